// hmg_fused.hip -- fused, LDS-tiled V-cycle kernels for gfx950.
//
// Each kernel performs the same per-node arithmetic as the one-pass kernels
// of hmg_kernels.hip (FP64 arithmetic on fields stored in the level
// precision; the LDS tiles hold FP64 values), but stages a tile of the level
// plus a halo in LDS so that one launch does several dependent steps and
// every field is read from and written to HBM about once:
//
//   k_gs_down     zero-guess red-black Gauss-Seidel sweep (role A operator),
//                 residual (role B operator) and full weighting to the next
//                 coarser level (Section 5: pre-smoothing and restriction);
//                 the smoothed iterate u0 is stored only when asked for;
//   k_gs_up       recomputes u0 (it depends on f only), adds the bilinear
//                 correction from the coarser level and does one red-black
//                 sweep (Section 5: prolongation and post-smoothing);
//   k_gs_up_u0    the same from a stored u0 (cache-resident FP64 levels);
//   k_kacz_tb     S sweeps of 5-colour Kaczmarz relaxation on a tile with a
//                 halo of 10 S nodes (each colour pass moves information two
//                 nodes), from zero or from u + P e; its RESID form also
//                 restricts the residual (the last pre-smoothing launch);
//   k_kacz_level  a whole level with n <= 63 in one workgroup (a tuner
//                 candidate);
//   k_kacz_table  the per-level row table (k, 1/||a_p||^2);
//   k_bottom      one workgroup runs the whole V-cycle on the small levels
//                 (relaxation, transfers and the dense coarsest solve) with
//                 the iterates resident in LDS; its BASIS form builds the
//                 matrix of that cycle, which k_dense_apply applies.
//
// A tile's workgroup writes only its own nodes and reads its halo from the
// input arrays, which no workgroup of the same launch writes.  Workgroups
// take tiles in XCD-contiguous bands (xcd_tile).

#include "hmg_device.h"

#include <type_traits>

namespace hmgk {

// sum_{q != p} a_pq U_q for an LDS array with row length LW (node p at l),
// neighbours in the order left, right, down, up.  The cells of a region
// that lie outside the domain hold zero and the row gives a missing
// neighbour weight zero, so all four cells are read without tests.
template <typename T>
__device__ __forceinline__ C<T> offsum_z(const Row<T> &r, const C<T> *U, int l, int LW) {
    const C<T> ul = U[l - 1], ur = U[l + 1], ud = U[l - LW], uu = U[l + LW];
    C<T> s = cmk(T(0), T(0));
    s = cadd(s, cscale(r.wl, ul));
    s = cadd(s, cscale(r.wr, ur));
    s = cadd(s, cscale(r.wd, ud));
    s = cadd(s, cscale(r.wu, uu));
    return s;
}

// One Kaczmarz row update in LDS (Section 4): d = (f_p - a_p u) / ||a_p||^2,
// u += conj(a_p) d on the five cells of the row.  Cells outside the domain
// are zero with zero weight and stay zero.
__device__ __forceinline__ void kacz_row_lds(C<double> *U, int l, int LW, const Row<double> &r, C<double> fp,
                                             double invn) {
    const C<double> uc = U[l], ul = U[l - 1], ur = U[l + 1], ud = U[l - LW], uu = U[l + LW];
    C<double> s = cmk(0.0, 0.0);
    s = cadd(s, cscale(r.wl, ul));
    s = cadd(s, cscale(r.wr, ur));
    s = cadd(s, cscale(r.wd, ud));
    s = cadd(s, cscale(r.wu, uu));
    const C<double> res = csub(fp, cadd(cmul(cmk(r.dre, r.dim), uc), s));
    const C<double> d = cmk(res.x * invn, res.y * invn);
    U[l] = cmk(uc.x + (r.dre * d.x + r.dim * d.y), uc.y + (r.dre * d.y - r.dim * d.x));
    U[l - 1] = cadd(ul, cscale(r.wl, d));
    U[l + 1] = cadd(ur, cscale(r.wr, d));
    U[l - LW] = cadd(ud, cscale(r.wd, d));
    U[l + LW] = cadd(uu, cscale(r.wu, d));
}

// Bilinear interpolation (Section 5) of the four coarse values around fine
// node (i, j): e00 = e(I, J), e10 = e(I+1, J), e01 = e(I, J+1),
// e11 = e(I+1, J+1) with I = i/2, J = j/2.  Selects, not branches; the sums
// are those of the one-pass prolongation, in the same order.
__device__ __forceinline__ C<double> bilinear(C<double> e00, C<double> e10, C<double> e01, C<double> e11, int i,
                                              int j) {
    const bool xo = i & 1, yo = j & 1;
    const C<double> sx = xo ? cadd(e00, e10) : e00;
    const C<double> s = yo ? (xo ? cadd(cadd(sx, e01), e11) : cadd(e00, e01)) : sx;
    const double w = (xo ? 0.5 : 1.0) * (yo ? 0.5 : 1.0);
    return cscale(w, s);
}

// bilinear interpolation of a coarse field in global memory at fine node
// (i, j) of the domain; the four loads are unconditional (indices clamped
// into the coarse grid; a clamped value gets weight zero)
template <typename T>
__device__ __forceinline__ C<double> prolong_at(const C<T> *ec, int i, int j, int Mc) {
    const int I = i >> 1, J = j >> 1;
    const int I1 = min(I + 1, Mc - 1), J1 = min(J + 1, Mc - 1);
    const C<double> e00 = ldr<double>(ec, (size_t)J * Mc + I), e10 = ldr<double>(ec, (size_t)J * Mc + I1);
    const C<double> e01 = ldr<double>(ec, (size_t)J1 * Mc + I), e11 = ldr<double>(ec, (size_t)J1 * Mc + I1);
    return bilinear(e00, e10, e01, e11, i, j);
}

__device__ __forceinline__ int mirror(int x, int N) { return x < 0 ? -x : (x > N ? 2 * N - x : x); }

// Tile of a workgroup.  Workgroups are dealt to the 8 XCDs of the chip in
// launch order, round-robin; each XCD gets a contiguous run of tiles (in
// row-major tile order) so that neighbouring tiles, which read each other's
// halo cells, share one L2.  A bijection of [0, T) for any T.
__device__ __forceinline__ void xcd_tile(int &tx, int &ty) {
    constexpr int NX = 8;
    const int T = gridDim.x * gridDim.y, bid = blockIdx.y * gridDim.x + blockIdx.x;
    const int x = bid % NX, base = T / NX, rem = T % NX;
    const int t = x * base + min(x, rem) + bid / NX;
    tx = t % gridDim.x;
    ty = t / gridDim.x;
}

// Row of node (i, j) for a region that may (IN = false) or may not (IN =
// true, every node of the region at least one node inside the boundary)
// touch the domain boundary.  The interior form gives the same values as
// row_at (weights 1/H^2, no boundary term) without its per-node tests.
template <bool IN>
__device__ __forceinline__ Row<double> row_in(int i, int j, int N, double H, double ih2, double kp, double sigma) {
    if (!IN) return row_at<double>(i, j, N, H, ih2, kp, sigma);
    Row<double> r;
    const double k2 = kp * kp;
    r.dre = -4.0 * ih2 + k2;
    r.dim = k2 * sigma;
    r.wl = r.wr = r.wd = r.wu = ih2;
    return r;
}

// ===========================================================================
// Fused Gauss-Seidel kernels.  A tile of X x Y fine nodes (x0, y0 even) is
// processed with a halo of RH = 3 held in LDS.  Each thread owns fixed
// red and black nodes of the haloed region (colour-compressed: node q of a
// colour maps to line q / HW, every other column), loads their f and k once,
// all loads in flight together, and keeps them in registers across the
// dependent phases, which then touch only LDS.
// ===========================================================================
constexpr int GNT = 256;

template <int DX, int DY, int H = 3>
struct GsTile {
    static constexpr int X = DX, Y = DY;                // tile (even sides)
    static constexpr int RH = H, LW = DX + 2 * RH, LH = DY + 2 * RH;
    static constexpr int HW = LW / 2;                   // nodes of one colour per line
    static constexpr int NC = HW * LH;                  // nodes of one colour in the region
    static constexpr int NS = (NC + GNT - 1) / GNT;     // owned nodes per colour per thread

    // local coordinates of owned node (colour c, slot m) of thread tid
    static __device__ __forceinline__ bool owned(int tid, int c, int m, int &lx, int &ly) {
        int q = tid + GNT * m;
        ly = q / HW;
        lx = 2 * (q % HW) + ((ly + c) & 1);             // red: (lx + ly) even
        return q < NC;
    }
    // ring distance from the region border: node (lx, ly) is in tile + h iff
    // lx >= RH - h, lx < LW - RH + h, and the same for ly
    static __device__ __forceinline__ bool ring(int lx, int ly, int h) {
        return lx >= RH - h && ly >= RH - h && lx < LW - RH + h && ly < LH - RH + h;
    }
};
// the finest levels use the large tile (less halo per node, fewer HBM
// re-reads); levels that would get fewer than two large tiles per CU use the
// small one, so that more workgroups share the latency of the dependent phases
using GsBig = GsTile<64, 20>;
using GsSmall = GsTile<32, 12>;
// the down kernel holds fewer values per node and prefers narrow tiles on
// the finest levels too: 16 x 16, the tallest with one node of each colour
// per thread (11 x 22 = 242 per colour in the region; 16641 workgroups at
// n = 2047), measured faster than 16 x 14, 16 x 12, 16 x 10 (40.3, 43.2,
// 45.0, 46.1 us at n = 2047), 64 x 12 and 32 x 12
using GsDownBig = GsTile<16, 16>;
// the up kernel that reads the stored pre-smoothed iterate needs a halo of 2
using GsBig2 = GsTile<64, 20, 2>;
// the up kernel with the Bi-CGSTAB matrix-vector product needs its result on
// tile + 1: a halo of 4
using GsBigMV = GsTile<64, 20, 4>;
using GsSmall2 = GsTile<32, 12, 2>;
// levels that would get fewer than four small tiles per CU (n <= 511) use
// tiles of half the width: one node of each colour per thread, shorter
// dependent phases, more workgroups to overlap them (and on n <= 255 more
// of the otherwise idle CUs)
using GsTiny = GsTile<16, 12>;
using GsTiny2 = GsTile<16, 12, 2>;

// ===========================================================================
// k_gs_down: one zero-guess red-black sweep (sigma_A), residual (sigma_B) on
// tile + 1, full weighting to the coarse nodes of the tile.  The smoothed
// iterate stays on chip (written only when uo != null).
// ===========================================================================
template <class TL, bool IN, typename T, typename TF>
__device__ __forceinline__ void k_gs_down_body(GeoT g, double H, double ih2, const T *__restrict__ k, double sa, double sb,
                                                const C<TF> *__restrict__ f, C<T> *uo, C<T> *__restrict__ fc,
                                                int uo_black, C<double> *U, int tid, int x0, int y0, int sk) {
    const int ox = x0 - TL::RH, oy = y0 - TL::RH;
    auto outside = [&](int i, int j) { return !IN && (i < 0 || j < 0 || i > g.N || j > g.N); };
    auto mir = [&](int x, int n) { return IN ? x : mirror(x, n); };
    (void)mir;
    const int N = g.N, M = g.M;
    C<double> fr[2][TL::NS];
    double kr[2][TL::NS];
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int m = 0; m < TL::NS; ++m) {
            int lx, ly;
            bool own = TL::owned(tid, c, m, lx, ly);
            int i = ox + lx, j = oy + ly;
            if (own && i >= 0 && j >= 0 && i <= N && j <= N) {
                size_t p = (size_t)j * M + i;
                fr[c][m] = ldr<double>(f, p);
                kr[c][m] = (double)k[p];
            }
        }
    if (flag_set(sk)) return;
    // red on tile + 3 (zero guess: u = f / a_pp); cells outside the domain
    // are set to zero (missing neighbours of the rows below)
#pragma unroll
    for (int m = 0; m < TL::NS; ++m) {
        int lx, ly;
        bool own = TL::owned(tid, 0, m, lx, ly);
        int i = ox + lx, j = oy + ly;
        if (!own) continue;
        if (outside(i, j)) {
            U[ly * TL::LW + lx] = cmk(0.0, 0.0);
            continue;
        }
        Row<double> r = row_in<IN>(i, j, N, H, ih2, kr[0][m], sa);
        U[ly * TL::LW + lx] = cdiv(fr[0][m], r.dre, r.dim);
    }
    __syncthreads();
    // black on tile + 2
#pragma unroll
    for (int m = 0; m < TL::NS; ++m) {
        int lx, ly;
        bool own = TL::owned(tid, 1, m, lx, ly);
        int i = ox + lx, j = oy + ly;
        if (!own || !TL::ring(lx, ly, 2)) continue;
        int l = ly * TL::LW + lx;
        if (outside(i, j)) {
            U[l] = cmk(0.0, 0.0);
            continue;
        }
        Row<double> r = row_in<IN>(i, j, N, H, ih2, kr[1][m], sa);
        U[l] = cdiv(csub(fr[1][m], offsum_z(r, U, l, TL::LW)), r.dre, r.dim);
    }
    __syncthreads();
    // the smoothed iterate on the tile (only when asked for: the up kernel
    // recomputes it), on the black nodes alone when uo_black (all the up
    // kernel reads)
    if (uo) {
#pragma unroll
        for (int m = 0; m < (TL::X * TL::Y + GNT - 1) / GNT; ++m) {
            const int q = tid + GNT * m;
            int tx = q % TL::X, ty = q / TL::X;
            int i = x0 + tx, j = y0 + ty;
            if (q >= TL::X * TL::Y || (!IN && (i > N || j > N)) || (uo_black && !((i + j) & 1))) continue;
            uo[(size_t)j * M + i] = st_as<T>(U[(ty + TL::RH) * TL::LW + tx + TL::RH]);
        }
    }
    // residual with the role-(B) operator on tile + 1, kept in registers
    // until every thread has read the iterate, then stored over it
    C<double> res[2][TL::NS];
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int m = 0; m < TL::NS; ++m) {
            int lx, ly;
            bool own = TL::owned(tid, c, m, lx, ly);
            int i = ox + lx, j = oy + ly;
            if (!own || !TL::ring(lx, ly, 1) || outside(i, j)) continue;
            int l = ly * TL::LW + lx;
            Row<double> r = row_in<IN>(i, j, N, H, ih2, kr[c][m], sb);
            C<double> au = cadd(cmul(cmk(r.dre, r.dim), U[l]), offsum_z(r, U, l, TL::LW));
            res[c][m] = csub(fr[c][m], au);
        }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int m = 0; m < TL::NS; ++m) {
            int lx, ly;
            bool own = TL::owned(tid, c, m, lx, ly);
            int i = ox + lx, j = oy + ly;
            if (!own || !TL::ring(lx, ly, 1) || outside(i, j)) continue;
            U[ly * TL::LW + lx] = res[c][m];
        }
    __syncthreads();
    // full weighting for the coarse nodes of this tile
    {
        const int Nc = N / 2, Mc = Nc + 1;
        constexpr int CX = TL::X / 2, NCN = (TL::X / 2) * (TL::Y / 2);
#pragma unroll
        for (int m = 0; m < (NCN + GNT - 1) / GNT; ++m) {
            const int q = tid + GNT * m;
            if (q >= NCN) break;
            int I = x0 / 2 + q % CX, J = y0 / 2 + q / CX;
            if (I > Nc || J > Nc) continue;
            C<double> s = cmk(0.0, 0.0);
            for (int e = -1; e <= 1; ++e) {
                int j = mir(2 * J + e, N);
                for (int d = -1; d <= 1; ++d) {
                    int i = mir(2 * I + d, N);
                    double w = (double)((2 - (d < 0 ? -d : d)) * (2 - (e < 0 ? -e : e)));
                    s = cadd(s, cscale(w, U[(j - oy) * TL::LW + (i - ox)]));
                }
            }
            fc[(size_t)J * Mc + I] = st_as<T>(cscale(0.0625, s));
        }
    }
}

template <class TL, typename T, typename TF>
__global__ __launch_bounds__(GNT) void k_gs_down(GeoT g, double H, double ih2, const T *__restrict__ k, double sa,
                                                 double sb, const C<TF> *__restrict__ f, C<T> *uo,
                                                 C<T> *__restrict__ fc, int uo_black, const int *skip, long zs) {
    f = zsh(f, zs);
    uo = zsh(uo, zs);
    fc = zsh(fc, zs);
    skip = zsh(skip, zs);
    const int sk = flag_read(skip);
    __shared__ C<double> U[TL::LW * TL::LH];      // the iterate, then the residual on tile + 1
    const int tid = threadIdx.x;
    int tx, ty;
    xcd_tile(tx, ty);
    const int x0 = tx * TL::X, y0 = ty * TL::Y;
    const int N = g.N;
    // tiles whose region lies inside the domain skip the boundary tests
    if (x0 - TL::RH >= 1 && y0 - TL::RH >= 1 && x0 - TL::RH + TL::LW <= N && y0 - TL::RH + TL::LH <= N)
        k_gs_down_body<TL, true>(g, H, ih2, k, sa, sb, f, uo, fc, uo_black, U, tid, x0, y0, sk);
    else
        k_gs_down_body<TL, false>(g, H, ih2, k, sa, sb, f, uo, fc, uo_black, U, tid, x0, y0, sk);
}

// ===========================================================================
// k_gs_up: u0 = the zero-guess red-black sweep of k_gs_down (recomputed from
// f), u = u0 + P ec, then one red-black sweep; result to uo.  Regions shrink
// by one per dependent step: red u0 on tile + 3, black u0 plus correction on
// tile + 2, red on tile + 1, black on the tile.  The red half-sweep reads
// only black values, so red nodes never get the correction: their values
// before the sweep are overwritten unread (the result is that of u0 + P ec
// on every node).  Tiles whose
// region lies inside the domain run the phases without boundary tests (a
// branch per workgroup; the same values either way).
// ===========================================================================
template <class TL, bool IN, typename T, typename TU>
__device__ __forceinline__ void gs_up_phases(C<double> *U, int tid, int ox, int oy, int N, int M, int Mc, double H,
                                             double ih2, double sa, const C<double> (&fr)[2][TL::NS],
                                             const double (&kr)[2][TL::NS], const C<T> *__restrict__ ec,
                                             C<TU> *__restrict__ uo) {
    auto prolong = [&](int i, int j) { return prolong_at(ec, i, j, Mc); };
    auto outside = [&](int i, int j) { return !IN && (i < 0 || j < 0 || i > N || j > N); };
    // red u0 on tile + 3 (zero outside the domain)
#pragma unroll
    for (int m = 0; m < TL::NS; ++m) {
        int lx, ly;
        bool own = TL::owned(tid, 0, m, lx, ly);
        int i = ox + lx, j = oy + ly;
        if (!own) continue;
        if (outside(i, j)) {
            U[ly * TL::LW + lx] = cmk(0.0, 0.0);
            continue;
        }
        Row<double> r = row_in<IN>(i, j, N, H, ih2, kr[0][m], sa);
        U[ly * TL::LW + lx] = cdiv(fr[0][m], r.dre, r.dim);
    }
    __syncthreads();
    // black u0 on tile + 2, plus the correction on the black nodes
#pragma unroll
    for (int m = 0; m < TL::NS; ++m) {
        int lx, ly;
        bool own = TL::owned(tid, 1, m, lx, ly);
        int i = ox + lx, j = oy + ly;
        if (!own || !TL::ring(lx, ly, 2)) continue;
        int l = ly * TL::LW + lx;
        if (outside(i, j)) {
            U[l] = cmk(0.0, 0.0);
            continue;
        }
        Row<double> r = row_in<IN>(i, j, N, H, ih2, kr[1][m], sa);
        U[l] = cadd(cdiv(csub(fr[1][m], offsum_z(r, U, l, TL::LW)), r.dre, r.dim), prolong(i, j));
    }
    __syncthreads();
    // red on tile + 1 (the red half-sweep reads only black values, so the
    // correction is needed on the black nodes alone)
#pragma unroll
    for (int m = 0; m < TL::NS; ++m) {
        int lx, ly;
        bool own = TL::owned(tid, 0, m, lx, ly);
        int i = ox + lx, j = oy + ly;
        if (!own || !TL::ring(lx, ly, 1) || outside(i, j)) continue;
        int l = ly * TL::LW + lx;
        Row<double> r = row_in<IN>(i, j, N, H, ih2, kr[0][m], sa);
        U[l] = cdiv(csub(fr[0][m], offsum_z(r, U, l, TL::LW)), r.dre, r.dim);
    }
    __syncthreads();
    // black on the tile -> output; red tile nodes -> output
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int m = 0; m < TL::NS; ++m) {
            int lx, ly;
            bool own = TL::owned(tid, c, m, lx, ly);
            int i = ox + lx, j = oy + ly;
            if (!own || !TL::ring(lx, ly, 0) || (!IN && (i > N || j > N))) continue;
            int l = ly * TL::LW + lx;
            C<double> v = U[l];
            if (c == 1) {
                Row<double> r = row_in<IN>(i, j, N, H, ih2, kr[1][m], sa);
                v = cdiv(csub(fr[1][m], offsum_z(r, U, l, TL::LW)), r.dre, r.dim);
            }
            uo[(size_t)j * M + i] = st_as<TU>(v);
        }
}

// f and k of the nodes of tile (ox + RH, oy + RH) owned by thread tid
template <class TL, typename T, typename TF>
__device__ __forceinline__ void gs_load(int tid, int ox, int oy, int N, int M, const C<TF> *__restrict__ f,
                                        const T *__restrict__ k, C<double> (&fr)[2][TL::NS],
                                        double (&kr)[2][TL::NS]) {
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int m = 0; m < TL::NS; ++m) {
            int lx, ly;
            bool own = TL::owned(tid, c, m, lx, ly);
            int i = ox + lx, j = oy + ly;
            if (own && i >= 0 && j >= 0 && i <= N && j <= N) {
                size_t p = (size_t)j * M + i;
                fr[c][m] = ldr<double>(f, p);
                kr[c][m] = (double)k[p];
            }
        }
}

// ===========================================================================
// k_gs_up_mv: k_gs_up on the finest level of an FP64 solve, followed by the
// Bi-CGSTAB product with L of the result it writes (Section 6): the phases
// run one ring further out (red u0 on tile + 4, black u0 + correction on
// tile + 3, red on tile + 2, black on tile + 1), so that uo is known on tile
// + 1 in LDS; then mvo = L uo on the tile and the block's partial sums
//   KIND 1: (dot, mvo)                 (v = L p^ and (rh, v), for alpha)
//   KIND 2: (mvo, dot), (mvo, mvo)     (t = L s^, (t, s) and (t, t), for omega)
// with (a, b) = sum conj(a) b, written to partials[q * blocks + block] as the
// separate product kernels do.  The product kernel and its launch go away.
// uo may be null: then only mvo and the sums leave the kernel.
// ===========================================================================
template <bool IN, int KIND>
__device__ __forceinline__ void gs_up_mv_phases(C<double> *U, int tid, int ox, int oy, int N, int M, int Mc,
                                                double H, double ih2, double sa,
                                                const C<double> (&fr)[2][GsBigMV::NS],
                                                const double (&kr)[2][GsBigMV::NS],
                                                const C<double> *__restrict__ ec, C<double> *__restrict__ uo,
                                                C<double> *__restrict__ mvo, const C<double> *__restrict__ dot,
                                                double *partials, const double *__restrict__ k) {
    using TL = GsBigMV;
    auto prolong = [&](int i, int j) { return prolong_at(ec, i, j, Mc); };
    auto outside = [&](int i, int j) { return !IN && (i < 0 || j < 0 || i > N || j > N); };
    // red u0 on tile + 4 (zero outside the domain)
#pragma unroll
    for (int m = 0; m < TL::NS; ++m) {
        int lx, ly;
        bool own = TL::owned(tid, 0, m, lx, ly);
        int i = ox + lx, j = oy + ly;
        if (!own) continue;
        if (outside(i, j)) {
            U[ly * TL::LW + lx] = cmk(0.0, 0.0);
            continue;
        }
        Row<double> r = row_in<IN>(i, j, N, H, ih2, kr[0][m], sa);
        U[ly * TL::LW + lx] = cdiv(fr[0][m], r.dre, r.dim);
    }
    __syncthreads();
    // black u0 plus the correction on tile + 3
#pragma unroll
    for (int m = 0; m < TL::NS; ++m) {
        int lx, ly;
        bool own = TL::owned(tid, 1, m, lx, ly);
        int i = ox + lx, j = oy + ly;
        if (!own || !TL::ring(lx, ly, 3)) continue;
        int l = ly * TL::LW + lx;
        if (outside(i, j)) {
            U[l] = cmk(0.0, 0.0);
            continue;
        }
        Row<double> r = row_in<IN>(i, j, N, H, ih2, kr[1][m], sa);
        U[l] = cadd(cdiv(csub(fr[1][m], offsum_z(r, U, l, TL::LW)), r.dre, r.dim), prolong(i, j));
    }
    __syncthreads();
    // red on tile + 2; then black on tile + 1 (black reads red only, so it
    // writes its own cells in place)
#pragma unroll
    for (int m = 0; m < TL::NS; ++m) {
        int lx, ly;
        bool own = TL::owned(tid, 0, m, lx, ly);
        int i = ox + lx, j = oy + ly;
        if (!own || !TL::ring(lx, ly, 2) || outside(i, j)) continue;
        int l = ly * TL::LW + lx;
        Row<double> r = row_in<IN>(i, j, N, H, ih2, kr[0][m], sa);
        U[l] = cdiv(csub(fr[0][m], offsum_z(r, U, l, TL::LW)), r.dre, r.dim);
    }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < TL::NS; ++m) {
        int lx, ly;
        bool own = TL::owned(tid, 1, m, lx, ly);
        int i = ox + lx, j = oy + ly;
        if (!own || !TL::ring(lx, ly, 1) || outside(i, j)) continue;
        int l = ly * TL::LW + lx;
        Row<double> r = row_in<IN>(i, j, N, H, ih2, kr[1][m], sa);
        U[l] = cdiv(csub(fr[1][m], offsum_z(r, U, l, TL::LW)), r.dre, r.dim);
    }
    __syncthreads();
    // Results leave in row order: thread q of a pass takes tile node (q % X,
    // q / X), so each wave stores whole 1 KB row segments (a colour-ordered
    // store would leave every cache line in two halves, from two passes).
    constexpr int NT_TILE = TL::X * TL::Y, NP = (NT_TILE + GNT - 1) / GNT;
    if (uo) {
#pragma unroll
        for (int m = 0; m < NP; ++m) {
            const int q = tid + GNT * m;
            const int tx = q % TL::X, ty = q / TL::X, i = ox + TL::RH + tx, j = oy + TL::RH + ty;
            if (q >= NT_TILE || (!IN && (i > N || j > N))) continue;
            uo[(size_t)j * M + i] = U[(ty + TL::RH) * TL::LW + tx + TL::RH];
        }
    }
    // the product with L (sigma = 0) on the tile, in the same row order, with
    // the block's partial sums; k of the tile is read again (in row order,
    // from the cache: the tile's own k was loaded at the start) instead of
    // keeping colour-ordered values in registers across the pass
    constexpr int NV = KIND == 1 ? 2 : 3;
    // an opaque copy of tid: reusing the positions of the sweeps would keep
    // them live across every phase and push the kernel past 128 VGPRs (three
    // waves per SIMD instead of four)
    int tid2 = tid;
    asm volatile("" : "+v"(tid2));
    double acc[NV];
#pragma unroll
    for (int q = 0; q < NV; ++q) acc[q] = 0.0;
#pragma unroll
    for (int m = 0; m < NP; ++m) {
        const int q = tid2 + GNT * m;
        const int tx = q % TL::X, ty = q / TL::X, i = ox + TL::RH + tx, j = oy + TL::RH + ty;
        if (q >= NT_TILE || (!IN && (i > N || j > N))) continue;
        const size_t p = (size_t)j * M + i;
        const int l = (ty + TL::RH) * TL::LW + tx + TL::RH;
        const Row<double> r = row_in<IN>(i, j, N, H, ih2, k[p], 0.0);
        const C<double> v = cadd(cmul(cmk(r.dre, r.dim), U[l]), offsum_z(r, U, l, TL::LW));
        mvo[p] = v;
        const C<double> a = dot[p];
        if (KIND == 1) {
            acc[0] += a.x * v.x + a.y * v.y;      // conj(rh) v
            acc[NV - 1] += a.x * v.y - a.y * v.x;
        } else {
            acc[0] += v.x * a.x + v.y * a.y;      // conj(t) s
            acc[1] += v.x * a.y - v.y * a.x;
            acc[NV - 1] += v.x * v.x + v.y * v.y;
        }
    }
    block_partials<NV>(acc, partials);
}

template <int KIND>
__global__ __launch_bounds__(GNT) void k_gs_up_mv(GeoT g, double H, double ih2, const double *__restrict__ k,
                                                  double sa, const C<double> *__restrict__ f,
                                                  const C<double> *__restrict__ ec, C<double> *__restrict__ uo,
                                                  C<double> *__restrict__ mvo, const C<double> *__restrict__ dot,
                                                  double *partials, const int *skip, long zs) {
    using TL = GsBigMV;
    f = zsh(f, zs);
    ec = zsh(ec, zs);
    uo = zsh(uo, zs);
    mvo = zsh(mvo, zs);
    dot = zsh(dot, zs);
    partials = zsh(partials, zs);
    skip = zsh(skip, zs);
    const int sk = flag_read(skip);
    __shared__ C<double> U[TL::LW * TL::LH];
    const int tid = threadIdx.x;
    int tx, ty;
    xcd_tile(tx, ty);
    const int ox = tx * TL::X - TL::RH, oy = ty * TL::Y - TL::RH;
    const int N = g.N, M = g.M, Mc = N / 2 + 1;
    C<double> fr[2][TL::NS];
    double kr[2][TL::NS];
    gs_load<TL>(tid, ox, oy, N, M, f, k, fr, kr);
    if (flag_set(sk)) return;
    if (ox >= 1 && oy >= 1 && ox + TL::LW <= N && oy + TL::LH <= N)
        gs_up_mv_phases<true, KIND>(U, tid, ox, oy, N, M, Mc, H, ih2, sa, fr, kr, ec, uo, mvo, dot, partials, k);
    else
        gs_up_mv_phases<false, KIND>(U, tid, ox, oy, N, M, Mc, H, ih2, sa, fr, kr, ec, uo, mvo, dot, partials, k);
}

template <class TL, typename T, typename TF, typename TU>
__global__ __launch_bounds__(GNT) void k_gs_up(GeoT g, double H, double ih2, const T *__restrict__ k, double sa,
                                               const C<TF> *__restrict__ f, const C<T> *__restrict__ ec,
                                               C<TU> *__restrict__ uo, const int *skip, long zs) {
    f = zsh(f, zs);
    ec = zsh(ec, zs);
    uo = zsh(uo, zs);
    skip = zsh(skip, zs);
    const int sk = flag_read(skip);
    __shared__ C<double> U[TL::LW * TL::LH];
    const int tid = threadIdx.x;
    int tx, ty;
    xcd_tile(tx, ty);
    const int x0 = tx * TL::X, y0 = ty * TL::Y;
    const int ox = x0 - TL::RH, oy = y0 - TL::RH;
    const int N = g.N, M = g.M, Mc = N / 2 + 1;
    C<double> fr[2][TL::NS];
    double kr[2][TL::NS];
    gs_load<TL>(tid, ox, oy, N, M, f, k, fr, kr);
    if (flag_set(sk)) return;
    if (ox >= 1 && oy >= 1 && ox + TL::LW <= N && oy + TL::LH <= N)
        gs_up_phases<TL, true>(U, tid, ox, oy, N, M, Mc, H, ih2, sa, fr, kr, ec, uo);
    else
        gs_up_phases<TL, false>(U, tid, ox, oy, N, M, Mc, H, ih2, sa, fr, kr, ec, uo);
}

// ===========================================================================
// k_gs_up_u0: as k_gs_up, but the pre-smoothed iterate u0 is read from
// memory (written by k_gs_down) instead of recomputed: u = u0 + P ec on the
// black nodes of tile + 2 (red values are overwritten unread), red on tile
// + 1, black on the tile -> uo.  Used where u0 is stored without rounding
// (FP64 levels); three phases instead of four.
// ===========================================================================
template <class TL, bool IN, typename T, typename TF, typename TU>
__device__ __forceinline__ void k_gs_up_u0_body(GeoT g, double H, double ih2, const T *__restrict__ k, double sa,
                                                 const C<TF> *__restrict__ f, const C<T> *__restrict__ u0,
                                                 const C<T> *__restrict__ ec, C<TU> *__restrict__ uo,
                                                 C<double> *U, int tid, int x0, int y0, int sk) {
    const int ox = x0 - TL::RH, oy = y0 - TL::RH;
    auto outside = [&](int i, int j) { return !IN && (i < 0 || j < 0 || i > g.N || j > g.N); };
    auto mir = [&](int x, int n) { return IN ? x : mirror(x, n); };
    (void)mir;
    const int N = g.N, M = g.M, Mc = N / 2 + 1;
    // f and k of the nodes relaxed here (tile + 1), and u0 + P ec on tile + 2
    C<double> fr[2][TL::NS];
    double kr[2][TL::NS];
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int m = 0; m < TL::NS; ++m) {
            int lx, ly;
            bool own = TL::owned(tid, c, m, lx, ly);
            int i = ox + lx, j = oy + ly;
            if (!own) continue;
            const int l = ly * TL::LW + lx;
            if (outside(i, j)) {
                U[l] = cmk(0.0, 0.0);
                continue;
            }
            const size_t p = (size_t)j * M + i;
            if (TL::ring(lx, ly, 1)) {
                fr[c][m] = ldr<double>(f, p);
                kr[c][m] = (double)k[p];
            }
            // the red half-sweep reads only black values: red nodes need
            // neither u0 nor the correction (their cells are overwritten
            // on tile + 1 and never read elsewhere)
            U[l] = (c == 1) ? cadd(ldr<double>(u0, p), prolong_at(ec, i, j, Mc)) : cmk(0.0, 0.0);
        }
    if (flag_set(sk)) return;
    __syncthreads();
    // red on tile + 1
#pragma unroll
    for (int m = 0; m < TL::NS; ++m) {
        int lx, ly;
        bool own = TL::owned(tid, 0, m, lx, ly);
        int i = ox + lx, j = oy + ly;
        if (!own || !TL::ring(lx, ly, 1) || outside(i, j)) continue;
        int l = ly * TL::LW + lx;
        Row<double> r = row_in<IN>(i, j, N, H, ih2, kr[0][m], sa);
        U[l] = cdiv(csub(fr[0][m], offsum_z(r, U, l, TL::LW)), r.dre, r.dim);
    }
    __syncthreads();
    // black on the tile -> output; red tile nodes -> output
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int m = 0; m < TL::NS; ++m) {
            int lx, ly;
            bool own = TL::owned(tid, c, m, lx, ly);
            int i = ox + lx, j = oy + ly;
            if (!own || !TL::ring(lx, ly, 0) || (!IN && (i > N || j > N))) continue;
            int l = ly * TL::LW + lx;
            C<double> v = U[l];
            if (c == 1) {
                Row<double> r = row_in<IN>(i, j, N, H, ih2, kr[1][m], sa);
                v = cdiv(csub(fr[1][m], offsum_z(r, U, l, TL::LW)), r.dre, r.dim);
            }
            uo[(size_t)j * M + i] = st_as<TU>(v);
        }
}

template <class TL, typename T, typename TF, typename TU>
__global__ __launch_bounds__(GNT) void k_gs_up_u0(GeoT g, double H, double ih2, const T *__restrict__ k, double sa,
                                                  const C<TF> *__restrict__ f, const C<T> *__restrict__ u0,
                                                  const C<T> *__restrict__ ec, C<TU> *__restrict__ uo,
                                                  const int *skip, long zs) {
    static_assert(TL::RH == 2, "halo of two");
    f = zsh(f, zs);
    u0 = zsh(u0, zs);
    ec = zsh(ec, zs);
    uo = zsh(uo, zs);
    skip = zsh(skip, zs);
    const int sk = flag_read(skip);
    __shared__ C<double> U[TL::LW * TL::LH];
    const int tid = threadIdx.x;
    int tx, ty;
    xcd_tile(tx, ty);
    const int x0 = tx * TL::X, y0 = ty * TL::Y;
    const int N = g.N;
    // tiles whose region lies inside the domain skip the boundary tests
    if (x0 - TL::RH >= 1 && y0 - TL::RH >= 1 && x0 - TL::RH + TL::LW <= N && y0 - TL::RH + TL::LH <= N)
        k_gs_up_u0_body<TL, true>(g, H, ih2, k, sa, f, u0, ec, uo, U, tid, x0, y0, sk);
    else
        k_gs_up_u0_body<TL, false>(g, H, ih2, k, sa, f, u0, ec, uo, U, tid, x0, y0, sk);
}

// ===========================================================================
// k_kacz_tb: S sweeps of 5-colour Kaczmarz on a TS x TY tile (TY = TS unless
// given) held in LDS
// with a halo of RH = 10 S (each colour pass moves information two nodes).
// Pass q (colour q mod 5) updates the rows on tile + (RH - 2q - 1); after it
// u is exact on tile + (RH - 2q - 2), and after the last pass on the tile
// itself.  Each thread keeps the same row slots (line, column slot) in every
// pass, so a pass needs no division to find its rows.  Cells of the region
// outside the domain hold zero; two rows of one colour never share a cell
// (the five-point stars of one colour tile the plane), so a row reads and
// writes its five cells without tests and the padding stays zero.  Initial
// u: 0 (ui == null) or ui, plus P ec when ec != null.  The region is loaded
// CH cells per thread at a time with every global load of a batch issued
// before the first is used (indices clamped into the domain).  ktab, when
// given, holds (k_p, 1 / ||a_p||^2) for sigma (k_kacz_table); else both are
// formed here.
//
// RESID (the last pre-smoothing launch of a level, Section 5): the halo
// grows by two and the tile shrinks by four (the same LDS region), so that
// after the passes u is exact on tile + 2; the residual with sigma_b is
// formed on tile + 1 and full-weighted to the coarse nodes of the tile (fc),
// which replaces the separate residual and restriction kernel.
// ===========================================================================
template <typename T, int TS0, int S, int NT, bool RESID, int TY0 = TS0>
__global__ __launch_bounds__(NT) void k_kacz_tb(GeoT g, double H, double ih2, const T *__restrict__ k,
                                                const C<double> *__restrict__ ktab, double sig,
                                                double sigb, const C<T> *__restrict__ f,
                                                const C<T> *__restrict__ ui, const C<T> *__restrict__ ec,
                                                C<T> *__restrict__ uo, C<T> *__restrict__ fc, const int *skip,
                                                long zs) {
    f = zsh(f, zs);
    ui = zsh(ui, zs);
    ec = zsh(ec, zs);
    uo = zsh(uo, zs);
    fc = zsh(fc, zs);
    skip = zsh(skip, zs);
    const int sk = flag_read(skip);
    constexpr int TS = RESID ? TS0 - 4 : TS0, TY = RESID ? TY0 - 4 : TY0;
    constexpr int RH = 10 * S + (RESID ? 2 : 0), LW = TS + 2 * RH, LH = TY + 2 * RH;
    // f and (k, 1/||a_p||^2) of the region are staged in LDS when they fit
    // next to u
    constexpr bool STAGE = (size_t)LW * LH * (16 + 16 + 16) <= 160 * 1024;
    static_assert(STAGE || !RESID, "the fused residual needs the staged region");
    static_assert(TS % 2 == 0 && TY % 2 == 0, "tiles start on coarse nodes");
    constexpr int T5 = (LW - 2 + 4) / 5;              // row slots per line and colour
    constexpr int NSLOT = (LH - 2) * T5;              // slots per colour
    constexpr int NM = (NSLOT + NT - 1) / NT;         // slots per thread and colour
    constexpr int NL = (LW * LH + NT - 1) / NT;       // region cells per thread
    // cells per load batch: about 28 registers each in flight, within the
    // budget of NT threads per workgroup
    constexpr int CHMAX = NT >= 1024 ? 2 : 4;
    constexpr int CH = NL < CHMAX ? NL : CHMAX;
    __shared__ C<double> U[LW * LH];
    __shared__ C<double> FS[STAGE ? LW * LH : 1];
    __shared__ C<double> KS[STAGE ? LW * LH : 1];
    const int tid = threadIdx.x;
    int tx, ty;
    xcd_tile(tx, ty);
    const int x0 = tx * TS, y0 = ty * TY;
    const int ox = x0 - RH, oy = y0 - RH;
    const int N = g.N, M = g.M, Mc = N / 2 + 1;
    // FP64 fields with a row table: f and (k, 1/||a_p||^2) go straight from
    // memory into LDS (16 B per lane, lane-contiguous destinations within a
    // wave), bypassing registers.  Cells outside the domain get the clamped
    // copies, which no row reads.
    const bool dma = std::is_same<T, double>::value && STAGE && ktab != nullptr;
    if (dma) {
        const int wbase = tid & ~63;
        for (int kk = 0; kk < NL; ++kk) {
            const int q = tid + NT * kk;
            if (q < LW * LH) {
                const int i = min(max(ox + q % LW, 0), N), j = min(max(oy + q / LW, 0), N);
                const size_t p = (size_t)j * M + i;
                __builtin_amdgcn_global_load_lds((const void *)(f + p),
                                                 (__attribute__((address_space(3))) void *)&FS[wbase + NT * kk],
                                                 16, 0, 0);
                __builtin_amdgcn_global_load_lds((const void *)(ktab + p),
                                                 (__attribute__((address_space(3))) void *)&KS[wbase + NT * kk],
                                                 16, 0, 0);
            }
        }
    }
    for (int b0 = 0; b0 < NL; b0 += CH) {
        C<double> vu[CH], vf[CH], e[CH][4], vkn[CH];   // vkn: (k, 1/||a_p||^2) or (k, -)
#pragma unroll
        for (int s = 0; s < CH; ++s) {
            const int q = tid + NT * (b0 + s);
            const int i = min(max(ox + q % LW, 0), N), j = min(max(oy + q / LW, 0), N);
            const size_t p = (size_t)j * M + i;
            vu[s] = ui ? ldr<double>(ui, p) : cmk(0.0, 0.0);
            if (ec) {
                const int I = i >> 1, J = j >> 1, I1 = min(I + 1, Mc - 1), J1 = min(J + 1, Mc - 1);
                e[s][0] = ldr<double>(ec, (size_t)J * Mc + I);
                e[s][1] = ldr<double>(ec, (size_t)J * Mc + I1);
                e[s][2] = ldr<double>(ec, (size_t)J1 * Mc + I);
                e[s][3] = ldr<double>(ec, (size_t)J1 * Mc + I1);
            }
            if (STAGE && !dma) {
                vf[s] = ldr<double>(f, p);
                vkn[s] = ktab ? ktab[p] : cmk((double)k[p], 0.0);
            }
        }
#pragma unroll
        for (int s = 0; s < CH; ++s) {
            const int q = tid + NT * (b0 + s);
            if (q >= LW * LH) continue;
            const int i = ox + q % LW, j = oy + q / LW;
            const bool in = i >= 0 && j >= 0 && i <= N && j <= N;
            C<double> v = vu[s];
            if (ec) v = cadd(v, bilinear(e[s][0], e[s][1], e[s][2], e[s][3], i, j));
            U[q] = in ? v : cmk(0.0, 0.0);
            if (STAGE && !dma) {
                FS[q] = in ? vf[s] : cmk(0.0, 0.0);
                C<double> kn = vkn[s];
                if (!ktab) {
                    Row<double> r = row_at<double>(min(max(i, 0), N), min(max(j, 0), N), N, H, ih2, kn.x, sig);
                    double nrm =
                        r.dre * r.dre + r.dim * r.dim + r.wl * r.wl + r.wr * r.wr + r.wd * r.wd + r.wu * r.wu;
                    kn.y = 1.0 / nrm;
                }
                KS[q] = in ? kn : cmk(0.0, 0.0);
            }
        }
    }
    // row slots of this thread: line ly = 1 + s / T5, column slot t = s % T5;
    // for colour c the row sits at lx = 1 + ((c + a) mod 5) + 5 t with
    // a = (-(ox + 1) - 2 j) mod 5 fixed per line (lines outside the domain
    // get no slot)
    int sly[NM], sbase[NM], sa[NM];
#pragma unroll
    for (int m = 0; m < NM; ++m) {
        const int sl = tid + NT * m, ly = 1 + sl / T5, j = oy + ly;
        sly[m] = (sl < NSLOT && j >= 0 && j <= N) ? ly : -1;
        sbase[m] = 1 + 5 * (sl % T5);
        sa[m] = (((-(ox + 1) - 2 * j) % 5) + 5) % 5;
    }
    if (dma) __builtin_amdgcn_s_waitcnt(0);   // the direct loads have landed in LDS
    if (flag_set(sk)) return;
    __syncthreads();
#pragma unroll
    for (int pass = 0; pass < 5 * S; ++pass) {
        const int c = pass % 5;
        // rows on tile + (RH - 2 pass - 1)
        const int lo = 2 * pass + 1, hi = LW - 2 - 2 * pass, hiy = LH - 2 - 2 * pass;
#pragma unroll
        for (int m = 0; m < NM; ++m) {
            const int ly = sly[m];
            if (ly < lo || ly > hiy) continue;
            const int j = oy + ly;
            const int ca = c + sa[m];
            const int lx = (ca >= 5 ? ca - 5 : ca) + sbase[m];
            const int i = ox + lx;
            if (lx < lo || lx > hi || i < 0 || i > N) continue;
            const int l = ly * LW + lx;
            if (STAGE) {
                const C<double> kc = KS[l];
                const C<double> fp = FS[l];
                kacz_row_lds(U, l, LW, row_at<double>(i, j, N, H, ih2, kc.x, sig), fp, kc.y);
            } else {
                // (k, 1/||a_p||^2) from the row table when there is one, the
                // values the staged configurations read, so that every
                // configuration gives the same bits
                const size_t p = (size_t)j * M + i;
                C<double> kc;
                if (ktab) {
                    kc = ktab[p];
                } else {
                    const Row<double> r = row_at<double>(i, j, N, H, ih2, (double)k[p], sig);
                    kc = cmk((double)k[p], 1.0 / (r.dre * r.dre + r.dim * r.dim + r.wl * r.wl + r.wr * r.wr +
                                                  r.wd * r.wd + r.wu * r.wu));
                }
                kacz_row_lds(U, l, LW, row_at<double>(i, j, N, H, ih2, kc.x, sig), ldr<double>(f, p), kc.y);
            }
        }
        __syncthreads();
    }
    for (int q = tid; q < TS * TY; q += NT) {
        int i = x0 + q % TS, j = y0 + q / TS;
        if (i > N || j > N) continue;
        uo[(size_t)j * M + i] = st_as<T>(U[(j - oy) * LW + (i - ox)]);
    }
    if constexpr (RESID) {
        // residual f - A_{sigma_b} u on tile + 1, kept in registers until
        // every thread has read f, then stored over f
        constexpr int W1 = TS + 2, H1 = TY + 2, NR = (W1 * H1 + NT - 1) / NT;
        C<double> res[NR];
#pragma unroll
        for (int m = 0; m < NR; ++m) {
            const int q = tid + NT * m;
            const int lx = RH - 1 + q % W1, ly = RH - 1 + q / W1, i = ox + lx, j = oy + ly;
            if (q >= W1 * H1 || i < 0 || j < 0 || i > N || j > N) continue;
            const int l = ly * LW + lx;
            Row<double> r = row_at<double>(i, j, N, H, ih2, KS[l].x, sigb);
            res[m] = csub(FS[l], cadd(cmul(cmk(r.dre, r.dim), U[l]), offsum_z(r, U, l, LW)));
        }
        __syncthreads();
#pragma unroll
        for (int m = 0; m < NR; ++m) {
            const int q = tid + NT * m;
            const int lx = RH - 1 + q % W1, ly = RH - 1 + q / W1, i = ox + lx, j = oy + ly;
            if (q >= W1 * H1 || i < 0 || j < 0 || i > N || j > N) continue;
            FS[ly * LW + lx] = res[m];
        }
        __syncthreads();
        // full weighting (mirrored at the boundary) for the coarse nodes of
        // the tile
        const int Nc = N / 2, Mc = Nc + 1;
        constexpr int CX = TS / 2, CY = TY / 2;
        for (int q = tid; q < CX * CY; q += NT) {
            const int I = x0 / 2 + q % CX, J = y0 / 2 + q / CX;
            if (I > Nc || J > Nc) continue;
            C<double> sum = cmk(0.0, 0.0);
            for (int e = -1; e <= 1; ++e) {
                const int j = mirror(2 * J + e, N);
                for (int d = -1; d <= 1; ++d) {
                    const int i = mirror(2 * I + d, N);
                    const double w = (double)((2 - (d < 0 ? -d : d)) * (2 - (e < 0 ? -e : e)));
                    sum = cadd(sum, cscale(w, FS[(j - oy) * LW + (i - ox)]));
                }
            }
            fc[(size_t)J * Mc + I] = st_as<T>(cscale(0.0625, sum));
        }
    }
}

// ===========================================================================
// k_kacz_level: the whole level (n <= 63) in one workgroup of LNT threads.
// u lives in LDS with a ring of zero cells; each thread owns one row slot
// (line j, column block t) and keeps f and (k, 1/||a_p||^2) of the slot's
// five cells, one per colour, in registers.  `sweeps` 5-colour sweeps from
// ui (null: zero) plus P ec (null: none), then u to uo and, when fc != null,
// fc = R (f - A_{sigb} u) (the restriction of the level's pre-smoothing).
// No halo is recomputed: every pass updates exactly the rows of its colour.
// ===========================================================================
constexpr int LNT = 1024, LMAX = 65;          // threads; largest M = n + 2

template <typename T>
__global__ __launch_bounds__(LNT) void k_kacz_level(GeoT g, double H, double ih2, const T *__restrict__ k,
                                                   const C<double> *__restrict__ ktab, double sig, double sigb,
                                                   int sweeps, const C<T> *__restrict__ f,
                                                   const C<T> *__restrict__ ui, const C<T> *__restrict__ ec,
                                                   C<T> *__restrict__ uo, C<T> *__restrict__ fc,
                                                   const int *skip) {
    if (skip && *skip) return;
    constexpr int PW = LMAX + 2;
    __shared__ C<double> U[PW * PW];          // node (i, j) at (j + 1) * pw + i + 1
    __shared__ C<double> KS[LMAX * LMAX];     // (k, 1/||a_p||^2); later the residual
    const int tid = threadIdx.x;
    const int N = g.N, M = g.M, pw = M + 2, Mc = N / 2 + 1;
    const int W5 = (M + 4) / 5;
    // slot of this thread: line j, cells i = 5 t + r (r = 0..4); the colour
    // of cell r is (i + 2 j) mod 5
    const int j = tid / W5, t = tid % W5;
    const bool slot = tid < M * W5;
    C<double> fr[5];
#pragma unroll
    for (int r = 0; r < 5; ++r) fr[r] = ldr<double>(f, (size_t)min(j, N) * M + min(5 * t + r, N));
    // u: zero ring, ui + P ec inside; the row table
    for (int q = tid; q < pw * pw; q += LNT) {
        const int i = q % pw - 1, jq = q / pw - 1;
        C<double> v = cmk(0.0, 0.0);
        if (i >= 0 && jq >= 0 && i <= N && jq <= N) {
            const size_t p = (size_t)jq * M + i;
            if (ui) v = ldr<double>(ui, p);
            if (ec) v = cadd(v, prolong_at(ec, i, jq, Mc));
            C<double> kn;
            if (ktab) {
                kn = ktab[p];
            } else {
                kn.x = (double)k[p];
                Row<double> rw = row_at<double>(i, jq, N, H, ih2, kn.x, sig);
                kn.y = 1.0 / (rw.dre * rw.dre + rw.dim * rw.dim + rw.wl * rw.wl + rw.wr * rw.wr +
                              rw.wd * rw.wd + rw.wu * rw.wu);
            }
            KS[p] = kn;
        }
        U[q] = v;
    }
    __syncthreads();
    const int a5 = (((-2 * j) % 5) + 5) % 5;
    for (int s = 0; s < sweeps; ++s) {
#pragma unroll 1
        for (int c = 0; c < 5; ++c) {
            // the slot's cell of colour c: r = (c - 2 j) mod 5
            const int r = c + a5 >= 5 ? c + a5 - 5 : c + a5;
            const int i = 5 * t + r;
            if (slot && i <= N) {
                C<double> fp = fr[0];
#pragma unroll
                for (int q = 1; q < 5; ++q)
                    if (q == r) fp = fr[q];
                const C<double> kp = KS[j * M + i];
                kacz_row_lds(U, (j + 1) * pw + i + 1, pw, row_at<double>(i, j, N, H, ih2, kp.x, sig), fp, kp.y);
            }
            __syncthreads();
        }
    }
    for (int q = tid; q < M * M; q += LNT) {
        const int i = q % M, jq = q / M;
        uo[q] = st_as<T>(U[(jq + 1) * pw + i + 1]);
    }
    if (!fc) return;
    // residual with sigma_b at the slot's cells (kept in registers until every
    // thread has read the table), stored over the table, then full weighting
    C<double> res[5];
    if (slot) {
#pragma unroll
        for (int r = 0; r < 5; ++r) {
            const int i = 5 * t + r;
            if (i > N) continue;
            const int l = (j + 1) * pw + i + 1;
            Row<double> rw = row_at<double>(i, j, N, H, ih2, KS[j * M + i].x, sigb);
            res[r] = csub(fr[r], cadd(cmul(cmk(rw.dre, rw.dim), U[l]), offsum_z(rw, U, l, pw)));
        }
    }
    __syncthreads();
    if (slot) {
#pragma unroll
        for (int r = 0; r < 5; ++r)
            if (5 * t + r <= N) KS[j * M + 5 * t + r] = res[r];
    }
    __syncthreads();
    for (int q = tid; q < Mc * Mc; q += LNT) {
        const int I = q % Mc, J = q / Mc;
        C<double> sum = cmk(0.0, 0.0);
        for (int e = -1; e <= 1; ++e) {
            const int jj = mirror(2 * J + e, N);
            for (int d = -1; d <= 1; ++d) {
                const int ii = mirror(2 * I + d, N);
                const double w = (double)((2 - (d < 0 ? -d : d)) * (2 - (e < 0 ? -e : e)));
                sum = cadd(sum, cscale(w, KS[jj * M + ii]));
            }
        }
        fc[q] = st_as<T>(cscale(0.0625, sum));
    }
}

// (k_p, 1 / ||a_p||^2) of the rows of A_sigma on a level: fixed for a grid,
// formed once for each Kaczmarz level and read by k_kacz_tb.
template <typename T>
__global__ __launch_bounds__(NT) void k_kacz_table(GeoT g, double H, double ih2, const T *__restrict__ k,
                                                   double sig, C<double> *__restrict__ tab) {
    const size_t p = (size_t)blockIdx.x * NT + threadIdx.x;
    if (p >= (size_t)g.M * g.M) return;
    const int i = (int)(p % g.M), j = (int)(p / g.M);
    const double kp = (double)k[p];
    Row<double> r = row_at<double>(i, j, g.N, H, ih2, kp, sig);
    double nrm = r.dre * r.dre + r.dim * r.dim + r.wl * r.wl + r.wr * r.wr + r.wd * r.wd + r.wu * r.wu;
    tab[p] = cmk(kp, 1.0 / nrm);
}

// ===========================================================================
// k_bottom: the V-cycle on levels lb..L-1 (n <= 31) in one workgroup of BNT
// threads.  Every field of every bottom level (u, f and k) lives in LDS, so
// the dependent colour passes never wait on global memory; only the first
// level's f (input), the coarsest inverse and the output touch it.  The
// iterates are stored with a ring of zero cells around the domain (row
// length M + 2), so the stencil rows read and write their cells without
// tests; the inverse's entries used by a thread are loaded into registers at
// the start and arrive while the down leg runs.
// ===========================================================================
constexpr int BNT = 256;
constexpr int BOT_C_ELEMS = 4096;     // complex slots (u and f of every level)
constexpr int BOT_K_ELEMS = 4096;     // real slots (k and a reciprocal of every level)
constexpr int CPARTS = 3;             // threads per row of the coarsest solve
constexpr int CPRE = 27;              // inverse entries a thread keeps in registers

template <typename T>
struct BotLevel {
    int n, M, N;
    double H, ih2, sa, sb;
    const T *k;
    int sm, pre, post;
    int uoff, foff, koff;
};

template <typename T>
struct BotPlan {
    int nlev;
    BotLevel<T> L[BOT_MAXL];
    const C<double> *ainv;
};

// padded position of node (i, j) of a level with M nodes per line
__device__ __forceinline__ int bpad(int i, int j, int M) { return (j + 1) * (M + 2) + i + 1; }

// K holds k of the level followed by IV: 1 / |a_pp|^2 (Gauss-Seidel levels)
// or 1 / ||a_p||^2 (Kaczmarz levels), computed once per launch.
template <typename T>
__device__ void bot_relax(const BotLevel<T> &L, C<double> *SM, const double *KS, int sweeps, bool zero) {
    const int tid = threadIdx.x, M = L.M, N = L.N, MM = M * M, PW = M + 2;
    C<double> *U = SM + L.uoff;
    const C<double> *F = SM + L.foff;
    const double *K = KS + L.koff;
    const double *IV = K + MM;
    if (zero && (L.sm != HMG_SM_GS_DEV || sweeps == 0)) {
        for (int p = tid; p < PW * PW; p += BNT) U[p] = cmk(0.0, 0.0);
        __syncthreads();
    }
    if (L.sm == HMG_SM_GS_DEV) {
        for (int s = 0; s < sweeps; ++s)
            for (int colour = 0; colour < 2; ++colour) {
                bool zg = zero && s == 0 && colour == 0;
                for (int p = tid; p < MM; p += BNT) {
                    int i = p % M, j = p / M;
                    if (((i + j) & 1) != colour) continue;
                    const int l = bpad(i, j, M);
                    Row<double> r = row_at<double>(i, j, N, L.H, L.ih2, K[p], L.sa);
                    C<double> num = F[p];
                    if (!zg) num = csub(num, offsum_z(r, U, l, PW));
                    const double inv = IV[p];
                    U[l] = cmk((num.x * r.dre + num.y * r.dim) * inv, (num.y * r.dre - num.x * r.dim) * inv);
                }
                __syncthreads();
            }
    } else {
        const int W5 = (M + 4) / 5;
        // fixed row slots: q = tid + BNT m -> line j = q / W5, column slot
        // 5 (q % W5); computed once, not per pass
        constexpr int BM = 2;     // M * W5 <= 33 * 7 < BM * BNT on bottom levels
        int qj[BM], q5[BM];
#pragma unroll
        for (int m = 0; m < BM; ++m) {
            int q = tid + BNT * m;
            qj[m] = (q < M * W5) ? q / W5 : -1;
            q5[m] = 5 * (q % W5);
        }
        for (int s = 0; s < sweeps; ++s)
            for (int c = 0; c < 5; ++c) {
#pragma unroll
                for (int m = 0; m < BM; ++m) {
                    const int j = qj[m];
                    if (j < 0) continue;
                    const int i = ((c - 2 * j) % 5 + 5) % 5 + q5[m];
                    if (i > N) continue;
                    const int p = j * M + i;
                    kacz_row_lds(U, bpad(i, j, M), PW, row_at<double>(i, j, N, L.H, L.ih2, K[p], L.sa), F[p],
                                 IV[p]);
                }
                __syncthreads();
            }
    }
}

// BASIS: workgroup b runs the cycle on the unit vector e_b and writes the
// result as column b of the row-major matrix uo (m x m, m = M^2 of the first
// bottom level): the cycle from a zero guess is linear in f, so these columns
// form the matrix of the whole bottom cycle.
template <typename T, typename TF, typename TU, bool BASIS>
__global__ __launch_bounds__(BNT) void k_bottom(BotPlan<T> P, const C<TF> *__restrict__ fg, C<TU> *__restrict__ uo,
                                                const int *skip) {
    if (skip && *skip) return;
    __shared__ C<double> SM[BOT_C_ELEMS];
    __shared__ double KS[BOT_K_ELEMS];
    // level parameters are indexed at run time: keep them in LDS, not in
    // (spilled) registers
    __shared__ BotLevel<T> PL[BOT_MAXL];
    const int tid = threadIdx.x;
    const int last = P.nlev - 1;
    // this thread's share of the coarsest solve: row cr, columns
    // [c0, c0 + CPRE) of the inverse (column-major), requested first
    const int mco = P.L[last].M * P.L[last].M;
    const int chunk = (mco + CPARTS - 1) / CPARTS;
    const int cr = tid % (BNT / CPARTS), cpart = tid / (BNT / CPARTS);
    const int cc0 = min(cpart, CPARTS - 1) * chunk;
    const bool cpre = chunk <= CPRE;
    C<double> ainv_r[CPRE];
    if (cpre) {
#pragma unroll
        for (int t = 0; t < CPRE; ++t) {
            const int c = min(cc0 + t, mco - 1), r = min(cr, mco - 1);
            ainv_r[t] = P.ainv[(size_t)c * mco + r];
        }
    }
    if (tid < P.nlev) PL[tid] = P.L[tid];
    for (int q = tid; q < BOT_C_ELEMS; q += BNT) SM[q] = cmk(0.0, 0.0);
    __syncthreads();
    // stage k of every level, the reciprocals of the relaxation rows and the
    // first level's f
    for (int l = 0; l <= last; ++l) {
        const BotLevel<T> &L = PL[l];
        const int MM = L.M * L.M;
        for (int p = tid; p < MM; p += BNT) {
            double kp = (double)L.k[p];
            KS[L.koff + p] = kp;
            Row<double> r = row_at<double>(p % L.M, p / L.M, L.N, L.H, L.ih2, kp, L.sa);
            double d2 = r.dre * r.dre + r.dim * r.dim;
            if (L.sm != HMG_SM_GS_DEV) d2 += r.wl * r.wl + r.wr * r.wr + r.wd * r.wd + r.wu * r.wu;
            KS[L.koff + MM + p] = 1.0 / d2;
        }
    }
    for (int p = tid; p < PL[0].M * PL[0].M; p += BNT)
        SM[PL[0].foff + p] = BASIS ? cmk(p == (int)blockIdx.x ? 1.0 : 0.0, 0.0) : ldr<double>(fg, p);
    __syncthreads();
    // down: pre-relaxation, residual, full weighting into the next f
    for (int l = 0; l < last; ++l) {
        const BotLevel<T> &L = PL[l];
        bot_relax<T>(L, SM, KS, L.pre, true);
        const BotLevel<T> &Cl = PL[l + 1];
        const C<double> *U = SM + L.uoff;
        const C<double> *F = SM + L.foff;
        const double *K = KS + L.koff;
        const int PW = L.M + 2;
        for (int qc = tid; qc < Cl.M * Cl.M; qc += BNT) {
            int I = qc % Cl.M, J = qc / Cl.M;
            C<double> s = cmk(0.0, 0.0);
            for (int e = -1; e <= 1; ++e) {
                int j = mirror(2 * J + e, L.N);
                for (int d = -1; d <= 1; ++d) {
                    int i = mirror(2 * I + d, L.N);
                    int p = j * L.M + i, l2 = bpad(i, j, L.M);
                    Row<double> r = row_at<double>(i, j, L.N, L.H, L.ih2, K[p], L.sb);
                    C<double> res = csub(F[p], cadd(cmul(cmk(r.dre, r.dim), U[l2]), offsum_z(r, U, l2, PW)));
                    double w = (double)((2 - (d < 0 ? -d : d)) * (2 - (e < 0 ? -e : e)));
                    s = cadd(s, cscale(w, res));
                }
            }
            SM[Cl.foff + qc] = cscale(0.0625, s);
        }
        __syncthreads();
    }
    // coarsest: u = A^{-1} f in FP64; row r is split over CPARTS threads
    // (column ranges), partial sums combined in a fixed order
    {
        __shared__ C<double> part[CPARTS][BNT / CPARTS];
        const BotLevel<T> &L = PL[last];
        const int m = mco;
        const C<double> *F = SM + L.foff;
        for (int base = 0; base < m; base += BNT / CPARTS) {
            const int r = base + cr;
            if (cpart < CPARTS) {
                C<double> acc = cmk(0.0, 0.0);
                if (r < m) {
                    const int c1 = min(m, cc0 + chunk);
                    if (cpre && base == 0) {
#pragma unroll
                        for (int t = 0; t < CPRE; ++t)
                            if (cc0 + t < c1) acc = cadd(acc, cmul(ainv_r[t], F[cc0 + t]));
                    } else {
                        for (int c = cc0; c < c1; ++c) acc = cadd(acc, cmul(P.ainv[(size_t)c * m + r], F[c]));
                    }
                }
                part[cpart][cr] = acc;
            }
            __syncthreads();
            if (tid < BNT / CPARTS && base + tid < m) {
                C<double> acc = part[0][tid];
                for (int q = 1; q < CPARTS; ++q) acc = cadd(acc, part[q][tid]);
                const int rr = base + tid;
                SM[L.uoff + bpad(rr % L.M, rr / L.M, L.M)] = acc;
            }
            __syncthreads();
        }
    }
    // up: bilinear correction, post-relaxation
    for (int l = last - 1; l >= 0; --l) {
        const BotLevel<T> &L = PL[l];
        const BotLevel<T> &Cl = PL[l + 1];
        C<double> *U = SM + L.uoff;
        const C<double> *E = SM + Cl.uoff;
        const int PWc = Cl.M + 2;
        for (int p = tid; p < L.M * L.M; p += BNT) {
            const int i = p % L.M, j = p / L.M;
            const int qc = bpad(i >> 1, j >> 1, Cl.M);   // coarse (I, J); its right and upper
                                                          // neighbours may be zero ring cells
            const int l2 = bpad(i, j, L.M);
            U[l2] = cadd(U[l2], bilinear(E[qc], E[qc + 1], E[qc + PWc], E[qc + PWc + 1], i, j));
        }
        __syncthreads();
        bot_relax<T>(L, SM, KS, L.post, false);
    }
    const BotLevel<T> &L0 = PL[0];
    const int m0 = L0.M * L0.M;
    for (int p = tid; p < m0; p += BNT) {
        const C<double> v = SM[L0.uoff + bpad(p % L0.M, p / L0.M, L0.M)];
        if (BASIS) uo[(size_t)p * m0 + blockIdx.x] = st_as<TU>(v);
        else uo[p] = st_as<TU>(v);
    }
}

// ===========================================================================
// k_dense_apply: u = B f for the dense bottom-cycle matrix B (row-major,
// complex FP64, m <= DMAX).  One workgroup per row: thread t takes columns
// t, t + DNT, ... (all of its loads issued together), then a fixed-order
// wave butterfly and a fixed-order sum over the waves.  f is read straight
// from memory (every workgroup reads the same m values, which stay in L2).
// ===========================================================================
constexpr int DNT = 256, DMAX = 33 * 33, DPT = (DMAX + DNT - 1) / DNT;

template <typename TF, typename TU>
__global__ __launch_bounds__(DNT) void k_dense_apply(const C<double> *__restrict__ B, int m,
                                                     const C<TF> *__restrict__ f, C<TU> *__restrict__ u,
                                                     const int *skip, long zs) {
    f = zsh(f, zs);
    u = zsh(u, zs);
    skip = zsh(skip, zs);
    const int sk = flag_read(skip);
    __shared__ double part[2][DNT / 64];
    const int tid = threadIdx.x, r = blockIdx.x;
    const C<double> *row = B + (size_t)r * m;
    C<double> b[DPT], x[DPT];
#pragma unroll
    for (int q = 0; q < DPT; ++q) {
        const int c = min(tid + DNT * q, m - 1);
        b[q] = row[c];
        x[q] = ldr<double>(f, c);
    }
    if (flag_set(sk)) return;
    double ax = 0.0, ay = 0.0;
#pragma unroll
    for (int q = 0; q < DPT; ++q) {
        if (tid + DNT * q >= m) continue;
        ax += b[q].x * x[q].x - b[q].y * x[q].y;
        ay += b[q].x * x[q].y + b[q].y * x[q].x;
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        ax += __shfl_xor(ax, off, 64);
        ay += __shfl_xor(ay, off, 64);
    }
    if ((tid & 63) == 0) {
        part[0][tid >> 6] = ax;
        part[1][tid >> 6] = ay;
    }
    __syncthreads();
    if (tid == 0) {
        double sx = part[0][0], sy = part[1][0];
        for (int w = 1; w < DNT / 64; ++w) {
            sx += part[0][w];
            sy += part[1][w];
        }
        u[r] = st_as<TU>(cmk(sx, sy));
    }
}

// ===========================================================================
// launchers
// ===========================================================================
static inline GeoT geo_t(const Geo &g) { return GeoT{g.n, g.M, g.N}; }

// the small tile when the large one would give fewer than two workgroups per CU
static bool gs_small(const Geo &g) {
    return (size_t)((g.M + GsBig::X - 1) / GsBig::X) * ((g.M + GsBig::Y - 1) / GsBig::Y) < 512;
}
static bool gs_tiny(const Geo &g) {
    return (size_t)((g.M + GsSmall::X - 1) / GsSmall::X) * ((g.M + GsSmall::Y - 1) / GsSmall::Y) < 1024;
}

template <class TL>
static dim3 gs_grid(const Geo &g, int nz = 1) {
    return dim3((g.M + TL::X - 1) / TL::X, (g.M + TL::Y - 1) / TL::Y, nz);
}

template <typename T, typename TF>
static void gs_down_t(hipStream_t s, const Geo &g, const void *k, double sa, double sb, const void *f, void *uo,
                      void *fc, bool uo_black, const int *skip, Bz bz) {
    if (gs_tiny(g))
        k_gs_down<GsTiny, T, TF><<<gs_grid<GsTiny>(g, bz.nz), GNT, 0, s>>>(
            geo_t(g), g.H, 1.0 / (g.H * g.H), (const T *)k, sa, sb, (const C<TF> *)f, (C<T> *)uo, (C<T> *)fc,
            uo_black ? 1 : 0, skip, bz.zs);
    else if (gs_small(g))
        k_gs_down<GsSmall, T, TF><<<gs_grid<GsSmall>(g, bz.nz), GNT, 0, s>>>(
            geo_t(g), g.H, 1.0 / (g.H * g.H), (const T *)k, sa, sb, (const C<TF> *)f, (C<T> *)uo, (C<T> *)fc,
            uo_black ? 1 : 0, skip, bz.zs);
    else
        k_gs_down<GsDownBig, T, TF><<<gs_grid<GsDownBig>(g, bz.nz), GNT, 0, s>>>(
            geo_t(g), g.H, 1.0 / (g.H * g.H), (const T *)k, sa, sb, (const C<TF> *)f, (C<T> *)uo, (C<T> *)fc,
            uo_black ? 1 : 0, skip, bz.zs);
}

void launch_gs_down(Prec p, bool f64in, hipStream_t s, const Geo &g, const void *k, double sa, double sb,
                    const void *f, void *uo, void *fc, const int *skip, bool uo_black, Bz bz) {
    if (p == P64) gs_down_t<double, double>(s, g, k, sa, sb, f, uo, fc, uo_black, skip, bz);
    else if (f64in) gs_down_t<float, double>(s, g, k, sa, sb, f, uo, fc, uo_black, skip, bz);
    else gs_down_t<float, float>(s, g, k, sa, sb, f, uo, fc, uo_black, skip, bz);
}

template <typename T, typename TF, typename TU>
static void gs_up_t(hipStream_t s, const Geo &g, const void *k, double sa, const void *f, const void *u0,
                    const void *ec, void *uo, const int *skip, Bz bz) {
    const double ih2 = 1.0 / (g.H * g.H);
    if (u0) {
        if (gs_tiny(g))
            k_gs_up_u0<GsTiny2, T, TF, TU><<<gs_grid<GsTiny2>(g, bz.nz), GNT, 0, s>>>(
                geo_t(g), g.H, ih2, (const T *)k, sa, (const C<TF> *)f, (const C<T> *)u0, (const C<T> *)ec,
                (C<TU> *)uo, skip, bz.zs);
        else if (gs_small(g))
            k_gs_up_u0<GsSmall2, T, TF, TU><<<gs_grid<GsSmall2>(g, bz.nz), GNT, 0, s>>>(
                geo_t(g), g.H, ih2, (const T *)k, sa, (const C<TF> *)f, (const C<T> *)u0, (const C<T> *)ec,
                (C<TU> *)uo, skip, bz.zs);
        else
            k_gs_up_u0<GsBig2, T, TF, TU><<<gs_grid<GsBig2>(g, bz.nz), GNT, 0, s>>>(
                geo_t(g), g.H, ih2, (const T *)k, sa, (const C<TF> *)f, (const C<T> *)u0, (const C<T> *)ec,
                (C<TU> *)uo, skip, bz.zs);
        return;
    }
    if (gs_tiny(g))
        k_gs_up<GsTiny, T, TF, TU><<<gs_grid<GsTiny>(g, bz.nz), GNT, 0, s>>>(
            geo_t(g), g.H, 1.0 / (g.H * g.H), (const T *)k, sa, (const C<TF> *)f, (const C<T> *)ec, (C<TU> *)uo, skip,
            bz.zs);
    else if (gs_small(g))
        k_gs_up<GsSmall, T, TF, TU><<<gs_grid<GsSmall>(g, bz.nz), GNT, 0, s>>>(
            geo_t(g), g.H, 1.0 / (g.H * g.H), (const T *)k, sa, (const C<TF> *)f, (const C<T> *)ec, (C<TU> *)uo, skip,
            bz.zs);
    else
        k_gs_up<GsBig, T, TF, TU><<<gs_grid<GsBig>(g, bz.nz), GNT, 0, s>>>(
            geo_t(g), g.H, 1.0 / (g.H * g.H), (const T *)k, sa, (const C<TF> *)f, (const C<T> *)ec, (C<TU> *)uo, skip,
            bz.zs);
}

bool gs_up_mv_ok(Prec p, const Geo &g) { return p == P64 && !gs_small(g) && g.n > 511; }
int gs_up_mv_blocks(const Geo &g) {
    const dim3 tg = gs_grid<GsBigMV>(g);
    return (int)(tg.x * tg.y);
}
void launch_gs_up_mv(hipStream_t s, int kind, const Geo &g, const void *k, double sa, const void *f,
                     const void *ec, void *uo, void *mvo, const void *dot, double *partials, const int *skip,
                     Bz bz) {
    const double ih2 = 1.0 / (g.H * g.H);
    if (kind == 1)
        k_gs_up_mv<1><<<gs_grid<GsBigMV>(g, bz.nz), GNT, 0, s>>>(
            geo_t(g), g.H, ih2, (const double *)k, sa, (const C<double> *)f, (const C<double> *)ec,
            (C<double> *)uo, (C<double> *)mvo, (const C<double> *)dot, partials, skip, bz.zs);
    else
        k_gs_up_mv<2><<<gs_grid<GsBigMV>(g, bz.nz), GNT, 0, s>>>(
            geo_t(g), g.H, ih2, (const double *)k, sa, (const C<double> *)f, (const C<double> *)ec,
            (C<double> *)uo, (C<double> *)mvo, (const C<double> *)dot, partials, skip, bz.zs);
}

void launch_gs_up(Prec p, bool io64, hipStream_t s, const Geo &g, const void *k, double sa, const void *f,
                  const void *u0, const void *ec, void *uo, const int *skip, Bz bz) {
    if (p == P64) gs_up_t<double, double, double>(s, g, k, sa, f, u0, ec, uo, skip, bz);
    else if (io64) gs_up_t<float, double, double>(s, g, k, sa, f, u0, ec, uo, skip, bz);
    else gs_up_t<float, float, float>(s, g, k, sa, f, u0, ec, uo, skip, bz);
}

template <typename T, int TS, int S, int NT, int TY = TS>
static void kacz_tb_t(hipStream_t s, const Geo &g, const void *k, const double *tab, double sig, const void *f,
                      const void *ui, const void *ec, void *uo, const int *skip, Bz bz) {
    dim3 grid((g.M + TS - 1) / TS, (g.M + TY - 1) / TY, bz.nz);
    k_kacz_tb<T, TS, S, NT, false, TY><<<grid, NT, 0, s>>>(geo_t(g), g.H, 1.0 / (g.H * g.H), (const T *)k,
                                                       (const C<double> *)tab, sig, 0.0, (const C<T> *)f,
                                                       (const C<T> *)ui, (const C<T> *)ec, (C<T> *)uo, nullptr,
                                                       skip, bz.zs);
}

// the RESID form of a configuration: tile TS - 4, halo 10 S + 2
template <typename T, int TS, int S, int NT, int TY = TS>
static void kacz_tb_resid_t(hipStream_t s, const Geo &g, const void *k, const double *tab, double sig, double sigb,
                            const void *f, const void *ui, void *uo, void *fc, const int *skip, Bz bz) {
    constexpr int T4 = TS - 4, Y4 = TY - 4;
    dim3 grid((g.M + T4 - 1) / T4, (g.M + Y4 - 1) / Y4, bz.nz);
    k_kacz_tb<T, TS, S, NT, true, TY><<<grid, NT, 0, s>>>(geo_t(g), g.H, 1.0 / (g.H * g.H), (const T *)k,
                                                      (const C<double> *)tab, sig, sigb, (const C<T> *)f,
                                                      (const C<T> *)ui, nullptr, (C<T> *)uo, (C<T> *)fc, skip,
                                                      bz.zs);
}

// Tile configurations offered to the tuner: (tile width, sweeps per launch,
// threads per workgroup, tile height, tile height of the RESID launch before
// its shrink by four).  The last one halves the tile height: about 20 % fewer
// rows per colour pass and workgroup at the price of more workgroups (153
// instead of 81 at n = 127), which the latency-bound passes favour.
const KaczCfg kKaczCfgs[KACZ_NCFG] = {{32, 1, 512, 32, 32},  {32, 2, 1024, 32, 32}, {16, 2, 512, 16, 16},
                                      {16, 4, 1024, 16, 16}, {16, 2, 1024, 16, 16}, {16, 1, 512, 16, 16},
                                      {32, 1, 1024, 32, 32}, {16, 2, 1024, 8, 12}};

// The LDS tile holds FP64 values in either storage precision.
bool kacz_cfg_fits(Prec, int cfg) {
    const KaczCfg &c = kKaczCfgs[cfg];
    int lw = c.ts + 20 * c.sweeps, lh = c.ty + 20 * c.sweeps;
    return (size_t)lw * lh * 16 <= 160 * 1024;
}

template <typename T>
static void kacz_tb_any(int cfg, hipStream_t s, const Geo &g, const void *k, const double *tab, double sig,
                        const void *f, const void *ui, const void *ec, void *uo, const int *skip, Bz bz) {
    switch (cfg) {
    case 0: kacz_tb_t<T, 32, 1, 512>(s, g, k, tab, sig, f, ui, ec, uo, skip, bz); break;
    case 1: kacz_tb_t<T, 32, 2, 1024>(s, g, k, tab, sig, f, ui, ec, uo, skip, bz); break;
    case 2: kacz_tb_t<T, 16, 2, 512>(s, g, k, tab, sig, f, ui, ec, uo, skip, bz); break;
    case 3: kacz_tb_t<T, 16, 4, 1024>(s, g, k, tab, sig, f, ui, ec, uo, skip, bz); break;
    case 4: kacz_tb_t<T, 16, 2, 1024>(s, g, k, tab, sig, f, ui, ec, uo, skip, bz); break;
    case 5: kacz_tb_t<T, 16, 1, 512>(s, g, k, tab, sig, f, ui, ec, uo, skip, bz); break;
    case 7: kacz_tb_t<T, 16, 2, 1024, 8>(s, g, k, tab, sig, f, ui, ec, uo, skip, bz); break;
    default: kacz_tb_t<T, 32, 1, 1024>(s, g, k, tab, sig, f, ui, ec, uo, skip, bz); break;
    }
}

void launch_kacz_tb(Prec p, int cfg, hipStream_t s, const Geo &g, const void *k, const double *tab, double sig,
                    const void *f, const void *ui, const void *ec, void *uo, const int *skip, Bz bz) {
    if (p == P64) kacz_tb_any<double>(cfg, s, g, k, tab, sig, f, ui, ec, uo, skip, bz);
    else kacz_tb_any<float>(cfg, s, g, k, tab, sig, f, ui, ec, uo, skip, bz);
}

bool kacz_level_fits(const Geo &g) { return g.M <= LMAX; }

void launch_kacz_level(Prec p, hipStream_t s, const Geo &g, const void *k, const double *tab, double sig,
                       double sigb, int sweeps, const void *f, const void *ui, const void *ec, void *uo, void *fc,
                       const int *skip) {
    const double ih2 = 1.0 / (g.H * g.H);
    if (p == P64)
        k_kacz_level<double><<<1, LNT, 0, s>>>(geo_t(g), g.H, ih2, (const double *)k, (const C<double> *)tab, sig,
                                               sigb, sweeps, (const C<double> *)f, (const C<double> *)ui,
                                               (const C<double> *)ec, (C<double> *)uo, (C<double> *)fc, skip);
    else
        k_kacz_level<float><<<1, LNT, 0, s>>>(geo_t(g), g.H, ih2, (const float *)k, (const C<double> *)tab, sig,
                                              sigb, sweeps, (const C<float> *)f, (const C<float> *)ui,
                                              (const C<float> *)ec, (C<float> *)uo, (C<float> *)fc, skip);
}

void launch_kacz_table(Prec p, hipStream_t s, const Geo &g, const void *k, double sig, double *tab) {
    const unsigned nb = (unsigned)(((size_t)g.M * g.M + NT - 1) / NT);
    if (p == P64)
        k_kacz_table<double><<<nb, NT, 0, s>>>(geo_t(g), g.H, 1.0 / (g.H * g.H), (const double *)k, sig,
                                                (C<double> *)tab);
    else
        k_kacz_table<float><<<nb, NT, 0, s>>>(geo_t(g), g.H, 1.0 / (g.H * g.H), (const float *)k, sig,
                                               (C<double> *)tab);
}

// Configurations whose region is staged in LDS have a RESID form.
bool kacz_cfg_resid(int cfg) {
    const KaczCfg &c = kKaczCfgs[cfg];
    int lw = c.ts + 20 * c.sweeps, lh = c.rty + 20 * c.sweeps;
    return (size_t)lw * lh * 48 <= 160 * 1024;
}

template <typename T>
static void kacz_resid_any(int cfg, hipStream_t s, const Geo &g, const void *k, const double *tab, double sig,
                           double sigb, const void *f, const void *ui, void *uo, void *fc, const int *skip, Bz bz) {
    switch (cfg) {
    case 0: kacz_tb_resid_t<T, 32, 1, 512>(s, g, k, tab, sig, sigb, f, ui, uo, fc, skip, bz); break;
    case 2: kacz_tb_resid_t<T, 16, 2, 512>(s, g, k, tab, sig, sigb, f, ui, uo, fc, skip, bz); break;
    case 4: kacz_tb_resid_t<T, 16, 2, 1024>(s, g, k, tab, sig, sigb, f, ui, uo, fc, skip, bz); break;
    case 5: kacz_tb_resid_t<T, 16, 1, 512>(s, g, k, tab, sig, sigb, f, ui, uo, fc, skip, bz); break;
    case 7: kacz_tb_resid_t<T, 16, 2, 1024, 12>(s, g, k, tab, sig, sigb, f, ui, uo, fc, skip, bz); break;
    default: kacz_tb_resid_t<T, 32, 1, 1024>(s, g, k, tab, sig, sigb, f, ui, uo, fc, skip, bz); break;
    }
}

void launch_kacz_tb_resid(Prec p, int cfg, hipStream_t s, const Geo &g, const void *k, const double *tab,
                          double sig, double sigb, const void *f, const void *ui, void *uo, void *fc,
                          const int *skip, Bz bz) {
    if (p == P64) kacz_resid_any<double>(cfg, s, g, k, tab, sig, sigb, f, ui, uo, fc, skip, bz);
    else kacz_resid_any<float>(cfg, s, g, k, tab, sig, sigb, f, ui, uo, fc, skip, bz);
}

int bottom_complex_slots() { return BOT_C_ELEMS; }
int bottom_real_slots() { return BOT_K_ELEMS; }

template <typename T>
static BotPlan<T> bot_plan(const BottomDesc &d) {
    BotPlan<T> P;
    P.nlev = d.nlev;
    P.ainv = (const C<double> *)d.ainv_t;
    for (int l = 0; l < d.nlev; ++l) {
        BotLevel<T> &L = P.L[l];
        const BottomLevelDesc &D = d.L[l];
        L.n = D.n;
        L.M = D.n + 2;
        L.N = D.n + 1;
        L.H = D.H;
        L.ih2 = 1.0 / (D.H * D.H);
        L.sa = D.sa;
        L.sb = D.sb;
        L.k = (const T *)D.k;
        L.sm = D.sm;
        L.pre = D.pre;
        L.post = D.post;
        L.uoff = D.uoff;
        L.foff = D.foff;
        L.koff = D.koff;
    }
    return P;
}

template <typename T, typename TF, typename TU>
static void bottom_t(hipStream_t s, const BottomDesc &d, const void *f, void *uo, const int *skip) {
    k_bottom<T, TF, TU, false><<<1, BNT, 0, s>>>(bot_plan<T>(d), (const C<TF> *)f, (C<TU> *)uo, skip);
}

int bottom_matrix_size(const BottomDesc &d) { return (d.L[0].n + 2) * (d.L[0].n + 2); }

// The matrix of the bottom cycle (row-major complex FP64, m x m), one
// workgroup per column.
void launch_bottom_basis(Prec p, hipStream_t s, const BottomDesc &d, double *B) {
    const int m = bottom_matrix_size(d);
    if (p == P64)
        k_bottom<double, double, double, true><<<m, BNT, 0, s>>>(bot_plan<double>(d), nullptr, (C<double> *)B,
                                                                 nullptr);
    else
        k_bottom<float, double, double, true><<<m, BNT, 0, s>>>(bot_plan<float>(d), nullptr, (C<double> *)B,
                                                                nullptr);
}

void launch_dense_apply(Prec p, bool io64, hipStream_t s, const double *B, int m, const void *f, void *u,
                        const int *skip, Bz bz) {
    dim3 grid(m, 1, bz.nz);
    const C<double> *b = (const C<double> *)B;
    if (p == P64 || io64)
        k_dense_apply<double, double><<<grid, DNT, 0, s>>>(b, m, (const C<double> *)f, (C<double> *)u, skip, bz.zs);
    else
        k_dense_apply<float, float><<<grid, DNT, 0, s>>>(b, m, (const C<float> *)f, (C<float> *)u, skip, bz.zs);
}

void launch_bottom(Prec p, bool io64, hipStream_t s, const BottomDesc &d, const void *f, void *uo, const int *skip) {
    if (p == P64) bottom_t<double, double, double>(s, d, f, uo, skip);
    else if (io64) bottom_t<float, double, double>(s, d, f, uo, skip);
    else bottom_t<float, float, float>(s, d, f, uo, skip);
}

}  // namespace hmgk
