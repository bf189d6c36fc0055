// hmg_fused.hip -- fused, LDS-tiled V-cycle kernels for gfx950.
//
// Each kernel performs the same per-node arithmetic as the one-pass kernels
// of hmg_kernels.hip, in the same order (FP64 arithmetic on fields stored in
// the level precision; the LDS tiles hold FP64 values), but stages a tile of
// the level plus a halo in LDS so that one launch does several dependent
// steps and every field is read from and written to HBM once:
//
//   k_gs_down    zero-guess red-black Gauss-Seidel sweep (role A operator),
//                residual (role B operator) and full weighting to the next
//                coarser level (Section 5: pre-smoothing and restriction);
//                the smoothed iterate stays on chip;
//   k_gs_up      recomputes that iterate (it depends on f only), adds the
//                bilinear correction from the coarser level and does one
//                red-black sweep (Section 5: prolongation and post-smoothing);
//   k_kacz_tb    S sweeps of 5-colour Kaczmarz relaxation on a tile with a
//                halo of 10 S nodes (each colour pass moves information two
//                nodes), optionally starting from zero or from u + P e;
//   k_bottom     one workgroup runs the whole V-cycle on the small levels
//                (relaxation, transfers and the dense coarsest solve) with
//                the iterates resident in LDS.
//
// A tile's workgroup writes only its own nodes and reads its halo from the
// input arrays, which no workgroup of the same launch writes.

#include "hmg_device.h"

namespace hmgk {

// sum_{q != p} a_pq U_q for an LDS array with row length LW (node p at l)
template <typename T>
__device__ __forceinline__ C<T> offsum_l(const Row<T> &r, const C<T> *U, int l, int LW, int i, int j, int N) {
    C<T> s = cmk(T(0), T(0));
    if (i > 0) s = cadd(s, cscale(r.wl, U[l - 1]));
    if (i < N) s = cadd(s, cscale(r.wr, U[l + 1]));
    if (j > 0) s = cadd(s, cscale(r.wd, U[l - LW]));
    if (j < N) s = cadd(s, cscale(r.wu, U[l + LW]));
    return s;
}

// bilinear interpolation of the coarse correction at fine node (i, j)
template <typename T>
__device__ __forceinline__ C<double> prolong_at(const C<T> *ec, int i, int j, int Mc) {
    int I = i >> 1, J = j >> 1;
    size_t q = (size_t)J * Mc + I;
    if (!(i & 1) && !(j & 1)) return ldr<double>(ec, q);
    if ((i & 1) && !(j & 1)) return cscale(0.5, cadd(ldr<double>(ec, q), ldr<double>(ec, q + 1)));
    if (!(i & 1) && (j & 1)) return cscale(0.5, cadd(ldr<double>(ec, q), ldr<double>(ec, q + Mc)));
    return cscale(0.25, cadd(cadd(cadd(ldr<double>(ec, q), ldr<double>(ec, q + 1)), ldr<double>(ec, q + Mc)),
                             ldr<double>(ec, q + Mc + 1)));
}

__device__ __forceinline__ int mirror(int x, int N) { return x < 0 ? -x : (x > N ? 2 * N - x : x); }

// ===========================================================================
// Fused Gauss-Seidel kernels.  A tile of GDX x GDY fine nodes (x0, y0 even)
// is processed with a halo of RH = 3 held in LDS.  Each thread owns fixed
// red and black nodes of the haloed region (colour-compressed: node q of a
// colour maps to line q / HW, every other column), loads their f and k once,
// all loads in flight together, and keeps them in registers across the
// dependent phases, which then touch only LDS.
// ===========================================================================
constexpr int GDX = 64, GDY = 20, GNT = 256;
constexpr int GRH = 3, GLW = GDX + 2 * GRH, GLH = GDY + 2 * GRH;
constexpr int GHW = GLW / 2;                       // nodes of one colour per line
constexpr int GNC = GHW * GLH;                     // nodes of one colour in the region
constexpr int GNS = (GNC + GNT - 1) / GNT;         // owned nodes per colour per thread

// local coordinates of owned node (colour c, slot m) of thread tid
__device__ __forceinline__ bool gs_owned(int tid, int c, int m, int &lx, int &ly) {
    int q = tid + GNT * m;
    ly = q / GHW;
    lx = 2 * (q % GHW) + ((ly + c) & 1);            // red: (lx + ly) even
    return q < GNC;
}

// ring distance from the region border: node (lx, ly) is in tile + h iff
// lx >= GRH - h, lx < GLW - GRH + h, and the same for ly
__device__ __forceinline__ bool in_ring(int lx, int ly, int h) {
    return lx >= GRH - h && ly >= GRH - h && lx < GLW - GRH + h && ly < GLH - GRH + h;
}

// ===========================================================================
// k_gs_down: one zero-guess red-black sweep (sigma_A), residual (sigma_B) on
// tile + 1, full weighting to the coarse nodes of the tile.  The smoothed
// iterate stays on chip (written only when uo != null).
// ===========================================================================
template <typename T, typename TF>
__global__ __launch_bounds__(GNT) void k_gs_down(GeoT g, double H, double ih2, const T *__restrict__ k, double sa,
                                                 double sb, const C<TF> *__restrict__ f, C<T> *uo,
                                                 C<T> *__restrict__ fc, const int *skip) {
    if (skip && *skip) return;
    __shared__ C<double> U[GLW * GLH];      // the iterate, then the residual on tile + 1
    const int tid = threadIdx.x;
    const int x0 = blockIdx.x * GDX, y0 = blockIdx.y * GDY;
    const int ox = x0 - GRH, oy = y0 - GRH;
    const int N = g.N, M = g.M;
    C<double> fr[2][GNS];
    double kr[2][GNS];
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int m = 0; m < GNS; ++m) {
            int lx, ly;
            bool own = gs_owned(tid, c, m, lx, ly);
            int i = ox + lx, j = oy + ly;
            if (own && i >= 0 && j >= 0 && i <= N && j <= N) {
                size_t p = (size_t)j * M + i;
                fr[c][m] = ldr<double>(f, p);
                kr[c][m] = (double)k[p];
            }
        }
    // red on tile + 3 (zero guess: u = f / a_pp)
#pragma unroll
    for (int m = 0; m < GNS; ++m) {
        int lx, ly;
        bool own = gs_owned(tid, 0, m, lx, ly);
        int i = ox + lx, j = oy + ly;
        if (!own || i < 0 || j < 0 || i > N || j > N) continue;
        Row<double> r = row_at<double>(i, j, N, H, ih2, kr[0][m], sa);
        U[ly * GLW + lx] = cdiv(fr[0][m], r.dre, r.dim);
    }
    __syncthreads();
    // black on tile + 2
#pragma unroll
    for (int m = 0; m < GNS; ++m) {
        int lx, ly;
        bool own = gs_owned(tid, 1, m, lx, ly);
        int i = ox + lx, j = oy + ly;
        if (!own || !in_ring(lx, ly, 2) || i < 0 || j < 0 || i > N || j > N) continue;
        int l = ly * GLW + lx;
        Row<double> r = row_at<double>(i, j, N, H, ih2, kr[1][m], sa);
        U[l] = cdiv(csub(fr[1][m], offsum_l(r, U, l, GLW, i, j, N)), r.dre, r.dim);
    }
    __syncthreads();
    // the smoothed iterate on the tile (only when asked for: the up kernel
    // recomputes it)
    if (uo) {
#pragma unroll
        for (int m = 0; m < GDX * GDY / GNT; ++m) {
            const int q = tid + GNT * m;
            int tx = q % GDX, ty = q / GDX;
            int i = x0 + tx, j = y0 + ty;
            if (i > N || j > N) continue;
            uo[(size_t)j * M + i] = st_as<T>(U[(ty + GRH) * GLW + tx + GRH]);
        }
    }
    // residual with the role-(B) operator on tile + 1, kept in registers
    // until every thread has read the iterate, then stored over it
    C<double> res[2][GNS];
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int m = 0; m < GNS; ++m) {
            int lx, ly;
            bool own = gs_owned(tid, c, m, lx, ly);
            int i = ox + lx, j = oy + ly;
            if (!own || !in_ring(lx, ly, 1) || i < 0 || j < 0 || i > N || j > N) continue;
            int l = ly * GLW + lx;
            Row<double> r = row_at<double>(i, j, N, H, ih2, kr[c][m], sb);
            C<double> au = cadd(cmul(cmk(r.dre, r.dim), U[l]), offsum_l(r, U, l, GLW, i, j, N));
            res[c][m] = csub(fr[c][m], au);
        }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int m = 0; m < GNS; ++m) {
            int lx, ly;
            bool own = gs_owned(tid, c, m, lx, ly);
            int i = ox + lx, j = oy + ly;
            if (!own || !in_ring(lx, ly, 1) || i < 0 || j < 0 || i > N || j > N) continue;
            U[ly * GLW + lx] = res[c][m];
        }
    __syncthreads();
    // full weighting for the coarse nodes of this tile
    {
        const int Nc = N / 2, Mc = Nc + 1;
        constexpr int CX = GDX / 2, NCN = (GDX / 2) * (GDY / 2);
#pragma unroll
        for (int m = 0; m < (NCN + GNT - 1) / GNT; ++m) {
            const int q = tid + GNT * m;
            if (q >= NCN) break;
            int I = x0 / 2 + q % CX, J = y0 / 2 + q / CX;
            if (I > Nc || J > Nc) continue;
            C<double> s = cmk(0.0, 0.0);
            for (int e = -1; e <= 1; ++e) {
                int j = mirror(2 * J + e, N);
                for (int d = -1; d <= 1; ++d) {
                    int i = mirror(2 * I + d, N);
                    double w = (double)((2 - (d < 0 ? -d : d)) * (2 - (e < 0 ? -e : e)));
                    s = cadd(s, cscale(w, U[(j - oy) * GLW + (i - ox)]));
                }
            }
            fc[(size_t)J * Mc + I] = st_as<T>(cscale(0.0625, s));
        }
    }
}

// ===========================================================================
// k_gs_up: u0 = the zero-guess red-black sweep of k_gs_down (recomputed from
// f), u = u0 + P ec, then one red-black sweep; result to uo.  Regions shrink
// by one per dependent step: red u0 on tile + 3, black u0 on tile + 2,
// correction on tile + 2, red on tile + 1, black on the tile.
// ===========================================================================
template <typename T, typename TF, typename TU>
__global__ __launch_bounds__(GNT) void k_gs_up(GeoT g, double H, double ih2, const T *__restrict__ k, double sa,
                                               const C<TF> *__restrict__ f, const C<T> *__restrict__ ec,
                                               C<TU> *__restrict__ uo, const int *skip) {
    if (skip && *skip) return;
    __shared__ C<double> U[GLW * GLH];
    const int tid = threadIdx.x;
    const int x0 = blockIdx.x * GDX, y0 = blockIdx.y * GDY;
    const int ox = x0 - GRH, oy = y0 - GRH;
    const int N = g.N, M = g.M, Mc = N / 2 + 1;
    C<double> fr[2][GNS];
    double kr[2][GNS];
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int m = 0; m < GNS; ++m) {
            int lx, ly;
            bool own = gs_owned(tid, c, m, lx, ly);
            int i = ox + lx, j = oy + ly;
            if (own && i >= 0 && j >= 0 && i <= N && j <= N) {
                size_t p = (size_t)j * M + i;
                fr[c][m] = ldr<double>(f, p);
                kr[c][m] = (double)k[p];
            }
        }
    // red u0 on tile + 3
#pragma unroll
    for (int m = 0; m < GNS; ++m) {
        int lx, ly;
        bool own = gs_owned(tid, 0, m, lx, ly);
        int i = ox + lx, j = oy + ly;
        if (!own || i < 0 || j < 0 || i > N || j > N) continue;
        Row<double> r = row_at<double>(i, j, N, H, ih2, kr[0][m], sa);
        U[ly * GLW + lx] = cdiv(fr[0][m], r.dre, r.dim);
    }
    __syncthreads();
    // black u0 on tile + 2, plus the correction on the black nodes
#pragma unroll
    for (int m = 0; m < GNS; ++m) {
        int lx, ly;
        bool own = gs_owned(tid, 1, m, lx, ly);
        int i = ox + lx, j = oy + ly;
        if (!own || !in_ring(lx, ly, 2) || i < 0 || j < 0 || i > N || j > N) continue;
        int l = ly * GLW + lx;
        Row<double> r = row_at<double>(i, j, N, H, ih2, kr[1][m], sa);
        U[l] = cadd(cdiv(csub(fr[1][m], offsum_l(r, U, l, GLW, i, j, N)), r.dre, r.dim),
                    prolong_at(ec, i, j, Mc));
    }
    __syncthreads();
    // the correction on the red nodes of tile + 2 (after every black u0 has
    // read the uncorrected red values)
#pragma unroll
    for (int m = 0; m < GNS; ++m) {
        int lx, ly;
        bool own = gs_owned(tid, 0, m, lx, ly);
        int i = ox + lx, j = oy + ly;
        if (!own || !in_ring(lx, ly, 2) || i < 0 || j < 0 || i > N || j > N) continue;
        int l = ly * GLW + lx;
        U[l] = cadd(U[l], prolong_at(ec, i, j, Mc));
    }
    __syncthreads();
    // red on tile + 1
#pragma unroll
    for (int m = 0; m < GNS; ++m) {
        int lx, ly;
        bool own = gs_owned(tid, 0, m, lx, ly);
        int i = ox + lx, j = oy + ly;
        if (!own || !in_ring(lx, ly, 1) || i < 0 || j < 0 || i > N || j > N) continue;
        int l = ly * GLW + lx;
        Row<double> r = row_at<double>(i, j, N, H, ih2, kr[0][m], sa);
        U[l] = cdiv(csub(fr[0][m], offsum_l(r, U, l, GLW, i, j, N)), r.dre, r.dim);
    }
    __syncthreads();
    // black on the tile -> output; red tile nodes -> output
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int m = 0; m < GNS; ++m) {
            int lx, ly;
            bool own = gs_owned(tid, c, m, lx, ly);
            int i = ox + lx, j = oy + ly;
            if (!own || !in_ring(lx, ly, 0) || i > N || j > N) continue;
            int l = ly * GLW + lx;
            C<double> v = U[l];
            if (c == 1) {
                Row<double> r = row_at<double>(i, j, N, H, ih2, kr[1][m], sa);
                v = cdiv(csub(fr[1][m], offsum_l(r, U, l, GLW, i, j, N)), r.dre, r.dim);
            }
            uo[(size_t)j * M + i] = st_as<TU>(v);
        }
}

// ===========================================================================
// k_kacz_tb: S sweeps of 5-colour Kaczmarz on a TS x TS tile held in LDS
// with a halo of RH = 10 S (each colour pass moves information two nodes).
// Pass q (colour q mod 5) updates the rows on tile + (RH - 2q - 1); after it
// u is exact on tile + (RH - 2q - 2), and after the last pass on the tile
// itself.  Each thread keeps the same row slots (line, column slot) in every
// pass, so a pass needs no division to find its rows.  Initial u: 0 (ui ==
// null) or ui, plus P ec when ec != null.
// ===========================================================================
constexpr int KNT = 512;

template <typename T, int TS, int S>
__global__ __launch_bounds__(KNT) void k_kacz_tb(GeoT g, double H, double ih2, const T *__restrict__ k, double sig,
                                                 const C<T> *__restrict__ f, const C<T> *__restrict__ ui,
                                                 const C<T> *__restrict__ ec, C<T> *__restrict__ uo,
                                                 const int *skip) {
    if (skip && *skip) return;
    constexpr int RH = 10 * S, LW = TS + 2 * RH;
    // f and (k, 1/||a_p||^2) of the region are staged in LDS when they fit
    // next to u
    constexpr bool STAGE = (size_t)LW * LW * (16 + 16 + 16) <= 160 * 1024;
    constexpr int T5 = (LW - 2 + 4) / 5;              // row slots per line and colour
    constexpr int NSLOT = (LW - 2) * T5;              // slots per colour
    constexpr int NM = (NSLOT + KNT - 1) / KNT;       // slots per thread and colour
    __shared__ C<double> U[LW * LW];
    __shared__ C<double> FS[STAGE ? LW * LW : 1];
    __shared__ C<double> KS[STAGE ? LW * LW : 1];
    const int tid = threadIdx.x;
    const int x0 = blockIdx.x * TS, y0 = blockIdx.y * TS;
    const int ox = x0 - RH, oy = y0 - RH;
    const int N = g.N, M = g.M, Mc = N / 2 + 1;
    for (int q = tid; q < LW * LW; q += KNT) {
        int i = ox + q % LW, j = oy + q / LW;
        if (i < 0 || j < 0 || i > N || j > N) continue;
        size_t p = (size_t)j * M + i;
        C<double> v = ui ? ldr<double>(ui, p) : cmk(0.0, 0.0);
        if (ec) v = cadd(v, prolong_at(ec, i, j, Mc));
        U[q] = v;
        if (STAGE) {
            FS[q] = ldr<double>(f, p);
            double kp = (double)k[p];
            Row<double> r = row_at<double>(i, j, N, H, ih2, kp, sig);
            double nrm = r.dre * r.dre + r.dim * r.dim + r.wl * r.wl + r.wr * r.wr + r.wd * r.wd + r.wu * r.wu;
            KS[q] = cmk(kp, 1.0 / nrm);
        }
    }
    // row slots of this thread: line ly = 1 + s / T5, column slot t = s % T5;
    // for colour c the row sits at lx = 1 + ((c - i1 - 2 j) mod 5) + 5 t
    int sly[NM], sbase[NM];
#pragma unroll
    for (int m = 0; m < NM; ++m) {
        int sl = tid + KNT * m;
        sly[m] = (sl < NSLOT) ? 1 + sl / T5 : -1;
        sbase[m] = 5 * (sl % T5);
    }
    __syncthreads();
    for (int pass = 0; pass < 5 * S; ++pass) {
        const int c = pass % 5;
        const int lo = 2 * pass + 1, hi = LW - 2 - 2 * pass;   // rows on tile + (RH - 2 pass - 1)
#pragma unroll
        for (int m = 0; m < NM; ++m) {
            const int ly = sly[m];
            if (ly < lo || ly > hi) continue;
            const int j = oy + ly;
            const int lx = 1 + (((c - (ox + 1) - 2 * j) % 5) + 5) % 5 + sbase[m];
            const int i = ox + lx;
            if (lx < lo || lx > hi || i < 0 || j < 0 || i > N || j > N) continue;
            const int l = ly * LW + lx;
            size_t p = (size_t)j * M + i;
            C<double> kc = STAGE ? KS[l] : cmk((double)k[p], 0.0);
            Row<double> r = row_at<double>(i, j, N, H, ih2, kc.x, sig);
            C<double> fp = STAGE ? FS[l] : ldr<double>(f, p);
            C<double> res = csub(fp, cadd(cmul(cmk(r.dre, r.dim), U[l]), offsum_l(r, U, l, LW, i, j, N)));
            double invn = kc.y;
            if (!STAGE) {
                double nrm = r.dre * r.dre + r.dim * r.dim + r.wl * r.wl + r.wr * r.wr + r.wd * r.wd + r.wu * r.wu;
                invn = 1.0 / nrm;
            }
            C<double> d = cmk(res.x * invn, res.y * invn);
            C<double> up = U[l];
            U[l] = cmk(up.x + (r.dre * d.x + r.dim * d.y), up.y + (r.dre * d.y - r.dim * d.x));
            if (i > 0) U[l - 1] = cadd(U[l - 1], cscale(r.wl, d));
            if (i < N) U[l + 1] = cadd(U[l + 1], cscale(r.wr, d));
            if (j > 0) U[l - LW] = cadd(U[l - LW], cscale(r.wd, d));
            if (j < N) U[l + LW] = cadd(U[l + LW], cscale(r.wu, d));
        }
        __syncthreads();
    }
    for (int q = tid; q < TS * TS; q += KNT) {
        int i = x0 + q % TS, j = y0 + q / TS;
        if (i > N || j > N) continue;
        uo[(size_t)j * M + i] = st_as<T>(U[(j - oy) * LW + (i - ox)]);
    }
}

// ===========================================================================
// k_bottom: the V-cycle on levels lb..L-1 (n <= 31) in one workgroup of BNT
// threads.  Every field of every bottom level (u, f and k) lives in LDS, so
// the dependent colour passes never wait on global memory; only the first
// level's f (input), the coarsest inverse and the output touch it.
// ===========================================================================
constexpr int BNT = 256;
constexpr int BOT_C_ELEMS = 4096;     // complex slots (u and f of every level)
constexpr int BOT_K_ELEMS = 4096;     // real slots (k and a reciprocal of every level)

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

// K holds k of the level followed by IV: 1 / |a_pp|^2 (Gauss-Seidel levels)
// or 1 / ||a_p||^2 (Kaczmarz levels), computed once per launch.
template <typename T>
__device__ void bot_relax(const BotLevel<T> &L, C<double> *SM, const double *KS, int sweeps, bool zero) {
    const int tid = threadIdx.x, M = L.M, N = L.N, MM = M * M;
    C<double> *U = SM + L.uoff;
    const C<double> *F = SM + L.foff;
    const double *K = KS + L.koff;
    const double *IV = K + MM;
    if (zero && (L.sm != HMG_SM_GS_DEV || sweeps == 0)) {
        for (int p = tid; p < MM; p += BNT) U[p] = cmk(0.0, 0.0);
        __syncthreads();
    }
    if (L.sm == HMG_SM_GS_DEV) {
        for (int s = 0; s < sweeps; ++s)
            for (int colour = 0; colour < 2; ++colour) {
                bool zg = zero && s == 0 && colour == 0;
                for (int p = tid; p < MM; p += BNT) {
                    int i = p % M, j = p / M;
                    if (((i + j) & 1) != colour) continue;
                    Row<double> r = row_at<double>(i, j, N, L.H, L.ih2, K[p], L.sa);
                    C<double> num = F[p];
                    if (!zg) num = csub(num, offsum_l(r, U, p, M, i, j, N));
                    const double inv = IV[p];
                    U[p] = cmk((num.x * r.dre + num.y * r.dim) * inv, (num.y * r.dre - num.x * r.dim) * inv);
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
                    int p = j * M + i;
                    Row<double> r = row_at<double>(i, j, N, L.H, L.ih2, K[p], L.sa);
                    C<double> res = csub(F[p], cadd(cmul(cmk(r.dre, r.dim), U[p]), offsum_l(r, U, p, M, i, j, N)));
                    const double invn = IV[p];
                    C<double> d = cmk(res.x * invn, res.y * invn);
                    C<double> up = U[p];
                    U[p] = cmk(up.x + (r.dre * d.x + r.dim * d.y), up.y + (r.dre * d.y - r.dim * d.x));
                    if (i > 0) U[p - 1] = cadd(U[p - 1], cscale(r.wl, d));
                    if (i < N) U[p + 1] = cadd(U[p + 1], cscale(r.wr, d));
                    if (j > 0) U[p - M] = cadd(U[p - M], cscale(r.wd, d));
                    if (j < N) U[p + M] = cadd(U[p + M], cscale(r.wu, d));
                }
                __syncthreads();
            }
    }
}

template <typename T, typename TF, typename TU>
__global__ __launch_bounds__(BNT) void k_bottom(BotPlan<T> P, const C<TF> *__restrict__ fg, C<TU> *__restrict__ uo,
                                                const int *skip) {
    if (skip && *skip) return;
    __shared__ C<double> SM[BOT_C_ELEMS];
    __shared__ double KS[BOT_K_ELEMS];
    // level parameters are indexed at run time: keep them in LDS, not in
    // (spilled) registers
    __shared__ BotLevel<T> PL[BOT_MAXL];
    const int tid = threadIdx.x;
    if (tid < P.nlev) PL[tid] = P.L[tid];
    __syncthreads();
    const int last = P.nlev - 1;
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
    for (int p = tid; p < PL[0].M * PL[0].M; p += BNT) SM[PL[0].foff + p] = ldr<double>(fg, p);
    __syncthreads();
    // down: pre-relaxation, residual, full weighting into the next f
    for (int l = 0; l < last; ++l) {
        const BotLevel<T> &L = PL[l];
        bot_relax<T>(L, SM, KS, L.pre, true);
        const BotLevel<T> &Cl = PL[l + 1];
        const C<double> *U = SM + L.uoff;
        const C<double> *F = SM + L.foff;
        const double *K = KS + L.koff;
        for (int qc = tid; qc < Cl.M * Cl.M; qc += BNT) {
            int I = qc % Cl.M, J = qc / Cl.M;
            C<double> s = cmk(0.0, 0.0);
            for (int e = -1; e <= 1; ++e) {
                int j = mirror(2 * J + e, L.N);
                for (int d = -1; d <= 1; ++d) {
                    int i = mirror(2 * I + d, L.N);
                    int p = j * L.M + i;
                    Row<double> r = row_at<double>(i, j, L.N, L.H, L.ih2, K[p], L.sb);
                    C<double> res = csub(F[p], cadd(cmul(cmk(r.dre, r.dim), U[p]), offsum_l(r, U, p, L.M, i, j, L.N)));
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
        constexpr int CPARTS = 3;
        __shared__ C<double> part[CPARTS][BNT];
        const BotLevel<T> &L = PL[last];
        const int m = L.M * L.M;
        const int chunk = (m + CPARTS - 1) / CPARTS;
        const C<double> *F = SM + L.foff;
        for (int base = 0; base < m; base += BNT / CPARTS) {
            const int r = base + tid % (BNT / CPARTS), part_id = tid / (BNT / CPARTS);
            if (part_id < CPARTS) {
                C<double> acc = cmk(0.0, 0.0);
                if (r < m) {
                    const int c0 = part_id * chunk, c1 = min(m, c0 + chunk);
                    for (int c = c0; c < c1; ++c) acc = cadd(acc, cmul(P.ainv[(size_t)c * m + r], F[c]));
                }
                part[part_id][tid % (BNT / CPARTS)] = acc;
            }
            __syncthreads();
            if (tid < BNT / CPARTS && base + tid < m) {
                C<double> acc = part[0][tid];
                for (int q = 1; q < CPARTS; ++q) acc = cadd(acc, part[q][tid]);
                SM[L.uoff + base + tid] = acc;
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
        for (int p = tid; p < L.M * L.M; p += BNT) {
            int i = p % L.M, j = p / L.M;
            U[p] = cadd(U[p], prolong_at(E, i, j, Cl.M));
        }
        __syncthreads();
        bot_relax<T>(L, SM, KS, L.post, false);
    }
    const BotLevel<T> &L0 = PL[0];
    for (int p = tid; p < L0.M * L0.M; p += BNT) uo[p] = st_as<TU>(SM[L0.uoff + p]);
}

// ===========================================================================
// launchers
// ===========================================================================
static inline GeoT geo_t(const Geo &g) { return GeoT{g.n, g.M, g.N}; }

template <typename T, typename TF>
static void gs_down_t(hipStream_t s, const Geo &g, const void *k, double sa, double sb, const void *f, void *uo,
                      void *fc, const int *skip) {
    dim3 grid((g.M + GDX - 1) / GDX, (g.M + GDY - 1) / GDY);
    k_gs_down<T, TF><<<grid, GNT, 0, s>>>(geo_t(g), g.H, 1.0 / (g.H * g.H), (const T *)k, sa, sb,
                                          (const C<TF> *)f, (C<T> *)uo, (C<T> *)fc, skip);
}

void launch_gs_down(Prec p, bool f64in, hipStream_t s, const Geo &g, const void *k, double sa, double sb,
                    const void *f, void *uo, void *fc, const int *skip) {
    if (p == P64) gs_down_t<double, double>(s, g, k, sa, sb, f, uo, fc, skip);
    else if (f64in) gs_down_t<float, double>(s, g, k, sa, sb, f, uo, fc, skip);
    else gs_down_t<float, float>(s, g, k, sa, sb, f, uo, fc, skip);
}

template <typename T, typename TF, typename TU>
static void gs_up_t(hipStream_t s, const Geo &g, const void *k, double sa, const void *f, const void *ec, void *uo,
                    const int *skip) {
    dim3 grid((g.M + GDX - 1) / GDX, (g.M + GDY - 1) / GDY);
    k_gs_up<T, TF, TU><<<grid, GNT, 0, s>>>(geo_t(g), g.H, 1.0 / (g.H * g.H), (const T *)k, sa, (const C<TF> *)f,
                                            (const C<T> *)ec, (C<TU> *)uo, skip);
}

void launch_gs_up(Prec p, bool io64, hipStream_t s, const Geo &g, const void *k, double sa, const void *f,
                  const void *ec, void *uo, const int *skip) {
    if (p == P64) gs_up_t<double, double, double>(s, g, k, sa, f, ec, uo, skip);
    else if (io64) gs_up_t<float, double, double>(s, g, k, sa, f, ec, uo, skip);
    else gs_up_t<float, float, float>(s, g, k, sa, f, ec, uo, skip);
}

template <typename T, int TS, int S>
static void kacz_tb_t(hipStream_t s, const Geo &g, const void *k, double sig, const void *f, const void *ui,
                      const void *ec, void *uo, const int *skip) {
    dim3 grid((g.M + TS - 1) / TS, (g.M + TS - 1) / TS);
    k_kacz_tb<T, TS, S><<<grid, KNT, 0, s>>>(geo_t(g), g.H, 1.0 / (g.H * g.H), (const T *)k, sig,
                                             (const C<T> *)f, (const C<T> *)ui, (const C<T> *)ec, (C<T> *)uo,
                                             skip);
}

// Tile configurations offered to the tuner: (tile side, sweeps per launch).
const KaczCfg kKaczCfgs[KACZ_NCFG] = {{32, 1}, {32, 2}, {16, 2}, {16, 4}};

// The LDS tile holds FP64 values in either storage precision.
bool kacz_cfg_fits(Prec, int cfg) {
    const KaczCfg &c = kKaczCfgs[cfg];
    int lw = c.ts + 20 * c.sweeps;
    return (size_t)lw * lw * 16 <= 160 * 1024;
}

void launch_kacz_tb(Prec p, int cfg, hipStream_t s, const Geo &g, const void *k, double sig, const void *f,
                    const void *ui, const void *ec, void *uo, const int *skip) {
    if (p == P64) {
        switch (cfg) {
        case 0: kacz_tb_t<double, 32, 1>(s, g, k, sig, f, ui, ec, uo, skip); break;
        case 1: kacz_tb_t<double, 32, 2>(s, g, k, sig, f, ui, ec, uo, skip); break;
        case 2: kacz_tb_t<double, 16, 2>(s, g, k, sig, f, ui, ec, uo, skip); break;
        default: kacz_tb_t<double, 16, 4>(s, g, k, sig, f, ui, ec, uo, skip); break;
        }
    } else {
        switch (cfg) {
        case 0: kacz_tb_t<float, 32, 1>(s, g, k, sig, f, ui, ec, uo, skip); break;
        case 1: kacz_tb_t<float, 32, 2>(s, g, k, sig, f, ui, ec, uo, skip); break;
        case 2: kacz_tb_t<float, 16, 2>(s, g, k, sig, f, ui, ec, uo, skip); break;
        default: kacz_tb_t<float, 16, 4>(s, g, k, sig, f, ui, ec, uo, skip); break;
        }
    }
}

int bottom_complex_slots() { return BOT_C_ELEMS; }
int bottom_real_slots() { return BOT_K_ELEMS; }

template <typename T, typename TF, typename TU>
static void bottom_t(hipStream_t s, const BottomDesc &d, const void *f, void *uo, const int *skip) {
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
    k_bottom<T, TF, TU><<<1, BNT, 0, s>>>(P, (const C<TF> *)f, (C<TU> *)uo, skip);
}

void launch_bottom(Prec p, bool io64, hipStream_t s, const BottomDesc &d, const void *f, void *uo, const int *skip) {
    if (p == P64) bottom_t<double, double, double>(s, d, f, uo, skip);
    else if (io64) bottom_t<float, double, double>(s, d, f, uo, skip);
    else bottom_t<float, float, float>(s, d, f, uo, skip);
}

}  // namespace hmgk
