// hmg_lex.hip -- lexicographic Gauss-Seidel and Kaczmarz sweeps (Section 4:
// the smoothers are analysed, and run by the paper, in lexicographic order,
// x fastest).  These give the results of the sequential sweeps, computed as
// a wavefront; the default schedule's coloured sweeps are the parallel
// alternative.
//
// Order.  A sweep visits the rows (i, j) with j outer and i inner.  In the
// skewed coordinate c = i + j the 5-point neighbours of (c, j) are (c -+ 1, j)
// (left, right), (c - 1, j - 1) (down) and (c + 1, j + 1) (up).
//   Gauss-Seidel reads the new values of left and down and the old values of
//   right and up: all rows with the same c are independent, and processing
//   c = 0, 1, 2, ... reproduces the sequential sweep.
//   Kaczmarz row p changes u on the whole stencil of p, so two rows interact
//   whenever their stencils meet (Manhattan distance <= 2).  The earlier row
//   of such a pair always has the smaller t = c + j = i + 2j, and rows with
//   equal t are at distance >= 3: processing t = 0, 1, 2, ... reproduces the
//   sequential sweep.
// Every dependency of row (c, j) points to a row with c' <= c and j' <= j, so
// rectangular tiles of the skewed plane (TC columns of c by TR rows of j) are
// processed in diagonal order a + b = 0, 1, 2, ... (tile (a, b)): one launch
// per diagonal; tiles of one diagonal touch disjoint node sets (their rows
// are pairwise at distance >= 3) except for two corner halo cells, which the
// kernel reads but neither uses nor writes back.
//
// Kernel.  One tile per workgroup of four waves.  The tile's u with a
// one-cell halo ring, its f and the constants of its rows (Gauss-Seidel:
// conj(a_pp) / |a_pp|^2; Kaczmarz: a_pp and 1 / ||a_p||^2) are staged in LDS
// by all four waves, every thread issuing all of its loads before its first
// LDS store (rows of the skewed tile are contiguous runs of a grid row in
// HBM, so the loads are coalesced).  The first wave then steps through the
// tile, lane = tile row (Gauss-Seidel: TC steps, all lanes on column c;
// Kaczmarz: TC + TR - 1 steps, lane l on column t - l), and all four waves
// write back what changed.  Arithmetic is FP64 as in the other kernels; u is
// rounded to the level precision at every store, as the coloured kernels do.

#include "hmg_device.h"

namespace hmgk {

constexpr int LX_TR = 64;            // rows per tile = lanes of the computing wave
constexpr int LX_TC = 32;            // skewed columns per tile
constexpr int LX_NT = 256;           // threads per workgroup (staging and write-back)
constexpr int LX_UH = LX_TR + 2;     // staged rows of u (halo ring)
constexpr int LX_UW = LX_TC + 3;     // staged columns of u: TC + 2, padded to an odd 16-byte stride
constexpr int LX_FW = LX_TC + 1;     // row stride of the staged f and row constants (odd)
constexpr int LX_UCELLS = LX_UH * (LX_TC + 2);
constexpr int LX_UPER = (LX_UCELLS + LX_NT - 1) / LX_NT;   // u cells per thread
constexpr int LX_FPER = LX_TR * LX_TC / LX_NT;             // f and k values per thread
static_assert(LX_TR * LX_TC % LX_NT == 0, "f and k cells divide over the threads");

// End of one wavefront step: order this step's LDS stores before the next
// step's LDS loads of other lanes of the same wave.
__device__ __forceinline__ void wave_step() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <typename T>
__device__ __forceinline__ C<double> lds_c(const C<T> &v) {
    return cmk((double)v.x, (double)v.y);
}

template <typename T, bool KACZ>
__global__ __launch_bounds__(LX_NT) void k_lex(GeoT g, double H, double ih2, const T *__restrict__ k, double sigma,
                                               const C<T> *__restrict__ f, C<T> *u, int diag, int b_lo,
                                               const int *skip) {
    if (skip && *skip) return;
    __shared__ C<T> U[LX_UH][LX_UW];
    __shared__ C<T> F[LX_TR][LX_FW];
    // per-node constants of the row, formed while staging (off the steps'
    // dependency chain): Gauss-Seidel conj(a_pp) / |a_pp|^2; Kaczmarz a_pp
    // and 1 / ||a_p||^2
    __shared__ double RW[LX_TR][LX_FW][3];
    const int b = b_lo + (int)blockIdx.x, a = diag - b;
    const int c0 = a * LX_TC, j0 = b * LX_TR, tid = threadIdx.x;

    // u with the halo ring: cell (jj, cc) holds node (i, j) = (c0 - 1 + cc - j, j0 - 1 + jj),
    // zero outside the grid (the matching weights of row_at are zero there).
    // All loads first, then the LDS stores.
    C<T> uv[LX_UPER], fv[LX_FPER];
    T kv[LX_FPER];
#pragma unroll
    for (int t = 0; t < LX_UPER; ++t) {
        const int q = t * LX_NT + tid, jj = q / (LX_TC + 2), cc = q - jj * (LX_TC + 2);
        const int j = j0 - 1 + jj, i = c0 - 1 + cc - j;
        uv[t] = (q < LX_UCELLS && j >= 0 && j <= g.N && i >= 0 && i <= g.N) ? u[(size_t)j * g.M + i]
                                                                          : cmk(T(0), T(0));
    }
#pragma unroll
    for (int t = 0; t < LX_FPER; ++t) {
        const int q = t * LX_NT + tid, jl = q / LX_TC, cl = q - jl * LX_TC;
        const int j = j0 + jl, i = c0 + cl - j;
        const bool in = j <= g.N && i >= 0 && i <= g.N;
        const size_t p = in ? (size_t)j * g.M + i : 0;
        fv[t] = in ? f[p] : cmk(T(0), T(0));
        kv[t] = in ? k[p] : T(1);
    }
#pragma unroll
    for (int t = 0; t < LX_UPER; ++t) {
        const int q = t * LX_NT + tid, jj = q / (LX_TC + 2), cc = q - jj * (LX_TC + 2);
        if (q < LX_UCELLS) U[jj][cc] = uv[t];
    }
#pragma unroll
    for (int t = 0; t < LX_FPER; ++t) {
        const int q = t * LX_NT + tid, jl = q / LX_TC, cl = q - jl * LX_TC;
        const int j = j0 + jl, i = c0 + cl - j;
        F[jl][cl] = fv[t];
        const Row<double> r = row_at<double>(i, j, g.N, H, ih2, (double)kv[t], sigma);
        if (KACZ) {
            RW[jl][cl][0] = r.dre;
            RW[jl][cl][1] = r.dim;
            RW[jl][cl][2] = 1.0 / (r.dre * r.dre + r.dim * r.dim + r.wl * r.wl + r.wr * r.wr + r.wd * r.wd +
                                   r.wu * r.wu);
        } else {
            const double inv = 1.0 / (r.dre * r.dre + r.dim * r.dim);
            RW[jl][cl][0] = r.dre * inv;
            RW[jl][cl][1] = -r.dim * inv;
        }
    }
    __syncthreads();

    // Only the first wave computes.  Between steps its lanes exchange values
    // through LDS; a wave's LDS operations complete in issue order, so
    // wavefront-scope fences (which keep the compiler from moving LDS accesses
    // across them) order each step's stores before the next step's loads.
    // The other waves wait at the barrier that follows.
    if (tid < LX_TR) {
        const int lane = tid, j = j0 + lane, jj = lane + 1;
        if (!KACZ) {
            for (int s = 0; s < LX_TC; ++s) {
                const int i = c0 + s - j, cc = s + 1;
                if (j <= g.N && i >= 0 && i <= g.N) {
                    const Row<double> r = row_at<double>(i, j, g.N, H, ih2, 0.0, 0.0);   // weights only
                    // neighbours in the order left, right, down, up
                    C<double> o = cscale(r.wl, lds_c(U[jj][cc - 1]));
                    o = cadd(o, cscale(r.wr, lds_c(U[jj][cc + 1])));
                    o = cadd(o, cscale(r.wd, lds_c(U[jj - 1][cc - 1])));
                    o = cadd(o, cscale(r.wu, lds_c(U[jj + 1][cc + 1])));
                    U[jj][cc] = st_as<T>(cmul(csub(lds_c(F[lane][s]), o), cmk(RW[lane][s][0], RW[lane][s][1])));
                }
                wave_step();
            }
        } else {
            // delta = (f_p - (A u)_p) / ||a_p||^2, u_q += conj(a_pq) delta on the stencil of p
            for (int s = 0; s < LX_TC + LX_TR - 1; ++s) {
                const int cl = s - lane, i = c0 + cl - j, cc = cl + 1;
                if (cl >= 0 && cl < LX_TC && j <= g.N && i >= 0 && i <= g.N) {
                    Row<double> r = row_at<double>(i, j, g.N, H, ih2, 0.0, 0.0);   // weights only
                    r.dre = RW[lane][cl][0];
                    r.dim = RW[lane][cl][1];
                    const C<double> up = lds_c(U[jj][cc]), ul = lds_c(U[jj][cc - 1]), ur = lds_c(U[jj][cc + 1]);
                    const C<double> ud = lds_c(U[jj - 1][cc - 1]), uu = lds_c(U[jj + 1][cc + 1]);
                    C<double> o = cscale(r.wl, ul);
                    o = cadd(o, cscale(r.wr, ur));
                    o = cadd(o, cscale(r.wd, ud));
                    o = cadd(o, cscale(r.wu, uu));
                    const C<double> res = csub(lds_c(F[lane][cl]), cadd(cmul(cmk(r.dre, r.dim), up), o));
                    const double rn = RW[lane][cl][2];
                    const C<double> d = cmk(res.x * rn, res.y * rn);
                    U[jj][cc] = st_as<T>(cmk(up.x + (r.dre * d.x + r.dim * d.y), up.y + (r.dre * d.y - r.dim * d.x)));
                    if (i > 0) U[jj][cc - 1] = st_as<T>(cadd(ul, cscale(r.wl, d)));
                    if (i < g.N) U[jj][cc + 1] = st_as<T>(cadd(ur, cscale(r.wr, d)));
                    if (j > 0) U[jj - 1][cc - 1] = st_as<T>(cadd(ud, cscale(r.wd, d)));
                    if (j < g.N) U[jj + 1][cc + 1] = st_as<T>(cadd(uu, cscale(r.wu, d)));
                }
                wave_step();
            }
        }
    }
    __syncthreads();

    if (!KACZ) {
        for (int q = tid; q < LX_TR * LX_TC; q += LX_NT) {
            const int jl = q / LX_TC, cl = q - jl * LX_TC;
            const int jg = j0 + jl, i = c0 + cl - jg;
            if (jg <= g.N && i >= 0 && i <= g.N) u[(size_t)jg * g.M + i] = U[jl + 1][cl + 1];
        }
        return;
    }
    // Kaczmarz: write back the union of the rows' stencils: the staged
    // rectangle less the corners (0, TC), (0, TC+1), (TR+1, 0), (TR+1, 1); two
    // of those belong to the tiles that run concurrently
    for (int q = tid; q < LX_UCELLS; q += LX_NT) {
        const int rj = q / (LX_TC + 2), cc = q - rj * (LX_TC + 2);
        if ((rj == 0 && cc >= LX_TC) || (rj == LX_UH - 1 && cc <= 1)) continue;
        const int jg = j0 - 1 + rj, i = c0 - 1 + cc - jg;
        if (jg >= 0 && jg <= g.N && i >= 0 && i <= g.N) u[(size_t)jg * g.M + i] = U[rj][cc];
    }
}

// Tiles of diagonal d that hold at least one node: b in [lo, hi] (lo > hi
// when none).  Tile (a, b) covers c in [a TC, a TC + TC), j in [b TR, b TR + TR);
// it holds a node iff its largest i = c - j is >= 0 and its smallest is <= N.
static void lex_tiles(int N, int d, int NA, int NB, int &lo, int &hi) {
    lo = 0;
    hi = -1;
    bool seen = false;
    for (int b = (d - NA + 1 > 0 ? d - NA + 1 : 0); b <= (d < NB - 1 ? d : NB - 1); ++b) {
        const int c0 = (d - b) * LX_TC, j0 = b * LX_TR, j1 = (j0 + LX_TR - 1 < N) ? j0 + LX_TR - 1 : N;
        if (c0 + LX_TC - 1 - j0 >= 0 && c0 - j1 <= N) {
            if (!seen) lo = b;
            seen = true;
            hi = b;
        }
    }
}

template <typename T, bool KACZ>
static void lex_t(hipStream_t s, const Geo &g, const void *k, double sigma, const void *f, void *u,
                  const int *skip) {
    const double H = g.H, ih2 = 1.0 / (g.H * g.H);
    const int NA = (2 * g.N + LX_TC) / LX_TC, NB = (g.N + LX_TR) / LX_TR;
    const GeoT gt{g.n, g.M, g.N};
    for (int d = 0; d < NA + NB - 1; ++d) {
        int lo, hi;
        lex_tiles(g.N, d, NA, NB, lo, hi);
        if (hi < lo) continue;
        k_lex<T, KACZ><<<hi - lo + 1, LX_NT, 0, s>>>(gt, H, ih2, (const T *)k, sigma, (const C<T> *)f, (C<T> *)u,
                                                     d, lo, skip);
    }
}

void launch_lex_sweep(Prec p, int kacz, hipStream_t s, const Geo &g, const void *k, double sigma, const void *f,
                      void *u, const int *skip) {
    if (p == P64) {
        if (kacz) lex_t<double, true>(s, g, k, sigma, f, u, skip);
        else lex_t<double, false>(s, g, k, sigma, f, u, skip);
    } else {
        if (kacz) lex_t<float, true>(s, g, k, sigma, f, u, skip);
        else lex_t<float, false>(s, g, k, sigma, f, u, skip);
    }
}

}  // namespace hmgk
