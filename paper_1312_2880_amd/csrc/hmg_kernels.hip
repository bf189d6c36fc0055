// hmg_kernels.hip -- gfx950 kernels of the multigrid-preconditioned
// Bi-CGSTAB Helmholtz solver (Livshits, arXiv:1312.2880).
//
// Layout: every field of a level is dense (n+2) x (n+2), x fastest; complex
// values are interleaved (re, im) in the level precision T (double or
// float).  Threads are laid out 64 x 4 per block so that each 64-wide wave
// reads 64 consecutive nodes of one grid row.
//
//
// The discrete operator and complex helpers are in hmg_device.h.

#include "hmg_device.h"

#include <cstring>

namespace hmgk {

// ---------------------------------------------------------------------------
// Operator apply: out = A_sigma u
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(NT) void k_apply(GeoT g, double H, double ih2, const T *__restrict__ k, double sigma,
                                              const C<T> *__restrict__ u, C<T> *__restrict__ out) {
    int i = blockIdx.x * BX + threadIdx.x;
    int j = blockIdx.y * BY + threadIdx.y;
    if (i > g.N || j > g.N) return;
    size_t p = (size_t)j * g.M + i;
    Row<double> r = row_at<double>(i, j, g.N, H, ih2, (double)k[p], sigma);
    out[p] = st_as<T>(row_apply(r, u, i, j, g.N, g.M));
}

// ---------------------------------------------------------------------------
// Red-black Gauss-Seidel half sweep (Section 4 relaxation, red = (i+j) even).
// u_p <- (f_p - sum_{q != p} a_pq u_q) / a_pp for every node of one colour;
// nodes of one colour are not coupled, so the update is order independent.
// zero_guess (colour 0 of a first sweep): the other colour counts as zero.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(NT) void k_gs_colour(GeoT g, double H, double ih2, const T *__restrict__ k,
                                                  double sigma, const C<T> *__restrict__ f, C<T> *u, int colour,
                                                  int zero_guess, const int *skip) {
    if (skip && *skip) return;
    int j = blockIdx.y * BY + threadIdx.y;
    int i = 2 * (blockIdx.x * BX + threadIdx.x) + ((colour + j) & 1);
    if (i > g.N || j > g.N) return;
    size_t p = (size_t)j * g.M + i;
    Row<double> r = row_at<double>(i, j, g.N, H, ih2, (double)k[p], sigma);
    C<double> num = ldr<double>(f, p);
    if (!zero_guess) num = csub(num, offsum(r, u, i, j, g.N, g.M));
    u[p] = st_as<T>(cdiv(num, r.dre, r.dim));
}

// ---------------------------------------------------------------------------
// 5-colour Kaczmarz pass (Section 4: relaxation of the normal equations,
// row-action form).  For every row p with (i + 2j) mod 5 == colour:
//   delta = (f_p - (A u)_p) / ||a_p||^2,  u_q += conj(a_pq) delta, q in row p.
// Rows of one colour are >= 3 apart, so their stencils are disjoint.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(NT) void k_kacz_colour(GeoT g, double H, double ih2, const T *__restrict__ k,
                                                    double sigma, const C<T> *__restrict__ f, C<T> *u, int colour,
                                                    const int *skip) {
    if (skip && *skip) return;
    int j = blockIdx.y * BY + threadIdx.y;
    int i0 = ((colour - 2 * j) % 5 + 5) % 5;
    int i = i0 + 5 * (blockIdx.x * BX + threadIdx.x);
    if (i > g.N || j > g.N) return;
    size_t p = (size_t)j * g.M + i;
    Row<double> r = row_at<double>(i, j, g.N, H, ih2, (double)k[p], sigma);
    C<double> res = csub(ldr<double>(f, p), row_apply(r, u, i, j, g.N, g.M));
    double nrm = r.dre * r.dre + r.dim * r.dim + r.wl * r.wl + r.wr * r.wr + r.wd * r.wd + r.wu * r.wu;
    C<double> d = cmk(res.x / nrm, res.y / nrm);
    C<double> up = ldr<double>(u, p);
    u[p] = st_as<T>(cmk(up.x + (r.dre * d.x + r.dim * d.y), up.y + (r.dre * d.y - r.dim * d.x)));
    if (i > 0) u[p - 1] = st_as<T>(cadd(ldr<double>(u, p - 1), cscale(r.wl, d)));
    if (i < g.N) u[p + 1] = st_as<T>(cadd(ldr<double>(u, p + 1), cscale(r.wr, d)));
    if (j > 0) u[p - g.M] = st_as<T>(cadd(ldr<double>(u, p - g.M), cscale(r.wd, d)));
    if (j < g.N) u[p + g.M] = st_as<T>(cadd(ldr<double>(u, p + g.M), cscale(r.wu, d)));
}

template <typename T>
__global__ __launch_bounds__(256) void k_fill_zero(C<T> *u, size_t count, const int *skip, long zs) {
    u = zsh(u, zs);
    skip = zsh(skip, zs);
    if (skip && *skip) return;
    size_t q = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (q < count) u[q] = cmk(T(0), T(0));
}

// ---------------------------------------------------------------------------
// Residual + full weighting (Section 5): fc(I,J) = (1/16) sum_{d,e} (2-|d|)
// (2-|e|) r(2I+d, 2J+e), r = f - A_sigma u, fine values outside the grid
// mirrored (r(-1) = r(1), r(N+1) = r(N-1)).  One thread per coarse node.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(NT) void k_residual_fw(GeoT g, double H, double ih2, const T *__restrict__ k,
                                                    double sigma, const C<T> *__restrict__ f,
                                                    const C<T> *__restrict__ u, C<T> *__restrict__ fc,
                                                    const int *skip, long zs) {
    f = zsh(f, zs);
    u = zsh(u, zs);
    fc = zsh(fc, zs);
    skip = zsh(skip, zs);
    if (skip && *skip) return;
    int Nc = g.N / 2, Mc = Nc + 1;
    int I = blockIdx.x * BX + threadIdx.x;
    int J = blockIdx.y * BY + threadIdx.y;
    if (I > Nc || J > Nc) return;
    C<double> s = cmk(0.0, 0.0);
    for (int e = -1; e <= 1; ++e) {
        int j = 2 * J + e;
        j = (j < 0) ? -j : ((j > g.N) ? 2 * g.N - j : j);
        for (int d = -1; d <= 1; ++d) {
            int i = 2 * I + d;
            i = (i < 0) ? -i : ((i > g.N) ? 2 * g.N - i : i);
            size_t p = (size_t)j * g.M + i;
            Row<double> r = row_at<double>(i, j, g.N, H, ih2, (double)k[p], sigma);
            C<double> res = csub(ldr<double>(f, p), row_apply(r, u, i, j, g.N, g.M));
            double w = (double)((2 - (d < 0 ? -d : d)) * (2 - (e < 0 ? -e : e)));
            s = cadd(s, cscale(w, res));
        }
    }
    fc[(size_t)J * Mc + I] = st_as<T>(cscale(0.0625, s));
}

// ---------------------------------------------------------------------------
// Bilinear prolongation + correction (Section 5): u += P ec.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(NT) void k_prolong_add(GeoT g, const C<T> *__restrict__ ec, C<T> *u,
                                                    const int *skip, long zs) {
    ec = zsh(ec, zs);
    u = zsh(u, zs);
    skip = zsh(skip, zs);
    if (skip && *skip) return;
    int i = blockIdx.x * BX + threadIdx.x;
    int j = blockIdx.y * BY + threadIdx.y;
    if (i > g.N || j > g.N) return;
    int Mc = g.N / 2 + 1;
    int I = i >> 1, J = j >> 1;
    size_t q = (size_t)J * Mc + I;
    C<double> e;
    if (!(i & 1) && !(j & 1)) {
        e = ldr<double>(ec, q);
    } else if ((i & 1) && !(j & 1)) {
        e = cscale(0.5, cadd(ldr<double>(ec, q), ldr<double>(ec, q + 1)));
    } else if (!(i & 1) && (j & 1)) {
        e = cscale(0.5, cadd(ldr<double>(ec, q), ldr<double>(ec, q + Mc)));
    } else {
        e = cscale(0.25, cadd(cadd(cadd(ldr<double>(ec, q), ldr<double>(ec, q + 1)), ldr<double>(ec, q + Mc)),
                              ldr<double>(ec, q + Mc + 1)));
    }
    size_t p = (size_t)j * g.M + i;
    u[p] = st_as<T>(cadd(ldr<double>(u, p), e));
}

// ---------------------------------------------------------------------------
// Coarsest level: u = A_c^{-1} f with the inverse precomputed in FP64
// (stored transposed, ainv_t[c*m + r] = inv[r][c], so that consecutive
// threads read consecutive rows).  One workgroup.
// ---------------------------------------------------------------------------
constexpr int MAX_COARSE = 33 * 33;

template <typename T>
__global__ __launch_bounds__(256) void k_coarsest(int m, const C<double> *__restrict__ ainv_t,
                                                  const C<T> *__restrict__ f, C<T> *__restrict__ u,
                                                  const int *skip) {
    if (skip && *skip) return;
    __shared__ C<double> fs[MAX_COARSE];
    for (int q = threadIdx.x; q < m; q += 256) fs[q] = ldr<double>(f, q);
    __syncthreads();
    for (int r = threadIdx.x; r < m; r += 256) {
        C<double> acc = cmk(0.0, 0.0);
        for (int c = 0; c < m; ++c) acc = cadd(acc, cmul(ainv_t[(size_t)c * m + r], fs[c]));
        u[r] = st_as<T>(acc);
    }
}

__global__ __launch_bounds__(256) void k_to_float(const C<double> *__restrict__ src, C<float> *__restrict__ dst,
                                                  size_t count, const int *skip, long zs) {
    src = zsh(src, zs);
    dst = zsh(dst, zs);
    skip = zsh(skip, zs);
    if (skip && *skip) return;
    size_t q = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (q < count) dst[q] = cmk((float)src[q].x, (float)src[q].y);
}

__global__ __launch_bounds__(256) void k_to_double(const C<float> *__restrict__ src, C<double> *__restrict__ dst,
                                                   size_t count, const int *skip, long zs) {
    src = zsh(src, zs);
    dst = zsh(dst, zs);
    skip = zsh(skip, zs);
    if (skip && *skip) return;
    size_t q = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (q < count) dst[q] = cmk((double)src[q].x, (double)src[q].y);
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
static inline GeoT geot(const Geo &g) { return GeoT{g.n, g.M, g.N}; }
static inline dim3 grid2(int nx, int ny, int nz = 1) { return dim3((nx + BX - 1) / BX, (ny + BY - 1) / BY, nz); }

template <typename T>
static void apply_t(hipStream_t s, const Geo &g, const void *k, double sigma, const void *u, void *out) {
    double H = g.H, ih2 = 1.0 / (g.H * g.H);
    k_apply<T><<<grid2(g.M, g.M), dim3(BX, BY), 0, s>>>(geot(g), H, ih2, (const T *)k, sigma,
                                                         (const C<T> *)u, (C<T> *)out);
}
void launch_apply(Prec p, hipStream_t s, const Geo &g, const void *k, double sigma, const void *u, void *out) {
    if (p == P64) apply_t<double>(s, g, k, sigma, u, out);
    else apply_t<float>(s, g, k, sigma, u, out);
}

template <typename T>
static void gs_t(hipStream_t s, const Geo &g, const void *k, double sigma, const void *f, void *u, int colour,
                 int zero_guess, const int *skip) {
    double H = g.H, ih2 = 1.0 / (g.H * g.H);
    k_gs_colour<T><<<grid2((g.M + 1) / 2, g.M), dim3(BX, BY), 0, s>>>(
        geot(g), H, ih2, (const T *)k, sigma, (const C<T> *)f, (C<T> *)u, colour, zero_guess, skip);
}
void launch_gs_colour(Prec p, hipStream_t s, const Geo &g, const void *k, double sigma, const void *f, void *u,
                      int colour, int zero_guess, const int *skip) {
    if (p == P64) gs_t<double>(s, g, k, sigma, f, u, colour, zero_guess, skip);
    else gs_t<float>(s, g, k, sigma, f, u, colour, zero_guess, skip);
}

template <typename T>
static void kacz_t(hipStream_t s, const Geo &g, const void *k, double sigma, const void *f, void *u, int colour,
                   const int *skip) {
    double H = g.H, ih2 = 1.0 / (g.H * g.H);
    k_kacz_colour<T><<<grid2((g.M + 4) / 5, g.M), dim3(BX, BY), 0, s>>>(
        geot(g), H, ih2, (const T *)k, sigma, (const C<T> *)f, (C<T> *)u, colour, skip);
}
void launch_kacz_colour(Prec p, hipStream_t s, const Geo &g, const void *k, double sigma, const void *f, void *u,
                        int colour, const int *skip) {
    if (p == P64) kacz_t<double>(s, g, k, sigma, f, u, colour, skip);
    else kacz_t<float>(s, g, k, sigma, f, u, colour, skip);
}

void launch_fill_zero(Prec p, hipStream_t s, void *u, size_t count, const int *skip, Bz bz) {
    dim3 nb((unsigned)((count + 255) / 256), 1, bz.nz);
    if (p == P64) k_fill_zero<double><<<nb, 256, 0, s>>>((C<double> *)u, count, skip, bz.zs);
    else k_fill_zero<float><<<nb, 256, 0, s>>>((C<float> *)u, count, skip, bz.zs);
}

template <typename T>
static void rfw_t(hipStream_t s, const Geo &g, const void *k, double sigma, const void *f, const void *u, void *fc,
                  const int *skip, Bz bz) {
    double H = g.H, ih2 = 1.0 / (g.H * g.H);
    int Mc = g.N / 2 + 1;
    k_residual_fw<T><<<grid2(Mc, Mc, bz.nz), dim3(BX, BY), 0, s>>>(geot(g), H, ih2, (const T *)k, sigma,
                                                                    (const C<T> *)f, (const C<T> *)u, (C<T> *)fc,
                                                                    skip, bz.zs);
}
void launch_residual_fw(Prec p, hipStream_t s, const Geo &g, const void *k, double sigma, const void *f,
                        const void *u, void *fc, const int *skip, Bz bz) {
    if (p == P64) rfw_t<double>(s, g, k, sigma, f, u, fc, skip, bz);
    else rfw_t<float>(s, g, k, sigma, f, u, fc, skip, bz);
}

void launch_prolong_add(Prec p, hipStream_t s, const Geo &g, const void *ec, void *u, const int *skip, Bz bz) {
    if (p == P64)
        k_prolong_add<double><<<grid2(g.M, g.M, bz.nz), dim3(BX, BY), 0, s>>>(geot(g), (const C<double> *)ec,
                                                                              (C<double> *)u, skip, bz.zs);
    else
        k_prolong_add<float><<<grid2(g.M, g.M, bz.nz), dim3(BX, BY), 0, s>>>(geot(g), (const C<float> *)ec,
                                                                             (C<float> *)u, skip, bz.zs);
}

void launch_coarsest(Prec p, hipStream_t s, int m, const double *ainv_t, const void *f, void *u, const int *skip) {
    if (p == P64)
        k_coarsest<double><<<1, 256, 0, s>>>(m, (const C<double> *)ainv_t, (const C<double> *)f, (C<double> *)u,
                                             skip);
    else
        k_coarsest<float><<<1, 256, 0, s>>>(m, (const C<double> *)ainv_t, (const C<float> *)f, (C<float> *)u,
                                            skip);
}

void launch_convert(hipStream_t s, int to_float, const void *src, void *dst, size_t count, const int *skip, Bz bz) {
    dim3 nb((unsigned)((count + 255) / 256), 1, bz.nz);
    if (to_float) k_to_float<<<nb, 256, 0, s>>>((const C<double> *)src, (C<float> *)dst, count, skip, bz.zs);
    else k_to_double<<<nb, 256, 0, s>>>((const C<float> *)src, (C<double> *)dst, count, skip, bz.zs);
}

// ===========================================================================
// Bi-CGSTAB (Section 6), FP64 on the finest grid.  Right preconditioning:
//   p = r + beta (p - omega v);  ph = B p;  v = L ph;  alpha = rho / (rh, v)
//   s = r - alpha v  (half step; stop if ||s|| <= rtol ||b||, x += alpha ph)
//   sh = B s;  t = L sh;  omega = (t, s) / (t, t)
//   x += alpha ph + omega sh;  r = s - omega t;  rho' = (rh, r)
//   beta = (rho' / rho)(alpha / omega)
// Inner products (a, b) = sum conj(a) b.  Each reduction writes one partial
// per block (fixed block order) and a single-block kernel sums the partials
// in a fixed order, so results do not depend on scheduling.
// ===========================================================================

// Single 256-thread block: total of each of NV partial rows.  Thread t sums
// entries t, t + 256, ... in eight interleaved accumulators (independent
// loads in flight instead of one dependent chain), combined in a fixed
// order, then a fixed tree across the block: the result depends only on nb.
// Accumulator u of thread t takes the entries t + u NT + 8 NT r below nb in
// increasing r.  Up to FIN_R rounds, every entry of every row is loaded
// before the first add (one memory round trip instead of one per round and
// row: the partials come from another kernel, through the last-level
// cache); the adds keep that order, so the sums are the same bit for bit.
constexpr int FIN_R = 3;
template <int NV>
__device__ __forceinline__ void finalize_sums(const double *partials, int nb, double *tot) {
    double v[NV];
    int tid = threadIdx.y * BX + threadIdx.x;
    if (nb <= FIN_R * 8 * NT) {
        double e[NV][FIN_R][8];
#pragma unroll
        for (int q = 0; q < NV; ++q)
#pragma unroll
            for (int r = 0; r < FIN_R; ++r)
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int b = tid + u * NT + 8 * NT * r;
                    e[q][r][u] = b < nb ? partials[(size_t)q * nb + b] : 0.0;
                }
#pragma unroll
        for (int q = 0; q < NV; ++q) {
            double a[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int r = 0; r < FIN_R; ++r)
#pragma unroll
                for (int u = 0; u < 8; ++u)
                    if (tid + u * NT + 8 * NT * r < nb) a[u] += e[q][r][u];
            v[q] = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
        }
    } else {
#pragma unroll
        for (int q = 0; q < NV; ++q) {
            const double *P = partials + (size_t)q * nb;
            double a[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
            int b = tid;
            for (; b + 7 * NT < nb; b += 8 * NT) {
#pragma unroll
                for (int u = 0; u < 8; ++u) a[u] += P[b + u * NT];
            }
#pragma unroll
            for (int u = 0; u < 8; ++u)
                if (b + u * NT < nb) a[u] += P[b + u * NT];
            v[q] = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
        }
    }
    __shared__ double out[NV];
    block_sum<NV>(v, out);
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NV; ++q) tot[q] = out[q];
}

// Each thread of a Bi-CGSTAB kernel covers KRY rows (fewer blocks, so fewer
// partial sums for the single-block finalisation).
constexpr int KRY = 4;

struct KDev {
    C<double> *b, *x, *r, *rh, *p, *v, *s, *t, *ph, *sh;
    double *partials, *hist;
    KState *st;
    int    *done_host;
};

static inline KDev kdev(const Krylov &K) {
    return KDev{(C<double> *)K.b,  (C<double> *)K.x, (C<double> *)K.r,  (C<double> *)K.rh,
                (C<double> *)K.p,  (C<double> *)K.v, (C<double> *)K.s,  (C<double> *)K.t,
                (C<double> *)K.ph, (C<double> *)K.sh, K.partials, K.hist, K.st, K.done_host};
}

// The pointers of right-hand side blockIdx.z in a batched launch: the
// vectors, partial sums and scalars of the slots lie zs bytes apart, the
// residual histories hz bytes, the pinned done flags one int.
__device__ __forceinline__ KDev kz(KDev K, long zs, long hz) {
    K.b = zsh(K.b, zs);
    K.x = zsh(K.x, zs);
    K.r = zsh(K.r, zs);
    K.rh = zsh(K.rh, zs);
    K.p = zsh(K.p, zs);
    K.v = zsh(K.v, zs);
    K.s = zsh(K.s, zs);
    K.t = zsh(K.t, zs);
    K.ph = zsh(K.ph, zs);
    K.sh = zsh(K.sh, zs);
    K.partials = zsh(K.partials, zs);
    K.hist = zsh(K.hist, hz);
    K.st = zsh(K.st, zs);
    K.done_host = zsh(K.done_host, zs ? (long)sizeof(int) : 0L);
    return K;
}

// The host polls the done flag of a running solve through a pinned copy
// that the kernels changing it write (a vector store to host memory), so no
// copy is queued behind every iteration.
__device__ __forceinline__ void publish_done(const KDev &K) {
    if (K.done_host) *(volatile int *)K.done_host = K.st->done;
}

__device__ __forceinline__ C<double> cdivc(C<double> a, C<double> b) { return cdiv(a, b.x, b.y); }
__device__ __forceinline__ C<double> ld2(const double *p) { return cmk(p[0], p[1]); }
__device__ __forceinline__ void st2(double *p, C<double> z) { p[0] = z.x; p[1] = z.y; }

// ---- init: r = b - L x (or r = b, x = 0), rh = r, p = v = 0 --------------
__global__ __launch_bounds__(NT) void k_kry_init(GeoT g, double H, double ih2, const double *__restrict__ k,
                                                 KDev K_, long zs, long hz, int x0_given) {
    const KDev K = kz(K_, zs, hz);
    int i = blockIdx.x * BX + threadIdx.x;
    double v[2] = {0.0, 0.0};
    for (int rr = 0; rr < KRY; ++rr) {
        int j = (blockIdx.y * KRY + rr) * BY + threadIdx.y;
        if (i > g.N || j > g.N) continue;
        size_t p = (size_t)j * g.M + i;
        C<double> bp = K.b[p], rp;
        if (x0_given) {
            Row<double> r = row_at<double>(i, j, g.N, H, ih2, k[p], 0.0);
            rp = csub(bp, row_apply(r, K.x, i, j, g.N, g.M));
        } else {
            K.x[p] = cmk(0.0, 0.0);
            rp = bp;
        }
        K.r[p] = rp;
        K.rh[p] = rp;
        K.p[p] = cmk(0.0, 0.0);
        K.v[p] = cmk(0.0, 0.0);
        v[0] += bp.x * bp.x + bp.y * bp.y;
        v[1] += rp.x * rp.x + rp.y * rp.y;
    }
    block_partials<2>(v, K.partials);
}

__global__ __launch_bounds__(NT) void k_kry_init_fin(KDev K_, long zs, long hz, int nb, double rtol, int maxhalf, int hist_cap,
                                                     int force_bd, int true_every, int nan_at) {
    const KDev K = kz(K_, zs, hz);
    double tot[2];
    finalize_sums<2>(K.partials, nb, tot);
    if (threadIdx.x || threadIdx.y) return;
    KState *s = K.st;
    double bn = sqrt(tot[0]);
    if (bn == 0.0) bn = 1.0;
    s->bnorm = bn;
    s->rnorm2 = tot[1];
    s->rhat_norm2 = tot[1];
    s->rho[0] = tot[1]; s->rho[1] = 0.0;
    s->rho_old[0] = 1.0; s->rho_old[1] = 0.0;
    s->alpha[0] = 1.0; s->alpha[1] = 0.0;
    s->omega[0] = 1.0; s->omega[1] = 0.0;
    s->beta[0] = 0.0; s->beta[1] = 0.0;
    s->rtol = rtol;
    s->halfsteps = 0;
    s->maxhalf = maxhalf;
    s->restart = 1;          // first p-update: p = r (p = v = 0, beta = rho)
    s->half_exit = 0;
    s->restarts = 0;
    s->hist_cap = hist_cap;
    s->force_bd = force_bd;
    s->true_every = true_every;
    s->nan_at = nan_at;
    s->fullits = 0;
    s->check = 0;
    double rel = sqrt(tot[1]) / bn;
    if (hist_cap > 0) K.hist[0] = rel;
    s->done = (rel <= rtol) ? 1 : 0;
    s->stop = s->done;
    s->true_rel = -1.0;
    publish_done(K);
}

// ---- p = r + beta (p - omega v); on restart rh = r and p = r ----------------
__global__ __launch_bounds__(NT) void k_kry_update_p(GeoT g, KDev K_, long zs, long hz) {
    const KDev K = kz(K_, zs, hz);
    const KState *s = K.st;
    const int done = flag_read(&s->done);
    int i = blockIdx.x * BX + threadIdx.x;
    const int restart = s->restart;
    C<double> beta = ld2(s->beta), omega = ld2(s->omega);
    C<double> r[KRY], pv[KRY], vv[KRY];
#pragma unroll
    for (int rr = 0; rr < KRY; ++rr) {
        int j = (blockIdx.y * KRY + rr) * BY + threadIdx.y;
        if (i > g.N || j > g.N) continue;
        size_t p = (size_t)j * g.M + i;
        r[rr] = K.r[p];
        pv[rr] = K.p[p];
        vv[rr] = K.v[p];
    }
    if (flag_set(done)) return;
#pragma unroll
    for (int rr = 0; rr < KRY; ++rr) {
        int j = (blockIdx.y * KRY + rr) * BY + threadIdx.y;
        if (i > g.N || j > g.N) continue;
        size_t p = (size_t)j * g.M + i;
        if (restart) {
            K.rh[p] = r[rr];
            K.p[p] = r[rr];
        } else {
            K.p[p] = cadd(r[rr], cmul(beta, csub(pv[rr], cmul(omega, vv[rr]))));
        }
    }
}

// ---- v = L ph, partial (rh, v) ----------------------------------------------
__global__ __launch_bounds__(NT) void k_kry_matvec_alpha(GeoT g, double H, double ih2, const double *__restrict__ k,
                                                         KDev K_, long zs, long hz) {
    const KDev K = kz(K_, zs, hz);
    if (K.st->done) return;
    int i = blockIdx.x * BX + threadIdx.x;
    double v[2] = {0.0, 0.0};
    for (int rr = 0; rr < KRY; ++rr) {
        int j = (blockIdx.y * KRY + rr) * BY + threadIdx.y;
        if (i > g.N || j > g.N) continue;
        size_t p = (size_t)j * g.M + i;
        Row<double> r = row_at<double>(i, j, g.N, H, ih2, k[p], 0.0);
        C<double> vp = row_apply(r, K.ph, i, j, g.N, g.M);
        K.v[p] = vp;
        C<double> a = K.rh[p];
        v[0] += a.x * vp.x + a.y * vp.y;      // conj(a) * vp
        v[1] += a.x * vp.y - a.y * vp.x;
    }
    block_partials<2>(v, K.partials);
}

__global__ __launch_bounds__(NT) void k_kry_alpha_fin(KDev K_, long zs, long hz, int nb) {
    const KDev K = kz(K_, zs, hz);
    const int done = flag_read(&K.st->done);
    double tot[2];
    finalize_sums<2>(K.partials, nb, tot);
    if (flag_set(done) || threadIdx.x || threadIdx.y) return;
    KState *s = K.st;
    s->restart = 0;
    st2(s->alpha, cdivc(ld2(s->rho), cmk(tot[0], tot[1])));
}

// ---- s = r - alpha v, partial ||s||^2 ----------------------------------------
__global__ __launch_bounds__(NT) void k_kry_update_s(GeoT g, KDev K_, long zs, long hz) {
    const KDev K = kz(K_, zs, hz);
    const int done = flag_read(&K.st->done);
    int i = blockIdx.x * BX + threadIdx.x;
    const C<double> alpha = ld2(K.st->alpha);
    C<double> r[KRY], vv[KRY];
#pragma unroll
    for (int rr = 0; rr < KRY; ++rr) {
        int j = (blockIdx.y * KRY + rr) * BY + threadIdx.y;
        if (i > g.N || j > g.N) continue;
        size_t p = (size_t)j * g.M + i;
        r[rr] = K.r[p];
        vv[rr] = K.v[p];
    }
    if (flag_set(done)) return;
    double v[1] = {0.0};
#pragma unroll
    for (int rr = 0; rr < KRY; ++rr) {
        int j = (blockIdx.y * KRY + rr) * BY + threadIdx.y;
        if (i > g.N || j > g.N) continue;
        size_t p = (size_t)j * g.M + i;
        C<double> sp = csub(r[rr], cmul(alpha, vv[rr]));
        K.s[p] = sp;
        v[0] += sp.x * sp.x + sp.y * sp.y;
    }
    block_partials<1>(v, K.partials);
}

__global__ __launch_bounds__(NT) void k_kry_s_fin(KDev K_, long zs, long hz, int nb) {
    const KDev K = kz(K_, zs, hz);
    const int done = flag_read(&K.st->done);
    double tot[1];
    finalize_sums<1>(K.partials, nb, tot);
    if (flag_set(done) || threadIdx.x || threadIdx.y) return;
    KState *s = K.st;
    s->halfsteps += 1;
    s->snorm2 = tot[0];
    double rel = sqrt(tot[0]) / s->bnorm;
    if (s->halfsteps < s->hist_cap) K.hist[s->halfsteps] = rel;
    if (!isfinite(rel)) {   // not finite: end with the iterate of the last full step
        s->done = 3;
        s->stop = 1;
        publish_done(K);
        return;
    }
    if (rel <= s->rtol) {
        s->half_exit = 1;
        s->stop = 1;
    }
}

// ---- t = L sh, partials (t, s), (t, t) -----------------------------------------
__global__ __launch_bounds__(NT) void k_kry_matvec_omega(GeoT g, double H, double ih2, const double *__restrict__ k,
                                                         KDev K_, long zs, long hz) {
    const KDev K = kz(K_, zs, hz);
    if (K.st->stop) return;
    int i = blockIdx.x * BX + threadIdx.x;
    double v[3] = {0.0, 0.0, 0.0};
    for (int rr = 0; rr < KRY; ++rr) {
        int j = (blockIdx.y * KRY + rr) * BY + threadIdx.y;
        if (i > g.N || j > g.N) continue;
        size_t p = (size_t)j * g.M + i;
        Row<double> r = row_at<double>(i, j, g.N, H, ih2, k[p], 0.0);
        C<double> tp = row_apply(r, K.sh, i, j, g.N, g.M);
        K.t[p] = tp;
        C<double> sp = K.s[p];
        v[0] += tp.x * sp.x + tp.y * sp.y;    // conj(t) s
        v[1] += tp.x * sp.y - tp.y * sp.x;
        v[2] += tp.x * tp.x + tp.y * tp.y;
    }
    block_partials<3>(v, K.partials);
}

__global__ __launch_bounds__(NT) void k_kry_omega_fin(KDev K_, long zs, long hz, int nb) {
    const KDev K = kz(K_, zs, hz);
    const int stop = flag_read(&K.st->stop);
    double tot[3];
    finalize_sums<3>(K.partials, nb, tot);
    if (flag_set(stop) || threadIdx.x || threadIdx.y) return;
    st2(K.st->omega, cdivc(cmk(tot[0], tot[1]), cmk(tot[2], 0.0)));
}

// ---- x += alpha ph + omega sh; r = s - omega t; partials ||r||^2, (rh, r) -----
__global__ __launch_bounds__(NT) void k_kry_update_xr(GeoT g, KDev K_, long zs, long hz) {
    const KDev K = kz(K_, zs, hz);
    const KState *s = K.st;
    const int done = flag_read(&s->done);
    const int half = s->half_exit;
    const C<double> alpha = ld2(s->alpha), omega = ld2(s->omega);
    int i = blockIdx.x * BX + threadIdx.x;
    double v[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int rr = 0; rr < KRY; ++rr) {
        int j = (blockIdx.y * KRY + rr) * BY + threadIdx.y;
        const bool in = i <= g.N && j <= g.N;
        size_t p = in ? (size_t)j * g.M + i : 0;
        // the first row's fields are requested before the flag is tested
        const C<double> xp = K.x[p], php = K.ph[p];
        if (rr == 0 && flag_set(done)) return;
        if (!in) continue;
        if (half) {
            K.x[p] = cadd(xp, cmul(alpha, php));
        } else {
            K.x[p] = cadd(xp, cadd(cmul(alpha, php), cmul(omega, K.sh[p])));
            C<double> rp = csub(K.s[p], cmul(omega, K.t[p]));
            K.r[p] = rp;
            C<double> a = K.rh[p];
            v[0] += rp.x * rp.x + rp.y * rp.y;
            v[1] += a.x * rp.x + a.y * rp.y;  // conj(rh) r
            v[2] += a.x * rp.y - a.y * rp.x;
        }
    }
    if (!half) block_partials<3>(v, K.partials);
}

// ---- the same with the update of x kept in the preconditioner's input space:
// y += alpha p + omega s (y in the p^ buffer), x = x + B y formed once at the
// end (k_kry_fold).  B is linear and fixed, so x is the same as with
// x += alpha p^ + omega s^ in exact arithmetic, and p^, s^ need not be stored.
__global__ __launch_bounds__(NT) void k_kry_update_yr(GeoT g, KDev K_, long zs, long hz) {
    const KDev K = kz(K_, zs, hz);
    const KState *s = K.st;
    const int done = flag_read(&s->done);
    const int half = s->half_exit;
    const C<double> alpha = ld2(s->alpha), omega = ld2(s->omega);
    C<double> *y = K.ph;
    int i = blockIdx.x * BX + threadIdx.x;
    double v[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int rr = 0; rr < KRY; ++rr) {
        int j = (blockIdx.y * KRY + rr) * BY + threadIdx.y;
        const bool in = i <= g.N && j <= g.N;
        size_t p = in ? (size_t)j * g.M + i : 0;
        // the first row's fields are requested before the flag is tested
        const C<double> yp = y[p], pp = K.p[p];
        if (rr == 0 && flag_set(done)) return;
        if (!in) continue;
        if (half) {
            y[p] = cadd(yp, cmul(alpha, pp));
        } else {
            const C<double> sp = K.s[p];
            y[p] = cadd(yp, cadd(cmul(alpha, pp), cmul(omega, sp)));
            C<double> rp = csub(sp, cmul(omega, K.t[p]));
            K.r[p] = rp;
            C<double> a = K.rh[p];
            v[0] += rp.x * rp.x + rp.y * rp.y;
            v[1] += a.x * rp.x + a.y * rp.y;  // conj(rh) r
            v[2] += a.x * rp.y - a.y * rp.x;
        }
    }
    if (!half) block_partials<3>(v, K.partials);
}

// ---- x += z (z = B y in the s^ buffer), y = 0 --------------------------------
__global__ __launch_bounds__(NT) void k_kry_fold(GeoT g, KDev K_, long zs, long hz) {
    const KDev K = kz(K_, zs, hz);
    int i = blockIdx.x * BX + threadIdx.x;
    for (int rr = 0; rr < KRY; ++rr) {
        int j = (blockIdx.y * KRY + rr) * BY + threadIdx.y;
        if (i > g.N || j > g.N) continue;
        size_t p = (size_t)j * g.M + i;
        K.x[p] = cadd(K.x[p], K.sh[p]);
        K.ph[p] = cmk(0.0, 0.0);
    }
}

__global__ __launch_bounds__(NT) void k_kry_iter_fin(KDev K_, long zs, long hz, int nb) {
    const KDev K = kz(K_, zs, hz);
    KState *s = K.st;
    const int done = flag_read(&s->done);
    const int half = s->half_exit;
    double tot[3];
    finalize_sums<3>(K.partials, nb, tot);     // unused after a half step
    if (flag_set(done)) return;
    if (half) {
        if (threadIdx.x == 0 && threadIdx.y == 0) {
            s->done = 1;
            s->stop = 1;
            publish_done(K);
        }
        return;
    }
    if (threadIdx.x || threadIdx.y) return;
    s->halfsteps += 1;
    s->rnorm2 = tot[0];
    double rn = sqrt(tot[0]);
    if (s->nan_at > 0 && s->halfsteps == 2 * s->nan_at) rn = __builtin_nan("");
    double rel = rn / s->bnorm;
    if (s->halfsteps < s->hist_cap) K.hist[s->halfsteps] = rel;
    if (!isfinite(rel)) {
        s->done = 3;
        s->stop = 1;
        publish_done(K);
        return;
    }
    if (rel <= s->rtol) {
        s->done = 1;
        s->stop = 1;
        publish_done(K);
        return;
    }
    if (s->halfsteps >= s->maxhalf) {
        s->done = 2;
        s->stop = 1;
        publish_done(K);
        return;
    }
    if (s->true_every > 0 && ++s->fullits % s->true_every == 0) {
        // the check kernels that follow recompute r and restart from it
        s->check = 1;
        return;
    }
    C<double> rho_new = cmk(tot[1], tot[2]);
    double mag = sqrt(rho_new.x * rho_new.x + rho_new.y * rho_new.y);
    if (mag <= 1e-14 * sqrt(s->rhat_norm2) * rn || s->halfsteps == 2 * s->force_bd) {
        // breakdown (or the one forced after iteration force_bd): restart
        // with rh = r
        s->restart = 1;
        s->restarts += 1;
        s->rho[0] = tot[0]; s->rho[1] = 0.0;
        s->rho_old[0] = 1.0; s->rho_old[1] = 0.0;
        s->alpha[0] = 1.0; s->alpha[1] = 0.0;
        s->omega[0] = 1.0; s->omega[1] = 0.0;
        s->rhat_norm2 = tot[0];
        return;
    }
    C<double> rho = ld2(s->rho);
    C<double> beta = cmul(cdivc(rho_new, rho), cdivc(ld2(s->alpha), ld2(s->omega)));
    st2(s->beta, beta);
    st2(s->rho_old, rho);
    st2(s->rho, rho_new);
}

// ---- true residual r = b - L x, ||r||^2 ----------------------------------------
__global__ __launch_bounds__(NT) void k_kry_true(GeoT g, double H, double ih2, const double *__restrict__ k,
                                                 KDev K_, long zs, long hz) {
    const KDev K = kz(K_, zs, hz);
    int i = blockIdx.x * BX + threadIdx.x;
    double v[1] = {0.0};
    for (int rr = 0; rr < KRY; ++rr) {
        int j = (blockIdx.y * KRY + rr) * BY + threadIdx.y;
        if (i > g.N || j > g.N) continue;
        size_t p = (size_t)j * g.M + i;
        Row<double> r = row_at<double>(i, j, g.N, H, ih2, k[p], 0.0);
        C<double> rp = csub(K.b[p], row_apply(r, K.x, i, j, g.N, g.M));
        K.r[p] = rp;
        v[0] += rp.x * rp.x + rp.y * rp.y;
    }
    block_partials<1>(v, K.partials);
}

__global__ __launch_bounds__(NT) void k_kry_true_fin(KDev K_, long zs, long hz, int nb) {
    const KDev K = kz(K_, zs, hz);
    double tot[1];
    finalize_sums<1>(K.partials, nb, tot);
    if (threadIdx.x || threadIdx.y) return;
    KState *s = K.st;
    s->rnorm2 = tot[0];
    s->true_rel = sqrt(tot[0]) / s->bnorm;
}

// restart from the recomputed residual: rh = r, p = r on the next update
__global__ void k_kry_restart(KDev K_, long zs, long hz) {
    const KDev K = kz(K_, zs, hz);
    KState *s = K.st;
    s->restart = 1;
    s->restarts += 1;
    s->rho[0] = s->rnorm2; s->rho[1] = 0.0;
    s->rho_old[0] = 1.0; s->rho_old[1] = 0.0;
    s->alpha[0] = 1.0; s->alpha[1] = 0.0;
    s->omega[0] = 1.0; s->omega[1] = 0.0;
    s->rhat_norm2 = s->rnorm2;
    s->done = 0;
    s->half_exit = 0;
    s->stop = 0;
    publish_done(K);
}

// ---- the periodic true-residual check (only when iter_fin marked it due) --
__global__ __launch_bounds__(NT) void k_kry_check_true(GeoT g, double H, double ih2, const double *__restrict__ k,
                                                       KDev K_, long zs, long hz) {
    const KDev K = kz(K_, zs, hz);
    if (!K.st->check) return;
    int i = blockIdx.x * BX + threadIdx.x;
    double v[1] = {0.0};
    for (int rr = 0; rr < KRY; ++rr) {
        int j = (blockIdx.y * KRY + rr) * BY + threadIdx.y;
        if (i > g.N || j > g.N) continue;
        size_t p = (size_t)j * g.M + i;
        Row<double> r = row_at<double>(i, j, g.N, H, ih2, k[p], 0.0);
        C<double> rp = csub(K.b[p], row_apply(r, K.x, i, j, g.N, g.M));
        K.r[p] = rp;
        v[0] += rp.x * rp.x + rp.y * rp.y;
    }
    block_partials<1>(v, K.partials);
}

__global__ __launch_bounds__(NT) void k_kry_check_fin(KDev K_, long zs, long hz, int nb) {
    const KDev K = kz(K_, zs, hz);
    KState *s = K.st;
    if (!s->check) return;
    double tot[1];
    finalize_sums<1>(K.partials, nb, tot);
    if (threadIdx.x || threadIdx.y) return;
    s->check = 0;
    s->rnorm2 = tot[0];
    const double rel = sqrt(tot[0]) / s->bnorm;
    s->true_rel = rel;
    if (!isfinite(rel)) {
        s->done = 3;
        s->stop = 1;
    } else if (rel <= s->rtol) {
        s->done = 1;        // confirmed again by the solve's final check
        s->stop = 1;
    } else {
        s->restart = 1;
        s->restarts += 1;
        s->rho[0] = tot[0]; s->rho[1] = 0.0;
        s->rho_old[0] = 1.0; s->rho_old[1] = 0.0;
        s->alpha[0] = 1.0; s->alpha[1] = 0.0;
        s->omega[0] = 1.0; s->omega[1] = 0.0;
        s->rhat_norm2 = tot[0];
    }
    publish_done(K);
}

static inline dim3 kgrid(const Geo &g, int nz = 1) {
    return dim3((g.M + BX - 1) / BX, (g.M + BY * KRY - 1) / (BY * KRY), nz);
}

int krylov_nblocks(const Geo &g) {
    dim3 gr = kgrid(g);
    return (int)(gr.x * gr.y);
}

static inline void hk(const Geo &g, double &H, double &ih2) { H = g.H; ih2 = 1.0 / (g.H * g.H); }

// Every launcher below runs on one solve slot K, or batched (kb.nz > 1) on the
// kb.nz slots from K on.
static inline dim3 one(int nz) { return dim3(1, 1, nz); }

void kry_init(hipStream_t s, const Geo &g, const double *k, const Krylov &K, int x0_given, double rtol,
              int maxhalf, int force_bd, int true_every, int nan_at, Kz kb) {
    double H, ih2;
    hk(g, H, ih2);
    KDev d = kdev(K);
    k_kry_init<<<kgrid(g, kb.nz), dim3(BX, BY), 0, s>>>(geot(g), H, ih2, k, d, kb.zs, kb.hz, x0_given);
    // the history buffer holds maxhalf + 2 entries (allocated by the caller)
    k_kry_init_fin<<<one(kb.nz), dim3(BX, BY), 0, s>>>(d, kb.zs, kb.hz, K.nblocks, rtol, maxhalf, maxhalf + 2, force_bd,
                                                    true_every, nan_at);
}
void kry_checkpoint(hipStream_t s, const Geo &g, const double *k, const Krylov &K, Kz kb) {
    double H, ih2;
    hk(g, H, ih2);
    KDev d = kdev(K);
    k_kry_check_true<<<kgrid(g, kb.nz), dim3(BX, BY), 0, s>>>(geot(g), H, ih2, k, d, kb.zs, kb.hz);
    k_kry_check_fin<<<one(kb.nz), dim3(BX, BY), 0, s>>>(d, kb.zs, kb.hz, K.nblocks);
}
void kry_update_p(hipStream_t s, const Geo &g, const Krylov &K, Kz kb) {
    k_kry_update_p<<<kgrid(g, kb.nz), dim3(BX, BY), 0, s>>>(geot(g), kdev(K), kb.zs, kb.hz);
}
void kry_matvec_alpha(hipStream_t s, const Geo &g, const double *k, const Krylov &K, Kz kb) {
    double H, ih2;
    hk(g, H, ih2);
    KDev d = kdev(K);
    k_kry_matvec_alpha<<<kgrid(g, kb.nz), dim3(BX, BY), 0, s>>>(geot(g), H, ih2, k, d, kb.zs, kb.hz);
    k_kry_alpha_fin<<<one(kb.nz), dim3(BX, BY), 0, s>>>(d, kb.zs, kb.hz, K.nblocks);
}
// partial sums of nv quantities over nb blocks -> out[0..2] (zero-padded)
__global__ __launch_bounds__(NT) void k_sum_partials(const double *partials, int nb, int nv, double *out) {
    double tot[3];
    if (nv == 2) finalize_sums<2>(partials, nb, tot);
    else finalize_sums<3>(partials, nb, tot);
    if (threadIdx.x || threadIdx.y) return;
    for (int q = 0; q < 3; ++q) out[q] = q < nv ? tot[q] : 0.0;
}
void launch_sum_partials(hipStream_t s, const double *partials, int nb, int nv, double *out) {
    k_sum_partials<<<1, dim3(BX, BY), 0, s>>>(partials, nb, nv, out);
}
void kry_alpha_fin(hipStream_t s, const Krylov &K, int nb, Kz kb) {
    k_kry_alpha_fin<<<one(kb.nz), dim3(BX, BY), 0, s>>>(kdev(K), kb.zs, kb.hz, nb);
}
void kry_omega_fin(hipStream_t s, const Krylov &K, int nb, Kz kb) {
    k_kry_omega_fin<<<one(kb.nz), dim3(BX, BY), 0, s>>>(kdev(K), kb.zs, kb.hz, nb);
}
void kry_update_s(hipStream_t s, const Geo &g, const Krylov &K, Kz kb) {
    KDev d = kdev(K);
    k_kry_update_s<<<kgrid(g, kb.nz), dim3(BX, BY), 0, s>>>(geot(g), d, kb.zs, kb.hz);
    k_kry_s_fin<<<one(kb.nz), dim3(BX, BY), 0, s>>>(d, kb.zs, kb.hz, K.nblocks);
}
void kry_matvec_omega(hipStream_t s, const Geo &g, const double *k, const Krylov &K, Kz kb) {
    double H, ih2;
    hk(g, H, ih2);
    KDev d = kdev(K);
    k_kry_matvec_omega<<<kgrid(g, kb.nz), dim3(BX, BY), 0, s>>>(geot(g), H, ih2, k, d, kb.zs, kb.hz);
    k_kry_omega_fin<<<one(kb.nz), dim3(BX, BY), 0, s>>>(d, kb.zs, kb.hz, K.nblocks);
}
void kry_update_xr(hipStream_t s, const Geo &g, const Krylov &K, Kz kb) {
    KDev d = kdev(K);
    k_kry_update_xr<<<kgrid(g, kb.nz), dim3(BX, BY), 0, s>>>(geot(g), d, kb.zs, kb.hz);
    k_kry_iter_fin<<<one(kb.nz), dim3(BX, BY), 0, s>>>(d, kb.zs, kb.hz, K.nblocks);
}
void kry_update_yr(hipStream_t s, const Geo &g, const Krylov &K, Kz kb) {
    KDev d = kdev(K);
    k_kry_update_yr<<<kgrid(g, kb.nz), dim3(BX, BY), 0, s>>>(geot(g), d, kb.zs, kb.hz);
    k_kry_iter_fin<<<one(kb.nz), dim3(BX, BY), 0, s>>>(d, kb.zs, kb.hz, K.nblocks);
}
void kry_fold(hipStream_t s, const Geo &g, const Krylov &K) {
    k_kry_fold<<<kgrid(g), dim3(BX, BY), 0, s>>>(geot(g), kdev(K), 0L, 0L);
}
void kry_true_residual(hipStream_t s, const Geo &g, const double *k, const Krylov &K) {
    double H, ih2;
    hk(g, H, ih2);
    KDev d = kdev(K);
    k_kry_true<<<kgrid(g), dim3(BX, BY), 0, s>>>(geot(g), H, ih2, k, d, 0L, 0L);
    k_kry_true_fin<<<1, dim3(BX, BY), 0, s>>>(d, 0L, 0L, K.nblocks);
}
void kry_restart_from_true(hipStream_t s, const Krylov &K) { k_kry_restart<<<1, 1, 0, s>>>(kdev(K), 0L, 0L); }

}  // namespace hmgk
