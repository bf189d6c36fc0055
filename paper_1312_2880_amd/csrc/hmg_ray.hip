// hmg_ray.hip -- the ray correction of Section 6.1 on the finest grid.
//
// Near-kernel error is a sum over the 8 directions j = 1..8 of plane waves
// exp(i kr (cos(j pi/4) x + sin(j pi/4) y)) times smooth ray functions.  The
// ray functions are bilinear on a vertex-centred ray grid (nr interior nodes
// per side over the fine grid's square, cells of c fine intervals), so the
// correction space is spanned by P e_(d,a) = wave_d(x) phi_a(x) and the
// correction of z for a right-hand side r is the Galerkin one:
//     z += P A^{-1} P^H (r - L z),   A = P^H L P.
// Kernels (all FP64, batched over right-hand sides by blockIdx.z):
//   k_ray_restrict  w = r - L z on a patch of P x P fine nodes inside one ray
//                   cell and its 8 x 4 partial sums conj(wave_d) phi_a w for
//                   the cell's corners (one record of 64 doubles per patch);
//   k_ray_gather    b(d, a) = the sum of its records over the cells around a,
//                   in a fixed order (results do not depend on scheduling);
//   k_ray_solve     a = A^{-1} b (dense inverse, one workgroup per row);
//   k_ray_prolong   z += sum_d wave_d (bilinear interpolation of a_d).
// The wave factors are products of two 1-D tables formed on the host,
// wave_d(i h, j h) = ex[d][i] ey[d][j].

#include "hmg_device.h"

namespace hmgk {

__device__ __forceinline__ C<double> cconjmul(C<double> a, C<double> b) {   // conj(a) b
    return cmk(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}

// the ray cell of fine index i (cells [I c, (I + 1) c), the last one closed)
// and the position in it, as the weight of the cell's upper corner
__device__ __forceinline__ void ray_cell(int i, const RayGeo &R, int &I, double &w) {
    I = min(i / R.c, R.Nr - 1);
    w = (double)(i - I * R.c) / (double)R.c;
}

template <int P>
__global__ __launch_bounds__(P *P) void k_ray_restrict(RayGeo R, double H, double ih2, const double *__restrict__ k,
                                                       const C<double> *__restrict__ ex,
                                                       const C<double> *__restrict__ ey,
                                                       const C<double> *__restrict__ r,
                                                       const C<double> *__restrict__ z, double *__restrict__ part,
                                                       const int *skip, long zs) {
    r = zsh(r, zs);
    z = zsh(z, zs);
    part = zsh(part, zs);
    skip = zsh(skip, zs);
    const int sk = flag_read(skip);
    constexpr int NTH = P * P, NW = NTH / 64;
    __shared__ double red[64][NW];
    const int tx = threadIdx.x % P, ty = threadIdx.x / P;
    const int i = blockIdx.x * P + tx, j = blockIdx.y * P + ty;
    const bool in = i <= R.N && j <= R.N;
    C<double> w = cmk(0.0, 0.0);
    if (in) {
        const size_t p = (size_t)j * R.M + i;
        const Row<double> row = row_at<double>(i, j, R.N, H, ih2, k[p], 0.0);
        const C<double> lz = row_apply(row, z, i, j, R.N, R.M);
        w = r ? csub(r[p], lz) : cmk(-lz.x, -lz.y);
    }
    if (flag_set(sk)) return;
    int I, J;
    double wx, wy;
    ray_cell(min(i, R.N), R, I, wx);
    ray_cell(min(j, R.N), R, J, wy);
    const double h4[4] = {(1.0 - wx) * (1.0 - wy), wx * (1.0 - wy), (1.0 - wx) * wy, wx * wy};
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int d = 0; d < 8; ++d) {
        C<double> t = cmk(0.0, 0.0);
        if (in) t = cconjmul(cmul(ex[d * R.M + i], ey[d * R.M + j]), w);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            double vx = h4[q] * t.x, vy = h4[q] * t.y;
            for (int off = 32; off > 0; off >>= 1) {
                vx += __shfl_xor(vx, off, 64);
                vy += __shfl_xor(vy, off, 64);
            }
            if (lane == 0) {
                red[(q * 8 + d) * 2][wave] = vx;
                red[(q * 8 + d) * 2 + 1][wave] = vy;
            }
        }
    }
    __syncthreads();
    if (threadIdx.x < 64) {
        double v = red[threadIdx.x][0];
        for (int q = 1; q < NW; ++q) v += red[threadIdx.x][q];
        part[(size_t)(blockIdx.y * R.np + blockIdx.x) * 64 + threadIdx.x] = v;
    }
}

// b(d, a), a = JA Mr + IA: the records of every patch of the (up to four)
// cells that have a as a corner, cells and patches in a fixed order
__global__ __launch_bounds__(256) void k_ray_gather(RayGeo R, const double *__restrict__ part,
                                                    C<double> *__restrict__ b, const int *skip, long zs) {
    part = zsh(part, zs);
    b = zsh(b, zs);
    skip = zsh(skip, zs);
    if (skip && *skip) return;
    const int K = 8 * R.Mr * R.Mr;
    const int t = blockIdx.x * 256 + threadIdx.x;
    if (t >= K) return;
    const int d = t / (R.Mr * R.Mr), a = t % (R.Mr * R.Mr), IA = a % R.Mr, JA = a / R.Mr;
    const int pc = R.c / R.P;    // patches per cell side (the last cell has one more)
    double sx = 0.0, sy = 0.0;
    for (int J = JA - 1; J <= JA; ++J) {
        if (J < 0 || J >= R.Nr) continue;
        const int py0 = J * pc, py1 = (J == R.Nr - 1) ? R.np : py0 + pc;
        for (int I = IA - 1; I <= IA; ++I) {
            if (I < 0 || I >= R.Nr) continue;
            const int px0 = I * pc, px1 = (I == R.Nr - 1) ? R.np : px0 + pc;
            const int q = (IA - I) + 2 * (JA - J);
            for (int py = py0; py < py1; ++py)
                for (int px = px0; px < px1; ++px) {
                    const double *rec = part + (size_t)(py * R.np + px) * 64 + (q * 8 + d) * 2;
                    sx += rec[0];
                    sy += rec[1];
                }
        }
    }
    b[t] = cmk(sx, sy);
}

// a = A^{-1} b, A^{-1} dense row-major (K x K): one workgroup per row, fixed-
// order sums
__global__ __launch_bounds__(256) void k_ray_solve(const C<double> *__restrict__ Ainv, int K,
                                                   const C<double> *__restrict__ b, C<double> *__restrict__ a,
                                                   const int *skip, long zs) {
    b = zsh(b, zs);
    a = zsh(a, zs);
    skip = zsh(skip, zs);
    if (skip && *skip) return;
    __shared__ double red[2][4];
    const int row = blockIdx.x, tid = threadIdx.x;
    const C<double> *Ar = Ainv + (size_t)row * K;
    double sx = 0.0, sy = 0.0;
    for (int c = tid; c < K; c += 256) {
        const C<double> v = cmul(Ar[c], b[c]);
        sx += v.x;
        sy += v.y;
    }
    for (int off = 32; off > 0; off >>= 1) {
        sx += __shfl_xor(sx, off, 64);
        sy += __shfl_xor(sy, off, 64);
    }
    if ((tid & 63) == 0) {
        red[0][tid >> 6] = sx;
        red[1][tid >> 6] = sy;
    }
    __syncthreads();
    if (tid == 0) a[row] = cmk(((red[0][0] + red[0][1]) + red[0][2]) + red[0][3],
                               ((red[1][0] + red[1][1]) + red[1][2]) + red[1][3]);
}

// z += sum_d wave_d (bilinear interpolation of a_d)
__global__ __launch_bounds__(256) void k_ray_prolong(RayGeo R, const C<double> *__restrict__ ex,
                                                     const C<double> *__restrict__ ey,
                                                     const C<double> *__restrict__ a, C<double> *__restrict__ z,
                                                     const int *skip, long zs) {
    a = zsh(a, zs);
    z = zsh(z, zs);
    skip = zsh(skip, zs);
    const int sk = flag_read(skip);
    const int i = blockIdx.x * 64 + (threadIdx.x & 63), j = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (i > R.N || j > R.N) return;
    const size_t p = (size_t)j * R.M + i;
    const C<double> z0 = z[p];
    if (flag_set(sk)) return;
    int I, J;
    double wx, wy;
    ray_cell(i, R, I, wx);
    ray_cell(j, R, J, wy);
    const int a00 = J * R.Mr + I, MM = R.Mr * R.Mr;
    C<double> acc = cmk(0.0, 0.0);
#pragma unroll
    for (int d = 0; d < 8; ++d) {
        const C<double> *ad = a + (size_t)d * MM;
        const C<double> e0 = cadd(cscale(1.0 - wx, ad[a00]), cscale(wx, ad[a00 + 1]));
        const C<double> e1 = cadd(cscale(1.0 - wx, ad[a00 + R.Mr]), cscale(wx, ad[a00 + R.Mr + 1]));
        const C<double> e = cadd(cscale(1.0 - wy, e0), cscale(wy, e1));
        acc = cadd(acc, cmul(cmul(ex[d * R.M + i], ey[d * R.M + j]), e));
    }
    z[p] = cadd(z0, acc);
}

// unit vector e_col of length K (the setup's ray coefficients)
__global__ __launch_bounds__(256) void k_ray_unit(C<double> *a, int K, int col) {
    const int t = blockIdx.x * 256 + threadIdx.x;
    if (t < K) a[t] = cmk(t == col ? 1.0 : 0.0, 0.0);
}

// column col of A = P^H L P from b = P^H (0 - L P e_col) (negated)
__global__ __launch_bounds__(256) void k_ray_column(const C<double> *__restrict__ b, C<double> *__restrict__ A,
                                                    int K, int col) {
    const int t = blockIdx.x * 256 + threadIdx.x;
    if (t < K) A[(size_t)t * K + col] = cmk(-b[t].x, -b[t].y);
}

static inline dim3 fine_grid(const RayGeo &R, int nz) { return dim3((R.M + 63) / 64, (R.M + 3) / 4, nz); }

void launch_ray_correct(hipStream_t s, const RayGeo &R, double H, const double *k, const void *ex, const void *ey,
                        const double *Ainv, const void *r, void *z, double *part, void *b, void *a,
                        const int *skip, Bz bz) {
    const double ih2 = 1.0 / (H * H);
    const int K = 8 * R.Mr * R.Mr;
    const dim3 pg(R.np, R.np, bz.nz);
    if (R.P == 16)
        k_ray_restrict<16><<<pg, 256, 0, s>>>(R, H, ih2, k, (const C<double> *)ex, (const C<double> *)ey,
                                              (const C<double> *)r, (const C<double> *)z, part, skip, bz.zs);
    else
        k_ray_restrict<8><<<pg, 64, 0, s>>>(R, H, ih2, k, (const C<double> *)ex, (const C<double> *)ey,
                                            (const C<double> *)r, (const C<double> *)z, part, skip, bz.zs);
    k_ray_gather<<<dim3((K + 255) / 256, 1, bz.nz), 256, 0, s>>>(R, part, (C<double> *)b, skip, bz.zs);
    k_ray_solve<<<dim3(K, 1, bz.nz), 256, 0, s>>>((const C<double> *)Ainv, K, (const C<double> *)b, (C<double> *)a,
                                                  skip, bz.zs);
    k_ray_prolong<<<fine_grid(R, bz.nz), 256, 0, s>>>(R, (const C<double> *)ex, (const C<double> *)ey,
                                                      (const C<double> *)a, (C<double> *)z, skip, bz.zs);
}

void launch_ray_column(hipStream_t s, const RayGeo &R, double H, const double *k, const void *ex, const void *ey,
                       void *zfine, double *part, void *b, void *a, void *A, int col) {
    const double ih2 = 1.0 / (H * H);
    const int K = 8 * R.Mr * R.Mr;
    (void)hipMemsetAsync(zfine, 0, (size_t)R.M * R.M * 16, s);
    k_ray_unit<<<(K + 255) / 256, 256, 0, s>>>((C<double> *)a, K, col);
    k_ray_prolong<<<fine_grid(R, 1), 256, 0, s>>>(R, (const C<double> *)ex, (const C<double> *)ey,
                                                  (const C<double> *)a, (C<double> *)zfine, nullptr, 0);
    const dim3 pg(R.np, R.np, 1);
    if (R.P == 16)
        k_ray_restrict<16><<<pg, 256, 0, s>>>(R, H, ih2, k, (const C<double> *)ex, (const C<double> *)ey, nullptr,
                                              (const C<double> *)zfine, part, nullptr, 0);
    else
        k_ray_restrict<8><<<pg, 64, 0, s>>>(R, H, ih2, k, (const C<double> *)ex, (const C<double> *)ey, nullptr,
                                            (const C<double> *)zfine, part, nullptr, 0);
    k_ray_gather<<<(K + 255) / 256, 256, 0, s>>>(R, part, (C<double> *)b, nullptr, 0);
    k_ray_column<<<(K + 255) / 256, 256, 0, s>>>((const C<double> *)b, (C<double> *)A, K, col);
}

}  // namespace hmgk
