// hmg_device.h -- device-side helpers shared by the kernel translation units
// of libhmg: complex arithmetic in the level precision and the rows of the
// discrete operator.
//
// Discrete operator (Section 1, eq:diff / eq:disc / eq:mh), for node p =
// (i, j) on a level with spacing H and N = n+1 intervals:
//   a_pp = (-4 + 2 i k_p H b_p) / H^2 + k_p^2 (1 + i sigma)
//   a_pq = w_pq / H^2,  w_pq = 2 for the inward neighbour across a boundary
//                       face of p, 1 otherwise,
// with b_p the number of boundary faces of p.  This is the 5-point stencil
// with the Sommerfeld condition du/dn - i k u = 0 closed by central-
// difference ghost points; sigma = 0 gives L, sigma = beta gives M.
#pragma once

#include "hmg_internal.h"

#include <type_traits>

namespace hmgk {


template <typename T>
struct __attribute__((aligned(2 * sizeof(T)))) C {
    T x, y;
};

template <typename T> __device__ __forceinline__ C<T> cmk(T a, T b) { C<T> z; z.x = a; z.y = b; return z; }
template <typename T> __device__ __forceinline__ C<T> cadd(C<T> a, C<T> b) { return cmk(a.x + b.x, a.y + b.y); }
template <typename T> __device__ __forceinline__ C<T> csub(C<T> a, C<T> b) { return cmk(a.x - b.x, a.y - b.y); }
template <typename T> __device__ __forceinline__ C<T> cscale(T s, C<T> a) { return cmk(s * a.x, s * a.y); }
template <typename T> __device__ __forceinline__ C<T> cmul(C<T> a, C<T> b) {
    return cmk(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// 1 / x for a positive normal x: the hardware reciprocal (about 24 correct
// bits) refined by two Newton-Raphson steps r <- r + r (1 - x r), each of
// which doubles the correct bits; five instructions instead of the
// scale/fix-up sequence of an IEEE division.
__device__ __forceinline__ double rcp_pos(double x) {
    double r = __builtin_amdgcn_rcp(x);
    double e = __builtin_fma(-x, r, 1.0);
    r = __builtin_fma(r, e, r);
    e = __builtin_fma(-x, r, 1.0);
    return __builtin_fma(r, e, r);
}
__device__ __forceinline__ float rcp_pos(float x) { return 1.0f / x; }

// a / (dre + i dim), (dre, dim) != 0
template <typename T> __device__ __forceinline__ C<T> cdiv(C<T> a, T dre, T dim) {
    T inv = rcp_pos(dre * dre + dim * dim);
    return cmk((a.x * dre + a.y * dim) * inv, (a.y * dre - a.x * dim) * inv);
}

// a / (dre + i dim) with inv = 1 / (dre^2 + dim^2) computed by the caller
template <typename T> __device__ __forceinline__ C<T> cdivr(C<T> a, T dre, T dim, T inv) {
    return cmk((a.x * dre + a.y * dim) * inv, (a.y * dre - a.x * dim) * inv);
}

constexpr int BX = 64, BY = 4, NT = BX * BY;

// Row p of A_sigma: diagonal (dre + i dim) and neighbour weights / H^2.
template <typename T>
struct Row {
    T dre, dim, wl, wr, wd, wu;
};

template <typename T>
__device__ __forceinline__ Row<T> row_at(int i, int j, int N, T H, T ih2, T kp, T sigma) {
    Row<T> r;
    int b = (i == 0) + (i == N) + (j == 0) + (j == N);
    T k2 = kp * kp;
    r.dre = T(-4) * ih2 + k2;
    r.dim = T(2) * kp * H * T(b) * ih2 + k2 * sigma;
    r.wl = (i > 0) ? ((i == N) ? T(2) : T(1)) * ih2 : T(0);
    r.wr = (i < N) ? ((i == 0) ? T(2) : T(1)) * ih2 : T(0);
    r.wd = (j > 0) ? ((j == N) ? T(2) : T(1)) * ih2 : T(0);
    r.wu = (j < N) ? ((j == 0) ? T(2) : T(1)) * ih2 : T(0);
    return r;
}

// Fields are stored in the level precision T (double or float); every
// kernel computes in R = double and rounds only when it stores, so that the
// stencil sums (terms of size |u| / H^2 that cancel) keep FP64 accuracy.
template <typename R, typename T>
__device__ __forceinline__ C<R> ldr(const C<T> *a, size_t p) {
    C<T> v = a[p];
    return cmk((R)v.x, (R)v.y);
}
template <typename T, typename R>
__device__ __forceinline__ C<T> st_as(C<R> v) {
    return cmk((T)v.x, (T)v.y);
}

// sum_{q != p} a_pq u_q, neighbours in the order left, right, down, up
template <typename R, typename T>
__device__ __forceinline__ C<R> offsum(const Row<R> &r, const C<T> *u, int i, int j, int N, int M) {
    C<R> s = cmk(R(0), R(0));
    size_t p = (size_t)j * M + i;
    if (i > 0) s = cadd(s, cscale(r.wl, ldr<R>(u, p - 1)));
    if (i < N) s = cadd(s, cscale(r.wr, ldr<R>(u, p + 1)));
    if (j > 0) s = cadd(s, cscale(r.wd, ldr<R>(u, p - M)));
    if (j < N) s = cadd(s, cscale(r.wu, ldr<R>(u, p + M)));
    return s;
}

template <typename R, typename T>
__device__ __forceinline__ C<R> row_apply(const Row<R> &r, const C<T> *u, int i, int j, int N, int M) {
    C<R> up = ldr<R>(u, (size_t)j * M + i);
    return cadd(cmul(cmk(r.dre, r.dim), up), offsum(r, u, i, j, N, M));
}

struct GeoT {
    int n, M, N;
};

// Pointer p of right-hand side blockIdx.z in a batched launch (zs bytes
// between right-hand sides; null stays null).  The offset is applied to a
// byte pointer, not an integer, so the compiler keeps knowing that p points
// to global memory (global, not flat, loads and stores).
template <typename T>
__device__ __forceinline__ T *zsh(T *p, long zs) {
    using B = typename std::conditional<std::is_const<T>::value, const char, char>::type;
    return p ? reinterpret_cast<T *>(reinterpret_cast<B *>(p) + (size_t)blockIdx.z * (size_t)zs) : p;
}

// Launches queued past convergence see a device flag and return.  The flag
// is read together with a kernel's first loads instead of before them (one
// memory latency less on the path of every launch): flag_read issues the
// load, flag_set tests it once the kernel's loads are in flight, and a
// launch that returns waits for its loads before it ends.  No launch stores
// anything before the test.
static __device__ int kNoFlag = 0;   // read (never written) where a launch has no flag
__device__ __forceinline__ int flag_read(const int *flag) { return *(flag ? flag : &kNoFlag); }
__device__ __forceinline__ bool flag_set(int v) {
    if (v) {
        __builtin_amdgcn_s_waitcnt(0);
        return true;
    }
    return false;
}

// Sum NV values over a 256-thread block; result valid in thread 0.
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double *out) {
    __shared__ double red[NV][NT / 64];
    int tid = threadIdx.y * BX + threadIdx.x;
    int lane = tid & 63, wave = tid >> 6;
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        double x = v[q];
        for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
        if (lane == 0) red[q][wave] = x;
    }
    __syncthreads();
    if (tid == 0) {
#pragma unroll
        for (int q = 0; q < NV; ++q) {
            double x = red[q][0];
            for (int w = 1; w < NT / 64; ++w) x += red[q][w];
            out[q] = x;
        }
    }
}

// Writes the block's NV sums to partials[q * nblocks + block].
template <int NV>
__device__ __forceinline__ void block_partials(double (&v)[NV], double *partials) {
    double tot[NV];
    block_sum<NV>(v, tot);
    int nb = gridDim.x * gridDim.y;
    int b = blockIdx.y * gridDim.x + blockIdx.x;
    if (threadIdx.x == 0 && threadIdx.y == 0) {
#pragma unroll
        for (int q = 0; q < NV; ++q) partials[(size_t)q * nb + b] = tot[q];
    }
}


}  // namespace hmgk
