// Stage (c) of the windowed evaluation and its transposes:
//   interp : f_j      = sum_{r in {-m+1..m}^3} g[(u_j + r) mod n] prod_d w_d(r_d)
//   spread : g[u_j+r] += f_j prod_d w_d(r_d)                 (adjoint, atomics)
//   grad   : d f_j/d x_{j,d} = n_d sum_r g[...] w_d'(r_d) prod_{e != d} w_e(r_e)
// with u_j = floor(n x_j) and w_d(r) = phi((n x_j)_d - u_d - r)/phi(0) taken
// from per-offset polynomials in the cell fraction (see api.hip).  The cell
// and fraction are formed in FP64 in both precisions.
//
// One thread per point over the tile-sorted point list: neighbouring lanes
// hold neighbouring points, so their (2m)^3 stencils overlap in L1/L2.
#include "internal.h"

namespace nfft3 {

constexpr int kIpThreads = 256;

template <typename T, int W>
__device__ __forceinline__ void window_weights(T f, const T *__restrict__ coef, int deg, T *w) {
    const T y = (T)2 * f - (T)1;
#pragma unroll
    for (int r = 0; r < W; ++r) w[r] = coef[r * (deg + 1) + deg];
    for (int q = deg - 1; q >= 0; --q) {
#pragma unroll
        for (int r = 0; r < W; ++r) w[r] = w[r] * y + coef[r * (deg + 1) + q];
    }
}

// Values and derivatives d/df (= d/dt of the window) of the same polynomials.
template <typename T, int W>
__device__ __forceinline__ void window_weights_d(T f, const T *__restrict__ coef, int deg, T *w, T *dw) {
    const T y = (T)2 * f - (T)1;
#pragma unroll
    for (int r = 0; r < W; ++r) { w[r] = coef[r * (deg + 1) + deg]; dw[r] = (T)0; }
    for (int q = deg - 1; q >= 0; --q) {
#pragma unroll
        for (int r = 0; r < W; ++r) {
            dw[r] = dw[r] * y + w[r];
            w[r] = w[r] * y + coef[r * (deg + 1) + q];
        }
    }
#pragma unroll
    for (int r = 0; r < W; ++r) dw[r] *= (T)2;
}

// Cell index (already wrapped to [0,n)) of the first stencil point and the
// fraction, from the folded FP64 coordinate.
template <typename T>
__device__ __forceinline__ void cell_frac(double x, int n, int m, int &start, T &frac) {
    const double t = (double)n * x;
    const double u = floor(t);
    frac = (T)(t - u);
    int s = (int)u - m + 1;
    s %= n;
    start = s < 0 ? s + n : s;
}

template <int W>
__device__ __forceinline__ void stencil_index(int start, int n, int *idx) {
#pragma unroll
    for (int r = 0; r < W; ++r) {
        int v = start + r;
        idx[r] = v >= n ? v - n : v;
    }
}

template <typename T, int W>
__global__ void __launch_bounds__(kIpThreads)
interp_gm_kernel(const double *__restrict__ xs, const int *__restrict__ perm, int M,
                 const c_t<T> *__restrict__ grid, int n0, int n1, int n2, const T *__restrict__ coef,
                 int deg, c_t<T> *__restrict__ out) {
    constexpr int m = W / 2;
    const int j = blockIdx.x * kIpThreads + threadIdx.x;
    if (j >= M) return;
    T w0[W], w1[W], w2[W];
    int i0[W], i1[W], i2[W];
    {
        int s;
        T f;
        cell_frac<T>(xs[3 * j + 0], n0, m, s, f);
        window_weights<T, W>(f, coef, deg, w0);
        stencil_index<W>(s, n0, i0);
        cell_frac<T>(xs[3 * j + 1], n1, m, s, f);
        window_weights<T, W>(f, coef, deg, w1);
        stencil_index<W>(s, n1, i1);
        cell_frac<T>(xs[3 * j + 2], n2, m, s, f);
        window_weights<T, W>(f, coef, deg, w2);
        stencil_index<W>(s, n2, i2);
    }
    const int64_t plane = (int64_t)n1 * n2;
    T ar = 0, ai = 0;
#pragma unroll 1
    for (int a = 0; a < W; ++a) {
        const c_t<T> *pl = grid + i0[a] * plane;
        T br = 0, bi = 0;
        for (int b = 0; b < W; ++b) {
            const c_t<T> *row = pl + (int64_t)i1[b] * n2;
            T cr = 0, ci = 0;
#pragma unroll
            for (int c = 0; c < W; ++c) {
                const c_t<T> g = row[i2[c]];
                cr += w2[c] * g.x;
                ci += w2[c] * g.y;
            }
            br += w1[b] * cr;
            bi += w1[b] * ci;
        }
        ar += w0[a] * br;
        ai += w0[a] * bi;
    }
    out[perm[j]] = cmk<T>(ar, ai);
}

template <typename T>
__device__ __forceinline__ void atomic_add_c(c_t<T> *p, T re, T im) {
    unsafeAtomicAdd(&p->x, re);
    unsafeAtomicAdd(&p->y, im);
}

template <typename T, int W>
__global__ void __launch_bounds__(kIpThreads)
spread_gm_kernel(const double *__restrict__ xs, const int *__restrict__ perm, int M,
                 const c_t<T> *__restrict__ f, c_t<T> *__restrict__ grid, int n0, int n1, int n2,
                 const T *__restrict__ coef, int deg) {
    constexpr int m = W / 2;
    const int j = blockIdx.x * kIpThreads + threadIdx.x;
    if (j >= M) return;
    T w0[W], w1[W], w2[W];
    int i0[W], i1[W], i2[W];
    {
        int s;
        T fr;
        cell_frac<T>(xs[3 * j + 0], n0, m, s, fr);
        window_weights<T, W>(fr, coef, deg, w0);
        stencil_index<W>(s, n0, i0);
        cell_frac<T>(xs[3 * j + 1], n1, m, s, fr);
        window_weights<T, W>(fr, coef, deg, w1);
        stencil_index<W>(s, n1, i1);
        cell_frac<T>(xs[3 * j + 2], n2, m, s, fr);
        window_weights<T, W>(fr, coef, deg, w2);
        stencil_index<W>(s, n2, i2);
    }
    const c_t<T> v = f[perm[j]];
    const int64_t plane = (int64_t)n1 * n2;
#pragma unroll 1
    for (int a = 0; a < W; ++a) {
        c_t<T> *pl = grid + i0[a] * plane;
        const T ar = w0[a] * v.x, ai = w0[a] * v.y;
        for (int b = 0; b < W; ++b) {
            c_t<T> *row = pl + (int64_t)i1[b] * n2;
            const T br = w1[b] * ar, bi = w1[b] * ai;
#pragma unroll
            for (int c = 0; c < W; ++c) atomic_add_c<T>(row + i2[c], w2[c] * br, w2[c] * bi);
        }
    }
}

template <typename T, int W>
__global__ void __launch_bounds__(kIpThreads)
grad_gm_kernel(const double *__restrict__ xs, const int *__restrict__ perm, int M,
               const c_t<T> *__restrict__ grid, int n0, int n1, int n2, const T *__restrict__ coef,
               int deg, const c_t<T> *__restrict__ G, double *__restrict__ grad_x) {
    constexpr int m = W / 2;
    const int j = blockIdx.x * kIpThreads + threadIdx.x;
    if (j >= M) return;
    T w0[W], w1[W], w2[W], d0[W], d1[W], d2[W];
    int i0[W], i1[W], i2[W];
    {
        int s;
        T f;
        cell_frac<T>(xs[3 * j + 0], n0, m, s, f);
        window_weights_d<T, W>(f, coef, deg, w0, d0);
        stencil_index<W>(s, n0, i0);
        cell_frac<T>(xs[3 * j + 1], n1, m, s, f);
        window_weights_d<T, W>(f, coef, deg, w1, d1);
        stencil_index<W>(s, n1, i1);
        cell_frac<T>(xs[3 * j + 2], n2, m, s, f);
        window_weights_d<T, W>(f, coef, deg, w2, d2);
        stencil_index<W>(s, n2, i2);
    }
    const int64_t plane = (int64_t)n1 * n2;
    // D0 = sum d0 w1 w2 g, D1 = sum w0 d1 w2 g, D2 = sum w0 w1 d2 g
    T D0r = 0, D0i = 0, D1r = 0, D1i = 0, D2r = 0, D2i = 0;
#pragma unroll 1
    for (int a = 0; a < W; ++a) {
        const c_t<T> *pl = grid + i0[a] * plane;
        T vr = 0, vi = 0, ur = 0, ui = 0, tr = 0, ti = 0;   // w1*s, d1*s, w1*t
        for (int b = 0; b < W; ++b) {
            const c_t<T> *row = pl + (int64_t)i1[b] * n2;
            T sr = 0, si = 0, qr = 0, qi = 0;                // sum w2 g, sum d2 g
#pragma unroll
            for (int c = 0; c < W; ++c) {
                const c_t<T> g = row[i2[c]];
                sr += w2[c] * g.x;
                si += w2[c] * g.y;
                qr += d2[c] * g.x;
                qi += d2[c] * g.y;
            }
            vr += w1[b] * sr; vi += w1[b] * si;
            ur += d1[b] * sr; ui += d1[b] * si;
            tr += w1[b] * qr; ti += w1[b] * qi;
        }
        D0r += d0[a] * vr; D0i += d0[a] * vi;
        D1r += w0[a] * ur; D1i += w0[a] * ui;
        D2r += w0[a] * tr; D2i += w0[a] * ti;
    }
    const int pj = perm[j];
    const c_t<T> g = G[pj];
    // Re(conj(G) D) = G.x D.x + G.y D.y, times n_d (dt/dx)
    grad_x[3 * (int64_t)pj + 0] = (double)n0 * ((double)g.x * (double)D0r + (double)g.y * (double)D0i);
    grad_x[3 * (int64_t)pj + 1] = (double)n1 * ((double)g.x * (double)D1r + (double)g.y * (double)D1i);
    grad_x[3 * (int64_t)pj + 2] = (double)n2 * ((double)g.x * (double)D2r + (double)g.y * (double)D2i);
}

__global__ void zero_kernel(float4 *p, int64_t count) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = make_float4(0.f, 0.f, 0.f, 0.f);
}

int launch_zero(nfft3_plan_impl *p, void *buf, size_t bytes) {
    const int64_t count = (int64_t)(bytes / 16);
    if (count == 0) return NFFT3_OK;
    hipLaunchKernelGGL(zero_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, p->stream,
                       (float4 *)buf, count);
    NFFT3_LAUNCH_CHECK("zero_kernel");
    return NFFT3_OK;
}

// ------------------------------------------------------------ dispatch ----
template <typename T, int W>
static int interp_w(nfft3_plan_impl *p, const void *grid, void *f) {
    const int M = (int)p->M;
    if (M == 0) return NFFT3_OK;
    hipLaunchKernelGGL((interp_gm_kernel<T, W>), dim3((M + kIpThreads - 1) / kIpThreads), dim3(kIpThreads), 0,
                       p->stream, p->xs, p->perm, M, (const c_t<T> *)grid, (int)p->n[0], (int)p->n[1],
                       (int)p->n[2], (const T *)p->wcoef, p->deg, (c_t<T> *)f);
    NFFT3_LAUNCH_CHECK("interp_gm_kernel");
    return NFFT3_OK;
}

template <typename T, int W>
static int spread_w(nfft3_plan_impl *p, const void *f, void *grid) {
    const int M = (int)p->M;
    if (M == 0) return NFFT3_OK;
    hipLaunchKernelGGL((spread_gm_kernel<T, W>), dim3((M + kIpThreads - 1) / kIpThreads), dim3(kIpThreads), 0,
                       p->stream, p->xs, p->perm, M, (const c_t<T> *)f, (c_t<T> *)grid, (int)p->n[0],
                       (int)p->n[1], (int)p->n[2], (const T *)p->wcoef, p->deg);
    NFFT3_LAUNCH_CHECK("spread_gm_kernel");
    return NFFT3_OK;
}

template <typename T, int W>
static int grad_w(nfft3_plan_impl *p, const void *grid, const void *G, double *gx) {
    const int M = (int)p->M;
    if (M == 0) return NFFT3_OK;
    hipLaunchKernelGGL((grad_gm_kernel<T, W>), dim3((M + kIpThreads - 1) / kIpThreads), dim3(kIpThreads), 0,
                       p->stream, p->xs, p->perm, M, (const c_t<T> *)grid, (int)p->n[0], (int)p->n[1],
                       (int)p->n[2], (const T *)p->wcoef, p->deg, (const c_t<T> *)G, gx);
    NFFT3_LAUNCH_CHECK("grad_gm_kernel");
    return NFFT3_OK;
}

#define NFFT3_DISPATCH_M(FN, T, ...)                     \
    switch (p->m) {                                      \
        case 1: return FN<T, 2>(p, __VA_ARGS__);         \
        case 2: return FN<T, 4>(p, __VA_ARGS__);         \
        case 3: return FN<T, 6>(p, __VA_ARGS__);         \
        case 4: return FN<T, 8>(p, __VA_ARGS__);         \
        case 5: return FN<T, 10>(p, __VA_ARGS__);        \
        case 6: return FN<T, 12>(p, __VA_ARGS__);        \
        case 7: return FN<T, 14>(p, __VA_ARGS__);        \
        case 8: return FN<T, 16>(p, __VA_ARGS__);        \
        case 9: return FN<T, 18>(p, __VA_ARGS__);        \
        case 10: return FN<T, 20>(p, __VA_ARGS__);       \
        default: return NFFT3_ERR_INVALID_ARG;           \
    }

int launch_interp(nfft3_plan_impl *p, const void *grid, void *f) {
    if (p->dtype == NFFT3_C128) { NFFT3_DISPATCH_M(interp_w, double, grid, f) }
    NFFT3_DISPATCH_M(interp_w, float, grid, f)
}

int launch_spread(nfft3_plan_impl *p, const void *f, void *grid) {
    if (p->dtype == NFFT3_C128) { NFFT3_DISPATCH_M(spread_w, double, f, grid) }
    NFFT3_DISPATCH_M(spread_w, float, f, grid)
}

int launch_grad(nfft3_plan_impl *p, const void *grid, const void *G, double *gx) {
    if (p->dtype == NFFT3_C128) { NFFT3_DISPATCH_M(grad_w, double, grid, G, gx) }
    NFFT3_DISPATCH_M(grad_w, float, grid, G, gx)
}

}  // namespace nfft3
