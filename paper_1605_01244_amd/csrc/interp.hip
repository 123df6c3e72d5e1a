// Stage (c) of the windowed evaluation and its transposes:
//   interp : f_j      = sum_{r in {-m+1..m}^3} g[(u_j + r) mod n] prod_d w_d(r_d)
//   spread : g[u_j+r] += f_j prod_d w_d(r_d)                      (adjoint)
//   grad   : d f_j/d x_{j,d} = n_d sum_r g[...] w_d'(r_d) prod_{e != d} w_e(r_e)
// with u_j = floor(n x_j) and w_d(r) = phi((n x_j)_d - u_d - r)/phi(0) from the
// per-offset window polynomials in the cell fraction (see api.hip).  Cell and
// fraction are formed in FP64 in both precisions.
//
// Plane streaming.  Points are sorted by (tile, z-cell), a tile being a
// By x Bx block of (y, x) cells; a work item is at most 256 points of one tile
// column (one point per thread).  The workgroup walks the grid planes
// z = zmin-m+1 .. zmax+m of its item; each plane's (By+2m-1) x (Bx+2m-1)
// region (the tile plus the stencil halo, wrapped periodically) is staged in
// LDS, double-buffered, with the next plane's global loads issued into
// registers before the current plane is consumed.  A thread whose point has
// the plane inside its stencil adds w0 * sum_{r1,r2} w1 w2 g from LDS; the y/x
// weights live in registers for the whole item, the z weight is one polynomial
// per plane.  The spread kernel accumulates each plane in LDS with LDS atomics
// and flushes it to the grid with global atomics.
#include "internal.h"

namespace nfft3 {

constexpr int kPsThreads = kItemPts;   // one point per thread
constexpr int kMaxPF = kMaxPlane / kPsThreads;   // staged plane elements per thread

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

// one window piece (offset index r) and optionally its derivative
template <typename T>
__device__ __forceinline__ T piece(const T *c, int deg, T f) {
    const T y = (T)2 * f - (T)1;
    T w = c[deg];
    for (int q = deg - 1; q >= 0; --q) w = w * y + c[q];
    return w;
}
template <typename T>
__device__ __forceinline__ T piece_d(const T *c, int deg, T f, T &dw) {
    const T y = (T)2 * f - (T)1;
    T w = c[deg], d = (T)0;
    for (int q = deg - 1; q >= 0; --q) { d = d * y + w; w = w * y + c[q]; }
    dw = (T)2 * d;
    return w;
}

// cell index in [0, n) and fraction of a folded coordinate
template <typename T>
__device__ __forceinline__ int cell_frac(double x, int n, T &frac) {
    const double t = (double)n * x;
    const double u = floor(t);
    frac = (T)(t - u);
    int c = (int)u;
    if (c < 0) c += n;
    return c >= n ? c - n : c;
}

__device__ __forceinline__ int wrapi(int v, int n) {
    v %= n;
    return v < 0 ? v + n : v;
}

struct PSArgs {
    const double *xs;
    const int *perm;
    const int4 *items;
    const void *grid;       // interp/grad source
    void *grid_out;         // spread target
    const void *vals;       // spread: f; grad: G
    void *out;              // interp: f; grad: grad_x
    const void *coef;
    int deg;
    int n0, n1, n2;
    int By, Bx, ntx;
};

// Per-workgroup setup shared by the three kernels.
struct PSItem {
    int y0, x0;          // first cell of the tile
    int p;               // sorted index of this thread's point
    bool active;
    int zbeg, nplanes;   // planes zbeg .. zbeg+nplanes-1 (unwrapped)
    int PY, PX, psz;
};

__device__ __forceinline__ PSItem ps_item(const PSArgs &a, int m) {
    PSItem it;
    const int4 item = a.items[blockIdx.x];
    const int ty = item.x / a.ntx, tx = item.x - ty * a.ntx;
    it.y0 = ty * a.By;
    it.x0 = tx * a.Bx;
    it.p = item.y + threadIdx.x;
    it.active = it.p < item.z;
    // points of an item are sorted by z-cell: the first and last give the range
    float dummy;
    const int zmin = cell_frac<float>(a.xs[3 * item.y], a.n0, dummy);
    const int zmax = cell_frac<float>(a.xs[3 * (item.z - 1)], a.n0, dummy);
    it.zbeg = zmin - m + 1;
    it.nplanes = zmax - zmin + 2 * m;
    it.PY = a.By + 2 * m - 1;
    it.PX = a.Bx + 2 * m - 1;
    it.psz = it.PY * it.PX;
    return it;
}

// Offsets (within a plane) of the elements this thread stages.
__device__ __forceinline__ void ps_offsets(const PSArgs &a, const PSItem &it, int m, int *off) {
#pragma unroll
    for (int k = 0; k < kMaxPF; ++k) {
        const int e = threadIdx.x + k * kPsThreads;
        if (e < it.psz) {
            const int ly = e / it.PX, lx = e - ly * it.PX;
            const int gy = wrapi(it.y0 - m + 1 + ly, a.n1);
            const int gx = wrapi(it.x0 - m + 1 + lx, a.n2);
            off[k] = gy * a.n2 + gx;
        } else {
            off[k] = 0;
        }
    }
}

// Staged values are kept as separate real/imaginary arrays: an array of the
// HIP complex vector type is not promoted to registers for double.
template <typename T>
__device__ __forceinline__ void ps_fetch(const c_t<T> *__restrict__ grid, const PSItem &it, const int *off,
                                         int64_t zoff, T *rr, T *ri) {
#pragma unroll
    for (int k = 0; k < kMaxPF; ++k) {
        const int e = threadIdx.x + k * kPsThreads;
        if (e < it.psz) {
            const c_t<T> g = grid[zoff + off[k]];
            rr[k] = g.x;
            ri[k] = g.y;
        }
    }
}

template <typename T>
__device__ __forceinline__ void ps_store(c_t<T> *buf, const PSItem &it, const T *rr, const T *ri) {
#pragma unroll
    for (int k = 0; k < kMaxPF; ++k) {
        const int e = threadIdx.x + k * kPsThreads;
        if (e < it.psz) buf[e] = cmk<T>(rr[k], ri[k]);
    }
}

// ------------------------------------------------------------ interp ----
template <typename T, int W>
__global__ void __launch_bounds__(kPsThreads) interp_ps_kernel(PSArgs a) {
    constexpr int m = W / 2;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const PSItem it = ps_item(a, m);
    c_t<T> *buf0 = reinterpret_cast<c_t<T> *>(smem_raw);
    c_t<T> *buf1 = buf0 + it.psz;
    T *scoef = reinterpret_cast<T *>(buf1 + it.psz);
    const T *coef = (const T *)a.coef;
    const int nc = W * (a.deg + 1);
    for (int i = threadIdx.x; i < nc; i += kPsThreads) scoef[i] = coef[i];

    T w1[W], w2[W];
    T f0 = 0;
    int zc = 0, yo = 0, xo = 0;
    if (it.active) {
        const double *xp = a.xs + 3 * it.p;
        T f1, f2;
        zc = cell_frac<T>(xp[0], a.n0, f0);
        const int yc = cell_frac<T>(xp[1], a.n1, f1);
        const int xc = cell_frac<T>(xp[2], a.n2, f2);
        yo = yc - it.y0;
        xo = xc - it.x0;
        window_weights<T, W>(f1, coef, a.deg, w1);
        window_weights<T, W>(f2, coef, a.deg, w2);
    }
    const int zlo = zc - m + 1 - it.zbeg;   // first plane index of this point's stencil

    int off[kMaxPF];
    ps_offsets(a, it, m, off);
    const c_t<T> *grid = (const c_t<T> *)a.grid;
    const int64_t plane = (int64_t)a.n1 * a.n2;
    T rr[kMaxPF], ri[kMaxPF];
    ps_fetch<T>(grid, it, off, (int64_t)wrapi(it.zbeg, a.n0) * plane, rr, ri);
    ps_store<T>(buf0, it, rr, ri);
    __syncthreads();

    T ar = 0, ai = 0;
    for (int i = 0; i < it.nplanes; ++i) {
        const bool more = i + 1 < it.nplanes;
        if (more) ps_fetch<T>(grid, it, off, (int64_t)wrapi(it.zbeg + i + 1, a.n0) * plane, rr, ri);
        const c_t<T> *pl = (i & 1) ? buf1 : buf0;
        const int r0 = i - zlo;
        if (it.active && r0 >= 0 && r0 < W) {
            const T w0 = piece<T>(scoef + r0 * (a.deg + 1), a.deg, f0);
            T sr = 0, si = 0;
            const c_t<T> *base = pl + yo * it.PX + xo;
#pragma unroll 2
            for (int r1 = 0; r1 < W; ++r1) {
                const c_t<T> *row = base + r1 * it.PX;
                T cr = 0, ci = 0;
#pragma unroll
                for (int r2 = 0; r2 < W; ++r2) {
                    const c_t<T> g = row[r2];
                    cr += w2[r2] * g.x;
                    ci += w2[r2] * g.y;
                }
                sr += w1[r1] * cr;
                si += w1[r1] * ci;
            }
            ar += w0 * sr;
            ai += w0 * si;
        }
        if (more) ps_store<T>((i & 1) ? buf0 : buf1, it, rr, ri);
        __syncthreads();
    }
    if (it.active) ((c_t<T> *)a.out)[a.perm[it.p]] = cmk<T>(ar, ai);
}

// ------------------------------------------------------------- grad ----
template <typename T, int W>
__global__ void __launch_bounds__(kPsThreads) grad_ps_kernel(PSArgs a) {
    constexpr int m = W / 2;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const PSItem it = ps_item(a, m);
    c_t<T> *buf0 = reinterpret_cast<c_t<T> *>(smem_raw);
    c_t<T> *buf1 = buf0 + it.psz;
    T *scoef = reinterpret_cast<T *>(buf1 + it.psz);
    const T *coef = (const T *)a.coef;
    const int nc = W * (a.deg + 1);
    for (int i = threadIdx.x; i < nc; i += kPsThreads) scoef[i] = coef[i];

    T w1[W], w2[W], d1[W], d2[W];
    T f0 = 0;
    int zc = 0, yo = 0, xo = 0;
    if (it.active) {
        const double *xp = a.xs + 3 * it.p;
        T f1, f2;
        zc = cell_frac<T>(xp[0], a.n0, f0);
        const int yc = cell_frac<T>(xp[1], a.n1, f1);
        const int xc = cell_frac<T>(xp[2], a.n2, f2);
        yo = yc - it.y0;
        xo = xc - it.x0;
        window_weights_d<T, W>(f1, coef, a.deg, w1, d1);
        window_weights_d<T, W>(f2, coef, a.deg, w2, d2);
    }
    const int zlo = zc - m + 1 - it.zbeg;
    int off[kMaxPF];
    ps_offsets(a, it, m, off);
    const c_t<T> *grid = (const c_t<T> *)a.grid;
    const int64_t plane = (int64_t)a.n1 * a.n2;
    T rr[kMaxPF], ri[kMaxPF];
    ps_fetch<T>(grid, it, off, (int64_t)wrapi(it.zbeg, a.n0) * plane, rr, ri);
    ps_store<T>(buf0, it, rr, ri);
    __syncthreads();

    // D0 = sum d0 w1 w2 g, D1 = sum w0 d1 w2 g, D2 = sum w0 w1 d2 g
    T D0r = 0, D0i = 0, D1r = 0, D1i = 0, D2r = 0, D2i = 0;
    for (int i = 0; i < it.nplanes; ++i) {
        const bool more = i + 1 < it.nplanes;
        if (more) ps_fetch<T>(grid, it, off, (int64_t)wrapi(it.zbeg + i + 1, a.n0) * plane, rr, ri);
        const c_t<T> *pl = (i & 1) ? buf1 : buf0;
        const int r0 = i - zlo;
        if (it.active && r0 >= 0 && r0 < W) {
            T dw0;
            const T w0 = piece_d<T>(scoef + r0 * (a.deg + 1), a.deg, f0, dw0);
            T vr = 0, vi = 0, ur = 0, ui = 0, tr = 0, ti = 0;
            const c_t<T> *base = pl + yo * it.PX + xo;
            for (int r1 = 0; r1 < W; ++r1) {
                const c_t<T> *row = base + r1 * it.PX;
                T sr = 0, si = 0, qr = 0, qi = 0;
#pragma unroll
                for (int r2 = 0; r2 < W; ++r2) {
                    const c_t<T> g = row[r2];
                    sr += w2[r2] * g.x;
                    si += w2[r2] * g.y;
                    qr += d2[r2] * g.x;
                    qi += d2[r2] * g.y;
                }
                vr += w1[r1] * sr; vi += w1[r1] * si;
                ur += d1[r1] * sr; ui += d1[r1] * si;
                tr += w1[r1] * qr; ti += w1[r1] * qi;
            }
            D0r += dw0 * vr; D0i += dw0 * vi;
            D1r += w0 * ur;  D1i += w0 * ui;
            D2r += w0 * tr;  D2i += w0 * ti;
        }
        if (more) ps_store<T>((i & 1) ? buf0 : buf1, it, rr, ri);
        __syncthreads();
    }
    if (it.active) {
        const int pj = a.perm[it.p];
        const c_t<T> g = ((const c_t<T> *)a.vals)[pj];
        double *gx = (double *)a.out + 3 * (int64_t)pj;
        // Re(conj(G) D) = G.x D.x + G.y D.y, times n_d (dt/dx)
        gx[0] = (double)a.n0 * ((double)g.x * (double)D0r + (double)g.y * (double)D0i);
        gx[1] = (double)a.n1 * ((double)g.x * (double)D1r + (double)g.y * (double)D1i);
        gx[2] = (double)a.n2 * ((double)g.x * (double)D2r + (double)g.y * (double)D2i);
    }
}

// ------------------------------------------------------------ spread ----
template <typename T, int W>
__global__ void __launch_bounds__(kPsThreads) spread_ps_kernel(PSArgs a) {
    constexpr int m = W / 2;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const PSItem it = ps_item(a, m);
    c_t<T> *acc = reinterpret_cast<c_t<T> *>(smem_raw);
    T *scoef = reinterpret_cast<T *>(acc + it.psz);
    const T *coef = (const T *)a.coef;
    const int nc = W * (a.deg + 1);
    for (int i = threadIdx.x; i < nc; i += kPsThreads) scoef[i] = coef[i];
    for (int e = threadIdx.x; e < it.psz; e += kPsThreads) acc[e] = cmk<T>(0, 0);

    T w1[W], w2[W];
    T f0 = 0;
    int zc = 0, yo = 0, xo = 0;
    c_t<T> v = cmk<T>(0, 0);
    if (it.active) {
        const double *xp = a.xs + 3 * it.p;
        T f1, f2;
        zc = cell_frac<T>(xp[0], a.n0, f0);
        const int yc = cell_frac<T>(xp[1], a.n1, f1);
        const int xc = cell_frac<T>(xp[2], a.n2, f2);
        yo = yc - it.y0;
        xo = xc - it.x0;
        window_weights<T, W>(f1, coef, a.deg, w1);
        window_weights<T, W>(f2, coef, a.deg, w2);
        v = ((const c_t<T> *)a.vals)[a.perm[it.p]];
    }
    const int zlo = zc - m + 1 - it.zbeg;
    int off[kMaxPF];
    ps_offsets(a, it, m, off);
    c_t<T> *grid = (c_t<T> *)a.grid_out;
    const int64_t plane = (int64_t)a.n1 * a.n2;
    __syncthreads();

    for (int i = 0; i < it.nplanes; ++i) {
        const int r0 = i - zlo;
        if (it.active && r0 >= 0 && r0 < W) {
            const T w0 = piece<T>(scoef + r0 * (a.deg + 1), a.deg, f0);
            const T vr = w0 * v.x, vi = w0 * v.y;
            c_t<T> *base = acc + yo * it.PX + xo;
            for (int r1 = 0; r1 < W; ++r1) {
                c_t<T> *row = base + r1 * it.PX;
                const T br = w1[r1] * vr, bi = w1[r1] * vi;
#pragma unroll
                for (int r2 = 0; r2 < W; ++r2) {
                    atomicAdd(&row[r2].x, w2[r2] * br);
                    atomicAdd(&row[r2].y, w2[r2] * bi);
                }
            }
        }
        __syncthreads();
        // flush this plane to the grid and clear it
        const int64_t zoff = (int64_t)wrapi(it.zbeg + i, a.n0) * plane;
#pragma unroll
        for (int k = 0; k < kMaxPF; ++k) {
            const int e = threadIdx.x + k * kPsThreads;
            if (e < it.psz) {
                const c_t<T> s = acc[e];
                if (s.x != (T)0 || s.y != (T)0) {
                    unsafeAtomicAdd(&grid[zoff + off[k]].x, s.x);
                    unsafeAtomicAdd(&grid[zoff + off[k]].y, s.y);
                    acc[e] = cmk<T>(0, 0);
                }
            }
        }
        __syncthreads();
    }
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
static PSArgs ps_args(nfft3_plan_impl *p) {
    PSArgs a;
    a.xs = p->xs;
    a.perm = p->perm;
    a.items = p->sub.items;
    a.grid = nullptr;
    a.grid_out = nullptr;
    a.vals = nullptr;
    a.out = nullptr;
    a.coef = p->wcoef;
    a.deg = p->deg;
    a.n0 = (int)p->n[0];
    a.n1 = (int)p->n[1];
    a.n2 = (int)p->n[2];
    a.By = p->bins.By;
    a.Bx = p->bins.Bx;
    a.ntx = p->bins.ntx;
    return a;
}

static size_t ps_lds(nfft3_plan_impl *p, int nbuf) {
    const int W = 2 * p->m;
    const size_t psz = (size_t)(p->bins.By + W - 1) * (p->bins.Bx + W - 1);
    return nbuf * psz * p->elt + (size_t)W * (p->deg + 1) * (p->elt / 2);
}

template <typename T, int W>
static int interp_w(nfft3_plan_impl *p, const void *grid, void *f) {
    if (p->M == 0 || p->sub.count == 0) return NFFT3_OK;
    PSArgs a = ps_args(p);
    a.grid = grid;
    a.out = f;
    const size_t lds = ps_lds(p, 2);
    allow_lds((const void *)interp_ps_kernel<T, W>, lds);
    hipLaunchKernelGGL((interp_ps_kernel<T, W>), dim3((unsigned)p->sub.count), dim3(kPsThreads), lds, p->stream, a);
    NFFT3_LAUNCH_CHECK("interp_ps_kernel");
    return NFFT3_OK;
}

template <typename T, int W>
static int spread_w(nfft3_plan_impl *p, const void *f, void *grid) {
    if (p->M == 0 || p->sub.count == 0) return NFFT3_OK;
    PSArgs a = ps_args(p);
    a.vals = f;
    a.grid_out = grid;
    const size_t lds = ps_lds(p, 1);
    allow_lds((const void *)spread_ps_kernel<T, W>, lds);
    hipLaunchKernelGGL((spread_ps_kernel<T, W>), dim3((unsigned)p->sub.count), dim3(kPsThreads), lds, p->stream, a);
    NFFT3_LAUNCH_CHECK("spread_ps_kernel");
    return NFFT3_OK;
}

template <typename T, int W>
static int grad_w(nfft3_plan_impl *p, const void *grid, const void *G, double *gx) {
    if (p->M == 0 || p->sub.count == 0) return NFFT3_OK;
    PSArgs a = ps_args(p);
    a.grid = grid;
    a.vals = G;
    a.out = gx;
    const size_t lds = ps_lds(p, 2);
    allow_lds((const void *)grad_ps_kernel<T, W>, lds);
    hipLaunchKernelGGL((grad_ps_kernel<T, W>), dim3((unsigned)p->sub.count), dim3(kPsThreads), lds, p->stream, a);
    NFFT3_LAUNCH_CHECK("grad_ps_kernel");
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
