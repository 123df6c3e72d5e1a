// Device code of the window sums (plane streaming over (tile, z)-sorted
// points), shared by the stand-alone kernels and the persistent batched
// kernel.  See interp.hip for the scheme.
#pragma once
#include "internal.h"

namespace nfft3 {

constexpr int kPsThreads = kItemPts;   // one point per thread

// Staged plane elements per thread for window width W: the plane region is
// at most (kMaxTile + W - 1)^2 elements.
template <int W>
constexpr int ps_nf() {
    return ((kMaxTile + W - 1) * (kMaxTile + W - 1) + kPsThreads - 1) / kPsThreads;
}

template <typename T>
using vec2_t = T __attribute__((ext_vector_type(2)));

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
    int pad8;               // pad the plane row stride to 8 mod 16 elements
};

// Per-workgroup setup shared by the three kernels.
struct PSItem {
    int y0, x0;          // first cell of the tile
    int p;               // sorted index of this thread's point
    bool active;
    int zbeg, nplanes;   // planes zbeg .. zbeg+nplanes-1 (unwrapped)
    int PY, PX, psz;
    int PXp;             // LDS row stride of the plane (padded)
};

// Work-item order: the hardware hands consecutive workgroups to the 8 XCDs in
// turn; map them so that each XCD walks a contiguous run of items (consecutive
// items of one tile column share 2m-1 halo planes, which then hit its L2).
__device__ __forceinline__ int xcd_item(int b, int G) {
    const int q = G / 8, r = G % 8;
    const int x = b % 8, i = b / 8;
    return x < r ? x * (q + 1) + i : r * (q + 1) + (x - r) * q + i;
}

// Geometry of the points [lo, hi) (sorted indices) of tile `tile`.
__device__ __forceinline__ PSItem ps_range(const PSArgs &a, int m, int tile, int lo, int hi) {
    PSItem it;
    const int ty = tile / a.ntx, tx = tile - ty * a.ntx;
    it.y0 = ty * a.By;
    it.x0 = tx * a.Bx;
    it.p = lo + threadIdx.x;
    it.active = it.p < hi;
    // points are sorted by z-cell: the first and last give the range
    float dummy;
    const int zmin = cell_frac<float>(a.xs[3 * lo], a.n0, dummy);
    const int zmax = cell_frac<float>(a.xs[3 * (hi - 1)], a.n0, dummy);
    it.zbeg = zmin - m + 1;
    it.nplanes = zmax - zmin + 2 * m;
    it.PY = a.By + 2 * m - 1;
    it.PX = a.Bx + 2 * m - 1;
    it.psz = it.PY * it.PX;
    it.PXp = a.pad8 ? it.PX + ((8 - it.PX % 16) + 16) % 16 : it.PX;
    return it;
}

__device__ __forceinline__ PSItem ps_item(const PSArgs &a, int m, int4 &item) {
    item = a.items[xcd_item(blockIdx.x, gridDim.x)];
    return ps_range(a, m, item.x, item.y, item.z);
}

// Offsets (within a plane) of the elements this thread stages; slots past
// the region point at element 0 so that every slot can be loaded.
template <int NF>
__device__ __forceinline__ void ps_offsets(const PSArgs &a, const PSItem &it, int m, int *off) {
#pragma unroll
    for (int k = 0; k < NF; ++k) {
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

// The loads are unconditional (no branch between them), so all NF are in
// flight together and the wait falls at the LDS store after the plane's
// compute; the values are held as native two-element vectors, which stay in
// registers for both precisions.
template <typename T, int NF>
__device__ __forceinline__ void ps_fetch(const c_t<T> *__restrict__ grid, const int *off, int64_t zoff,
                                         vec2_t<T> *v) {
    const vec2_t<T> *g = reinterpret_cast<const vec2_t<T> *>(grid) + zoff;
#pragma unroll
    for (int k = 0; k < NF; ++k) v[k] = g[off[k]];
}

template <typename T, int NF>
__device__ __forceinline__ void ps_store(c_t<T> *buf, const PSItem &it, const vec2_t<T> *v) {
    vec2_t<T> *b = reinterpret_cast<vec2_t<T> *>(buf);
#pragma unroll
    for (int k = 0; k < NF; ++k) {
        const int e = threadIdx.x + k * kPsThreads;
        if (e < it.psz) b[e] = v[k];
    }
}

// LDS bank spreading.  Lane l of a wavefront natively takes sorted point
// base + 64 w + l (z-adjacent points, so the wave is active on the same
// planes).  The stencil read of an instruction is, per lane, plane element
// (row + yo) * PX + (col + xo): the bank a lane hits is fixed by its class
// c = (yo * PX + xo) mod 16.  Sorting the wave's 64 points by class and
// dealing them out transposed (sorted position p -> lane 16 (p mod 4) + p/4)
// gives each 16-lane (and 8-lane) issue group distinct classes when the
// classes are balanced, instead of random ones.  Returns the lane-local index
// (0..255) of the point this thread takes.
__device__ __forceinline__ int wave_spread(const PSArgs &a, const PSItem &it, int base, int end) {
    const int lane = threadIdx.x & 63, wbase = threadIdx.x & ~63;
    const int pk = base + threadIdx.x;
    const bool valid = pk < end;
    int c = 16;                     // invalid lanes sort last
    if (valid) {
        float f;
        const int yc = cell_frac<float>(a.xs[3 * pk + 1], a.n1, f);
        const int xc = cell_frac<float>(a.xs[3 * pk + 2], a.n2, f);
        c = ((yc - it.y0) * it.PX + (xc - it.x0)) & 15;
    }
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    int pos = 0, rank = 0;
#pragma unroll
    for (int q = 0; q <= 16; ++q) {
        const uint64_t mq = __ballot(c == q);
        if (q < c) pos += __popcll(mq);
        if (q == c) rank = __popcll(mq & below);
    }
    pos += rank;                    // position in class-sorted order, 0..63
    const int tgt = 16 * (pos & 3) + (pos >> 2);
    const int src = __builtin_amdgcn_ds_permute(tgt << 2, lane);
    return wbase + src;
}

// ------------------------------------------------------------ interp ----
// Point slot k of thread t is sorted index item.y + k*256 + t: each slot's
// wavefronts hold z-adjacent points, so they are active on the same planes.
template <typename T, int W, int PPT>
__device__ __forceinline__ void interp_body(const PSArgs &a, int item_index, unsigned char *smem_raw) {
    constexpr int m = W / 2;
    const int4 item = a.items[item_index];
    const PSItem it = ps_range(a, m, item.x, item.y, item.z);
    c_t<T> *buf0 = reinterpret_cast<c_t<T> *>(smem_raw);
    c_t<T> *buf1 = buf0 + it.psz;
    T *scoef = reinterpret_cast<T *>(buf1 + it.psz);
    const T *coef = (const T *)a.coef;
    const int nc = W * (a.deg + 1);
    for (int i = threadIdx.x; i < nc; i += kPsThreads) scoef[i] = coef[i];

    T w1[PPT][W], w2[PPT][W];
    T f0[PPT], ar[PPT], ai[PPT];
    int zlo[PPT], pofs[PPT], pidx[PPT];
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        const int pk = item.y + k * kPsThreads + wave_spread(a, it, item.y + k * kPsThreads, item.z);
        pidx[k] = pk;
        ar[k] = 0;
        ai[k] = 0;
        zlo[k] = -4 * W;     // never active
        pofs[k] = -1;
        f0[k] = 0;
        if (pk < item.z) {
            const double *xp = a.xs + 3 * pk;
            T f1, f2;
            const int zc = cell_frac<T>(xp[0], a.n0, f0[k]);
            const int yc = cell_frac<T>(xp[1], a.n1, f1);
            const int xc = cell_frac<T>(xp[2], a.n2, f2);
            pofs[k] = (yc - it.y0) * it.PX + (xc - it.x0);
            zlo[k] = zc - m + 1 - it.zbeg;      // first plane index of the stencil
            window_weights<T, W>(f1, coef, a.deg, w1[k]);
            window_weights<T, W>(f2, coef, a.deg, w2[k]);
        }
    }

    constexpr int NF = ps_nf<W>();
    int off[NF];
    ps_offsets<NF>(a, it, m, off);
    const c_t<T> *grid = (const c_t<T> *)a.grid;
    const int64_t plane = (int64_t)a.n1 * a.n2;
    vec2_t<T> stage[NF];
    ps_fetch<T, NF>(grid, off, (int64_t)wrapi(it.zbeg, a.n0) * plane, stage);
    ps_store<T, NF>(buf0, it, stage);
    __syncthreads();

    for (int i = 0; i < it.nplanes; ++i) {
        const bool more = i + 1 < it.nplanes;
        if (more) ps_fetch<T, NF>(grid, off, (int64_t)wrapi(it.zbeg + i + 1, a.n0) * plane, stage);
        const c_t<T> *pl = (i & 1) ? buf1 : buf0;
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            const int r0 = i - zlo[k];
            if (r0 >= 0 && r0 < W) {
                const T w0 = piece<T>(scoef + r0 * (a.deg + 1), a.deg, f0[k]);
                T sr = 0, si = 0;
                const c_t<T> *base = pl + pofs[k];
#pragma unroll
                for (int r1 = 0; r1 < W; ++r1) {
                    const c_t<T> *row = base + r1 * it.PX;
                    T cr = 0, ci = 0;
#pragma unroll
                    for (int r2 = 0; r2 < W; ++r2) {
                        const c_t<T> g = row[r2];
                        cr += w2[k][r2] * g.x;
                        ci += w2[k][r2] * g.y;
                    }
                    sr += w1[k][r1] * cr;
                    si += w1[k][r1] * ci;
                }
                ar[k] += w0 * sr;
                ai[k] += w0 * si;
            }
        }
        if (more) ps_store<T, NF>((i & 1) ? buf0 : buf1, it, stage);
        __syncthreads();
    }
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        const int pk = pidx[k];
        if (pk < item.z) ((c_t<T> *)a.out)[a.perm[pk]] = cmk<T>(ar[k], ai[k]);
    }
}


inline PSArgs ps_args(const nfft3_plan_impl *p) {
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
    a.pad8 = 0;
    return a;
}

// LDS bytes of the window-sum kernels: nbuf staged planes + the coefficients.
inline size_t ps_lds(const nfft3_plan_impl *p, int nbuf) {
    const int W = 2 * p->m;
    const size_t psz = (size_t)(p->bins.By + W - 1) * (p->bins.Bx + W - 1);
    return nbuf * psz * p->elt + (size_t)W * (p->deg + 1) * (p->elt / 2);
}

}  // namespace nfft3
