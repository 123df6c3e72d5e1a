// Device code of the window sums (plane streaming over (tile, z)-sorted
// points), shared by the single-plan kernels (interp.hip) and the batched
// window-sum launch (batch.hip).  See interp.hip for the scheme.
#pragma once
#include <numeric>

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

// The window sums keep the pieces in LDS as rows of a fixed length ZC (a
// whole number of 16-byte units, zero above the degree), so a piece is a few
// 16-byte reads and an unrolled Horner chain; the leading zeros pass through
// the chain exactly, so the value is the one of piece().  elt = bytes of one
// complex element.
constexpr int zrow_len(int elt, int W) { return elt == 8 ? 12 : (W <= 4 ? 20 : 16); }

template <typename T, int ZC>
__device__ __forceinline__ T piece_fixed(const T *c, T f) {
    using V = T __attribute__((ext_vector_type(16 / sizeof(T))));
    constexpr int E = 16 / sizeof(T);
    const V *cv = reinterpret_cast<const V *>(c);
    T k[ZC];
#pragma unroll
    for (int u = 0; u < ZC / E; ++u) {
        const V v = cv[u];
#pragma unroll
        for (int e = 0; e < E; ++e) k[u * E + e] = v[e];
    }
    const T y = (T)2 * f - (T)1;
    T w = k[ZC - 1];
#pragma unroll
    for (int q = ZC - 2; q >= 0; --q) w = w * y + k[q];
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
    int pxp;                // interp: LDS row stride of a staged plane (elements); 0 = unpadded
    int qinv;               // interp: inverse of (row stride in 16-B units / D) mod 16/D
    int fmask;              // fields: derivative axes written after the field (bit d = axis d)
    int64_t fstride;        // fields: elements between consecutive output blocks (M)
    int unit;               // bit 0: axis 0 is a unit axis (one plane, weight 1); bit 1: axis 1 too
    int gdim;               // grad: components per point written (the last gdim axes)
};

// What the window-sum body computes at each point.
constexpr int kModeValue = 0;    // f_j
constexpr int kModeGrad = 1;     // Re(conj(G_j) d f_j/d x_{j,d}), d = 0, 1, 2
constexpr int kModeFields = 2;   // f_j and the derivative fields d f_j/d x_{j,d} of fmask

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
__device__ __forceinline__ PSItem ps_range(const PSArgs &a, int m, int tile, int lo, int hi, bool rows1 = false) {
    PSItem it;
    const int ty = tile / a.ntx, tx = tile - ty * a.ntx;
    it.y0 = ty * a.By;
    it.x0 = tx * a.Bx;
    it.p = lo + threadIdx.x;
    it.active = it.p < hi;
    // points are sorted by z-cell: the first and last give the range
    float dummy;
    const int zmin = cell_frac<float>(a.xs[3 * (int64_t)lo], a.n0, dummy);
    const int zmax = cell_frac<float>(a.xs[3 * ((int64_t)hi - 1)], a.n0, dummy);
    it.zbeg = zmin - m + 1;
    it.nplanes = zmax - zmin + 2 * m;
    if (a.unit & 1) {       // unit axis 0: the one plane, weight 1
        it.zbeg = 0;
        it.nplanes = 1;
    }
    it.PY = rows1 ? 1 : a.By + 2 * m - 1;    // rows1: only the region's first row is read
    it.PX = a.Bx + 2 * m - 1;
    it.psz = it.PY * it.PX;
    it.PXp = a.pxp ? a.pxp : it.PX;
    return it;
}

__device__ __forceinline__ PSItem ps_item(const PSArgs &a, int m, int4 &item) {
    item = a.items[xcd_item(blockIdx.x, gridDim.x)];
    return ps_range(a, m, item.x, item.y, item.z);
}

// Offsets (within a plane) of the elements this thread stages; slots past
// the region point at element 0 so that every slot can be loaded.  lidx is
// the element's LDS index in a plane of row stride it.PXp.
template <int NF>
__device__ __forceinline__ void ps_offsets(const PSArgs &a, const PSItem &it, int m, int *off, int *lidx) {
#pragma unroll
    for (int k = 0; k < NF; ++k) {
        const int e = threadIdx.x + k * kPsThreads;
        if (e < it.psz) {
            const int ly = e / it.PX, lx = e - ly * it.PX;
            const int gy = wrapi(it.y0 - m + 1 + ly, a.n1);
            const int gx = wrapi(it.x0 - m + 1 + lx, a.n2);
            off[k] = gy * a.n2 + gx;
            lidx[k] = ly * it.PXp + lx;
        } else {
            off[k] = 0;
            lidx[k] = 0;
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

// Direct staging for unpadded complex<double> planes: each 16-byte element
// goes from global memory straight into LDS (buffer_load_dwordx4 ... lds;
// lane l of a wavefront writes the l-th 16 bytes after the wavefront's LDS
// base), so no registers hold the next plane.  The buffer resource spans one
// plane (offsets past it would read zero).  Completion is tracked by vmcnt:
// wait for it before the barrier that publishes the plane.  (The buffer form
// keeps the LDS counter free for selective waits on the stencil reads.)
template <int NF>
__device__ __forceinline__ void ps_fetch_lds(const c_t<double> *__restrict__ plane, int plane_bytes,
                                             const PSItem &it, const int *off, c_t<double> *buf) {
    const __amdgpu_buffer_rsrc_t rsrc =
        __builtin_amdgcn_make_buffer_rsrc((void *)plane, (short)0, plane_bytes, 0x00020000);
    const int wbase = threadIdx.x & ~63;
#pragma unroll
    for (int k = 0; k < NF; ++k) {
        const int e = threadIdx.x + k * kPsThreads;
        if (e < it.psz)
            __builtin_amdgcn_raw_ptr_buffer_load_lds(
                rsrc, (__attribute__((address_space(3))) void *)(buf + k * kPsThreads + wbase), 16, off[k] * 16, 0,
                0, 0);
    }
}

template <typename T, int NF>
__device__ __forceinline__ void ps_store(c_t<T> *buf, const PSItem &it, const int *lidx, const vec2_t<T> *v) {
    vec2_t<T> *b = reinterpret_cast<vec2_t<T> *>(buf);
#pragma unroll
    for (int k = 0; k < NF; ++k) {
        const int e = threadIdx.x + k * kPsThreads;
        if (e < it.psz) b[lidx[k]] = v[k];
    }
}

// ------------------------------------------------------------ interp ----
// Stencil reads without LDS bank conflicts.
//
// gfx950 serves a 16-byte-per-lane LDS read 16 lanes per clock; two lanes of
// one 16-lane group conflict when their addresses share a 16-byte bank group
// (address/16 mod 16).  The stencil is read in 16-byte units: one
// complex<double>, or an aligned pair of complex<float>.  complex<float>
// planes are staged twice, as is (first buffer) and shifted by one element
// (second buffer, element e at e + 1): a stencil row of W values starting on
// an even column is W/2 aligned pairs of the first copy, one starting on an
// odd column W/2 aligned pairs of the second, so no read carries a value
// outside the stencil.  At row step j a lane reads stencil row (j + t) mod W;
// the plane row stride RU (in units) is chosen with W*RU = 0 mod 16, so the
// bank group of its k-th unit at step j is u + RU*t + RU*j + k mod 16, u being
// the stencil's first unit.  RU*t runs over the multiples of
// D = 16/gcd(W, 16) (= gcd(RU, 16)), so each lane picks the rotation t that
// puts it on a target group of its own within its coset u mod D; with D = 1
// (complex<double>, m = 8) every 16-lane group reads conflict-free.  The y
// weights are rotated with the rows, once per point.

template <typename T> struct LdsUnit;
template <> struct LdsUnit<double> {
    using type = vec2_t<double>;
    static constexpr int EPU = 1;     // elements per 16-byte unit
};
template <> struct LdsUnit<float> {
    using type = float __attribute__((ext_vector_type(4)));
    static constexpr int EPU = 2;
};

constexpr int cgcd(int a, int b) { return b ? cgcd(b, a % b) : a; }

// 0: every item walks up; 1: odd items walk down; 2: odd items longer than
// 3 window widths walk down
constexpr int kInterpWalk = 1;

// largest divisor of n that is at most 7 (a chunk of stencil-row reads)
constexpr int row_chunk(int n) {
    for (int c = 7; c > 1; --c)
        if (n % c == 0) return c;
    return 1;
}

// Chunks of stencil-row reads issued ahead of the one being consumed.  The
// complex<double> form (16 reads of 16 B per row, two waves per SIMD) needs
// them in flight; the complex<float> form (5 reads per row, more waves)
// runs fastest with the compiler's own schedule (measured on MI355X).
template <typename T>
constexpr int interp_lookahead(int ch) {
    return sizeof(T) == 4 ? 0 : (15 / ch - 1 < 2 ? 15 / ch - 1 : 2);
}

// w[j] <- w[(j + t) mod W] for 0 <= t < NT (NT a power of two <= W).  The
// selects are done on the bit patterns: a select between two elements of the
// same array would otherwise be folded into one load at a lane-dependent
// index, which moves the array out of registers.
__device__ __forceinline__ float bitsel(bool c, float a, float b) {
    const unsigned m = c ? ~0u : 0u;
    return __uint_as_float((__float_as_uint(a) & m) | (__float_as_uint(b) & ~m));
}
__device__ __forceinline__ double bitsel(bool c, double a, double b) {
    const unsigned long long m = c ? ~0ull : 0ull;
    return __longlong_as_double((long long)(((unsigned long long)__double_as_longlong(a) & m) |
                                            ((unsigned long long)__double_as_longlong(b) & ~m)));
}

template <typename T, int W, int NT>
__device__ __forceinline__ void rotate_rows(T *w, int t) {
#pragma unroll
    for (int b = 1; b < NT; b <<= 1) {
        const bool on = (t & b) != 0;
        T tmp[W];
#pragma unroll
        for (int j = 0; j < W; ++j) tmp[j] = bitsel(on, w[(j + b) % W], w[j]);
#pragma unroll
        for (int j = 0; j < W; ++j) w[j] = tmp[j];
    }
}

// Direction of an item's walk over its planes.  Consecutive items of a tile
// column overlap in the 2m-1 planes at the top of one and the bottom of the
// next, and are dispatched together (see xcd_item): walking them in opposite
// directions makes both read the shared planes at about the same time, so
// the second read can hit in L2.
__device__ __forceinline__ bool interp_walk_down(int item, int nplanes, int W) {
    return kInterpWalk == 1 ? (item & 1) != 0 : kInterpWalk == 2 ? ((item & 1) != 0 && nplanes > 3 * W) : false;
}

// Point slot k of thread t is sorted index item.y + k*256 + t: each slot's
// wavefronts hold z-adjacent points, so they are active on the same planes.
// Derivative modes (kModeGrad, kModeFields) also form the derivative sums
// D_0 = sum w0' w1 w2 g, D_1 = sum w0 w1' w2 g, D_2 = sum w0 w1 w2' g (so
// d f_j / d x_{j,d} = n_d D_d): the y derivative weights rotate with the y
// weights and the x derivative weights are shifted like the x weights, so the
// reads are the same.  kModeGrad writes grad_x[j, d] = n_d Re(conj(G_j) D_d),
// kModeFields the field and the derivative fields n_d D_d of a.fmask.

// ROW1 (value mode of a one-dimensional plan, unit axes 0 and 1): every
// stencil row of the region is grid row 0 and only the first carries weight
// 1, so one row is staged and read, without rotation.
template <typename T, int W, int PPT, int MODE, bool ROW1 = false>
__device__ __forceinline__ void interp_range(const PSArgs &a, int item_index, const int4 item,
                                             unsigned char *smem_raw) {
    constexpr int m = W / 2;
    using U = typename LdsUnit<T>::type;
    constexpr int EPU = LdsUnit<T>::EPU;
    constexpr bool TWIN = EPU == 2;                // complex<float>: aligned + shifted copy
    constexpr bool GRAD = MODE != kModeValue;      // derivative sums
    constexpr int NR = EPU == 1 ? W : W / 2;       // units read per stencil row
    constexpr int NW = NR * EPU;                   // column weights per row
    constexpr int D = 16 / cgcd(W, 16);            // cosets of bank groups
    constexpr int NT = 16 / D;                     // distinct rotations
    static_assert(!ROW1 || MODE == kModeValue, "one-row walk in the value mode only");
    const PSItem it = ps_range(a, m, item.x, item.y, item.z, ROW1);
    const int RU = it.PXp / EPU;
    const int bufsz = it.PY * it.PXp;
    c_t<T> *buf0 = reinterpret_cast<c_t<T> *>(smem_raw);
    c_t<T> *buf1 = buf0 + bufsz;
    // pieces: rows of ZC coefficients (16-byte aligned) when the degree fits
    constexpr int ZC = zrow_len((int)sizeof(c_t<T>), W);
    const bool zfix = !GRAD && a.deg < ZC;
    const int zrow = zfix ? ZC : a.deg + 1;
    T *scoef = reinterpret_cast<T *>(smem_raw + ((2 * (size_t)bufsz * sizeof(c_t<T>) + 15) & ~(size_t)15));
    const T *coef = (const T *)a.coef;
    for (int i = threadIdx.x; i < W * zrow; i += kPsThreads) {
        const int r = i / zrow, q = i - r * zrow;
        scoef[i] = q <= a.deg ? coef[r * (a.deg + 1) + q] : (T)0;
    }

    const int lane = threadIdx.x & 63;
    const uint64_t below = lane ? (~0ull >> (64 - lane)) : 0ull;
    const uint64_t gmask = 0xFFFFull << (16 * (lane >> 4));
    const uint64_t hmask = 0xFFull << (8 * (lane >> 3));    // 8-lane half of the group
    constexpr int WG = GRAD ? W : 1, NWG = GRAD ? NW : 1;
    T w1[PPT][W], wt[PPT][NW];
    T d1[PPT][WG], dt[PPT][NWG];                   // GRAD: derivative weights
    T f0[PPT], ar[PPT], ai[PPT];
    T vr[PPT], vi[PPT];                            // kModeFields: the value
    T g1r[PPT], g1i[PPT], g2r[PPT], g2i[PPT];      // GRAD: D_1, D_2 (ar, ai hold D_0)
    int zlo[PPT], ub0[PPT], ub1[PPT], tt[PPT];
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        const int pk = item.y + k * kPsThreads + threadIdx.x;
        const bool active = pk < item.z;
        ar[k] = 0;
        ai[k] = 0;
        vr[k] = vi[k] = 0;
        g1r[k] = g1i[k] = g2r[k] = g2i[k] = 0;
        zlo[k] = -4 * W;     // never active
        f0[k] = 0;
        int s = 0;           // stencil's first element in the plane
        T w2[W], e2[WG];
#pragma unroll
        for (int r = 0; r < W; ++r) { w1[k][r] = 0; w2[r] = 0; }
#pragma unroll
        for (int r = 0; r < WG; ++r) { d1[k][r] = 0; e2[r] = 0; }
        if (active) {
            const double *xp = a.xs + 3 * (int64_t)pk;
            T f1, f2;
            const int zc = cell_frac<T>(xp[0], a.n0, f0[k]);
            const int yc = cell_frac<T>(xp[1], a.n1, f1);
            const int xc = cell_frac<T>(xp[2], a.n2, f2);
            s = (yc - it.y0) * it.PXp + (xc - it.x0);
            zlo[k] = (a.unit & 1) ? 0 : zc - m + 1 - it.zbeg;      // first plane index of the stencil
            if constexpr (GRAD) {
                window_weights_d<T, W>(f1, coef, a.deg, w1[k], d1[k]);
                window_weights_d<T, W>(f2, coef, a.deg, w2, e2);
            } else {
                if constexpr (!ROW1) window_weights<T, W>(f1, coef, a.deg, w1[k]);
                window_weights<T, W>(f2, coef, a.deg, w2);
            }
            if (a.unit & 2) {   // unit axis 1: every region row is grid row 0; weight 1 on one
#pragma unroll
                for (int r = 0; r < W; ++r) w1[k][r] = r == 0 ? (T)1 : (T)0;
#pragma unroll
                for (int r = 0; r < WG; ++r) d1[k][r] = 0;
            }
        }
        // first unit of the stencil row: complex<double> at s; complex<float>
        // with an even first column in the first copy (buf0) at s/2, with an
        // odd one in the shifted copy (buf1, element e at e + 1), (bufsz + s + 1)/2
        // units from buf0
        const int u = TWIN ? ((s & 1) ? (bufsz + s + 1) / 2 : s / 2) : s;
#pragma unroll
        for (int c = 0; c < NW; ++c) {
            wt[k][c] = w2[c];
            if constexpr (GRAD) dt[k][c] = e2[c];
        }
        // rank within the lane's coset and 16-lane group -> target bank group.
        // Two cosets: ranks are taken per 8-lane half and the halves get
        // disjoint target ranges (cs + 2 {0..3} and cs + 8 + 2 {0..3}), so the
        // targets are distinct within each half as well as within the group
        // (measured 2% faster than group-wide ranks for complex<float>, m = 4).
        // A coset holding more than 4 lanes of a half shares targets: the
        // cosets follow the stencils' columns and are not balanced.
        const int cs = u & (D - 1);
        int rank = 0;
#pragma unroll
        for (int c = 0; c < D; ++c) {
            const uint64_t mc = __ballot(active && cs == c);
            if (cs == c) rank = __popcll(mc & (D == 2 ? hmask : gmask) & below);
        }
        const int target = D == 2 ? cs + 2 * ((rank & 3) + 4 * ((lane >> 3) & 1)) : cs + D * (rank & (NT - 1));
        const int delta = (target - u) & 15;   // a multiple of D
        const int t = ROW1 ? 0 : ((delta / D) * a.qinv) & (NT - 1);
        if constexpr (!ROW1) rotate_rows<T, W, NT>(w1[k], t);
        if constexpr (GRAD) rotate_rows<T, W, NT>(d1[k], t);
        tt[k] = t;
        ub0[k] = u + t * RU;
        ub1[k] = ub0[k] - W * RU;
    }

    constexpr int NF = ps_nf<W>();
    int off[NF], lidx[NF];
    ps_offsets<NF>(a, it, m, off, lidx);
    const c_t<T> *grid = (const c_t<T> *)a.grid;
    const int64_t plane = (int64_t)a.n1 * a.n2;
    // complex<double> planes with an odd row length need no padding: stage
    // them directly (the host sets the row stride to PX in that case)
    constexpr bool kDirect = EPU == 1 && W == 16;
    vec2_t<T> stage[kDirect ? 1 : NF];
    const int plane_bytes = (int)(plane * (int64_t)sizeof(c_t<T>));
    // plane order: see interp_walk_down
    const bool down = interp_walk_down(item_index, it.nplanes, W);
    const int np = it.nplanes;
    if constexpr (kDirect) {
        ps_fetch_lds<NF>((const c_t<double> *)grid + (int64_t)wrapi(it.zbeg + (down ? np - 1 : 0), a.n0) * plane,
                         plane_bytes, it, off, (c_t<double> *)buf0);
        __builtin_amdgcn_s_waitcnt(0);
    } else {
        ps_fetch<T, NF>(grid, off, (int64_t)wrapi(it.zbeg + (down ? np - 1 : 0), a.n0) * plane, stage);
        ps_store<T, NF>(buf0, it, lidx, stage);
        if constexpr (TWIN) ps_store<T, NF>(buf1 + 1, it, lidx, stage);
    }
    __syncthreads();

    for (int st = 0; st < np; ++st) {
        const int i = down ? np - 1 - st : st;      // plane index of this step
        const bool more = st + 1 < np;
        if (more) {
            const int64_t zoff = (int64_t)wrapi(it.zbeg + (down ? i - 1 : i + 1), a.n0) * plane;
            if constexpr (kDirect)
                ps_fetch_lds<NF>((const c_t<double> *)grid + zoff, plane_bytes, it, off,
                                 (c_t<double> *)((st & 1) ? buf0 : buf1));
            else
                ps_fetch<T, NF>(grid, off, zoff, stage);
        }
        const U *pl = reinterpret_cast<const U *>(TWIN ? buf0 : ((st & 1) ? buf1 : buf0));
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            const int r0 = i - zlo[k];
            if (r0 >= 0 && r0 < W) {
                T dw0 = 0;
                T w0;
                if (a.unit & 1) w0 = 1;
                else if constexpr (GRAD) w0 = piece_d<T>(scoef + r0 * zrow, a.deg, f0[k], dw0);
                else if (zfix) w0 = piece_fixed<T, ZC>(scoef + r0 * ZC, f0[k]);
                else w0 = piece<T>(scoef + r0 * zrow, a.deg, f0[k]);
                T sr = 0, si = 0;
                T ur = 0, ui = 0, vr2 = 0, vi2 = 0;      // GRAD: sum d1 c, sum w1 q
                // Reads are software-pipelined in chunks of CH units of a
                // row: chunk q + LA is issued before chunk q is consumed, and
                // the scheduling barriers keep that order.  At most
                // (LA + 1) * CH <= 15 reads are outstanding, the most the LDS
                // counter can wait on selectively.
                constexpr int CH = row_chunk(NR);
                constexpr int S = NR / CH;             // chunks per row
                // (the derivative mode holds twice the weights: one chunk ahead)
                constexpr int LA = GRAD ? (interp_lookahead<T>(CH) > 0 ? 1 : 0) : interp_lookahead<T>(CH);
                constexpr int NQ = ROW1 ? S : W * S;      // ROW1: the first row only
                U g[LA + 1][CH];
#pragma unroll
                for (int q = 0; q < LA; ++q) {
                    const int j = q / S;
                    const U *row = pl + ((j + tt[k] < W) ? ub0[k] : ub1[k]) + j * RU + (q % S) * CH;
#pragma unroll
                    for (int c = 0; c < CH; ++c) g[q][c] = row[c];
                }
                T cr = 0, ci = 0, qr = 0, qi = 0;
#pragma unroll
                for (int q = 0; q < NQ; ++q) {
                    if (q + LA < NQ) {
                        const int q1 = q + LA, j1 = q1 / S;
                        const U *row = pl + ((j1 + tt[k] < W) ? ub0[k] : ub1[k]) + j1 * RU + (q1 % S) * CH;
#pragma unroll
                        for (int c = 0; c < CH; ++c) g[q1 % (LA + 1)][c] = row[c];
                    }
                    if constexpr (LA > 0) __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                    for (int c = 0; c < CH; ++c) {
                        const U v = g[q % (LA + 1)][c];
                        const int cc = (q % S) * CH + c;
                        if constexpr (EPU == 1) {
                            cr += wt[k][cc] * v.x;
                            ci += wt[k][cc] * v.y;
                            if constexpr (GRAD) {
                                qr += dt[k][cc] * v.x;
                                qi += dt[k][cc] * v.y;
                            }
                        } else {
                            cr += wt[k][2 * cc] * v.x;
                            ci += wt[k][2 * cc] * v.y;
                            cr += wt[k][2 * cc + 1] * v.z;
                            ci += wt[k][2 * cc + 1] * v.w;
                            if constexpr (GRAD) {
                                qr += dt[k][2 * cc] * v.x;
                                qi += dt[k][2 * cc] * v.y;
                                qr += dt[k][2 * cc + 1] * v.z;
                                qi += dt[k][2 * cc + 1] * v.w;
                            }
                        }
                    }
                    if (q % S == S - 1) {
                        if constexpr (ROW1) {
                            sr += cr;
                            si += ci;
                        } else {
                            sr += w1[k][q / S] * cr;
                            si += w1[k][q / S] * ci;
                        }
                        if constexpr (GRAD) {
                            ur += d1[k][q / S] * cr;
                            ui += d1[k][q / S] * ci;
                            vr2 += w1[k][q / S] * qr;
                            vi2 += w1[k][q / S] * qi;
                            qr = 0;
                            qi = 0;
                        }
                        cr = 0;
                        ci = 0;
                    }
                    if constexpr (LA > 0) __builtin_amdgcn_sched_barrier(0);
                }
                if constexpr (GRAD) {
                    ar[k] += dw0 * sr;    // D_0
                    ai[k] += dw0 * si;
                    g1r[k] += w0 * ur;    // D_1
                    g1i[k] += w0 * ui;
                    g2r[k] += w0 * vr2;   // D_2
                    g2i[k] += w0 * vi2;
                    if constexpr (MODE == kModeFields) {
                        vr[k] += w0 * sr;
                        vi[k] += w0 * si;
                    }
                } else {
                    ar[k] += w0 * sr;
                    ai[k] += w0 * si;
                }
            }
        }
        if constexpr (kDirect) {
            __builtin_amdgcn_s_waitcnt(0);
        } else if constexpr (TWIN) {
            __syncthreads();      // every read of this plane is done
            if (more) {
                ps_store<T, NF>(buf0, it, lidx, stage);
                ps_store<T, NF>(buf1 + 1, it, lidx, stage);
            }
        } else {
            if (more) ps_store<T, NF>((st & 1) ? buf0 : buf1, it, lidx, stage);
        }
        __syncthreads();
    }
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        const int pk = item.y + k * kPsThreads + threadIdx.x;
        if (pk >= item.z) continue;
        const int pj = a.perm[pk];
        if constexpr (MODE == kModeFields) {
            c_t<T> *o = (c_t<T> *)a.out;
            o[pj] = cmk<T>(vr[k], vi[k]);
            int64_t at = a.fstride + pj;
            if (a.fmask & 1) { o[at] = cmk<T>((T)a.n0 * ar[k], (T)a.n0 * ai[k]); at += a.fstride; }
            if (a.fmask & 2) { o[at] = cmk<T>((T)a.n1 * g1r[k], (T)a.n1 * g1i[k]); at += a.fstride; }
            if (a.fmask & 4) o[at] = cmk<T>((T)a.n2 * g2r[k], (T)a.n2 * g2i[k]);
        } else if constexpr (GRAD) {
            // Re(conj(G) D) = G.x D.x + G.y D.y, times n_d (dt/dx)
            const c_t<T> g = ((const c_t<T> *)a.vals)[pj];
            // the last gdim components (a plan of fewer axes drops its unit axes)
            double *gx = (double *)a.out + (int64_t)a.gdim * pj;
            const int c0 = 3 - a.gdim;     // component of axis d is gx[d - c0]
            if (c0 == 0) gx[0] = (double)a.n0 * ((double)g.x * (double)ar[k] + (double)g.y * (double)ai[k]);
            if (c0 <= 1) gx[1 - c0] = (double)a.n1 * ((double)g.x * (double)g1r[k] + (double)g.y * (double)g1i[k]);
            gx[2 - c0] = (double)a.n2 * ((double)g.x * (double)g2r[k] + (double)g.y * (double)g2i[k]);
        } else {
            ((c_t<T> *)a.out)[pj] = cmk<T>(ar[k], ai[k]);
        }
    }
}


template <typename T, int W, int PPT, bool ROW1 = false>
__device__ __forceinline__ void interp_body(const PSArgs &a, int item_index, unsigned char *smem_raw) {
    interp_range<T, W, PPT, kModeValue, ROW1>(a, item_index, a.items[item_index], smem_raw);
}

// Derivative modes: one point per thread (to stay within two waves per SIMD
// without spills at m = 8); items of more points are taken 256 at a time.
template <typename T, int W, int MODE>
__device__ __forceinline__ void interp_body_der(const PSArgs &a, int item_index, unsigned char *smem_raw) {
    const int4 item = a.items[item_index];
    for (int lo = item.y; lo < item.z; lo += kPsThreads) {
        __syncthreads();
        interp_range<T, W, 1, MODE>(a, item_index, make_int4(item.x, lo, min(item.z, lo + kPsThreads), 0), smem_raw);
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
    a.pxp = 0;
    a.qinv = 0;
    a.fmask = 0;
    a.fstride = 0;
    a.unit = p->unit;
    a.gdim = p->dim;
    return a;
}

// Row stride of the interp kernel's staged planes: at least PX (+2 for
// complex<float>, whose shifted copy holds element PX - 1 at PX), a whole number RU
// of 16-byte units with gcd(RU mod 16, 16) = D = 16/gcd(W, 16); and the
// inverse of RU/D modulo 16/D.
inline void interp_layout(const nfft3_plan_impl *p, PSArgs &a) {
    const int W = 2 * p->m;
    const int epu = p->elt == 16 ? 1 : 2;
    const int PX = p->bins.Bx + W - 1;
    const int D = 16 / std::gcd(W, 16);
    int pxp = PX + (epu == 2 ? 2 : 0);
    for (;; ++pxp) {
        if (pxp % epu) continue;
        const int q = (pxp / epu) % 16;
        if (q != 0 && std::gcd(q, 16) == D) break;
    }
    const int NT = 16 / D;
    const int qd = ((pxp / epu) % 16) / D;
    int qinv = 0;
    for (int v = 0; v < NT; ++v)
        if ((qd * v) % NT == 1 % NT) { qinv = v; break; }
    a.pxp = pxp;
    a.qinv = qinv;
}

inline PSArgs interp_args(const nfft3_plan_impl *p) {
    PSArgs a = ps_args(p);
    interp_layout(p, a);
    return a;
}

// The direct (global -> LDS) staging of complex<double>, m = 8 writes each
// wavefront's elements contiguously, so it needs unpadded rows.
inline bool interp_layout_ok(const nfft3_plan_impl *p, const PSArgs &a) {
    return !(p->elt == 16 && p->m == 8) || a.pxp == p->bins.Bx + 2 * p->m - 1;
}

// LDS bytes of the interp kernel: two staged planes + the coefficient rows
// (16-byte aligned, zrow_len long when the degree fits).
inline size_t interp_lds(const nfft3_plan_impl *p, const PSArgs &a) {
    const int W = 2 * p->m;
    const size_t bufsz = (size_t)(p->bins.By + W - 1) * a.pxp;
    const int zrow = std::max(zrow_len(p->elt, W), p->deg + 1);
    return ((2 * bufsz * p->elt + 15) & ~(size_t)15) + (size_t)W * zrow * (p->elt / 2);
}

// LDS bytes of the window-sum kernels: nbuf staged planes + the coefficients.
inline size_t ps_lds(const nfft3_plan_impl *p, int nbuf) {
    const int W = 2 * p->m;
    const size_t psz = (size_t)(p->bins.By + W - 1) * (p->bins.Bx + W - 1);
    return nbuf * psz * p->elt + (size_t)W * (p->deg + 1) * (p->elt / 2);
}

// Dispatch on the half-width m to the stencil-width template W = 2m.
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

}  // namespace nfft3
