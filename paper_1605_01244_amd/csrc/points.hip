// Point preprocessing (the precomputation step of the windowed method):
// fold every point into [-1/2, 1/2) with the Euclidean remainder of
// Sec. 2.2.1, locate its grid cell u_d = floor(n_d x_d) in FP64, and sort the
// points with a counting sort (histogram -> exclusive scan -> scatter) by the
// key (tile, z-cell), where a tile is a By x Bx block of cells in the (y, x)
// plane and z (axis 0) varies fastest.  Each tile column is then cut into
// work items of at most maxpts points spanning at most kItemZ z-cells; a
// workgroup of the window-sum kernels takes one item and streams the z-planes
// of its tile (plus the stencil halo) through LDS.
#include <algorithm>

#include "internal.h"

namespace nfft3 {

constexpr int kPtThreads = 256;
constexpr int kScanBlock = 1024;     // elements per block of the scan
constexpr int kScanThreads = 256;

__device__ __forceinline__ double fold_unit(double v) {
    double r = v - rint(v);          // exact; in [-1/2, 1/2]
    return r >= 0.5 ? r - 1.0 : r;   // +1/2 belongs to the next period
}

struct BinGeom {
    double n0, n1, n2;
    int in0, in1, in2;
    int By, Bx;
    int nty, ntx;
};

__device__ __forceinline__ int cell_of(double r, double nd, int ind) {
    int c = (int)floor(nd * r);
    if (c < 0) c += ind;
    return c >= ind ? c - ind : c;
}

__device__ __forceinline__ int bin_of_point(const double *xp, const BinGeom &g) {
    const int c0 = cell_of(fold_unit(xp[0]), g.n0, g.in0);
    const int c1 = cell_of(fold_unit(xp[1]), g.n1, g.in1);
    const int c2 = cell_of(fold_unit(xp[2]), g.n2, g.in2);
    return ((c1 / g.By) * g.ntx + c2 / g.Bx) * g.in0 + c0;
}

__global__ void fill_int_kernel(int *p, int64_t count, int v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = v;
}

__global__ void __launch_bounds__(kPtThreads)
bin_count_kernel(const double *__restrict__ x, int64_t M, BinGeom g, int *__restrict__ counts,
                 int *__restrict__ bin_of, int *__restrict__ rank, int *__restrict__ flag) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= M) return;
    const double *xp = x + 3 * j;
    int b = 0;
    if (isfinite(xp[0]) && isfinite(xp[1]) && isfinite(xp[2])) {
        b = bin_of_point(xp, g);
    } else {
        atomicOr(flag, 1);
    }
    // counter copy of this workgroup (see kBinCopies)
    const int c = b * kBinCopies + (int)(blockIdx.x & (kBinCopies - 1));
    bin_of[j] = c;
    rank[j] = atomicAdd(&counts[c], 1);
}

// ---- exclusive scan: block-local scans, a scan of block sums, then add ------
__device__ __forceinline__ int block_exclusive_scan(int v, int *sh, int &total) {
    const int tid = threadIdx.x;
    sh[tid] = v;
    __syncthreads();
    for (int off = 1; off < kScanThreads; off <<= 1) {
        int t = tid >= off ? sh[tid - off] : 0;
        __syncthreads();
        sh[tid] += t;
        __syncthreads();
    }
    total = sh[kScanThreads - 1];
    int ex = sh[tid] - v;
    __syncthreads();
    return ex;
}

__global__ void __launch_bounds__(kScanThreads)
scan_blocks_kernel(const int *__restrict__ in, int *__restrict__ out, int *__restrict__ block_sums, int64_t n) {
    __shared__ int sh[kScanThreads];
    constexpr int per = kScanBlock / kScanThreads;
    const int64_t base = (int64_t)blockIdx.x * kScanBlock + threadIdx.x * per;
    int v[per];
    int s = 0;
#pragma unroll
    for (int i = 0; i < per; ++i) {
        v[i] = base + i < n ? in[base + i] : 0;
        s += v[i];
    }
    int total;
    int run = block_exclusive_scan(s, sh, total);
#pragma unroll
    for (int i = 0; i < per; ++i) {
        if (base + i < n) out[base + i] = run;
        run += v[i];
    }
    if (threadIdx.x == 0) block_sums[blockIdx.x] = total;
}

// single workgroup: exclusive scan of nb block sums in place; writes the total
__global__ void __launch_bounds__(kScanThreads)
scan_sums_kernel(int *__restrict__ sums, int64_t nb, int *__restrict__ total_out) {
    __shared__ int sh[kScanThreads];
    int carry = 0;
    for (int64_t start = 0; start < nb; start += kScanThreads) {
        const int64_t i = start + threadIdx.x;
        int v = i < nb ? sums[i] : 0;
        int total;
        int ex = block_exclusive_scan(v, sh, total);
        if (i < nb) sums[i] = carry + ex;
        carry += total;
    }
    if (threadIdx.x == 0) *total_out = carry;
}

__global__ void add_block_offsets_kernel(int *__restrict__ out, const int *__restrict__ sums, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] += sums[i / kScanBlock];
}

// exclusive scan of n ints (in -> out), out[n] = total; sums needs ceil(n/1024) ints
static int exclusive_scan(hipStream_t s, const int *in, int *out, int *sums, int64_t n) {
    if (n <= 0) {
        hipLaunchKernelGGL(fill_int_kernel, dim3(1), dim3(64), 0, s, out, (int64_t)1, 0);
        NFFT3_LAUNCH_CHECK("fill_int_kernel");
        return NFFT3_OK;
    }
    const int64_t nb = (n + kScanBlock - 1) / kScanBlock;
    hipLaunchKernelGGL(scan_blocks_kernel, dim3((unsigned)nb), dim3(kScanThreads), 0, s, in, out, sums, n);
    NFFT3_LAUNCH_CHECK("scan_blocks_kernel");
    hipLaunchKernelGGL(scan_sums_kernel, dim3(1), dim3(kScanThreads), 0, s, sums, nb, out + n);
    NFFT3_LAUNCH_CHECK("scan_sums_kernel");
    hipLaunchKernelGGL(add_block_offsets_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, out, sums, n);
    NFFT3_LAUNCH_CHECK("add_block_offsets_kernel");
    return NFFT3_OK;
}

__global__ void __launch_bounds__(kPtThreads)
scatter_kernel(const double *__restrict__ x, int64_t M, const int *__restrict__ offsets,
               const int *__restrict__ bin_of, const int *__restrict__ rank, double *__restrict__ xs,
               int *__restrict__ perm) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= M) return;
    const int64_t pos = (int64_t)offsets[bin_of[j]] + rank[j];
    const double *xp = x + 3 * j;
    xs[3 * pos + 0] = fold_unit(xp[0]);
    xs[3 * pos + 1] = fold_unit(xp[1]);
    xs[3 * pos + 2] = fold_unit(xp[2]);
    perm[pos] = (int)j;
}

int launch_exclusive_scan(hipStream_t s, const int *in, int *out, int *sums, int64_t n) {
    return exclusive_scan(s, in, out, sums, n);
}

// ---- two-level counting sort (tile, then z within the tile) ---------------
// One global atomic per point (the single-level sort above) runs at the
// device's atomic rate, and its scatter writes 24 bytes at a random place
// per point.  The two-level sort works on chunks of kSortChunk points per
// workgroup.  Level 1 keys by tile (input order -> tile order): a count pass
// writes each chunk's per-tile counts into a (tile, chunk) matrix, whose
// exclusive scan gives every (tile, chunk) run its final start (no
// atomics: one counter per tile would take an atomic from every chunk).
// Level 2 keys by z-cell within chunks that never cross a tile (tile order
// -> (tile, z) order); its bins are many and lightly contended, so a run is
// reserved with one global atomic per (chunk, bin).  A scatter pass ranks
// the chunk again in LDS (any order within a key will do: the run's length
// is what was counted), computes each point's destination, and then moves
// the data one field at a time through LDS: coalesced reads in the chunk's
// order, coalesced runs of writes in the sorted order.  The order within a
// (tile, z) bin depends on the atomics (as before).
constexpr int kSortChunk = 2048;                 // points per workgroup
constexpr int kSortPer = kSortChunk / kPtThreads;
constexpr int kSortMaxTiles = 8192;              // LDS counters of level 1
// (tile, chunk) counts of level 1 and (chunk, z) bases of level 2: at most
constexpr int64_t kSortMaxBases = int64_t(1) << 25;

__device__ __forceinline__ int point_tile(const double *xp, const BinGeom &g, bool &finite) {
    finite = isfinite(xp[0]) && isfinite(xp[1]) && isfinite(xp[2]);
    if (!finite) return 0;         // reported through the flag; the sort is then discarded
    const int c1 = cell_of(fold_unit(xp[1]), g.n1, g.in1);
    const int c2 = cell_of(fold_unit(xp[2]), g.n2, g.in2);
    return (c1 / g.By) * g.ntx + c2 / g.Bx;
}

// In-place exclusive scan of n LDS ints by the workgroup (kPtThreads
// threads, contiguous segments per thread); sh holds kPtThreads ints.
__device__ void lds_exclusive_scan(int *a, int n, int *sh) {
    const int per = (n + kPtThreads - 1) / kPtThreads;
    const int b = threadIdx.x * per, e = min(n, b + per);
    int sum = 0;
    for (int i = b; i < e; ++i) sum += a[i];
    int total;
    int run = block_exclusive_scan(sum, sh, total);
    for (int i = b; i < e; ++i) {
        const int v = a[i];
        a[i] = run;
        run += v;
    }
    __syncthreads();
}

// Move one field of a chunk into sorted order through LDS: value v[i] of
// the thread's i-th point goes to slot sl[i]; slot s (s = threadIdx + k 256)
// is written to out[dest[k]] (stride elements apart for interleaved output).
template <typename V>
__device__ __forceinline__ void stage_field(V *buf, const V *v, const int *sl, const int64_t *dest, int nv, V *out,
                                            int stride, int comp) {
#pragma unroll
    for (int i = 0; i < kSortPer; ++i)
        if (i * kPtThreads + (int)threadIdx.x < nv) buf[sl[i]] = v[i];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kSortPer; ++k) {
        const int s = k * kPtThreads + threadIdx.x;
        if (s < nv) out[dest[k] * stride + comp] = buf[s];
    }
    __syncthreads();
}

// level 1 count: counts[t * nchunks + chunk]
__global__ void __launch_bounds__(kPtThreads)
tile_count_kernel(const double *__restrict__ x, int64_t M, BinGeom g, int ntiles, int *__restrict__ counts,
                  int *__restrict__ flag) {
    extern __shared__ int cnt[];                 // ntiles
    for (int t = threadIdx.x; t < ntiles; t += kPtThreads) cnt[t] = 0;
    __syncthreads();
    const int64_t c0 = (int64_t)blockIdx.x * kSortChunk;
    bool bad = false;
#pragma unroll 4
    for (int i = 0; i < kSortPer; ++i) {
        const int64_t j = c0 + i * kPtThreads + threadIdx.x;
        if (j < M) {
            bool finite;
            const int t = point_tile(x + 3 * j, g, finite);
            bad = bad || !finite;
            atomicAdd(&cnt[t], 1);
        }
    }
    if (bad) atomicOr(flag, 1);
    __syncthreads();
    for (int t = threadIdx.x; t < ntiles; t += kPtThreads) counts[(int64_t)t * gridDim.x + blockIdx.x] = cnt[t];
}

// tile starts from the scanned (tile, chunk) matrix: tile_start[t] = run
// start of (t, chunk 0); tile_start[ntiles] = M
__global__ void tile_start_kernel(const int *__restrict__ starts, int nchunks, int ntiles, int M,
                                  int *__restrict__ tile_start) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < ntiles) tile_start[t] = starts[(int64_t)t * nchunks];
    if (t == ntiles) tile_start[t] = M;
}

// level 1 scatter: folded coordinates (three arrays), caller index and
// z-cell in tile order; each point is read once and held in registers
__global__ void __launch_bounds__(kPtThreads)
tile_scatter_kernel(const double *__restrict__ x, int64_t M, BinGeom g, int ntiles, const int *__restrict__ starts,
                    double *__restrict__ tx, int *__restrict__ tperm, int *__restrict__ tz) {
    extern __shared__ __align__(16) int sm[];    // ntiles offsets (8-byte aligned), then a field of the chunk
    __shared__ int sh[kPtThreads];
    int *lofs = sm;
    double *buf = (double *)(sm + ((ntiles + 1) & ~1));
    for (int t = threadIdx.x; t < ntiles; t += kPtThreads) lofs[t] = 0;
    __syncthreads();
    const int64_t c0 = (int64_t)blockIdx.x * kSortChunk;
    const int nv = (int)min<int64_t>(kSortChunk, M - c0);
    int key[kSortPer], sl[kSortPer], zc[kSortPer];
    double f[3][kSortPer];
#pragma unroll
    for (int i = 0; i < kSortPer; ++i) {
        const int li = i * kPtThreads + threadIdx.x;
        key[i] = 0;
        sl[i] = 0;
        zc[i] = 0;
        f[0][i] = f[1][i] = f[2][i] = 0.0;
        if (li < nv) {
            const double *xp = x + 3 * (c0 + li);
            const double a = xp[0], b = xp[1], c = xp[2];
            // a non-finite point goes to tile 0 at the origin (reported
            // through the flag by tile_count_kernel)
            if (isfinite(a) && isfinite(b) && isfinite(c)) {
                f[0][i] = fold_unit(a);
                f[1][i] = fold_unit(b);
                f[2][i] = fold_unit(c);
            }
            const int c1 = cell_of(f[1][i], g.n1, g.in1), c2 = cell_of(f[2][i], g.n2, g.in2);
            key[i] = (c1 / g.By) * g.ntx + c2 / g.Bx;
            zc[i] = cell_of(f[0][i], g.n0, g.in0);
            sl[i] = atomicAdd(&lofs[key[i]], 1);
        }
    }
    __syncthreads();
    lds_exclusive_scan(lofs, ntiles, sh);
    // destination of each slot: the (tile, chunk) run start + rank in the run
    int *dslot = (int *)buf;
#pragma unroll
    for (int i = 0; i < kSortPer; ++i) {
        const int li = i * kPtThreads + threadIdx.x;
        if (li < nv) {
            const int r = sl[i];
            sl[i] = lofs[key[i]] + r;
            dslot[sl[i]] = starts[(int64_t)key[i] * gridDim.x + blockIdx.x] + r;
        }
    }
    __syncthreads();
    int64_t dest[kSortPer];
#pragma unroll
    for (int k = 0; k < kSortPer; ++k) {
        const int s = k * kPtThreads + threadIdx.x;
        dest[k] = s < nv ? dslot[s] : 0;
    }
    __syncthreads();
    for (int d = 0; d < 3; ++d) stage_field<double>(buf, f[d], sl, dest, nv, tx + d * M, 1, 0);
    int *ibuf = (int *)buf;
    int v[kSortPer];
#pragma unroll
    for (int i = 0; i < kSortPer; ++i) v[i] = (int)(c0 + i * kPtThreads + threadIdx.x);
    stage_field<int>(ibuf, v, sl, dest, nv, tperm, 1, 0);
    stage_field<int>(ibuf, zc, sl, dest, nv, tz, 1, 0);
}

// chunks of level 2 per tile: ceil(count / kSortChunk)
__global__ void tile_chunks_kernel(const int *__restrict__ tile_start, int ntiles, int *__restrict__ nchunks) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < ntiles) nchunks[t] = (tile_start[t + 1] - tile_start[t] + kSortChunk - 1) / kSortChunk;
}

// chunk b of level 2 -> its tile (last t with chunk_start[t] <= b) and range
__device__ __forceinline__ bool level2_chunk(const int *__restrict__ chunk_start, const int *__restrict__ tile_start,
                                             int ntiles, int b, int &t, int &lo, int &hi) {
    if (b >= chunk_start[ntiles]) return false;
    int a = 0, z = ntiles - 1;
    while (a < z) {
        const int mid = (a + z + 1) >> 1;
        if (chunk_start[mid] <= b) a = mid;
        else z = mid - 1;
    }
    t = a;
    lo = tile_start[t] + (b - chunk_start[t]) * kSortChunk;
    hi = min(tile_start[t + 1], lo + kSortChunk);
    return true;
}

// level 2 count: chunk bases per (chunk, z) present
__global__ void __launch_bounds__(kPtThreads)
z_count_kernel(const int *__restrict__ tz, const int *__restrict__ tile_start, const int *__restrict__ chunk_start,
               int ntiles, int n0, int *__restrict__ bin_counts, int *__restrict__ chunk_base) {
    extern __shared__ int cnt[];                 // n0
    int t, lo, hi;
    if (!level2_chunk(chunk_start, tile_start, ntiles, blockIdx.x, t, lo, hi)) return;
    for (int z = threadIdx.x; z < n0; z += kPtThreads) cnt[z] = 0;
    __syncthreads();
    for (int64_t p = (int64_t)lo + threadIdx.x; p < hi; p += kPtThreads) atomicAdd(&cnt[tz[p]], 1);
    __syncthreads();
    int *bc = bin_counts + (int64_t)t * n0;
    int *cb = chunk_base + (int64_t)blockIdx.x * n0;
    for (int z = threadIdx.x; z < n0; z += kPtThreads)
        if (cnt[z]) cb[z] = atomicAdd(&bc[z], cnt[z]);
}

// level 2 scatter into (tile, z) order
__global__ void __launch_bounds__(kPtThreads)
z_scatter_kernel(const double *__restrict__ tx, const int *__restrict__ tperm, const int *__restrict__ tz,
                 int64_t M, const int *__restrict__ tile_start, const int *__restrict__ chunk_start, int ntiles,
                 int n0, const int *__restrict__ bin_start, const int *__restrict__ chunk_base,
                 double *__restrict__ xs, int *__restrict__ perm) {
    extern __shared__ __align__(16) int sm[];    // n0 offsets (8-byte aligned), then three fields of the chunk
    __shared__ int sh[kPtThreads];
    int t, lo, hi;
    if (!level2_chunk(chunk_start, tile_start, ntiles, blockIdx.x, t, lo, hi)) return;
    int *lofs = sm;
    double *buf = (double *)(sm + ((n0 + 1) & ~1));
    for (int z = threadIdx.x; z < n0; z += kPtThreads) lofs[z] = 0;
    __syncthreads();
    const int nv = hi - lo;
    int key[kSortPer], sl[kSortPer];
#pragma unroll
    for (int i = 0; i < kSortPer; ++i) {
        const int li = i * kPtThreads + threadIdx.x;
        key[i] = 0;
        sl[i] = 0;
        if (li < nv) {
            key[i] = tz[(int64_t)lo + li];
            sl[i] = atomicAdd(&lofs[key[i]], 1);
        }
    }
    __syncthreads();
    lds_exclusive_scan(lofs, n0, sh);
    const int *cb = chunk_base + (int64_t)blockIdx.x * n0;
    const int *bs = bin_start + (int64_t)t * n0;
    int *dslot = (int *)buf;
#pragma unroll
    for (int i = 0; i < kSortPer; ++i) {
        const int li = i * kPtThreads + threadIdx.x;
        if (li < nv) {
            const int r = sl[i];
            sl[i] = lofs[key[i]] + r;
            dslot[sl[i]] = bs[key[i]] + cb[key[i]] + r;
        }
    }
    __syncthreads();
    int64_t dest[kSortPer];
#pragma unroll
    for (int k = 0; k < kSortPer; ++k) {
        const int s = k * kPtThreads + threadIdx.x;
        dest[k] = s < nv ? dslot[s] : 0;
    }
    __syncthreads();
    // the three coordinates go through LDS together, so each point's 24
    // bytes are written at once (three strided passes would leave partly
    // written lines between passes)
#pragma unroll
    for (int i = 0; i < kSortPer; ++i) {
        const int li = i * kPtThreads + threadIdx.x;
        if (li < nv) {
#pragma unroll
            for (int d = 0; d < 3; ++d) buf[d * kSortChunk + sl[i]] = tx[d * M + lo + li];
        }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kSortPer; ++k) {
        const int s = k * kPtThreads + threadIdx.x;
        if (s < nv) {
            double *o = xs + 3 * dest[k];
            o[0] = buf[s];
            o[1] = buf[kSortChunk + s];
            o[2] = buf[2 * kSortChunk + s];
        }
    }
    __syncthreads();
    int v[kSortPer];
#pragma unroll
    for (int i = 0; i < kSortPer; ++i) {
        const int li = i * kPtThreads + threadIdx.x;
        v[i] = li < nv ? tperm[(int64_t)lo + li] : 0;
    }
    stage_field<int>((int *)buf, v, sl, dest, nv, perm, 1, 0);
}

// ---- points of a lower-dimensional plan -----------------------------------
// x3[j] = (0, .., 0, x[j][0], .., x[j][dim-1]): the leading unit axes take
// coordinate 0 (their only frequency is 0, so any value gives the same sum).
__global__ void __launch_bounds__(kPtThreads)
widen_points_kernel(const double *__restrict__ x, int64_t M, int dim, double *__restrict__ x3) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= 3 * M) return;
    const int64_t j = e / 3;
    const int c = (int)(e - 3 * j) - (3 - dim);
    x3[e] = c >= 0 ? x[j * dim + c] : 0.0;
}

int launch_widen_points(hipStream_t s, int64_t M, int dim, const double *x, double *x3) {
    if (M <= 0) return NFFT3_OK;
    hipLaunchKernelGGL(widen_points_kernel, dim3((unsigned)((3 * M + kPtThreads - 1) / kPtThreads)),
                       dim3(kPtThreads), 0, s, x, M, dim, x3);
    NFFT3_LAUNCH_CHECK("widen_points_kernel");
    return NFFT3_OK;
}

// ---- do the sorted points still describe x? ------------------------------
// Sorted position q holds fold(x[perm[q]]) from the last sort.  If every
// position still equals the fold of the caller's current coordinates (bit for
// bit), a new sort would yield the same bins and items, so it can be skipped.
// Any difference (or a NaN, which never compares equal) sets bit 1 of flag.
__global__ void __launch_bounds__(kPtThreads)
points_equal_kernel(const double *__restrict__ x, int64_t M, const double *__restrict__ xs,
                    const int *__restrict__ perm, int *__restrict__ flag) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= M) return;
    const int64_t j = perm[q];
    bool same = j >= 0 && j < M;
    if (same) {
        const double *xp = x + 3 * j;
        const double *sp = xs + 3 * q;
#pragma unroll
        for (int d = 0; d < 3; ++d)
            same = same && __double_as_longlong(fold_unit(xp[d])) == __double_as_longlong(sp[d]);
    }
    if (!same) atomicOr(flag + 1, 2);
}

int launch_points_equal(nfft3_plan_impl *p, int64_t M, const double *x, int *equal) {
    hipStream_t s = p->stream;
    hipLaunchKernelGGL(fill_int_kernel, dim3(1), dim3(256), 0, s, p->flag, (int64_t)16, 0);
    NFFT3_LAUNCH_CHECK("fill_int_kernel");
    if (M > 0) {
        hipLaunchKernelGGL(points_equal_kernel, dim3((unsigned)((M + kPtThreads - 1) / kPtThreads)),
                           dim3(kPtThreads), 0, s, x, M, p->xs, p->perm, p->flag);
        NFFT3_LAUNCH_CHECK("points_equal_kernel");
    }
    int w = 0;
    NFFT3_HIP_TRY(hipMemcpyAsync(&w, p->flag + 1, sizeof(int), hipMemcpyDeviceToHost, s));
    NFFT3_HIP_TRY(hipStreamSynchronize(s));
    *equal = (w & 2) ? 0 : 1;
    return NFFT3_OK;
}

__global__ void copy_int_kernel(const int *__restrict__ src, int *__restrict__ dst) { *dst = *src; }

// ---- work items: greedy walks over segments of each tile column ----------
// A tile column is cut into segments of kItemZ z-cells, one wave per
// segment: lane e loads the start of cell z0 + e (coalesced) and the cell
// counts follow by a shuffle; the greedy walk over the cells then runs on
// wave-uniform values (read lane by lane), and lane 0 writes the items: a new
// item starts when adding the next cell would exceed maxpts points, and a
// cell holding more than maxpts points becomes ceil(count/maxpts) items of
// its own.  Items never cross a segment boundary, so none spans more than
// kItemZ cells.  WRITE=false counts the items of each (tile, segment),
// WRITE=true emits (tile, p_lo, p_hi, 0) at the scanned offsets, i.e. in
// (tile, z) order.  (One thread per segment, walking 65 loaded starts, took
// 3x longer: few waves, and every load a different line.)
constexpr int kItemThreads = 64;         // one wave per segment
static_assert(kItemZ == kItemThreads, "one lane per cell of a segment");

template <bool WRITE>
__global__ void __launch_bounds__(kItemThreads)
items_kernel(const int *__restrict__ offsets, int copies, int ntiles, int n0, int nseg, int maxpts,
             int *__restrict__ item_count, const int *__restrict__ item_offset, int4 *__restrict__ items,
             int64_t cap, int *__restrict__ flag) {
    const int64_t q = blockIdx.x;
    if (q >= (int64_t)ntiles * nseg) return;
    const int tile = (int)(q / nseg), seg = (int)(q - (int64_t)tile * nseg);
    const int z0 = seg * kItemZ, z1 = min(n0, z0 + kItemZ);
    const int lane = threadIdx.x;
    // bin (tile, z) spans offsets[(tile n0 + z) K] .. offsets[(tile n0 + z + 1) K],
    // K = copies counters per bin
    const int *g = offsets + (int64_t)tile * n0 * copies;
    const int oz = g[(int64_t)min(z0 + lane, z1) * copies];
    const int oend = g[(int64_t)z1 * copies];
    // (the shuffle runs on every lane: under a branch, the last lane would
    // not take part, and its neighbour would read nothing from it)
    const int oright = __shfl_down(oz, 1);
    const int onext = lane + 1 < kItemThreads ? oright : oend;
    const int cnt = z0 + lane < z1 ? onext - oz : 0;
    const int64_t w = WRITE ? item_offset[q] : 0;
    const bool writer = WRITE && lane == 0;
    int k = 0, cur = 0, p_start = 0;
    for (int e = 0; e < z1 - z0; ++e) {
        const int c = __builtin_amdgcn_readlane(cnt, e);
        if (c == 0) continue;
        const int o = __builtin_amdgcn_readlane(oz, e);
        if (cur > 0 && cur + c > maxpts) {
            if (writer && w + k < cap) items[w + k] = make_int4(tile, p_start, p_start + cur, 0);
            ++k;
            cur = 0;
        }
        if (c > maxpts) {     // a dense cell on its own
            for (int s0 = 0; s0 < c; s0 += maxpts) {
                if (writer && w + k < cap) items[w + k] = make_int4(tile, o + s0, o + min(c, s0 + maxpts), 0);
                ++k;
            }
            continue;
        }
        if (cur == 0) p_start = o;
        cur += c;
    }
    if (cur > 0) {
        if (writer && w + k < cap) items[w + k] = make_int4(tile, p_start, p_start + cur, 0);
        ++k;
    }
    if (!WRITE && lane == 0) item_count[q] = k;
    // the list is sized by max_items; should it ever be short, report it
    if (writer && w + k > cap) atomicOr(flag, 4);
}

// Items of a tiling with ntiles tile columns of n0 cells for M points, at
// most: an item cut because the next (regular) cell would overflow it holds,
// with its successor in the segment, more than maxpts points, so such items
// number below 2 P / maxpts for the P points of regular cells; a dense cell
// of c points makes under 2 c / maxpts items and cuts at most one; each of
// the ceil(n0 / kItemZ) segments of a column ends one more.
int64_t max_items(int64_t M, int64_t ntiles, int64_t n0, int maxpts) {
    return 3 * ((M + maxpts - 1) / maxpts) + ntiles * (n0 / kItemZ + 2) + 1;
}

// Single-level sort (one global atomic per point, kBinCopies counters per
// bin): for tilings with more than kSortMaxTiles tiles, whose level-1 LDS
// histogram would not fit.
static int sort_single_level(nfft3_plan_impl *p, int64_t M, const double *x, const BinGeom &g) {
    const int64_t nb = p->bins.nbins * kBinCopies;   // counters: kBinCopies per bin
    hipStream_t s = p->stream;
    hipLaunchKernelGGL(fill_int_kernel, dim3((unsigned)((nb + 255) / 256)), dim3(256), 0, s, p->bins.counts, nb, 0);
    NFFT3_LAUNCH_CHECK("fill_int_kernel");
    const unsigned blocks = (unsigned)((M + kPtThreads - 1) / kPtThreads);
    if (M > 0) {
        hipLaunchKernelGGL(bin_count_kernel, dim3(blocks), dim3(kPtThreads), 0, s, x, M, g, p->bins.counts,
                           p->bin_of, p->rank, p->flag);
        NFFT3_LAUNCH_CHECK("bin_count_kernel");
    }
    int rc = exclusive_scan(s, p->bins.counts, p->bins.offsets, p->bins.scratch, nb);
    if (rc) return rc;
    if (M > 0) {
        hipLaunchKernelGGL(scatter_kernel, dim3(blocks), dim3(kPtThreads), 0, s, x, M, p->bins.offsets,
                           p->bin_of, p->rank, p->xs, p->perm);
        NFFT3_LAUNCH_CHECK("scatter_kernel");
    }
    return NFFT3_OK;
}

// Two-level sort (see tile_count_kernel); bins.offsets receives the nbins + 1
// bin starts.
static int sort_two_level(nfft3_plan_impl *p, int64_t M, const double *x, const BinGeom &g) {
    const int ntiles = g.nty * g.ntx;
    const int64_t nb = p->bins.nbins;
    hipStream_t s = p->stream;
    Bins &B = p->bins;
    const int chunks1 = (int)((M + kSortChunk - 1) / kSortChunk);
    hipLaunchKernelGGL(fill_int_kernel, dim3((unsigned)((nb + 255) / 256)), dim3(256), 0, s, B.counts, nb, 0);
    NFFT3_LAUNCH_CHECK("fill_int_kernel");
    const size_t lds1 = sizeof(int) * (((size_t)ntiles + 1) & ~(size_t)1) + sizeof(double) * kSortChunk;
    const size_t lds2 = sizeof(int) * (((size_t)g.in0 + 1) & ~(size_t)1) + 3 * sizeof(double) * kSortChunk;
    allow_lds((const void *)tile_count_kernel, sizeof(int) * ntiles);
    allow_lds((const void *)tile_scatter_kernel, lds1);
    allow_lds((const void *)z_scatter_kernel, lds2);
    if (M > 0) {
        // (tile, chunk) counts -> run starts in place
        hipLaunchKernelGGL(tile_count_kernel, dim3(chunks1), dim3(kPtThreads), sizeof(int) * ntiles, s, x, M, g,
                           ntiles, p->chunk_base, p->flag);
        NFFT3_LAUNCH_CHECK("tile_count_kernel");
        int rc = exclusive_scan(s, p->chunk_base, p->chunk_base, p->sort_scratch, (int64_t)chunks1 * ntiles);
        if (rc) return rc;
        hipLaunchKernelGGL(tile_start_kernel, dim3((unsigned)((ntiles + 256) / 256)), dim3(256), 0, s, p->chunk_base,
                           chunks1, ntiles, (int)M, B.tile_start);
        NFFT3_LAUNCH_CHECK("tile_start_kernel");
        hipLaunchKernelGGL(tile_scatter_kernel, dim3(chunks1), dim3(kPtThreads), lds1, s, x, M, g, ntiles,
                           p->chunk_base, p->tx, p->tperm, p->tz);
        NFFT3_LAUNCH_CHECK("tile_scatter_kernel");
    } else {
        hipLaunchKernelGGL(fill_int_kernel, dim3((unsigned)((ntiles + 256) / 256)), dim3(256), 0, s, B.tile_start,
                           (int64_t)ntiles + 1, 0);
        NFFT3_LAUNCH_CHECK("fill_int_kernel");
    }
    hipLaunchKernelGGL(tile_chunks_kernel, dim3((unsigned)((ntiles + 255) / 256)), dim3(256), 0, s, B.tile_start,
                       ntiles, B.tile_counts);
    NFFT3_LAUNCH_CHECK("tile_chunks_kernel");
    int rc = exclusive_scan(s, B.tile_counts, B.chunk_start, B.scratch, ntiles);
    if (rc) return rc;
    // level-2 chunks: at most one partial chunk per tile beyond M / kSortChunk
    // (blocks past the last chunk return at once)
    const int64_t chunks2 = (M + kSortChunk - 1) / kSortChunk + ntiles;
    if (M > 0) {
        hipLaunchKernelGGL(z_count_kernel, dim3((unsigned)chunks2), dim3(kPtThreads), sizeof(int) * g.in0, s, p->tz,
                           B.tile_start, B.chunk_start, ntiles, g.in0, B.counts, p->chunk_base);
        NFFT3_LAUNCH_CHECK("z_count_kernel");
    }
    rc = exclusive_scan(s, B.counts, B.offsets, B.scratch, nb);
    if (rc) return rc;
    if (M > 0) {
        hipLaunchKernelGGL(z_scatter_kernel, dim3((unsigned)chunks2), dim3(kPtThreads), lds2, s, p->tx, p->tperm,
                           p->tz, M, B.tile_start, B.chunk_start, ntiles, g.in0, B.offsets, p->chunk_base, p->xs,
                           p->perm);
        NFFT3_LAUNCH_CHECK("z_scatter_kernel");
    }
    return NFFT3_OK;
}

// Entries of the two-level sort's run buffer for M points (level 1: the
// (tile, chunk) matrix and its scan; then level 2: the (chunk, z) bases), or
// -1 when the plan's tiling or M calls for the single-level sort.
int64_t two_level_bases(const nfft3_plan_impl *p, int64_t M) {
    const int64_t ntiles = (int64_t)p->bins.nty * p->bins.ntx;
    if (ntiles > kSortMaxTiles) return -1;
    const int64_t c1 = (M + kSortChunk - 1) / kSortChunk;
    // level-1 (tile, chunk) matrix and its scan total, then level-2 (chunk, z) bases
    const int64_t need = std::max(c1 * ntiles + 1, (c1 + ntiles) * p->n[0]);
    return need <= kSortMaxBases ? need : -1;
}

int launch_set_points(nfft3_plan_impl *p, int64_t M, const double *x, int *flag_out) {
    BinGeom g;
    g.n0 = (double)p->n[0]; g.n1 = (double)p->n[1]; g.n2 = (double)p->n[2];
    g.in0 = (int)p->n[0]; g.in1 = (int)p->n[1]; g.in2 = (int)p->n[2];
    g.By = p->bins.By; g.Bx = p->bins.Bx;
    g.nty = p->bins.nty; g.ntx = p->bins.ntx;
    const int ntiles = p->bins.nty * p->bins.ntx;
    hipStream_t s = p->stream;
    hipLaunchKernelGGL(fill_int_kernel, dim3(1), dim3(256), 0, s, p->flag, (int64_t)16, 0);
    NFFT3_LAUNCH_CHECK("fill_int_kernel");
    const bool two = two_level_bases(p, M) >= 0;
    int rc = two ? sort_two_level(p, M, x, g) : sort_single_level(p, M, x, g);
    if (rc) return rc;
    const int copies = two ? 1 : kBinCopies;
    // work items: counted, scanned and written on the device into a list
    // sized for the most items M points can make
    const int64_t cap = max_items(M, ntiles, g.in0, p->sub.maxpts);
    if (cap > p->sub.cap) {
        (void)hipFree(p->sub.items);
        p->sub.items = nullptr;
        p->sub.cap = 0;
        NFFT3_HIP_TRY(hipMalloc(&p->sub.items, sizeof(int4) * (size_t)cap));
        p->sub.cap = cap;
    }
    const int nseg = (int)((g.in0 + kItemZ - 1) / kItemZ);
    const int64_t nws = (int64_t)ntiles * nseg;
    const unsigned tb = (unsigned)nws;        // one wave per (tile, segment)
    hipLaunchKernelGGL((items_kernel<false>), dim3(tb), dim3(kItemThreads), 0, s, p->bins.offsets, copies, ntiles, g.in0, nseg,
                       p->sub.maxpts, p->bins.tile_items, (const int *)nullptr, (int4 *)nullptr, (int64_t)0, p->flag);
    NFFT3_LAUNCH_CHECK("items_kernel");
    rc = exclusive_scan(s, p->bins.tile_items, p->bins.tile_item_off, p->bins.scratch, nws);
    if (rc) return rc;
    hipLaunchKernelGGL((items_kernel<true>), dim3(tb), dim3(kItemThreads), 0, s, p->bins.offsets, copies, ntiles, g.in0, nseg,
                       p->sub.maxpts, (int *)nullptr, (const int *)p->bins.tile_item_off, p->sub.items, p->sub.cap,
                       p->flag);
    NFFT3_LAUNCH_CHECK("items_kernel");
    // the item count sizes the window-sum launches; the flag reports
    // non-finite points: one copy and one synchronisation for both
    hipLaunchKernelGGL(copy_int_kernel, dim3(1), dim3(1), 0, s, p->bins.tile_item_off + nws, p->flag + 2);
    NFFT3_LAUNCH_CHECK("copy_int_kernel");
    int words[3] = {0, 0, 0};
    NFFT3_HIP_TRY(hipMemcpyAsync(words, p->flag, sizeof(words), hipMemcpyDeviceToHost, s));
    NFFT3_HIP_TRY(hipStreamSynchronize(s));
    const int nitems = words[2], flag = words[0];
    if (flag & 4) return NFFT3_ERR_INVALID_ARG;    // item list too short (never expected)
    p->sub.count = nitems;
    *flag_out = flag;
    return NFFT3_OK;
}

}  // namespace nfft3
