// Point preprocessing (the precomputation step of the windowed method):
// fold every point into [-1/2, 1/2) with the Euclidean remainder of
// Sec. 2.2.1, locate its grid cell u_d = floor(n_d x_d) in FP64, and sort the
// points with a counting sort (histogram -> exclusive scan -> scatter) by the
// key (tile, z-cell), where a tile is a By x Bx block of cells in the (y, x)
// plane and z (axis 0) varies fastest.  Each tile column is then cut into
// work items of at most maxpts points spanning at most kItemZ z-cells; a
// workgroup of the window-sum kernels takes one item and streams the z-planes
// of its tile (plus the stencil halo) through LDS.
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

// ---- two-level counting sort (tile, then z within the tile) ---------------
// One global atomic per point (the single-level sort above) runs at the
// device's atomic rate, and its scatter writes 24 bytes at a random place
// per point.  The two-level sort counts in LDS instead: a workgroup takes a
// chunk of kSortChunk points, ranks them within the chunk with LDS atomics
// per key, then reserves each key's run with one global atomic per (chunk,
// key) present; a point's rank in its key is the run's base plus its local
// rank.  Level 1 keys by tile and scatters the folded points into tile order;
// level 2 walks each tile's points in chunks that never cross a tile, keys
// them by z-cell and scatters them into (tile, z) order.  Every run of a
// chunk and key is contiguous, so the scatters write in runs.  The order
// within a (tile, z) bin depends on the atomics (as before).
constexpr int kSortChunk = 4096;                 // points per workgroup
constexpr int kSortPer = kSortChunk / kPtThreads;
constexpr int kSortMaxTiles = 8192;              // LDS: two ints per tile

// level 1: local ranks by tile, a global base per (chunk, tile) present
__global__ void __launch_bounds__(kPtThreads)
tile_rank_kernel(const double *__restrict__ x, int64_t M, BinGeom g, int ntiles, int *__restrict__ tile_counts,
                 int *__restrict__ trank, int *__restrict__ flag) {
    extern __shared__ int sh[];                  // [0, ntiles): counts, then bases
    int *cnt = sh, *base = sh + ntiles;
    for (int t = threadIdx.x; t < ntiles; t += kPtThreads) cnt[t] = 0;
    __syncthreads();
    const int64_t c0 = (int64_t)blockIdx.x * kSortChunk;
    int key[kSortPer], lr[kSortPer];
#pragma unroll
    for (int i = 0; i < kSortPer; ++i) {
        const int64_t j = c0 + i * kPtThreads + threadIdx.x;
        key[i] = -1;
        if (j < M) {
            const double *xp = x + 3 * j;
            int t = 0;
            if (isfinite(xp[0]) && isfinite(xp[1]) && isfinite(xp[2])) {
                const int c1 = cell_of(fold_unit(xp[1]), g.n1, g.in1);
                const int c2 = cell_of(fold_unit(xp[2]), g.n2, g.in2);
                t = (c1 / g.By) * g.ntx + c2 / g.Bx;
            } else {
                atomicOr(flag, 1);
            }
            key[i] = t;
            lr[i] = atomicAdd(&cnt[t], 1);
        }
    }
    __syncthreads();
    for (int t = threadIdx.x; t < ntiles; t += kPtThreads)
        if (cnt[t]) base[t] = atomicAdd(&tile_counts[t], cnt[t]);
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kSortPer; ++i) {
        const int64_t j = c0 + i * kPtThreads + threadIdx.x;
        if (key[i] >= 0) trank[j] = base[key[i]] + lr[i];
    }
}

// level 1 scatter: folded coordinates, caller index and z-cell in tile order
__global__ void __launch_bounds__(kPtThreads)
tile_scatter_kernel(const double *__restrict__ x, int64_t M, BinGeom g, const int *__restrict__ tile_start,
                    const int *__restrict__ trank, double *__restrict__ tx, int *__restrict__ tperm,
                    int *__restrict__ tz) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= M) return;
    const double *xp = x + 3 * j;
    double f0 = 0.0, f1 = 0.0, f2 = 0.0;
    // a non-finite point (reported through the flag; the sort's result is
    // then discarded) goes to tile 0 at the origin, as tile_rank_kernel put it
    if (isfinite(xp[0]) && isfinite(xp[1]) && isfinite(xp[2])) {
        f0 = fold_unit(xp[0]);
        f1 = fold_unit(xp[1]);
        f2 = fold_unit(xp[2]);
    }
    const int c1 = cell_of(f1, g.n1, g.in1), c2 = cell_of(f2, g.n2, g.in2);
    const int t = (c1 / g.By) * g.ntx + c2 / g.Bx;
    const int64_t pos = (int64_t)tile_start[t] + trank[j];
    tx[3 * pos + 0] = f0;
    tx[3 * pos + 1] = f1;
    tx[3 * pos + 2] = f2;
    tperm[pos] = (int)j;
    tz[pos] = cell_of(f0, g.n0, g.in0);
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

// level 2: local ranks by z-cell within a tile's chunk, a global base per
// (chunk, bin) present
__global__ void __launch_bounds__(kPtThreads)
z_rank_kernel(const int *__restrict__ tz, const int *__restrict__ tile_start, const int *__restrict__ chunk_start,
              int ntiles, int n0, int *__restrict__ bin_counts, int *__restrict__ zrank) {
    extern __shared__ int sh[];                  // [0, n0): counts, then bases
    int *cnt = sh, *base = sh + n0;
    int t, lo, hi;
    if (!level2_chunk(chunk_start, tile_start, ntiles, blockIdx.x, t, lo, hi)) return;
    for (int z = threadIdx.x; z < n0; z += kPtThreads) cnt[z] = 0;
    __syncthreads();
    int key[kSortPer], lr[kSortPer];
#pragma unroll
    for (int i = 0; i < kSortPer; ++i) {
        const int64_t p = (int64_t)lo + i * kPtThreads + threadIdx.x;
        key[i] = -1;
        if (p < hi) {
            key[i] = tz[p];
            lr[i] = atomicAdd(&cnt[key[i]], 1);
        }
    }
    __syncthreads();
    int *bc = bin_counts + (int64_t)t * n0;
    for (int z = threadIdx.x; z < n0; z += kPtThreads)
        if (cnt[z]) base[z] = atomicAdd(&bc[z], cnt[z]);
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kSortPer; ++i) {
        const int64_t p = (int64_t)lo + i * kPtThreads + threadIdx.x;
        if (key[i] >= 0) zrank[p] = base[key[i]] + lr[i];
    }
}

// level 2 scatter into (tile, z) order
__global__ void __launch_bounds__(kPtThreads)
z_scatter_kernel(const double *__restrict__ tx, const int *__restrict__ tperm, const int *__restrict__ tz,
                 const int *__restrict__ zrank, int64_t M, BinGeom g, const int *__restrict__ bin_start,
                 double *__restrict__ xs, int *__restrict__ perm) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= M) return;
    const double f0 = tx[3 * p + 0], f1 = tx[3 * p + 1], f2 = tx[3 * p + 2];
    const int c1 = cell_of(f1, g.n1, g.in1), c2 = cell_of(f2, g.n2, g.in2);
    const int t = (c1 / g.By) * g.ntx + c2 / g.Bx;
    const int64_t pos = (int64_t)bin_start[(int64_t)t * g.in0 + tz[p]] + zrank[p];
    xs[3 * pos + 0] = f0;
    xs[3 * pos + 1] = f1;
    xs[3 * pos + 2] = f2;
    perm[pos] = tperm[p];
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

// ---- work items: walk each tile column's z-cells (one wave per tile) ------
// A new item starts when adding the next cell would exceed maxpts points or
// the item would span more than kItemZ z-cells; a cell holding more than
// maxpts points becomes ceil(count/maxpts) items of its own.  WRITE=false
// counts the items of each tile, WRITE=true emits (tile, p_lo, p_hi, 0).
// The wave stages the tile's n0 + 1 bin starts in LDS with coalesced loads
// (when they fit), then one lane walks them: the walk is sequential, so
// reading its inputs from HBM one dependent load at a time dominated.
constexpr int kItemWaves = 4;            // tiles per workgroup

template <bool WRITE>
__global__ void __launch_bounds__(64 * kItemWaves)
items_kernel(const int *__restrict__ offsets, int copies, int ntiles, int n0, int maxpts,
             int *__restrict__ item_count, const int *__restrict__ item_offset, int4 *__restrict__ items,
             int use_lds) {
    extern __shared__ int sofs[];        // kItemWaves x (n0 + 1) bin starts
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int tile = blockIdx.x * kItemWaves + wave;
    const bool valid = tile < ntiles;
    // bin (tile, z) spans offsets[(tile n0 + z) K] .. offsets[(tile n0 + z + 1) K],
    // K = copies counters per bin
    const int *g = offsets + (int64_t)(valid ? tile : 0) * n0 * copies;
    const int *ofs = g;
    int stride = copies;
    if (use_lds) {
        int *sw = sofs + wave * (n0 + 1);
        if (valid)
            for (int z = lane; z <= n0; z += 64) sw[z] = g[(int64_t)z * copies];
        __syncthreads();
        ofs = sw;
        stride = 1;
    }
    if (!valid || lane != 0) return;
    int k = 0;
    int64_t w = WRITE ? item_offset[tile] : 0;
    int cur = 0, z_start = 0, p_start = 0;
    int onext = ofs[0];
    for (int z = 0; z < n0; ++z) {
        const int oz = onext;
        onext = ofs[(z + 1) * stride];
        const int c = onext - oz;
        if (c == 0) continue;
        if (cur > 0 && (cur + c > maxpts || z - z_start >= kItemZ)) {
            if (WRITE) items[w + k] = make_int4(tile, p_start, p_start + cur, 0);
            ++k;
            cur = 0;
        }
        if (c > maxpts) {     // a dense cell on its own
            for (int s = 0; s < c; s += maxpts) {
                if (WRITE) items[w + k] = make_int4(tile, oz + s, oz + min(c, s + maxpts), 0);
                ++k;
            }
            continue;
        }
        if (cur == 0) { z_start = z; p_start = oz; }
        cur += c;
    }
    if (cur > 0) {
        if (WRITE) items[w + k] = make_int4(tile, p_start, p_start + cur, 0);
        ++k;
    }
    if (!WRITE) item_count[tile] = k;
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

// Two-level sort (see tile_rank_kernel); bins.offsets receives the nbins + 1
// bin starts.
static int sort_two_level(nfft3_plan_impl *p, int64_t M, const double *x, const BinGeom &g) {
    const int ntiles = g.nty * g.ntx;
    const int64_t nb = p->bins.nbins;
    hipStream_t s = p->stream;
    Bins &B = p->bins;
    hipLaunchKernelGGL(fill_int_kernel, dim3((unsigned)((ntiles + 255) / 256)), dim3(256), 0, s, B.tile_counts,
                       (int64_t)ntiles, 0);
    NFFT3_LAUNCH_CHECK("fill_int_kernel");
    hipLaunchKernelGGL(fill_int_kernel, dim3((unsigned)((nb + 255) / 256)), dim3(256), 0, s, B.counts, nb, 0);
    NFFT3_LAUNCH_CHECK("fill_int_kernel");
    const unsigned chunks1 = (unsigned)((M + kSortChunk - 1) / kSortChunk);
    allow_lds((const void *)tile_rank_kernel, sizeof(int) * 2 * ntiles);
    if (M > 0) {
        hipLaunchKernelGGL(tile_rank_kernel, dim3(chunks1), dim3(kPtThreads), sizeof(int) * 2 * ntiles, s, x, M, g,
                           ntiles, B.tile_counts, p->bin_of, p->flag);
        NFFT3_LAUNCH_CHECK("tile_rank_kernel");
    }
    int rc = exclusive_scan(s, B.tile_counts, B.tile_start, B.scratch, ntiles);
    if (rc) return rc;
    const unsigned blocks = (unsigned)((M + kPtThreads - 1) / kPtThreads);
    if (M > 0) {
        hipLaunchKernelGGL(tile_scatter_kernel, dim3(blocks), dim3(kPtThreads), 0, s, x, M, g, B.tile_start,
                           p->bin_of, p->tx, p->tperm, p->tz);
        NFFT3_LAUNCH_CHECK("tile_scatter_kernel");
    }
    hipLaunchKernelGGL(tile_chunks_kernel, dim3((unsigned)((ntiles + 255) / 256)), dim3(256), 0, s, B.tile_start,
                       ntiles, B.tile_counts);
    NFFT3_LAUNCH_CHECK("tile_chunks_kernel");
    rc = exclusive_scan(s, B.tile_counts, B.chunk_start, B.scratch, ntiles);
    if (rc) return rc;
    // level-2 chunks: at most one partial chunk per tile beyond M / kSortChunk
    const int64_t chunks2 = (M + kSortChunk - 1) / kSortChunk + ntiles;
    if (M > 0) {
        hipLaunchKernelGGL(z_rank_kernel, dim3((unsigned)chunks2), dim3(kPtThreads), sizeof(int) * 2 * g.in0, s, p->tz,
                           B.tile_start, B.chunk_start, ntiles, g.in0, B.counts, p->rank);
        NFFT3_LAUNCH_CHECK("z_rank_kernel");
    }
    rc = exclusive_scan(s, B.counts, B.offsets, B.scratch, nb);
    if (rc) return rc;
    if (M > 0) {
        hipLaunchKernelGGL(z_scatter_kernel, dim3(blocks), dim3(kPtThreads), 0, s, p->tx, p->tperm, p->tz, p->rank, M,
                           g, B.offsets, p->xs, p->perm);
        NFFT3_LAUNCH_CHECK("z_scatter_kernel");
    }
    return NFFT3_OK;
}

bool two_level_sort(const nfft3_plan_impl *p) {
    return (int64_t)p->bins.nty * p->bins.ntx <= kSortMaxTiles;
}

int launch_set_points(nfft3_plan_impl *p, int64_t M, const double *x) {
    BinGeom g;
    g.n0 = (double)p->n[0]; g.n1 = (double)p->n[1]; g.n2 = (double)p->n[2];
    g.in0 = (int)p->n[0]; g.in1 = (int)p->n[1]; g.in2 = (int)p->n[2];
    g.By = p->bins.By; g.Bx = p->bins.Bx;
    g.nty = p->bins.nty; g.ntx = p->bins.ntx;
    const int ntiles = p->bins.nty * p->bins.ntx;
    hipStream_t s = p->stream;
    hipLaunchKernelGGL(fill_int_kernel, dim3(1), dim3(256), 0, s, p->flag, (int64_t)16, 0);
    NFFT3_LAUNCH_CHECK("fill_int_kernel");
    const bool two = two_level_sort(p);
    int rc = two ? sort_two_level(p, M, x, g) : sort_single_level(p, M, x, g);
    if (rc) return rc;
    const int copies = two ? 1 : kBinCopies;
    // work items
    const unsigned tb = (unsigned)((ntiles + kItemWaves - 1) / kItemWaves);
    const size_t ilds = sizeof(int) * kItemWaves * ((size_t)g.in0 + 1);
    const int use_lds = ilds <= 64 * 1024 ? 1 : 0;
    hipLaunchKernelGGL((items_kernel<false>), dim3(tb), dim3(64 * kItemWaves), use_lds ? ilds : 0, s, p->bins.offsets,
                       copies, ntiles, g.in0, p->sub.maxpts, p->bins.tile_items, (const int *)nullptr,
                       (int4 *)nullptr, use_lds);
    NFFT3_LAUNCH_CHECK("items_kernel");
    rc = exclusive_scan(s, p->bins.tile_items, p->bins.tile_item_off, p->bins.scratch, ntiles);
    if (rc) return rc;
    // the item count is needed on the host to size the item list and the launches
    int nitems = 0;
    NFFT3_HIP_TRY(hipMemcpyAsync(&nitems, p->bins.tile_item_off + ntiles, sizeof(int), hipMemcpyDeviceToHost, s));
    NFFT3_HIP_TRY(hipStreamSynchronize(s));
    if (nitems > p->sub.cap) {
        (void)hipFree(p->sub.items);
        p->sub.items = nullptr;
        p->sub.cap = 0;
        NFFT3_HIP_TRY(hipMalloc(&p->sub.items, sizeof(int4) * (size_t)std::max(nitems, 1)));
        p->sub.cap = nitems;
    }
    p->sub.count = nitems;
    if (nitems > 0) {
        hipLaunchKernelGGL((items_kernel<true>), dim3(tb), dim3(64 * kItemWaves), use_lds ? ilds : 0, s,
                           p->bins.offsets, copies, ntiles, g.in0, p->sub.maxpts, (int *)nullptr,
                           (const int *)p->bins.tile_item_off, p->sub.items, use_lds);
        NFFT3_LAUNCH_CHECK("items_kernel");
    }
    return NFFT3_OK;
}

}  // namespace nfft3
