// Point preprocessing (the precomputation step of the windowed method):
// fold every point into [-1/2, 1/2) with the Euclidean remainder of
// Sec. 2.2.1, locate its grid cell u_d = floor(n_d x_d) in FP64, and sort the
// points by grid tile with a counting sort (histogram -> exclusive scan ->
// scatter).  The sorted copy keeps the folded FP64 coordinates and the
// permutation back to the caller's order, so a workgroup of the window-sum
// kernels touches one compact region of the grid.
#include "internal.h"

namespace nfft3 {

constexpr int kPtThreads = 256;
constexpr int kScanThreads = 1024;

__device__ __forceinline__ double fold_unit(double v) {
    double r = v - rint(v);          // exact; in [-1/2, 1/2]
    return r >= 0.5 ? r - 1.0 : r;   // +1/2 belongs to the next period
}

struct BinGeom {
    double n0, n1, n2;
    int in0, in1, in2;
    int B0, B1, B2;
    int nb0, nb1, nb2;
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
    return ((c0 / g.B0) * g.nb1 + c1 / g.B1) * g.nb2 + c2 / g.B2;
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
    bin_of[j] = b;
    rank[j] = atomicAdd(&counts[b], 1);
}

// Exclusive scan of nb counts by one workgroup (nb is at most a few 1e5).
__global__ void __launch_bounds__(kScanThreads)
scan_kernel(const int *__restrict__ counts, int *__restrict__ offsets, int64_t nb) {
    __shared__ int part[kScanThreads];
    const int tid = threadIdx.x;
    const int64_t per = (nb + kScanThreads - 1) / kScanThreads;
    const int64_t lo = min<int64_t>(nb, tid * per), hi = min<int64_t>(nb, lo + per);
    int s = 0;
    for (int64_t i = lo; i < hi; ++i) s += counts[i];
    part[tid] = s;
    __syncthreads();
    for (int off = 1; off < kScanThreads; off <<= 1) {
        int v = tid >= off ? part[tid - off] : 0;
        __syncthreads();
        part[tid] += v;
        __syncthreads();
    }
    int run = part[tid] - s;   // exclusive prefix of this chunk
    for (int64_t i = lo; i < hi; ++i) {
        offsets[i] = run;
        run += counts[i];
    }
    if (tid == kScanThreads - 1) offsets[nb] = part[tid];
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

int launch_set_points(nfft3_plan_impl *p, int64_t M, const double *x) {
    BinGeom g;
    g.n0 = (double)p->n[0]; g.n1 = (double)p->n[1]; g.n2 = (double)p->n[2];
    g.in0 = (int)p->n[0]; g.in1 = (int)p->n[1]; g.in2 = (int)p->n[2];
    g.B0 = p->bins.B[0]; g.B1 = p->bins.B[1]; g.B2 = p->bins.B[2];
    g.nb0 = p->bins.nb[0]; g.nb1 = p->bins.nb[1]; g.nb2 = p->bins.nb[2];
    const int64_t nb = p->bins.nbins;
    hipLaunchKernelGGL(fill_int_kernel, dim3((unsigned)((nb + 255) / 256)), dim3(256), 0, p->stream,
                       p->bins.counts, nb, 0);
    NFFT3_LAUNCH_CHECK("fill_int_kernel");
    hipLaunchKernelGGL(fill_int_kernel, dim3(1), dim3(256), 0, p->stream, p->flag, (int64_t)16, 0);
    NFFT3_LAUNCH_CHECK("fill_int_kernel");
    const unsigned blocks = (unsigned)((M + kPtThreads - 1) / kPtThreads);
    if (M > 0) {
        hipLaunchKernelGGL(bin_count_kernel, dim3(blocks), dim3(kPtThreads), 0, p->stream, x, M, g,
                           p->bins.counts, p->bin_of, p->rank, p->flag);
        NFFT3_LAUNCH_CHECK("bin_count_kernel");
    }
    hipLaunchKernelGGL(scan_kernel, dim3(1), dim3(kScanThreads), 0, p->stream, p->bins.counts,
                       p->bins.offsets, nb);
    NFFT3_LAUNCH_CHECK("scan_kernel");
    if (M > 0) {
        hipLaunchKernelGGL(scatter_kernel, dim3(blocks), dim3(kPtThreads), 0, p->stream, x, M,
                           p->bins.offsets, p->bin_of, p->rank, p->xs, p->perm);
        NFFT3_LAUNCH_CHECK("scatter_kernel");
    }
    return NFFT3_OK;
}

}  // namespace nfft3
