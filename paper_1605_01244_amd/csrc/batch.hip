// Batched evaluation of many plans (own N, own points; same dtype, sigma, m)
// and of their derivative fields.
//
// Each (plan, field) pair is a transform with four stages: the row pass
// (deconvolve + zero-pad + FFT along axis 2), the column passes along axes 1
// and 0, and the window sums.  The batch runs as four launches, one per
// stage, each covering the work items (row blocks, column tiles, point items)
// of EVERY transform: workgroup b finds its transform t by a binary search in
// the per-stage prefix table of item counts and runs item b - first[t] with
// t's arguments.  Kernel boundaries order the stages, so no workgroup ever
// waits on another.  The stage bodies are the ones of the single-plan kernels
// (same launch shapes), so a batched result equals the sequential one bit for
// bit.
#include <algorithm>
#include <vector>

#include "fft_dev.h"
#include "interp_dev.h"

namespace nfft3 {

constexpr int kStages = 4;
constexpr int kBRowThreads = 256;
constexpr int kBColThreads = 512;

struct BatchXform {
    RowArgs rows;
    ColArgs c1, c0;
    PSArgs ip;
    int gx1, gx0;
    int ntile[kStages];
};

// transform of block b: last t with first[t] <= b (first has X + 1 entries)
__device__ __forceinline__ int batch_find(const int *__restrict__ first, int X, int b) {
    int lo = 0, hi = X - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (first[mid] <= b) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

template <typename T>
__global__ void __launch_bounds__(kBRowThreads)
batch_rows_kernel(const BatchXform *__restrict__ xf, const int *__restrict__ first, int X) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int t = batch_find(first, X, blockIdx.x);
    rows_any<T, 0, kBRowThreads>(xf[t].rows, blockIdx.x - first[t], smem_raw);
}

template <typename T, int AXIS>
__global__ void __launch_bounds__(kBColThreads)
batch_cols_kernel(const BatchXform *__restrict__ xf, const int *__restrict__ first, int X) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int t = batch_find(first, X, blockIdx.x);
    const int tile = blockIdx.x - first[t];
    if (AXIS == 1) {
        const int gx = xf[t].gx1;
        cols_any<T, true, kBColThreads, 16>(xf[t].c1, tile % gx, tile / gx, smem_raw);
    } else {
        const int gx = xf[t].gx0;
        cols_any<T, true, kBColThreads, 16>(xf[t].c0, tile % gx, tile / gx, smem_raw);
    }
}

template <typename T, int W, int PPT>
__global__ void __launch_bounds__(kPsThreads)
batch_interp_kernel(const BatchXform *__restrict__ xf, const int *__restrict__ first, int X) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int t = batch_find(first, X, blockIdx.x);
    interp_body<T, W, PPT>(xf[t].ip, blockIdx.x - first[t], smem_raw);
}

// device-side descriptors of the batched launcher (grown as needed, kept)
static void *g_batch_buf = nullptr;
static size_t g_batch_cap = 0;

template <typename T, int W, int PPT>
static int batch_launch(int T_, nfft3_plan_impl *const *plans, const void *const *fhat, void *const *out, int mask) {
    std::vector<int> fields = {-1};
    for (int d = 0; d < 3; ++d)
        if (mask & (1 << d)) fields.push_back(d);
    const int F = (int)fields.size();
    const int X = T_ * F;
    std::vector<BatchXform> xf((size_t)X);
    size_t lds[kStages] = {0, 0, 0, 0};
    hipStream_t stream = plans[0]->stream;
    for (int t = 0; t < T_; ++t) {
        nfft3_plan_impl *p = plans[t];
        while ((int)p->extra_grids.size() < F - 1) {
            void *g = nullptr;
            NFFT3_HIP_TRY(hipMalloc(&g, (size_t)p->n[0] * p->n[1] * p->n[2] * p->elt));
            p->extra_grids.push_back(g);
        }
        for (int f = 0; f < F; ++f) {
            BatchXform &b = xf[(size_t)t * F + f];
            void *grid = f == 0 ? p->grid : p->extra_grids[f - 1];
            b.rows = make_row_args<T>(p, fhat[t], grid, fields[f], kBRowThreads);
            b.c1 = make_col_args<T>(p, grid, 1, (int)p->N[1], (int)p->n[1], p->n[1] * p->n[2], kBColThreads, 16);
            b.c0 = make_col_args<T>(p, grid, 0, (int)p->N[0], (int)p->n[0], p->n[2], kBColThreads, 16);
            b.ip = interp_args(p);
            if (!interp_layout_ok(p, b.ip)) return NFFT3_ERR_INVALID_ARG;
            b.ip.grid = grid;
            b.ip.out = (char *)out[t] + (size_t)f * p->M * p->elt;
            b.gx1 = col_grid_x(b.c1);
            b.gx0 = col_grid_x(b.c0);
            b.ntile[0] = (int)row_blocks(p, b.rows);
            b.ntile[1] = b.gx1 * (int)p->N[0];
            b.ntile[2] = b.gx0 * (int)p->n[1];
            b.ntile[3] = (p->M > 0) ? (int)p->sub.count : 0;
            lds[0] = std::max(lds[0], row_lds<T>(b.rows));
            lds[1] = std::max(lds[1], col_lds<T>(b.c1));
            lds[2] = std::max(lds[2], col_lds<T>(b.c0));
            lds[3] = std::max(lds[3], interp_lds(p, b.ip));
        }
    }
    // per-stage prefix tables of item counts: first[s][t], X + 1 entries each
    std::vector<int> first((size_t)kStages * (X + 1));
    int total[kStages];
    for (int s = 0; s < kStages; ++s) {
        int acc = 0;
        for (int t = 0; t < X; ++t) {
            first[(size_t)s * (X + 1) + t] = acc;
            acc += xf[t].ntile[s];
        }
        first[(size_t)s * (X + 1) + X] = acc;
        total[s] = acc;
    }
    const size_t off_first = ((sizeof(BatchXform) * X + 255) / 256) * 256;
    const size_t need = off_first + sizeof(int) * first.size();
    if (need > g_batch_cap) {
        if (g_batch_buf) {
            NFFT3_HIP_TRY(hipStreamSynchronize(stream));
            hipFree(g_batch_buf);
        }
        g_batch_buf = nullptr;
        g_batch_cap = 0;
        NFFT3_HIP_TRY(hipMalloc(&g_batch_buf, need));
        g_batch_cap = need;
    }
    char *base = (char *)g_batch_buf;
    NFFT3_HIP_TRY(hipMemcpyAsync(base, xf.data(), sizeof(BatchXform) * X, hipMemcpyHostToDevice, stream));
    NFFT3_HIP_TRY(hipMemcpyAsync(base + off_first, first.data(), sizeof(int) * first.size(),
                                 hipMemcpyHostToDevice, stream));
    const BatchXform *dxf = (const BatchXform *)base;
    const int *dfirst = (const int *)(base + off_first);
    if (total[0] > 0) {
        hipLaunchKernelGGL(batch_rows_kernel<T>, dim3((unsigned)total[0]), dim3(kBRowThreads), lds[0], stream, dxf,
                           dfirst, X);
        NFFT3_LAUNCH_CHECK("batch_rows_kernel");
    }
    if (total[1] > 0) {
        allow_lds((const void *)batch_cols_kernel<T, 1>, lds[1]);
        hipLaunchKernelGGL((batch_cols_kernel<T, 1>), dim3((unsigned)total[1]), dim3(kBColThreads), lds[1], stream,
                           dxf, dfirst + (X + 1), X);
        NFFT3_LAUNCH_CHECK("batch_cols_kernel");
    }
    if (total[2] > 0) {
        allow_lds((const void *)batch_cols_kernel<T, 0>, lds[2]);
        hipLaunchKernelGGL((batch_cols_kernel<T, 0>), dim3((unsigned)total[2]), dim3(kBColThreads), lds[2], stream,
                           dxf, dfirst + 2 * (X + 1), X);
        NFFT3_LAUNCH_CHECK("batch_cols_kernel");
    }
    if (total[3] > 0) {
        allow_lds((const void *)batch_interp_kernel<T, W, PPT>, lds[3]);
        hipLaunchKernelGGL((batch_interp_kernel<T, W, PPT>), dim3((unsigned)total[3]), dim3(kPsThreads), lds[3],
                           stream, dxf, dfirst + 3 * (X + 1), X);
        NFFT3_LAUNCH_CHECK("batch_interp_kernel");
    }
    // the host descriptors above are copied from pageable memory; make sure
    // the copies are done before the vectors go away
    NFFT3_HIP_TRY(hipStreamSynchronize(stream));
    return NFFT3_OK;
}

template <typename T, int W>
static int batch_w(int T_, nfft3_plan_impl *const *plans, const void *const *fhat, void *const *out, int mask) {
    for (int t = 0; t < T_; ++t)
        if (plans[t]->sub.maxpts != plans[0]->sub.maxpts) return NFFT3_ERR_INVALID_ARG;
    if constexpr (W > 16) {
        return NFFT3_ERR_INVALID_ARG;
    } else {
        switch (plans[0]->sub.maxpts / kPsThreads) {
            case 1: return batch_launch<T, W, 1>(T_, plans, fhat, out, mask);
            case 2: return batch_launch<T, W, 2>(T_, plans, fhat, out, mask);
            default: return NFFT3_ERR_INVALID_ARG;
        }
    }
}

#define NFFT3_BATCH_M(T)                                          \
    switch (plans[0]->m) {                                        \
        case 1: return batch_w<T, 2>(T_, plans, fhat, out, mask);  \
        case 2: return batch_w<T, 4>(T_, plans, fhat, out, mask);  \
        case 3: return batch_w<T, 6>(T_, plans, fhat, out, mask);  \
        case 4: return batch_w<T, 8>(T_, plans, fhat, out, mask);  \
        case 5: return batch_w<T, 10>(T_, plans, fhat, out, mask); \
        case 6: return batch_w<T, 12>(T_, plans, fhat, out, mask); \
        case 7: return batch_w<T, 14>(T_, plans, fhat, out, mask); \
        case 8: return batch_w<T, 16>(T_, plans, fhat, out, mask); \
        default: return NFFT3_ERR_INVALID_ARG;                    \
    }

int launch_batch(int T_, nfft3_plan_impl *const *plans, const void *const *fhat, void *const *out, int mask) {
    if (plans[0]->dtype == NFFT3_C128) { NFFT3_BATCH_M(double) }
    NFFT3_BATCH_M(float)
}

}  // namespace nfft3
