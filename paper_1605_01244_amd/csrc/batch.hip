// Batched evaluation of many plans (own N, own points; same dtype, sigma, m)
// and of their derivative fields.
//
// complex<float>: each (plan, field) pair is a transform (the derivative
// fields through -2 pi i k_d fhat, one grid each); complex<double>: one
// transform per plan whose window sums also write the derivative fields
// (window derivative, as nfft3_trafo_fields).  A transform has four stages: the row pass
// (deconvolve + zero-pad + FFT along axis 2), the column passes along axes 1
// and 0, and the window sums.
//
// Two forms run the same stage bodies.  Per-length launches: each FFT stage
// runs as one launch per distinct transform length along its axis (a kernel
// specialised for that length, or one generic launch for lengths the
// compile-time engine does not cover), the window sums as one launch; each
// launch covers the work items (row blocks, column tiles, point items) of
// every transform in its group: workgroup b finds its transform by a binary
// search in the group's prefix table of item counts and runs item b -
// first[t] with that transform's arguments.  Kernel boundaries order the
// stages, so no workgroup ever waits on another.  The stage bodies and
// launch shapes are the ones of the single-plan kernels, so a batched result
// equals the sequential one bit for bit.  (A single kernel over all lengths
// holds every specialisation's code and ran several times slower.)
// Work queue: one launch of persistent workgroups over (transform, stage,
// tile) tickets (queue_impl.h); the same bodies (the column passes with 256
// threads and fewer columns per tile, which leaves each line's arithmetic
// unchanged), so its results equal the per-length form's bit for bit.
#include <algorithm>
#include <cstdlib>
#include <mutex>
#include <vector>

#include "batch_dev.h"

namespace nfft3 {

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

// group g of a stage: transforms ids[0 .. X), prefix table first[0 .. X]
template <typename T, int L>
__global__ void __launch_bounds__(kBRowThreads)
batch_rows_kernel(const BatchXform *__restrict__ xf, const int *__restrict__ ids, const int *__restrict__ first,
                  int X) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int g = batch_find(first, X, blockIdx.x);
    const RowArgs a = load_rows(&((cbx_t *)xf)[ids[g]].rows);
    if constexpr (L == 0) rows_body<T, 0, kBRowThreads>(a, blockIdx.x - first[g], smem_raw);
    else rows_body_s<T, 0, kBRowThreads, L, static_rows_nl<T>(L)>(a, blockIdx.x - first[g], smem_raw);
}

template <typename T, int AXIS, int L>
__global__ void __launch_bounds__(L == 0 ? kColsThreadsGeneric : kColsThreads)
batch_cols_kernel(const BatchXform *__restrict__ xf, const int *__restrict__ ids, const int *__restrict__ first,
                  int X) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int g = batch_find(first, X, blockIdx.x);
    cbx_t *b = (cbx_t *)xf + ids[g];
    const int tile = blockIdx.x - first[g];
    const ColArgs c = load_cols(AXIS == 1 ? &b->c1 : &b->c0);
    const int gx = AXIS == 1 ? b->gx1 : b->gx0;
    if constexpr (L == 0) cols_body<T, true, kColsThreadsGeneric, 16>(c, tile % gx, tile / gx, smem_raw);
    else cols_body_s<T, true, kColsThreads, L, static_cols_nl<T>(L)>(c, tile % gx, tile / gx, smem_raw);
}

template <typename T, int W, int PPT>
__global__ void __launch_bounds__(kPsThreads)
batch_interp_kernel(const BatchXform *__restrict__ xf, const int *__restrict__ ids, const int *__restrict__ first,
                    int X) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int g = batch_find(first, X, blockIdx.x);
    interp_body<T, W, PPT>(load_ps(&((cbx_t *)xf)[ids[g]].ip), blockIdx.x - first[g], smem_raw);
}

// complex<double> with derivative fields: the field and its derivative fields
// from the field's one grid (window derivative)
template <typename T, int W>
__global__ void __launch_bounds__(kPsThreads) __attribute__((amdgpu_waves_per_eu(2)))
batch_fields_kernel(const BatchXform *__restrict__ xf, const int *__restrict__ ids, const int *__restrict__ first,
                    int X) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int g = batch_find(first, X, blockIdx.x);
    interp_body_der<T, W, kModeFields>(load_ps(&((cbx_t *)xf)[ids[g]].ip), blockIdx.x - first[g], smem_raw);
}

// one launch of a stage over one group of transforms
struct BatchGroup {
    int stage;        // 0 rows, 1 cols axis 1, 2 cols axis 0, 3 window sums
    int len;          // static length, or 0 for the generic kernels
    std::vector<int> ids;
    size_t lds = 0;
    int total = 0;
    size_t off_ids = 0, off_first = 0;
};

template <typename T, int L>
static void launch_group_static(const BatchGroup &g, const BatchXform *dxf, const int *dids, const int *dfirst,
                                hipStream_t s) {
    const int X = (int)g.ids.size();
    if (g.stage == 0) {
        hipLaunchKernelGGL((batch_rows_kernel<T, L>), dim3((unsigned)g.total), dim3(kBRowThreads), g.lds, s, dxf,
                           dids, dfirst, X);
    } else if (g.stage == 1) {
        allow_lds((const void *)batch_cols_kernel<T, 1, L>, g.lds);
        hipLaunchKernelGGL((batch_cols_kernel<T, 1, L>), dim3((unsigned)g.total), dim3(L == 0 ? kColsThreadsGeneric : kColsThreads), g.lds, s,
                           dxf, dids, dfirst, X);
    } else {
        allow_lds((const void *)batch_cols_kernel<T, 0, L>, g.lds);
        hipLaunchKernelGGL((batch_cols_kernel<T, 0, L>), dim3((unsigned)g.total), dim3(L == 0 ? kColsThreadsGeneric : kColsThreads), g.lds, s,
                           dxf, dids, dfirst, X);
    }
}

template <typename T>
static void launch_group_fft(const BatchGroup &g, const BatchXform *dxf, const int *dids, const int *dfirst,
                             hipStream_t s) {
    switch (g.len) {
#define NFFT3_BATCH_LEN(L) \
        case L: launch_group_static<T, L>(g, dxf, dids, dfirst, s); return;
        NFFT3_STATIC_LENGTHS(NFFT3_BATCH_LEN)
#undef NFFT3_BATCH_LEN
        default: launch_group_static<T, 0>(g, dxf, dids, dfirst, s); return;
    }
}

// Launch descriptors.  The allocating call keeps one device buffer per GPU,
// grown as needed; the no-allocation call uses the file-scope array
// `scratch` below.  Each call holds its GPU's lock until its work has
// finished (the call synchronises before it returns), so calls on one GPU
// from several host threads run one after another and never share a buffer
// while it is in use.
constexpr int kMaxDevices = 64;
struct DescBuf {
    void *buf = nullptr;
    size_t cap = 0;
};
static std::mutex g_batch_mu[kMaxDevices];
static DescBuf g_desc[kMaxDevices];

// Descriptors of nfft3_batch_trafo_noalloc: a static device array, one copy
// per GPU, kept until the process ends.  Host code never passes `scratch`
// itself to a kernel or copy (on the host it only names the symbol): its
// device address on each GPU comes from hipGetSymbolAddress, taken once per
// device with that device current.
constexpr size_t kBatchScratchBytes = NFFT3_BATCH_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kBatchScratchBytes];
static void *g_scratch_ptr[kMaxDevices];

// the device address of `scratch` on GPU dev (caller holds g_batch_mu[dev] and
// has made dev the current device)
static int scratch_address(int dev, void **ptr) {
    if (!g_scratch_ptr[dev]) {
        void *a = nullptr;
        const hipError_t e = hipGetSymbolAddress(&a, HIP_SYMBOL(scratch));
        if (e != hipSuccess) {
            set_hip_error(e, "hipGetSymbolAddress(scratch)");
            return NFFT3_ERR_HIP;
        }
        g_scratch_ptr[dev] = a;
    }
    *ptr = g_scratch_ptr[dev];
    return NFFT3_OK;
}

// fills the queue's control words (a kernel, not a memset: safe under capture)
__global__ void __launch_bounds__(256) queue_reset_kernel(unsigned *ctl, int n) {
    for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) ctl[i] = 0;
}

// wall-clock ticks a queue wait may last: NFFT3_QUEUE_WAIT_US microseconds
// (default 2 s, at most one hour)
static int queue_wait_ticks(int dev, unsigned long long *ticks) {
    int khz = 0;
    NFFT3_HIP_TRY(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
    double us = 2e6;
    if (const char *e = std::getenv("NFFT3_QUEUE_WAIT_US")) us = std::min(std::max(0.0, std::atof(e)), 3.6e9);
    *ticks = (unsigned long long)(us * 1e-3 * (double)std::max(khz, 1));
    return NFFT3_OK;
}

// The work-queue form: segments of tickets stage-major (every transform's
// row pass, then every axis-1 pass, ...), each waiting for the previous
// stage of its own transform; one launch (after the control words are
// cleared).  Uses the allocating call's descriptor buffer; the caller holds
// the GPU's lock.
template <typename T, int W, int PPT>
static int queue_launch(const std::vector<BatchXform> &xf, size_t lds_ip, bool fields, hipStream_t stream,
                        int dev) {
    const int X = (int)xf.size();
    std::vector<QSeg> segs;
    int64_t total = 0;
    size_t lds = lds_ip;
    // tiles per ticket, per stage
    int cus = 0;
    NFFT3_HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    int64_t stage_tiles[kStages] = {0, 0, 0, 0};
    for (const BatchXform &b : xf)
        for (int s = 0; s < kStages; ++s) stage_tiles[s] += std::max(b.ntile[s], 0);
    int chunk[kStages];
    const int64_t per = (int64_t)kQTicketsPerCu * std::max(cus, 1);
    for (int s = 0; s < 3; ++s) chunk[s] = (int)std::min<int64_t>(kQChunkFftMax, std::max<int64_t>(1, stage_tiles[s] / per));
    chunk[3] = (sizeof(T) == 4 && stage_tiles[3] >= 8 * per) ? 2 : 1;
    auto chunk_of = [&](int s) { return chunk[s]; };
    auto tickets = [&](int ntile, int s) { return (ntile + chunk_of(s) - 1) / chunk_of(s); };
    for (int s = 0; s < kStages; ++s) {
        for (int x = 0; x < X; ++x) {
            const BatchXform &b = xf[x];
            if (s == 0) lds = std::max({lds, row_lds<T>(b.rows), col_lds<T>(b.c1), col_lds<T>(b.c0)});
            if (b.ntile[s] <= 0) continue;
            QSeg g;
            g.first = (int)total;
            g.x = x;
            g.stage = s;
            g.kind = s == 0 ? b.rows.n : s == 1 ? b.c1.n : s == 2 ? b.c0.n : 0;
            g.dep = -1;
            g.need = 0;
            g.ntile = b.ntile[s];
            g.chunk = chunk_of(s);
            for (int r = s - 1; r >= 0; --r) {
                if (b.ntile[r] > 0) {
                    g.dep = 4 * x + r;
                    g.need = tickets(b.ntile[r], r);
                    break;
                }
            }
            segs.push_back(g);
            total += tickets(b.ntile[s], s);
        }
    }
    if (total == 0) return NFFT3_OK;
    if (total > INT32_MAX) return NFFT3_ERR_INVALID_ARG;
    std::vector<int> tseg((size_t)total);
    for (size_t i = 0; i < segs.size(); ++i) {
        const int end = i + 1 < segs.size() ? segs[i + 1].first : (int)total;
        std::fill(tseg.begin() + segs[i].first, tseg.begin() + end, (int)i);
    }
    const size_t off_segs = ((sizeof(BatchXform) * X + 255) / 256) * 256;
    const size_t off_tseg = ((off_segs + sizeof(QSeg) * segs.size() + 255) / 256) * 256;
    const size_t off_ctl = ((off_tseg + sizeof(int) * tseg.size() + 255) / 256) * 256;
    const int nctl = kQDone + 4 * X;
    const size_t need = off_ctl + sizeof(unsigned) * nctl;
    DescBuf &d = g_desc[dev];
    if (need > d.cap) {
        // the previous call on this GPU synchronised before it released the lock
        (void)hipFree(d.buf);
        d.buf = nullptr;
        d.cap = 0;
        NFFT3_HIP_TRY(hipMalloc(&d.buf, need));
        d.cap = need;
    }
    char *base = (char *)d.buf;
    QueueLaunch q;
    q.args.xf = (const BatchXform *)base;
    q.args.segs = (const QSeg *)(base + off_segs);
    q.args.tseg = (const int *)(base + off_tseg);
    q.args.ctl = (unsigned *)(base + off_ctl);
    q.args.nseg = (int)segs.size();
    q.args.total = (int)total;
    int rc = queue_wait_ticks(dev, &q.args.wait_ticks);
    if (rc) return rc;
    q.lds = lds;
    q.W = W;
    q.ppt = PPT;
    q.fields = fields;
    NFFT3_HIP_TRY(hipMemcpyAsync(base, xf.data(), sizeof(BatchXform) * X, hipMemcpyHostToDevice, stream));
    NFFT3_HIP_TRY(hipMemcpyAsync(base + off_segs, segs.data(), sizeof(QSeg) * segs.size(), hipMemcpyHostToDevice,
                                 stream));
    NFFT3_HIP_TRY(hipMemcpyAsync(base + off_tseg, tseg.data(), sizeof(int) * tseg.size(), hipMemcpyHostToDevice,
                                 stream));
    hipLaunchKernelGGL(queue_reset_kernel, dim3((unsigned)std::min((nctl + 255) / 256, 1024)), dim3(256), 0,
                       stream, q.args.ctl, nctl);
    NFFT3_LAUNCH_CHECK("queue_reset_kernel");
    rc = sizeof(T) == 8 ? launch_queue_f64(q, stream) : launch_queue_f32(q, stream);
    unsigned aborted = 0;
    if (rc == NFFT3_OK)
        NFFT3_HIP_TRY(hipMemcpyAsync(&aborted, q.args.ctl + 1, sizeof(unsigned), hipMemcpyDeviceToHost, stream));
    // the host vectors above are copied from pageable memory; make sure the
    // copies are done before they go away
    NFFT3_HIP_TRY(hipStreamSynchronize(stream));
    if (rc) return rc;
    return aborted ? NFFT3_ERR_TIMEOUT : NFFT3_OK;
}

template <typename T, int W, int PPT>
static int batch_launch(int T_, nfft3_plan_impl *const *plans, const void *const *fhat, void *const *out, int mask,
                        int form) {
    const bool noalloc = form == kBatchNoAlloc, queue = form == kBatchQueue;
    const int dev = plans[0]->device;
    if (dev < 0 || dev >= kMaxDevices) return NFFT3_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lock(g_batch_mu[dev]);
    // allocations (allocating call) land on the plans' device
    int cur_dev = 0;
    NFFT3_HIP_TRY(hipGetDevice(&cur_dev));
    struct Restore {
        int dev;
        ~Restore() { (void)hipSetDevice(dev); }
    } restore{cur_dev};
    if (cur_dev != dev) NFFT3_HIP_TRY(hipSetDevice(dev));
    // complex<double>: derivative fields through the window derivative from
    // the field's grid (as nfft3_trafo_fields); complex<float>: one grid and
    // transform per field (spectral derivative)
    constexpr bool kDouble = sizeof(T) == 8;
    const bool der_fields = kDouble && mask != 0;
    std::vector<int> fields = {-1};
    for (int d = 0; d < 3; ++d)
        if (!der_fields && (mask & (1 << d))) fields.push_back(d);
    const int F = (int)fields.size();
    const int X = T_ * F;
    std::vector<BatchXform> xf((size_t)X);
    size_t lds_ip = 0;
    hipStream_t stream = plans[0]->stream;
    bool missing_grids = false;
    for (int t = 0; t < T_; ++t) {
        nfft3_plan_impl *p = plans[t];
        if (noalloc) {
            missing_grids = missing_grids || (int)p->extra_grids.size() < F - 1;
        } else {
            while ((int)p->extra_grids.size() < F - 1) {
                void *g = nullptr;
                NFFT3_HIP_TRY(hipMalloc(&g, (size_t)p->n[0] * p->n[1] * p->n[2] * p->elt));
                p->extra_grids.push_back(g);
            }
        }
        for (int f = 0; f < F; ++f) {
            BatchXform &b = xf[(size_t)t * F + f];
            // (a missing grid is reported below, before anything is launched)
            void *grid = (f == 0 || f - 1 >= (int)p->extra_grids.size()) ? p->grid : p->extra_grids[f - 1];
            b.rows = make_row_args<T>(p, fhat[t], grid, fields[f], kBRowThreads);
            b.c1 = make_col_args<T>(p, grid, 1, (int)p->N[1], (int)p->n[1], p->n[1] * p->n[2]);
            b.c0 = make_col_args<T>(p, grid, 0, (int)p->N[0], (int)p->n[0], p->n[2]);
            b.ip = interp_args(p);
            if (!interp_layout_ok(p, b.ip)) return NFFT3_ERR_INVALID_ARG;
            b.ip.grid = grid;
            b.ip.out = (char *)out[t] + (size_t)f * p->M * p->elt;
            if (der_fields) {
                b.ip.fmask = mask;
                b.ip.fstride = p->M;
            }
            b.gx1 = col_grid_x(b.c1);
            b.gx0 = col_grid_x(b.c0);
            b.ntile[0] = (int)row_blocks(p, b.rows);
            b.ntile[1] = b.gx1 * (int)p->N[0];
            b.ntile[2] = b.gx0 * (int)p->n[1];
            b.ntile[3] = (p->M > 0) ? (int)p->sub.count : 0;
            lds_ip = std::max(lds_ip, interp_lds(p, b.ip));
            if (queue) {
                // the queue's column tiles (256 threads); compile-time lengths only
                for (int ax = 0; ax < 3; ++ax)
                    if (!static_fft_len((int)p->n[ax])) return NFFT3_ERR_INVALID_ARG;
                if (b.rows.lpw != static_rows_nl<T>(b.rows.n)) return NFFT3_ERR_INVALID_ARG;
                b.c1.C = queue_cols_nl<T>(b.c1.n);
                b.c0.C = queue_cols_nl<T>(b.c0.n);
                if (b.c1.C > b.c1.ncols || b.c0.C > b.c0.ncols) return NFFT3_ERR_INVALID_ARG;
                b.gx1 = col_grid_x(b.c1);
                b.gx0 = col_grid_x(b.c0);
                b.ntile[1] = b.gx1 * (int)p->N[0];
                b.ntile[2] = b.gx0 * (int)p->n[1];
            }
        }
    }
    if (queue) return queue_launch<T, W, PPT>(xf, lds_ip, der_fields, stream, dev);
    // groups: per FFT stage one per distinct axis length (static lengths
    // only when the pass uses the compile-time engine's line counts), one for
    // the window sums
    std::vector<BatchGroup> groups;
    auto group_of = [&](int stage, int len) -> BatchGroup & {
        for (BatchGroup &g : groups)
            if (g.stage == stage && g.len == len) return g;
        groups.push_back(BatchGroup());
        groups.back().stage = stage;
        groups.back().len = len;
        return groups.back();
    };
    for (int t = 0; t < X; ++t) {
        const BatchXform &b = xf[t];
        if (b.ntile[0] > 0) {
            const int L = b.rows.n;
            const bool st = static_fft_len(L) && b.rows.lpw == static_rows_nl<T>(L);
            BatchGroup &g = group_of(0, st ? L : 0);
            g.ids.push_back(t);
            g.lds = std::max(g.lds, row_lds<T>(b.rows));
        }
        for (int ax = 1; ax <= 2; ++ax) {
            const ColArgs &c = ax == 1 ? b.c1 : b.c0;
            if (b.ntile[ax] <= 0) continue;
            const bool st = col_static<T>(c);
            BatchGroup &g = group_of(ax, st ? c.n : 0);
            g.ids.push_back(t);
            g.lds = std::max(g.lds, col_lds<T>(c));
        }
        if (b.ntile[3] > 0) {
            BatchGroup &g = group_of(3, 0);
            g.ids.push_back(t);
        }
    }
    // device layout: descriptors, then per group its ids and prefix table
    std::vector<int> ints;
    size_t off = ((sizeof(BatchXform) * X + 255) / 256) * 256;
    for (BatchGroup &g : groups) {
        g.off_ids = off + sizeof(int) * ints.size();
        for (int t : g.ids) ints.push_back(t);
        g.off_first = off + sizeof(int) * ints.size();
        int acc = 0;
        for (int t : g.ids) {
            ints.push_back(acc);
            acc += xf[t].ntile[g.stage];
        }
        ints.push_back(acc);
        g.total = acc;
        if (g.stage == 3) g.lds = lds_ip;
    }
    const size_t need = off + sizeof(int) * ints.size();
    char *base = nullptr;
    if (noalloc) {
        if (need > kBatchScratchBytes) return NFFT3_ERR_CAPACITY;
        if (missing_grids) return NFFT3_ERR_INVALID_ARG;
        void *sp = nullptr;
        const int rc = scratch_address(dev, &sp);
        if (rc) return rc;
        base = (char *)sp;
    } else {
        DescBuf &d = g_desc[dev];
        if (need > d.cap) {
            // the previous call on this GPU synchronised before it released the lock
            (void)hipFree(d.buf);
            d.buf = nullptr;
            d.cap = 0;
            NFFT3_HIP_TRY(hipMalloc(&d.buf, need));
            d.cap = need;
        }
        base = (char *)d.buf;
    }
    NFFT3_HIP_TRY(hipMemcpyAsync(base, xf.data(), sizeof(BatchXform) * X, hipMemcpyHostToDevice, stream));
    NFFT3_HIP_TRY(hipMemcpyAsync(base + off, ints.data(), sizeof(int) * ints.size(), hipMemcpyHostToDevice, stream));
    const BatchXform *dxf = (const BatchXform *)base;
    for (int stage = 0; stage < kStages; ++stage) {
        for (const BatchGroup &g : groups) {
            if (g.stage != stage || g.total == 0) continue;
            const int *dids = (const int *)(base + g.off_ids);
            const int *dfirst = (const int *)(base + g.off_first);
            if (stage < 3) {
                launch_group_fft<T>(g, dxf, dids, dfirst, stream);
                NFFT3_LAUNCH_CHECK("batch_fft_kernel");
            } else if (der_fields) {
                if constexpr (kDouble) {
                    allow_lds((const void *)batch_fields_kernel<T, W>, g.lds);
                    hipLaunchKernelGGL((batch_fields_kernel<T, W>), dim3((unsigned)g.total), dim3(kPsThreads),
                                       g.lds, stream, dxf, dids, dfirst, (int)g.ids.size());
                    NFFT3_LAUNCH_CHECK("batch_fields_kernel");
                }
            } else {
                allow_lds((const void *)batch_interp_kernel<T, W, PPT>, g.lds);
                hipLaunchKernelGGL((batch_interp_kernel<T, W, PPT>), dim3((unsigned)g.total), dim3(kPsThreads),
                                   g.lds, stream, dxf, dids, dfirst, (int)g.ids.size());
                NFFT3_LAUNCH_CHECK("batch_interp_kernel");
            }
        }
    }
    // the host descriptors above are copied from pageable memory; make sure
    // the copies are done before the vectors go away
    NFFT3_HIP_TRY(hipStreamSynchronize(stream));
    return NFFT3_OK;
}

template <typename T, int W>
static int batch_w(int T_, nfft3_plan_impl *const *plans, const void *const *fhat, void *const *out, int mask,
                   int form) {
    for (int t = 0; t < T_; ++t)
        if (plans[t]->sub.maxpts != plans[0]->sub.maxpts) return NFFT3_ERR_INVALID_ARG;
    if constexpr (W > 16) {
        return NFFT3_ERR_INVALID_ARG;
    } else {
        switch (plans[0]->sub.maxpts / kPsThreads) {
            case 1: return batch_launch<T, W, 1>(T_, plans, fhat, out, mask, form);
            case 2: return batch_launch<T, W, 2>(T_, plans, fhat, out, mask, form);
            default: return NFFT3_ERR_INVALID_ARG;
        }
    }
}

#define NFFT3_BATCH_M(T)                                          \
    switch (plans[0]->m) {                                        \
        case 1: return batch_w<T, 2>(T_, plans, fhat, out, mask, form);  \
        case 2: return batch_w<T, 4>(T_, plans, fhat, out, mask, form);  \
        case 3: return batch_w<T, 6>(T_, plans, fhat, out, mask, form);  \
        case 4: return batch_w<T, 8>(T_, plans, fhat, out, mask, form);  \
        case 5: return batch_w<T, 10>(T_, plans, fhat, out, mask, form); \
        case 6: return batch_w<T, 12>(T_, plans, fhat, out, mask, form); \
        case 7: return batch_w<T, 14>(T_, plans, fhat, out, mask, form); \
        case 8: return batch_w<T, 16>(T_, plans, fhat, out, mask, form); \
        default: return NFFT3_ERR_INVALID_ARG;                    \
    }

int launch_batch(int T_, nfft3_plan_impl *const *plans, const void *const *fhat, void *const *out, int mask,
                 int form) {
    if (plans[0]->dtype == NFFT3_C128) { NFFT3_BATCH_M(double) }
    NFFT3_BATCH_M(float)
}

}  // namespace nfft3
