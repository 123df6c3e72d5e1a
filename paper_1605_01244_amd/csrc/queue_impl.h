// The batched evaluation as one launch: persistent workgroups take tickets
// over (transform, stage, tile) from a device counter (layout in
// batch_dev.h).
//
// Progress.  Tickets are taken in increasing order and a task waits only for
// tasks of lower tickets (the previous stage of its own transform), each
// held by a workgroup that is already running; so the lowest unfinished
// ticket never waits, and the queue drains whatever the number of resident
// workgroups.
//
// Visibility.  After an FFT task every wave waits for its stores to complete
// (they are then in its XCD's L2); after the workgroup barrier wave 0 adds 1
// to the stage's done counter with a device-scope release (which writes the
// XCD's L2 back).  A task whose previous stage this workgroup has not yet
// seen finished reads the counter with device-scope acquire loads (which
// invalidate the CU's L1 and the XCD's L2 copies) before the workgroup's
// barrier.  The window sums publish nothing: no task depends on them.
//
// Every wait is bounded: a wait longer than wait_ticks of the wall clock (or
// one that sees the abort flag) sets the abort flag and ends its workgroup;
// the others stop taking tickets, and the host reports the abort.
//
// The FFT stage bodies are the compile-time engine's (the host admits only
// plans whose three lengths it covers), called (not inlined) so that one
// kernel holds every length without growing with the window-sum
// instantiations; each callee reloads its arguments as uniform values.  The
// window sums are inlined.
#pragma once
#include "batch_dev.h"

namespace nfft3 {

template <typename T, int L>
__device__ __attribute__((noinline)) void q_rows(const BatchXform *xf_, int x_, int blk_) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cbx_t *xf = uniform_xf(xf_);
    const int x = __builtin_amdgcn_readfirstlane(x_), blk = __builtin_amdgcn_readfirstlane(blk_);
    const RowArgs a = load_rows(&xf[x].rows);
    rows_body_s<T, 0, kQThreads, L, static_rows_nl<T>(L)>(a, blk, smem_raw);
}

template <typename T, int L>
__device__ __attribute__((noinline)) void q_cols(const BatchXform *xf_, int x_, int axis_, int tile_) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cbx_t *xf = uniform_xf(xf_);
    const int x = __builtin_amdgcn_readfirstlane(x_), tile = __builtin_amdgcn_readfirstlane(tile_);
    const bool a1 = __builtin_amdgcn_readfirstlane(axis_) == 1;
    const ColArgs c = load_cols(a1 ? &xf[x].c1 : &xf[x].c0);
    const int gx = a1 ? xf[x].gx1 : xf[x].gx0;
    cols_body_s<T, true, kQThreads, L, queue_cols_nl<T>(L)>(c, tile % gx, tile / gx, smem_raw);
}

template <typename T>
__device__ __forceinline__ void q_fft(const BatchXform *xf, const QSeg &sg, int task) {
    if (sg.stage == 0) {
        switch (sg.kind) {
#define NFFT3_Q_ROWS(L) \
            case L: q_rows<T, L>(xf, sg.x, task); return;
            NFFT3_STATIC_LENGTHS(NFFT3_Q_ROWS)
#undef NFFT3_Q_ROWS
            default: return;
        }
    }
    const int axis = sg.stage == 1 ? 1 : 0;
    switch (sg.kind) {
#define NFFT3_Q_COLS(L) \
        case L: q_cols<T, L>(xf, sg.x, axis, task); return;
        NFFT3_STATIC_LENGTHS(NFFT3_Q_COLS)
#undef NFFT3_Q_COLS
        default: return;
    }
}

// s_waitcnt with vmcnt(0) and no wait on the other counters (gfx9 encoding:
// vmcnt bits 3:0 and 15:14, expcnt 6:4, lgkmcnt 11:8)
constexpr int kWaitVmcnt0 = 0x0F70;

__device__ __forceinline__ unsigned q_load_acquire(unsigned *p) {
    return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned q_load_relaxed(unsigned *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Wave 0 of the workgroup, all 64 lanes together (every branch here is
// uniform across the wave): the next ticket whose dependency has finished,
// or -1 (queue empty, abort).  Lane 0's share of each atomic is the only
// nonzero one.  (A lane-0-only branch in this loop is not used: the
// compiler may merge the two lane-0 regions across the loop's back edge into
// a loop that the other lanes repeat, past the workgroup barrier, without
// lane 0.)
__device__ __forceinline__ int q_take(const QueueArgs &q, int &seg, int &ok_dep) {
    unsigned *abort_flag = q.ctl + 1;
    const unsigned one = (threadIdx.x & 63) == 0 ? 1u : 0u;
    if (__builtin_amdgcn_readfirstlane(q_load_relaxed(abort_flag))) return -1;
    const int t = (int)__builtin_amdgcn_readfirstlane(
        __hip_atomic_fetch_add(q.ctl, one, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    if (t >= q.total) return -1;
    seg = __builtin_amdgcn_readfirstlane(q.tseg[t]);
    const int dep = __builtin_amdgcn_readfirstlane(q.segs[seg].dep);
    // no dependency, or one this workgroup has already seen finished (its
    // acquire then made the stage's results visible here)
    if (dep < 0 || dep == ok_dep) return t;
    unsigned *d = q.ctl + kQDone + dep;
    const unsigned need = (unsigned)__builtin_amdgcn_readfirstlane(q.segs[seg].need);
    if (__builtin_amdgcn_readfirstlane(q_load_acquire(d)) < need) {
        const unsigned long long t0 = wall_clock64();
        while (__builtin_amdgcn_readfirstlane(q_load_acquire(d)) < need) {
            if (__builtin_amdgcn_readfirstlane(q_load_relaxed(abort_flag)) || wall_clock64() - t0 > q.wait_ticks) {
                __hip_atomic_store(abort_flag, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                return -1;
            }
            __builtin_amdgcn_s_sleep(2);
        }
    }
    ok_dep = dep;
    return t;
}

template <typename T, int W, int PPT, bool FIELDS>
__device__ __forceinline__ void queue_body(const QueueArgs &q) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ int s_take[2];
    // uniform within each wave: wave 0 takes the tickets
    const bool wave0 = __builtin_amdgcn_readfirstlane(threadIdx.x) < 64;
    const unsigned one = (threadIdx.x & 63) == 0 ? 1u : 0u;
    int ok_dep = -1;
    for (;;) {
        if (wave0) {
            int seg = 0;
            const int t = q_take(q, seg, ok_dep);
            s_take[0] = t;                 // every lane of wave 0 writes the same values
            s_take[1] = __builtin_amdgcn_readfirstlane(seg);
        }
        __syncthreads();
        const int t = __builtin_amdgcn_readfirstlane(s_take[0]);
        if (t < 0) break;
        // the segment as uniform values (its fields steer every branch below)
        const QSeg sg = load_uniform((__attribute__((address_space(4))) const QSeg *)q.segs +
                                     __builtin_amdgcn_readfirstlane(s_take[1]));
        const int c0 = (t - sg.first) * sg.chunk, c1 = min(c0 + sg.chunk, sg.ntile);
        if (sg.stage < 3) {
            for (int task = c0; task < c1; ++task) {
                if (task > c0) __syncthreads();       // LDS reuse between tiles
                q_fft<T>(q.xf, sg, task);
            }
            // publish the stage's stores: every wave waits for its own
            // stores to complete, then wave 0's release (one L2 writeback)
            // and count
            __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);
            __syncthreads();
            if (wave0)
                __hip_atomic_fetch_add(q.ctl + kQDone + 4 * sg.x + sg.stage, one, __ATOMIC_RELEASE,
                                       __HIP_MEMORY_SCOPE_AGENT);
        } else {
            // the window sums: nothing waits for them (the kernel's end
            // publishes the outputs)
            cbx_t *xf = uniform_xf(q.xf);
            const PSArgs a = load_ps(&xf[sg.x].ip);
            for (int task = c0; task < c1; ++task) {
                if (task > c0) __syncthreads();
                if constexpr (FIELDS) interp_body_der<T, W, kModeFields>(a, task, smem_raw);
                else interp_body<T, W, PPT>(a, task, smem_raw);
            }
            __syncthreads();
        }
    }
}

// waves per SIMD to hold: the complex<float> window sums up to m = 4 run at
// four (as their own kernel does), the others at two
template <typename T, int W>
constexpr int queue_waves() { return sizeof(T) == 4 && W <= 8 ? 4 : 2; }

template <typename T, int W, int PPT>
__global__ void __launch_bounds__(kQThreads) __attribute__((amdgpu_waves_per_eu(queue_waves<T, W>())))
batch_queue_kernel(QueueArgs q) {
    queue_body<T, W, PPT, false>(q);
}

// complex<double> with derivative fields (the window derivative, as the
// per-length form's fields kernel)
template <typename T, int W>
__global__ void __launch_bounds__(kQThreads) __attribute__((amdgpu_waves_per_eu(2)))
batch_queue_fields_kernel(QueueArgs q) {
    queue_body<T, W, 1, true>(q);
}

template <class K>
static int queue_run(K kernel, const QueueLaunch &q, hipStream_t s) {
    allow_lds((const void *)kernel, q.lds);
    int dev = 0, cus = 0, per = 0;
    NFFT3_HIP_TRY(hipGetDevice(&dev));
    NFFT3_HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    NFFT3_HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, (const void *)kernel, kQThreads, q.lds));
    if (per < 1) return NFFT3_ERR_INVALID_ARG;
    const int grid = (int)std::min<int64_t>((int64_t)cus * per, std::max(q.args.total, 1));
    hipLaunchKernelGGL(kernel, dim3((unsigned)grid), dim3(kQThreads), q.lds, s, q.args);
    NFFT3_LAUNCH_CHECK("batch_queue_kernel");
    return NFFT3_OK;
}

template <typename T>
static int launch_queue_t(const QueueLaunch &q, hipStream_t s) {
    if (q.fields) {
        if constexpr (sizeof(T) == 8) {
            switch (q.W) {
#define NFFT3_QF(W) \
                case W: return queue_run(batch_queue_fields_kernel<T, W>, q, s);
                NFFT3_QF(2) NFFT3_QF(4) NFFT3_QF(6) NFFT3_QF(8) NFFT3_QF(10) NFFT3_QF(12) NFFT3_QF(14) NFFT3_QF(16)
#undef NFFT3_QF
                default: return NFFT3_ERR_INVALID_ARG;
            }
        }
        return NFFT3_ERR_INVALID_ARG;
    }
    switch (q.W * 4 + q.ppt) {
#define NFFT3_QV(W)                                                              \
        case W * 4 + 1: return queue_run(batch_queue_kernel<T, W, 1>, q, s); \
        case W * 4 + 2: return queue_run(batch_queue_kernel<T, W, 2>, q, s);
        NFFT3_QV(2) NFFT3_QV(4) NFFT3_QV(6) NFFT3_QV(8) NFFT3_QV(10) NFFT3_QV(12) NFFT3_QV(14) NFFT3_QV(16)
#undef NFFT3_QV
        default: return NFFT3_ERR_INVALID_ARG;
    }
}

}  // namespace nfft3
