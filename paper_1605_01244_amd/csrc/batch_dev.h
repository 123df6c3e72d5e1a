// Launch descriptors of the batched evaluation, shared by the per-length
// launches (batch.hip) and the work-queue form (queue_impl.h).
#pragma once
#include "fft_dev.h"
#include "interp_dev.h"

namespace nfft3 {

constexpr int kStages = 4;
constexpr int kBRowThreads = 256;

// One transform (a plan and one of its fields): the arguments of its four
// stages and the number of tiles (row blocks, column tiles, point items) of
// each.
struct BatchXform {
    RowArgs rows;
    ColArgs c1, c0;
    PSArgs ip;
    int gx1, gx0;
    int ntile[kStages];
};

// ------------------------------------------------ descriptor loads ----
// Both forms read their descriptors from a device table.  The helpers below
// read them as uniform (scalar) values through the constant address space
// and keep their pointers marked as global memory, so that the stage bodies
// compile to global (not flat) accesses with uniform control flow, whether
// they are inlined into a kernel or called.
typedef __attribute__((address_space(4))) const BatchXform cbx_t;

// a copy of *p read as uniform (scalar) values
template <class S>
__device__ __forceinline__ S load_uniform(__attribute__((address_space(4))) const S *p) {
    static_assert(sizeof(S) % 4 == 0, "descriptor size");
    S v;
    const __attribute__((address_space(4))) int *src = (const __attribute__((address_space(4))) int *)p;
    int *dst = reinterpret_cast<int *>(&v);
#pragma unroll
    for (int i = 0; i < (int)(sizeof(S) / 4); ++i) dst[i] = src[i];
    return v;
}

// A descriptor pointer field reloaded as a global-memory pointer (the
// word-wise copy above loses that): accesses through it then compile to
// global, not flat, instructions, and loads at uniform addresses stay
// uniform.
template <class P>
__device__ __forceinline__ P *gptr_at(const __attribute__((address_space(4))) void *loc) {
    typedef __attribute__((address_space(1))) P *gptr;
    return (P *)*(const __attribute__((address_space(4))) gptr *)loc;
}
__device__ __forceinline__ RowArgs load_rows(__attribute__((address_space(4))) const RowArgs *src) {
    RowArgs a = load_uniform(src);
    a.in = gptr_at<const void>(&src->in);
    a.out = gptr_at<void>(&src->out);
    a.c0 = gptr_at<const void>(&src->c0);
    a.c1 = gptr_at<const void>(&src->c1);
    a.c2 = gptr_at<const void>(&src->c2);
    a.tw = gptr_at<const void>(&src->tw);
    a.stw = gptr_at<const void>(&src->stw);
    return a;
}
__device__ __forceinline__ ColArgs load_cols(__attribute__((address_space(4))) const ColArgs *src) {
    ColArgs a = load_uniform(src);
    a.data = gptr_at<void>(&src->data);
    a.tw = gptr_at<const void>(&src->tw);
    a.stw = gptr_at<const void>(&src->stw);
    return a;
}
__device__ __forceinline__ PSArgs load_ps(__attribute__((address_space(4))) const PSArgs *src) {
    PSArgs a = load_uniform(src);
    a.xs = gptr_at<const double>(&src->xs);
    a.perm = gptr_at<const int>(&src->perm);
    a.items = gptr_at<const int4>(&src->items);
    a.grid = gptr_at<const void>(&src->grid);
    a.grid_out = gptr_at<void>(&src->grid_out);
    a.vals = gptr_at<const void>(&src->vals);
    a.out = gptr_at<void>(&src->out);
    a.coef = gptr_at<const void>(&src->coef);
    return a;
}

// the descriptor table as a uniform constant-address pointer
__device__ __forceinline__ cbx_t *uniform_xf(const BatchXform *xf) {
    const uint64_t pa = (uint64_t)xf;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)pa);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(pa >> 32));
    return (cbx_t *)(((uint64_t)hi << 32) | lo);
}

// ------------------------------------------------------- work queue ----
// The work-queue form runs the whole batch as one launch of persistent
// workgroups that take tickets 0, 1, ... from a counter.  The tickets are
// laid out in segments: stage s of transform x holds ceil(ntile[s] / chunk)
// consecutive tickets of `chunk` tiles each, stage-major (every transform's
// row pass, then every axis-1 pass, ...), so a ticket depends only on
// tickets lower than itself: the earlier stage of its own transform.
struct QSeg {
    int first;     // first ticket
    int x;         // transform
    int stage;     // 0 rows, 1 cols axis 1, 2 cols axis 0, 3 window sums
    int kind;      // FFT stages: compile-time length
    int dep;       // index into the done counters of the stage waited for, or -1
    int need;      // tickets of that stage
    int ntile;     // tiles of this stage
    int chunk;     // tiles per ticket (consecutive tiles run by one workgroup)
};

// Control words (device, zeroed by the launch before the queue kernel):
// [0] next ticket, [1] abort flag, [kQDone + 4 x + s] finished tickets of
// stage s of transform x.
constexpr int kQDone = 64;

struct QueueArgs {
    const BatchXform *xf;
    const QSeg *segs;
    const int *tseg;     // segment of each ticket
    unsigned *ctl;
    int nseg;
    int total;
    unsigned long long wait_ticks;   // wall-clock ticks a wait may last
};

constexpr int kQThreads = 256;
// Tiles per ticket.  A ticket costs a device-scope atomic on one counter
// (and the scheduling around it), so short tiles are taken in runs: an FFT
// stage about 4 tickets per CU, each of at most kQChunkFftMax tiles; the
// complex<float> window sums two items per ticket when there are many.
constexpr int kQChunkFftMax = 128;
constexpr int kQTicketsPerCu = 4;
constexpr size_t kQColsLdsMax = 72 * 1024;

// Columns per tile of the queue's static-length column passes: 256 threads
// with at most 16 values each (the per-length kernels use 1024 threads), up
// to 256 contiguous bytes per row visit.
template <typename T>
constexpr int queue_cols_nl(int n) {
    int C = 256 / (int)sizeof(c_t<T>);
    while (C > 1 && C * (n + 1) * (int)sizeof(c_t<T>) > (int)kQColsLdsMax) C /= 2;
    const int f = st_lines_fit(n, 16, C, kQThreads);
    return f < C ? f : C;
}

struct QueueLaunch {
    QueueArgs args;
    size_t lds;
    int W, ppt;
    bool fields;
};
// one launch of the queue kernel (queue_f32.hip / queue_f64.hip)
int launch_queue_f32(const QueueLaunch &q, hipStream_t s);
int launch_queue_f64(const QueueLaunch &q, hipStream_t s);

}  // namespace nfft3
