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
