// Stage (a)+(b) of the windowed evaluation: deconvolution, zero-padding and
// the 3-D FFT on the oversampled grid, and the transposed pipeline for the
// adjoint.  Each axis is one pass of self-sorting (Stockham) radix-8/4/2/3/5/7
// FFTs held in LDS:
//   * the contiguous axis (2) runs lines = rows, loaded with unit stride;
//   * the strided axes (1, 0) run tiles of C adjacent columns, so every
//     global access is a C*elt-byte (128 B) contiguous segment, transposed
//     into LDS lines of padded stride n+1.
// Zero-padding is pruned: the forward passes only read the N_d nonzero
// inputs per line and write into the same grid buffer in place
//   pass 1 (axis 2): fhat (N0,N1,N2) -> grid[i0][i1][0..n2)   i0<N0, i1<N1
//   pass 2 (axis 1): grid[i0][0..N1)[x] -> grid[i0][0..n1)[x]  i0<N0
//   pass 3 (axis 0): grid[0..N0)[y][x] -> grid[0..n0)[y][x]
// and the adjoint keeps only the N_d outputs per line in reverse order.
// Leading unit axes (lower-dimensional plans, n_d = N_d = 1) have no pass.
// Compact index i of a pruned line holds frequency i - L/2, which sits at
// FFT position (i - L/2) mod n.
#include "fft_dev.h"

namespace nfft3 {

constexpr int kRowThreads = 256;

template <typename T, int MODE>
__global__ void __launch_bounds__(kRowThreads) fft_rows_kernel(RowArgs a) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    rows_body<T, MODE, kRowThreads>(a, blockIdx.x, smem_raw);
}

template <typename T, bool FWD>
__global__ void __launch_bounds__(kColsThreadsGeneric) fft_cols_kernel(ColArgs a) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cols_body<T, FWD, kColsThreadsGeneric, 16>(a, blockIdx.x, blockIdx.y, smem_raw);
}

// compile-time-engine passes (the lengths of static_fft_len)
template <typename T, int MODE, int N>
__global__ void __launch_bounds__(kRowThreads) fft_rows_kernel_s(RowArgs a) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    rows_body_s<T, MODE, kRowThreads, N, static_rows_nl<T>(N)>(a, blockIdx.x, smem_raw);
}

template <typename T, bool FWD, int N>
__global__ void __launch_bounds__(kColsThreads) fft_cols_kernel_s(ColArgs a) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cols_body_s<T, FWD, kColsThreads, N, static_cols_nl<T>(N)>(a, blockIdx.x, blockIdx.y, smem_raw);
}

template <typename T, int MODE, int N>
static void launch_rows_s(dim3 g, size_t lds, hipStream_t s, const RowArgs &a) {
    hipLaunchKernelGGL((fft_rows_kernel_s<T, MODE, N>), g, dim3(kRowThreads), lds, s, a);
}

template <typename T, bool FWD, int N>
static void launch_cols_s(dim3 g, size_t lds, hipStream_t s, const ColArgs &a) {
    allow_lds((const void *)fft_cols_kernel_s<T, FWD, N>, lds);
    hipLaunchKernelGGL((fft_cols_kernel_s<T, FWD, N>), g, dim3(kColsThreads), lds, s, a);
}

template <typename T, int MODE>
static bool rows_static(const RowArgs &a, dim3 g, size_t lds, hipStream_t s) {
    if (!static_fft_len(a.n) || a.lpw != static_rows_nl<T>(a.n)) return false;
    switch (a.n) {
#define NFFT3_ROWS_LAUNCH(L) \
        case L: launch_rows_s<T, MODE, L>(g, lds, s, a); return true;
        NFFT3_STATIC_LENGTHS(NFFT3_ROWS_LAUNCH)
#undef NFFT3_ROWS_LAUNCH
        default: return false;
    }
}

template <typename T, bool FWD>
static bool cols_static(const ColArgs &a, dim3 g, size_t lds, hipStream_t s) {
    if (!col_static<T>(a)) return false;
    switch (a.n) {
#define NFFT3_COLS_LAUNCH(L) \
        case L: launch_cols_s<T, FWD, L>(g, lds, s, a); return true;
        NFFT3_STATIC_LENGTHS(NFFT3_COLS_LAUNCH)
#undef NFFT3_COLS_LAUNCH
        default: return false;
    }
}

template <typename T>
static int rows_pass(nfft3_plan_impl *p, int mode, const void *in, void *out, int deriv) {
    RowArgs a = make_row_args<T>(p, in, out, deriv, kRowThreads);
    const int64_t nblk = row_blocks(p, a);
    const size_t lds = row_lds<T>(a);
    const bool done = mode == 0 ? rows_static<T, 0>(a, dim3((unsigned)nblk), lds, p->stream)
                                : rows_static<T, 1>(a, dim3((unsigned)nblk), lds, p->stream);
    if (done) {
        NFFT3_LAUNCH_CHECK("fft_rows_kernel_s");
        return NFFT3_OK;
    }
    if (mode == 0)
        hipLaunchKernelGGL((fft_rows_kernel<T, 0>), dim3((unsigned)nblk), dim3(kRowThreads), lds, p->stream, a);
    else
        hipLaunchKernelGGL((fft_rows_kernel<T, 1>), dim3((unsigned)nblk), dim3(kRowThreads), lds, p->stream, a);
    NFFT3_LAUNCH_CHECK("fft_rows_kernel");
    return NFFT3_OK;
}

template <typename T>
static int cols_pass(nfft3_plan_impl *p, int axis, bool fwd, int Lin, int Lout, int64_t n_outer,
                     int64_t s_outer) {
    ColArgs a = make_col_args<T>(p, p->grid, axis, Lin, Lout, s_outer);
    dim3 grid((unsigned)col_grid_x(a), (unsigned)n_outer);
    const size_t lds = col_lds<T>(a);
    const bool done = fwd ? cols_static<T, true>(a, grid, lds, p->stream)
                          : cols_static<T, false>(a, grid, lds, p->stream);
    if (done) {
        NFFT3_LAUNCH_CHECK("fft_cols_kernel_s");
        return NFFT3_OK;
    }
    if (fwd) {
        allow_lds((const void *)fft_cols_kernel<T, true>, lds);
        hipLaunchKernelGGL((fft_cols_kernel<T, true>), grid, dim3(kColsThreadsGeneric), lds, p->stream, a);
    } else {
        allow_lds((const void *)fft_cols_kernel<T, false>, lds);
        hipLaunchKernelGGL((fft_cols_kernel<T, false>), grid, dim3(kColsThreadsGeneric), lds, p->stream, a);
    }
    NFFT3_LAUNCH_CHECK("fft_cols_kernel");
    return NFFT3_OK;
}

template <typename T>
static int grid_forward(nfft3_plan_impl *p, const void *fhat, int deriv) {
    int rc = rows_pass<T>(p, 0, fhat, p->grid, deriv);
    if (rc) return rc;
    // (a unit axis, n = N = 1, has no pass: its transform is the identity)
    // axis 1: tiles over i0 < N0 (outer stride n1 n2)
    if (p->n[1] > 1) rc = cols_pass<T>(p, 1, true, (int)p->N[1], (int)p->n[1], p->N[0], p->n[1] * p->n[2]);
    if (rc) return rc;
    // axis 0: tiles over y < n1 (outer stride n2)
    if (p->n[0] > 1) rc = cols_pass<T>(p, 0, true, (int)p->N[0], (int)p->n[0], p->n[1], p->n[2]);
    return rc;
}

template <typename T>
static int grid_adjoint(nfft3_plan_impl *p, void *fhat) {
    int rc = NFFT3_OK;
    if (p->n[0] > 1) rc = cols_pass<T>(p, 0, false, (int)p->n[0], (int)p->N[0], p->n[1], p->n[2]);
    if (rc) return rc;
    if (p->n[1] > 1) rc = cols_pass<T>(p, 1, false, (int)p->n[1], (int)p->N[1], p->N[0], p->n[1] * p->n[2]);
    if (rc) return rc;
    return rows_pass<T>(p, 1, p->grid, fhat, -1);
}

int launch_grid_forward(nfft3_plan_impl *p, const void *fhat, void *grid, int deriv_axis) {
    void *saved = p->grid;
    p->grid = grid;
    int rc = p->dtype == NFFT3_C128 ? grid_forward<double>(p, fhat, deriv_axis)
                                    : grid_forward<float>(p, fhat, deriv_axis);
    p->grid = saved;
    return rc;
}

int launch_grid_adjoint(nfft3_plan_impl *p, void *grid, void *fhat) {
    void *saved = p->grid;
    p->grid = grid;
    int rc = p->dtype == NFFT3_C128 ? grid_adjoint<double>(p, fhat) : grid_adjoint<float>(p, fhat);
    p->grid = saved;
    return rc;
}

}  // namespace nfft3
