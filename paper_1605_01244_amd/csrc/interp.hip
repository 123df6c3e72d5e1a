// Stage (c) of the windowed evaluation and its derivative in the points:
//   interp : f_j      = sum_{r in {-m+1..m}^3} g[(u_j + r) mod n] prod_d w_d(r_d)
//   grad   : d f_j/d x_{j,d} = n_d sum_r g[...] w_d'(r_d) prod_{e != d} w_e(r_e)
//            (contracted with the cotangent G_j for the point gradient, or
//            written out as the derivative fields)
// (the adjoint, spreading, is in spread.hip)
// with u_j = floor(n x_j) and w_d(r) = phi((n x_j)_d - u_d - r)/phi(0) from the
// per-offset window polynomials in the cell fraction (see api.hip).  Cell and
// fraction are formed in FP64 in both precisions.
//
// Plane streaming.  Points are sorted by (tile, z-cell), a tile being a
// By x Bx block of (y, x) cells; a work item is at most 512 points (two per
// thread of a 256-thread workgroup; 256 through nfft3_set_tuning) of one tile
// column spanning at most 64 z-cells.  The workgroup walks the grid planes
// z = zmin-m+1 .. zmax+m of its item; each plane's (By+2m-1) x (Bx+2m-1)
// region (the tile plus the stencil halo, wrapped periodically) is staged in
// LDS, with the next plane's global loads issued before the current plane is
// consumed: complex<double> double-buffered (m = 8 by direct global-to-LDS
// loads), complex<float> as two copies (as is and shifted by one element) in
// one buffer.  A thread whose point has
// the plane inside its stencil adds w0 * sum_{r1,r2} w1 w2 g from LDS; the y/x
// weights live in registers for the whole item, the z weight is one polynomial
// per plane.  The spread kernel (spread.hip) walks the same items and planes.
#include "interp_dev.h"

namespace nfft3 {

template <typename T, int W, int PPT>
__global__ void __launch_bounds__(kPsThreads) interp_ps_kernel(PSArgs a) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    interp_body<T, W, PPT>(a, xcd_item(blockIdx.x, gridDim.x), smem_raw);
}

// one-dimensional plans (unit axes 0 and 1): one stencil row per point
template <typename T, int W, int PPT>
__global__ void __launch_bounds__(kPsThreads) interp_row1_kernel(PSArgs a) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    interp_body<T, W, PPT, true>(a, xcd_item(blockIdx.x, gridDim.x), smem_raw);
}

// ------------------------------------------------------- grad, fields ----
// The interp body in its derivative modes (rotated, conflict-free reads), one
// point per thread: items of more points are taken 256 at a time.
template <typename T, int W>
__global__ void __launch_bounds__(kPsThreads) __attribute__((amdgpu_waves_per_eu(2)))
grad_ps_kernel(PSArgs a) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    interp_body_der<T, W, kModeGrad>(a, xcd_item(blockIdx.x, gridDim.x), smem_raw);
}

// the field and its derivative fields from one grid (complex<double>: the
// window derivative meets the FP64 gates; see launch_fields)
template <typename T, int W>
__global__ void __launch_bounds__(kPsThreads) __attribute__((amdgpu_waves_per_eu(2)))
fields_ps_kernel(PSArgs a) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    interp_body_der<T, W, kModeFields>(a, xcd_item(blockIdx.x, gridDim.x), smem_raw);
}

// ------------------------------------------------------------ dispatch ----
template <typename T, int W, int PPT>
static int interp_ppt(nfft3_plan_impl *p, const void *grid, void *f) {
    PSArgs a = interp_args(p);
    if (!interp_layout_ok(p, a)) return NFFT3_ERR_INVALID_ARG;
    a.grid = grid;
    a.out = f;
    const size_t lds = interp_lds(p, a);
    if ((p->unit & 3) == 3) {
        allow_lds((const void *)interp_row1_kernel<T, W, PPT>, lds);
        hipLaunchKernelGGL((interp_row1_kernel<T, W, PPT>), dim3((unsigned)p->sub.count), dim3(kPsThreads), lds,
                           p->stream, a);
        NFFT3_LAUNCH_CHECK("interp_row1_kernel");
        return NFFT3_OK;
    }
    allow_lds((const void *)interp_ps_kernel<T, W, PPT>, lds);
    hipLaunchKernelGGL((interp_ps_kernel<T, W, PPT>), dim3((unsigned)p->sub.count), dim3(kPsThreads), lds,
                       p->stream, a);
    NFFT3_LAUNCH_CHECK("interp_ps_kernel");
    return NFFT3_OK;
}

template <typename T, int W>
static int interp_w(nfft3_plan_impl *p, const void *grid, void *f) {
    if (p->M == 0 || p->sub.count == 0) return NFFT3_OK;
    switch (p->sub.maxpts / kPsThreads) {
        case 1: return interp_ppt<T, W, 1>(p, grid, f);
        case 2: return interp_ppt<T, W, 2>(p, grid, f);
        default: return NFFT3_ERR_INVALID_ARG;
    }
}

template <typename T, int W>
static int grad_w(nfft3_plan_impl *p, const void *grid, const void *G, double *gx) {
    if (p->M == 0 || p->sub.count == 0) return NFFT3_OK;
    PSArgs a = interp_args(p);
    if (!interp_layout_ok(p, a)) return NFFT3_ERR_INVALID_ARG;
    a.grid = grid;
    a.vals = G;
    a.out = gx;
    const size_t lds = interp_lds(p, a);
    allow_lds((const void *)grad_ps_kernel<T, W>, lds);
    hipLaunchKernelGGL((grad_ps_kernel<T, W>), dim3((unsigned)p->sub.count), dim3(kPsThreads), lds, p->stream, a);
    NFFT3_LAUNCH_CHECK("grad_ps_kernel");
    return NFFT3_OK;
}

template <typename T, int W>
static int fields_w(nfft3_plan_impl *p, const void *grid, void *out, int mask) {
    if (p->M == 0 || p->sub.count == 0) return NFFT3_OK;
    PSArgs a = interp_args(p);
    if (!interp_layout_ok(p, a)) return NFFT3_ERR_INVALID_ARG;
    a.grid = grid;
    a.out = out;
    a.fmask = mask;
    a.fstride = p->M;
    const size_t lds = interp_lds(p, a);
    allow_lds((const void *)fields_ps_kernel<T, W>, lds);
    hipLaunchKernelGGL((fields_ps_kernel<T, W>), dim3((unsigned)p->sub.count), dim3(kPsThreads), lds, p->stream,
                       a);
    NFFT3_LAUNCH_CHECK("fields_ps_kernel");
    return NFFT3_OK;
}

int launch_fields(nfft3_plan_impl *p, const void *grid, void *out, int mask) {
    if (p->dtype != NFFT3_C128) return NFFT3_ERR_DTYPE;
    NFFT3_DISPATCH_M(fields_w, double, grid, out, mask)
}

int launch_interp(nfft3_plan_impl *p, const void *grid, void *f) {
    if (p->dtype == NFFT3_C128) { NFFT3_DISPATCH_M(interp_w, double, grid, f) }
    NFFT3_DISPATCH_M(interp_w, float, grid, f)
}

int launch_grad(nfft3_plan_impl *p, const void *grid, const void *G, double *gx) {
    if (p->dtype == NFFT3_C128) { NFFT3_DISPATCH_M(grad_w, double, grid, G, gx) }
    NFFT3_DISPATCH_M(grad_w, float, grid, G, gx)
}

}  // namespace nfft3
