// The series of eq. (fs) on a physical domain prod [a_d, b_d) (Sec. 2.2.1),
// and the evaluation within vortex tubes (Sec. 4.3).
//
// eq. (fs): psi(xi) = sum_k psihat_k prod_d exp(+2 pi i k_d (xi_d - a_d)/(b_d - a_d)) / sqrt(b_d - a_d)
// is the NFFT problem at zeta_d = mod((xi_d - a_d)/(a_d - b_d), 1) - 1/2
// (Euclidean remainder) with fhat_k = psihat_k (-1)^(k_0 + k_1 + k_2) /
// prod sqrt(b_d - a_d): with t = (xi - a)/(b - a), zeta = 1/2 - t mod 1 and
// exp(-2 pi i k zeta) = (-1)^k exp(2 pi i k t), whose sign the coefficient
// factor cancels.  Here k_d = i_d - N_d/2 for array index i_d.  A plan of
// fewer axes (the one- and two-dimensional series) takes a_d = 0, b_d = 1 on
// its unit axes, where k_d = 0 and both factors are 1.
//
// Tube refinement: start from the points of the regular grid X_N of the
// domain (x_{d,n} = a_d + n h_d) and rho = |psi|^2 there; for each threshold
// rhobar_l keep the current points with rho <= rhobar_l (flag, scan,
// compaction on the device), replace each by the 27 points of a regular
// grid of step h_d / 3^(l+1) centred on it, and evaluate rho there.
#include <algorithm>
#include <utility>

#include "internal.h"

namespace nfft3 {

struct Domain {
    double a[3];
    double inv[3];      // 1 / (a_d - b_d)
    double h[3];        // (b_d - a_d) / N_d
};

__device__ __forceinline__ double euclid_mod1(double v) {
    const double r = v - floor(v);
    return r >= 1.0 ? 0.0 : r;              // floor rounding can leave r = 1
}

// zeta = mod((xi - a)/(a - b), 1) - 1/2; NaN / Inf pass through (set_points
// reports them).  Points of dim coordinates: the plan's last dim axes.
__global__ void map_points_kernel(const double *__restrict__ xi, int64_t M, int dim, Domain D,
                                  double *__restrict__ zeta) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= dim * M) return;
    const int d = 3 - dim + (int)(e % dim);
    const double v = xi[e];
    zeta[e] = isfinite(v) ? euclid_mod1((v - D.a[d]) * D.inv[d]) - 0.5 : v;
}

// fhat_i = psihat_i (-1)^(sum_d i_d - N_d/2) scale
template <typename T>
__global__ void coeff_sign_kernel(const c_t<T> *__restrict__ psihat, int64_t N0, int64_t N1, int64_t N2, T scale,
                                  c_t<T> *__restrict__ fhat) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= N0 * N1 * N2) return;
    const int64_t i2 = e % N2, r = e / N2, i1 = r % N1, i0 = r / N1;
    const int64_t s = (i0 - N0 / 2) + (i1 - N1 / 2) + (i2 - N2 / 2);
    const T f = (s & 1) ? -scale : scale;
    const c_t<T> v = psihat[e];
    fhat[e] = cmk<T>(v.x * f, v.y * f);
}

// the points of X_N, C order of (n0, n1, n2)
__global__ void regular_grid_kernel(int64_t N0, int64_t N1, int64_t N2, Domain D, double *__restrict__ pts) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= N0 * N1 * N2) return;
    const int64_t n2 = e % N2, r = e / N2, n1 = r % N1, n0 = r / N1;
    pts[3 * e + 0] = D.a[0] + (double)n0 * D.h[0];
    pts[3 * e + 1] = D.a[1] + (double)n1 * D.h[1];
    pts[3 * e + 2] = D.a[2] + (double)n2 * D.h[2];
}

// rho = |psi|^2 (in FP64) and the keep flag rho <= rhobar
template <typename T>
__global__ void rho_flag_kernel(const c_t<T> *__restrict__ psi, int64_t M, double rhobar, double *__restrict__ rho,
                                int *__restrict__ keep) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= M) return;
    const c_t<T> v = psi[j];
    const double r = (double)v.x * (double)v.x + (double)v.y * (double)v.y;
    rho[j] = r;
    if (keep) keep[j] = r <= rhobar ? 1 : 0;
}

// the 27 points of step h / 3^level around each kept point (slot = scanned
// keep flag); neighbour (o0, o1, o2) in {-1, 0, 1}^3 at index 9 (o0 + 1) +
// 3 (o1 + 1) + o2 + 1
__global__ void refine_kernel(const double *__restrict__ pts, const int *__restrict__ keep,
                              const int *__restrict__ slot, int64_t M, Domain D, double div,
                              double *__restrict__ out) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= M || !keep[j]) return;
    const double c0 = pts[3 * j], c1 = pts[3 * j + 1], c2 = pts[3 * j + 2];
    const double s0 = D.h[0] / div, s1 = D.h[1] / div, s2 = D.h[2] / div;
    double *o = out + 81 * (int64_t)slot[j];
    for (int q = 0; q < 27; ++q) {
        const int o0 = q / 9 - 1, o1 = (q / 3) % 3 - 1, o2 = q % 3 - 1;
        o[3 * q + 0] = c0 + o0 * s0;
        o[3 * q + 1] = c1 + o1 * s1;
        o[3 * q + 2] = c2 + o2 * s2;
    }
}

static Domain make_domain(const nfft3_plan_impl *p, const double a[3], const double b[3]) {
    Domain D;
    for (int d = 0; d < 3; ++d) {
        D.a[d] = a[d];
        D.inv[d] = 1.0 / (a[d] - b[d]);
        D.h[d] = (b[d] - a[d]) / (double)p->N[d];
    }
    return D;
}

static int ensure(void **buf, int64_t *cap, int64_t need, size_t elt) {
    if (need <= *cap) return NFFT3_OK;
    (void)hipFree(*buf);
    *buf = nullptr;
    *cap = 0;
    NFFT3_HIP_TRY(hipMalloc(buf, (size_t)std::max<int64_t>(need, 1) * elt));
    *cap = need;
    return NFFT3_OK;
}

int launch_infft3(nfft3_plan_impl *p, const double a[3], const double b[3], const void *psihat, int64_t M,
                  const double *xi, void *psi) {
    const Domain D = make_domain(p, a, b);
    hipStream_t s = p->stream;
    InfftmScratch &S = p->infftm;
    int rc = ensure(&S.zeta, &S.zeta_cap, p->dim * M, sizeof(double));
    if (rc) return rc;
    const int64_t nc = p->N[0] * p->N[1] * p->N[2];
    rc = ensure(&S.fhat, &S.fhat_cap, nc, p->elt);
    if (rc) return rc;
    if (M > 0) {
        hipLaunchKernelGGL(map_points_kernel, dim3((unsigned)((p->dim * M + 255) / 256)), dim3(256), 0, s, xi, M,
                           p->dim, D, (double *)S.zeta);
        NFFT3_LAUNCH_CHECK("map_points_kernel");
    }
    double scale = 1.0;
    for (int d = 0; d < 3; ++d) scale /= sqrt(b[d] - a[d]);
    if (p->dtype == NFFT3_C128)
        hipLaunchKernelGGL(coeff_sign_kernel<double>, dim3((unsigned)((nc + 255) / 256)), dim3(256), 0, s,
                           (const c_t<double> *)psihat, p->N[0], p->N[1], p->N[2], scale, (c_t<double> *)S.fhat);
    else
        hipLaunchKernelGGL(coeff_sign_kernel<float>, dim3((unsigned)((nc + 255) / 256)), dim3(256), 0, s,
                           (const c_t<float> *)psihat, p->N[0], p->N[1], p->N[2], (float)scale,
                           (c_t<float> *)S.fhat);
    NFFT3_LAUNCH_CHECK("coeff_sign_kernel");
    rc = nfft3_set_points(static_cast<nfft3_plan_s *>(p), M, (const double *)S.zeta);
    if (rc) return rc;
    if (M == 0) return NFFT3_OK;
    return nfft3_trafo(static_cast<nfft3_plan_s *>(p), S.fhat, psi);
}

int launch_tube_refine(nfft3_plan_impl *p, const double a[3], const double b[3], const void *psihat, int levels,
                       const double *rhobar, int64_t cap, double *pts_out, double *rho_out, int64_t *count_out) {
    const Domain D = make_domain(p, a, b);
    hipStream_t s = p->stream;
    InfftmScratch &S = p->infftm;
    // level 0: the regular grid and rho there
    int64_t M = p->N[0] * p->N[1] * p->N[2];
    int rc = ensure(&S.pts, &S.pts_cap, 3 * M, sizeof(double));
    if (rc) return rc;
    hipLaunchKernelGGL(regular_grid_kernel, dim3((unsigned)((M + 255) / 256)), dim3(256), 0, s, p->N[0], p->N[1],
                       p->N[2], D, (double *)S.pts);
    NFFT3_LAUNCH_CHECK("regular_grid_kernel");
    for (int lev = 0; lev <= levels; ++lev) {
        rc = ensure(&S.psi, &S.psi_cap, M, p->elt);
        if (!rc) rc = ensure(&S.rho, &S.rho_cap, M, sizeof(double));
        if (!rc) rc = ensure(&S.keep, &S.keep_cap, M + 1, 2 * sizeof(int));   // flags, then their scan
        if (!rc) rc = ensure(&S.sums, &S.sums_cap, M / 1024 + 2, sizeof(int));
        if (rc) return rc;
        rc = launch_infft3(p, a, b, psihat, M, (const double *)S.pts, S.psi);
        if (rc) return rc;
        int *keep = (int *)S.keep;
        int *slot = keep + (M + 1);
        const double rb = lev < levels ? rhobar[lev] : 0.0;
        if (M > 0) {
            if (p->dtype == NFFT3_C128)
                hipLaunchKernelGGL(rho_flag_kernel<double>, dim3((unsigned)((M + 255) / 256)), dim3(256), 0, s,
                                   (const c_t<double> *)S.psi, M, rb, (double *)S.rho, lev < levels ? keep : nullptr);
            else
                hipLaunchKernelGGL(rho_flag_kernel<float>, dim3((unsigned)((M + 255) / 256)), dim3(256), 0, s,
                                   (const c_t<float> *)S.psi, M, rb, (double *)S.rho, lev < levels ? keep : nullptr);
            NFFT3_LAUNCH_CHECK("rho_flag_kernel");
        }
        if (lev == levels) break;
        // kept points -> slots; the count sizes the next level
        rc = launch_exclusive_scan(s, keep, slot, (int *)S.sums, M);
        if (rc) return rc;
        int kept = 0;
        NFFT3_HIP_TRY(hipMemcpyAsync(&kept, slot + M, sizeof(int), hipMemcpyDeviceToHost, s));
        NFFT3_HIP_TRY(hipStreamSynchronize(s));
        const int64_t M2 = 27 * (int64_t)kept;
        if (M2 > (int64_t)INT32_MAX) return NFFT3_ERR_CAPACITY;
        rc = ensure(&S.pts2, &S.pts2_cap, 3 * M2, sizeof(double));
        if (rc) return rc;
        if (M > 0) {
            hipLaunchKernelGGL(refine_kernel, dim3((unsigned)((M + 255) / 256)), dim3(256), 0, s,
                               (const double *)S.pts, keep, slot, M, D, pow(3.0, lev + 1), (double *)S.pts2);
            NFFT3_LAUNCH_CHECK("refine_kernel");
        }
        std::swap(S.pts, S.pts2);
        std::swap(S.pts_cap, S.pts2_cap);
        M = M2;
    }
    *count_out = M;
    if (M > cap) return NFFT3_ERR_CAPACITY;
    if (M > 0) {
        NFFT3_HIP_TRY(hipMemcpyAsync(pts_out, S.pts, sizeof(double) * 3 * M, hipMemcpyDeviceToDevice, s));
        NFFT3_HIP_TRY(hipMemcpyAsync(rho_out, S.rho, sizeof(double) * M, hipMemcpyDeviceToDevice, s));
    }
    return NFFT3_OK;
}

void free_infftm(nfft3_plan_impl *p) {
    InfftmScratch &S = p->infftm;
    void **bufs[] = {&S.zeta, &S.fhat, &S.pts, &S.pts2, &S.psi, &S.rho, &S.keep, &S.sums};
    for (void **b : bufs) {
        (void)hipFree(*b);
        *b = nullptr;
    }
    S = InfftmScratch();
}

}  // namespace nfft3
