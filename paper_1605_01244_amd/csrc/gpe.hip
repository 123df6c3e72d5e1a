// Time splitting pseudospectral (TSSP) integration of the Gross-Pitaevskii
// equation of Sec. 3.1,
//
//   d psi / dt = (i/2) Lap psi + (i/2) (1 - |psi|^2) psi,
//
// on the regular grid X_N of a periodic domain prod [a_d, b_d), by Strang
// splitting: half a step of the potential part, whose flow keeps |v| and is
// therefore exact, v <- exp((tau/2) (i/2) (1 - |v|^2)) v; a full step of the
// kinetic part, exact in Fourier space (each mode times
// exp(-i tau |kappa_k|^2 / 2), kappa_{k,d} = 2 pi k_d / (b_d - a_d), the
// eq. (Lambda) multipliers squared); half a step of the potential part.
// Consecutive half steps of the potential part are merged into one (exact,
// since |v| is kept).
//
// The Fourier transforms are the Stockham passes of the grid stage on an
// FFT-only plan with n = N (no oversampling, unit deconvolution factors),
// in place on the state: the adjoint pipeline (axis 0, axis 1, then rows)
// takes the grid values to sum_x psi_x exp(+2 pi i k.x/N), stored in FFT
// order on axes 0 and 1 and centred (index k + N_2/2) on axis 2; the
// forward pipeline (rows, axis 1, axis 0) reads that layout back with the
// opposite sign, so the pair is N0 N1 N2 times the identity.
#include "internal.h"

namespace nfft3 {

// v <- exp(i c (1 - |v|^2)) v
template <typename T>
__global__ void gpe_potential_kernel(c_t<T> *__restrict__ g, int64_t count, double c) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= count) return;
    const c_t<T> v = g[e];
    const T th = (T)c * ((T)1 - (v.x * v.x + v.y * v.y));
    T s, co;
    if constexpr (sizeof(T) == 8) sincos(th, &s, &co);
    else __sincosf(th, &s, &co);
    g[e] = cmk<T>(co * v.x - s * v.y, co * v.y + s * v.x);
}

// mode (i0, i1, i2) of the adjoint pipeline's layout times
// exp(-i tau |kappa|^2 / 2) / (N0 N1 N2); the phase is formed in FP64
template <typename T>
__global__ void gpe_kinetic_kernel(c_t<T> *__restrict__ g, int64_t N0, int64_t N1, int64_t N2, double w0, double w1,
                                   double w2, double tau, double norm) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= N0 * N1 * N2) return;
    const int64_t i2 = e % N2, r = e / N2, i1 = r % N1, i0 = r / N1;
    const double k0 = (double)(i0 < N0 / 2 ? i0 : i0 - N0);
    const double k1 = (double)(i1 < N1 / 2 ? i1 : i1 - N1);
    const double k2 = (double)(i2 - N2 / 2);
    const double kap = (w0 * k0) * (w0 * k0) + (w1 * k1) * (w1 * k1) + (w2 * k2) * (w2 * k2);
    double s, c;
    sincos(-0.5 * tau * kap, &s, &c);
    const T cs = (T)(c * norm), sn = (T)(s * norm);
    const c_t<T> v = g[e];
    g[e] = cmk<T>(cs * v.x - sn * v.y, cs * v.y + sn * v.x);
}

// v <- conj(v)
template <typename T>
__global__ void gpe_conj_kernel(const c_t<T> *__restrict__ in, c_t<T> *__restrict__ out, int64_t count) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= count) return;
    const c_t<T> v = in[e];
    out[e] = cmk<T>(v.x, -v.y);
}

// psihat[c0][c1][c2] (centred: frequency c_d - N_d/2) = conj(S) scale, S in
// the adjoint pipeline's layout (FFT order on axes 0, 1; centred on axis 2)
template <typename T>
__global__ void gpe_coeffs_kernel(const c_t<T> *__restrict__ S, int64_t N0, int64_t N1, int64_t N2, double scale,
                                  c_t<T> *__restrict__ psihat) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= N0 * N1 * N2) return;
    const int64_t c2 = e % N2, r = e / N2, c1 = r % N1, c0 = r / N1;
    const int64_t j0 = (c0 - N0 / 2 + N0) % N0, j1 = (c1 - N1 / 2 + N1) % N1;
    const c_t<T> v = S[(j0 * N1 + j1) * N2 + c2];
    psihat[e] = cmk<T>((T)(v.x * scale), (T)(-v.y * scale));
}

template <typename T>
static int gpe_potential(nfft3_gpe_impl *g, double half_steps) {
    const int64_t cnt = g->fp.N[0] * g->fp.N[1] * g->fp.N[2];
    const double c = 0.5 * (g->tau / 2) * half_steps;
    hipLaunchKernelGGL(gpe_potential_kernel<T>, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, g->fp.stream,
                       (c_t<T> *)g->state, cnt, c);
    NFFT3_LAUNCH_CHECK("gpe_potential_kernel");
    return NFFT3_OK;
}

template <typename T>
static int gpe_steps_t(nfft3_gpe_impl *g, int nsteps) {
    nfft3_plan_impl *p = &g->fp;
    const int64_t N0 = p->N[0], N1 = p->N[1], N2 = p->N[2], cnt = N0 * N1 * N2;
    const double two_pi = 6.283185307179586476925286766559;
    const double w0 = two_pi / g->len[0], w1 = two_pi / g->len[1], w2 = two_pi / g->len[2];
    const double norm = 1.0 / (double)cnt;
    for (int s = 0; s < nsteps; ++s) {
        int rc = gpe_potential<T>(g, s == 0 ? 1.0 : 2.0);     // the previous step's half merged in
        if (rc) return rc;
        rc = launch_grid_adjoint(p, g->state, g->state);
        if (rc) return rc;
        hipLaunchKernelGGL(gpe_kinetic_kernel<T>, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, p->stream,
                           (c_t<T> *)g->state, N0, N1, N2, w0, w1, w2, g->tau, norm);
        NFFT3_LAUNCH_CHECK("gpe_kinetic_kernel");
        rc = launch_grid_forward(p, g->state, g->state, -1);
        if (rc) return rc;
    }
    return nsteps > 0 ? gpe_potential<T>(g, 1.0) : NFFT3_OK;
}

int launch_gpe_steps(nfft3_gpe_impl *g, int nsteps) {
    return g->fp.dtype == NFFT3_C128 ? gpe_steps_t<double>(g, nsteps) : gpe_steps_t<float>(g, nsteps);
}

template <typename T>
static int gpe_coeffs_t(nfft3_gpe_impl *g, void *psihat) {
    nfft3_plan_impl *p = &g->fp;
    const int64_t N0 = p->N[0], N1 = p->N[1], N2 = p->N[2], cnt = N0 * N1 * N2;
    const unsigned blocks = (unsigned)((cnt + 255) / 256);
    hipLaunchKernelGGL(gpe_conj_kernel<T>, dim3(blocks), dim3(256), 0, p->stream, (const c_t<T> *)g->state,
                       (c_t<T> *)g->work, cnt);
    NFFT3_LAUNCH_CHECK("gpe_conj_kernel");
    int rc = launch_grid_adjoint(p, g->work, g->work);
    if (rc) return rc;
    double scale = 1.0;
    for (int d = 0; d < 3; ++d) scale *= sqrt(g->len[d]) / (double)p->N[d];
    hipLaunchKernelGGL(gpe_coeffs_kernel<T>, dim3(blocks), dim3(256), 0, p->stream, (const c_t<T> *)g->work, N0, N1,
                       N2, scale, (c_t<T> *)psihat);
    NFFT3_LAUNCH_CHECK("gpe_coeffs_kernel");
    return NFFT3_OK;
}

int launch_gpe_coeffs(nfft3_gpe_impl *g, void *psihat) {
    return g->fp.dtype == NFFT3_C128 ? gpe_coeffs_t<double>(g, psihat) : gpe_coeffs_t<float>(g, psihat);
}

}  // namespace nfft3
