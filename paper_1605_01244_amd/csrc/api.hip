// C ABI of libnfft3: argument validation, plan construction, host-side
// tables (deconvolution factors, window polynomials, FFT twiddles) and the
// orchestration of the device stages.  See include/nfft3.h for the contract.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <new>

#include "internal.h"

namespace nfft3 {

static thread_local std::string g_last_hip;

void set_hip_error(hipError_t e, const char *where) {
    g_last_hip = std::string(where) + ": " + hipGetErrorName(e) + " (" + hipGetErrorString(e) + ")";
}

void allow_lds(const void *kernel, size_t bytes) {
    // a failure here shows up as a launch error of the kernel, which is checked
    if (bytes > 65536) (void)hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

// ---------------------------------------------------------------------------
// Host tables
// ---------------------------------------------------------------------------

// Modified Bessel function I0 by its power series sum_q (x^2/4)^q / (q!)^2,
// summed in long double (all terms positive, no cancellation).
static long double i0_series(long double x) {
    const long double y = x * x / 4.0L;
    long double term = 1.0L, sum = 1.0L;
    for (int q = 1; q < 500; ++q) {
        term *= y / ((long double)q * (long double)q);
        sum += term;
        if (term < sum * 1e-21L) break;
    }
    return sum;
}

double bessel_i0(double x) { return (double)i0_series((long double)x); }

// Normalised Kaiser-Bessel window phi(t)/phi(0), |t| <= m, in the form
// (m/s) e^{b(s-m)} expm1(-2bs)/expm1(-2bm), s = sqrt(m^2 - t^2), which has no
// overflow for any m and no cancellation as s -> 0.
static long double kb_norm(long double t, int m, long double b) {
    long double at = fabsl(t);
    if (at > (long double)m) return 0.0L;
    long double s2 = ((long double)m - at) * ((long double)m + at);
    long double den = expm1l(-2.0L * b * m);
    if (s2 <= 0.0L) return (long double)m * expl(-b * m) * (2.0L * b) / (-den);
    long double s = sqrtl(s2);
    return ((long double)m / s) * expl(b * (s - m)) * (expm1l(-2.0L * b * s) / den);
}

// c[i] = phi(0) / I0(m sqrt(b^2 - (2 pi k / n)^2)), k = i - Nd/2, with
// phi(0) = sinh(b m)/(pi m): the reciprocal of n phihat(k) for the window
// normalised to phi(0) = 1.
void deconv_factors(int64_t Nd, int64_t nd, int m, double b, double *c) {
    const long double pi = 3.14159265358979323846264338327950288L;
    const long double phi0 = sinhl((long double)b * m) / (pi * m);
    for (int64_t i = 0; i < Nd; ++i) {
        long double k = (long double)(i - Nd / 2);
        long double w = 2.0L * pi * k / (long double)nd;
        long double arg = (long double)b * b - w * w;
        long double i0 = i0_series((long double)m * sqrtl(arg > 0 ? arg : 0));
        c[i] = (double)(phi0 / i0);
    }
}

// Chebyshev interpolation of each window piece on [0,1] (variable y = 2f-1),
// converted to monomials in y.  Picks the smallest degree whose error on a
// fine sample is below tol (relative to phi(0) = 1).  Returns the degree, or
// -1 if cap_deg is not enough.
int window_poly(int m, double b, double tol, int cap_deg, std::vector<double> &coef) {
    const long double pi = 3.14159265358979323846264338327950288L;
    const int R = 2 * m;
    for (int deg = 2; deg <= cap_deg; ++deg) {
        const int K = deg + 1;
        std::vector<long double> mono((size_t)R * K, 0.0L);
        for (int r = 0; r < R; ++r) {
            const int off = r - m + 1;
            // Chebyshev coefficients from values at the K Chebyshev nodes
            std::vector<long double> fv(K), ck(K, 0.0L);
            for (int i = 0; i < K; ++i) {
                long double y = cosl(pi * (i + 0.5L) / K);
                fv[i] = kb_norm((y + 1.0L) / 2.0L - off, m, b);
            }
            for (int k = 0; k < K; ++k) {
                long double s = 0.0L;
                for (int i = 0; i < K; ++i) s += fv[i] * cosl(pi * k * (i + 0.5L) / K);
                ck[k] = (k == 0 ? 1.0L : 2.0L) * s / K;
            }
            // monomial coefficients: accumulate c_k T_k(y) with T recurrence
            std::vector<long double> tkm(K, 0.0L), tk(K, 0.0L), tkp(K, 0.0L);
            tkm[0] = 1.0L;                 // T0
            if (K > 1) tk[1] = 1.0L;       // T1
            for (int j = 0; j < K; ++j) mono[(size_t)r * K + j] += ck[0] * tkm[j];
            if (K > 1)
                for (int j = 0; j < K; ++j) mono[(size_t)r * K + j] += ck[1] * tk[j];
            for (int k = 2; k < K; ++k) {
                for (int j = 0; j < K; ++j) tkp[j] = -tkm[j] + (j > 0 ? 2.0L * tk[j - 1] : 0.0L);
                for (int j = 0; j < K; ++j) mono[(size_t)r * K + j] += ck[k] * tkp[j];
                tkm.swap(tk);
                tk.swap(tkp);
            }
        }
        // check in double Horner (the device evaluates the same way)
        double err = 0.0;
        for (int r = 0; r < R && err <= tol; ++r) {
            const int off = r - m + 1;
            for (int s = 0; s <= 400; ++s) {
                double f = s / 400.0;
                double y = 2.0 * f - 1.0;
                double p = (double)mono[(size_t)r * K + deg];
                for (int q = deg - 1; q >= 0; --q) p = p * y + (double)mono[(size_t)r * K + q];
                double ex = (double)kb_norm((long double)f - off, m, b);
                err = std::max(err, fabs(p - ex));
            }
        }
        if (err <= tol) {
            coef.assign((size_t)R * K, 0.0);
            for (size_t i = 0; i < coef.size(); ++i) coef[i] = (double)mono[i];
            return deg;
        }
    }
    return -1;
}

// Radices 8, 4, 2, 3, 5 whose product is n (largest first).
bool factor_radices(int n, std::vector<int> &rad) {
    rad.clear();
    const int nr = st_nrad(n);
    if (nr < 1 || nr > 16) return false;
    for (int s = 0; s < nr; ++s) rad.push_back(st_radix(n, s));
    return true;
}

// ---------------------------------------------------------------------------
// Plan lifetime
// ---------------------------------------------------------------------------

static void free_points(nfft3_plan_impl *p) {
    (void)hipFree(p->xs); p->xs = nullptr;
    (void)hipFree(p->perm); p->perm = nullptr;
    (void)hipFree(p->bin_of); p->bin_of = nullptr;
    (void)hipFree(p->rank); p->rank = nullptr;
    (void)hipFree(p->tx); p->tx = nullptr;
    (void)hipFree(p->tperm); p->tperm = nullptr;
    (void)hipFree(p->tz); p->tz = nullptr;
    (void)hipFree(p->chunk_base); p->chunk_base = nullptr;
    (void)hipFree(p->sort_scratch); p->sort_scratch = nullptr;
    (void)hipFree(p->xin); p->xin = nullptr;
    p->chunk_base_cap = 0;
    p->cap_pts = 0;
    p->cap_xin = 0;
}

static void free_bins(nfft3_plan_impl *p) {
    (void)hipFree(p->bins.counts); p->bins.counts = nullptr;
    (void)hipFree(p->bins.offsets); p->bins.offsets = nullptr;
    (void)hipFree(p->bins.scratch); p->bins.scratch = nullptr;
    (void)hipFree(p->bins.tile_items); p->bins.tile_items = nullptr;
    (void)hipFree(p->bins.tile_item_off); p->bins.tile_item_off = nullptr;
    (void)hipFree(p->bins.tile_counts); p->bins.tile_counts = nullptr;
    (void)hipFree(p->bins.tile_start); p->bins.tile_start = nullptr;
    (void)hipFree(p->bins.chunk_start); p->bins.chunk_start = nullptr;
}
static void free_plan(nfft3_plan_impl *p) {
    if (!p) return;
    (void)hipFree(p->grid);
    for (void *g : p->extra_grids) (void)hipFree(g);
    for (int d = 0; d < 3; ++d) { (void)hipFree(p->cdec[d]); (void)hipFree(p->fft[d].tw); (void)hipFree(p->fft[d].stw); }
    (void)hipFree(p->wcoef);
    free_points(p);
    (void)hipFree(p->flag);
    free_bins(p);
    (void)hipFree(p->sub.items);
    free_infftm(p);
}

static int validate(const int64_t N[3], double sigma, int m, int dtype, int64_t n[3]) {
    if (dtype != NFFT3_C64 && dtype != NFFT3_C128) return NFFT3_ERR_DTYPE;
    if (!(sigma > 1.0) || !isfinite(sigma)) return NFFT3_ERR_INVALID_ARG;
    if (m < 1 || m > 10) return NFFT3_ERR_INVALID_ARG;
    for (int d = 0; d < 3; ++d) {
        // leading unit axes (N_0 = 1, or N_0 = N_1 = 1): lower-dimensional plans
        if (N[d] == 1 && d < 2 && (d == 0 || N[0] == 1)) {
            n[d] = 1;
            continue;
        }
        if (N[d] < 2 || (N[d] % 2) != 0 || N[d] > 4096) return NFFT3_ERR_INVALID_ARG;
        double nd = sigma * (double)N[d];
        int64_t ni = (int64_t)llround(nd);
        if (fabs(nd - (double)ni) > 1e-9 * nd) return NFFT3_ERR_INVALID_ARG;
        if (ni % 2 != 0 || ni > 2048 || ni < 2 * m) return NFFT3_ERR_INVALID_ARG;
        std::vector<int> rad;
        if (!factor_radices((int)ni, rad)) return NFFT3_ERR_INVALID_ARG;
        n[d] = ni;
    }
    return NFFT3_OK;
}

template <typename T>
static int upload_real(const std::vector<double> &v, void **dst) {
    std::vector<T> h(v.begin(), v.end());
    NFFT3_HIP_TRY(hipMalloc(dst, sizeof(T) * std::max<size_t>(h.size(), 1)));
    NFFT3_HIP_TRY(hipMemcpy(*dst, h.data(), sizeof(T) * h.size(), hipMemcpyHostToDevice));
    return NFFT3_OK;
}

template <typename T>
static int upload_stage_twiddles(int n, void **dst) {
    // per-stage tables of the compile-time power-of-two engine
    const long double pi = 3.14159265358979323846264338327950288L;
    const int size = st_tw_size(n);
    if (size == 0) return NFFT3_OK;
    std::vector<T> h(2 * (size_t)size, (T)0);
    for (int s = 1; s < st_nrad(n); ++s) {
        const int ns = st_ns(n, s), R = st_radix(n, s), off = st_tw_offset(n, s);
        for (int k = 0; k < ns; ++k)
            for (int r = 0; r < R; ++r) {
                const long long num = (long long)r * k, den = (long long)ns * R;
                long double re, im;
                if ((4 * num) % den == 0) {   // exact quarter points
                    const int qd = (int)(((4 * num) / den) % 4);
                    const long double qre[4] = {1, 0, -1, 0}, qim[4] = {0, -1, 0, 1};
                    re = qre[qd];
                    im = qim[qd];
                } else {
                    const long double a = -2.0L * pi * (long double)num / (long double)den;
                    re = cosl(a);
                    im = sinl(a);
                }
                h[2 * ((size_t)off + k * 8 + r)] = (T)re;
                h[2 * ((size_t)off + k * 8 + r) + 1] = (T)im;
            }
    }
    NFFT3_HIP_TRY(hipMalloc(dst, sizeof(T) * h.size()));
    NFFT3_HIP_TRY(hipMemcpy(*dst, h.data(), sizeof(T) * h.size(), hipMemcpyHostToDevice));
    return NFFT3_OK;
}

template <typename T>
static int upload_twiddles(int n, void **dst) {
    const long double pi = 3.14159265358979323846264338327950288L;
    std::vector<T> h(2 * (size_t)n);
    for (int k = 0; k < n; ++k) {
        // exp(-2 pi i k/n), angle reduced to the first octant by symmetry-free
        // long double evaluation (error ~1e-19, below either precision)
        long double a = -2.0L * pi * (long double)k / (long double)n;
        h[2 * k] = (T)cosl(a);
        h[2 * k + 1] = (T)sinl(a);
    }
    // exact values at the quarter points
    for (int k = 0; k < n; ++k) {
        if ((4LL * k) % n == 0) {
            int qd = (int)((4LL * k) / n);
            const T re[4] = {1, 0, -1, 0}, im[4] = {0, -1, 0, 1};
            h[2 * k] = re[qd];
            h[2 * k + 1] = im[qd];
        }
    }
    NFFT3_HIP_TRY(hipMalloc(dst, sizeof(T) * h.size()));
    NFFT3_HIP_TRY(hipMemcpy(*dst, h.data(), sizeof(T) * h.size(), hipMemcpyHostToDevice));
    return NFFT3_OK;
}

// Point tiles of edge T (at most kMaxTile, and small enough that the plane,
// tile + stencil halo, fits the window-sum kernels' staging of kMaxPlane
// elements) and the binning buffers sized for them.
static int alloc_bins(nfft3_plan_impl *p, int T) {
    while (T > 4 && (T + 2 * p->m - 1) * (T + 2 * p->m - 1) > kMaxPlane) T -= 4;
    free_bins(p);
    p->bins.By = (int)std::min<int64_t>(T, p->n[1]);
    p->bins.Bx = (int)std::min<int64_t>(T, p->n[2]);
    p->bins.nty = (int)((p->n[1] + p->bins.By - 1) / p->bins.By);
    p->bins.ntx = (int)((p->n[2] + p->bins.Bx - 1) / p->bins.Bx);
    const int64_t ntiles = (int64_t)p->bins.nty * p->bins.ntx;
    const int64_t nb = ntiles * p->n[0];
    p->bins.nbins = nb;
    const int64_t nc = nb * kBinCopies;
    // counter indices (bin copies + copy) and sorted positions are int
    if (nc + 1 > (int64_t)INT32_MAX) return NFFT3_ERR_INVALID_ARG;
    NFFT3_HIP_TRY(hipMalloc(&p->bins.counts, sizeof(int) * nc));
    NFFT3_HIP_TRY(hipMalloc(&p->bins.offsets, sizeof(int) * (nc + 1)));
    NFFT3_HIP_TRY(hipMalloc(&p->bins.scratch, sizeof(int) * (nc / 1024 + 2)));
    // work items are counted per (tile, segment of kItemZ z-cells)
    const int64_t nws = ntiles * ((p->n[0] + kItemZ - 1) / kItemZ);
    NFFT3_HIP_TRY(hipMalloc(&p->bins.tile_items, sizeof(int) * nws));
    NFFT3_HIP_TRY(hipMalloc(&p->bins.tile_item_off, sizeof(int) * (nws + 1)));
    NFFT3_HIP_TRY(hipMalloc(&p->bins.tile_counts, sizeof(int) * ntiles));
    NFFT3_HIP_TRY(hipMalloc(&p->bins.tile_start, sizeof(int) * (ntiles + 1)));
    NFFT3_HIP_TRY(hipMalloc(&p->bins.chunk_start, sizeof(int) * (ntiles + 1)));
    return NFFT3_OK;
}

static int build_plan(nfft3_plan_impl *p) {
    const bool f64 = p->dtype == NFFT3_C128;
    NFFT3_HIP_TRY(hipGetDevice(&p->device));
    const size_t total = (size_t)p->n[0] * p->n[1] * p->n[2];
    NFFT3_HIP_TRY(hipMalloc(&p->grid, total * p->elt));
    NFFT3_HIP_TRY(hipMalloc(&p->flag, 64));
    for (int d = 0; d < 3; ++d) {
        std::vector<double> c((size_t)p->N[d], 1.0);      // unit axis: exact, factor 1
        if (!(p->unit >> d & 1)) deconv_factors(p->N[d], p->n[d], p->m, p->b, c.data());
        int rc = f64 ? upload_real<double>(c, &p->cdec[d]) : upload_real<float>(c, &p->cdec[d]);
        if (rc) return rc;
        std::vector<int> rad;
        factor_radices((int)p->n[d], rad);
        p->fft[d].n = (int)p->n[d];
        p->fft[d].nrad = (int)rad.size();
        for (size_t i = 0; i < rad.size(); ++i) p->fft[d].radix[i] = rad[i];
        rc = f64 ? upload_twiddles<double>((int)p->n[d], &p->fft[d].tw)
                 : upload_twiddles<float>((int)p->n[d], &p->fft[d].tw);
        if (rc) return rc;
        rc = f64 ? upload_stage_twiddles<double>((int)p->n[d], &p->fft[d].stw)
                 : upload_stage_twiddles<float>((int)p->n[d], &p->fft[d].stw);
        if (rc) return rc;
    }
    std::vector<double> coef;
    const double tol = f64 ? 4e-16 : 2e-8;
    int deg = window_poly(p->m, p->b, tol, kMaxDeg, coef);
    if (deg < 0) deg = window_poly(p->m, p->b, f64 ? 2e-15 : 1e-7, kMaxDeg, coef);
    if (deg < 0) return NFFT3_ERR_INVALID_ARG;
    p->deg = deg;
    int rc = f64 ? upload_real<double>(coef, &p->wcoef) : upload_real<float>(coef, &p->wcoef);
    if (rc) return rc;
    // points per work item of the window sums (a thread holds the y/x
    // weights of every point it owns); 512 measured fastest for both forms
    // at N = 256^3, M = 1e7
    p->sub.maxpts = 2 * kItemPts;
    p->tile_req = kMaxTile;
    return alloc_bins(p, kMaxTile);
}



}  // namespace nfft3

using namespace nfft3;

extern "C" {

int nfft3_plan(nfft3_plan_t *out, const int64_t N[3], double sigma, int m, int dtype, void *stream) {
    if (!out) return NFFT3_ERR_NULL;
    *out = nullptr;
    if (!N) return NFFT3_ERR_NULL;
    int64_t n[3];
    int rc = validate(N, sigma, m, dtype, n);
    if (rc) return rc;
    nfft3_plan_s *p = new (std::nothrow) nfft3_plan_s();
    if (!p) return NFFT3_ERR_OOM;
    p->dtype = dtype;
    p->m = m;
    p->sigma = sigma;
    p->b = M_PI * (2.0 - 1.0 / sigma);
    for (int d = 0; d < 3; ++d) {
        p->N[d] = N[d];
        p->n[d] = n[d];
        if (N[d] == 1) p->unit |= 1 << d;
    }
    p->stream = (hipStream_t)stream;
    p->elt = dtype == NFFT3_C128 ? 16 : 8;
    rc = build_plan(p);
    if (rc) {
        free_plan(p);
        delete p;
        return rc;
    }
    *out = p;
    return NFFT3_OK;
}

int nfft3_plan_nd(nfft3_plan_t *out, int d, const int64_t *N, double sigma, int m, int dtype, void *stream) {
    if (!out) return NFFT3_ERR_NULL;
    *out = nullptr;
    if (!N) return NFFT3_ERR_NULL;
    if (d < 1 || d > 3) return NFFT3_ERR_INVALID_ARG;
    int64_t N3[3] = {1, 1, 1};
    for (int i = 0; i < d; ++i) {
        if (N[i] < 2) return NFFT3_ERR_INVALID_ARG;     // unit axes are the padding only
        N3[3 - d + i] = N[i];
    }
    int rc = nfft3_plan(out, N3, sigma, m, dtype, stream);
    if (rc == NFFT3_OK) (*out)->dim = d;
    return rc;
}

int nfft3_set_stream(nfft3_plan_t p, void *stream) {
    if (!p) return NFFT3_ERR_NULL;
    p->stream = (hipStream_t)stream;
    return NFFT3_OK;
}

int nfft3_destroy(nfft3_plan_t p) {
    if (!p) return NFFT3_OK;
    if (p->stream) (void)hipStreamSynchronize(p->stream);
    free_plan(p);
    delete p;
    return NFFT3_OK;
}

// Points of a plan with dim < 3 coordinates: widened on the device to the
// (M, 3) layout of the kernels (0 on the unit axes) in the plan's xin.
static int widen(nfft3_plan_impl *p, int64_t M, const double **x) {
    if (p->dim == 3 || M == 0) return NFFT3_OK;
    if (M > p->cap_xin) {
        (void)hipFree(p->xin);
        p->xin = nullptr;
        p->cap_xin = 0;
        NFFT3_HIP_TRY(hipMalloc(&p->xin, sizeof(double) * 3 * M));
        p->cap_xin = M;
    }
    int rc = launch_widen_points(p->stream, M, p->dim, *x, p->xin);
    if (rc) return rc;
    *x = p->xin;
    return NFFT3_OK;
}

// a derivative mask over the plan's own axes -> over the three kernel axes
static int kernel_mask(const nfft3_plan_impl *p, int mask, int *out) {
    if (mask < 0 || mask >= (1 << p->dim)) return NFFT3_ERR_INVALID_ARG;
    *out = mask << (3 - p->dim);
    return NFFT3_OK;
}

int nfft3_set_points(nfft3_plan_t p, int64_t M, const double *x) {
    if (!p) return NFFT3_ERR_NULL;
    if (M < 0 || M > (int64_t)INT32_MAX) return NFFT3_ERR_INVALID_ARG;
    if (M > 0 && !x) return NFFT3_ERR_NULL;
    p->have_points = false;
    p->M = 0;
    if (M > p->cap_pts) {
        free_points(p);
        NFFT3_HIP_TRY(hipMalloc(&p->xs, sizeof(double) * 3 * M));
        NFFT3_HIP_TRY(hipMalloc(&p->perm, sizeof(int) * M));
        NFFT3_HIP_TRY(hipMalloc(&p->bin_of, sizeof(int) * M));
        NFFT3_HIP_TRY(hipMalloc(&p->rank, sizeof(int) * M));
        NFFT3_HIP_TRY(hipMalloc(&p->tx, sizeof(double) * 3 * M));
        NFFT3_HIP_TRY(hipMalloc(&p->tperm, sizeof(int) * M));
        NFFT3_HIP_TRY(hipMalloc(&p->tz, sizeof(int) * M));
        p->cap_pts = M;
    }
    const int64_t bases = two_level_bases(p, M);
    if (bases > p->chunk_base_cap) {
        (void)hipFree(p->chunk_base);
        (void)hipFree(p->sort_scratch);
        p->chunk_base = nullptr;
        p->sort_scratch = nullptr;
        p->chunk_base_cap = 0;
        NFFT3_HIP_TRY(hipMalloc(&p->chunk_base, sizeof(int) * (size_t)bases));
        NFFT3_HIP_TRY(hipMalloc(&p->sort_scratch, sizeof(int) * (size_t)(bases / 1024 + 2)));
        p->chunk_base_cap = bases;
    }
    int rc = widen(p, M, &x);
    if (rc) return rc;
    int flag = 0;
    rc = launch_set_points(p, M, x, &flag);
    if (rc) return rc;
    if (flag & 1) return NFFT3_ERR_NONFINITE;
    p->M = M;
    p->have_points = true;
    p->epoch += 1;
    return NFFT3_OK;
}

int nfft3_points_unchanged(nfft3_plan_t p, int64_t M, const double *x, int *unchanged) {
    if (!p || !unchanged) return NFFT3_ERR_NULL;
    *unchanged = 0;
    if (M < 0) return NFFT3_ERR_INVALID_ARG;
    if (!p->have_points || M != p->M) return NFFT3_OK;
    if (M > 0 && !x) return NFFT3_ERR_NULL;
    int rc = widen(p, M, &x);
    if (rc) return rc;
    return launch_points_equal(p, M, x, unchanged);
}

int nfft3_trafo(nfft3_plan_t p, const void *fhat, void *f) {
    if (!p) return NFFT3_ERR_NULL;
    if (!p->have_points) return NFFT3_ERR_NO_POINTS;
    if (!fhat || (p->M > 0 && !f)) return NFFT3_ERR_NULL;
    int rc = launch_grid_forward(p, fhat, p->grid, -1);
    if (rc) return rc;
    return launch_interp(p, p->grid, f);
}

int nfft3_trafo_fields(nfft3_plan_t p, const void *fhat, void *out, int mask) {
    if (!p) return NFFT3_ERR_NULL;
    if (!p->have_points) return NFFT3_ERR_NO_POINTS;
    int rc0 = kernel_mask(p, mask, &mask);
    if (rc0) return rc0;
    if (!fhat || (p->M > 0 && !out)) return NFFT3_ERR_NULL;
    if (p->dtype == NFFT3_C128 && mask != 0) {
        // FP64: the derivative fields through the window derivative, from
        // the one grid of the field (the window's derivative error stays
        // within the FP64 gates; in FP32 the rounding of the grid is
        // amplified ~n_d-fold by the derivative, so FP32 takes the spectral
        // route below: one grid per field)
        int rc = launch_grid_forward(p, fhat, p->grid, -1);
        if (rc) return rc;
        return launch_fields(p, p->grid, out, mask);
    }
    char *o = (char *)out;
    for (int field = -1; field < 3; ++field) {
        if (field >= 0 && !(mask & (1 << field))) continue;
        int rc = launch_grid_forward(p, fhat, p->grid, field);
        if (rc) return rc;
        rc = launch_interp(p, p->grid, o);
        if (rc) return rc;
        o += (size_t)p->M * p->elt;
    }
    return NFFT3_OK;
}

int nfft3_adjoint(nfft3_plan_t p, const void *f, void *fhat) {
    if (!p) return NFFT3_ERR_NULL;
    if (!p->have_points) return NFFT3_ERR_NO_POINTS;
    if (!fhat || (p->M > 0 && !f)) return NFFT3_ERR_NULL;
    const size_t total = (size_t)p->n[0] * p->n[1] * p->n[2];
    int rc = launch_zero(p, p->grid, total * p->elt);
    if (rc) return rc;
    rc = launch_spread(p, f, p->grid);
    if (rc) return rc;
    return launch_grid_adjoint(p, p->grid, fhat);
}

int nfft3_grad_points(nfft3_plan_t p, const void *fhat, const void *G, double *grad_x) {
    if (!p) return NFFT3_ERR_NULL;
    if (!p->have_points) return NFFT3_ERR_NO_POINTS;
    if (!fhat || (p->M > 0 && (!G || !grad_x))) return NFFT3_ERR_NULL;
    int rc = launch_grid_forward(p, fhat, p->grid, -1);
    if (rc) return rc;
    return launch_grad(p, p->grid, G, grad_x);
}

static int batch_common(int T, const nfft3_plan_t *plans, const void *const *fhat, void *const *out, int mask,
                        int form) {
    if (T < 0 || mask < 0 || mask > 7) return NFFT3_ERR_INVALID_ARG;
    if (T == 0) return NFFT3_OK;
    if (!plans || !fhat || !out) return NFFT3_ERR_NULL;
    for (int t = 0; t < T; ++t) {
        if (!plans[t] || !fhat[t]) return NFFT3_ERR_NULL;
        if (!plans[t]->have_points) return NFFT3_ERR_NO_POINTS;
        if (plans[t]->M > 0 && !out[t]) return NFFT3_ERR_NULL;
        if (plans[t]->dtype != plans[0]->dtype) return NFFT3_ERR_DTYPE;
        if (plans[t]->m != plans[0]->m || plans[t]->sigma != plans[0]->sigma || plans[t]->m > 8)
            return NFFT3_ERR_INVALID_ARG;
        if (plans[t]->device != plans[0]->device) return NFFT3_ERR_INVALID_ARG;
        if (plans[t]->unit) return NFFT3_ERR_INVALID_ARG;     // three-dimensional plans only
        for (int u = 0; u < t; ++u)
            if (plans[u] == plans[t]) return NFFT3_ERR_INVALID_ARG;
    }
    std::vector<nfft3_plan_impl *> pl(plans, plans + T);
    return launch_batch(T, pl.data(), fhat, out, mask, form);
}

int nfft3_batch_trafo(int T, const nfft3_plan_t *plans, const void *const *fhat, void *const *out, int mask) {
    return batch_common(T, plans, fhat, out, mask, kBatchLaunches);
}

int nfft3_batch_trafo_queue(int T, const nfft3_plan_t *plans, const void *const *fhat, void *const *out, int mask) {
    return batch_common(T, plans, fhat, out, mask, kBatchQueue);
}

int nfft3_batch_trafo_noalloc(int T, const nfft3_plan_t *plans, const void *const *fhat, void *const *out,
                              int mask) {
    return batch_common(T, plans, fhat, out, mask, kBatchNoAlloc);
}

const char *nfft3_strerror(int code) {
    switch (code) {
        case NFFT3_OK: return "ok";
        case NFFT3_ERR_INVALID_ARG: return "invalid argument";
        case NFFT3_ERR_DTYPE: return "unsupported or mismatched dtype";
        case NFFT3_ERR_OOM: return "device out of memory";
        case NFFT3_ERR_NO_POINTS: return "no points set on the plan";
        case NFFT3_ERR_NONFINITE: return "non-finite point coordinate";
        case NFFT3_ERR_HIP: return "HIP runtime error";
        case NFFT3_ERR_NULL: return "NULL plan or pointer";
        case NFFT3_ERR_CAPACITY: return "launch descriptors exceed the static scratch of the no-allocation call";
        case NFFT3_ERR_TIMEOUT: return "a work-queue wait exceeded its time limit (the batch was abandoned)";
        default: return "unknown status";
    }
}

const char *nfft3_last_hip_error(void) { return g_last_hip.c_str(); }

// ---- Gross-Pitaevskii time splitting (Sec. 3.1) --------------------------------

static void free_gpe(nfft3_gpe_impl *g) {
    for (int d = 0; d < 3; ++d) {
        (void)hipFree(g->fp.cdec[d]);
        (void)hipFree(g->fp.fft[d].tw);
        (void)hipFree(g->fp.fft[d].stw);
        g->fp.cdec[d] = g->fp.fft[d].tw = g->fp.fft[d].stw = nullptr;
    }
    (void)hipFree(g->state);
    (void)hipFree(g->work);
    g->state = g->work = nullptr;
}

static int build_gpe(nfft3_gpe_impl *g) {
    nfft3_plan_impl *p = &g->fp;
    const bool f64 = p->dtype == NFFT3_C128;
    NFFT3_HIP_TRY(hipGetDevice(&p->device));
    for (int d = 0; d < 3; ++d) {
        std::vector<double> ones((size_t)p->N[d], 1.0);
        int rc = f64 ? upload_real<double>(ones, &p->cdec[d]) : upload_real<float>(ones, &p->cdec[d]);
        if (rc) return rc;
        std::vector<int> rad;
        factor_radices((int)p->n[d], rad);
        p->fft[d].n = (int)p->n[d];
        p->fft[d].nrad = (int)rad.size();
        for (size_t i = 0; i < rad.size(); ++i) p->fft[d].radix[i] = rad[i];
        rc = f64 ? upload_twiddles<double>((int)p->n[d], &p->fft[d].tw)
                 : upload_twiddles<float>((int)p->n[d], &p->fft[d].tw);
        if (rc) return rc;
        rc = f64 ? upload_stage_twiddles<double>((int)p->n[d], &p->fft[d].stw)
                 : upload_stage_twiddles<float>((int)p->n[d], &p->fft[d].stw);
        if (rc) return rc;
    }
    const size_t bytes = (size_t)p->N[0] * p->N[1] * p->N[2] * p->elt;
    NFFT3_HIP_TRY(hipMalloc(&g->state, bytes));
    NFFT3_HIP_TRY(hipMalloc(&g->work, bytes));
    return NFFT3_OK;
}

int nfft3_gpe_create(nfft3_gpe_t *out, const int64_t N[3], const double a[3], const double b[3], int dtype,
                     void *stream) {
    if (!out) return NFFT3_ERR_NULL;
    *out = nullptr;
    if (!N || !a || !b) return NFFT3_ERR_NULL;
    if (dtype != NFFT3_C64 && dtype != NFFT3_C128) return NFFT3_ERR_DTYPE;
    for (int d = 0; d < 3; ++d) {
        std::vector<int> rad;
        // at least two radix stages per axis (the passes run in place)
        if (N[d] < 16 || N[d] > 2048 || N[d] % 2 || !factor_radices((int)N[d], rad)) return NFFT3_ERR_INVALID_ARG;
        if (!std::isfinite(a[d]) || !std::isfinite(b[d]) || !(b[d] > a[d])) return NFFT3_ERR_INVALID_ARG;
    }
    auto *g = new (std::nothrow) nfft3_gpe_s();
    if (!g) return NFFT3_ERR_OOM;
    g->fp.dtype = dtype;
    g->fp.elt = dtype == NFFT3_C128 ? 16 : 8;
    g->fp.sigma = 1.0;
    g->fp.stream = (hipStream_t)stream;
    for (int d = 0; d < 3; ++d) {
        g->fp.N[d] = g->fp.n[d] = N[d];
        g->len[d] = b[d] - a[d];
    }
    const int rc = build_gpe(g);
    if (rc) {
        free_gpe(g);
        delete g;
        return rc;
    }
    *out = g;
    return NFFT3_OK;
}

int nfft3_gpe_set_stream(nfft3_gpe_t g, void *stream) {
    if (!g) return NFFT3_ERR_NULL;
    g->fp.stream = (hipStream_t)stream;
    return NFFT3_OK;
}

int nfft3_gpe_set_state(nfft3_gpe_t g, const void *psi) {
    if (!g || !psi) return NFFT3_ERR_NULL;
    const size_t bytes = (size_t)g->fp.N[0] * g->fp.N[1] * g->fp.N[2] * g->fp.elt;
    NFFT3_HIP_TRY(hipMemcpyAsync(g->state, psi, bytes, hipMemcpyDeviceToDevice, g->fp.stream));
    return NFFT3_OK;
}

int nfft3_gpe_get_state(nfft3_gpe_t g, void *psi) {
    if (!g || !psi) return NFFT3_ERR_NULL;
    const size_t bytes = (size_t)g->fp.N[0] * g->fp.N[1] * g->fp.N[2] * g->fp.elt;
    NFFT3_HIP_TRY(hipMemcpyAsync(psi, g->state, bytes, hipMemcpyDeviceToDevice, g->fp.stream));
    return NFFT3_OK;
}

int nfft3_gpe_step(nfft3_gpe_t g, double tau, int nsteps) {
    if (!g) return NFFT3_ERR_NULL;
    if (nsteps < 0 || !std::isfinite(tau)) return NFFT3_ERR_INVALID_ARG;
    g->tau = tau;
    return launch_gpe_steps(g, nsteps);
}

int nfft3_gpe_coeffs(nfft3_gpe_t g, void *psihat) {
    if (!g || !psihat) return NFFT3_ERR_NULL;
    return launch_gpe_coeffs(g, psihat);
}

int nfft3_gpe_destroy(nfft3_gpe_t g) {
    if (!g) return NFFT3_OK;
    if (g->fp.stream) (void)hipStreamSynchronize(g->fp.stream);
    free_gpe(g);
    delete g;
    return NFFT3_OK;
}

// ---- the series on a physical domain (Sec. 2.2.1) and vortex tubes (Sec. 4.3)

static bool domain_ok(const double a[3], const double b[3]) {
    for (int d = 0; d < 3; ++d)
        if (!std::isfinite(a[d]) || !std::isfinite(b[d]) || !(b[d] > a[d])) return false;
    return true;
}

int nfft3_infft3(nfft3_plan_t p, const double a[3], const double b[3], const void *psihat, int64_t M, const double *xi,
                 void *psi) {
    if (!p || !a || !b || !psihat) return NFFT3_ERR_NULL;
    if (M < 0 || M > (int64_t)INT32_MAX / 3) return NFFT3_ERR_INVALID_ARG;
    if (M > 0 && (!xi || !psi)) return NFFT3_ERR_NULL;
    // a, b hold one entry per plan axis; unit axes take [0, 1)
    double a3[3] = {0.0, 0.0, 0.0}, b3[3] = {1.0, 1.0, 1.0};
    for (int i = 0; i < p->dim; ++i) {
        a3[3 - p->dim + i] = a[i];
        b3[3 - p->dim + i] = b[i];
    }
    if (!domain_ok(a3, b3)) return NFFT3_ERR_INVALID_ARG;
    return launch_infft3(p, a3, b3, psihat, M, xi, psi);
}

int nfft3_tube_refine(nfft3_plan_t p, const double a[3], const double b[3], const void *psihat, int levels,
                      const double *rhobar, int64_t cap, double *pts, double *rho, int64_t *count) {
    if (!p || !a || !b || !psihat || !count) return NFFT3_ERR_NULL;
    *count = 0;
    if (levels < 0 || levels > 16 || cap < 0) return NFFT3_ERR_INVALID_ARG;
    if (levels > 0 && !rhobar) return NFFT3_ERR_NULL;
    if (cap > 0 && (!pts || !rho)) return NFFT3_ERR_NULL;
    if (!domain_ok(a, b)) return NFFT3_ERR_INVALID_ARG;
    if (p->unit || p->dim != 3) return NFFT3_ERR_INVALID_ARG;     // the refinement grids are three-dimensional
    if (p->N[0] * p->N[1] * p->N[2] > (int64_t)INT32_MAX / 3) return NFFT3_ERR_INVALID_ARG;
    return launch_tube_refine(p, a, b, psihat, levels, rhobar, cap, pts, rho, count);
}

// ---- evaluation at a rectilinear grid (Sec. 2.1) ----------------------------

static void free_rgrid(nfft3_rgrid_impl *g) {
    for (int d = 0; d < 3; ++d) { (void)hipFree(g->E[d]); g->E[d] = nullptr; }
    (void)hipFree(g->t1); g->t1 = nullptr;
    (void)hipFree(g->t2); g->t2 = nullptr;
    (void)hipFree(g->flag); g->flag = nullptr;
}

int nfft3_rgrid_plan(nfft3_rgrid_t *out, const int64_t N[3], const int64_t M[3], int dtype, void *stream) {
    if (!out) return NFFT3_ERR_NULL;
    *out = nullptr;
    if (!N || !M) return NFFT3_ERR_NULL;
    if (dtype != NFFT3_C64 && dtype != NFFT3_C128) return NFFT3_ERR_DTYPE;
    for (int d = 0; d < 3; ++d) {
        // leading unit axes (N_d = M_d = 1): the two- and one-dimensional forms
        if (N[d] == 1 && M[d] == 1 && d < 2 && (d == 0 || N[0] == 1)) continue;
        if (N[d] < 2 || N[d] % 2 || N[d] > kRgridMaxN) return NFFT3_ERR_INVALID_ARG;
        if (M[d] < 1 || M[d] > kRgridMaxM) return NFFT3_ERR_INVALID_ARG;
    }
    auto *g = new (std::nothrow) nfft3_rgrid_s();
    if (!g) return NFFT3_ERR_OOM;
    g->dtype = dtype;
    g->elt = dtype == NFFT3_C128 ? 16 : 8;
    g->stream = (hipStream_t)stream;
    for (int d = 0; d < 3; ++d) { g->N[d] = N[d]; g->M[d] = M[d]; }
    int rc = NFFT3_OK;
    auto fail = [&](int code) { free_rgrid(g); delete g; return code; };
    hipError_t e = hipGetDevice(&g->device);
    if (e != hipSuccess) { set_hip_error(e, "hipGetDevice"); return fail(NFFT3_ERR_HIP); }
    const size_t sizes[5] = {(size_t)(M[0] * N[0]), (size_t)(M[1] * N[1]), (size_t)(N[2] * M[2]),
                             (size_t)(N[0] * N[1] * M[2]), (size_t)(N[0] * M[1] * M[2])};
    void **dst[5] = {&g->E[0], &g->E[1], &g->E[2], &g->t1, &g->t2};
    for (int i = 0; i < 5; ++i) {
        e = hipMalloc(dst[i], sizes[i] * g->elt);
        if (e != hipSuccess) {
            set_hip_error(e, "hipMalloc (rectilinear grid)");
            return fail(e == hipErrorOutOfMemory ? NFFT3_ERR_OOM : NFFT3_ERR_HIP);
        }
    }
    e = hipMalloc(&g->flag, 64);
    if (e != hipSuccess) { set_hip_error(e, "hipMalloc (flag)"); return fail(NFFT3_ERR_OOM); }
    (void)rc;
    *out = g;
    return NFFT3_OK;
}

int nfft3_rgrid_set_stream(nfft3_rgrid_t g, void *stream) {
    if (!g) return NFFT3_ERR_NULL;
    g->stream = (hipStream_t)stream;
    return NFFT3_OK;
}

int nfft3_rgrid_set_axes(nfft3_rgrid_t g, const double *y0, const double *y1, const double *y2) {
    if (!g) return NFFT3_ERR_NULL;
    // a unit axis reads no coordinate (its pointer may be NULL)
    if ((!y0 && !(g->N[0] == 1 && g->M[0] == 1)) || (!y1 && !(g->N[1] == 1 && g->M[1] == 1)) || !y2)
        return NFFT3_ERR_NULL;
    g->have_axes = false;
    const double *y[3] = {y0, y1, y2};
    int rc = launch_rgrid_axes(g, y);
    if (rc) return rc;
    int flag = 0;
    NFFT3_HIP_TRY(hipMemcpyAsync(&flag, g->flag, sizeof(int), hipMemcpyDeviceToHost, g->stream));
    NFFT3_HIP_TRY(hipStreamSynchronize(g->stream));
    if (flag & 1) return NFFT3_ERR_NONFINITE;
    g->have_axes = true;
    return NFFT3_OK;
}

int nfft3_rgrid_eval(nfft3_rgrid_t g, const void *fhat, void *out) {
    if (!g) return NFFT3_ERR_NULL;
    if (!g->have_axes) return NFFT3_ERR_NO_POINTS;
    if (!fhat || !out) return NFFT3_ERR_NULL;
    return launch_rgrid_eval(g, fhat, out);
}

int nfft3_rgrid_destroy(nfft3_rgrid_t g) {
    if (!g) return NFFT3_OK;
    if (g->stream) (void)hipStreamSynchronize(g->stream);
    free_rgrid(g);
    delete g;
    return NFFT3_OK;
}

int nfft3_set_tuning(nfft3_plan_t p, int tile, int items) {
    if (!p) return NFFT3_ERR_NULL;
    if (tile != 0 && (tile < 8 || tile > kMaxTile || tile % 4 != 0)) return NFFT3_ERR_INVALID_ARG;
    if (items != 0 && items != kItemPts && items != 2 * kItemPts) return NFFT3_ERR_INVALID_ARG;
    int cur_tile = 0, cur_items = 0;
    nfft3_get_tuning(p, &cur_tile, &cur_items);
    if (tile == 0) tile = cur_tile;
    if (items == 0) items = cur_items;
    if (tile == cur_tile && items == cur_items) return NFFT3_OK;
    NFFT3_HIP_TRY(hipStreamSynchronize(p->stream));
    p->have_points = false;
    p->M = 0;
    p->sub.maxpts = items;
    if (tile != cur_tile) {
        p->tile_req = tile;
        return alloc_bins(p, tile);
    }
    return NFFT3_OK;
}

int nfft3_get_tuning(nfft3_plan_t p, int *tile, int *items) {
    if (!p) return NFFT3_ERR_NULL;
    if (tile) *tile = p->tile_req;
    if (items) *items = p->sub.maxpts;
    return NFFT3_OK;
}

int nfft3_autotune(nfft3_plan_t p, int64_t M, const double *x, const void *fhat, void *f, int reps, int *tile_out,
                   int *items_out) {
    if (!p) return NFFT3_ERR_NULL;
    if (!fhat || (M > 0 && (!x || !f))) return NFFT3_ERR_NULL;
    if (reps < 1) return NFFT3_ERR_INVALID_ARG;
    const int tiles[] = {16, 24, 32};
    const int items[] = {kItemPts, 2 * kItemPts};
    hipEvent_t e0 = nullptr, e1 = nullptr;
    NFFT3_HIP_TRY(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return NFFT3_ERR_HIP;
    }
    int best_t = 0, best_i = 0, rc = NFFT3_OK;
    float best = 0.f;
    for (int t : tiles) {
        for (int it : items) {
            rc = nfft3_set_tuning(p, t, it);
            if (!rc) rc = nfft3_set_points(p, M, x);
            if (!rc) rc = nfft3_trafo(p, fhat, f);     // warm-up
            std::vector<float> ms;
            for (int r = 0; r < reps && !rc; ++r) {
                if (hipEventRecord(e0, p->stream) != hipSuccess) { rc = NFFT3_ERR_HIP; break; }
                rc = nfft3_trafo(p, fhat, f);
                if (rc) break;
                if (hipEventRecord(e1, p->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
                    rc = NFFT3_ERR_HIP;
                    break;
                }
                float v = 0.f;
                if (hipEventElapsedTime(&v, e0, e1) != hipSuccess) { rc = NFFT3_ERR_HIP; break; }
                ms.push_back(v);
            }
            if (rc) break;
            std::sort(ms.begin(), ms.end());
            const float med = ms[ms.size() / 2];
            if (best_t == 0 || med < best) { best = med; best_t = t; best_i = it; }
        }
        if (rc) break;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    rc = nfft3_set_tuning(p, best_t, best_i);
    if (!rc) rc = nfft3_set_points(p, M, x);
    if (rc) return rc;
    if (tile_out) *tile_out = best_t;
    if (items_out) *items_out = best_i;
    return NFFT3_OK;
}

int nfft3_get_info(nfft3_plan_t p, int64_t n_out[3], int64_t *M_out) {
    if (!p) return NFFT3_ERR_NULL;
    if (n_out)
        for (int d = 0; d < 3; ++d) n_out[d] = p->n[d];
    if (M_out) *M_out = p->have_points ? p->M : 0;
    return NFFT3_OK;
}

int nfft3_stage_grid(nfft3_plan_t p, const void *fhat, int deriv_axis) {
    if (!p) return NFFT3_ERR_NULL;
    if (!fhat) return NFFT3_ERR_NULL;
    if (deriv_axis < -1 || deriv_axis > 2) return NFFT3_ERR_INVALID_ARG;
    return launch_grid_forward(p, fhat, p->grid, deriv_axis);
}

int nfft3_stage_interp(nfft3_plan_t p, void *f) {
    if (!p) return NFFT3_ERR_NULL;
    if (!p->have_points) return NFFT3_ERR_NO_POINTS;
    if (p->M > 0 && !f) return NFFT3_ERR_NULL;
    return launch_interp(p, p->grid, f);
}

int nfft3_stage_spread(nfft3_plan_t p, const void *f) {
    if (!p) return NFFT3_ERR_NULL;
    if (!p->have_points) return NFFT3_ERR_NO_POINTS;
    if (p->M > 0 && !f) return NFFT3_ERR_NULL;
    const size_t total = (size_t)p->n[0] * p->n[1] * p->n[2];
    int rc = launch_zero(p, p->grid, total * p->elt);
    if (rc) return rc;
    return launch_spread(p, f, p->grid);
}

int nfft3_grid_copy(nfft3_plan_t p, void *buf, int to_plan) {
    if (!p) return NFFT3_ERR_NULL;
    if (!buf) return NFFT3_ERR_NULL;
    const size_t bytes = (size_t)p->n[0] * p->n[1] * p->n[2] * p->elt;
    if (to_plan)
        NFFT3_HIP_TRY(hipMemcpyAsync(p->grid, buf, bytes, hipMemcpyDeviceToDevice, p->stream));
    else
        NFFT3_HIP_TRY(hipMemcpyAsync(buf, p->grid, bytes, hipMemcpyDeviceToDevice, p->stream));
    return NFFT3_OK;
}

int nfft3_deconv_factors(int64_t Nd, double sigma, int m, double *c) {
    if (!c) return NFFT3_ERR_NULL;
    if (Nd < 2 || Nd % 2 || !(sigma > 1.0) || m < 1 || m > 10) return NFFT3_ERR_INVALID_ARG;
    double nd = sigma * (double)Nd;
    deconv_factors(Nd, (int64_t)llround(nd), m, M_PI * (2.0 - 1.0 / sigma), c);
    return NFFT3_OK;
}

int nfft3_window_poly(int m, double sigma, int dtype, int cap_deg, double *coef, int *deg) {
    if (!coef || !deg) return NFFT3_ERR_NULL;
    if (m < 1 || m > 10 || !(sigma > 1.0) || cap_deg < 2) return NFFT3_ERR_INVALID_ARG;
    if (dtype != NFFT3_C64 && dtype != NFFT3_C128) return NFFT3_ERR_DTYPE;
    std::vector<double> c;
    double b = M_PI * (2.0 - 1.0 / sigma);
    int d = window_poly(m, b, dtype == NFFT3_C128 ? 4e-16 : 2e-8, std::min(cap_deg, kMaxDeg), c);
    if (d < 0) d = window_poly(m, b, dtype == NFFT3_C128 ? 2e-15 : 1e-7, std::min(cap_deg, kMaxDeg), c);
    if (d < 0) return NFFT3_ERR_INVALID_ARG;
    memcpy(coef, c.data(), sizeof(double) * c.size());
    *deg = d;
    return NFFT3_OK;
}

}  // extern "C"
