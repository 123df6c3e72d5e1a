// Internal declarations shared by the translation units of libnfft3.
// Device code targets gfx950 (CDNA4): 64-lane wavefronts, 160 KiB LDS per CU.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/nfft3.h"

namespace nfft3 {

// ----------------------------------------------------------------------------
// Complex helpers.  Complex values are the HIP vector types float2 / double2
// (interleaved re, im), so a complex load is one 8- or 16-byte access.
// ----------------------------------------------------------------------------
template <typename T> struct cplx;
template <> struct cplx<float> { using type = float2; };
template <> struct cplx<double> { using type = double2; };
template <typename T> using c_t = typename cplx<T>::type;

template <typename T>
__device__ __forceinline__ c_t<T> cmk(T re, T im) { c_t<T> r; r.x = re; r.y = im; return r; }
template <typename C>
__device__ __forceinline__ C cadd(C a, C b) { a.x += b.x; a.y += b.y; return a; }
template <typename C>
__device__ __forceinline__ C csub(C a, C b) { a.x -= b.x; a.y -= b.y; return a; }
template <typename C>
__device__ __forceinline__ C cmul(C a, C b) {
    C r;
    r.x = a.x * b.x - a.y * b.y;
    r.y = a.x * b.y + a.y * b.x;
    return r;
}
// a * conj(b)
template <typename C>
__device__ __forceinline__ C cmulc(C a, C b) {
    C r;
    r.x = a.x * b.x + a.y * b.y;
    r.y = a.y * b.x - a.x * b.y;
    return r;
}

// ----------------------------------------------------------------------------
// Window polynomials: for stencil offset index r (0..2m-1) and cell fraction
// f in [0,1), w_r(f) = sum_q coef[r*(deg+1)+q] y^q, y = 2f - 1.
// ----------------------------------------------------------------------------
constexpr int kMaxM = 16;
constexpr int kMaxDeg = 24;

// ----------------------------------------------------------------------------
// Plan
// ----------------------------------------------------------------------------
struct FftAxisPlan {
    int n = 0;                // transform length
    int nrad = 0;             // number of radix stages
    int radix[16] = {0};      // radices in application order
    void *tw = nullptr;       // device twiddles exp(-2 pi i k/n), k = 0..n-1 (c_t<T>)
    void *stw = nullptr;      // per-stage twiddle tables of the compile-time engine (st_tw_offset)
};

// Radix plan of a length n = 2^a 3^b 5^c 7^d, in application order: radix-8
// stages, then one radix-4 or radix-2 stage for a mod 3 = 2 or 1 (two
// radix-4 stages instead of 8 x 2 when a mod 3 = 1 and a >= 4), then the
// radix-3, radix-5 and radix-7 stages.  The host's FFT plans and the
// compile-time engine both use it.
constexpr int st_nrad(int n) {
    int a = 0;
    while (n % 2 == 0) { n /= 2; ++a; }
    int q = a / 3, r = a % 3, c = 0;
    if (r == 1 && q > 0) { q -= 1; r = 4; }
    c = q + (r == 4 ? 2 : (r ? 1 : 0));
    while (n % 3 == 0) { n /= 3; ++c; }
    while (n % 5 == 0) { n /= 5; ++c; }
    while (n % 7 == 0) { n /= 7; ++c; }
    return n == 1 ? c : -1;
}
constexpr int st_radix(int n, int s) {
    int a = 0;
    while (n % 2 == 0) { n /= 2; ++a; }
    int q = a / 3, r = a % 3;
    if (r == 1 && q > 0) { q -= 1; r = 4; }
    if (s < q) return 8;
    s -= q;
    if (r == 4) { if (s < 2) return 4; s -= 2; }
    else if (r == 2) { if (s < 1) return 4; s -= 1; }
    else if (r == 1) { if (s < 1) return 2; s -= 1; }
    int b = 0, c = 0;
    while (n % 3 == 0) { n /= 3; ++b; }
    while (n % 5 == 0) { n /= 5; ++c; }
    return s < b ? 3 : (s < b + c ? 5 : 7);
}
// product of the radices before stage s (the Stockham span Ns)
constexpr int st_ns(int n, int s) {
    int ns = 1;
    for (int i = 0; i < s; ++i) ns *= st_radix(n, i);
    return ns;
}
// Stage s >= 1 twiddles of the compile-time engine: entry [k * 8 + r] =
// exp(-2 pi i r k / (Ns R)), k < Ns, r < R; this is the offset of stage s's
// table.
constexpr int st_tw_offset(int n, int s) {
    int off = 0;
    for (int i = 1; i < s; ++i) off += st_ns(n, i) * 8;
    return off;
}
constexpr int st_tw_size(int n) { return st_nrad(n) > 0 ? st_tw_offset(n, st_nrad(n)) : 0; }

// Points are sorted by (tile, z-cell); a tile is By x Bx cells of the (y, x)
// plane.  Work items for the window-sum kernels are at most Subproblems::maxpts
// points (a multiple of the kItemPts threads of a workgroup) of one tile
// column spanning at most kItemZ z-cells.
constexpr int kItemPts = 256;
constexpr int kItemZ = 64;
constexpr int kMaxPlane = 12 * kItemPts;   // staged plane elements per workgroup
constexpr int kMaxTile = 32;               // By, Bx never exceed this
// The counting sort keeps kBinCopies counters per (tile, z) bin, interleaved
// (bin b, copy c at b kBinCopies + c), a workgroup using copy blockIdx mod
// kBinCopies: clustered points send hundreds of atomic increments to the same
// bins, and spreading them over copies divides that contention (8 copies ran
// the binning of 1e7 clustered points 24% slower than 32).  Each point's rank
// is within its copy; the scan over all counters keeps a bin's copies
// contiguous, so a bin still owns one contiguous range of sorted points.
constexpr int kBinCopies = 32;

struct Bins {
    int By = 32, Bx = 32;     // tile size in cells (y, x)
    int nty = 0, ntx = 0;     // tiles per axis
    int64_t nbins = 0;        // nty * ntx * n0
    int *counts = nullptr;    // point counts, kBinCopies counters per bin (single-level sort) or one (two-level) (device)
    int *offsets = nullptr;   // exclusive scan of counts: bin starts (device)
    int *scratch = nullptr;   // block sums of the scans
    int *tile_counts = nullptr;     // two-level sort: points (then level-2 chunks) per tile
    int *tile_start = nullptr;      // exclusive scan of the points per tile, ntiles + 1
    int *chunk_start = nullptr;     // exclusive scan of the chunks per tile, ntiles + 1
    int *tile_items = nullptr;      // items per (tile, segment of kItemZ z-cells) (device)
    int *tile_item_off = nullptr;   // exclusive scan of tile_items, one more entry (device)
};

struct Subproblems {
    int maxpts = 1024;        // points per item at most (points per thread x 256)
    int64_t count = 0;        // number of work items
    int4 *items = nullptr;    // (tile, first sorted index, end sorted index, 0) (device)
    int64_t cap = 0;
};

// Scratch of the physical-domain calls (infftm.hip), grown as needed.
struct InfftmScratch {
    void *zeta = nullptr;  int64_t zeta_cap = 0;   // mapped points (doubles)
    void *fhat = nullptr;  int64_t fhat_cap = 0;   // signed, scaled coefficients (elements)
    void *pts = nullptr;   int64_t pts_cap = 0;    // tube: current points (doubles)
    void *pts2 = nullptr;  int64_t pts2_cap = 0;   // tube: refined points (doubles)
    void *psi = nullptr;   int64_t psi_cap = 0;    // tube: values (elements)
    void *rho = nullptr;   int64_t rho_cap = 0;    // tube: |psi|^2 (doubles)
    void *keep = nullptr;  int64_t keep_cap = 0;   // tube: flags and their scan (int pairs)
    void *sums = nullptr;  int64_t sums_cap = 0;   // tube: block sums of the scan (ints)
};

struct nfft3_plan_impl {
    int dtype = NFFT3_C128;
    int m = 8;
    double sigma = 2.0;
    double b = 0.0;
    int64_t N[3] = {0, 0, 0};
    int64_t n[3] = {0, 0, 0};
    hipStream_t stream = nullptr;
    int device = 0;
    size_t elt = 16;          // bytes per complex element
    // Lower-dimensional transforms: a plan of d < 3 axes is the 3-D plan with
    // 3 - d leading unit axes (N = n = 1: frequency 0 only, so the sum over
    // such an axis is exact and needs no window).  dim = coordinates per
    // caller point; unit bit d = axis d is a unit axis.
    int dim = 3;
    int unit = 0;
    double *xin = nullptr;    // dim < 3: caller points widened to (M,3)
    int64_t cap_xin = 0;

    void *grid = nullptr;     // n0 n1 n2 complex
    std::vector<void *> extra_grids;   // batched derivative fields
    void *cdec[3] = {nullptr, nullptr, nullptr};   // deconvolution factors (real T)
    FftAxisPlan fft[3];
    void *wcoef = nullptr;    // window polynomial coefficients (real T), 2m*(deg+1)
    int deg = 0;

    // points
    int64_t M = 0;
    bool have_points = false;
    int64_t cap_pts = 0;
    double *xs = nullptr;     // sorted folded points, (M,3)
    int *perm = nullptr;      // sorted position -> caller index
    int *bin_of = nullptr;    // per caller index: bin id / rank in tile (scratch)
    int *rank = nullptr;      // rank inside bin (scratch)
    double *tx = nullptr;     // two-level sort: folded points in tile order (scratch, (M,3))
    int *tperm = nullptr;     // two-level sort: caller index in tile order (scratch)
    int *tz = nullptr;        // two-level sort: z-cell in tile order (scratch)
    int *chunk_base = nullptr;      // two-level sort: runs per (chunk, key) (scratch)
    int *sort_scratch = nullptr;    // two-level sort: block sums of the run scan
    int64_t chunk_base_cap = 0;
    int *flag = nullptr;      // device status word (non-finite points)
    Bins bins;
    int tile_req = kMaxTile;  // requested tile edge (By, Bx may be smaller)
    Subproblems sub;
    int64_t epoch = 0;        // bumps at every set_points
    InfftmScratch infftm;     // nfft3_infft3 / nfft3_tube_refine
};

// Evaluation at a rectilinear grid (Sec. 2.1): three complex matrix products.
constexpr int64_t kRgridMaxN = 1 << 14;   // coefficients per axis
constexpr int64_t kRgridMaxM = 1 << 20;   // grid points per axis
struct nfft3_rgrid_impl {
    int dtype = NFFT3_C128;
    int64_t N[3] = {0, 0, 0};   // coefficients
    int64_t M[3] = {0, 0, 0};   // grid points per axis
    hipStream_t stream = nullptr;
    int device = 0;
    size_t elt = 16;
    void *E[3] = {nullptr, nullptr, nullptr};   // E0 (M0 x N0), E1 (M1 x N1), E2^T (N2 x M2)
    void *t1 = nullptr;         // N0 N1 M2 (after the sum over k2)
    void *t2 = nullptr;         // N0 M1 M2 (after the sum over k1)
    int *flag = nullptr;        // device status word (non-finite coordinates)
    bool have_axes = false;
};

// Gross-Pitaevskii time splitting (gpe.hip): an FFT-only plan (n = N, unit
// deconvolution factors) whose grid passes transform the state in place.
struct nfft3_gpe_impl {
    nfft3_plan_impl fp;
    void *state = nullptr;      // psi on X_N (N0 N1 N2 complex, C order)
    void *work = nullptr;       // coefficient output scratch
    double tau = 0.0;
    double len[3] = {0, 0, 0};  // b_d - a_d
};

// Raise a kernel's dynamic-LDS limit above the 64 KiB default when needed.
void allow_lds(const void *kernel, size_t bytes);

// error helpers ---------------------------------------------------------------
void set_hip_error(hipError_t e, const char *where);
#define NFFT3_HIP_TRY(expr)                                              \
    do {                                                                 \
        hipError_t _e = (expr);                                          \
        if (_e != hipSuccess) {                                          \
            ::nfft3::set_hip_error(_e, #expr);                           \
            return (_e == hipErrorOutOfMemory) ? NFFT3_ERR_OOM : NFFT3_ERR_HIP; \
        }                                                                \
    } while (0)
#define NFFT3_LAUNCH_CHECK(where)                                        \
    do {                                                                 \
        hipError_t _e = hipGetLastError();                               \
        if (_e != hipSuccess) {                                          \
            ::nfft3::set_hip_error(_e, where);                           \
            return NFFT3_ERR_HIP;                                        \
        }                                                                \
    } while (0)

// host-side tables (api.hip) ---------------------------------------------------
double bessel_i0(double x);
void deconv_factors(int64_t Nd, int64_t nd, int m, double b, double *c);
int window_poly(int m, double b, double tol, int cap_deg, std::vector<double> &coef);
bool factor_radices(int n, std::vector<int> &rad);

// stage launchers ---------------------------------------------------------------
// FFT (fft.hip)
int launch_grid_forward(nfft3_plan_impl *p, const void *fhat, void *grid, int deriv_axis);
int launch_grid_adjoint(nfft3_plan_impl *p, void *grid, void *fhat);
// points (points.hip)
// sorts the points and cuts the work items; *flag = the device status word
// (bit 0: a non-finite coordinate).  Synchronises the plan's stream once.
int launch_set_points(nfft3_plan_impl *p, int64_t M, const double *x, int *flag);
// chunk bases the two-level sort needs for M points, -1 if it is not used
int64_t two_level_bases(const nfft3_plan_impl *p, int64_t M);
// *equal = 1 when the sorted points are those of x (no new sort needed)
int launch_widen_points(hipStream_t s, int64_t M, int dim, const double *x, double *x3);
int launch_points_equal(nfft3_plan_impl *p, int64_t M, const double *x, int *equal);
// window sums and their point derivative (interp.hip)
int launch_interp(nfft3_plan_impl *p, const void *grid, void *f);
int launch_grad(nfft3_plan_impl *p, const void *grid, const void *G, double *grad_x);
// complex<double> only: the field and the derivative fields of mask from one grid
int launch_fields(nfft3_plan_impl *p, const void *grid, void *out, int mask);
// spreading, the adjoint window step, and the grid fill (spread.hip)
int launch_spread(nfft3_plan_impl *p, const void *f, void *grid);
int launch_zero(nfft3_plan_impl *p, void *buf, size_t bytes);
// batch (batch.hip)
// forms of the batch: per-length launches (descriptors in a library buffer or
// in the static array), or one work-queue launch
enum { kBatchLaunches = 0, kBatchNoAlloc = 1, kBatchQueue = 2 };
int launch_batch(int T, nfft3_plan_impl *const *plans, const void *const *fhat, void *const *out,
                 int deriv_mask, int form);

// exclusive scan of n ints (in -> out, out[n] = total; in place allowed);
// sums holds ceil(n / 1024) ints (points.hip)
int launch_exclusive_scan(hipStream_t s, const int *in, int *out, int *sums, int64_t n);
// physical domain and vortex tubes (infftm.hip)
int launch_infft3(nfft3_plan_impl *p, const double a[3], const double b[3], const void *psihat, int64_t M,
                  const double *xi, void *psi);
int launch_tube_refine(nfft3_plan_impl *p, const double a[3], const double b[3], const void *psihat, int levels,
                       const double *rhobar, int64_t cap, double *pts, double *rho, int64_t *count);
void free_infftm(nfft3_plan_impl *p);
// GPE time splitting (gpe.hip)
int launch_gpe_steps(nfft3_gpe_impl *g, int nsteps);
int launch_gpe_coeffs(nfft3_gpe_impl *g, void *psihat);
// rectilinear grid (rgrid.hip)
int launch_rgrid_axes(nfft3_rgrid_impl *g, const double *const y[3]);
int launch_rgrid_eval(nfft3_rgrid_impl *g, const void *fhat, void *out);

}  // namespace nfft3

struct nfft3_plan_s : nfft3::nfft3_plan_impl {};
struct nfft3_rgrid_s : nfft3::nfft3_rgrid_impl {};
struct nfft3_gpe_s : nfft3::nfft3_gpe_impl {};
