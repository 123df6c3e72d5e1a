// Adjoint window step (spreading), the transpose of the window sums:
//   g[(u_j + r) mod n] += f_j prod_d w_d(r_d),  r in {-m+1..m}^3,
// over the same work items (points sorted by (tile, z-cell)) and the same
// plane walk as the window sums (interp.hip): each plane's tile region plus
// halo is accumulated in LDS and then added to the grid, whose halo cells
// neighbouring items share, with global atomics.
#include "interp_dev.h"

namespace nfft3 {

// The plane accumulator in LDS holds 64-bit fixed-point values: on gfx950 an
// LDS float atomic add runs ~15x slower than an LDS 64-bit integer atomic
// add (measured), whatever the address pattern.  A chunk of at most 512
// points (PPT per thread; slot k of thread t is sorted index lo + k 256 + t)
// is accumulated at scale 2^k, k = 53 - e with max|f| < 2^e, so every
// contribution |f w0 w1 w2| 2^k (window values <= 1) is below 2^53 and any
// sum of at most 512 of them stays below 2^62.  A contribution p = a b is
// rounded to the nearest integer by three fused multiply-adds and integer
// adds, without conversion instructions.  With C = 1.5 2^52 the doubles in
// [2^52, 2^53] are the integers and adjacent doubles have adjacent bit
// patterns, so y = fma(a, b/4, C) holds q1 = rint(p/4) as bits(y) - bits(C)
// (|p/4| < 2^51; C's low word is zero, so only the high word is adjusted);
// fma(y, -4, 5C) = C - 4 q1 exactly; z = fma(a, b, C - 4 q1) holds
// rint(p - 4 q1), |.| <= 2, in its low word; and rint(p) = 4 q1 +
// rint(p - 4 q1), with one rounding of the exact product.  The error is at
// most 2^(e-54), half an FP64 ulp of the chunk's largest value (2^-53 max|f|
// up to the 1.0001 margin on the scale).  The largest value is taken in f's
// own precision, so any finite range works (1e-300 and 1e300 alike); NaN and
// infinite values are kept out of the sums and turn the result into NaN.  Each plane is flushed once per
// chunk: converted back (exact power-of-two scaling) and added to the grid
// with global atomics, whose rate bounds the kernel when a 512-point item is
// taken in two chunks, hence two points per thread (one walk and one flush
// per item) where the registers allow.
__device__ __forceinline__ unsigned long long fixed_fma(double a, double b4, double b) {
    constexpr double C = 6755399441055744.0;          // 1.5 2^52
    const double y = __fma_rn(a, b4, C);              // C + q1, q1 = rint(a b / 4)
    const double t = __fma_rn(y, -4.0, 5.0 * C);      // C - 4 q1 (exact)
    const double z = __fma_rn(a, b, t);               // C + rint(a b - 4 q1), |.| <= 2
    const unsigned hi = (unsigned)__double2hiint(y) - 0x43380000u;
    const unsigned long long q1 = ((unsigned long long)hi << 32) | (unsigned)__double2loint(y);
    return (q1 << 2) + (unsigned long long)(long long)__double2loint(z);
}

template <typename T, int W, int PPT>
__global__ void __launch_bounds__(kPsThreads) spread_ps_kernel(PSArgs a) {
    constexpr int m = W / 2;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ T wmax[kPsThreads / 64];
    const int4 item = a.items[xcd_item(blockIdx.x, gridDim.x)];
    for (int lo = item.y; lo < item.z; lo += kPsThreads * PPT) {
    __syncthreads();
    const int hi = min(item.z, lo + kPsThreads * PPT);
    const PSItem it = ps_range(a, m, item.x, lo, hi);
    unsigned long long *acc = reinterpret_cast<unsigned long long *>(smem_raw);   // (re, im) per element
    T *scoef = reinterpret_cast<T *>(acc + 2 * it.psz);
    const T *coef = (const T *)a.coef;
    const int nc = W * (a.deg + 1);
    for (int i = threadIdx.x; i < nc; i += kPsThreads) scoef[i] = coef[i];
    for (int e = threadIdx.x; e < 2 * it.psz; e += kPsThreads) acc[e] = 0ull;

    // W = 16: lane l of each 16-lane group walks its stencil rows starting at
    // row t, chosen so that all its atomics fall in bank group l mod 16
    // offset by a step-dependent constant.  Element e's 16-byte bank group is
    // e mod 16; at step (j, r2) a lane adds to element c + ((j + t) mod 16) PX
    // + r2 (c its stencil's first element), which is c + t PX + j PX + r2 mod
    // 16; the region's row length PX = B + 2m - 1 is odd, hence invertible
    // mod 16, and t = (l - c) PX^-1 mod 16 makes c + t PX = l.  The row
    // weights are rotated with the rows, once per point.
    constexpr bool ROT = W == 16;
    const int pxinv = (it.PX * (2 - it.PX * it.PX)) & 15;   // PX^-1 mod 16
    T w1[PPT][W], w2[PPT][W];
    T f0[PPT];
    int zlo[PPT], base[PPT], rot[PPT];
    c_t<T> v[PPT];
    T amax = 0;             // the chunk's largest |Re f|, |Im f|, in f's precision
    bool bad = false;       // a NaN or infinite value in the chunk
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        const int pk = lo + k * kPsThreads + threadIdx.x;
        f0[k] = 0;
        zlo[k] = -4 * W;     // never active
        base[k] = 0;
        rot[k] = 0;
        v[k] = cmk<T>(0, 0);
#pragma unroll
        for (int r = 0; r < W; ++r) { w1[k][r] = 0; w2[k][r] = 0; }
        if (pk < hi) {
            const double *xp = a.xs + 3 * (int64_t)pk;
            T f1, f2;
            const int zc = cell_frac<T>(xp[0], a.n0, f0[k]);
            const int yc = cell_frac<T>(xp[1], a.n1, f1);
            const int xc = cell_frac<T>(xp[2], a.n2, f2);
            zlo[k] = (a.unit & 1) ? 0 : zc - m + 1 - it.zbeg;
            base[k] = 2 * ((yc - it.y0) * it.PX + (xc - it.x0));
            window_weights<T, W>(f1, coef, a.deg, w1[k]);
            window_weights<T, W>(f2, coef, a.deg, w2[k]);
            if (a.unit & 2) {   // unit axis 1: every region row is grid row 0; weight 1 on one
#pragma unroll
                for (int r = 0; r < W; ++r) w1[k][r] = r == 0 ? (T)1 : (T)0;
            }
            if constexpr (ROT) {
                rot[k] = (((int)(threadIdx.x & 15) - (base[k] >> 1)) * pxinv) & 15;
                rotate_rows<T, W, 16>(w1[k], rot[k]);
            }
            v[k] = ((const c_t<T> *)a.vals)[a.perm[pk]];
            if (!isfinite(v[k].x) || !isfinite(v[k].y)) {
                bad = true;
                v[k] = cmk<T>(0, 0);
            }
            amax = fmax(amax, fmax(fabs(v[k].x), fabs(v[k].y)));
        }
    }
    // chunk scale 2^ks: 2^ks max|f| < 2^53
    for (int off = 32; off > 0; off >>= 1) amax = fmax(amax, __shfl_xor(amax, off));
    if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = amax;
    constexpr int NF = ps_nf<W>();
    int off[NF], lidx[NF];
    ps_offsets<NF>(a, it, m, off, lidx);
    c_t<T> *grid = (c_t<T> *)a.grid_out;
    const int64_t plane = (int64_t)a.n1 * a.n2;
    const bool chunk_bad = __syncthreads_or(bad);
    T bmax = 0;
#pragma unroll
    for (int w = 0; w < kPsThreads / 64; ++w) bmax = fmax(bmax, wmax[w]);
    // 2^ex > 1.0001 bmax (the margin covers window values a rounding above
    // 1), taken without forming 1.0001 bmax, which could overflow
    int ex = 0;
    if (bmax > 0) {
        const double mant = frexp((double)bmax, &ex);   // bmax = mant 2^ex, mant in [1/2, 1)
        if (mant * 1.0001 >= 1.0) ++ex;
    }
    const int ks = 53 - ex;
    double vr0[PPT], vi0[PPT];
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        vr0[k] = ldexp((double)v[k].x, ks);
        vi0[k] = ldexp((double)v[k].y, ks);
    }

    for (int i = 0; i < it.nplanes; ++i) {
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            const int r0 = i - zlo[k];
            if (r0 >= 0 && r0 < W) {
                const double w0 = (a.unit & 1) ? 1.0 : (double)piece<T>(scoef + r0 * (a.deg + 1), a.deg, f0[k]);
                const double vr = w0 * vr0[k], vi = w0 * vi0[k];
                for (int r1 = 0; r1 < W; ++r1) {
                    const int rr = ROT ? (r1 + rot[k]) & 15 : r1;
                    unsigned long long *row = acc + base[k] + 2 * rr * it.PX;
                    const double br = (double)w1[k][r1] * vr, bi = (double)w1[k][r1] * vi;
                    const double br4 = 0.25 * br, bi4 = 0.25 * bi;
#pragma unroll
                    for (int r2 = 0; r2 < W; ++r2) {
                        const double w2d = (double)w2[k][r2];
                        atomicAdd(&row[2 * r2], fixed_fma(w2d, br4, br));
                        atomicAdd(&row[2 * r2 + 1], fixed_fma(w2d, bi4, bi));
                    }
                }
            }
        }
        __syncthreads();
        // flush this plane to the grid and clear it
        const int64_t zoff = (int64_t)wrapi(it.zbeg + i, a.n0) * plane;
#pragma unroll
        for (int kk = 0; kk < NF; ++kk) {
            const int e = threadIdx.x + kk * kPsThreads;
            if (e < it.psz) {
                const long long sr = (long long)acc[2 * e], si = (long long)acc[2 * e + 1];
                if (sr != 0 || si != 0) {
                    unsafeAtomicAdd(&grid[zoff + off[kk]].x, (T)ldexp((double)sr, -ks));
                    unsafeAtomicAdd(&grid[zoff + off[kk]].y, (T)ldexp((double)si, -ks));
                    acc[2 * e] = 0ull;
                    acc[2 * e + 1] = 0ull;
                }
            }
        }
        __syncthreads();
    }
    // A NaN or infinite value was left out of the fixed-point sums; one NaN
    // in the grid makes every coefficient of the adjoint NaN (the adjoint FFT
    // sums every grid value into every coefficient), as the arithmetic would.
    if (chunk_bad && threadIdx.x == 0)
        unsafeAtomicAdd(&grid[(int64_t)wrapi(it.zbeg, a.n0) * plane + off[0]].x, (T)NAN);
    }
}

__global__ void zero_kernel(float4 *p, int64_t count) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = make_float4(0.f, 0.f, 0.f, 0.f);
}

int launch_zero(nfft3_plan_impl *p, void *buf, size_t bytes) {
    const int64_t count = (int64_t)(bytes / 16);
    if (count == 0) return NFFT3_OK;
    hipLaunchKernelGGL(zero_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, p->stream,
                       (float4 *)buf, count);
    NFFT3_LAUNCH_CHECK("zero_kernel");
    return NFFT3_OK;
}

// ------------------------------------------------------------ dispatch ----
template <typename T, int W>
static int spread_w(nfft3_plan_impl *p, const void *f, void *grid) {
    if (p->M == 0 || p->sub.count == 0) return NFFT3_OK;
    PSArgs a = ps_args(p);
    a.vals = f;
    a.grid_out = grid;
    // 16 bytes (two 64-bit fixed-point values) per staged element + the coefficients
    const size_t psz = (size_t)(p->bins.By + W - 1) * (p->bins.Bx + W - 1);
    const size_t lds = psz * 16 + (size_t)W * (p->deg + 1) * sizeof(T);
    // Two points per thread (complex<float> up to m = 4, complex<double> up
    // to m = 8): a 512-point item is walked and flushed once, not twice; the
    // global-atomic flush of every plane otherwise bounds the kernel.  Wider
    // complex<float> stencils keep one (registers).
    constexpr int PPT = (sizeof(T) == 4 ? W <= 8 : W <= 16) ? 2 : 1;
    allow_lds((const void *)spread_ps_kernel<T, W, PPT>, lds);
    hipLaunchKernelGGL((spread_ps_kernel<T, W, PPT>), dim3((unsigned)p->sub.count), dim3(kPsThreads), lds,
                       p->stream, a);
    NFFT3_LAUNCH_CHECK("spread_ps_kernel");
    return NFFT3_OK;
}

int launch_spread(nfft3_plan_impl *p, const void *f, void *grid) {
    if (p->dtype == NFFT3_C128) { NFFT3_DISPATCH_M(spread_w, double, f, grid) }
    NFFT3_DISPATCH_M(spread_w, float, f, grid)
}

}  // namespace nfft3
