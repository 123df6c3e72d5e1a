// Evaluation of the series at a rectilinear grid (Sec. 2.1):
//
//   F[i0, i1, i2] = sum_k fhat_k e0[i0, k0] e1[i1, k1] e2[i2, k2],
//   e_d[i, k] = exp(-2 pi i k y_d[i]),  k = -N_d/2 .. N_d/2 - 1,
//
// in the NFFT sign on the unit period (the convention of nfft3_trafo).  As in
// Sec. 2.1 the nested sums are three dense complex matrix products, one per
// axis, the contiguous axis first:
//
//   t1[(k0, k1), i2] = sum_k2 fhat[(k0, k1), k2] e2^T[k2, i2]     (N0 N1 x N2) (N2 x M2)
//   t2[k0][i1, i2]   = sum_k1 e1[i1, k1] t1[k0][k1, i2]           N0 x (M1 x N1) (N1 x M2)
//   F[i0, (i1, i2)]  = sum_k0 e0[i0, k0] t2[k0, (i1, i2)]         (M0 x N0) (N0 x M1 M2)
//
// All three are row-major C = A B products, so one kernel serves them: a
// complex GEMM on the matrix cores (v_mfma_f64_16x16x4f64 / v_mfma_f32_16x16x4f32)
// with each complex product taken as three real ones (Gauss's form, as in
// the 3M complex GEMMs): P1 = Ar Br, P2 = Ai Bi, P3 = (Ar + Ai)(Br + Bi),
// Re C = P1 - P2, Im C = P3 - P1 - P2.  Its rounding error is bounded by a
// small multiple of eps sum |A||B| (|A| = |Ar| + |Ai|), the componentwise
// bound of the four-product form up to a constant; it issues 3/4 of the
// matrix operations (measured 18-20% faster on the 256^3 -> 321^3 chain).  The E^d tables are formed
// on the device from the coordinates with the phase k y reduced mod 1 in one
// fused multiply-add (rounded once), so their error does not grow with |k y|.
#include "internal.h"

namespace nfft3 {

typedef double dx4_t __attribute__((ext_vector_type(4)));
typedef float fx4_t __attribute__((ext_vector_type(4)));

template <typename T> struct Mfma;
// Operand layout (both): A[i][k] in lane i + 16 k, B[k][j] in lane j + 16 k.
// Result element r of lane l holds D[row(l / 16, r)][l % 16]; the row order
// differs between the two (checked on gfx950 with a one-wave probe).
template <> struct Mfma<double> {
    using acc = dx4_t;
    static __device__ __forceinline__ acc fma(double a, double b, acc c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lk, int r) { return lk + 4 * r; }
};
template <> struct Mfma<float> {
    using acc = fx4_t;
    static __device__ __forceinline__ acc fma(float a, float b, acc c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lk, int r) { return 4 * lk + r; }
};

__global__ void rgrid_flag_kernel(int *flag) {
    if (threadIdx.x < 16) flag[threadIdx.x] = 0;
}

// ------------------------------------------------------------ tables ----
// E[i][k] (row-major M x N, trans = 0) or E^T[k][i] (N x M, trans = 1) of
// exp(-2 pi i (k - N/2) y_i).  A non-finite coordinate sets *flag.
template <typename T>
__global__ void rgrid_table_kernel(const double *__restrict__ y, int64_t Md, int Nd, int trans,
                                   c_t<T> *__restrict__ E, int *__restrict__ flag) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= Md * Nd) return;
    int64_t i, k;
    if (trans) { k = e / Md; i = e - k * Md; }
    else { i = e / Nd; k = e - i * Nd; }
    const double yi = y[i];
    if (!isfinite(yi)) {
        atomicOr(flag, 1);
        E[e] = cmk<T>((T)0, (T)0);
        return;
    }
    const double kf = (double)(k - Nd / 2);
    // k y - n for the integer n nearest the rounded product, in one fused
    // operation: the exact product less n, rounded once (|r| <= 1/2 + ulp).
    // (Written as one fma so that no contraction of the surrounding
    // expressions can change it.)
    const double r = fma(kf, yi, -rint(kf * yi));
    double s, c;
    sincospi(2.0 * r, &s, &c);
    E[e] = cmk<T>((T)c, (T)-s);
}

// ------------------------------------------------------------- GEMM ----
// C[b] (M x N) = A[b] (M x K) B[b] (K x N), complex, row-major with row
// strides lda / ldb / ldc and batch strides sa / sb / sc (elements).
struct GemmArgs {
    const void *A;
    const void *B;
    void *C;
    int64_t M, N, K;
    int64_t lda, ldb, ldc;
    int64_t sa, sb, sc;
    int64_t tiles_m, tiles_n;
};

// C tile of a workgroup: BM x BN, four waves of BM/2 x BN/2 (2 x 2).  64 x
// 64 (2 x 2 blocks per wave, two waves per SIMD) ran the 256^3 -> 321^3
// chain fastest: 128 x 128 (FP32) and 128 x 64 (FP64) tiles, with four
// times the operand reuse per LDS read, hold one wave per SIMD and took
// 1.79 / 3.21 ms against 1.57 / 3.03 ms.
template <typename T> struct GemmTile;
template <> struct GemmTile<double> { static constexpr int BM = 64, BN = 64; };
template <> struct GemmTile<float> { static constexpr int BM = 64, BN = 64; };
constexpr int kGK = 16;        // contraction depth per LDS stage
constexpr int kGThreads = 256;
constexpr int kGPad = 1;       // LDS row padding (elements)

// One workgroup per (batch, row tile, column tile).  The A tile (BM x 16) and
// B tile (16 x BN) are staged in LDS as separate real and imaginary planes,
// A transposed (k-major) so that the 16 lanes of an MFMA operand row read
// consecutive words; the next K stage is loaded into registers while the
// current one is consumed.  Wave w owns the BM/2 x BN/2 quadrant (w / 2,
// w % 2): IB x JB MFMA blocks of 16 x 16, each with the three accumulators
// P1, P2, P3 (operand and result layouts: see Mfma); every operand read from
// LDS feeds JB (A) or IB (B) blocks.
template <typename T, int BM, int BN>
__global__ void __launch_bounds__(kGThreads) rgrid_gemm_kernel(GemmArgs g) {
    using C2 = c_t<T>;
    using Acc = typename Mfma<T>::acc;
    constexpr int IB = BM / 32, JB = BN / 32;
    constexpr int QA = BM * kGK / kGThreads, QB = BN * kGK / kGThreads;
    __shared__ T As[2][kGK][BM + kGPad];   // [re/im][k][row]
    __shared__ T Bs[2][kGK][BN + kGPad];   // [re/im][k][col]

    const int64_t tiles = g.tiles_m * g.tiles_n;
    const int64_t bidx = blockIdx.x;
    const int64_t batch = bidx / tiles;
    const int64_t rem = bidx - batch * tiles;
    const int64_t tm = rem / g.tiles_n, tn = rem - tm * g.tiles_n;
    const int64_t row0 = tm * BM, col0 = tn * BN;
    const C2 *A = (const C2 *)g.A + batch * g.sa;
    const C2 *B = (const C2 *)g.B + batch * g.sb;
    C2 *C = (C2 *)g.C + batch * g.sc;

    const int t = threadIdx.x;
    const int lane = t & 63, wave = t >> 6;
    const int lr = lane & 15, lk = lane >> 4;
    const int wr = (wave >> 1) * (BM / 2), wc = (wave & 1) * (BN / 2);

    // register staging: QA A and QB B elements per thread per stage
    C2 ra[QA], rb[QB];
    auto load_stage = [&](int64_t k0) {
#pragma unroll
        for (int q = 0; q < QA; ++q) {
            const int e = t + q * kGThreads;
            const int ar = e >> 4, ak = e & 15;          // A: BM rows x 16 k
            const int64_t gr = row0 + ar, gk = k0 + ak;
            ra[q] = (gr < g.M && gk < g.K) ? A[gr * g.lda + gk] : cmk<T>((T)0, (T)0);
        }
#pragma unroll
        for (int q = 0; q < QB; ++q) {
            const int e = t + q * kGThreads;
            const int bk = e / BN, bc = e % BN;          // B: 16 k x BN cols
            const int64_t hk = k0 + bk, hc = col0 + bc;
            rb[q] = (hk < g.K && hc < g.N) ? B[hk * g.ldb + hc] : cmk<T>((T)0, (T)0);
        }
    };
    auto store_stage = [&]() {
#pragma unroll
        for (int q = 0; q < QA; ++q) {
            const int e = t + q * kGThreads;
            const int ar = e >> 4, ak = e & 15;
            As[0][ak][ar] = ra[q].x;
            As[1][ak][ar] = ra[q].y;
        }
#pragma unroll
        for (int q = 0; q < QB; ++q) {
            const int e = t + q * kGThreads;
            const int bk = e / BN, bc = e % BN;
            Bs[0][bk][bc] = rb[q].x;
            Bs[1][bk][bc] = rb[q].y;
        }
    };

    Acc p1[IB][JB], p2[IB][JB], p3[IB][JB];
#pragma unroll
    for (int i = 0; i < IB; ++i)
#pragma unroll
        for (int j = 0; j < JB; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) { p1[i][j][r] = 0; p2[i][j][r] = 0; p3[i][j][r] = 0; }
    // 16 x 16 blocks wholly outside C (in the last row or column tile) issue
    // no MFMAs: a 321-wide output then costs 21 blocks per axis, not 24
    bool live[IB][JB];
#pragma unroll
    for (int i = 0; i < IB; ++i)
#pragma unroll
        for (int j = 0; j < JB; ++j) live[i][j] = row0 + wr + i * 16 < g.M && col0 + wc + j * 16 < g.N;

    load_stage(0);
    for (int64_t k0 = 0; k0 < g.K; k0 += kGK) {
        __syncthreads();                 // previous stage consumed
        store_stage();
        __syncthreads();
        if (k0 + kGK < g.K) load_stage(k0 + kGK);
#pragma unroll
        for (int kk = 0; kk < kGK; kk += 4) {
            T a_r[IB], a_i[IB], a_s[IB], b_r[JB], b_i[JB], b_s[JB];
#pragma unroll
            for (int i = 0; i < IB; ++i) {
                a_r[i] = As[0][kk + lk][wr + i * 16 + lr];
                a_i[i] = As[1][kk + lk][wr + i * 16 + lr];
                a_s[i] = a_r[i] + a_i[i];
            }
#pragma unroll
            for (int j = 0; j < JB; ++j) {
                b_r[j] = Bs[0][kk + lk][wc + j * 16 + lr];
                b_i[j] = Bs[1][kk + lk][wc + j * 16 + lr];
                b_s[j] = b_r[j] + b_i[j];
            }
#pragma unroll
            for (int i = 0; i < IB; ++i)
#pragma unroll
                for (int j = 0; j < JB; ++j) {
                    if (!live[i][j]) continue;
                    p1[i][j] = Mfma<T>::fma(a_r[i], b_r[j], p1[i][j]);
                    p2[i][j] = Mfma<T>::fma(a_i[i], b_i[j], p2[i][j]);
                    p3[i][j] = Mfma<T>::fma(a_s[i], b_s[j], p3[i][j]);
                }
        }
    }
#pragma unroll
    for (int i = 0; i < IB; ++i)
#pragma unroll
        for (int j = 0; j < JB; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t gr = row0 + wr + i * 16 + Mfma<T>::row(lk, r);
                const int64_t gc = col0 + wc + j * 16 + lr;
                const T v1 = p1[i][j][r], v2 = p2[i][j][r];
                if (gr < g.M && gc < g.N) C[gr * g.ldc + gc] = cmk<T>(v1 - v2, p3[i][j][r] - v1 - v2);
            }
}

template <typename T>
static int launch_gemm(hipStream_t s, const void *A, const void *B, void *C, int64_t M, int64_t N, int64_t K,
                       int64_t lda, int64_t ldb, int64_t ldc, int64_t batch, int64_t sa, int64_t sb, int64_t sc) {
    if (M <= 0 || N <= 0 || batch <= 0) return NFFT3_OK;
    GemmArgs g;
    g.A = A; g.B = B; g.C = C;
    g.M = M; g.N = N; g.K = K;
    g.lda = lda; g.ldb = ldb; g.ldc = ldc;
    g.sa = sa; g.sb = sb; g.sc = sc;
    constexpr int BM = GemmTile<T>::BM, BN = GemmTile<T>::BN;
    g.tiles_m = (M + BM - 1) / BM;
    g.tiles_n = (N + BN - 1) / BN;
    const int64_t blocks = g.tiles_m * g.tiles_n * batch;
    if (blocks > (int64_t)INT32_MAX) return NFFT3_ERR_INVALID_ARG;
    hipLaunchKernelGGL((rgrid_gemm_kernel<T, BM, BN>), dim3((unsigned)blocks), dim3(kGThreads), 0, s, g);
    NFFT3_LAUNCH_CHECK("rgrid_gemm_kernel");
    return NFFT3_OK;
}

// ------------------------------------------------------------- host ----
// Leading unit axes (N_d = M_d = 1: frequency 0 only, factor 1) make the
// two- and one-dimensional forms; their products are skipped.
static bool rgrid_unit(const nfft3_rgrid_impl *g, int d) { return g->N[d] == 1 && g->M[d] == 1; }

static int rgrid_tables(nfft3_rgrid_impl *g, const double *const y[3]) {
    hipLaunchKernelGGL(rgrid_flag_kernel, dim3(1), dim3(64), 0, g->stream, g->flag);
    NFFT3_LAUNCH_CHECK("rgrid_flag_kernel");
    for (int d = 0; d < 3; ++d) {
        if (rgrid_unit(g, d)) continue;          // no table: its product is skipped
        const int64_t cnt = g->M[d] * g->N[d];
        const unsigned blocks = (unsigned)((cnt + 255) / 256);
        const int trans = d == 2 ? 1 : 0;
        if (g->dtype == NFFT3_C128)
            hipLaunchKernelGGL(rgrid_table_kernel<double>, dim3(blocks), dim3(256), 0, g->stream, y[d], g->M[d],
                               (int)g->N[d], trans, (c_t<double> *)g->E[d], g->flag);
        else
            hipLaunchKernelGGL(rgrid_table_kernel<float>, dim3(blocks), dim3(256), 0, g->stream, y[d], g->M[d],
                               (int)g->N[d], trans, (c_t<float> *)g->E[d], g->flag);
        NFFT3_LAUNCH_CHECK("rgrid_table_kernel");
    }
    return NFFT3_OK;
}

int launch_rgrid_axes(nfft3_rgrid_impl *g, const double *const y[3]) { return rgrid_tables(g, y); }

template <typename T>
static int rgrid_eval_t(nfft3_rgrid_impl *g, const void *fhat, void *out) {
    const int64_t N0 = g->N[0], N1 = g->N[1], N2 = g->N[2];
    const int64_t M0 = g->M[0], M1 = g->M[1], M2 = g->M[2];
    hipStream_t s = g->stream;
    const bool u0 = rgrid_unit(g, 0), u1 = u0 && rgrid_unit(g, 1);
    // sum over k2: (N0 N1 x N2) (N2 x M2)
    int rc = launch_gemm<T>(s, fhat, g->E[2], u1 ? out : g->t1, N0 * N1, M2, N2, N2, M2, M2, 1, 0, 0, 0);
    if (rc || u1) return rc;
    // sum over k1, for every k0: (M1 x N1) (N1 x M2)
    rc = launch_gemm<T>(s, g->E[1], g->t1, u0 ? out : g->t2, M1, M2, N1, N1, M2, M2, N0, 0, N1 * M2, M1 * M2);
    if (rc || u0) return rc;
    // sum over k0: (M0 x N0) (N0 x M1 M2)
    return launch_gemm<T>(s, g->E[0], g->t2, out, M0, M1 * M2, N0, N0, M1 * M2, M1 * M2, 1, 0, 0, 0);
}

int launch_rgrid_eval(nfft3_rgrid_impl *g, const void *fhat, void *out) {
    if (g->dtype == NFFT3_C128) return rgrid_eval_t<double>(g, fhat, out);
    return rgrid_eval_t<float>(g, fhat, out);
}

}  // namespace nfft3
