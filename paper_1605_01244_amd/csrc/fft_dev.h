// Device code of the FFT passes (deconvolve + zero-pad + Stockham passes and
// the transposed adjoint passes), shared by the single-plan pass kernels
// (fft.hip) and the batched per-length launches (batch.hip).  See fft.hip for
// the pass structure.
#pragma once
#include "internal.h"

namespace nfft3 {

constexpr int kMaxStages = 16;

struct RadixList {
    int nrad;
    int r[kMaxStages];
};

// ---------------------------------------------------------------- DFTs ----
// In-place DFT of R values with kernel exp(sgn 2 pi i / R), sgn = FWD ? -1 : +1.
template <typename C, bool FWD>
__device__ __forceinline__ C mul_i(C a) {  // multiply by sgn*i
    C r;
    if (FWD) { r.x = a.y; r.y = -a.x; }    // -i * a
    else { r.x = -a.y; r.y = a.x; }        // +i * a
    return r;
}

template <typename T, bool FWD>
__device__ __forceinline__ void dft2(c_t<T> *v) {
    c_t<T> a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
}

template <typename T, bool FWD>
__device__ __forceinline__ void dft4(c_t<T> *v) {
    c_t<T> c0 = cadd(v[0], v[2]), c1 = csub(v[0], v[2]);
    c_t<T> c2 = cadd(v[1], v[3]), c3 = mul_i<c_t<T>, FWD>(csub(v[1], v[3]));
    v[0] = cadd(c0, c2);
    v[2] = csub(c0, c2);
    v[1] = cadd(c1, c3);
    v[3] = csub(c1, c3);
}

template <typename T, bool FWD>
__device__ __forceinline__ void dft8(c_t<T> *v) {
    const T h = (T)0.70710678118654752440084436210485;
    c_t<T> a[4], b[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) { a[r] = cadd(v[r], v[r + 4]); b[r] = csub(v[r], v[r + 4]); }
    // b_r *= w^r, w = exp(sgn 2 pi i/8)
    {
        c_t<T> t = b[1];   // w = h (1 + sgn i)
        b[1] = FWD ? cmk<T>(h * (t.x + t.y), h * (t.y - t.x)) : cmk<T>(h * (t.x - t.y), h * (t.y + t.x));
        b[2] = mul_i<c_t<T>, FWD>(b[2]);
        t = b[3];          // w^3 = h (-1 + sgn i)
        b[3] = FWD ? cmk<T>(h * (t.y - t.x), -h * (t.x + t.y)) : cmk<T>(-h * (t.x + t.y), h * (t.x - t.y));
    }
    dft4<T, FWD>(a);
    dft4<T, FWD>(b);
#pragma unroll
    for (int r = 0; r < 4; ++r) { v[2 * r] = a[r]; v[2 * r + 1] = b[r]; }
}

template <typename T, bool FWD>
__device__ __forceinline__ void dft3(c_t<T> *v) {
    const T s3 = (T)0.86602540378443864676372317075294;   // sqrt(3)/2
    c_t<T> t = cadd(v[1], v[2]);
    c_t<T> u = mul_i<c_t<T>, FWD>(csub(v[1], v[2]));
    c_t<T> x0 = v[0];
    v[0] = cadd(x0, t);
    c_t<T> a = cmk<T>(x0.x - (T)0.5 * t.x, x0.y - (T)0.5 * t.y);
    v[1] = cmk<T>(a.x + s3 * u.x, a.y + s3 * u.y);
    v[2] = cmk<T>(a.x - s3 * u.x, a.y - s3 * u.y);
}

template <typename T, bool FWD>
__device__ __forceinline__ void dft5(c_t<T> *v) {
    // X_k = sum_r x_r w^{rk}, w = exp(sgn 2 pi i/5); real/imag parts of w, w^2
    const T c1 = (T)0.30901699437494742410229341718282, c2 = (T)-0.80901699437494742410229341718282;
    const T s1 = (T)0.95105651629515357211643933337938, s2 = (T)0.58778525229247312916870595463907;
    c_t<T> a1 = cadd(v[1], v[4]), b1 = csub(v[1], v[4]);
    c_t<T> a2 = cadd(v[2], v[3]), b2 = csub(v[2], v[3]);
    c_t<T> x0 = v[0];
    c_t<T> p1 = cmk<T>(x0.x + c1 * a1.x + c2 * a2.x, x0.y + c1 * a1.y + c2 * a2.y);
    c_t<T> p2 = cmk<T>(x0.x + c2 * a1.x + c1 * a2.x, x0.y + c2 * a1.y + c1 * a2.y);
    // q1 = sgn i (s1 b1 + s2 b2), q2 = sgn i (s2 b1 - s1 b2)
    c_t<T> q1 = mul_i<c_t<T>, FWD>(cmk<T>(s1 * b1.x + s2 * b2.x, s1 * b1.y + s2 * b2.y));
    c_t<T> q2 = mul_i<c_t<T>, FWD>(cmk<T>(s2 * b1.x - s1 * b2.x, s2 * b1.y - s1 * b2.y));
    v[0] = cadd(x0, cadd(a1, a2));
    v[1] = cadd(p1, q1);
    v[4] = csub(p1, q1);
    v[2] = cadd(p2, q2);
    v[3] = csub(p2, q2);
}

template <typename T, bool FWD>
__device__ __forceinline__ void dft7(c_t<T> *v) {
    // pairs a_k = x_k + x_{7-k}, b_k = x_k - x_{7-k}; X_m = x_0 + sum_k cos(2 pi k m/7) a_k
    // + sgn i sum_k sin(2 pi k m/7) b_k and X_{7-m} the same with - sgn i
    const T c1 = (T)0.6234898018587335305250048840042398, c2 = (T)-0.2225209339563144042889025644967948,
            c3 = (T)-0.9009688679024191262361023195074451;
    const T s1 = (T)0.7818314824680298087084445266740578, s2 = (T)0.9749279121818236070181316829939312,
            s3 = (T)0.4338837391175581204757683328483588;
    const c_t<T> a1 = cadd(v[1], v[6]), b1 = csub(v[1], v[6]);
    const c_t<T> a2 = cadd(v[2], v[5]), b2 = csub(v[2], v[5]);
    const c_t<T> a3 = cadd(v[3], v[4]), b3 = csub(v[3], v[4]);
    const c_t<T> x0 = v[0];
    auto lin3 = [](T p, c_t<T> u, T q, c_t<T> w, T r, c_t<T> z) {
        return cmk<T>(p * u.x + q * w.x + r * z.x, p * u.y + q * w.y + r * z.y);
    };
    const c_t<T> p1 = cadd(x0, lin3(c1, a1, c2, a2, c3, a3));
    const c_t<T> p2 = cadd(x0, lin3(c2, a1, c3, a2, c1, a3));
    const c_t<T> p3 = cadd(x0, lin3(c3, a1, c1, a2, c2, a3));
    const c_t<T> q1 = mul_i<c_t<T>, FWD>(lin3(s1, b1, s2, b2, s3, b3));
    const c_t<T> q2 = mul_i<c_t<T>, FWD>(lin3(s2, b1, -s3, b2, -s1, b3));
    const c_t<T> q3 = mul_i<c_t<T>, FWD>(lin3(s3, b1, -s1, b2, s2, b3));
    v[0] = cadd(x0, cadd(a1, cadd(a2, a3)));
    v[1] = cadd(p1, q1);
    v[6] = csub(p1, q1);
    v[2] = cadd(p2, q2);
    v[5] = csub(p2, q2);
    v[3] = cadd(p3, q3);
    v[4] = csub(p3, q3);
}

template <typename T, int R, bool FWD>
__device__ __forceinline__ void dft_small(c_t<T> *v) {
    if constexpr (R == 2) dft2<T, FWD>(v);
    else if constexpr (R == 3) dft3<T, FWD>(v);
    else if constexpr (R == 4) dft4<T, FWD>(v);
    else if constexpr (R == 5) dft5<T, FWD>(v);
    else if constexpr (R == 7) dft7<T, FWD>(v);
    else dft8<T, FWD>(v);
}

// ------------------------------------------------------ Stockham engine ----
// Radix-R stage over `nlines` lines of length n: butterfly j of a line reads
// x[j + r n/R], twiddles by W^{r (j mod Ns) n/(Ns R)} (W = exp(-+2 pi i/n)) and
// writes its R results to (j/Ns) Ns R + (j mod Ns) + r Ns.  The first stage
// reads its inputs through `ld` straight from global memory (zero-padding is
// never loaded), the last stage writes through `st` straight to global memory
// (for the last stage Ns = n/R, so the outputs land at j + r n/R); only the
// stages in between go through LDS, in place: every read of a stage completes
// (barrier) before any of its writes.
//
// Butterfly -> (line, j) mapping: LINE_FAST puts consecutive lanes on
// consecutive lines (strided-axis tiles: lines are adjacent columns in memory,
// so a wave's loads are contiguous); otherwise consecutive lanes take
// consecutive j of one line (contiguous rows).
template <bool LINE_FAST>
__device__ __forceinline__ void bt_map(int bt, int nlines, int nbl, int &line, int &j) {
    if (LINE_FAST) { j = bt / nlines; line = bt - j * nlines; }
    else { line = bt / nbl; j = bt - line * nbl; }
}

template <typename T, int R, int VMAX, int NT, bool FWD, bool LINE_FAST, bool FIRST, bool LAST, class LD, class ST>
__device__ __forceinline__ void fft_stage(c_t<T> *buf, int ls, int nlines, int n, int Ns,
                                          const c_t<T> *__restrict__ tw, LD &ld, ST &st) {
    constexpr int BMAX = VMAX / R;
    const int tid = threadIdx.x;
    const int nbl = n / R;
    const int NB = nlines * nbl;
    c_t<T> v[BMAX][R];
#pragma unroll
    for (int i = 0; i < BMAX; ++i) {
        const int bt = tid + i * NT;
        if (bt < NB) {
            int line, j;
            bt_map<LINE_FAST>(bt, nlines, nbl, line, j);
            if (FIRST) {
#pragma unroll
                for (int r = 0; r < R; ++r) v[i][r] = ld(line, j + r * nbl);
            } else {
                const c_t<T> *src = buf + line * ls;
#pragma unroll
                for (int r = 0; r < R; ++r) v[i][r] = src[j + r * nbl];
            }
        }
    }
    if (!FIRST && !LAST) __syncthreads();
    const int step = n / (Ns * R);
#pragma unroll
    for (int i = 0; i < BMAX; ++i) {
        const int bt = tid + i * NT;
        if (bt < NB) {
            int line, j;
            bt_map<LINE_FAST>(bt, nlines, nbl, line, j);
            const int k = j % Ns;
            if (!FIRST && Ns > 1) {
#pragma unroll
                for (int r = 1; r < R; ++r) {
                    const c_t<T> w = tw[r * k * step];
                    v[i][r] = FWD ? cmul(v[i][r], w) : cmulc(v[i][r], w);
                }
            }
            dft_small<T, R, FWD>(v[i]);
            if (LAST) {
#pragma unroll
                for (int r = 0; r < R; ++r) st(line, j + r * nbl, v[i][r]);
            } else {
                c_t<T> *dst = buf + line * ls;
                const int base = (j / Ns) * Ns * R + k;
#pragma unroll
                for (int r = 0; r < R; ++r) dst[base + r * Ns] = v[i][r];
            }
        }
    }
    if (!LAST) __syncthreads();
}

template <typename T, int VMAX, int NT, bool FWD, bool LINE_FAST, bool FIRST, bool LAST, class LD, class ST>
__device__ __forceinline__ void fft_stage_r(int R, c_t<T> *buf, int ls, int nlines, int n, int Ns,
                                            const c_t<T> *__restrict__ tw, LD &ld, ST &st) {
    switch (R) {
        case 8: fft_stage<T, 8, VMAX, NT, FWD, LINE_FAST, FIRST, LAST>(buf, ls, nlines, n, Ns, tw, ld, st); break;
        case 4: fft_stage<T, 4, VMAX, NT, FWD, LINE_FAST, FIRST, LAST>(buf, ls, nlines, n, Ns, tw, ld, st); break;
        case 2: fft_stage<T, 2, VMAX, NT, FWD, LINE_FAST, FIRST, LAST>(buf, ls, nlines, n, Ns, tw, ld, st); break;
        case 3: fft_stage<T, 3, VMAX, NT, FWD, LINE_FAST, FIRST, LAST>(buf, ls, nlines, n, Ns, tw, ld, st); break;
        case 7: fft_stage<T, 7, VMAX, NT, FWD, LINE_FAST, FIRST, LAST>(buf, ls, nlines, n, Ns, tw, ld, st); break;
        default: fft_stage<T, 5, VMAX, NT, FWD, LINE_FAST, FIRST, LAST>(buf, ls, nlines, n, Ns, tw, ld, st); break;
    }
}

template <typename T, int VMAX, int NT, bool FWD, bool LINE_FAST, class LD, class ST>
__device__ __forceinline__ void fft_lines(c_t<T> *buf, int ls, int nlines, int n, const RadixList &rl,
                                          const c_t<T> *__restrict__ tw, LD &ld, ST &st) {
    if (rl.nrad == 1) {
        fft_stage_r<T, VMAX, NT, FWD, LINE_FAST, true, true>(rl.r[0], buf, ls, nlines, n, 1, tw, ld, st);
        return;
    }
    int Ns = rl.r[0];
    fft_stage_r<T, VMAX, NT, FWD, LINE_FAST, true, false>(rl.r[0], buf, ls, nlines, n, 1, tw, ld, st);
    for (int s = 1; s + 1 < rl.nrad; ++s) {
        fft_stage_r<T, VMAX, NT, FWD, LINE_FAST, false, false>(rl.r[s], buf, ls, nlines, n, Ns, tw, ld, st);
        Ns *= rl.r[s];
    }
    fft_stage_r<T, VMAX, NT, FWD, LINE_FAST, false, true>(rl.r[rl.nrad - 1], buf, ls, nlines, n, Ns, tw, ld, st);
}

// ------------------------------------------------ compile-time engine ----
// The same Stockham stages with n, the radices (st_radix), the spans Ns, the
// lines per workgroup NL and the LDS line stride LS known at compile time:
// the index math folds to constant divisions (shifts and masks for powers
// of two), and a stage's twiddles come from its own table (8 entries per k,
// so one butterfly's are contiguous).
template <typename T, int N, int S, int NL, int LS, int NT, bool FWD, bool LINE_FAST, class LD, class ST>
__device__ __forceinline__ void sfft_stage(c_t<T> *buf, const c_t<T> *__restrict__ stw, LD &ld, ST &st) {
    constexpr int R = st_radix(N, S), NS = st_ns(N, S), NRAD = st_nrad(N);
    constexpr bool FIRST = S == 0, LAST = S == NRAD - 1;
    constexpr int NBL = N / R, NB = NL * NBL, BPT = (NB + NT - 1) / NT;
    const int tid = threadIdx.x;
    c_t<T> v[BPT][R];
#pragma unroll
    for (int i = 0; i < BPT; ++i) {
        const int bt = tid + i * NT;
        if (NB % NT == 0 || bt < NB) {
            const int j = LINE_FAST ? bt / NL : bt % NBL;
            const int line = LINE_FAST ? bt % NL : bt / NBL;
            if constexpr (FIRST) {
#pragma unroll
                for (int r = 0; r < R; ++r) v[i][r] = ld(line, j + r * NBL);
            } else {
                const c_t<T> *src = buf + line * LS + j;
#pragma unroll
                for (int r = 0; r < R; ++r) v[i][r] = src[r * NBL];
            }
        }
    }
    if constexpr (!FIRST && !LAST) __syncthreads();
#pragma unroll
    for (int i = 0; i < BPT; ++i) {
        const int bt = tid + i * NT;
        if (NB % NT == 0 || bt < NB) {
            const int j = LINE_FAST ? bt / NL : bt % NBL;
            const int line = LINE_FAST ? bt % NL : bt / NBL;
            const int k = j % NS;
            if constexpr (!FIRST) {
                const c_t<T> *w = stw + st_tw_offset(N, S) + k * 8;
#pragma unroll
                for (int r = 1; r < R; ++r) v[i][r] = FWD ? cmul(v[i][r], w[r]) : cmulc(v[i][r], w[r]);
            }
            dft_small<T, R, FWD>(v[i]);
            if constexpr (LAST) {
#pragma unroll
                for (int r = 0; r < R; ++r) st(line, j + r * NBL, v[i][r]);
            } else {
                c_t<T> *dst = buf + line * LS + (j - k) * R + k;   // (j / Ns) Ns R + j mod Ns
#pragma unroll
                for (int r = 0; r < R; ++r) dst[r * NS] = v[i][r];
            }
        }
    }
    if constexpr (!LAST) __syncthreads();
}

template <typename T, int N, int S, int NL, int LS, int NT, bool FWD, bool LINE_FAST, class LD, class ST>
__device__ __forceinline__ void sfft_lines(c_t<T> *buf, const c_t<T> *__restrict__ stw, LD &ld, ST &st) {
    sfft_stage<T, N, S, NL, LS, NT, FWD, LINE_FAST>(buf, stw, ld, st);
    if constexpr (S + 1 < st_nrad(N)) sfft_lines<T, N, S + 1, NL, LS, NT, FWD, LINE_FAST>(buf, stw, ld, st);
}

// Column passes of the compile-time engine: workgroup size, and the LDS
// bound of one tile (lines of n + 1 values).  A tile spans 256 contiguous
// bytes of every row it visits: along axis 0 consecutive rows lie one plane
// (n1 n2 values, 2 MB and more) apart, so each row visit is a separate page
// translation, and 128-byte segments ran that pass at ~60% of the axis-1
// pass's bandwidth.  The generic engine keeps 128-byte segments, 512
// threads and an 80 KB tile (its double-precision body spills at 1024).
constexpr int kColsThreads = 1024;
constexpr size_t kColsLdsMax = 144 * 1024;
constexpr int kColsThreadsGeneric = 512;
constexpr size_t kColsLdsMaxGeneric = 80 * 1024;

// Lengths served by the compile-time engine, and its lines per workgroup:
// the row count equals what make_row_args finds with lines_fit over the same
// radix plan, and make_col_args takes the column count from here, so host
// and device agree.
constexpr bool static_fft_len(int n) {
    return n == 64 || n == 80 || n == 96 || n == 128 || n == 160 || n == 192 || n == 256 || n == 320 || n == 384 ||
           n == 512;
}
constexpr int st_lines_fit(int n, int vmax, int cap, int nthreads) {
    int best = 1;
    for (int L = 1; L <= cap; ++L) {
        bool ok = true;
        for (int s = 0; s < st_nrad(n); ++s) {
            const int R = st_radix(n, s);
            const int per = (L * (n / R) + nthreads - 1) / nthreads;
            if (per > vmax / R) { ok = false; break; }
        }
        if (!ok) break;
        best = L;
    }
    return best;
}
template <typename T>
constexpr int static_rows_nl(int n) {
    int cap = 32768 / (n * (int)sizeof(c_t<T>));
    cap = cap < 1 ? 1 : (cap > 64 ? 64 : cap);
    return st_lines_fit(n, 16, cap, 256);
}
template <typename T>
constexpr int static_cols_nl(int n) {
    int C = 256 / (int)sizeof(c_t<T>);
    while (C > 1 && C * (n + 1) * (int)sizeof(c_t<T>) > (int)kColsLdsMax) C /= 2;
    const int f = st_lines_fit(n, 16, C, kColsThreads);
    return f < C ? f : C;
}

// FFT position -> compact index of a pruned line of L entries (frequency
// k = pos or pos - n; kept when -L/2 <= k < L/2), or -1.
__device__ __forceinline__ int compact_of(int pos, int L, int n) {
    const int k = pos < n / 2 ? pos : pos - n;
    return (k >= -L / 2 && k < L / 2) ? k + L / 2 : -1;
}

// -------------------------------------------------------- row passes ----
// MODE 0 (forward, first pass): rows (i0,i1) of fhat deconvolved by
//   c0[i0] c1[i1] c2[i2] (times -2 pi i k_d for a derivative field) at FFT
//   position of i2; all n outputs stored to grid rows (i0,i1).
// MODE 1 (adjoint, last pass): grid rows (i0,i1) transformed with + sign; the
//   N2 kept outputs times c0 c1 c2 stored to fhat.
struct RowArgs {
    const void *in;
    void *out;
    const void *c0, *c1, *c2;
    const void *tw;
    const void *stw;             // stage tables of the compile-time engine
    int n, N0, N1, N2;
    int64_t grid_s0, grid_s1;   // grid strides of i0, i1 (elements)
    int lpw;                     // rows per workgroup
    int deriv;                   // -1 or axis
    RadixList rl;
};

template <typename T, int MODE, int NT>
__device__ __forceinline__ void rows_body(const RowArgs &a, int blk, unsigned char *smem_raw) {
    c_t<T> *buf = reinterpret_cast<c_t<T> *>(smem_raw);
    const int n = a.n;
    const int64_t nrows = (int64_t)a.N0 * a.N1;
    const int64_t row0 = (int64_t)blk * a.lpw;
    const int nl = (int)min<int64_t>(a.lpw, nrows - row0);
    const T *c0 = (const T *)a.c0, *c1 = (const T *)a.c1, *c2 = (const T *)a.c2;
    const T twopi = (T)6.283185307179586476925286766559;
    const int N0 = a.N0, N1 = a.N1, N2 = a.N2, deriv = a.deriv;
    const int64_t s0 = a.grid_s0, s1 = a.grid_s1;

    // rows handled here are (i0, i1) = divmod(row0 + line, N1); 32-bit index math
    const int rbase = (int)row0;
    if (MODE == 0) {
        const c_t<T> *fhat = (const c_t<T> *)a.in;
        c_t<T> *grid = (c_t<T> *)a.out;
        auto ld = [&](int line, int pos) -> c_t<T> {
            const int i2 = compact_of(pos, N2, n);
            if (i2 < 0) return cmk<T>(0, 0);
            const int row = rbase + line;
            const int i0 = row / N1, i1 = row - i0 * N1;
            c_t<T> v = fhat[(int64_t)row * N2 + i2];
            const T s = c0[i0] * c1[i1] * c2[i2];
            v.x *= s;
            v.y *= s;
            if (deriv >= 0) {   // times -2 pi i k_d
                const int kd = deriv == 0 ? i0 - N0 / 2 : deriv == 1 ? i1 - N1 / 2 : i2 - N2 / 2;
                const T f = twopi * (T)kd;
                v = cmk<T>(f * v.y, -f * v.x);
            }
            return v;
        };
        auto st = [&](int line, int pos, c_t<T> v) {
            const int row = rbase + line;
            const int i0 = row / N1, i1 = row - i0 * N1;
            grid[i0 * s0 + i1 * s1 + pos] = v;
        };
        fft_lines<T, 16, NT, true, false>(buf, n, nl, n, a.rl, (const c_t<T> *)a.tw, ld, st);
    } else {
        const c_t<T> *grid = (const c_t<T> *)a.in;
        c_t<T> *fhat = (c_t<T> *)a.out;
        auto ld = [&](int line, int pos) -> c_t<T> {
            const int row = rbase + line;
            const int i0 = row / N1, i1 = row - i0 * N1;
            return grid[i0 * s0 + i1 * s1 + pos];
        };
        auto st = [&](int line, int pos, c_t<T> v) {
            const int o = compact_of(pos, N2, n);
            if (o < 0) return;
            const int row = rbase + line;
            const int i0 = row / N1, i1 = row - i0 * N1;
            const T s = c0[i0] * c1[i1] * c2[o];
            v.x *= s;
            v.y *= s;
            fhat[(int64_t)row * N2 + o] = v;
        };
        fft_lines<T, 16, NT, false, false>(buf, n, nl, n, a.rl, (const c_t<T> *)a.tw, ld, st);
    }
}

// Row pass with the compile-time engine: n = N, NL rows per workgroup (the
// last workgroup may hold fewer: the others are masked).
template <typename T, int MODE, int NT, int N, int NL>
__device__ __forceinline__ void rows_body_s(const RowArgs &a, int blk, unsigned char *smem_raw) {
    c_t<T> *buf = reinterpret_cast<c_t<T> *>(smem_raw);
    const int nrows = a.N0 * a.N1;
    const int rbase = blk * NL;
    const int nl = min(NL, nrows - rbase);
    const T *c0 = (const T *)a.c0, *c1 = (const T *)a.c1, *c2 = (const T *)a.c2;
    const T twopi = (T)6.283185307179586476925286766559;
    const int N0 = a.N0, N1 = a.N1, N2 = a.N2, deriv = a.deriv;
    const int s0 = (int)a.grid_s0, s1 = (int)a.grid_s1;
    const c_t<T> *stw = (const c_t<T> *)a.stw;
    if (MODE == 0) {
        const c_t<T> *fhat = (const c_t<T> *)a.in;
        c_t<T> *grid = (c_t<T> *)a.out;
        auto ld = [&](int line, int pos) -> c_t<T> {
            const int i2 = compact_of(pos, N2, N);
            if (i2 < 0 || line >= nl) return cmk<T>(0, 0);
            const int row = rbase + line;
            const int i0 = row / N1, i1 = row - i0 * N1;
            c_t<T> v = fhat[(int64_t)row * N2 + i2];
            const T s = c0[i0] * c1[i1] * c2[i2];
            v.x *= s;
            v.y *= s;
            if (deriv >= 0) {   // times -2 pi i k_d
                const int kd = deriv == 0 ? i0 - N0 / 2 : deriv == 1 ? i1 - N1 / 2 : i2 - N2 / 2;
                const T f = twopi * (T)kd;
                v = cmk<T>(f * v.y, -f * v.x);
            }
            return v;
        };
        auto st = [&](int line, int pos, c_t<T> v) {
            if (line >= nl) return;
            const int row = rbase + line;
            const int i0 = row / N1, i1 = row - i0 * N1;
            grid[(int64_t)i0 * s0 + i1 * s1 + pos] = v;
        };
        sfft_lines<T, N, 0, NL, N, NT, true, false>(buf, stw, ld, st);
    } else {
        const c_t<T> *grid = (const c_t<T> *)a.in;
        c_t<T> *fhat = (c_t<T> *)a.out;
        auto ld = [&](int line, int pos) -> c_t<T> {
            if (line >= nl) return cmk<T>(0, 0);
            const int row = rbase + line;
            const int i0 = row / N1, i1 = row - i0 * N1;
            return grid[(int64_t)i0 * s0 + i1 * s1 + pos];
        };
        auto st = [&](int line, int pos, c_t<T> v) {
            const int o = compact_of(pos, N2, N);
            if (o < 0 || line >= nl) return;
            const int row = rbase + line;
            const int i0 = row / N1, i1 = row - i0 * N1;
            const T s = c0[i0] * c1[i1] * c2[o];
            v.x *= s;
            v.y *= s;
            fhat[(int64_t)row * N2 + o] = v;
        };
        sfft_lines<T, N, 0, NL, N, NT, false, false>(buf, stw, ld, st);
    }
}

// ----------------------------------------------------- column passes ----
// In-place transform along a strided axis of tiles of C adjacent columns.
// Column c of tile (outer, x0) has element i at
//   data[outer * s_outer + i * s_axis + x0 + c].
// Input: Lin entries (compact, at their FFT positions) or all n; output: all
// n or the Lout compact entries.
struct ColArgs {
    void *data;
    const void *tw;
    const void *stw;
    int n, Lin, Lout;
    int ncols;          // contiguous extent (columns)
    int C;              // columns per tile
    int64_t s_axis, s_outer;
    RadixList rl;
};

template <typename T, bool FWD, int NT, int VMAX>
__device__ __forceinline__ void cols_body(const ColArgs &a, int bx, int by, unsigned char *smem_raw) {
    c_t<T> *buf = reinterpret_cast<c_t<T> *>(smem_raw);
    const int n = a.n, C = a.C;
    const int ls = n + 1;   // padded line stride
    const int x0 = bx * C;
    const int nc = min(C, a.ncols - x0);
    c_t<T> *data = (c_t<T> *)a.data + (int64_t)by * a.s_outer + x0;
    const int Lin = a.Lin, Lout = a.Lout;
    const int64_t sa = a.s_axis;
    auto ld = [&](int c, int pos) -> c_t<T> {
        if (c >= nc) return cmk<T>(0, 0);
        int i = pos;
        if (Lin < n) {
            i = compact_of(pos, Lin, n);
            if (i < 0) return cmk<T>(0, 0);
        }
        return data[(int64_t)i * sa + c];
    };
    auto st = [&](int c, int pos, c_t<T> v) {
        if (c >= nc) return;
        int o = pos;
        if (Lout < n) {
            o = compact_of(pos, Lout, n);
            if (o < 0) return;
        }
        data[(int64_t)o * sa + c] = v;
    };
    fft_lines<T, VMAX, NT, FWD, true>(buf, ls, C, n, a.rl, (const c_t<T> *)a.tw, ld, st);
}


// Column pass with the compile-time engine: n = N, C = NC columns per tile.
template <typename T, bool FWD, int NT, int N, int NC>
__device__ __forceinline__ void cols_body_s(const ColArgs &a, int bx, int by, unsigned char *smem_raw) {
    c_t<T> *buf = reinterpret_cast<c_t<T> *>(smem_raw);
    const int x0 = bx * NC;
    const int nc = min(NC, a.ncols - x0);
    c_t<T> *data = (c_t<T> *)a.data + (int64_t)by * a.s_outer + x0;
    const int Lin = a.Lin, Lout = a.Lout;
    const int64_t sa = a.s_axis;
    auto ld = [&](int c, int pos) -> c_t<T> {
        if (c >= nc) return cmk<T>(0, 0);
        int i = pos;
        if (Lin < N) {
            i = compact_of(pos, Lin, N);
            if (i < 0) return cmk<T>(0, 0);
        }
        return data[(int64_t)i * sa + c];
    };
    auto st = [&](int c, int pos, c_t<T> v) {
        if (c >= nc) return;
        int o = pos;
        if (Lout < N) {
            o = compact_of(pos, Lout, N);
            if (o < 0) return;
        }
        data[(int64_t)o * sa + c] = v;
    };
    sfft_lines<T, N, 0, NC, N + 1, NT, FWD, true>(buf, (const c_t<T> *)a.stw, ld, st);
}

// The lengths the compile-time engine is instantiated for (2^a 3^b 5^c
// oversampled lengths of the common coefficient sizes).
#define NFFT3_STATIC_LENGTHS(X) X(64) X(80) X(96) X(128) X(160) X(192) X(256) X(320) X(384) X(512)

// Largest number of lines such that every stage fits VMAX values per thread.
inline int lines_fit(const FftAxisPlan &f, int vmax, int cap, int nthreads) {
    int best = 1;
    for (int L = 1; L <= cap; ++L) {
        bool ok = true;
        for (int s = 0; s < f.nrad; ++s) {
            const int R = f.radix[s];
            const int NB = L * (f.n / R);
            const int per = (NB + nthreads - 1) / nthreads;
            if (per > vmax / R) { ok = false; break; }
        }
        if (ok) best = L;
        else break;
    }
    return best;
}

inline RadixList radix_list(const FftAxisPlan &f) {
    RadixList rl;
    rl.nrad = f.nrad;
    for (int i = 0; i < kMaxStages; ++i) rl.r[i] = i < f.nrad ? f.radix[i] : 0;
    return rl;
}

// Column tiles may use more than 64 KiB of LDS (gfx950 has 160 KiB per CU).

// Row-pass arguments (mode 0: forward first pass into `grid`; mode 1: adjoint
// last pass from `grid`) for workgroups of nthreads threads.
template <typename T>
inline RowArgs make_row_args(const nfft3_plan_impl *p, const void *in, void *out, int deriv, int nthreads) {
    const FftAxisPlan &f = p->fft[2];
    RowArgs a;
    a.in = in;
    a.out = out;
    a.c0 = p->cdec[0];
    a.c1 = p->cdec[1];
    a.c2 = p->cdec[2];
    a.tw = f.tw;
    a.stw = f.stw;
    a.n = f.n;
    a.N0 = (int)p->N[0];
    a.N1 = (int)p->N[1];
    a.N2 = (int)p->N[2];
    a.grid_s0 = p->n[1] * p->n[2];
    a.grid_s1 = p->n[2];
    a.deriv = deriv;
    a.rl = radix_list(f);
    const int cap = std::max(1, (int)(32768 / (f.n * sizeof(c_t<T>))));
    a.lpw = lines_fit(f, 16, std::max(1, std::min(cap, 64)), nthreads);
    return a;
}
inline int64_t row_blocks(const nfft3_plan_impl *p, const RowArgs &a) {
    return (p->N[0] * p->N[1] + a.lpw - 1) / a.lpw;
}
template <typename T>
inline size_t row_lds(const RowArgs &a) { return (size_t)a.lpw * a.n * sizeof(c_t<T>); }

// Column-pass arguments over `grid` for workgroups of nthreads threads with
// at most vmax values per thread.
template <typename T>
inline ColArgs make_col_args(const nfft3_plan_impl *p, void *grid, int axis, int Lin, int Lout, int64_t s_outer) {
    const FftAxisPlan &f = p->fft[axis];
    ColArgs a;
    a.data = grid;
    a.tw = f.tw;
    a.stw = f.stw;
    a.n = f.n;
    a.Lin = Lin;
    a.Lout = Lout;
    a.ncols = (int)p->n[2];
    a.s_axis = axis == 0 ? p->n[1] * p->n[2] : p->n[2];
    a.s_outer = s_outer;
    a.rl = radix_list(f);
    if (static_fft_len(f.n) && static_cols_nl<T>(f.n) <= a.ncols) {
        a.C = static_cols_nl<T>(f.n);
        return a;
    }
    // generic engine: 128-byte column segments, bounded by LDS and registers
    int C = (int)(128 / sizeof(c_t<T>));
    while (C > 1 && (size_t)C * (f.n + 1) * sizeof(c_t<T>) > kColsLdsMaxGeneric) C /= 2;
    C = std::min(C, lines_fit(f, 16, C, kColsThreadsGeneric));
    C = std::min<int>(C, a.ncols);
    a.C = C;
    return a;
}
// whether a column pass runs on the compile-time engine, and its workgroup size
template <typename T>
inline bool col_static(const ColArgs &a) { return static_fft_len(a.n) && a.C == static_cols_nl<T>(a.n); }
template <typename T>
inline int col_threads(const ColArgs &a) { return col_static<T>(a) ? kColsThreads : kColsThreadsGeneric; }
template <typename T>
inline size_t col_lds(const ColArgs &a) { return (size_t)a.C * (a.n + 1) * sizeof(c_t<T>); }
inline int col_grid_x(const ColArgs &a) { return (a.ncols + a.C - 1) / a.C; }

}  // namespace nfft3
