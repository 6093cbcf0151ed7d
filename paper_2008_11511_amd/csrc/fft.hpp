// fft.hpp - device building blocks for batched complex64 power-of-two FFTs
// on gfx950 (wave64).
//
// A length-N 1D transform is done by T = N/E threads that each hold E
// elements in registers.  It runs as a sequence of self-sorting (Stockham)
// passes of radix R_p (product = N): in each pass a thread performs E/R_p
// radix-R_p butterflies on elements N/R_p apart, after a twiddle by
// exp(sign 2 pi i r k / (R_p L)) (L = product of the earlier radices,
// k = butterfly index mod L), and the results are exchanged through LDS
// between passes.  The in-register radix-2/4/8/16 DFTs use compile-time
// constant twiddles.  The inverse transform runs the radices in reverse
// order, so that the element-to-register layout a forward transform leaves
// behind is exactly the input layout of the inverse (the column kernel
// chains forward -> modulus -> inverse without touching memory).
//
// The transforms here are unnormalised; callers fold the unitary 1/N of a
// 2D transform into their own pointwise step.
#pragma once

#include <hip/hip_runtime.h>

namespace ptycho {

// ---------------------------------------------------------------- complex --
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
// The products below name their fused multiply-adds explicitly, so that
// every kernel that forms a product rounds it the same way whatever the
// compiler's contraction would choose for the surrounding code: two kernels
// fed the same values (say an integer window and a sub-pixel window whose
// fraction is zero) then give the same bits.
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(__builtin_fmaf(a.x, b.x, -(a.y * b.y)), __builtin_fmaf(a.x, b.y, a.y * b.x));
}
// conj(a) * b
__device__ __forceinline__ float2 cmulc(float2 a, float2 b) {
    return make_float2(__builtin_fmaf(a.x, b.x, a.y * b.y), __builtin_fmaf(a.x, b.y, -(a.y * b.x)));
}
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
__device__ __forceinline__ float cnorm(float2 a) { return __builtin_fmaf(a.x, a.x, a.y * a.y); }

// multiply by exp(DIR * i pi / 2): -i for the forward sign, +i for inverse
template <int DIR>
__device__ __forceinline__ float2 rot90(float2 a) {
    if constexpr (DIR < 0) return make_float2(a.y, -a.x);
    else return make_float2(-a.y, a.x);
}

// multiply by exp(DIR * 2 pi i * M / 16), M known at compile time
template <int M, int DIR>
__device__ __forceinline__ float2 tw16(float2 a) {
    constexpr int m = M & 15;
    // cos / sin of 2 pi m / 16
    constexpr float C[16] = {1.0f, 0.92387953251128674f, 0.70710678118654752f, 0.38268343236508977f,
                             0.0f, -0.38268343236508977f, -0.70710678118654752f, -0.92387953251128674f,
                             -1.0f, -0.92387953251128674f, -0.70710678118654752f, -0.38268343236508977f,
                             0.0f, 0.38268343236508977f, 0.70710678118654752f, 0.92387953251128674f};
    constexpr float S[16] = {0.0f, 0.38268343236508977f, 0.70710678118654752f, 0.92387953251128674f,
                             1.0f, 0.92387953251128674f, 0.70710678118654752f, 0.38268343236508977f,
                             0.0f, -0.38268343236508977f, -0.70710678118654752f, -0.92387953251128674f,
                             -1.0f, -0.92387953251128674f, -0.70710678118654752f, -0.38268343236508977f};
    if constexpr (m == 0) {
        return a;
    } else if constexpr (m == 4) {
        return rot90<DIR>(a);
    } else if constexpr (m == 8) {
        return make_float2(-a.x, -a.y);
    } else if constexpr (m == 12) {
        return rot90<-DIR>(a);
    } else if constexpr (m == 2 || m == 6 || m == 10 || m == 14) {
        // (+-1 +- i)/sqrt2: two adds and two multiplies
        constexpr float c = C[m];
        constexpr float s = (DIR < 0 ? -1.0f : 1.0f) * S[m];
        return make_float2(c * a.x - s * a.y, c * a.y + s * a.x);
    } else {
        constexpr float c = C[m];
        constexpr float s = (DIR < 0 ? -1.0f : 1.0f) * S[m];
        return make_float2(c * a.x - s * a.y, c * a.y + s * a.x);
    }
}

// In-register DFT of length R on u[0..R-1] (natural order in and out).
template <int R, int DIR>
struct Dft;

template <int DIR>
struct Dft<1, DIR> {
    __device__ __forceinline__ static void run(float2 *) {}
};

template <int DIR>
struct Dft<2, DIR> {
    __device__ __forceinline__ static void run(float2 *u) {
        float2 a = u[0];
        u[0] = cadd(a, u[1]);
        u[1] = csub(a, u[1]);
    }
};

template <int DIR>
struct Dft<4, DIR> {
    __device__ __forceinline__ static void run(float2 *u) {
        float2 t0 = cadd(u[0], u[2]);
        float2 t1 = csub(u[0], u[2]);
        float2 t2 = cadd(u[1], u[3]);
        float2 t3 = rot90<DIR>(csub(u[1], u[3]));
        u[0] = cadd(t0, t2);
        u[2] = csub(t0, t2);
        u[1] = cadd(t1, t3);
        u[3] = csub(t1, t3);
    }
};

// radix-2 split of an even-length DFT: even/odd halves, then combine
template <int R, int DIR>
struct Dft {
    static_assert(R == 8 || R == 16, "radix");
    __device__ __forceinline__ static void run(float2 *u) {
        float2 e[R / 2], o[R / 2];
#pragma unroll
        for (int i = 0; i < R / 2; ++i) {
            e[i] = u[2 * i];
            o[i] = u[2 * i + 1];
        }
        Dft<R / 2, DIR>::run(e);
        Dft<R / 2, DIR>::run(o);
        combine<0>(u, e, o);
    }
    template <int K>
    __device__ __forceinline__ static void combine(float2 *u, const float2 *e, const float2 *o) {
        if constexpr (K < R / 2) {
            float2 t = tw16<K * (16 / R), DIR>(o[K]);
            u[K] = cadd(e[K], t);
            u[K + R / 2] = csub(e[K], t);
            combine<K + 1>(u, e, o);
        }
    }
};

// ------------------------------------------------------- size configuration --
// A transform plan: N points, E elements per thread (T = N/E threads per
// transform) and the radices of the forward passes (the inverse runs them in
// reverse).  Every radix divides E.
template <int N, int E>
struct FftCfg {
    static constexpr int T = N / E;
    static constexpr int R0 = (N == 8) ? 8 : (N == 16) ? 16 : (N == 32) ? 8 : (N == 64) ? 8
                            : (N == 512) ? 8 : (N == 2048) ? 16 : (E == 16 ? 16 : 8);
    static constexpr int R1 = (N <= 16) ? 1 : (N == 32) ? 4 : (N == 64) ? 8 : (N == 128) ? (E == 16 ? 8 : 4)
                            : (N == 512) ? 8 : (N == 2048) ? 16 : (E == 16 ? 16 : 8);
    static constexpr int R2 = (N == 128 || N == 256) ? (E == 16 ? 1 : 4) : (N == 512) ? 8 : (N == 1024) ? 4
                            : (N == 2048) ? 8 : 1;
    static constexpr int R3 = (N == 1024 && E == 8) ? 4 : 1;
    static constexpr int P = 1 + (R1 > 1) + (R2 > 1) + (R3 > 1);
    static_assert(R0 * R1 * R2 * R3 == N, "radices must multiply to N");
    static_assert(E % R0 == 0 && E % R1 == 0 && E % R2 == 0 && E % R3 == 0, "every radix must divide E");
};

template <int N, int E, int DIR, int P>
struct Radix {
    using C = FftCfg<N, E>;
    static constexpr int fwd(int p) { return p == 0 ? C::R0 : p == 1 ? C::R1 : p == 2 ? C::R2 : C::R3; }
    static constexpr int value = DIR < 0 ? fwd(P) : fwd(C::P - 1 - P);
};

template <int N, int E, int DIR> struct FirstRadix { static constexpr int value = Radix<N, E, DIR, 0>::value; };
template <int N, int E, int DIR> struct LastRadix { static constexpr int value = Radix<N, E, DIR, FftCfg<N, E>::P - 1>::value; };

// Index (along the transform) of register e of thread t: with R the radix of
// the pass that reads (first) or writes (last) the registers,
// u[b*R + r] <-> x[t + b*T + r*N/R].
template <int N, int E, int R>
__device__ __forceinline__ constexpr int elem_index(int t, int e) {
    constexpr int T = N / E;
    return t + (e / R) * T + (e % R) * (N / R);
}
template <int N, int E, int DIR>
__device__ __forceinline__ int in_index(int t, int e) { return elem_index<N, E, FirstRadix<N, E, DIR>::value>(t, e); }
template <int N, int E, int DIR>
__device__ __forceinline__ int out_index(int t, int e) { return elem_index<N, E, LastRadix<N, E, DIR>::value>(t, e); }

// Twiddle table exp(-2 pi i m / 2048), m = 0..2047, filled once per device
// (read-only for kernels, so loads can be shared between probe modes).  Each
// translation unit that runs transforms holds its own copy (internal
// linkage) and fills it through its set_twiddles entry.
constexpr int TW_MAX = 2048;
namespace {
__constant__ float2 g_twiddle[TW_MAX];
}

template <int DIR>
__device__ __forceinline__ float2 twiddle(int m_of_table) {
    float2 w = g_twiddle[m_of_table];
    if constexpr (DIR > 0) w.y = -w.y;
    return w;
}

// w[r] = w1^r for r = 1..R-1 from one table load, by a balanced product tree
// (at most 4 multiplications deep).
template <int R, int DIR>
__device__ __forceinline__ void twiddle_powers(int m_of_table, float2 *w) {
    w[1] = twiddle<DIR>(m_of_table);
    if constexpr (R > 2) {
        w[2] = cmul(w[1], w[1]);
        w[3] = cmul(w[2], w[1]);
    }
    if constexpr (R > 4) {
        w[4] = cmul(w[2], w[2]);
        w[5] = cmul(w[4], w[1]);
        w[6] = cmul(w[4], w[2]);
        w[7] = cmul(w[4], w[3]);
    }
    if constexpr (R > 8) {
        w[8] = cmul(w[4], w[4]);
#pragma unroll
        for (int r = 9; r < 16; ++r) w[r] = cmul(w[8], w[r - 8]);
    }
}

// All passes of one length-N transform held by thread t (0 <= t < N/E).
// `Lds` provides ld(idx), st(idx, v) and sync() for this transform's
// private N-element exchange buffer.
template <int N, int E, int DIR, int P, int L, class Lds>
__device__ __forceinline__ void fft_pass(float2 *u, int t, Lds &lds) {
    using C = FftCfg<N, E>;
    constexpr int T = N / E, R = Radix<N, E, DIR, P>::value;
    if constexpr (P > 0) {
#pragma unroll
        for (int b = 0; b < E / R; ++b) {
            const int i = t + b * T;
#pragma unroll
            for (int r = 0; r < R; ++r) u[b * R + r] = lds.ld(i + r * (N / R));
        }
    }
#pragma unroll
    for (int b = 0; b < E / R; ++b) {
        if constexpr (L > 1) {
            const int i = t + b * T;
            const int k = i & (L - 1);
            // exp(DIR 2 pi i r k / (R L)) = (table[k * TW_MAX / (R L)])^r
            float2 w[R];
            twiddle_powers<R, DIR>(k * (TW_MAX / (R * L)), w);
#pragma unroll
            for (int r = 1; r < R; ++r) u[b * R + r] = cmul(u[b * R + r], w[r]);
        }
        Dft<R, DIR>::run(u + b * R);
    }
    if constexpr (P + 1 < C::P) {
        lds.sync();
#pragma unroll
        for (int b = 0; b < E / R; ++b) {
            const int i = t + b * T;
            const int k = i & (L - 1);
            const int j = (i - k) * R + k;
#pragma unroll
            for (int r = 0; r < R; ++r) lds.st(j + r * L, u[b * R + r]);
        }
        lds.sync();
        fft_pass<N, E, DIR, P + 1, L * R>(u, t, lds);
    }
}

template <int N, int E, int DIR, class Lds>
__device__ __forceinline__ void fft1d(float2 *u, int t, Lds &lds) {
    fft_pass<N, E, DIR, 0, 1>(u, t, lds);
}

// K independent transforms (one per probe mode) held by the same thread, run
// pass by pass together: one barrier pair and one set of twiddles per pass
// serve all K.  lds[k] is the exchange buffer of transform k.
template <int N, int E, int DIR, int P, int L, int K, class Lds>
__device__ __forceinline__ void fftk_pass(float2 (&u)[K][E], int t, Lds *lds) {
    using C = FftCfg<N, E>;
    constexpr int T = N / E, R = Radix<N, E, DIR, P>::value;
    if constexpr (P > 0) {
#pragma unroll
        for (int k = 0; k < K; ++k)
#pragma unroll
            for (int b = 0; b < E / R; ++b) {
                const int i = t + b * T;
#pragma unroll
                for (int r = 0; r < R; ++r) u[k][b * R + r] = lds[k].ld(i + r * (N / R));
            }
    }
#pragma unroll
    for (int b = 0; b < E / R; ++b) {
        if constexpr (L > 1) {
            const int i = t + b * T;
            const int q = i & (L - 1);
            float2 w[R];
            twiddle_powers<R, DIR>(q * (TW_MAX / (R * L)), w);
#pragma unroll
            for (int k = 0; k < K; ++k)
#pragma unroll
                for (int r = 1; r < R; ++r) u[k][b * R + r] = cmul(u[k][b * R + r], w[r]);
        }
#pragma unroll
        for (int k = 0; k < K; ++k) Dft<R, DIR>::run(u[k] + b * R);
    }
    if constexpr (P + 1 < C::P) {
        lds[0].sync();
#pragma unroll
        for (int b = 0; b < E / R; ++b) {
            const int i = t + b * T;
            const int q = i & (L - 1);
            const int j = (i - q) * R + q;
#pragma unroll
            for (int k = 0; k < K; ++k)
#pragma unroll
                for (int r = 0; r < R; ++r) lds[k].st(j + r * L, u[k][b * R + r]);
        }
        lds[0].sync();
        fftk_pass<N, E, DIR, P + 1, L * R, K>(u, t, lds);
    }
}

template <int N, int E, int DIR, int K, class Lds>
__device__ __forceinline__ void fftk(float2 (&u)[K][E], int t, Lds *lds) {
    fftk_pass<N, E, DIR, 0, 1, K>(u, t, lds);
}

// LDS exchange buffer for a transform along a contiguous row: element x of
// row `row` lives at row*(N + N/16) + x + x/16 (one pad slot per 16).
template <int N>
struct RowLds {
    float2 *base;
    __device__ __forceinline__ RowLds(float2 *lds, int row) : base(lds + row * (N + N / 16)) {}
    __device__ __forceinline__ float2 ld(int x) const { return base[x + (x >> 4)]; }
    __device__ __forceinline__ void st(int x, float2 v) { base[x + (x >> 4)] = v; }
    __device__ __forceinline__ void sync() const { __syncthreads(); }
    static constexpr int floats2_per_row = N + N / 16;
};

// LDS exchange buffer for a transform along a column: element y of local
// column `col` lives at row v(y), column col, rows CB float2 wide.  v permutes
// y within aligned groups of G = 32/CB rows (the rows one 64-bank cycle
// holds) by an XOR of higher bits, so that lanes whose rows differ by 1, 4 or
// 8 - the strides of the radix-8/4 passes - hit distinct bank groups.
template <int N, int CB>
struct ColLds {
    static constexpr int G = (CB >= 32) ? 1 : 32 / CB;
    float2 *base;
    ColLds() = default;
    __device__ __forceinline__ ColLds(float2 *lds, int col) : base(lds + col) {}
    __device__ __forceinline__ static int row(int y) {
        if constexpr (G == 1) return y;
        else return (y & ~(G - 1)) | ((y ^ (y >> 2) ^ (y >> 3)) & (G - 1));
    }
    __device__ __forceinline__ float2 ld(int y) const { return base[row(y) * CB]; }
    __device__ __forceinline__ void st(int y, float2 v) { base[row(y) * CB] = v; }
    __device__ __forceinline__ void sync() const { __syncthreads(); }
    static constexpr int floats2 = N * CB;
};

}  // namespace ptycho
