// stack_kernels.hpp - the frame-size templated kernels of one stack: the row
// passes, the column pass and the plain batched FFT.  Each frame size is
// instantiated in a translation unit of its own (inst_N.hip).
#pragma once

#include "common.hpp"

namespace ptycho {

// ============================================================ row passes ===

// Forward row FFT of the stack's exit waves.  Block = RB consecutive rows of
// the flattened (slot, y) row index of one probe mode (blockIdx.y); thread =
// (row, t).  The object view is re-read per mode from the caches.
template <int N, int MODE, bool NF, bool SUB>
__global__ __launch_bounds__(256) void k_rows_fwd(StackArgs a) {
    using G = RowGeom<N>;
    constexpr int E = G::E, T = G::T, RB = G::RB;
    __shared__ float2 lds[G::LDS_F2];
    const int tid = threadIdx.x, rr = tid / T, t = tid % T;
    const int k = blockIdx.y;
    const int g = xcd_block(blockIdx.x, gridDim.x) * RB + rr;
    const bool active = g < a.S * N;
    const int gg = active ? g : a.S * N - 1;
    const int s = gg / N, y = gg % N;
    const int j = a.order[a.s0 + s];
    const int2 o = a.offs[j];
    const size_t orow = (size_t)(o.x + y) * a.Nx + o.y;
    RowLds<N> L(lds, rr);
    // line search: A = P O, B = P dO + dP O, C = dP dO; IN_LS2 forms B and C
    // only (A is the gradient pass's kept row transform)
    constexpr bool LSM = (MODE == IN_LS) || (MODE == IN_LS2);
    constexpr int SETS = (MODE == IN_LS) ? 3 : (MODE == IN_LS2) ? 2 : 1;
    const float2 *prow = a.probe + ((size_t)k * N + y) * N;
    const float2 *drow = LSM ? a.dprobe + ((size_t)k * N + y) * N : nullptr;
    // The three line-search rows held together need 3E complex registers;
    // at 2048 points each set is formed and transformed on its own instead
    // (the object and probe rows are read again, from the caches).
    constexpr bool SPLIT = LSM && N >= 2048;
    float2 u[SPLIT ? 1 : SETS][E];
    // the object view (and the line search's direction view) at column x:
    // integer windows read the row, sub-pixel windows (SUB) interpolate
    ViewRow vr{};
    if constexpr (SUB) vr = view_row(a.Ny, a.Nx, o, a.frac[j], y);
#pragma unroll
    for (int set = 0; set < SETS; ++set) {
        const int sl = SPLIT ? 0 : set;
        auto fill = [&](auto view) {
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const int x = in_index<N, E, -1>(t, e);
                const float2 ov = view(a.obj, x);
                const float2 p = prow[x];
                if constexpr (SPLIT) {
                    const float2 dv = view(a.dobj, x), dp = drow[x];
                    const int q = (MODE == IN_LS2) ? set + 1 : set;
                    u[0][e] = q == 0 ? cmul(ov, p) : q == 1 ? cadd(cmul(dv, p), cmul(ov, dp)) : cmul(dv, dp);
                } else if constexpr (MODE == IN_LS2) {
                    const float2 dv = view(a.dobj, x);
                    const float2 dp = drow[x];
                    u[0][e] = cadd(cmul(dv, p), cmul(ov, dp));
                    u[1][e] = cmul(dv, dp);
                } else if constexpr (MODE == IN_LS) {
                    const float2 dv = view(a.dobj, x);
                    const float2 dp = drow[x];
                    u[0][e] = cmul(ov, p);
                    u[1][e] = cadd(cmul(dv, p), cmul(ov, dp));
                    u[2][e] = cmul(dv, dp);
                } else if constexpr (MODE == IN_DM) {
                    const float2 phi = cmul(ov, p);
                    // the old exit waves are read once: non-temporal
                    const float2 ps = ld_stream(a.psi + (((size_t)j * a.K + k) * N + y) * N + x);
                    u[0][e] = make_float2(2.0f * phi.x - ps.x, 2.0f * phi.y - ps.y);
                } else {
                    u[0][e] = cmul(ov, p);
                }
            }
        };
        if (SPLIT || set == 0) {
            if constexpr (SUB) fill([&](const float2 *b, int x) { return view_at(b, vr, x); });
            else fill([&](const float2 *b, int x) { return b[orow + x]; });
        }
        const int tt = SPLIT ? opaque(t) : t;
        fft1d<N, E, -1>(u[sl], tt, L);
        if constexpr (NF) {
            // Dx: the x factor of the transfer function, then back to x
            const float2 *qx = a.prop + N;
            const int t1 = opaque(tt);
#pragma unroll
            for (int e = 0; e < E; ++e) u[sl][e] = cmul(u[sl][e], qx[out_index<N, E, -1>(t1, e)]);
            fft1d<N, E, +1>(u[sl], t1, L);
        }
        float2 *dst = (MODE == IN_PHI ? a.fwd : a.scr) + ((size_t)s * SETS * a.K + set * a.K + k) * N * N;
        if (active) {
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const int x = NF ? out_index<N, E, +1>(t, e) : out_index<N, E, -1>(t, e);
                st_stream(dst + scr_at<N>(y, x), u[sl][e]);
            }
        }
    }
}


// Inverse row FFT of the stack scratch and the real-space epilogue.  A block
// has TPM threads (whole wavefronts) per probe mode, all on the same RQ rows.
// Outputs:
// OUT_SCR the exit waves back into the scratch, OUT_STORE into psi_out
// [J][K][N][N], OUT_DM Phi + u into psi_out, OUT_NONE nothing.  With WQ the
// block also writes q = sum_k conj(P_k) Psi_k (the modes summed through LDS),
// the frame's term of the object numerator, to qbuf, so that the object
// gather reads one plane per frame instead of K exit waves and K probe
// values.
template <int N, int K, int MODE, bool WQ, bool NF, bool SUB>
__global__ __launch_bounds__(InvRowGeom<N>::TPM * K) void k_rows_inv(StackArgs a) {
    using G = InvRowGeom<N>;
    constexpr int E = G::E, T = G::T, RQ = G::RQ;
    __shared__ float2 lds[K * RQ * G::ROW_F2];
    const int k = threadIdx.x / G::TPM, lane = threadIdx.x % G::TPM, rr = lane / T, t = lane % T;
    const int g = xcd_block(blockIdx.x, gridDim.x) * RQ + rr;
    const bool active = g < a.S * N;
    const int gg = active ? g : a.S * N - 1;
    const int s = gg / N, y = gg % N;
    const int j = a.order[a.s0 + s];
    RowLds<N> L(lds, k * RQ + rr);

    float2 *src = a.scr + ((size_t)s * K + k) * N * N;
    float2 u[E];
#pragma unroll
    for (int e = 0; e < E; ++e)          // read once: non-temporal, the caches keep the views and the probe
        u[e] = ld_stream(src + scr_at<N>(y, NF ? in_index<N, E, -1>(t, e) : in_index<N, E, +1>(t, e)));
    if constexpr (NF) {
        // Dx^-1: forward transform, the conjugate x factor, inverse below
        fft1d<N, E, -1>(u, t, L);
        const float2 *qx = a.prop + N;
#pragma unroll
        for (int e = 0; e < E; ++e) u[e] = cmulc(qx[out_index<N, E, -1>(t, e)], u[e]);
    }
    const float2 *prow = a.probe + ((size_t)k * N + y) * N;
    const size_t prow_psi = (((size_t)j * K + k) * N + y) * N;
    size_t orow = 0;
    if constexpr (MODE == OUT_DM) {
        const int2 o = a.offs[j];
        orow = (size_t)(o.x + y) * a.Nx + o.y;
    }
    ViewRow vr{};
    if constexpr (SUB) vr = view_row(a.Ny, a.Nx, a.offs[j], a.frac[j], y);
    // The DM form loads the object view and the probe row before the
    // transform, so that their latency overlaps its passes (loads cannot move
    // across the transform's barriers): measured 10% faster at 256 points
    // with 3 modes and 22% at 512 with 4.  Sub-pixel views (four object
    // values per pixel) and the near field would hold too many registers.
    constexpr bool PF = MODE == OUT_DM && !NF && !SUB;
    constexpr bool PP = PF;
    float2 ovp[PF ? E : 1], pvp[PP ? E : 1];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int x = out_index<N, E, +1>(t, e);
        if constexpr (PF) ovp[e] = SUB ? view_at(a.obj, vr, x) : a.obj[orow + x];
        if constexpr (PP) pvp[e] = prow[x];
    }
    fft1d<N, E, +1>(u, t, L);
    float2 qk[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int x = out_index<N, E, +1>(t, e);
        float2 v = u[e];
        float2 pe;
        if constexpr (PP) pe = pvp[e];
        else pe = prow[x];
        if constexpr (MODE == OUT_DM) {
            float2 oe;
            if constexpr (PF) oe = ovp[e];
            else oe = SUB ? view_at(a.obj, vr, x) : a.obj[orow + x];
            if (active) v = cadd(cmul(oe, pe), v);
        }
        if (active) {
            if constexpr (MODE == OUT_SCR) src[scr_at<N>(y, x)] = v;
            if constexpr (MODE == OUT_STORE || MODE == OUT_DM) st_stream(a.psi_out + prow_psi + x, v);
        }
        if constexpr (WQ) qk[e] = cmulc(pe, v);
    }
    if constexpr (WQ) {
        __syncthreads();                 // the transforms' LDS reads are done
#pragma unroll
        for (int e = 0; e < E; ++e) L.st(out_index<N, E, +1>(t, e), qk[e]);
        __syncthreads();
        // the threads of mode k sum and write the pixels of their elements
        // e = k, k + K, ...
        if (active) {
            float2 *qrow = a.qbuf + ((size_t)s * N + y) * N;
#pragma unroll
            for (int e = 0; e < E; ++e) {
                if (e % K != k) continue;
                const int x = out_index<N, E, +1>(t, e);
                float2 q = RowLds<N>(lds, rr).ld(x);
#pragma unroll
                for (int m = 1; m < K; ++m) q = cadd(q, RowLds<N>(lds, m * RQ + rr).ld(x));
                st_stream(qrow + x, q);
            }
        }
    }
}
// ========================================================== column pass ===
// OP_CORR writes (s - 1) F(X) instead of s F(X): since P_F(X) = X + F^-1((s-1) F(X))
// (s = 1 at bad pixels), the DM update Psi + P_F(2 Phi - Psi) - Phi equals
// Phi + F^-1((s - 1) F(2 Phi - Psi)), which the inverse row pass forms from the
// views alone, without reading the old exit waves again.

// Exchange buffers of the read-only column pass: the line search's three
// transforms of a mode run pass by pass together while their buffers fit
// 96 KiB of LDS, one after the other through one buffer beyond that.
template <int N, int OP>
struct ColSeqBufs {
    static constexpr int SETS = (OP == OP_LS || OP == OP_LS2) ? 3 : 1;
    static constexpr int value = ((size_t)SETS * ColGeom<N>::LDS_F2 * 8 <= 96 * 1024) ? SETS : 1;
};

// Waves per SIMD a column kernel is compiled for: the DM form with up to 3
// modes fits 128 registers without spilling, which gives 4 waves instead of
// 3 (measured faster); the near-field pass at 2048 points with one mode gets
// 4 waves too, so that two of its 512-thread blocks share a CU (a 32-byte
// spill; measured faster); the others keep the compiler's choice.
template <int N, int K, int OP, bool NF>
struct ColMinWaves {
    static constexpr int value = ((!NF && ColJoint<N, K>::SEQ && N <= 256 && K <= 3 && OP == OP_CORR) ||
                                  (NF && N >= 2048 && K == 1)) ? 4 : 1;
};

// Row (y) index of register e of thread t at the detector-plane step: after
// the forward transform in the far field (a frequency), after the forward
// and inverse transforms in the near field (a pixel).
template <int N, int E, bool NF>
__device__ __forceinline__ int det_row(int t, int e) {
    return NF ? in_index<N, E, -1>(t, e) : out_index<N, E, -1>(t, e);
}

// The column transforms of all K modes, forward (DIR -1) or inverse (+1):
// joint pass by pass, or one mode after the other through one buffer.
template <int N, int E, int DIR, int K, bool SEQ, class Lds>
__device__ __forceinline__ void col_transforms(float2 (&u)[K][E], int t, Lds *L) {
    if constexpr (SEQ) {
        __syncthreads();     // earlier transforms' last LDS reads are done
#pragma unroll
        for (int k = 0; k < K; ++k) fft1d<N, E, DIR>(u[k], t, L[k]);
    } else {
        fftk<N, E, DIR, K>(u, t, L);
    }
}

// Near field: multiply the column spectra by Qy (CONJ: its conjugate).
template <int N, int E, int K, int NSET, bool CONJ>
__device__ __forceinline__ void apply_qy(float2 (&u)[K][E], const float2 *qy, int t) {
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const float2 w = qy[out_index<N, E, -1>(t, e)];
#pragma unroll
        for (int k = 0; k < NSET; ++k) u[k][e] = CONJ ? cmulc(w, u[k][e]) : cmul(u[k][e], w);
    }
}

// Column FFTs of all K modes held together in registers, the Fourier-space
// step and (project / grad) the inverse column FFTs, written back in place.
template <int N, int K, int OP, bool NF>
__global__ __launch_bounds__(ColGeom<N>::THREADS, (ColMinWaves<N, K, OP, NF>::value)) void k_cols_joint(StackArgs a) {
    using G = ColGeom<N>;
    constexpr int E = G::E, CB = G::CB;
    extern __shared__ float2 lds_dyn[];
    const int tid = threadIdx.x, cl = tid % CB, t = tid / CB;
    const int blk = xcd_block(blockIdx.x, gridDim.x);
    const int g = blk * CB + cl;
    const bool active = g < a.S * N;
    const int gg = active ? g : a.S * N - 1;
    const int s = gg / N, c = gg % N;
    const int j = a.order[a.s0 + s];
    constexpr bool SEQ = ColJoint<N, K>::SEQ;
    ColLds<N, CB> L[K];
#pragma unroll
    for (int k = 0; k < K; ++k) L[k] = ColLds<N, CB>(lds_dyn + (SEQ ? 0 : k) * G::LDS_F2, cl);
    // far field: the unitary 1/N^2 of the forward and inverse 2D transforms;
    // near field: folded into the transfer-function factors
    constexpr float nrm = NF ? 1.0f : 1.0f / ((float)N * (float)N);

    // far field from 512 points (two waves per SIMD, latency-bound) the stack
    // is read non-temporally: 4000 x 512^2 x 4 modes, columns 25.2 -> 23.8 ms
    // per DM cycle; at 256 points it made the pass 5% slower
    constexpr bool NT = !NF && N >= 512;
    float2 u[K][E];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const float2 *src = a.colin + ((size_t)(s * K + k) * N) * N + scr_at<N>(0, c);
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const float2 *at = src + in_index<N, E, -1>(t, e) * ScrTile<N>::W;
            u[k][e] = NT ? ld_stream(at) : *at;
        }
    }
    // the data of the pixels this thread will own after the transform are
    // loaded now: loads cannot move across the transform's barriers
    const float *io = a.iobs + (size_t)j * N * N + c;
    float iobv[E];
    bool badv[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int q = det_row<N, E, NF>(t, e);
        iobv[e] = io[(size_t)q * N];
        badv[e] = a.mask != nullptr && a.mask[q * N + c] != 0;
    }
    col_transforms<N, E, -1, K, SEQ>(u, t, L);
    if constexpr (NF) {
        // Dy: to the detector plane
        const int t1 = opaque(t);
        apply_qy<N, E, K, K, false>(u, a.prop, t1);
        col_transforms<N, E, +1, K, SEQ>(u, t1, L);
    }

    double acc = 0.0;
#pragma unroll
    for (int e = 0; e < E; ++e) {
        float inten = 0.0f;
#pragma unroll
        for (int k = 0; k < K; ++k) inten += cnorm(u[k][e]);
        // the background (L2-resident, usually absent) is read here rather
        // than with Iobs, so that it holds no registers across the transform
        inten = inten * nrm + (a.bg != nullptr ? a.bg[det_row<N, E, NF>(t, e) * N + c] : 0.0f);
        const bool bad = badv[e];
        const float iob = iobv[e];
        float sc;
        if constexpr (OP == OP_PROJECT) {
            const float r = iob / fmaxf(inten, a.eps);
            sc = bad ? nrm : sqrtf(r) * nrm;
            if (a.s2 != nullptr && active) a.s2[((size_t)s * N + det_row<N, E, NF>(t, e)) * N + c] = bad ? 1.0f : r;
        } else if constexpr (OP == OP_CORR) {
            sc = bad ? 0.0f : (sqrtf(iob / fmaxf(inten, a.eps)) - 1.0f) * nrm;
        } else {
            const float ifl = fmaxf(inten, a.eps);
            sc = bad ? 0.0f : (1.0f - iob / ifl) * nrm;
            if (!bad && active) acc += (double)llk_term(ifl, iob);
        }
#pragma unroll
        for (int k = 0; k < K; ++k) u[k][e] = cscale(u[k][e], sc);
    }
    const int t3 = NF ? opaque(t) : t;
    if constexpr (NF) {
        // Dy^-1: back from the detector plane (the inverse transform below)
        const int t2 = opaque(t);
        col_transforms<N, E, -1, K, SEQ>(u, t2, L);
        apply_qy<N, E, K, K, true>(u, a.prop, t2);
    }
    col_transforms<N, E, +1, K, SEQ>(u, t3, L);
    if (active) {
#pragma unroll
        for (int k = 0; k < K; ++k) {
            float2 *dst = a.scr + ((size_t)(s * K + k) * N) * N + scr_at<N>(0, c);
#pragma unroll
            for (int e = 0; e < E; ++e) dst[out_index<N, E, +1>(t, e) * ScrTile<N>::W] = u[k][e];
        }
    }
    if constexpr (OP == OP_GRAD) {
        const double r = block_sum(acc);
        if (threadIdx.x == 0) a.red[blk] = r;
    }
}

// Column FFTs one mode at a time for the read-only Fourier-space steps:
// LLK, calculated intensity, and the line-search terms I0, I1, I2.  The
// transforms' inputs are read once, non-temporally (line search at 500 x
// 256^2 x 3 modes: ML cycle 2.34 -> 2.31 ms).
template <int N, int OP, bool NF>
__global__ __launch_bounds__(ColGeom<N>::THREADS) void k_cols_seq(StackArgs a) {
    using G = ColGeom<N>;
    constexpr int E = G::E, CB = G::CB;
    extern __shared__ float2 lds_dyn[];
    const int tid = threadIdx.x, cl = tid % CB, t = tid / CB;
    const int blk = xcd_block(blockIdx.x, gridDim.x);
    const int g = blk * CB + cl;
    const bool active = g < a.S * N;
    const int gg = active ? g : a.S * N - 1;
    const int s = gg / N, c = gg % N;
    const int j = a.order[a.s0 + s];
    constexpr float nrm = NF ? 1.0f : 1.0f / ((float)N * (float)N);
    constexpr int SETS = ColSeqBufs<N, OP>::SETS;
    constexpr bool ONE_BUF = ColSeqBufs<N, OP>::value == 1 && SETS > 1;

    float i0[E], i1[E], i2[E];
#pragma unroll
    for (int e = 0; e < E; ++e) i0[e] = i1[e] = i2[e] = 0.0f;
    // the SETS transforms of a mode run pass by pass together
    ColLds<N, CB> Ls[SETS];
#pragma unroll
    for (int set = 0; set < SETS; ++set) Ls[set] = ColLds<N, CB>(lds_dyn + (ONE_BUF ? 0 : set) * G::LDS_F2, cl);
    // set `set` of mode k: A from the kept row transforms (OP_LS2) or the
    // scratch, B and C from the scratch
    auto src_of = [&](int set, int k) -> const float2 * {
        if constexpr (OP == OP_LS2) {
            if (set == 0) return a.colin + ((size_t)(s * a.K + k) * N) * N + scr_at<N>(0, c);
            return a.scr + ((size_t)(s * 2 * a.K + (set - 1) * a.K + k) * N) * N + scr_at<N>(0, c);
        }
        return a.colin + ((size_t)(s * SETS * a.K + set * a.K + k) * N) * N + scr_at<N>(0, c);
    };
    for (int k = 0; k < a.K; ++k) {
        if constexpr (ONE_BUF) {
            // one transform at a time (large N): keep A, fold B and C into
            // the sums as soon as each is transformed
            float2 A[1][E], V[1][E];
            auto load_transform = [&](float2 (&v)[1][E], int set) {
                const float2 *src = src_of(set, k);
#pragma unroll
                for (int e = 0; e < E; ++e) v[0][e] = ld_stream(src + in_index<N, E, -1>(t, e) * ScrTile<N>::W);
                const int t0 = opaque(t);
                col_transforms<N, E, -1, 1, false>(v, t0, Ls);
                if constexpr (NF) {
                    const int t1 = opaque(t);
                    apply_qy<N, E, 1, 1, false>(v, a.prop, t1);
                    col_transforms<N, E, +1, 1, false>(v, t1, Ls);
                }
            };
            load_transform(A, 0);
            load_transform(V, 1);
#pragma unroll
            for (int e = 0; e < E; ++e) {
                i0[e] += cnorm(A[0][e]);
                i1[e] += 2.0f * cmulc(A[0][e], V[0][e]).x;
                i2[e] += cnorm(V[0][e]);
            }
            load_transform(V, 2);
#pragma unroll
            for (int e = 0; e < E; ++e) i2[e] += 2.0f * cmulc(A[0][e], V[0][e]).x;
            continue;
        }
        float2 u[SETS][E];
#pragma unroll
        for (int set = 0; set < SETS; ++set) {
            const float2 *src = src_of(set, k);
#pragma unroll
            for (int e = 0; e < E; ++e) u[set][e] = ld_stream(src + in_index<N, E, -1>(t, e) * ScrTile<N>::W);
        }
        col_transforms<N, E, -1, SETS, ONE_BUF>(u, t, Ls);
        if constexpr (NF) {
            const int t1 = opaque(t);
            apply_qy<N, E, SETS, SETS, false>(u, a.prop, t1);
            col_transforms<N, E, +1, SETS, ONE_BUF>(u, t1, Ls);
        }
#pragma unroll
        for (int e = 0; e < E; ++e) {
            i0[e] += cnorm(u[0][e]);
            if constexpr (OP == OP_LS || OP == OP_LS2) {
                const float2 ab = cmulc(u[0][e], u[1][e]);
                const float2 ac = cmulc(u[0][e], u[2][e]);
                i1[e] += 2.0f * ab.x;
                i2[e] += cnorm(u[1][e]) + 2.0f * ac.x;
            }
        }
    }
    const float *io = a.iobs + (size_t)j * N * N + c;
    double acc0 = 0.0, acc1 = 0.0;
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int q = det_row<N, E, NF>(t, e);
        const float inten = i0[e] * nrm + (a.bg != nullptr ? a.bg[q * N + c] : 0.0f);
        if constexpr (OP == OP_ICALC) {
            if (active) a.icalc[((size_t)j * N + q) * N + c] = inten;
        } else {
            const bool bad = a.mask != nullptr && a.mask[q * N + c] != 0;
            if (bad || !active) continue;
            const float iob = io[(size_t)q * N];
            const float ifl = fmaxf(inten, a.eps);
            if constexpr (OP == OP_LLK) {
                acc0 += (double)llk_model_term(a.llk_model, ifl, iob);
            } else {
                const float d1 = 1.0f - iob / ifl;
                const float d2 = (iob / ifl) / ifl;
                const float j1 = i1[e] * nrm, j2 = i2[e] * nrm;
                acc0 += (double)(d1 * j1);
                acc1 += (double)(d2 * j1 * j1 + 2.0f * d1 * j2);
            }
        }
    }
    if constexpr (OP == OP_LLK) {
        const double r = block_sum(acc0);
        if (threadIdx.x == 0) a.red[blk] = r;
    } else if constexpr (OP == OP_LS || OP == OP_LS2) {
        const double r0 = block_sum(acc0);
        const double r1 = block_sum(acc1);
        if (threadIdx.x == 0) {
            a.red[2 * blk] = r0;
            a.red[2 * blk + 1] = r1;
        }
    }
}

// Plain batched FFT along rows / columns (standalone 2D transform).  Both
// passes remap their blocks so that each XCD takes a contiguous range: the
// column blocks that share 128-byte row lines (and neighbouring rows) are then
// served by one L2 (2048-point frames: 3.9 -> 5.0 TB/s).
template <int N, int DIR>
__global__ __launch_bounds__(256) void k_fft_rows(float2 *data, long rows) {
    using G = RowGeom<N>;
    constexpr int E = G::E, T = G::T, RB = G::RB;
    __shared__ float2 lds[G::LDS_F2];
    const int tid = threadIdx.x, rr = tid / T, t = tid % T;
    const long g = (long)xcd_block(blockIdx.x, gridDim.x) * RB + rr;
    const bool active = g < rows;
    float2 *row = data + (size_t)(active ? g : rows - 1) * N;
    RowLds<N> L(lds, rr);
    float2 u[E];
#pragma unroll
    for (int e = 0; e < E; ++e) u[e] = row[in_index<N, E, DIR>(t, e)];
    fft1d<N, E, DIR>(u, t, L);
    if (active) {
#pragma unroll
        for (int e = 0; e < E; ++e) row[out_index<N, E, DIR>(t, e)] = u[e];
    }
}

// Geometry of the standalone column transform, which reads row-major frames:
// from 128 points up a block takes 16 adjacent columns (128-byte row
// segments; 8 at 2048 points), with 16 elements per thread from 1024 points
// so that the block stays within 1024 threads.
template <int N>
struct FftColGeom {
    static constexpr int E = (N >= 1024) ? 16 : col_e(N), T = N / E;
    static constexpr int CB = (N >= 2048) ? 8 : (N >= 128) ? 16 : col_cb(N);
    static constexpr int THREADS = CB * T;
    static constexpr int LDS_F2 = (FftCfg<N, E>::P > 1) ? N * CB : 1;
    static_assert(THREADS <= 1024, "one block");
};

template <int N, int DIR>
__global__ __launch_bounds__(FftColGeom<N>::THREADS) void k_fft_cols(float2 *data, long count, float scale) {
    using G = FftColGeom<N>;
    constexpr int E = G::E, CB = G::CB;
    extern __shared__ float2 lds_dyn[];
    const int tid = threadIdx.x, cl = tid % CB, t = tid / CB;
    const long g = (long)xcd_block(blockIdx.x, gridDim.x) * CB + cl;
    const bool active = g < count * N;
    const long gg = active ? g : count * N - 1;
    const long f = gg / N;
    const int c = (int)(gg % N);
    float2 *col = data + (size_t)f * N * N + c;
    ColLds<N, CB> L(lds_dyn, cl);
    float2 u[E];
#pragma unroll
    for (int e = 0; e < E; ++e) u[e] = col[(size_t)in_index<N, E, DIR>(t, e) * N];
    fft1d<N, E, DIR>(u, t, L);
    if (active) {
#pragma unroll
        for (int e = 0; e < E; ++e) col[(size_t)out_index<N, E, DIR>(t, e) * N] = cscale(u[e], scale);
    }
}


}  // namespace ptycho
