// kernels.hpp - gfx950 kernels of the ptychography hot path.
//
// One cycle over a stack of S frames runs as
//   rows_fwd : object view x probe (or 2*Phi - Psi for DM), 1D FFT along x
//              of every row of every mode -> stack scratch
//   cols     : 1D FFT along y of every column of every mode, the Fourier-space
//              step (modulus projection, ML gradient weighting, LLK, line
//              search terms), and the inverse 1D FFT along y, in registers
//   rows_inv : inverse 1D FFT along x and the real-space epilogue (AP: keep
//              the projected exit wave; DM: Psi + P_F(2Phi - Psi) - Phi)
//   gather_obj / gather_probe : overlap-update numerators and denominators,
//              each output pixel summed by exactly one thread in a fixed
//              frame order (no atomics, bitwise reproducible)
// and, once per cycle, max-reductions and the normalisation with inertia.
//
// Near field (template flag NF): the detector sees D = F^-1 Q F instead of F,
// with the Fresnel transfer function Q(u, v) = Qy(u) Qx(v) separable, so
// D = Dy Dx with Dx = F_x^-1 Qx F_x acting on rows alone and Dy on columns
// alone.  Each row or column pass then runs its forward transform, the
// transfer-function factor and the inverse transform back to back in
// registers, and the detector-plane step sits between the column pass's two
// propagations: the same three passes over memory as the far field, twice the
// transforms.
#pragma once

#include "fft.hpp"

namespace ptycho {

// ------------------------------------------------------------- geometry ---
// The size rules as plain functions of N (the host uses them for the
// workspace layout; the geometry structs below use them for the kernels).
constexpr int row_e(int n) { return (n >= 128 || n == 16) ? 16 : 8; }
constexpr int row_rb(int n) { return 256 / (n / row_e(n)); }
constexpr int col_e(int n) { return (n == 16 || n >= 2048) ? 16 : 8; }
constexpr int col_cb(int n) {
    return (n >= 1024) ? 4 : (n >= 256) ? 8 : ((256 / (n / col_e(n))) > 16 ? 256 / (n / col_e(n)) : 16);
}
constexpr int scr_tile_w(int n) { return col_cb(n) < n ? col_cb(n) : n; }

// Row transforms: 16 elements per thread from N = 128 up (fewer LDS passes),
// RB rows per 256-thread block.
template <int N, int E_ = row_e(N)>
struct RowGeom {
    static constexpr int E = E_, T = N / E, RB = 256 / T, THREADS = 256;
    static constexpr int LDS_F2 = (FftCfg<N, E>::P > 1) ? RB * (N + N / 16) : 1;
};
// The inverse row pass runs whole wavefronts per probe mode over the same RQ
// rows (one wavefront while a row has at most 64 threads, else T threads),
// so that the modes of a pixel meet in one block.
template <int N>
struct InvRowGeom {
    static constexpr int E = RowGeom<N>::E, T = N / E;
    static constexpr int TPM = T > 64 ? T : 64;     // threads per mode
    static constexpr int RQ = TPM / T;
    static constexpr int ROW_F2 = N + N / 16;        // one RowLds row
};
// Column transforms keep all K modes in registers at once, so they use 8
// elements per thread (16 at N = 16 and N = 2048), CB adjacent columns per
// block (a 128-byte row segment at CB = 16; 4 columns from N = 1024 keep the
// block at 512 threads, so that a thread may hold 256 registers).
template <int N>
struct ColGeom {
    static constexpr int E = col_e(N), T = N / E;
    static constexpr int CB = col_cb(N);
    static constexpr int THREADS = CB * T;
    static constexpr int LDS_F2 = (FftCfg<N, E>::P > 1) ? N * CB : 1;   // one transform buffer
};

// The joint column pass runs the K transforms pass by pass together (one
// barrier pair per pass, K exchange buffers) while their buffers fit 32 KiB
// of LDS; beyond that the transforms run one after the other through a
// single buffer: more barriers, but more blocks per CU and fewer registers
// (measured faster at 256 points with 3 modes and at 512 points).
template <int N, int K>
struct ColJoint {
    static constexpr bool SEQ = (size_t)K * ColGeom<N>::LDS_F2 * 8 > 32 * 1024;
    static constexpr int BUFS = SEQ ? 1 : K;
};

constexpr int ilog2(int v) { return v <= 1 ? 0 : 1 + ilog2(v / 2); }

// Layout of one frame-mode plane of the stack scratch: column tiles of W
// adjacent columns, each tile holding rows 0..N-1 of its W columns (W
// elements per row, rows consecutive).  A column block then reads and writes
// one contiguous N*W range, and each row pass writes, for every tile, runs
// of W elements over consecutive rows.  W = N is the row-major layout; the
// exit waves the caller stores are always row-major.
template <int N>
struct ScrTile {
    static constexpr int W = scr_tile_w(N);
    static constexpr int LW = ilog2(W);
    static_assert((1 << LW) == W, "tile width is a power of two");
};
template <int N>
__device__ __forceinline__ int scr_at(int y, int x) {
    constexpr int W = ScrTile<N>::W;
    return ((x / W) * N + y) * W + (x % W);
}
// The same with the tile width's log2 known at run time (lw = log2 N: row-major).
__device__ __forceinline__ size_t tiled_at(int y, int x, int n, int lw) {
    return ((size_t)((x >> lw) * n + y) << lw) + (x & ((1 << lw) - 1));
}

// Blocks are dispatched to the 8 XCDs round-robin (block i on XCD i % 8), each
// XCD with its own L2.  This remap gives every XCD a contiguous range of
// logical blocks, so neighbouring column blocks that share 128-byte lines
// (and neighbouring rows of one frame) are served by the same L2.
__device__ __forceinline__ int xcd_block(int b, int nb) {
    const int full = nb & ~7;
    if (b >= full) return b;
    return (b & 7) * (full >> 3) + (b >> 3);
}

// Streaming load: data read once (exit waves in the gathers) are marked
// non-temporal so that they do not evict the data the gathers reuse from L2
// (the probe, the object rows).
__device__ __forceinline__ float2 ld_stream(const float2 *p) {
    return make_float2(__builtin_nontemporal_load(&p->x), __builtin_nontemporal_load(&p->y));
}

// Streaming store: data written once and not read again before much more
// has passed through the caches: the exit waves, the forward rows' stack and
// the per-frame object terms.  (The column pass's output, read by the next
// pass right away, is stored normally: measured faster.)
__device__ __forceinline__ void st_stream(float2 *p, float2 v) {
    __builtin_nontemporal_store(v.x, &p->x);
    __builtin_nontemporal_store(v.y, &p->y);
}

// An opaque copy of an index: transforms chained back to back (near field)
// then cannot share their twiddle loads, which would keep the twiddles of one
// transform in registers through the next ones.
__device__ __forceinline__ int opaque(int v) {
    asm volatile("" : "+v"(v));
    return v;
}

// Object tile of the atomic-free object gather.
constexpr int OTILE_Y = 16, OTILE_X = 64;

// ------------------------------------------------------------ arguments ---
struct StackArgs {
    int Ny, Nx, K, S, s0;
    const int2 *offs;            // [J] (oy, ox)
    const int *order;            // slot -> frame
    const float2 *obj, *probe;
    const float2 *dobj, *dprobe; // line-search direction
    const float2 *psi;           // DM state read  [J][K][N][N]
    float2 *psi_out;             // DM state write [J][K][N][N]
    float2 *scr;                 // stack scratch [S][sets*K][N][N] (column tiles)
    float2 *qbuf;                // per slot sum_k conj(P_k) Psi_k, [S][N][N] row-major
    const float *iobs;           // [J][N][N]
    const float *bg;             // incoherent background [N][N] or null
    float *s2;                   // AP background refinement: s^2 per slot [S][N][N], or null
    const unsigned char *mask;   // [N][N] or null
    const float2 *prop;          // near field: [2][N] Qy(u) / N, Qx(v) / N (FFT order), or null
    float *icalc;                // [J][N][N] (icalc op)
    double *red;                 // per-block partial sums of this launch
    float eps;
    int llk_model;               // noise model of OP_LLK (LlkModel)
};


// --------------------------------------------------------- reductions -----
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    return v;
}
__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_down(v, o, 64));
    return v;
}
// Fixed-order block sum; result valid in thread 0.
__device__ __forceinline__ double block_sum(double v) {
    __shared__ double sh[16];
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sh[w] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < (int)(blockDim.x + 63) / 64; ++i) r += sh[i];
    return r;
}
__device__ __forceinline__ float block_max(float v) {
    __shared__ float shm[16];
    v = wave_max(v);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) shm[w] = v;
    __syncthreads();
    float r = 0.0f;
    for (int i = 0; i < (int)(blockDim.x + 63) / 64; ++i) r = fmaxf(r, shm[i]);
    return r;   // valid in every thread
}

// Poisson term I - Iobs + Iobs ln(Iobs/I) computed as I f(t), t = (Iobs-I)/I,
// f(t) = (1+t) log1p(t) - t, with the series t^2/2 - t^3/6 + t^4/12 for
// |t| < 1e-2 so that fp32 keeps its relative accuracy near a perfect fit.
__device__ __forceinline__ float llk_term(float inten, float iob) {
    if (iob <= 0.0f) return inten;
    const float t = (iob - inten) / inten;
    float f;
    if (fabsf(t) < 1e-2f) f = t * t * (0.5f - t * (1.0f / 6.0f - t * (1.0f / 12.0f)));
    else f = (1.0f + t) * log1pf(t) - t;
    return inten * f;
}

// Noise models of the reported likelihood, each the negative log-density
// difference to a perfect fit: Poisson (above), Gaussian with variance
// Iobs + 1, and Gaussian amplitudes with variance 1/4 ("Euclidean"), whose
// difference of square roots is formed as (I - Iobs) / (sqrt I + sqrt Iobs)
// to keep fp32 accuracy near the fit.
enum LlkModel { LLK_POISSON = 0, LLK_GAUSSIAN = 1, LLK_EUCLIDEAN = 2 };
__device__ __forceinline__ float llk_model_term(int model, float inten, float iob) {
    if (model == LLK_GAUSSIAN) {
        const float d = inten - iob;
        return d * d / (2.0f * (iob + 1.0f));
    }
    if (model == LLK_EUCLIDEAN) {
        const float ob = fmaxf(iob, 0.0f);
        const float den = sqrtf(inten) + sqrtf(ob);
        const float a = den > 0.0f ? (inten - ob) / den : 0.0f;
        return 2.0f * a * a;
    }
    return llk_term(inten, iob);
}

// ============================================================ row passes ===
enum RowIn { IN_PHI = 0, IN_DM = 1, IN_LS = 2, IN_DATA = 3 };

// Forward row FFT of the stack's exit waves.  Block = RB consecutive rows of
// the flattened (slot, y) row index of one probe mode (blockIdx.y); thread =
// (row, t).  The object view is re-read per mode from the caches.
template <int N, int MODE, bool NF>
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
    constexpr int SETS = (MODE == IN_LS) ? 3 : 1;
    const float2 *prow = a.probe + ((size_t)k * N + y) * N;
    const float2 *drow = (MODE == IN_LS) ? a.dprobe + ((size_t)k * N + y) * N : nullptr;
    // The three line-search rows held together need 3E complex registers;
    // at 2048 points each set is formed and transformed on its own instead
    // (the object and probe rows are read again, from the caches).
    constexpr bool SPLIT = (MODE == IN_LS) && N >= 2048;
    float2 u[SPLIT ? 1 : SETS][E];
#pragma unroll
    for (int set = 0; set < SETS; ++set) {
        const int sl = SPLIT ? 0 : set;
        if (SPLIT || set == 0) {
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const int x = in_index<N, E, -1>(t, e);
                const float2 ov = a.obj[orow + x];
                const float2 p = prow[x];
                if constexpr (SPLIT) {
                    const float2 dv = a.dobj[orow + x], dp = drow[x];
                    u[0][e] = set == 0 ? cmul(ov, p) : set == 1 ? cadd(cmul(dv, p), cmul(ov, dp)) : cmul(dv, dp);
                } else if constexpr (MODE == IN_LS) {
                    const float2 dv = a.dobj[orow + x];
                    const float2 dp = drow[x];
                    u[0][e] = cmul(ov, p);
                    u[1][e] = cadd(cmul(dv, p), cmul(ov, dp));
                    u[2][e] = cmul(dv, dp);
                } else if constexpr (MODE == IN_DM) {
                    const float2 phi = cmul(ov, p);
                    const float2 ps = a.psi[(((size_t)j * a.K + k) * N + y) * N + x];
                    u[0][e] = make_float2(2.0f * phi.x - ps.x, 2.0f * phi.y - ps.y);
                } else {
                    u[0][e] = cmul(ov, p);
                }
            }
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
        float2 *dst = a.scr + ((size_t)s * SETS * a.K + set * a.K + k) * N * N;
        if (active) {
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const int x = NF ? out_index<N, E, +1>(t, e) : out_index<N, E, -1>(t, e);
                st_stream(dst + scr_at<N>(y, x), u[sl][e]);
            }
        }
    }
}

enum RowOut { OUT_SCR = 0, OUT_DM = 1, OUT_STORE = 2, OUT_NONE = 3 };

// Inverse row FFT of the stack scratch and the real-space epilogue.  A block
// has TPM threads (whole wavefronts) per probe mode, all on the same RQ rows.
// Outputs:
// OUT_SCR the exit waves back into the scratch, OUT_STORE into psi_out
// [J][K][N][N], OUT_DM Phi + u into psi_out, OUT_NONE nothing.  With WQ the
// block also writes q = sum_k conj(P_k) Psi_k (the modes summed through LDS),
// the frame's term of the object numerator, to qbuf, so that the object
// gather reads one plane per frame instead of K exit waves and K probe
// values.
template <int N, int K, int MODE, bool WQ, bool NF>
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
    for (int e = 0; e < E; ++e) u[e] = src[scr_at<N>(y, NF ? in_index<N, E, -1>(t, e) : in_index<N, E, +1>(t, e))];
    if constexpr (NF) {
        // Dx^-1: forward transform, the conjugate x factor, inverse below
        fft1d<N, E, -1>(u, t, L);
        const float2 *qx = a.prop + N;
#pragma unroll
        for (int e = 0; e < E; ++e) u[e] = cmulc(qx[out_index<N, E, -1>(t, e)], u[e]);
    }
    fft1d<N, E, +1>(u, t, L);
    const float2 *prow = a.probe + ((size_t)k * N + y) * N;
    const size_t prow_psi = (((size_t)j * K + k) * N + y) * N;
    size_t orow = 0;
    if constexpr (MODE == OUT_DM) {
        const int2 o = a.offs[j];
        orow = (size_t)(o.x + y) * a.Nx + o.y;
    }
    float2 qk[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int x = out_index<N, E, +1>(t, e);
        float2 v = u[e];
        if constexpr (MODE == OUT_DM) {
            if (active) v = cadd(cmul(a.obj[orow + x], prow[x]), v);
        }
        if (active) {
            if constexpr (MODE == OUT_SCR) src[scr_at<N>(y, x)] = v;
            if constexpr (MODE == OUT_STORE || MODE == OUT_DM) st_stream(a.psi_out + prow_psi + x, v);
        }
        if constexpr (WQ) qk[e] = cmulc(prow[x], v);
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

// AP background refinement: bsum[i] (+)= sum over the stack's slots of s^2
// (slot order), then bg[i] *= bsum[i] / J once all stacks are in.
__global__ __launch_bounds__(256) void k_bg_accum(const float *s2, int S, long n2, double *bsum, int first) {
    for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < n2; i += (long)gridDim.x * 256) {
        double v = first ? 0.0 : bsum[i];
        for (int s = 0; s < S; ++s) v += (double)s2[(size_t)s * n2 + i];
        bsum[i] = v;
    }
}
__global__ __launch_bounds__(256) void k_bg_finish(float *bg, const double *bsum, long n2, double J) {
    for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < n2; i += (long)gridDim.x * 256)
        bg[i] = (float)((double)bg[i] * (bsum[i] / J));
}

// Position refinement (Psi2PosShift): block j accumulates, over frame j's
// pixels and modes, the 2x2 least-squares system of its position shift,
// chi = Psi - P O ~ d_y P dO/dy + d_x P dO/dx, with the object gradient by
// centred differences (one-sided on the object's border), and writes
// out[j] = (d_y, d_x, S_yy + S_xx).
struct PosShiftArgs {
    int N, K, Ny, Nx;
    const int2 *offs;             // [J] (oy, ox)
    const float2 *obj, *probe, *psi;
    double *out;                  // [J][3]
};

__device__ __forceinline__ float2 obj_diff(const float2 *o, int i, int lo_step, int hi_step, bool at_lo,
                                           bool at_hi) {
    if (at_lo) return csub(o[i + hi_step], o[i]);
    if (at_hi) return csub(o[i], o[i - lo_step]);
    return cscale(csub(o[i + hi_step], o[i - lo_step]), 0.5f);
}

__global__ __launch_bounds__(256) void k_pos_shift(PosShiftArgs a) {
    const int j = blockIdx.x, N = a.N;
    const int2 o = a.offs[j];
    const long n2 = (long)N * N;
    double syy = 0.0, sxx = 0.0, sxy = 0.0, by = 0.0, bx = 0.0;
    for (long idx = threadIdx.x; idx < n2; idx += 256) {
        const int y = (int)(idx / N), x = (int)(idx % N);
        const int Y = o.x + y, X = o.y + x;
        const int i = Y * a.Nx + X;
        const float2 ov = a.obj[i];
        const float2 gy = obj_diff(a.obj, i, a.Nx, a.Nx, Y == 0, Y == a.Ny - 1);
        const float2 gx = obj_diff(a.obj, i, 1, 1, X == 0, X == a.Nx - 1);
        float fyy = 0.0f, fxx = 0.0f, fxy = 0.0f, fby = 0.0f, fbx = 0.0f;
        for (int k = 0; k < a.K; ++k) {
            const float2 p = a.probe[k * n2 + idx];
            const float2 ps = a.psi[((size_t)j * a.K + k) * n2 + idx];
            const float2 chi = csub(ps, cmul(p, ov));
            const float2 Gy = cmul(p, gy), Gx = cmul(p, gx);
            fyy += cnorm(Gy);
            fxx += cnorm(Gx);
            fxy += cmulc(Gy, Gx).x;
            fby += cmulc(Gy, chi).x;
            fbx += cmulc(Gx, chi).x;
        }
        syy += fyy;
        sxx += fxx;
        sxy += fxy;
        by += fby;
        bx += fbx;
    }
    syy = block_sum(syy);
    sxx = block_sum(sxx);
    sxy = block_sum(sxy);
    by = block_sum(by);
    bx = block_sum(bx);
    if (threadIdx.x == 0) {
        const double det = syy * sxx - sxy * sxy;
        double dy = 0.0, dx = 0.0;
        if (det > 0.0 && det > 1e-12 * syy * sxx) {
            dy = (sxx * by - sxy * bx) / det;
            dx = (syy * bx - sxy * by) / det;
        }
        a.out[3 * j] = dy;
        a.out[3 * j + 1] = dx;
        a.out[3 * j + 2] = syy + sxx;
    }
}

// flag[0] = 1 if any of a[0 .. n) is not finite (flag cleared beforehand;
// every writer stores the same value).
__global__ __launch_bounds__(256) void k_check_finite(const float *a, long n, int *flag) {
    bool bad = false;
    for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long)gridDim.x * 256) bad |= !isfinite(a[i]);
    if (bad) flag[0] = 1;
}
__global__ void k_clear_flag(int *flag) { flag[0] = 0; }

// dst = J * (number of mask pixels equal to 0); every pixel if mask is null.
__global__ __launch_bounds__(256) void k_count_good(const unsigned char *mask, int n2, double J, double *dst) {
    double c = 0.0;
    for (int i = threadIdx.x; i < n2; i += 256) c += (mask == nullptr || mask[i] == 0) ? 1.0 : 0.0;
    c = block_sum(c);
    if (threadIdx.x == 0) dst[0] = c * J;
}

// sum over modes of |P_k|^2 per probe pixel (the object denominator's term)
__global__ __launch_bounds__(256) void k_probe_intensity(const float2 *probe, int K, long n2, float *pint) {
    for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < n2; i += (long)gridDim.x * 256) {
        float v = 0.0f;
        for (int k = 0; k < K; ++k) v += cnorm(probe[k * n2 + i]);
        pint[i] = v;
    }
}

// ========================================================== column pass ===
// OP_CORR writes (s - 1) F(X) instead of s F(X): since P_F(X) = X + F^-1((s-1) F(X))
// (s = 1 at bad pixels), the DM update Psi + P_F(2 Phi - Psi) - Phi equals
// Phi + F^-1((s - 1) F(2 Phi - Psi)), which the inverse row pass forms from the
// views alone, without reading the old exit waves again.
enum ColOp { OP_PROJECT = 0, OP_GRAD = 1, OP_LLK = 2, OP_ICALC = 3, OP_LS = 4, OP_CORR = 5 };

// Exchange buffers of the read-only column pass: the line search's three
// transforms of a mode run pass by pass together while their buffers fit
// 96 KiB of LDS, one after the other through one buffer beyond that.
template <int N, int OP>
struct ColSeqBufs {
    static constexpr int SETS = (OP == OP_LS) ? 3 : 1;
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

    float2 u[K][E];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const float2 *src = a.scr + ((size_t)(s * K + k) * N) * N + scr_at<N>(0, c);
#pragma unroll
        for (int e = 0; e < E; ++e) u[k][e] = src[in_index<N, E, -1>(t, e) * ScrTile<N>::W];
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
// LLK, calculated intensity, and the line-search terms I0, I1, I2.
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
    for (int k = 0; k < a.K; ++k) {
        if constexpr (ONE_BUF) {
            // one transform at a time (large N): keep A, fold B and C into
            // the sums as soon as each is transformed
            float2 A[1][E], V[1][E];
            auto load_transform = [&](float2 (&v)[1][E], int set) {
                const float2 *src = a.scr + ((size_t)(s * SETS * a.K + set * a.K + k) * N) * N + scr_at<N>(0, c);
#pragma unroll
                for (int e = 0; e < E; ++e) v[0][e] = src[in_index<N, E, -1>(t, e) * ScrTile<N>::W];
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
            const float2 *src = a.scr + ((size_t)(s * SETS * a.K + set * a.K + k) * N) * N + scr_at<N>(0, c);
#pragma unroll
            for (int e = 0; e < E; ++e) u[set][e] = src[in_index<N, E, -1>(t, e) * ScrTile<N>::W];
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
            if constexpr (OP == OP_LS) {
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
    } else if constexpr (OP == OP_LS) {
        const double r0 = block_sum(acc0);
        const double r1 = block_sum(acc1);
        if (threadIdx.x == 0) {
            a.red[2 * blk] = r0;
            a.red[2 * blk + 1] = r1;
        }
    }
}

// ============================================================== gathers ===
// Object numerator/denominator by object tile: block b sums, for every pixel
// of tile tiles[b], the frames of entries [tptr[b], tptr[b+1]) in list order;
// each entry is (slot, oy, ox, 0).  A frame adds q = sum_k conj(P_k) Psi_k
// (from the inverse row pass) to the numerator and sum_k |P_k|^2 to the
// denominator.  Blocks are listed with the most covering frames first, so
// light border tiles fill in at the end; a long list is split into chunks
// whose partial sums k_obj_chunk_reduce adds in order.
struct ObjTileArgs {
    int N, Ny, Nx, ntx;
    const int *tiles;             // block -> tile
    const int *tptr;              // block -> entry range
    const int *pslot;             // block -> partial slot, -1: add to the sums directly
    const int4 *tent;
    const float *pint;            // [N][N] sum_k |P_k|^2
    const float2 *q;              // [S][N][N]
    float2 *numO;
    float *denO;
    float2 *pnum;                 // partial sums [slot][OTILE_Y * OTILE_X]
    float *pden;
};

__global__ __launch_bounds__(256) void k_gather_obj(ObjTileArgs a) {
    const int tile = a.tiles[blockIdx.x];
    const int ty = tile / a.ntx, tx = tile % a.ntx;
    const int col = threadIdx.x % OTILE_X, r0 = threadIdx.x / OTILE_X;
    constexpr int RSTEP = 256 / OTILE_X;            // row phases per block
    const int px = tx * OTILE_X + col;
    constexpr int PY = OTILE_Y / RSTEP;
    constexpr int FU = 4;                            // frames per iteration
    float2 acc[PY];
    float den[PY];
#pragma unroll
    for (int i = 0; i < PY; ++i) {
        acc[i] = make_float2(0.0f, 0.0f);
        den[i] = 0.0f;
    }
    const int N = a.N;
    const size_t fsz = (size_t)N * N;
    const int f0 = a.tptr[blockIdx.x], f1 = a.tptr[blockIdx.x + 1];
    // FU frames per iteration: all loads are issued before any is summed
    // (the per-pixel order of the sum is unchanged).  Out-of-window pixels
    // and missing frames read a clamped in-window address and are weighted
    // 0, so the body is branch-free.
    for (int f = f0; f < f1; f += FU) {
        float2 v[FU][PY];
        float d[FU][PY], m[FU][PY];
#pragma unroll
        for (int h = 0; h < FU; ++h) {
            const bool have = f + h < f1;
            const int4 e = a.tent[have ? f + h : f];
            const int x = px - e.z;
            const bool xin = (unsigned)x < (unsigned)N && have;
            const int xc = min(max(x, 0), N - 1);
            const float2 *qs = a.q + (size_t)e.x * fsz;
#pragma unroll
            for (int i = 0; i < PY; ++i) {
                const int y = ty * OTILE_Y + r0 + RSTEP * i - e.y;
                m[h][i] = (xin && (unsigned)y < (unsigned)N) ? 1.0f : 0.0f;
                const size_t pix = (size_t)min(max(y, 0), N - 1) * N + xc;
                v[h][i] = qs[pix];
                d[h][i] = a.pint[pix];
            }
        }
#pragma unroll
        for (int h = 0; h < FU; ++h)
#pragma unroll
            for (int i = 0; i < PY; ++i) {
                acc[i].x += m[h][i] * v[h][i].x;
                acc[i].y += m[h][i] * v[h][i].y;
                den[i] += m[h][i] * d[h][i];
            }
    }
    const int slot = a.pslot[blockIdx.x];
    if (slot >= 0) {
#pragma unroll
        for (int i = 0; i < PY; ++i) {
            const size_t q = (size_t)slot * (OTILE_Y * OTILE_X) + (r0 + RSTEP * i) * OTILE_X + col;
            a.pnum[q] = acc[i];
            a.pden[q] = den[i];
        }
        return;
    }
    if (px >= a.Nx) return;
#pragma unroll
    for (int i = 0; i < PY; ++i) {
        const int py = ty * OTILE_Y + r0 + RSTEP * i;
        if (py >= a.Ny) continue;
        const size_t op = (size_t)py * a.Nx + px;
        const float2 n0 = a.numO[op];
        a.numO[op] = make_float2(n0.x + acc[i].x, n0.y + acc[i].y);
        a.denO[op] += den[i];
    }
}

// Sums of the chunk partials of split tiles, added to the object sums: block
// b handles tile rtile[b] whose chunks occupy partial slots rfirst[b] ..
// rfirst[b] + rcount[b] - 1.
__global__ __launch_bounds__(256) void k_obj_chunk_reduce(const int *rtile, const int *rfirst, const int *rcount,
                                                          const float2 *pnum, const float *pden, float2 *numO,
                                                          float *denO, int ntx, int Ny, int Nx) {
    const int tile = rtile[blockIdx.x], first = rfirst[blockIdx.x], n = rcount[blockIdx.x];
    const int ty = tile / ntx, tx = tile % ntx;
    for (int q = threadIdx.x; q < OTILE_Y * OTILE_X; q += 256) {
        const int py = ty * OTILE_Y + q / OTILE_X, px = tx * OTILE_X + q % OTILE_X;
        float2 s = make_float2(0.0f, 0.0f);
        float d = 0.0f;
        for (int c = 0; c < n; ++c) {
            const size_t i = (size_t)(first + c) * (OTILE_Y * OTILE_X) + q;
            s.x += pnum[i].x;
            s.y += pnum[i].y;
            d += pden[i];
        }
        if (py >= Ny || px >= Nx) continue;
        const size_t op = (size_t)py * Nx + px;
        const float2 n0 = numO[op];
        numO[op] = make_float2(n0.x + s.x, n0.y + s.y);
        denO[op] += d;
    }
}

// Probe numerator/denominator over the frames order[q0 .. q0+nq), with the
// given object: one thread per probe pixel, all K modes (the object value of
// a frame is read once for the K modes); the range is split into gridDim.z
// chunks whose partial sums k_probe_reduce adds in chunk order.  Exit waves
// are read from the stack scratch by slot (FROM_SCR, slot = q - q0) or from
// stored exit waves [J][K][N][N] by frame.  The order is the plan's
// spatially compact one, so object rows are reused in L2.
struct ProbeAllArgs {
    int N, K, q0, nq, Nx;
    int lw;             // log2 of the exit waves' tile width (log2 N: row-major)
    const int2 *offs;
    const int *order;
    const float2 *obj;
    const float2 *psi;
    float2 *part_num;   // [C][K][N*N]
    float *part_den;    // [C][N*N]
};

template <int K, bool FROM_SCR>
__global__ __launch_bounds__(256) void k_gather_probe(ProbeAllArgs a) {
    const int N = a.N;
    const int idx = xcd_block(blockIdx.x, gridDim.x) * 256 + threadIdx.x;
    const int c = blockIdx.z, C = gridDim.z;
    if (idx >= N * N) return;
    const int y = idx / N, x = idx % N;
    const size_t fsz = (size_t)N * N;
    const size_t vpix = tiled_at(y, x, N, a.lw);
    const int j0 = (int)((long)c * a.nq / C), j1 = (int)((long)(c + 1) * a.nq / C);
    float2 acc[K];
#pragma unroll
    for (int k = 0; k < K; ++k) acc[k] = make_float2(0.0f, 0.0f);
    float den = 0.0f;
    for (int q = j0; q < j1; ++q) {
        const int j = a.order[a.q0 + q];
        const int2 o = a.offs[j];
        const float2 ov = a.obj[(size_t)(o.x + y) * a.Nx + o.y + x];
        const float2 *ps = a.psi + (size_t)(FROM_SCR ? q : j) * K * fsz + vpix;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const float2 cv = cmulc(ov, ld_stream(ps + k * fsz));
            acc[k].x += cv.x;
            acc[k].y += cv.y;
        }
        den += cnorm(ov);
    }
#pragma unroll
    for (int k = 0; k < K; ++k) a.part_num[((size_t)c * K + k) * fsz + idx] = acc[k];
    a.part_den[(size_t)c * fsz + idx] = den;
}

// numP, denP (=, or += with accumulate) the chunk partials in chunk order.
__global__ __launch_bounds__(256) void k_probe_reduce(const float2 *part_num, const float *part_den, int C, int K,
                                                      long n2, float2 *numP, float *denP, int accumulate) {
    const long np = n2 * K;
    for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < np; i += (long)gridDim.x * 256) {
        float2 s = accumulate ? numP[i] : make_float2(0.0f, 0.0f);
        for (int c = 0; c < C; ++c) {
            const float2 v = part_num[(size_t)c * np + i];
            s.x += v.x;
            s.y += v.y;
        }
        numP[i] = s;
        if (i < n2) {
            float d = accumulate ? denP[i] : 0.0f;
            for (int c = 0; c < C; ++c) d += part_den[(size_t)c * n2 + i];
            denP[i] = d;
        }
    }
}

// ====================================================== normalisation ===
// Per-block maxima of the object and probe denominators.
__global__ __launch_bounds__(256) void k_max_partial(const float *denO, long nO, const float *denP,
                                                     long nP, float *part) {
    float mo = 0.0f, mp = 0.0f;
    for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < nO; i += (long)gridDim.x * 256)
        mo = fmaxf(mo, denO[i]);
    for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < nP; i += (long)gridDim.x * 256)
        mp = fmaxf(mp, denP[i]);
    mo = block_max(mo);
    mp = block_max(mp);
    if (threadIdx.x == 0) {
        part[blockIdx.x] = mo;
        part[gridDim.x + blockIdx.x] = mp;
    }
}

__device__ __forceinline__ void reduce_partials(const float *part, int npart, float &mo, float &mp) {
    float a = 0.0f, b = 0.0f;
    for (int i = threadIdx.x; i < npart; i += blockDim.x) {
        a = fmaxf(a, part[i]);
        b = fmaxf(b, part[npart + i]);
    }
    mo = block_max(a);
    mp = block_max(b);
}

// O <- (numO + a O)/(denO + a), a = dO * max(denO); same for every probe mode.
__global__ __launch_bounds__(256) void k_normalize(float2 *obj, const float2 *numO, const float *denO,
                                                   long nO, float2 *probe, const float2 *numP,
                                                   const float *denP, int n2, int K, const float *part,
                                                   int npart, float dO, float dP, unsigned upd) {
    float mo, mp;
    reduce_partials(part, npart, mo, mp);
    const float ao = dO * mo, ap = dP * mp;
    if (upd & 1u) {
        for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < nO; i += (long)gridDim.x * 256) {
            const float d = denO[i] + ao;
            if (d > 0.0f) {
                const float2 n = numO[i], o = obj[i];
                const float r = 1.0f / d;
                obj[i] = make_float2((n.x + ao * o.x) * r, (n.y + ao * o.y) * r);
            }
        }
    }
    if (upd & 2u) {
        const long np = (long)n2 * K;
        for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < np; i += (long)gridDim.x * 256) {
            const float d = denP[i % n2] + ap;
            if (d > 0.0f) {
                const float2 n = numP[i], p = probe[i];
                const float r = 1.0f / d;
                probe[i] = make_float2((n.x + ap * p.x) * r, (n.y + ap * p.y) * r);
            }
        }
    }
}

// ======================================================== small kernels ===
__global__ __launch_bounds__(256) void k_zero(float4 *p, long n16) {
    for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < n16; i += (long)gridDim.x * 256)
        p[i] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
}

// psi[j][k] = O_j * P_k for all frames (DM start).
__global__ __launch_bounds__(256) void k_psi_init(const float2 *obj, const float2 *probe, const int2 *offs,
                                                  float2 *psi, int N, int K, int Nx, long total) {
    for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < total; i += (long)gridDim.x * 256) {
        const long n2 = (long)N * N;
        const int pix = (int)(i % n2);
        const long jk = i / n2;
        const int k = (int)(jk % K);
        const int j = (int)(jk / K);
        const int y = pix / N, x = pix % N;
        const int2 o = offs[j];
        psi[i] = cmul(obj[(size_t)(o.x + y) * Nx + o.y + x], probe[(size_t)k * n2 + pix]);
    }
}

// Sum of `n` partials (fixed order, one block) into out[0] (+= if accumulate).
__global__ __launch_bounds__(256) void k_sum_partials(const double *red, long n, int stride, double *out,
                                                      int accumulate) {
    double v = 0.0;
    for (long i = threadIdx.x; i < n; i += 256) v += red[i * stride];
    v = block_sum(v);
    if (threadIdx.x == 0) out[0] = accumulate ? out[0] + v : v;
}

// Plain batched FFT along rows / columns (standalone 2D transform).
template <int N, int DIR>
__global__ __launch_bounds__(256) void k_fft_rows(float2 *data, long rows) {
    using G = RowGeom<N>;
    constexpr int E = G::E, T = G::T, RB = G::RB;
    __shared__ float2 lds[G::LDS_F2];
    const int tid = threadIdx.x, rr = tid / T, t = tid % T;
    const long g = (long)blockIdx.x * RB + rr;
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

template <int N, int DIR>
__global__ __launch_bounds__(ColGeom<N>::THREADS) void k_fft_cols(float2 *data, long count, float scale) {
    using G = ColGeom<N>;
    constexpr int E = G::E, CB = G::CB;
    extern __shared__ float2 lds_dyn[];
    const int tid = threadIdx.x, cl = tid % CB, t = tid / CB;
    const long g = (long)blockIdx.x * CB + cl;
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
