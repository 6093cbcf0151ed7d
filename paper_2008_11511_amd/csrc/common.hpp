// common.hpp - device code shared by the gfx950 kernels of the ptychography
// hot path: size rules, the stack-scratch layout, kernel arguments,
// reductions and likelihood terms.
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
// Two adjacent complex values in one 16-byte non-temporal load (p 16-byte
// aligned).
typedef float f32x4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ float4 ld_stream2(const float2 *p) {
    const f32x4 v = __builtin_nontemporal_load((const f32x4 *)p);
    return make_float4(v.x, v.y, v.z, v.w);
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

// Sub-pixel window view: frame corner (oy, ox) + (fy, fx) with fractions in
// [0, 1); the view of row y at column x is the bilinear interpolation
//   (1-fy)(1-fx) O[r0][c] + (1-fy) fx O[r0][c+1] + fy (1-fx) O[r1][c] + fy fx O[r1][c+1]
// with r0 = oy + y, c = ox + x.  The neighbour row and column are clamped to
// the object: beyond it their weight is 0 (a corner is at most Ny - N, where
// its fraction is 0).  With zero fractions the view is O[r0][c] exactly.
struct ViewRow {
    size_t i0, i1;               // offsets of object rows r0 and r1 (clamped), at column ox
    float w00, w01, w10, w11;
    int xlast;                   // last object column, relative to ox
};
__device__ __forceinline__ ViewRow view_row(int Ny, int Nx, int2 o, float2 f, int y) {
    ViewRow v;
    const int r0 = o.x + y, r1 = min(r0 + 1, Ny - 1);
    v.i0 = (size_t)r0 * Nx + o.y;
    v.i1 = (size_t)r1 * Nx + o.y;
    v.w00 = (1.0f - f.x) * (1.0f - f.y);
    v.w01 = (1.0f - f.x) * f.y;
    v.w10 = f.x * (1.0f - f.y);
    v.w11 = f.x * f.y;
    v.xlast = Nx - 1 - o.y;
    return v;
}
// The view of array `base` (object grid) at column x of the row.
__device__ __forceinline__ float2 view_at(const float2 *base, const ViewRow &v, int x) {
    const int x1 = min(x + 1, v.xlast);
    const float2 a = base[v.i0 + x], b = base[v.i0 + x1], c = base[v.i1 + x], d = base[v.i1 + x1];
    return make_float2(v.w00 * a.x + v.w01 * b.x + v.w10 * c.x + v.w11 * d.x,
                       v.w00 * a.y + v.w01 * b.y + v.w10 * c.y + v.w11 * d.y);
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
    float2 *fwd;                 // where the forward row pass writes (the scratch, or
                                 // the kept row transforms of the ML cycle), [S][K][N][N]
    const float2 *colin;         // where the column pass reads its first set, [S][K][N][N]
    float2 *qbuf;                // per slot sum_k conj(P_k) Psi_k, [S][N][N] row-major
    const float *iobs;           // [J][N][N]
    const float *bg;             // incoherent background [N][N] or null
    float *s2;                   // AP background refinement: s^2 per slot [S][N][N], or null
    const unsigned char *mask;   // [N][N] or null
    const float2 *prop;          // near field: [2][N] Qy(u) / N, Qx(v) / N (FFT order), or null
    const float2 *frac;          // sub-pixel windows: [J] (fy, fx) of each frame's corner, or null
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

// Operation selectors of the stack kernels (also used by the host).
enum RowIn { IN_PHI = 0, IN_DM = 1, IN_LS = 2, IN_DATA = 3, IN_LS2 = 4 };
enum RowOut { OUT_SCR = 0, OUT_DM = 1, OUT_STORE = 2, OUT_NONE = 3 };
enum ColOp { OP_PROJECT = 0, OP_GRAD = 1, OP_LLK = 2, OP_ICALC = 3, OP_LS = 4, OP_CORR = 5, OP_LS2 = 6 };

}  // namespace ptycho
