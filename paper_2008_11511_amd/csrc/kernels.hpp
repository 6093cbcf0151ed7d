// kernels.hpp - kernels that do not depend on the frame size: the object and
// probe gathers, normalisation, reductions, position shifts, background
// refinement and small helpers.  Compiled once, in ptycho.hip.
#pragma once

#include "common.hpp"

namespace ptycho {


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

// Position refinement (Psi2PosShift): the 2x2 least-squares system of each
// frame's position shift, chi = dPsi ~ d_y P dO/dy + d_x P dO/dx, with the
// object gradient by centred differences (one-sided on the object's border)
// taken at the frame's view (interpolated like the view for sub-pixel
// windows).  The exit-wave change is chi = Psi - P O_view from projected exit
// waves (AP), or chi = scale * Psi from a gradient wave (ML, scale = -1/2).
// Block f CH + c sums the five terms over rows [c R, c R + R) of frame f of
// the launch; k_pos_shift_finish adds a frame's chunks in order and solves.
struct PosShiftArgs {
    int N, K, Ny, Nx;
    int R, CH;                    // rows per chunk, chunks per frame
    int lgN;                      // log2 N
    const int2 *offs;             // [J] (oy, ox)
    const float2 *frac;           // [J] sub-pixel fractions, or null
    const int *order;             // launch frame f -> frame j (order[s0 + f]), or null: j = f
    int s0, nf;                   // first launch frame, frames in the launch
    const float2 *obj, *probe, *psi;
    int lw;                       // log2 of psi's tile width (log2 N: row-major)
    bool by_slot;                 // psi indexed by launch frame f (stack scratch), else by frame j
    bool ml;                      // chi = chi_scale * psi (else psi - P O_view)
    float chi_scale;
    double *part;                 // [J][CH][5], indexed by frame j
};

// Partial sums of the position-shift systems, one chunk of R rows of F
// frames per block (the same pixels of each, so that one probe load serves
// the F frames).  The derivatives of the object are the centred
// differences inside the object and one-sided ones on its border:
// (O[hi] - O[lo]) / (hi - lo) with lo, hi the neighbours clamped to the
// object.
//
// One thread walks down two adjacent columns (x, x + 1) of its chunk, in each
// of its F frames, and keeps the object rows its pixels need in registers.  Per row of the walk it
// loads the object values X-1 .. X+2 (and X+3 for sub-pixel windows) of one
// new row (clamped to the object) and forms, for both pixels, the row's view
// along x and that of its x derivative,
//   H(Y') = sum_b w_b O[Y'][X+b],   D(Y') = sum_b w_b dO/dx[Y'][X+b]
// (w = (1 - fx, fx); integer windows: one term, w = 1).  A pixel at object
// row Y then takes everything from rows Y-1 .. Y+2 (v = (1 - fy, fy)):
//   view  = sum_a v_a H(Y+a)
//   dO/dx = sum_a v_a D(Y+a)
//   dO/dy = sum_a v_a (H(hi(Y+a)) - H(lo(Y+a))) / (hi - lo)
// i.e. the bilinear views of the object and of its two derivatives.  The two
// columns' exit waves and probe values arrive in one 16-byte load each.
struct RawRow {
    float2 v[5];                 // O[Y][clamp(X - 1 + i)]
};
struct ShiftRow {
    float2 h[2], d[2];           // per pixel of the pair
};
template <bool SUB>
__device__ __forceinline__ RawRow load_row(const float2 *o, int Nx, int Y, int X) {
    const float2 *row = o + (size_t)Y * Nx;
    RawRow r;
    r.v[0] = row[max(X - 1, 0)];
    r.v[1] = row[X];
    r.v[2] = row[min(X + 1, Nx - 1)];
    r.v[3] = row[min(X + 2, Nx - 1)];
    r.v[4] = SUB ? row[min(X + 3, Nx - 1)] : make_float2(0.0f, 0.0f);
    return r;
}
// dO/dx at column c, whose clamped neighbours are r.v[i - 1] and r.v[i + 1]
__device__ __forceinline__ float2 row_dx(const RawRow &r, int i, int c, int Nx) {
    return cscale(csub(r.v[i + 1], r.v[i - 1]), (min(c + 1, Nx - 1) - max(c - 1, 0) == 2) ? 0.5f : 1.0f);
}
template <bool SUB>
__device__ __forceinline__ ShiftRow make_row(const RawRow &r, int Nx, int X, float wx0, float wx1) {
    ShiftRow w;
#pragma unroll
    for (int p = 0; p < 2; ++p) {
        const int i = 1 + p, c = X + p;
        const float2 d0 = row_dx(r, i, c, Nx);
        if constexpr (!SUB) {
            w.h[p] = r.v[i];
            w.d[p] = d0;
        } else {
            // the second column min(c + 1, Nx - 1) weighs fx, which is 0
            // whenever c is the object's last column
            const float2 d1 = row_dx(r, i + 1, c + 1, Nx);
            const float2 b = r.v[i], e = r.v[i + 1];
            w.h[p] = make_float2(__builtin_fmaf(wx1, e.x, wx0 * b.x), __builtin_fmaf(wx1, e.y, wx0 * b.y));
            w.d[p] = make_float2(__builtin_fmaf(wx1, d1.x, wx0 * d0.x), __builtin_fmaf(wx1, d1.y, wx0 * d0.y));
        }
    }
    return w;
}

template <int K, bool SUB, int F>
__global__ __launch_bounds__(256) void k_pos_shift_part(PosShiftArgs a) {
    // the chunks of a frame, and neighbouring frames, on one XCD: their
    // object rows overlap and are served by that XCD's L2
    const int b = xcd_block(blockIdx.x, gridDim.x);
    const int c = b % a.CH, fg = b / a.CH, N = a.N;
    const size_t n2 = (size_t)N * N;
    // F frames per block, the same pixels of each: one probe load serves all
    // F.  A block past the last frame repeats it and drops its sums.
    int jf[F];
    int2 of[F];
    float vy0[F], vy1[F], wx0[F], wx1[F];
    const float2 *psf[F];
#pragma unroll
    for (int i = 0; i < F; ++i) {
        const int f = min(fg * F + i, a.nf - 1);
        jf[i] = a.order != nullptr ? a.order[a.s0 + f] : f;
        of[i] = a.offs[jf[i]];
        const float2 fr = SUB ? a.frac[jf[i]] : make_float2(0.0f, 0.0f);
        vy0[i] = 1.0f - fr.x;
        vy1[i] = fr.x;
        wx0[i] = 1.0f - fr.y;
        wx1[i] = fr.y;
        psf[i] = a.psi + (size_t)(a.by_slot ? f : jf[i]) * K * n2;
    }
    // the thread's column pairs: one pair of ceil(R / G) rows (G = 256 / (N/2)
    // row groups) up to N = 512, N / 512 pairs of R rows beyond
    const int tid = threadIdx.x, lgP = a.lgN - 1, NP = N >> 1;
    int npair, rows, x0, ylo;
    if (NP <= 256) {
        const int G = 256 >> lgP, rt = (a.R + G - 1) / G, gi = tid >> lgP;
        x0 = 2 * (tid & (NP - 1));
        ylo = gi * rt;
        rows = max(0, min(a.R - ylo, rt));
        npair = rows > 0 ? 1 : 0;     // groups past the chunk's rows read nothing
    } else {
        npair = NP >> 8;
        x0 = 2 * tid;
        ylo = 0;
        rows = a.R;
    }
    // the newest object row a pixel at row Y needs: Y + 1, or Y + 2 for
    // sub-pixel windows
    constexpr int LEAD = SUB ? 2 : 1;
    const int ylast = a.Ny - 1;
    // fp32 sums over the thread's pixels (at most 64 terms per frame at every
    // N), fp64 from the block sum on
    float fyy[F], fxx[F], fxy[F], fby[F], fbx[F];
#pragma unroll
    for (int i = 0; i < F; ++i) fyy[i] = fxx[i] = fxy[i] = fby[i] = fbx[i] = 0.0f;
    for (int m = 0; m < npair; ++m) {
        const int x = x0 + (m << 9);
        const int y0 = c * a.R + ylo, ylast_px = y0 + rows - 1;
        // each step loads the next pixel row's exit waves and probe and the
        // object rows after the windows while it works on the current row,
        // and folds the modes of the loaded row as its last act
        auto load_px = [&](int y, float4 (&ps)[F][K], float4 (&pr)[K]) {
            const size_t pix = tiled_at(y, x, N, a.lw);
#pragma unroll
            for (int k = 0; k < K; ++k) {
                pr[k] = *(const float4 *)(a.probe + (size_t)k * n2 + (size_t)y * N + x);
#pragma unroll
                for (int i = 0; i < F; ++i)     // read once: non-temporal, to keep L2 for the object
                    ps[i][k] = ld_stream2(psf[i] + (size_t)k * n2 + pix);
            }
        };
        // the modes enter through Q = sum_k conj(P_k) Psi_k and
        // P2 = sum_k |P_k|^2: sum_k |P_k g|^2 = P2 |g|^2 and
        // sum_k conj(P_k g) chi_k = conj(g) c with c = Q - P2 O_view (AP) or
        // c = scale Q (ML); a row is carried to the next step as Q and P2 of
        // its two pixels, not as its exit-wave and probe values
        auto fold = [&](const float4 (&ps)[F][K], const float4 (&pr)[K], float2 (&q)[F][2], float (&p2)[2]) {
#pragma unroll
            for (int p = 0; p < 2; ++p) {
                p2[p] = 0.0f;
#pragma unroll
                for (int i = 0; i < F; ++i) q[i][p] = make_float2(0.0f, 0.0f);
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    const float2 pk = p ? make_float2(pr[k].z, pr[k].w) : make_float2(pr[k].x, pr[k].y);
                    p2[p] += cnorm(pk);
#pragma unroll
                    for (int i = 0; i < F; ++i) {
                        const float2 sk = p ? make_float2(ps[i][k].z, ps[i][k].w) : make_float2(ps[i][k].x, ps[i][k].y);
                        const float2 mk = cmulc(pk, sk);
                        q[i][p] = make_float2(q[i][p].x + mk.x, q[i][p].y + mk.y);
                    }
                }
            }
        };
        float2 qc[F][2];
        float p2c[2];
        {
            float4 ps[F][K], pr[K];
            load_px(y0, ps, pr);
            fold(ps, pr, qc, p2c);
        }
        RawRow rn[F];
        ShiftRow wm[F], w0[F], w1[F];
#pragma unroll
        for (int i = 0; i < F; ++i) {
            const int X = of[i].y + x, Y0 = of[i].x + y0;
            rn[i] = load_row<SUB>(a.obj, a.Nx, min(Y0 + LEAD, ylast), X);
            // rows Y-1, Y (and Y+1) of the first pixel row, clamped
            wm[i] = make_row<SUB>(load_row<SUB>(a.obj, a.Nx, max(Y0 - 1, 0), X), a.Nx, X, wx0[i], wx1[i]);
            w0[i] = make_row<SUB>(load_row<SUB>(a.obj, a.Nx, Y0, X), a.Nx, X, wx0[i], wx1[i]);
            w1[i] = ShiftRow{};
            if constexpr (SUB)
                w1[i] = make_row<SUB>(load_row<SUB>(a.obj, a.Nx, min(Y0 + 1, ylast), X), a.Nx, X, wx0[i], wx1[i]);
        }
        for (int r = 0; r < rows; ++r) {
            const int y = y0 + r;
            // prefetch (the last step loads its own row again, in bounds)
            float4 ps2[F][K], pr2[K];
            load_px(min(y + 1, ylast_px), ps2, pr2);
            RawRow rn2[F];
#pragma unroll
            for (int i = 0; i < F; ++i)
                rn2[i] = load_row<SUB>(a.obj, a.Nx, min(of[i].x + y + 1 + LEAD, ylast), of[i].y + x);
#pragma unroll
            for (int i = 0; i < F; ++i) {
                const int X = of[i].y + x, Y = of[i].x + y;
                const ShiftRow wl = make_row<SUB>(rn[i], a.Nx, X, wx0[i], wx1[i]);     // row Y + LEAD
                const int Ym = max(Y - 1, 0), Y1 = min(Y + 1, ylast), Y2 = min(Y + 2, ylast);
                const float sy0 = (Y1 - Ym == 2) ? 0.5f : 1.0f, sy1 = (Y2 - Y == 2) ? 0.5f : 1.0f;
#pragma unroll
                for (int p = 0; p < 2; ++p) {
                    float2 ov, gy, gx;
                    if constexpr (SUB) {
                        const float2 gy0 = cscale(csub(w1[i].h[p], wm[i].h[p]), sy0);
                        const float2 gy1 = cscale(csub(wl.h[p], w0[i].h[p]), sy1);
                        ov = make_float2(__builtin_fmaf(vy1[i], w1[i].h[p].x, vy0[i] * w0[i].h[p].x),
                                         __builtin_fmaf(vy1[i], w1[i].h[p].y, vy0[i] * w0[i].h[p].y));
                        gx = make_float2(__builtin_fmaf(vy1[i], w1[i].d[p].x, vy0[i] * w0[i].d[p].x),
                                         __builtin_fmaf(vy1[i], w1[i].d[p].y, vy0[i] * w0[i].d[p].y));
                        gy = make_float2(__builtin_fmaf(vy1[i], gy1.x, vy0[i] * gy0.x),
                                         __builtin_fmaf(vy1[i], gy1.y, vy0[i] * gy0.y));
                    } else {
                        ov = w0[i].h[p];
                        gx = w0[i].d[p];
                        gy = cscale(csub(wl.h[p], wm[i].h[p]), sy0);
                    }
                    const float2 q = qc[i][p];
                    const float p2 = p2c[p];
                    const float2 cc = a.ml ? cscale(q, a.chi_scale) : csub(q, cscale(ov, p2));
                    fyy[i] += p2 * cnorm(gy);
                    fxx[i] += p2 * cnorm(gx);
                    fxy[i] += p2 * cmulc(gy, gx).x;
                    fby[i] += cmulc(gy, cc).x;
                    fbx[i] += cmulc(gx, cc).x;
                }
                // slide the window down one row
                wm[i] = w0[i];
                if constexpr (SUB) {
                    w0[i] = w1[i];
                    w1[i] = wl;
                } else {
                    w0[i] = wl;
                }
                rn[i] = rn2[i];
            }
            fold(ps2, pr2, qc, p2c);
        }
    }
#pragma unroll
    for (int i = 0; i < F; ++i) {
        const double syy = block_sum((double)fyy[i]);
        const double sxx = block_sum((double)fxx[i]);
        const double sxy = block_sum((double)fxy[i]);
        const double by = block_sum((double)fby[i]);
        const double bx = block_sum((double)fbx[i]);
        if (threadIdx.x == 0 && fg * F + i < a.nf) {
            double *d = a.part + ((size_t)jf[i] * a.CH + c) * 5;
            d[0] = syy;
            d[1] = sxx;
            d[2] = sxy;
            d[3] = by;
            d[4] = bx;
        }
    }
}

// out[j] = (d_y, d_x, S_yy + S_xx) from the chunks of frames order[s0 + f]
// (or f), f < nf; d = 0 when the 2x2 system is singular.
__global__ __launch_bounds__(256) void k_pos_shift_finish(const double *part, int CH, const int *order, int s0, int nf,
                                                          double *out) {
    const int f = blockIdx.x * 256 + threadIdx.x;
    if (f >= nf) return;
    const int j = order != nullptr ? order[s0 + f] : f;
    double s[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int c = 0; c < CH; ++c)
        for (int m = 0; m < 5; ++m) s[m] += part[((size_t)j * CH + c) * 5 + m];
    const double syy = s[0], sxx = s[1], sxy = s[2], by = s[3], bx = s[4];
    const double det = syy * sxx - sxy * sxy;
    double dy = 0.0, dx = 0.0;
    if (det > 0.0 && det > 1e-12 * syy * sxx) {
        dy = (sxx * by - sxy * bx) / det;
        dx = (syy * bx - sxy * by) / det;
    }
    out[3 * (size_t)j] = dy;
    out[3 * (size_t)j + 1] = dx;
    out[3 * (size_t)j + 2] = syy + sxx;
}

// Window tables from real corners t (double [J][2]): offs = floor(t) clamped
// to the object, frac = t - offs in float, 0 at the last corner.
__global__ __launch_bounds__(256) void k_windows(const double *t, int J, int n, int Ny, int Nx, int2 *offs,
                                                 float2 *frac) {
    for (int j = blockIdx.x * 256 + threadIdx.x; j < J; j += gridDim.x * 256) {
        const double ty = t[2 * (size_t)j], tx = t[2 * (size_t)j + 1];
        const int oy = min(max((int)floor(ty), 0), Ny - n), ox = min(max((int)floor(tx), 0), Nx - n);
        offs[j] = make_int2(oy, ox);
        frac[j] = make_float2((float)fmin(fmax(ty - oy, 0.0), oy == Ny - n ? 0.0 : 1.0),
                              (float)fmin(fmax(tx - ox, 0.0), ox == Nx - n ? 0.0 : 1.0));
    }
}

// Positions relative to the object centre from real corners: p = t - c + N/2.
__global__ __launch_bounds__(256) void k_corners_to_positions(const double *t, int J, double cy, double cx,
                                                              double *pos) {
#pragma clang fp contract(off)
    for (int j = blockIdx.x * 256 + threadIdx.x; j < J; j += gridDim.x * 256) {
        pos[2 * (size_t)j] = t[2 * (size_t)j] - cy;
        pos[2 * (size_t)j + 1] = t[2 * (size_t)j + 1] - cx;
    }
}

// Position update of the refinement (Section 4: frames move by the shift
// estimated from the exit waves, except frames whose object gradient is too
// weak to tell a shift, and the total move from the starting positions is
// bounded).  One block: the median of the frames' gradient energies by an
// exact radix selection over their bit patterns (non-negative doubles order
// as unsigned integers), then, for every frame j and axis a,
//   keep_j = e_j >= min_grad * median(e)
//   p'     = p + mult * (keep_j ? d : 0)
//   out    = p0 + clamp(p' - p0, -max_shift, max_shift)
// with the median of an even count the mean of the two middle values.  The
// arithmetic is not contracted into fused multiply-adds, so every step
// rounds as written.  out may alias pos.
constexpr int POSUPD_THREADS = 1024;

// The k-th smallest (0-based) of the non-negative doubles v[stride * i],
// i < n, as its bit pattern; every thread of the block returns it.
__device__ unsigned long long select_kth_nonneg(const double *v, int n, int stride, int k, unsigned *hist,
                                                unsigned long long *s_prefix, int *s_rank) {
    unsigned long long prefix = 0ull;
    int rank = k;
    for (int sh = 56; sh >= 0; sh -= 8) {
        const unsigned long long decided = (sh == 56) ? 0ull : (~0ull << (sh + 8));
        for (int i = threadIdx.x; i < 256; i += blockDim.x) hist[i] = 0u;
        __syncthreads();
        for (int i = threadIdx.x; i < n; i += blockDim.x) {
            const unsigned long long key = (unsigned long long)__double_as_longlong(v[(size_t)stride * i]);
            if ((key & decided) == prefix) atomicAdd(&hist[(key >> sh) & 255ull], 1u);
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            int below = 0, b = 0;
            for (; b < 255; ++b) {
                if (below + (int)hist[b] > rank) break;
                below += (int)hist[b];
            }
            *s_prefix = prefix | ((unsigned long long)b << sh);
            *s_rank = rank - below;
        }
        __syncthreads();
        prefix = *s_prefix;
        rank = *s_rank;
        __syncthreads();
    }
    return prefix;
}

__global__ __launch_bounds__(POSUPD_THREADS) void k_update_positions(int J, const double *pos, const double *pos0,
                                                                     const double *shifts, double mult,
                                                                     double max_shift, double min_grad,
                                                                     double *out) {
#pragma clang fp contract(off)
    __shared__ unsigned hist[256];
    __shared__ unsigned long long s_prefix;
    __shared__ int s_rank;
    const unsigned long long lo = select_kth_nonneg(shifts + 2, J, 3, (J - 1) / 2, hist, &s_prefix, &s_rank);
    const unsigned long long hi = select_kth_nonneg(shifts + 2, J, 3, J / 2, hist, &s_prefix, &s_rank);
    const double median = (__longlong_as_double((long long)lo) + __longlong_as_double((long long)hi)) / 2.0;
    const double threshold = min_grad * median;
    for (int j = threadIdx.x; j < J; j += blockDim.x) {
        const bool keep = shifts[3 * (size_t)j + 2] >= threshold;
#pragma unroll
        for (int ax = 0; ax < 2; ++ax) {
            const double step = keep ? shifts[3 * (size_t)j + ax] : 0.0;
            const double moved = pos[2 * (size_t)j + ax] + mult * step;
            const double p0 = pos0[2 * (size_t)j + ax];
            const double d = fmin(fmax(moved - p0, -max_shift), max_shift);
            out[2 * (size_t)j + ax] = p0 + d;
        }
    }
}

// Frame tables of a plan-free call: offs[j] = the caller's offsets clamped
// to the object (flag[0] = 1 if any window was outside it), order[j] = j.
__global__ __launch_bounds__(256) void k_frame_tables(const int *offsets, int J, int n, int ny, int nx, int2 *offs,
                                                      int *order, int *flag) {
    bool bad = false;
    for (int j = blockIdx.x * 256 + threadIdx.x; j < J; j += gridDim.x * 256) {
        const int oy = offsets[2 * j], ox = offsets[2 * j + 1];
        const int cy = min(max(oy, 0), ny - n), cx = min(max(ox, 0), nx - n);
        bad |= (cy != oy) || (cx != ox);
        offs[j] = make_int2(cy, cx);
        order[j] = j;
    }
    if (bad) flag[0] = 1;
}

// dst[0] = NaN when flag[0] is set.
__global__ void k_nan_if_flagged(double *dst, const int *flag) {
    if (flag[0] != 0) dst[0] = __longlong_as_double(0x7ff8000000000000ll);
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
    const int2 *offs;             // sub-pixel windows: frame corners by frame (entry .w) ...
    const float2 *frac;           // ... and their fractions, or null (integer windows: entries)
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
    if (a.frac != nullptr) {
        // sub-pixel windows: object pixel (py, px) takes w_ab q(py - oy - a, px - ox - b) from every
        // frame, the adjoint of the bilinear view (the same weights), and w_ab sum_k |P_k|^2 at the
        // same place for the denominator; the frame's corner comes from the device tables
        for (int f = f0; f < f1; ++f) {
            const int jf = a.tent[f].w;
            const int2 o = a.offs[jf];
            const float2 fr = a.frac[jf];
            const float2 *qs = a.q + (size_t)a.tent[f].x * fsz;
            const float wy[2] = {1.0f - fr.x, fr.x}, wx[2] = {1.0f - fr.y, fr.y};
#pragma unroll
            for (int i = 0; i < PY; ++i) {
                const int y = ty * OTILE_Y + r0 + RSTEP * i - o.x, x = px - o.y;
#pragma unroll
                for (int ay = 0; ay < 2; ++ay)
#pragma unroll
                    for (int bx = 0; bx < 2; ++bx) {
                        const int yy = y - ay, xx = x - bx;
                        if ((unsigned)yy < (unsigned)N && (unsigned)xx < (unsigned)N) {
                            const float w = wy[ay] * wx[bx];
                            const size_t pix = (size_t)yy * N + xx;
                            const float2 v = qs[pix];
                            acc[i].x += w * v.x;
                            acc[i].y += w * v.y;
                            den[i] += w * a.pint[pix];
                        }
                    }
            }
        }
    } else {
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
    int N, K, q0, nq, Nx, Ny;
    const float2 *frac;  // sub-pixel windows [J], or null
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
        const float2 ov = a.frac != nullptr ? view_at(a.obj, view_row(a.Ny, a.Nx, o, a.frac[j], y), x)
                                            : a.obj[(size_t)(o.x + y) * a.Nx + o.y + x];
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
                                                  const float2 *frac, float2 *psi, int N, int K, int Ny, int Nx,
                                                  long total) {
    for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < total; i += (long)gridDim.x * 256) {
        const long n2 = (long)N * N;
        const int pix = (int)(i % n2);
        const long jk = i / n2;
        const int k = (int)(jk % K);
        const int j = (int)(jk / K);
        const int y = pix / N, x = pix % N;
        const int2 o = offs[j];
        const float2 ov = frac != nullptr ? view_at(obj, view_row(Ny, Nx, o, frac[j], y), x)
                                          : obj[(size_t)(o.x + y) * Nx + o.y + x];
        psi[i] = cmul(ov, probe[(size_t)k * n2 + pix]);
    }
}

// Sum of `n` partials (fixed order, one block of SUM_THREADS) into out[0]
// (+= if accumulate).  Each thread keeps four running sums over its
// elements i = t + SUM_THREADS m, m = 0, 1, 2, 3 taken in turn, so that four
// loads are in flight per thread; the order depends on n alone.
constexpr int SUM_THREADS = 1024;
__global__ __launch_bounds__(SUM_THREADS) void k_sum_partials(const double *red, long n, int stride, double *out,
                                                              int accumulate) {
    constexpr long T = SUM_THREADS;
    double v0 = 0.0, v1 = 0.0, v2 = 0.0, v3 = 0.0;
    long i = threadIdx.x;
    for (; i + 3 * T < n; i += 4 * T) {
        v0 += red[i * stride];
        v1 += red[(i + T) * stride];
        v2 += red[(i + 2 * T) * stride];
        v3 += red[(i + 3 * T) * stride];
    }
    for (; i < n; i += T) v0 += red[i * stride];
    const double v = block_sum((v0 + v1) + (v2 + v3));
    if (threadIdx.x == 0) out[0] = accumulate ? out[0] + v : v;
}


}  // namespace ptycho
