// mlcg.hpp - device side of the conjugate-gradient maximum-likelihood cycle.
//
// All scalars of the iteration (beta, the probe preconditioning scale, the
// line-search coefficients and the step) live in device memory, so a run of
// ML cycles is enqueued without any host synchronisation.  Every reduction
// is a fixed-order two-level sum (per-block partials, then one block).
#pragma once

#include "kernels.hpp"

namespace ptycho {

// device scalar slots (double)
enum {
    CG_LLK = 0,    // LLK at the current point (from the gradient pass)
    CG_L1 = 1,     // L'(0) along the direction
    CG_L2 = 2,     // L''(0)
    CG_ZG = 3,     // <z, g> of the previous cycle
    CG_HAVE = 4,   // 1 once a direction exists
    CG_BETA = 5,
    CG_S = 6,      // probe preconditioning scale max(denO)/max(denP)
    CG_GAMMA = 7,
    CG_NSCAL = 16
};
constexpr int CG_NPART = 256;   // blocks of the inner-product reduction

__global__ void k_cg_reset(double *scal) {
    if (threadIdx.x < CG_NSCAL) scal[threadIdx.x] = 0.0;
}

__global__ __launch_bounds__(256) void k_scale_copy(float2 *dst, const float2 *src, long n, float s) {
    for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long)gridDim.x * 256)
        dst[i] = cscale(src[i], s);
}

// Partials of <gO,gO>, <gO,gO_prev>, <gP,gP>, <gP,gP_prev> with g = 2 * sums,
// blocks not being updated counting as zero.
__global__ __launch_bounds__(256) void k_cg_dots(const float2 *sumO, const float2 *gprevO, long no,
                                                 const float2 *sumP, const float2 *gprevP, long np, unsigned upd,
                                                 double *part) {
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    if (upd & 1u) {
        for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < no; i += (long)gridDim.x * 256) {
            const float2 g = cscale(sumO[i], 2.0f), q = gprevO[i];
            a0 += (double)g.x * g.x + (double)g.y * g.y;
            a1 += (double)g.x * q.x + (double)g.y * q.y;
        }
    }
    if (upd & 2u) {
        for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < np; i += (long)gridDim.x * 256) {
            const float2 g = cscale(sumP[i], 2.0f), q = gprevP[i];
            a2 += (double)g.x * g.x + (double)g.y * g.y;
            a3 += (double)g.x * q.x + (double)g.y * q.y;
        }
    }
    a0 = block_sum(a0);
    a1 = block_sum(a1);
    a2 = block_sum(a2);
    a3 = block_sum(a3);
    if (threadIdx.x == 0) {
        part[4 * blockIdx.x + 0] = a0;
        part[4 * blockIdx.x + 1] = a1;
        part[4 * blockIdx.x + 2] = a2;
        part[4 * blockIdx.x + 3] = a3;
    }
}

// beta (Polak-Ribiere, clipped at 0) and the preconditioning scale s.
__global__ __launch_bounds__(256) void k_cg_beta(const double *part, const float *maxpart, int nmax, double *scal,
                                                 double *hist_slot) {
    double a[4];
    for (int m = 0; m < 4; ++m) {
        double v = 0.0;
        for (int i = threadIdx.x; i < CG_NPART; i += 256) v += part[4 * i + m];
        a[m] = block_sum(v);
    }
    float mo, mp;
    reduce_partials(maxpart, nmax, mo, mp);
    if (threadIdx.x == 0) {
        const double s = mp > 0.0f ? (double)mo / (double)mp : 1.0;
        const double zg = a[0] + s * a[2];
        double beta = 0.0;
        if (scal[CG_HAVE] != 0.0 && scal[CG_ZG] > 0.0) {
            beta = (a[0] - a[1] + s * (a[2] - a[3])) / scal[CG_ZG];
            if (!(beta > 0.0)) beta = 0.0;
        }
        scal[CG_BETA] = beta;
        scal[CG_S] = s;
        scal[CG_ZG] = zg;
        scal[CG_HAVE] = 1.0;
        if (hist_slot) hist_slot[0] = scal[CG_LLK];
    }
}

// d <- -(gO, s gP) + beta d;  g_prev <- g.
__global__ __launch_bounds__(256) void k_cg_direction(const float2 *sumO, float2 *gprevO, float2 *dO, long no,
                                                      const float2 *sumP, float2 *gprevP, float2 *dP, long np,
                                                      unsigned upd, const double *scal) {
    const float beta = (float)scal[CG_BETA];
    const float s = (float)scal[CG_S];
    for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < no; i += (long)gridDim.x * 256) {
        const float2 g = (upd & 1u) ? cscale(sumO[i], 2.0f) : make_float2(0.0f, 0.0f);
        float2 d = make_float2(-g.x, -g.y);
        if (beta != 0.0f) {
            const float2 dp = dO[i];
            d.x += beta * dp.x;
            d.y += beta * dp.y;
        }
        dO[i] = d;
        gprevO[i] = g;
    }
    for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < np; i += (long)gridDim.x * 256) {
        const float2 g = (upd & 2u) ? cscale(sumP[i], 2.0f) : make_float2(0.0f, 0.0f);
        float2 d = make_float2(-s * g.x, -s * g.y);
        if (beta != 0.0f) {
            const float2 dp = dP[i];
            d.x += beta * dp.x;
            d.y += beta * dp.y;
        }
        dP[i] = d;
        gprevP[i] = g;
    }
}

// x <- x + gamma d with gamma = -L'(0)/L''(0) (0 unless L''(0) > 0).
__global__ __launch_bounds__(256) void k_cg_step(float2 *obj, const float2 *dO, long no, float2 *probe,
                                                 const float2 *dP, long np, unsigned upd, double *scal) {
    const double l1 = scal[CG_L1], l2 = scal[CG_L2];
    const double gd = (l2 > 0.0 && isfinite(l1) && isfinite(l2)) ? -l1 / l2 : 0.0;
    const float gamma = (float)gd;
    if (blockIdx.x == 0 && threadIdx.x == 0) scal[CG_GAMMA] = gd;
    if (upd & 1u) {
        for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < no; i += (long)gridDim.x * 256) {
            const float2 d = dO[i], o = obj[i];
            obj[i] = make_float2(o.x + gamma * d.x, o.y + gamma * d.y);
        }
    }
    if (upd & 2u) {
        for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < np; i += (long)gridDim.x * 256) {
            const float2 d = dP[i], p = probe[i];
            probe[i] = make_float2(p.x + gamma * d.x, p.y + gamma * d.y);
        }
    }
}

}  // namespace ptycho
