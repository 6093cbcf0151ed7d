// passes.hpp - the frame-size specific host passes: launches of the stack
// kernels for frame size N over all stacks of a plan.  Included by exactly
// one translation unit per N (inst_N.hip), which defines the NPass table of
// that size with PTYCHO_DEFINE_PASSES(N).
#pragma once

#include "plan.hpp"
#include "stack_kernels.hpp"

namespace ptycho {

// Kernels whose dynamic LDS exceeds 64 KiB must opt in once per process.
template <class KernelT>
static hipError_t set_dyn_lds(KernelT kern, size_t bytes) {
    if (bytes <= 64 * 1024) return hipSuccess;
    return hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

template <int N>
static int rows_blocks(int sn) {
    return (int)(((long)sn * N + RowGeom<N>::RB - 1) / RowGeom<N>::RB);
}
template <int N>
static int cols_blocks(int sn) {
    return (int)(((long)sn * N + ColGeom<N>::CB - 1) / ColGeom<N>::CB);
}

template <int N, int K, int OP, bool NF>
static void launch_cols_joint(const StackArgs &a, hipStream_t s) {
    const size_t lds = sizeof(float2) * ColGeom<N>::LDS_F2 * ColJoint<N, K>::BUFS;
    static const hipError_t attr = set_dyn_lds(k_cols_joint<N, K, OP, NF>, lds);
    (void)attr;
    hipLaunchKernelGGL((k_cols_joint<N, K, OP, NF>), dim3(cols_blocks<N>(a.S)), dim3(ColGeom<N>::THREADS), lds, s,
                       a);
}
template <int N, int OP, bool NF>
static void launch_cols_seq(const StackArgs &a, hipStream_t s) {
    const size_t lds = sizeof(float2) * ColGeom<N>::LDS_F2 * ColSeqBufs<N, OP>::value;
    static const hipError_t attr = set_dyn_lds(k_cols_seq<N, OP, NF>, lds);
    (void)attr;
    hipLaunchKernelGGL((k_cols_seq<N, OP, NF>), dim3(cols_blocks<N>(a.S)), dim3(ColGeom<N>::THREADS), lds, s, a);
}

// Forward row pass of input form MODE: the sub-pixel-window instance when the
// plan's windows interpolate, the integer one otherwise.
template <int N, int MODE, bool NF>
static void launch_rows_fwd(const StackArgs &a, dim3 grid, hipStream_t s) {
    if (a.frac != nullptr) hipLaunchKernelGGL((k_rows_fwd<N, MODE, NF, true>), grid, dim3(256), 0, s, a);
    else hipLaunchKernelGGL((k_rows_fwd<N, MODE, NF, false>), grid, dim3(256), 0, s, a);
}

template <int N, int K, int MODE, bool NF>
static void launch_rows_inv(const StackArgs &a, bool wq, hipStream_t s) {
    const dim3 grid((unsigned)(((long)a.S * N + InvRowGeom<N>::RQ - 1) / InvRowGeom<N>::RQ));
    const dim3 block(InvRowGeom<N>::TPM * K);
    // only the DM epilogue reads the view
    if (MODE == OUT_DM && a.frac != nullptr) {
        if (wq) hipLaunchKernelGGL((k_rows_inv<N, K, MODE, true, NF, MODE == OUT_DM>), grid, block, 0, s, a);
        else hipLaunchKernelGGL((k_rows_inv<N, K, MODE, false, NF, MODE == OUT_DM>), grid, block, 0, s, a);
        return;
    }
    if (wq) hipLaunchKernelGGL((k_rows_inv<N, K, MODE, true, NF, false>), grid, block, 0, s, a);
    else hipLaunchKernelGGL((k_rows_inv<N, K, MODE, false, NF, false>), grid, block, 0, s, a);
}

// One pass over all stacks: forward rows, column op, inverse rows and the
// per-stack gathers.  kind: 0 = AP projection, 1 = DM, 2 = ML gradient.
// Exit waves go to `psi` (all frames) when it is given, else stay in the
// stack scratch.  acc selects the sums taken per stack: the object sums
// (from the inverse row pass's per-frame terms), the probe sums (only for
// the gradient, whose two sums are taken at the same point; they read the
// exit waves from the scratch).
template <int N, int K, bool NF>
static int project_pass_nk(ptycho_plan_s *p, const float *obj, const float *probe, float *psi, int kind,
                           unsigned acc, bool upd_bg, float2 *keep) {
    const int J = p->d.n_frames, S = p->L.S;
    hipStream_t s = p->stream;
    const bool store = (psi != nullptr);
    const bool wq = (acc & ACC_OBJ) != 0;
    if (wq) {
        Timed tm(p, TC_OTHER);
        const int st = launch_probe_intensity(p, probe);
        if (st) return st;
    }
    for (int sidx = 0; sidx < p->L.nstacks; ++sidx) {
        const int s0 = sidx * S, sn = std::min(S, J - s0);
        StackArgs a = stack_args(p, s0, sn, obj, probe);
        a.psi = (const float2 *)psi;
        a.psi_out = (float2 *)psi;
        a.red = p->red + (size_t)sidx * p->L.maxb;
        if (upd_bg) a.s2 = p->s2;
        if (keep) a.fwd = keep + (size_t)s0 * K * N * N;
        a.colin = a.fwd;
        const dim3 rg(rows_blocks<N>(sn), p->d.n_modes);
        {
            Timed tm(p, TC_ROWS_FWD);
            if (kind == 1) launch_rows_fwd<N, IN_DM, NF>(a, rg, s);
            else launch_rows_fwd<N, IN_PHI, NF>(a, rg, s);
        }
        {
            Timed tm(p, TC_COLS);
            if (kind == 2) launch_cols_joint<N, K, OP_GRAD, NF>(a, s);
            else if (kind == 1) launch_cols_joint<N, K, OP_CORR, NF>(a, s);
            else launch_cols_joint<N, K, OP_PROJECT, NF>(a, s);
        }
        if (upd_bg) {
            Timed tm(p, TC_OTHER);
            const int st = launch_bg_accum(p, sn, sidx == 0 ? 1 : 0);
            if (st) return st;
        }
        {
            Timed tm(p, TC_ROWS_INV);
            if (kind == 1) launch_rows_inv<N, K, OUT_DM, NF>(a, wq, s);
            else if (store) launch_rows_inv<N, K, OUT_STORE, NF>(a, wq, s);
            else if (acc & ACC_PROBE) launch_rows_inv<N, K, OUT_SCR, NF>(a, wq, s);
            else launch_rows_inv<N, K, OUT_NONE, NF>(a, wq, s);
        }
        LAUNCHCHK();
        int st = PTYCHO_OK;
        // ML position shifts from the gradient wave left in the scratch
        if (kind == 2 && p->shifts_in_grad) st = launch_ml_shifts(p, obj, probe, s0, sn);
        if (!st && (acc & ACC_OBJ)) st = object_sums(p, sidx);
        if (!st && (acc & ACC_PROBE)) st = probe_sums(p, obj, p->scr, s0, sn, true, true);
        if (st) return st;
    }
    return PTYCHO_OK;
}

template <int N>
static int project_pass_n(ptycho_plan_s *p, const float *obj, const float *probe, float *psi, int kind,
                          unsigned acc, bool upd_bg, float2 *keep) {
    return with_k(p->d.n_modes, [&](auto kk) {
        return with_nf(p, [&](auto nf) {
            return project_pass_nk<N, decltype(kk)::value, decltype(nf)::value>(p, obj, probe, psi, kind, acc,
                                                                                  upd_bg, keep);
        });
    });
}

// Read-only forward passes: LLK, icalc, line search.
template <int N, int OP, bool NF>
static int forward_pass_op(ptycho_plan_s *p, const float *obj, const float *probe, const float *dobj,
                           const float *dprobe, float *icalc, int llk_model, const float2 *keep) {
    const bool ls = (OP == OP_LS || OP == OP_LS2);
    const Layout &Lp = p->L;
    const int J = p->d.n_frames;
    const int S = (OP == OP_LS2) ? Lp.S_ls2 : ls ? Lp.S_ls : Lp.S;
    const int nst = (OP == OP_LS2) ? Lp.nstacks_ls2 : ls ? Lp.nstacks_ls : Lp.nstacks;
    const int maxb = (OP == OP_LS2) ? Lp.maxb_ls2 : ls ? Lp.maxb_ls : Lp.maxb;
    hipStream_t s = p->stream;
    for (int sidx = 0; sidx < nst; ++sidx) {
        const int s0 = sidx * S, sn = std::min(S, J - s0);
        StackArgs a = stack_args(p, s0, sn, obj, probe);
        a.dobj = (const float2 *)dobj;
        a.dprobe = (const float2 *)dprobe;
        a.icalc = icalc;
        a.llk_model = llk_model;
        a.red = p->red + (size_t)sidx * maxb * (ls ? 2 : 1);
        if (OP == OP_LS2) a.colin = keep + (size_t)s0 * p->d.n_modes * N * N;
        const dim3 rg(rows_blocks<N>(sn), p->d.n_modes);
        {
            Timed tm(p, TC_ROWS_FWD);
            if (OP == OP_LS2) launch_rows_fwd<N, IN_LS2, NF>(a, rg, s);
            else if (ls) launch_rows_fwd<N, IN_LS, NF>(a, rg, s);
            else launch_rows_fwd<N, IN_PHI, NF>(a, rg, s);
        }
        {
            Timed tm(p, TC_COLS);
            launch_cols_seq<N, OP, NF>(a, s);
        }
        LAUNCHCHK();
    }
    return PTYCHO_OK;
}

template <int N>
static int forward_pass_n(ptycho_plan_s *p, int op, const float *obj, const float *probe, const float *dobj,
                          const float *dprobe, float *icalc, int llk_model, const float2 *keep) {
    return with_nf(p, [&](auto nf) {
        constexpr bool NF = decltype(nf)::value;
        switch (op) {
            case OP_LLK: return forward_pass_op<N, OP_LLK, NF>(p, obj, probe, dobj, dprobe, icalc, llk_model, keep);
            case OP_ICALC: return forward_pass_op<N, OP_ICALC, NF>(p, obj, probe, dobj, dprobe, icalc, llk_model, keep);
            case OP_LS: return forward_pass_op<N, OP_LS, NF>(p, obj, probe, dobj, dprobe, icalc, llk_model, keep);
            case OP_LS2: return forward_pass_op<N, OP_LS2, NF>(p, obj, probe, dobj, dprobe, icalc, llk_model, keep);
            default: return fail(PTYCHO_E_INVALID, "internal: unknown forward op");
        }
    });
}

template <int N>
static int fft2_n(int32_t count, float *data, int32_t dir, hipStream_t s) {
    const long rows = (long)count * N;
    const int rb = (int)((rows + RowGeom<N>::RB - 1) / RowGeom<N>::RB);
    using FG = FftColGeom<N>;
    const int cbk = (int)((rows + FG::CB - 1) / FG::CB);
    const size_t lds = sizeof(float2) * FG::LDS_F2;
    const float scale = 1.0f / (float)N;
    if (dir < 0) {
        static const hipError_t attr = set_dyn_lds(k_fft_cols<N, -1>, lds);
        (void)attr;
        hipLaunchKernelGGL((k_fft_rows<N, -1>), dim3(rb), dim3(256), 0, s, (float2 *)data, rows);
        hipLaunchKernelGGL((k_fft_cols<N, -1>), dim3(cbk), dim3(FG::THREADS), lds, s, (float2 *)data,
                           (long)count, scale);
    } else {
        static const hipError_t attr = set_dyn_lds(k_fft_cols<N, 1>, lds);
        (void)attr;
        hipLaunchKernelGGL((k_fft_rows<N, 1>), dim3(rb), dim3(256), 0, s, (float2 *)data, rows);
        hipLaunchKernelGGL((k_fft_cols<N, 1>), dim3(cbk), dim3(FG::THREADS), lds, s, (float2 *)data,
                           (long)count, scale);
    }
    LAUNCHCHK();
    return PTYCHO_OK;
}

static hipError_t set_twiddles_here(const float2 *host) {
    return hipMemcpyToSymbol(HIP_SYMBOL(g_twiddle), host, sizeof(float2) * TW_MAX);
}

}  // namespace ptycho

// The table is built inside a host function, so that the device compilation
// emits no host data but still instantiates the kernels the passes launch.
#define PTYCHO_DEFINE_PASSES(NN)                                                                       \
    namespace ptycho {                                                                                \
    const NPass *passes_##NN() {                                                                      \
        static const NPass t = {NN, project_pass_n<NN>, forward_pass_n<NN>, fft2_n<NN>, set_twiddles_here}; \
        return &t;                                                                                    \
    }                                                                                                 \
    }
