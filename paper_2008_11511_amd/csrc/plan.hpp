// plan.hpp - host-side internals shared by the library's translation units:
// the plan structure, its workspace layout, per-kernel-class timing, error
// reporting, and the table of frame-size specific passes (one translation
// unit per frame size, inst_N.hip, instantiates the stack kernels for N).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <string>
#include <type_traits>
#include <vector>

#include "ptycho.h"
#include "common.hpp"

namespace ptycho {

// ------------------------------------------------------------------ errors --
// Records the message for ptycho_last_error() and returns code.
int fail(int code, const std::string &msg);

#define HIPCHK(x)                                                                              \
    do {                                                                                       \
        hipError_t e_ = (x);                                                                   \
        if (e_ != hipSuccess) return ::ptycho::fail(PTYCHO_E_HIP, std::string(#x) + ": " + hipGetErrorString(e_)); \
    } while (0)
#define LAUNCHCHK()                                                                            \
    do {                                                                                       \
        hipError_t e_ = hipGetLastError();                                                     \
        if (e_ != hipSuccess) return ::ptycho::fail(PTYCHO_E_HIP, std::string("kernel launch: ") + hipGetErrorString(e_)); \
    } while (0)

template <class F>
static int with_k(int k, F &&f) {
    switch (k) {
        case 1: return f(std::integral_constant<int, 1>());
        case 2: return f(std::integral_constant<int, 2>());
        case 3: return f(std::integral_constant<int, 3>());
        case 4: return f(std::integral_constant<int, 4>());
        default: return fail(PTYCHO_E_UNSUPPORTED, "unsupported number of probe modes");
    }
}

constexpr size_t ALIGN = 256;
inline size_t up(size_t x) { return (x + ALIGN - 1) / ALIGN * ALIGN; }
inline int grid_for(long n) { return (int)std::max(1L, std::min((n + 255) / 256, 4096L)); }

struct Layout {
    int S, nstacks, S_ls, nstacks_ls, maxb, maxb_ls, pchunks;
    int S_ls2, nstacks_ls2, maxb_ls2;   // line search with kept A (two sets per slot)
    size_t nlist_ints, npslots;   // object-gather block/reduce lists, partial slots
    size_t nent_max, nfr_max, nred;
    size_t off_offs, off_order, off_lists, off_ent_fr, off_opart, off_scr, off_q, off_pint, off_numO, off_denO,
        off_numP, off_denP, off_pnum, off_pden, off_part, off_red, off_scal, off_s2, off_bsum, off_prop,
        off_pspart, off_shift, off_pos, off_pos0, off_frac, total;
    int pos_chunks;               // row chunks per frame of the position-shift sums
};

// Per-kernel-class timing with HIP events on the plan's stream.
enum { TC_ROWS_FWD = 0, TC_COLS = 1, TC_ROWS_INV = 2, TC_GATHER_OBJ = 3, TC_GATHER_PROBE = 4,
       TC_PROBE_ALL = 5, TC_NORMALIZE = 6, TC_OTHER = 7, TC_N = 8 };

struct TimingLog {
    bool on = false;
    unsigned mask = 0;      // classes recorded (bit c: class c)
    std::vector<hipEvent_t> pool;
    std::vector<int> cls;   // class of event pair i (events 2i, 2i+1)
    size_t used = 0;        // pairs recorded
};

}  // namespace ptycho

struct ptycho_plan_s {
    ptycho_desc_t d;
    ptycho::TimingLog timing;
    ptycho::Layout L;
    hipStream_t stream;
    const float *iobs;
    const uint8_t *mask;
    char *ws;
    int2 *offs;
    int *order;
    int4 *ent_fr;
    int *lists;          // device copy of h_lists
    float2 *opnum;       // object-gather chunk partials
    float *opden;
    float2 *scr, *q, *numO, *numP, *pnum;
    float *bg = nullptr;     // caller's background [N][N] (set_background), or null
    float *s2 = nullptr;     // [S][N][N] with PTYCHO_FLAG_BACKGROUND
    double *bsum = nullptr;  // [N][N]
    float2 *prop = nullptr;  // [2][N] with PTYCHO_FLAG_NEAR_FIELD
    bool nf_ready = false;   // Fresnel parameters set
    double *pspart = nullptr;    // position-shift partial sums [J][pos_chunks][5]
    double *shifts = nullptr;    // [J][3] shifts of the last refinement step
    // PTYCHO_FLAG_POSITIONS: real window corners t (current and start),
    // their fractions, the update parameters; pos_ready once set
    double *pos = nullptr, *pos0 = nullptr;
    float2 *frac = nullptr;
    bool pos_ready = false;
    double pos_mult = 1.0, pos_min_grad = 0.1;
    bool shifts_in_grad = false; // the gradient pass also takes the ML position shifts
    std::vector<float2> h_prop;
    std::vector<double> h_pos;   // host copies of the uploaded corners and fractions
    std::vector<float2> h_frac;
    float *pint, *denO, *denP, *pden, *part;
    double *red, *scal;
    int ntx, nty;
    // Object-gather lists.  A list is a run of blocks (tile, entry range,
    // partial slot or -1) followed by a run of reductions (split tile, first
    // slot, count), stored in h_lists; GatherList gives the offsets.
    struct GatherList {
        int nb, blk_tile, blk_ptr, blk_slot, nr, red_tile, red_first, red_count;
    };
    std::vector<GatherList> stack_lists;
    std::vector<int> h_lists;
    // host copies kept alive for the asynchronous uploads
    std::vector<int2> h_offs;
    std::vector<int> h_order;
    std::vector<int4> h_fr;
};

namespace ptycho {

// Records an event pair around the launches made while it is alive.
struct Timed {
    ptycho_plan_s *p;
    int c;
    size_t pair;
    bool rec = false;
    Timed(ptycho_plan_s *p_, int c_) : p(p_), c(c_), pair(0) {
        TimingLog &t = p->timing;
        if (!t.on || !((t.mask >> c) & 1u)) return;
        pair = t.used++;
        while (t.pool.size() < 2 * t.used) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) { t.on = false; return; }
            t.pool.push_back(e);
        }
        if (t.cls.size() < t.used) t.cls.resize(t.used);
        t.cls[pair] = c;
        (void)hipEventRecord(t.pool[2 * pair], p->stream);
        rec = true;
    }
    ~Timed() {
        TimingLog &t = p->timing;
        if (rec && t.on) (void)hipEventRecord(t.pool[2 * pair + 1], p->stream);
    }
};

// Calls f(std::true_type) on a near-field plan, f(std::false_type) otherwise.
template <class F>
static int with_nf(const ptycho_plan_s *p, F &&f) {
    if (p->prop) return f(std::true_type{});
    return f(std::false_type{});
}

// Which sums a projection pass accumulates.
enum { ACC_OBJ = 1, ACC_PROBE = 2 };

// Helpers defined in ptycho.hip, used by the frame-size specific passes.
StackArgs stack_args(ptycho_plan_s *p, int s0, int sn, const float *obj, const float *probe);
int object_sums(ptycho_plan_s *p, int sidx);
int probe_sums(ptycho_plan_s *p, const float *obj, const float2 *psi, int q0, int nq, bool from_scr,
               bool accumulate);
int launch_probe_intensity(ptycho_plan_s *p, const float *probe);
int launch_bg_accum(ptycho_plan_s *p, int sn, int first);
// ML position shifts of the stack's slots s0 .. s0+sn from the gradient wave
// the inverse row pass left in the stack scratch.
int launch_ml_shifts(ptycho_plan_s *p, const float *obj, const float *probe, int s0, int sn);

// The passes of one frame size N (inst_N.hip).
struct NPass {
    int n;
    // One pass over all stacks (kind: 0 AP projection, 1 DM, 2 ML gradient)
    // with the per-stack sums selected by acc.
    // keep (nullable): [J][K][N][N] column-tiled buffer that receives the
    // forward row transforms of every frame (slot order), read by the column
    // pass from there; the ML cycle's line search reuses them.
    int (*project)(ptycho_plan_s *p, const float *obj, const float *probe, float *psi, int kind, unsigned acc,
                   bool upd_bg, float2 *keep);
    // Read-only forward pass of column op `op` (OP_LLK, OP_ICALC, OP_LS, and
    // OP_LS2: the line search with A read from `keep`).
    int (*forward)(ptycho_plan_s *p, int op, const float *obj, const float *probe, const float *dobj,
                   const float *dprobe, float *icalc, int llk_model, const float2 *keep);
    // Plain batched unitary 2D FFT.
    int (*fft2)(int32_t count, float *data, int32_t dir, hipStream_t s);
    // Copies the twiddle table into this translation unit's constant memory
    // (current device).
    hipError_t (*set_twiddles)(const float2 *host);
};

}  // namespace ptycho
