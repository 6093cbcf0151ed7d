// ptycho.hip - host side of the C ABI declared in include/ptycho.h.
//
// A plan holds the index tables of one scan (integer offsets, the frame
// order in which stacks are formed, and for every stack the list of object
// tiles it touches with, per tile, the covering frames), carved from the
// caller's workspace together with the stack scratch, the per-cycle overlap
// sums and the reduction partials.  Every entry point validates on the host,
// then enqueues kernels on the plan's stream and returns.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <deque>
#include <mutex>
#include <string>
#include <vector>

#include "ptycho.h"
#include "plan.hpp"
#include "kernels.hpp"
#include "mlcg.hpp"

using namespace ptycho;

// ------------------------------------------------------------------ errors --
static thread_local std::string g_err;
int ptycho::fail(int code, const std::string &msg) {
    g_err = msg;
    return code;
}

extern "C" const char *ptycho_last_error(void) { return g_err.c_str(); }

// ------------------------------------------------------ frame-size table --
// The stack kernels of each frame size live in a translation unit of their
// own (inst_N.hip).  PTYCHO_KERNEL_N_MAX (a build option of the host-only
// sanitizer test, whose program launches nothing) limits the sizes linked
// in; the library is built with all of them.
#ifndef PTYCHO_KERNEL_N_MAX
#define PTYCHO_KERNEL_N_MAX 2048
#endif
namespace ptycho {
const NPass *passes_8();
#if PTYCHO_KERNEL_N_MAX >= 16
const NPass *passes_16();
const NPass *passes_32();
const NPass *passes_64();
const NPass *passes_128();
const NPass *passes_256();
const NPass *passes_512();
const NPass *passes_1024();
const NPass *passes_2048();
#endif
}  // namespace ptycho

static const NPass *(*const g_passes[])() = {
    passes_8,
#if PTYCHO_KERNEL_N_MAX >= 16
    passes_16, passes_32, passes_64, passes_128, passes_256, passes_512, passes_1024, passes_2048,
#endif
};

static bool supported_n(int n) {
    return n == 8 || n == 16 || n == 32 || n == 64 || n == 128 || n == 256 || n == 512 || n == 1024 || n == 2048;
}

// The passes of frame size n, or null (with the error recorded).
static const NPass *passes_for(int n) {
    for (auto get : g_passes)
        if (get()->n == n) return get();
    fail(PTYCHO_E_UNSUPPORTED, supported_n(n) ? "frame size not compiled into this library" : "unsupported frame size");
    return nullptr;
}

// --------------------------------------------------------------- twiddles --
static std::mutex g_tw_mu;
static std::vector<int> g_tw_done;

static int ensure_twiddles() {
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_tw_mu);
    if ((int)g_tw_done.size() <= dev) g_tw_done.resize(dev + 1, 0);
    if (g_tw_done[dev]) return PTYCHO_OK;
    std::vector<float2> h(TW_MAX);
    for (int m = 0; m < TW_MAX; ++m) {
        const double a = -2.0 * M_PI * (double)m / (double)TW_MAX;
        h[m] = make_float2((float)std::cos(a), (float)std::sin(a));
    }
    for (auto get : g_passes) HIPCHK(get()->set_twiddles(h.data()));
    HIPCHK(hipDeviceSynchronize());
    g_tw_done[dev] = 1;
    return PTYCHO_OK;
}

static constexpr int NPART = 512;       // blocks of the max-reduction
static constexpr int NSCAL = 64;        // device scalars
static constexpr int SC_NOBS = 0;       //   unmasked pixels of all frames (double)

// Frame chunks of the all-frame probe gather: enough blocks to fill the
// chip (about 4096), never more chunks than frames.
static int probe_chunks(const ptycho_desc_t &d) {
    const long blocks = (long)((d.n * d.n + 255) / 256);
    long c = (4096 + blocks - 1) / blocks;
    c = std::max(1L, std::min(c, 32L));
    return (int)std::min<long>(c, d.n_frames);
}

// Object margin of a frame's tile coverage: windows of a positions plan move
// up to max_shift pixels and view one more row and column.
static int window_margin(const ptycho_desc_t &d) {
    return (d.flags & PTYCHO_FLAG_POSITIONS) ? (int)std::ceil((double)d.max_shift) + 1 : 0;
}

// Frames per thread of the position-shift sums: the frames share each probe
// load (two: 0.32 -> 0.295 ms per call at 1000 x 256^2 x 3 modes; three
// frames leave two waves per SIMD and are slower).
static constexpr int SHIFT_FRAMES = 2;
// Rows per chunk of the position-shift sums: about 16384 pixels per block.
static int pos_rows(int n) { return std::max(1, std::min(n, 16384 / n)); }

// Frames per launch.  The stack kernels are bandwidth-bound and do not keep
// data in cache from one launch to the next, so larger launches (fewer
// launches, smaller tails, one object gather per cycle) are faster; the
// scratch is sized to up to 32 GiB of the 288 GB of HBM, one stack for a
// 4000-frame scan of 512^2 frames with 4 modes (AP and DM cycles 4% faster
// than in stacks of 256 frames).
static int auto_stack(const ptycho_desc_t &d) {
    if (d.stack > 0) return std::min(d.stack, d.n_frames);
    const double per = (double)d.n_modes * d.n * d.n * 8.0;
    int s = (int)std::floor((32.0 * 1024 * 1024 * 1024) / per);
    s = std::max(1, std::min(s, d.n_frames));
    return s;
}

static Layout layout_for(const ptycho_desc_t &d) {
    Layout L{};
    const int J = d.n_frames, N = d.n, K = d.n_modes;
    L.S = auto_stack(d);
    L.nstacks = (J + L.S - 1) / L.S;
    L.S_ls = std::max(1, L.S / 3);
    L.nstacks_ls = (J + L.S_ls - 1) / L.S_ls;
    // the scratch holds max(S, 3 S_ls) frame-modes per mode; two sets per slot
    L.S_ls2 = std::max(1, std::min(J, std::max(L.S, 3 * L.S_ls) / 2));
    L.nstacks_ls2 = (J + L.S_ls2 - 1) / L.S_ls2;
    const int cb = col_cb(N);
    L.maxb = (int)(((long)L.S * N + cb - 1) / cb);
    L.maxb_ls = (int)(((long)L.S_ls * N + cb - 1) / cb);
    L.maxb_ls2 = (int)(((long)L.S_ls2 * N + cb - 1) / cb);
    const int mg = window_margin(d);
    const long ty = (N + 2 * mg + OTILE_Y - 1) / OTILE_Y + 1, tx = (N + 2 * mg + OTILE_X - 1) / OTILE_X + 1;
    L.nfr_max = (size_t)J * ty * tx;
    const long ntx = (d.obj_nx + OTILE_X - 1) / OTILE_X, nty = (d.obj_ny + OTILE_Y - 1) / OTILE_Y;
    const long ntiles = ntx * nty;
    L.nent_max = std::min((size_t)L.nstacks * ntiles, L.nfr_max);
    // object-gather lists per stack: per block tile, entry range, partial
    // slot (plus one end pointer per list); per split tile: tile, first
    // slot, count
    const size_t nb_st = L.nent_max + L.nfr_max / 16 + L.nstacks;
    L.nlist_ints = 3 * nb_st + 3 * L.nent_max + 2;
    L.npslots = std::min<size_t>(8192, L.nfr_max / 8 + 1);
    L.nred = std::max({(size_t)L.nstacks * L.maxb, (size_t)L.nstacks_ls * L.maxb_ls * 2,
                       (size_t)L.nstacks_ls2 * L.maxb_ls2 * 2});
    L.pchunks = probe_chunks(d);
    L.pos_chunks = N / pos_rows(N);
    const size_t n2 = (size_t)N * N, no = (size_t)d.obj_ny * d.obj_nx;
    size_t o = 0;
    L.off_offs = o; o = up(o + sizeof(int2) * J);
    L.off_order = o; o = up(o + sizeof(int) * J);
    L.off_lists = o; o = up(o + sizeof(int) * L.nlist_ints);
    L.off_ent_fr = o; o = up(o + sizeof(int4) * L.nfr_max);
    L.off_opart = o; o = up(o + (sizeof(float2) + sizeof(float)) * L.npslots * OTILE_Y * OTILE_X);
    L.off_scr = o; o = up(o + sizeof(float2) * (size_t)std::max(L.S, 3 * L.S_ls) * K * n2);
    L.off_q = o; o = up(o + sizeof(float2) * (size_t)L.S * n2);
    L.off_pint = o; o = up(o + sizeof(float) * n2);
    L.off_numO = o; o = up(o + sizeof(float2) * no);
    L.off_denO = o; o = up(o + sizeof(float) * no);
    L.off_numP = o; o = up(o + sizeof(float2) * K * n2);
    L.off_denP = o; o = up(o + sizeof(float) * n2);
    L.off_pnum = o; o = up(o + sizeof(float2) * (size_t)L.pchunks * K * n2);
    L.off_pden = o; o = up(o + sizeof(float) * (size_t)L.pchunks * n2);
    L.off_part = o; o = up(o + sizeof(float) * 2 * NPART);
    L.off_red = o; o = up(o + sizeof(double) * L.nred);
    L.off_scal = o; o = up(o + sizeof(double) * NSCAL);
    // background refinement (AP): s^2 of a stack's frames and their sums
    const bool bgu = (d.flags & PTYCHO_FLAG_BACKGROUND) != 0;
    L.off_s2 = o; o = up(o + (bgu ? sizeof(float) * (size_t)L.S * n2 : 0));
    L.off_bsum = o; o = up(o + (bgu ? sizeof(double) * n2 : 0));
    // near field: the transfer-function factors Qy / N, Qx / N
    const bool nfg = (d.flags & PTYCHO_FLAG_NEAR_FIELD) != 0;
    L.off_prop = o; o = up(o + (nfg ? sizeof(float2) * 2 * (size_t)N : 0));
    // position refinement: shift partials and shifts; real corners and
    // fractions of a positions plan
    L.off_pspart = o; o = up(o + sizeof(double) * 5 * (size_t)L.pos_chunks * J);
    L.off_shift = o; o = up(o + sizeof(double) * 3 * (size_t)J);
    const bool pst = (d.flags & PTYCHO_FLAG_POSITIONS) != 0;
    L.off_pos = o; o = up(o + (pst ? sizeof(double) * 2 * (size_t)J : 0));
    L.off_pos0 = o; o = up(o + (pst ? sizeof(double) * 2 * (size_t)J : 0));
    L.off_frac = o; o = up(o + (pst ? sizeof(float2) * (size_t)J : 0));
    L.total = o;
    return L;
}

// ---------------------------------------------------------------- validate --
static int check_desc(const ptycho_desc_t *d) {
    if (!d) return fail(PTYCHO_E_INVALID, "null descriptor");
    if (!supported_n(d->n)) return fail(PTYCHO_E_UNSUPPORTED, "frame size must be a power of two from 8 to 2048");
    if (d->n_modes < 1 || d->n_modes > 4) return fail(PTYCHO_E_UNSUPPORTED, "probe modes must be 1..4");
    if (d->n_frames < 1) return fail(PTYCHO_E_INVALID, "n_frames must be >= 1");
    if (d->obj_ny < d->n || d->obj_nx < d->n) return fail(PTYCHO_E_INVALID, "object smaller than a frame");
    if ((long)d->obj_ny * d->obj_nx > (1L << 31) - 1) return fail(PTYCHO_E_INVALID, "object too large");
    if (d->stack < 0) return fail(PTYCHO_E_INVALID, "negative stack");
    if (!(d->obj_inertia >= 0.0f) || !(d->probe_inertia >= 0.0f)) return fail(PTYCHO_E_INVALID, "negative inertia");
    if (!(d->icalc_floor > 0.0f)) return fail(PTYCHO_E_INVALID, "icalc_floor must be > 0");
    if (d->flags & ~(PTYCHO_FLAG_BACKGROUND | PTYCHO_FLAG_NEAR_FIELD | PTYCHO_FLAG_POSITIONS))
        return fail(PTYCHO_E_INVALID, "unknown descriptor flag");
    if ((d->flags & PTYCHO_FLAG_POSITIONS) && !(d->max_shift >= 0.0f && d->max_shift <= 0.25f * d->n))
        return fail(PTYCHO_E_INVALID, "max_shift must be within [0, N/4] pixels");
    return PTYCHO_OK;
}

// ------------------------------------------------------------- host entries --
extern "C" int ptycho_offsets_from_positions(const double *pos, int32_t J, int32_t n, int32_t ny, int32_t nx,
                                             int32_t *out) {
    if (!pos || !out) return fail(PTYCHO_E_INVALID, "null pointer");
    if (J < 0 || n < 1 || ny < n || nx < n) return fail(PTYCHO_E_INVALID, "bad sizes");
    std::vector<int32_t> tmp((size_t)J * 2);
    const double cy = ny / 2.0, cx = nx / 2.0;
    for (int32_t j = 0; j < J; ++j) {
        const double fy = std::floor(cy + pos[2 * j] + 0.5), fx = std::floor(cx + pos[2 * j + 1] + 0.5);
        if (!std::isfinite(fy) || !std::isfinite(fx)) return fail(PTYCHO_E_BOUNDS, "non-finite position");
        const double oy = fy - (double)(n / 2), ox = fx - (double)(n / 2);
        if (oy < 0 || ox < 0 || oy > ny - n || ox > nx - n)
            return fail(PTYCHO_E_BOUNDS, "scan position window outside the object (frame " + std::to_string(j) + ")");
        tmp[2 * j] = (int32_t)oy;
        tmp[2 * j + 1] = (int32_t)ox;
    }
    std::memcpy(out, tmp.data(), sizeof(int32_t) * tmp.size());
    return PTYCHO_OK;
}

extern "C" int ptycho_windows_from_positions(const double *pos, int32_t J, int32_t n, int32_t ny, int32_t nx,
                                             int32_t *offsets, double *frac) {
    if (!pos || !offsets || !frac) return fail(PTYCHO_E_INVALID, "null pointer");
    if (J < 0 || n < 1 || ny < n || nx < n) return fail(PTYCHO_E_INVALID, "bad sizes");
    std::vector<int32_t> o((size_t)J * 2);
    std::vector<double> f((size_t)J * 2);
    const double c[2] = {ny / 2.0, nx / 2.0};
    const int lim[2] = {ny - n, nx - n};
    for (int32_t j = 0; j < J; ++j)
        for (int ax = 0; ax < 2; ++ax) {
            const double t = c[ax] + pos[2 * j + ax] - n / 2.0;
            if (!(t >= 0.0) || !(t <= (double)lim[ax]))
                return fail(PTYCHO_E_BOUNDS, "scan position window outside the object (frame " + std::to_string(j) + ")");
            const double fl = std::floor(t);
            o[2 * j + ax] = (int32_t)fl;
            f[2 * j + ax] = t - fl;
        }
    std::memcpy(offsets, o.data(), sizeof(int32_t) * o.size());
    std::memcpy(frac, f.data(), sizeof(double) * f.size());
    return PTYCHO_OK;
}

extern "C" int ptycho_workspace_bytes(const ptycho_desc_t *d, size_t *bytes) {
    int st = check_desc(d);
    if (st) return st;
    if (!bytes) return fail(PTYCHO_E_INVALID, "null output");
    *bytes = layout_for(*d).total;
    return PTYCHO_OK;
}

static uint32_t spread_bits(uint32_t v) {
    v &= 0xffffu;
    v = (v | (v << 8)) & 0x00ff00ffu;
    v = (v | (v << 4)) & 0x0f0f0f0fu;
    v = (v | (v << 2)) & 0x33333333u;
    v = (v | (v << 1)) & 0x55555555u;
    return v;
}

// Host-side index tables of a plan: frame order, object-gather lists.  No
// GPU work; shared by ptycho_plan and ptycho_plan_dry_run.
static int build_host_tables(ptycho_plan_s *p, const Layout &L, const int32_t *offsets) {
    const ptycho_desc_t *d = &p->d;
    const int J = d->n_frames, N = d->n;
    const int mg = window_margin(*d);
    // frame order: Morton (Z) order of the window corners, so that every
    // stack covers a compact patch of the object
    p->h_offs.resize(J);
    std::vector<std::pair<uint64_t, int>> key(J);
    for (int j = 0; j < J; ++j) {
        p->h_offs[j] = make_int2(offsets[2 * j], offsets[2 * j + 1]);
        const uint32_t z = spread_bits((uint32_t)offsets[2 * j]) << 1 | spread_bits((uint32_t)offsets[2 * j + 1]);
        key[j] = {((uint64_t)z << 32) | (uint32_t)j, j};
    }
    std::sort(key.begin(), key.end());
    p->h_order.resize(J);
    for (int j = 0; j < J; ++j) p->h_order[j] = key[j].second;

    // Object-gather lists: per stack, the touched object tiles with, per
    // tile, entries (slot, oy, ox) of the covering frames in slot order.
    // Tiles with the most entries come first; a tile with more than F entries
    // (F ~ entries / 4096, at least 16) is split into chunks of at most F
    // whose partial sums a reduction adds in chunk order, so no block carries
    // a much longer serial frame loop than the others.
    const int ntiles = p->ntx * p->nty;
    std::vector<std::vector<int4>> per_tile(ntiles);
    int max_slots = 0;
    auto emit_list = [&](std::vector<int> &tiles, std::vector<int4> &ents, size_t ent_base) {
        std::stable_sort(tiles.begin(), tiles.end(),
                         [&](int a, int b) { return per_tile[a].size() > per_tile[b].size(); });
        size_t total = 0;
        for (int t : tiles) total += per_tile[t].size();
        const int F = (int)std::max<size_t>(16, (total + 4095) / 4096);
        std::vector<int> bt, bp, bs, rt, rf, rc;
        int slots = 0;
        for (int t : tiles) {
            auto &v = per_tile[t];
            const int n = (int)v.size();
            const int nch = (n + F - 1) / F;
            if (nch > 1) {
                rt.push_back(t);
                rf.push_back(slots);
                rc.push_back(nch);
            }
            for (int c = 0; c < nch; ++c) {
                bt.push_back(t);
                bp.push_back((int)(ents.size() - ent_base) + c * F);
                bs.push_back(nch > 1 ? slots + c : -1);
            }
            if (nch > 1) slots += nch;
            ents.insert(ents.end(), v.begin(), v.end());
            v.clear();
        }
        bp.push_back((int)(ents.size() - ent_base));
        max_slots = std::max(max_slots, slots);
        ptycho_plan_s::GatherList gl{};
        auto put = [&](const std::vector<int> &x) {
            const int at = (int)p->h_lists.size();
            p->h_lists.insert(p->h_lists.end(), x.begin(), x.end());
            return at;
        };
        gl.nb = (int)bt.size();
        gl.blk_tile = put(bt);
        gl.blk_ptr = put(bp);
        gl.blk_slot = put(bs);
        gl.nr = (int)rt.size();
        gl.red_tile = put(rt);
        gl.red_first = put(rf);
        gl.red_count = put(rc);
        return gl;
    };
    std::vector<int> touched;
    for (int sidx = 0; sidx < L.nstacks; ++sidx) {
        const int s0 = sidx * L.S, sn = std::min(L.S, J - s0);
        touched.clear();
        for (int s = 0; s < sn; ++s) {
            const int jf = p->h_order[s0 + s];
            const int2 o = p->h_offs[jf];
            const int y0 = std::max(0, o.x - mg), y1 = std::min(d->obj_ny - 1, o.x + N - 1 + mg);
            const int x0 = std::max(0, o.y - mg), x1 = std::min(d->obj_nx - 1, o.y + N - 1 + mg);
            for (int ty = y0 / OTILE_Y; ty <= y1 / OTILE_Y; ++ty)
                for (int tx = x0 / OTILE_X; tx <= x1 / OTILE_X; ++tx) {
                    auto &v = per_tile[ty * p->ntx + tx];
                    if (v.empty()) touched.push_back(ty * p->ntx + tx);
                    v.push_back(make_int4(s, o.x, o.y, jf));
                }
        }
        std::sort(touched.begin(), touched.end());
        p->stack_lists.push_back(emit_list(touched, p->h_fr, 0));
    }
    if (p->h_fr.size() > L.nfr_max || p->h_lists.size() > L.nlist_ints ||
        (size_t)max_slots > L.npslots) {
        return fail(PTYCHO_E_WORKSPACE, "internal: object-gather lists exceed their bound");
    }
    return PTYCHO_OK;
}

// Page-locked staging of the plan tables, one buffer per process used as a
// ring.  A copy from pageable host memory can make the host wait for the
// stream; from the ring it is a plain asynchronous DMA.  Each use records an
// event, and a region is reused only once the uses overlapping it are done.
// Tables larger than the ring are copied from the plan's own host vectors.
struct StagingRing {
    static constexpr size_t CAP = size_t(64) << 20;
    std::mutex m;
    char *buf = nullptr;
    bool failed = false;
    size_t head = 0;
    struct Use { size_t a, b; hipEvent_t ev; };
    std::deque<Use> uses;
};
static StagingRing g_ring;

struct HostPart { void *dst; const void *src; size_t bytes; };

static hipError_t upload_tables(const std::vector<HostPart> &parts, hipStream_t stream) {
    size_t total = 0;
    for (const HostPart &h : parts) total += up(h.bytes);
    StagingRing &r = g_ring;
    std::lock_guard<std::mutex> lk(r.m);
    if (!r.buf && !r.failed) {
        if (hipHostMalloc((void **)&r.buf, StagingRing::CAP, hipHostMallocDefault) != hipSuccess) {
            r.buf = nullptr;
            r.failed = true;
            (void)hipGetLastError();
        }
    }
    if (!r.buf || total > StagingRing::CAP) {
        for (const HostPart &h : parts) {
            if (!h.bytes) continue;
            hipError_t e = hipMemcpyAsync(h.dst, h.src, h.bytes, hipMemcpyHostToDevice, stream);
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    }
    // drop finished uses; wrap; wait for the uses that overlap the region
    while (!r.uses.empty() && hipEventQuery(r.uses.front().ev) == hipSuccess) {
        (void)hipEventDestroy(r.uses.front().ev);
        r.uses.pop_front();
    }
    if (r.head + total > StagingRing::CAP) r.head = 0;
    const size_t a = r.head, b = r.head + total;
    for (;;) {
        bool overlap = false;
        for (const StagingRing::Use &u : r.uses) overlap |= (u.a < b && a < u.b);
        if (!overlap) break;
        hipError_t e = hipEventSynchronize(r.uses.front().ev);
        (void)hipEventDestroy(r.uses.front().ev);
        r.uses.pop_front();
        if (e != hipSuccess) return e;
    }
    size_t o = a;
    for (const HostPart &h : parts) {
        if (!h.bytes) continue;
        std::memcpy(r.buf + o, h.src, h.bytes);
        hipError_t e = hipMemcpyAsync(h.dst, r.buf + o, h.bytes, hipMemcpyHostToDevice, stream);
        if (e != hipSuccess) return e;
        o += up(h.bytes);
    }
    hipEvent_t ev;
    hipError_t e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventRecord(ev, stream);
    if (e != hipSuccess) {
        // without an event the region cannot be tracked: wait for the copies
        (void)hipStreamSynchronize(stream);
        return e;
    }
    r.uses.push_back({a, b, ev});
    r.head = b;
    return hipSuccess;
}

extern "C" int ptycho_plan(const ptycho_desc_t *d, const int32_t *offsets, const float *iobs,
                                  const uint8_t *mask, void *ws, size_t ws_bytes, void *stream,
                                  ptycho_plan_t *out) {
    int st = check_desc(d);
    if (st) return st;
    if (!offsets || !iobs || !out) return fail(PTYCHO_E_INVALID, "null pointer");
    const Layout L = layout_for(*d);
    if (!ws) return fail(PTYCHO_E_WORKSPACE, "null workspace");
    if (((uintptr_t)ws) % ALIGN) return fail(PTYCHO_E_WORKSPACE, "workspace not 256-byte aligned");
    if (ws_bytes < L.total) return fail(PTYCHO_E_WORKSPACE, "workspace too small");
    const int J = d->n_frames, N = d->n;
    for (int j = 0; j < J; ++j) {
        const int oy = offsets[2 * j], ox = offsets[2 * j + 1];
        if (oy < 0 || ox < 0 || oy > d->obj_ny - N || ox > d->obj_nx - N)
            return fail(PTYCHO_E_BOUNDS, "frame window outside the object (frame " + std::to_string(j) + ")");
    }
    auto *p = new ptycho_plan_s();
    p->d = *d;
    p->L = L;
    p->stream = (hipStream_t)stream;
    p->iobs = iobs;
    p->mask = mask;
    p->ws = (char *)ws;
    p->offs = (int2 *)(p->ws + L.off_offs);
    p->order = (int *)(p->ws + L.off_order);
    p->lists = (int *)(p->ws + L.off_lists);
    p->ent_fr = (int4 *)(p->ws + L.off_ent_fr);
    p->opnum = (float2 *)(p->ws + L.off_opart);
    p->opden = (float *)(p->opnum + L.npslots * OTILE_Y * OTILE_X);
    p->scr = (float2 *)(p->ws + L.off_scr);
    p->q = (float2 *)(p->ws + L.off_q);
    p->pint = (float *)(p->ws + L.off_pint);
    p->numO = (float2 *)(p->ws + L.off_numO);
    p->denO = (float *)(p->ws + L.off_denO);
    p->numP = (float2 *)(p->ws + L.off_numP);
    p->denP = (float *)(p->ws + L.off_denP);
    p->pnum = (float2 *)(p->ws + L.off_pnum);
    p->pden = (float *)(p->ws + L.off_pden);
    p->part = (float *)(p->ws + L.off_part);
    p->red = (double *)(p->ws + L.off_red);
    p->scal = (double *)(p->ws + L.off_scal);
    if (d->flags & PTYCHO_FLAG_BACKGROUND) {
        p->s2 = (float *)(p->ws + L.off_s2);
        p->bsum = (double *)(p->ws + L.off_bsum);
    }
    if (d->flags & PTYCHO_FLAG_NEAR_FIELD) p->prop = (float2 *)(p->ws + L.off_prop);
    p->pspart = (double *)(p->ws + L.off_pspart);
    p->shifts = (double *)(p->ws + L.off_shift);
    if (d->flags & PTYCHO_FLAG_POSITIONS) {
        p->pos = (double *)(p->ws + L.off_pos);
        p->pos0 = (double *)(p->ws + L.off_pos0);
        p->frac = (float2 *)(p->ws + L.off_frac);
    }
    p->ntx = (d->obj_nx + OTILE_X - 1) / OTILE_X;
    p->nty = (d->obj_ny + OTILE_Y - 1) / OTILE_Y;

    st = build_host_tables(p, L, offsets);
    if (!st) st = ensure_twiddles();
    if (st) {
        delete p;
        return st;
    }
    hipError_t e = upload_tables({{p->offs, p->h_offs.data(), sizeof(int2) * J},
                                  {p->order, p->h_order.data(), sizeof(int) * J},
                                  {p->lists, p->h_lists.data(), sizeof(int) * p->h_lists.size()},
                                  {p->ent_fr, p->h_fr.data(), sizeof(int4) * p->h_fr.size()}},
                                 p->stream);
    if (e == hipSuccess) {
        // number of unmasked pixels of all frames, kept on the device (the
        // plan never waits for its stream)
        hipLaunchKernelGGL(k_count_good, dim3(1), dim3(256), 0, p->stream, mask, N * N, (double)J,
                           p->scal + SC_NOBS);
        e = hipGetLastError();
    }
    if (e != hipSuccess) {
        delete p;
        return fail(PTYCHO_E_HIP, std::string("plan upload: ") + hipGetErrorString(e));
    }
    *out = p;
    return PTYCHO_OK;
}

extern "C" int ptycho_plan_dry_run(const ptycho_desc_t *d, const int32_t *offsets, size_t *table_bytes) {
    int st = check_desc(d);
    if (st) return st;
    if (!offsets || !table_bytes) return fail(PTYCHO_E_INVALID, "null pointer");
    const Layout L = layout_for(*d);
    const int J = d->n_frames, N = d->n;
    for (int j = 0; j < J; ++j) {
        const int oy = offsets[2 * j], ox = offsets[2 * j + 1];
        if (oy < 0 || ox < 0 || oy > d->obj_ny - N || ox > d->obj_nx - N)
            return fail(PTYCHO_E_BOUNDS, "frame window outside the object (frame " + std::to_string(j) + ")");
    }
    ptycho_plan_s p{};
    p.d = *d;
    p.L = L;
    p.ntx = (d->obj_nx + OTILE_X - 1) / OTILE_X;
    p.nty = (d->obj_ny + OTILE_Y - 1) / OTILE_Y;
    st = build_host_tables(&p, L, offsets);
    if (st) return st;
    *table_bytes = sizeof(int) * p.h_lists.size() + sizeof(int4) * p.h_fr.size() +
                   sizeof(int) * p.h_order.size() + sizeof(int2) * p.h_offs.size();
    return PTYCHO_OK;
}

extern "C" int ptycho_plan_set_background(ptycho_plan_t p, float *bg) {
    if (!p) return fail(PTYCHO_E_INVALID, "null plan");
    p->bg = bg;
    return PTYCHO_OK;
}

extern "C" int ptycho_plan_set_near_field(ptycho_plan_t p, double fy, double fx) {
    if (!p) return fail(PTYCHO_E_INVALID, "null plan");
    if (!p->prop) return fail(PTYCHO_E_INVALID, "a near-field plan needs PTYCHO_FLAG_NEAR_FIELD");
    if (!std::isfinite(fy) || !std::isfinite(fx)) return fail(PTYCHO_E_INVALID, "non-finite Fresnel parameter");
    const int N = p->d.n;
    // exp(-i f u'^2) / N in double, the phase reduced modulo 2 pi first
    std::vector<float2> h(2 * (size_t)N);
    const double two_pi = 6.283185307179586476925286766559;
    for (int axis = 0; axis < 2; ++axis) {
        const double f = axis == 0 ? fy : fx;
        for (int u = 0; u < N; ++u) {
            const double us = (u < N / 2) ? u : u - N;
            const double ph = std::fmod(f * us * us, two_pi);
            h[(size_t)axis * N + u] = make_float2((float)(std::cos(ph) / N), (float)(-std::sin(ph) / N));
        }
    }
    p->h_prop.swap(h);
    hipError_t e = upload_tables({{p->prop, p->h_prop.data(), sizeof(float2) * p->h_prop.size()}}, p->stream);
    if (e != hipSuccess) return fail(PTYCHO_E_HIP, std::string("near-field table upload: ") + hipGetErrorString(e));
    p->nf_ready = true;
    return PTYCHO_OK;
}

// Entry points that propagate need the Fresnel parameters of a near-field plan.
static int check_geometry(const ptycho_plan_s *p) {
    if (p->prop && !p->nf_ready)
        return fail(PTYCHO_E_INVALID, "near-field plan without Fresnel parameters (ptycho_plan_set_near_field)");
    return PTYCHO_OK;
}

extern "C" int ptycho_plan_set_stream(ptycho_plan_t p, void *stream) {
    if (!p) return fail(PTYCHO_E_INVALID, "null plan");
    p->stream = (hipStream_t)stream;
    return PTYCHO_OK;
}

extern "C" int ptycho_plan_stack(ptycho_plan_t p, int32_t *s) {
    if (!p || !s) return fail(PTYCHO_E_INVALID, "null pointer");
    *s = p->L.S;
    return PTYCHO_OK;
}

extern "C" int ptycho_plan_destroy(ptycho_plan_t p) {
    if (p)
        for (hipEvent_t e : p->timing.pool) (void)hipEventDestroy(e);
    delete p;
    return PTYCHO_OK;
}

extern "C" int ptycho_plan_timing(ptycho_plan_t p, int32_t classes) {
    if (!p) return fail(PTYCHO_E_INVALID, "null plan");
    if (classes < 0 || classes >= (1 << TC_N)) return fail(PTYCHO_E_INVALID, "bad timing class mask");
    p->timing.on = classes != 0;
    p->timing.mask = (unsigned)classes;
    if (classes) p->timing.used = 0;
    return PTYCHO_OK;
}

extern "C" int ptycho_plan_timing_read(ptycho_plan_t p, int32_t cls, double *ms_total, int64_t *launches) {
    if (!p || !ms_total || !launches) return fail(PTYCHO_E_INVALID, "null pointer");
    if (cls < 0 || cls >= TC_N) return fail(PTYCHO_E_INVALID, "bad timing class");
    TimingLog &t = p->timing;
    double tot = 0.0;
    int64_t n = 0;
    if (t.used) HIPCHK(hipEventSynchronize(t.pool[2 * t.used - 1]));
    for (size_t i = 0; i < t.used; ++i) {
        if (t.cls[i] != cls) continue;
        float ms = 0.0f;
        HIPCHK(hipEventElapsedTime(&ms, t.pool[2 * i], t.pool[2 * i + 1]));
        tot += ms;
        ++n;
    }
    *ms_total = tot;
    *launches = n;
    return PTYCHO_OK;
}

// ----------------------------------------------------------------- passes --
static int launch_shifts(ptycho_plan_s *p, const float *obj, const float *probe, const float2 *psi, int lw,
                         bool by_slot, const int *order, int s0, int nf, bool ml, double *out);
static int move_positions(ptycho_plan_s *p);

static int zero_async(void *ptr, size_t bytes, hipStream_t s) {
    // plain fill kernel (no memset nodes, so the work can be graph-captured)
    if (bytes % 16) return fail(PTYCHO_E_INVALID, "internal: zero size");
    const long n16 = (long)(bytes / 16);
    hipLaunchKernelGGL(k_zero, dim3(grid_for(n16)), dim3(256), 0, s, (float4 *)ptr, n16);
    LAUNCHCHK();
    return PTYCHO_OK;
}

StackArgs ptycho::stack_args(ptycho_plan_s *p, int s0, int sn, const float *obj, const float *probe) {
    StackArgs a{};
    a.Ny = p->d.obj_ny;
    a.Nx = p->d.obj_nx;
    a.K = p->d.n_modes;
    a.S = sn;
    a.s0 = s0;
    a.offs = p->offs;
    a.order = p->order;
    a.obj = (const float2 *)obj;
    a.probe = (const float2 *)probe;
    a.scr = p->scr;
    a.fwd = p->scr;
    a.colin = p->scr;
    a.qbuf = p->q;
    a.iobs = p->iobs;
    a.bg = p->bg;
    a.mask = p->mask;
    a.prop = p->prop;
    a.frac = p->pos_ready ? p->frac : nullptr;
    a.eps = p->d.icalc_floor;
    return a;
}

// log2 of the tile width of exit waves at psi: the stack scratch is stored in
// column tiles, caller-stored exit waves are row-major.
static int psi_tile_log2(const ptycho_plan_s *p, const float2 *psi) {
    const int n = p->d.n;
    if (psi != p->scr) return ilog2(n);
    return ilog2(scr_tile_w(n));
}

// Object sums of one stack, added to the running sums, from the stack's
// per-frame numerator terms q (written by the inverse row pass) and the
// probe intensity image.
int ptycho::object_sums(ptycho_plan_s *p, int sidx) {
    const ptycho_plan_s::GatherList &gl = p->stack_lists[sidx];
    if (gl.nb <= 0) return PTYCHO_OK;
    ObjTileArgs a{};
    a.N = p->d.n;
    a.Ny = p->d.obj_ny;
    a.Nx = p->d.obj_nx;
    a.ntx = p->ntx;
    a.tiles = p->lists + gl.blk_tile;
    a.tptr = p->lists + gl.blk_ptr;
    a.pslot = p->lists + gl.blk_slot;
    a.tent = p->ent_fr;
    a.pint = p->pint;
    a.q = p->q;
    a.numO = p->numO;
    a.denO = p->denO;
    a.pnum = p->opnum;
    a.pden = p->opden;
    a.offs = p->offs;
    a.frac = p->pos_ready ? p->frac : nullptr;
    Timed tm(p, TC_GATHER_OBJ);
    hipLaunchKernelGGL(k_gather_obj, dim3(gl.nb), dim3(256), 0, p->stream, a);
    if (gl.nr > 0) {
        const int *L0 = p->lists;
        hipLaunchKernelGGL(k_obj_chunk_reduce, dim3(gl.nr), dim3(256), 0, p->stream, L0 + gl.red_tile,
                           L0 + gl.red_first, L0 + gl.red_count, p->opnum, p->opden, p->numO, p->denO, p->ntx,
                           p->d.obj_ny, p->d.obj_nx);
    }
    LAUNCHCHK();
    return PTYCHO_OK;
}

// Probe sums over frames order[q0 .. q0+nq) with the given object, from the
// stack scratch (slots) or stored exit waves (frames); deterministic chunked
// reduction, written or added to the running sums.
int ptycho::probe_sums(ptycho_plan_s *p, const float *obj, const float2 *psi, int q0, int nq, bool from_scr,
                      bool accumulate) {
    ProbeAllArgs a{};
    a.N = p->d.n;
    a.K = p->d.n_modes;
    a.q0 = q0;
    a.nq = nq;
    a.Nx = p->d.obj_nx;
    a.Ny = p->d.obj_ny;
    a.frac = p->pos_ready ? p->frac : nullptr;
    a.lw = psi_tile_log2(p, psi);
    a.offs = p->offs;
    a.order = p->order;
    a.obj = (const float2 *)obj;
    a.psi = psi;
    a.part_num = p->pnum;
    a.part_den = p->pden;
    const long n2 = (long)a.N * a.N;
    const int chunks = std::max(1, std::min(p->L.pchunks, nq));
    dim3 grid((unsigned)((n2 + 255) / 256), 1, chunks);
    Timed tm(p, from_scr ? TC_GATHER_PROBE : TC_PROBE_ALL);
    with_k(a.K, [&](auto kk) {
        constexpr int K = decltype(kk)::value;
        if (from_scr) hipLaunchKernelGGL((k_gather_probe<K, true>), grid, dim3(256), 0, p->stream, a);
        else hipLaunchKernelGGL((k_gather_probe<K, false>), grid, dim3(256), 0, p->stream, a);
        return (int)PTYCHO_OK;
    });
    hipLaunchKernelGGL(k_probe_reduce, dim3(grid_for(n2 * a.K)), dim3(256), 0, p->stream, p->pnum, p->pden, chunks,
                       a.K, n2, p->numP, p->denP, accumulate ? 1 : 0);
    LAUNCHCHK();
    return PTYCHO_OK;
}

static int zero_sums(ptycho_plan_s *p, unsigned acc) {
    const size_t no = (size_t)p->d.obj_ny * p->d.obj_nx, n2 = (size_t)p->d.n * p->d.n;
    int st = PTYCHO_OK;
    if (acc & ACC_OBJ) {
        st = zero_async(p->numO, up(sizeof(float2) * no), p->stream);
        if (!st) st = zero_async(p->denO, up(sizeof(float) * no), p->stream);
    }
    if (!st && (acc & ACC_PROBE)) {
        st = zero_async(p->numP, up(sizeof(float2) * p->d.n_modes * n2), p->stream);
        if (!st) st = zero_async(p->denP, up(sizeof(float) * n2), p->stream);
    }
    return st;
}

// Probe intensity image sum_k |P_k|^2 (the object denominator's term).
int ptycho::launch_probe_intensity(ptycho_plan_s *p, const float *probe) {
    const long n2 = (long)p->d.n * p->d.n;
    hipLaunchKernelGGL(k_probe_intensity, dim3(grid_for(n2)), dim3(256), 0, p->stream, (const float2 *)probe,
                       p->d.n_modes, n2, p->pint);
    LAUNCHCHK();
    return PTYCHO_OK;
}

// AP background refinement: the s^2 sums of one stack of sn frames.
int ptycho::launch_bg_accum(ptycho_plan_s *p, int sn, int first) {
    const long n2 = (long)p->d.n * p->d.n;
    hipLaunchKernelGGL(k_bg_accum, dim3(grid_for(n2)), dim3(256), 0, p->stream, p->s2, sn, n2, p->bsum, first);
    LAUNCHCHK();
    return PTYCHO_OK;
}

static int normalize(ptycho_plan_s *p, float *obj, float *probe, unsigned upd) {
    const long no = (long)p->d.obj_ny * p->d.obj_nx, n2 = (long)p->d.n * p->d.n;
    Timed tm(p, TC_NORMALIZE);
    hipLaunchKernelGGL(k_max_partial, dim3(NPART), dim3(256), 0, p->stream, p->denO, (upd & 1u) ? no : 0L,
                       p->denP, (upd & 2u) ? n2 : 0L, p->part);
    const long work = std::max((upd & 1u) ? no : 0L, (upd & 2u) ? n2 * p->d.n_modes : 0L);
    hipLaunchKernelGGL(k_normalize, dim3(grid_for(work)), dim3(256), 0, p->stream,
                       (float2 *)obj, p->numO, p->denO, no, (float2 *)probe, p->numP, p->denP, (int)n2,
                       p->d.n_modes, p->part, NPART, p->d.obj_inertia, p->d.probe_inertia, upd);
    LAUNCHCHK();
    return PTYCHO_OK;
}

static int check_plan_ptrs(ptycho_plan_t p, const void *a, const void *b) {
    if (!p) return fail(PTYCHO_E_INVALID, "null plan");
    if (!a || !b) return fail(PTYCHO_E_INVALID, "null object or probe");
    return PTYCHO_OK;
}

// The same for the entry points that propagate to the detector.
static int check_prop_ptrs(ptycho_plan_t p, const void *a, const void *b) {
    const int st = check_plan_ptrs(p, a, b);
    return st ? st : check_geometry(p);
}

// The position-shift kernel reads two pixels' exit waves and probe values in
// one 16-byte load.
static int check_shift_align(const void *probe, const void *psi) {
    if (((uintptr_t)probe | (uintptr_t)psi) % 16)
        return fail(PTYCHO_E_INVALID, "position shifts need 16-byte aligned probe and exit waves");
    return PTYCHO_OK;
}

// AP (kind 0) or DM (kind 1) cycles: projection with the per-stack object
// sums, object normalisation, then the probe sums over all frames with the
// new object and the probe normalisation.
static int run_cycles(ptycho_plan_t p, float *obj, float *probe, float *psi, int n_cycles, uint32_t upd, int kind) {
    int st = check_prop_ptrs(p, obj, probe);
    if (st) return st;
    if (n_cycles < 0) return fail(PTYCHO_E_INVALID, "negative cycle count");
    if (upd & ~(kind == 0 ? 15u : 3u)) return fail(PTYCHO_E_INVALID, "unknown update flag");
    const bool upd_pos = (upd & PTYCHO_UPDATE_POSITIONS) != 0;
    if (upd_pos && !p->pos_ready)
        return fail(PTYCHO_E_INVALID, "a position update needs a plan with positions (ptycho_plan_set_positions)");
    if (upd_pos && !psi) return fail(PTYCHO_E_INVALID, "a position update needs exit-wave storage (psi)");
    if (upd_pos && (st = check_shift_align(probe, psi))) return st;
    const bool upd_bg = (upd & PTYCHO_UPDATE_BACKGROUND) != 0;
    if (upd_bg && !p->bg) return fail(PTYCHO_E_INVALID, "a background update needs a background (set_background)");
    if (upd_bg && !p->s2)
        return fail(PTYCHO_E_INVALID, "a background update needs a plan created with PTYCHO_FLAG_BACKGROUND");
    if (kind == 1 && !psi) return fail(PTYCHO_E_INVALID, "null psi");
    if (kind == 0 && (upd & 2u) && !psi)
        return fail(PTYCHO_E_INVALID, "an AP probe update needs exit-wave storage (psi)");
    const NPass *np = passes_for(p->d.n);
    if (!np) return PTYCHO_E_UNSUPPORTED;
    const long n2 = (long)p->d.n * p->d.n;
    for (int c = 0; c < n_cycles; ++c) {
        int s2 = PTYCHO_OK;
        if (upd & 1u) s2 = zero_sums(p, ACC_OBJ);
        if (!s2) s2 = np->project(p, obj, probe, psi, kind, (upd & 1u) ? ACC_OBJ : 0u, upd_bg, nullptr);
        if (!s2 && upd_bg) {
            // every stack was projected with the old background
            Timed tm(p, TC_OTHER);
            hipLaunchKernelGGL(k_bg_finish, dim3(grid_for(n2)), dim3(256), 0, p->stream, p->bg, p->bsum, n2,
                               (double)p->d.n_frames);
            s2 = hipGetLastError() == hipSuccess ? PTYCHO_OK : fail(PTYCHO_E_HIP, "background update launch");
        }
        if (!s2 && (upd & 1u)) s2 = normalize(p, obj, probe, 1u);
        if (!s2 && (upd & 2u)) s2 = probe_sums(p, obj, (const float2 *)psi, 0, p->d.n_frames, false, false);
        if (!s2 && (upd & 2u)) s2 = normalize(p, obj, probe, 2u);
        // positions: shifts of the projected exit waves against the new
        // object and probe, then the move
        if (!s2 && upd_pos)
            s2 = launch_shifts(p, obj, probe, (const float2 *)psi, ilog2(p->d.n), false, nullptr, 0, p->d.n_frames,
                               false, p->shifts);
        if (!s2 && upd_pos) s2 = move_positions(p);
        if (s2) return s2;
    }
    return PTYCHO_OK;
}

extern "C" int ptycho_ap_cycle(ptycho_plan_t p, float *obj, float *probe, float *psi, int32_t n_cycles,
                               uint32_t upd) {
    return run_cycles(p, obj, probe, psi, n_cycles, upd, 0);
}

extern "C" int ptycho_dm_cycle(ptycho_plan_t p, float *obj, float *probe, float *psi, int32_t n_cycles,
                               uint32_t upd) {
    return run_cycles(p, obj, probe, psi, n_cycles, upd, 1);
}

extern "C" int ptycho_psi_init(ptycho_plan_t p, const float *obj, const float *probe, float *psi) {
    int st = check_plan_ptrs(p, obj, probe);
    if (st) return st;
    if (!psi) return fail(PTYCHO_E_INVALID, "null psi");
    const long total = (long)p->d.n_frames * p->d.n_modes * p->d.n * p->d.n;
    hipLaunchKernelGGL(k_psi_init, dim3(grid_for(total)), dim3(256), 0, p->stream, (const float2 *)obj,
                       (const float2 *)probe, p->offs, p->pos_ready ? p->frac : nullptr, (float2 *)psi, p->d.n,
                       p->d.n_modes, p->d.obj_ny, p->d.obj_nx, total);
    LAUNCHCHK();
    return PTYCHO_OK;
}

// A read-only forward pass of column op `op` through the frame-size table.
static int forward_pass(ptycho_plan_s *p, int op, const float *obj, const float *probe, const float *dobj,
                        const float *dprobe, float *icalc, int llk_model = LLK_POISSON,
                        const float2 *keep = nullptr) {
    const NPass *np = passes_for(p->d.n);
    if (!np) return PTYCHO_E_UNSUPPORTED;
    return np->forward(p, op, obj, probe, dobj, dprobe, icalc, llk_model, keep);
}

static int zero_red(ptycho_plan_s *p) { return zero_async(p->red, up(sizeof(double) * p->L.nred), p->stream); }

// llk_dev[0] = sum of the reduction partials, llk_dev[1] = number of good pixels
__global__ void k_copy_scalar(double *dst, const double *src) { dst[0] = src[0]; }

static int llk_into(ptycho_plan_t p, const float *obj, const float *probe, double *llk, int model) {
    int st = zero_red(p);
    if (st) return st;
    st = forward_pass(p, OP_LLK, obj, probe, nullptr, nullptr, nullptr, model);
    if (st) return st;
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(SUM_THREADS), 0, p->stream, p->red, (long)p->L.nred, 1, llk, 0);
    hipLaunchKernelGGL(k_copy_scalar, dim3(1), dim3(1), 0, p->stream, llk + 1, p->scal + SC_NOBS);
    LAUNCHCHK();
    return PTYCHO_OK;
}

extern "C" int ptycho_llk(ptycho_plan_t p, const float *obj, const float *probe, double *llk) {
    int st = check_prop_ptrs(p, obj, probe);
    if (st) return st;
    if (!llk) return fail(PTYCHO_E_INVALID, "null llk output");
    return llk_into(p, obj, probe, llk, LLK_POISSON);
}

extern "C" int ptycho_llk_model(ptycho_plan_t p, const float *obj, const float *probe, int32_t model,
                                double *llk) {
    int st = check_prop_ptrs(p, obj, probe);
    if (st) return st;
    if (!llk) return fail(PTYCHO_E_INVALID, "null llk output");
    if (model != LLK_POISSON && model != LLK_GAUSSIAN && model != LLK_EUCLIDEAN)
        return fail(PTYCHO_E_INVALID, "unknown noise model");
    return llk_into(p, obj, probe, llk, model);
}

// Position-shift sums of nf frames (launch frame f -> frame order[s0 + f], or
// f when order is null) from exit waves psi (AP: projected, chi = psi - P O;
// ML: a gradient wave, chi = -1/2 psi), then the shifts of those frames into
// out [J][3].
static int launch_shifts(ptycho_plan_s *p, const float *obj, const float *probe, const float2 *psi, int lw,
                         bool by_slot, const int *order, int s0, int nf, bool ml, double *out) {
    PosShiftArgs a{};
    a.N = p->d.n;
    a.K = p->d.n_modes;
    a.Ny = p->d.obj_ny;
    a.Nx = p->d.obj_nx;
    a.R = pos_rows(a.N);
    a.CH = p->L.pos_chunks;
    a.lgN = ilog2(a.N);
    a.offs = p->offs;
    a.frac = p->pos_ready ? p->frac : nullptr;
    a.order = order;
    a.s0 = s0;
    a.nf = nf;
    a.obj = (const float2 *)obj;
    a.probe = (const float2 *)probe;
    a.psi = psi;
    a.lw = lw;
    a.by_slot = by_slot;
    a.ml = ml;
    a.chi_scale = -0.5f;
    a.part = p->pspart;
    Timed tm(p, TC_OTHER);
    constexpr int F = SHIFT_FRAMES;
    const dim3 grid((unsigned)a.CH * (unsigned)((nf + F - 1) / F));
    const bool sub = a.frac != nullptr;
    switch (a.K * 2 + (sub ? 1 : 0)) {
        case 2: hipLaunchKernelGGL((k_pos_shift_part<1, false, F>), grid, dim3(256), 0, p->stream, a); break;
        case 3: hipLaunchKernelGGL((k_pos_shift_part<1, true, F>), grid, dim3(256), 0, p->stream, a); break;
        case 4: hipLaunchKernelGGL((k_pos_shift_part<2, false, F>), grid, dim3(256), 0, p->stream, a); break;
        case 5: hipLaunchKernelGGL((k_pos_shift_part<2, true, F>), grid, dim3(256), 0, p->stream, a); break;
        case 6: hipLaunchKernelGGL((k_pos_shift_part<3, false, F>), grid, dim3(256), 0, p->stream, a); break;
        case 7: hipLaunchKernelGGL((k_pos_shift_part<3, true, F>), grid, dim3(256), 0, p->stream, a); break;
        case 8: hipLaunchKernelGGL((k_pos_shift_part<4, false, F>), grid, dim3(256), 0, p->stream, a); break;
        case 9: hipLaunchKernelGGL((k_pos_shift_part<4, true, F>), grid, dim3(256), 0, p->stream, a); break;
        default: return fail(PTYCHO_E_INVALID, "internal: modes outside 1..4");
    }
    hipLaunchKernelGGL(k_pos_shift_finish, dim3((nf + 255) / 256), dim3(256), 0, p->stream, p->pspart, a.CH, order,
                       s0, nf, out);
    LAUNCHCHK();
    return PTYCHO_OK;
}

int ptycho::launch_ml_shifts(ptycho_plan_s *p, const float *obj, const float *probe, int s0, int sn) {
    return launch_shifts(p, obj, probe, p->scr, ilog2(scr_tile_w(p->d.n)), true, p->order, s0, sn, true, p->shifts);
}

extern "C" int ptycho_position_shifts(ptycho_plan_t p, const float *obj, const float *probe, const float *psi,
                                      double *out) {
    int st = check_plan_ptrs(p, obj, probe);
    if (st) return st;
    if (!psi || !out) return fail(PTYCHO_E_INVALID, "null psi or output");
    if ((st = check_shift_align(probe, psi))) return st;
    return launch_shifts(p, obj, probe, (const float2 *)psi, ilog2(p->d.n), false, nullptr, 0, p->d.n_frames, false,
                         out);
}

// The plan's positions move by its last shifts (filter, step, bound), then
// its window tables follow.
static int move_positions(ptycho_plan_s *p) {
    Timed tm(p, TC_OTHER);
    hipLaunchKernelGGL(k_update_positions, dim3(1), dim3(POSUPD_THREADS), 0, p->stream, p->d.n_frames, p->pos,
                       p->pos0, p->shifts, p->pos_mult, (double)p->d.max_shift, p->pos_min_grad, p->pos);
    hipLaunchKernelGGL(k_windows, dim3(grid_for(p->d.n_frames)), dim3(256), 0, p->stream, p->pos, p->d.n_frames,
                       p->d.n, p->d.obj_ny, p->d.obj_nx, p->offs, p->frac);
    LAUNCHCHK();
    return PTYCHO_OK;
}

extern "C" int ptycho_plan_set_positions(ptycho_plan_t p, const double *pos, double mult, double min_grad) {
    if (!p || !pos) return fail(PTYCHO_E_INVALID, "null pointer");
    if (!p->pos) return fail(PTYCHO_E_INVALID, "positions need a plan created with PTYCHO_FLAG_POSITIONS");
    if (!std::isfinite(mult) || !std::isfinite(min_grad) || !(min_grad >= 0.0))
        return fail(PTYCHO_E_INVALID, "mult and min_grad must be finite, min_grad >= 0");
    const ptycho_desc_t &d = p->d;
    const int J = d.n_frames, N = d.n;
    const double c[2] = {d.obj_ny / 2.0, d.obj_nx / 2.0};
    const int lim[2] = {d.obj_ny - N, d.obj_nx - N};
    const double ms = d.max_shift;
    std::vector<double> t((size_t)J * 2);
    std::vector<float2> fr(J);
    for (int j = 0; j < J; ++j) {
        float f2[2];
        for (int ax = 0; ax < 2; ++ax) {
            const double tv = c[ax] + pos[2 * j + ax] - N / 2.0;
            if (!std::isfinite(tv)) return fail(PTYCHO_E_INVALID, "non-finite position");
            const int oref = ax == 0 ? p->h_offs[j].x : p->h_offs[j].y;
            if (std::floor(tv) != (double)oref)
                return fail(PTYCHO_E_INVALID, "positions do not match the plan's window corners (frame " +
                                                  std::to_string(j) + ")");
            if (tv - ms < 0.0 || tv + ms > (double)lim[ax])
                return fail(PTYCHO_E_BOUNDS, "a window moved by max_shift would leave the object (frame " +
                                                 std::to_string(j) + ")");
            t[2 * j + ax] = tv;
            f2[ax] = (float)(tv - std::floor(tv));
        }
        fr[j] = make_float2(f2[0], f2[1]);
    }
    p->h_pos.swap(t);
    p->h_frac.swap(fr);
    hipError_t e = upload_tables({{p->pos, p->h_pos.data(), sizeof(double) * p->h_pos.size()},
                                  {p->pos0, p->h_pos.data(), sizeof(double) * p->h_pos.size()},
                                  {p->frac, p->h_frac.data(), sizeof(float2) * p->h_frac.size()}},
                                 p->stream);
    if (e != hipSuccess) return fail(PTYCHO_E_HIP, std::string("position upload: ") + hipGetErrorString(e));
    p->pos_mult = mult;
    p->pos_min_grad = min_grad;
    p->pos_ready = true;
    return PTYCHO_OK;
}

extern "C" int ptycho_plan_positions(ptycho_plan_t p, double *out) {
    if (!p || !out) return fail(PTYCHO_E_INVALID, "null pointer");
    if (!p->pos_ready) return fail(PTYCHO_E_INVALID, "the plan has no positions (ptycho_plan_set_positions)");
    const ptycho_desc_t &d = p->d;
    hipLaunchKernelGGL(k_corners_to_positions, dim3(grid_for(d.n_frames)), dim3(256), 0, p->stream, p->pos,
                       d.n_frames, d.obj_ny / 2.0 - d.n / 2.0, d.obj_nx / 2.0 - d.n / 2.0, out);
    LAUNCHCHK();
    return PTYCHO_OK;
}

extern "C" int ptycho_refine_positions(ptycho_plan_t p, const float *obj, const float *probe, const float *psi,
                                       double *shifts) {
    int st = check_plan_ptrs(p, obj, probe);
    if (st) return st;
    if (!psi) return fail(PTYCHO_E_INVALID, "null psi");
    if (!p->pos_ready) return fail(PTYCHO_E_INVALID, "the plan has no positions (ptycho_plan_set_positions)");
    if ((st = check_shift_align(probe, psi))) return st;
    st = launch_shifts(p, obj, probe, (const float2 *)psi, ilog2(p->d.n), false, nullptr, 0, p->d.n_frames, false,
                       p->shifts);
    if (!st) st = move_positions(p);
    if (!st && shifts)
        HIPCHK(hipMemcpyAsync(shifts, p->shifts, sizeof(double) * 3 * p->d.n_frames, hipMemcpyDeviceToDevice,
                              p->stream));
    return st;
}

extern "C" int ptycho_update_positions(int32_t n_frames, const double *pos, const double *pos0, const double *shifts,
                                       double mult, double max_shift, double min_grad, double *pos_out,
                                       void *stream) {
    if (n_frames < 1) return fail(PTYCHO_E_INVALID, "n_frames must be >= 1");
    if (!pos || !pos0 || !shifts || !pos_out) return fail(PTYCHO_E_INVALID, "null pointer");
    if (!std::isfinite(mult) || !std::isfinite(max_shift) || !(max_shift >= 0.0) || !std::isfinite(min_grad) ||
        !(min_grad >= 0.0))
        return fail(PTYCHO_E_INVALID, "mult, max_shift and min_grad must be finite, the last two >= 0");
    hipLaunchKernelGGL(k_update_positions, dim3(1), dim3(POSUPD_THREADS), 0, (hipStream_t)stream, (int)n_frames, pos,
                       pos0, shifts, mult, max_shift, min_grad, pos_out);
    LAUNCHCHK();
    return PTYCHO_OK;
}

extern "C" int ptycho_check_finite(ptycho_plan_t p, const float *obj, const float *probe, int32_t *flag) {
    int st = check_plan_ptrs(p, obj, probe);
    if (st) return st;
    if (!flag) return fail(PTYCHO_E_INVALID, "null flag");
    const long no = 2L * p->d.obj_ny * p->d.obj_nx, np = 2L * p->d.n_modes * p->d.n * p->d.n;
    Timed tm(p, TC_OTHER);
    hipLaunchKernelGGL(k_clear_flag, dim3(1), dim3(1), 0, p->stream, (int *)flag);
    hipLaunchKernelGGL(k_check_finite, dim3(grid_for(no)), dim3(256), 0, p->stream, obj, no, (int *)flag);
    hipLaunchKernelGGL(k_check_finite, dim3(grid_for(np)), dim3(256), 0, p->stream, probe, np, (int *)flag);
    LAUNCHCHK();
    return PTYCHO_OK;
}

extern "C" int ptycho_icalc(ptycho_plan_t p, const float *obj, const float *probe, float *icalc) {
    int st = check_prop_ptrs(p, obj, probe);
    if (st) return st;
    if (!icalc) return fail(PTYCHO_E_INVALID, "null icalc output");
    return forward_pass(p, OP_ICALC, obj, probe, nullptr, nullptr, icalc);
}

// Gradient pass: sums in numO/numP (and denominators), LLK partials in red.
// keep (nullable) receives the forward row transforms of every frame.
static int grad_pass(ptycho_plan_s *p, const float *obj, const float *probe, float2 *keep = nullptr) {
    int st = zero_sums(p, ACC_OBJ | ACC_PROBE);
    if (!st) st = zero_red(p);
    if (st) return st;
    const NPass *np = passes_for(p->d.n);
    if (!np) return PTYCHO_E_UNSUPPORTED;
    return np->project(p, obj, probe, nullptr, 2, ACC_OBJ | ACC_PROBE, false, keep);
}

extern "C" int ptycho_ml_grad(ptycho_plan_t p, const float *obj, const float *probe, float *g_obj, float *g_probe,
                              double *llk) {
    int st = check_prop_ptrs(p, obj, probe);
    if (st) return st;
    if (!g_obj || !g_probe) return fail(PTYCHO_E_INVALID, "null gradient output");
    st = grad_pass(p, obj, probe);
    if (st) return st;
    const long no = (long)p->d.obj_ny * p->d.obj_nx, np = (long)p->d.n_modes * p->d.n * p->d.n;
    hipLaunchKernelGGL(k_scale_copy, dim3(grid_for(no)), dim3(256), 0, p->stream, (float2 *)g_obj, p->numO, no, 2.0f);
    hipLaunchKernelGGL(k_scale_copy, dim3(grid_for(np)), dim3(256), 0, p->stream, (float2 *)g_probe, p->numP, np, 2.0f);
    if (llk) {
        hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(SUM_THREADS), 0, p->stream, p->red, (long)p->L.nred, 1, llk, 0);
        hipLaunchKernelGGL(k_copy_scalar, dim3(1), dim3(1), 0, p->stream, llk + 1, p->scal + SC_NOBS);
    }
    LAUNCHCHK();
    return PTYCHO_OK;
}

// Line-search coefficients; with keep (the gradient pass's row transforms at
// the same point) the pass forms and row-transforms only B and C.
static int ls_pass(ptycho_plan_s *p, const float *obj, const float *probe, const float *dobj, const float *dprobe,
                   double *coef, const float2 *keep = nullptr) {
    int st = zero_red(p);
    if (st) return st;
    st = keep ? forward_pass(p, OP_LS2, obj, probe, dobj, dprobe, nullptr, LLK_POISSON, keep)
              : forward_pass(p, OP_LS, obj, probe, dobj, dprobe, nullptr);
    if (st) return st;
    const long n = (long)p->L.nred / 2;
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(SUM_THREADS), 0, p->stream, p->red, n, 2, coef, 0);
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(SUM_THREADS), 0, p->stream, p->red + 1, n, 2, coef + 1, 0);
    LAUNCHCHK();
    return PTYCHO_OK;
}

extern "C" int ptycho_ml_linesearch(ptycho_plan_t p, const float *obj, const float *probe, const float *dobj,
                                    const float *dprobe, double *coef) {
    int st = check_prop_ptrs(p, obj, probe);
    if (st) return st;
    if (!dobj || !dprobe || !coef) return fail(PTYCHO_E_INVALID, "null direction or output");
    return ls_pass(p, obj, probe, dobj, dprobe, coef);
}

// ------------------------------------------------------------ CG ML cycle --
// State of the CG iteration: scalars, direction and previous gradient of the
// object and probe, inner-product partials, and the forward row transforms
// of every frame at the current point (kept by the gradient pass for the
// line search, which then forms only its two other transforms).
static size_t ml_state_bytes(const ptycho_desc_t &d) {
    const size_t no = (size_t)d.obj_ny * d.obj_nx, np = (size_t)d.n_modes * d.n * d.n;
    return up(sizeof(double) * CG_NSCAL) + 2 * up(sizeof(float2) * no) + 2 * up(sizeof(float2) * np) +
           up(sizeof(double) * 4 * CG_NPART) + up(sizeof(float2) * np * d.n_frames);
}

extern "C" int ptycho_ml_state_bytes(ptycho_plan_t p, size_t *bytes) {
    if (!p || !bytes) return fail(PTYCHO_E_INVALID, "null pointer");
    *bytes = ml_state_bytes(p->d);
    return PTYCHO_OK;
}

extern "C" int ptycho_ml_cycle(ptycho_plan_t p, float *obj, float *probe, void *state, int32_t n_cycles,
                               uint32_t upd, int32_t reset, double *hist) {
    int st = check_prop_ptrs(p, obj, probe);
    if (st) return st;
    if (!state) return fail(PTYCHO_E_INVALID, "null state");
    if (((uintptr_t)state) % ALIGN) return fail(PTYCHO_E_WORKSPACE, "state not 256-byte aligned");
    if (n_cycles < 0) return fail(PTYCHO_E_INVALID, "negative cycle count");
    if (upd & ~11u) return fail(PTYCHO_E_INVALID, "unknown update flag");
    const bool upd_pos = (upd & PTYCHO_UPDATE_POSITIONS) != 0;
    if (upd_pos && !p->pos_ready)
        return fail(PTYCHO_E_INVALID, "a position update needs a plan with positions (ptycho_plan_set_positions)");
    if (upd_pos && (st = check_shift_align(probe, nullptr))) return st;
    upd &= 3u;
    const size_t no = (size_t)p->d.obj_ny * p->d.obj_nx, np = (size_t)p->d.n_modes * p->d.n * p->d.n;
    char *b = (char *)state;
    double *scal = (double *)b;
    b += up(sizeof(double) * CG_NSCAL);
    float2 *d_o = (float2 *)b;
    b += up(sizeof(float2) * no);
    float2 *g_o = (float2 *)b;
    b += up(sizeof(float2) * no);
    float2 *d_p = (float2 *)b;
    b += up(sizeof(float2) * np);
    float2 *g_p = (float2 *)b;
    b += up(sizeof(float2) * np);
    double *cpart = (double *)b;
    b += up(sizeof(double) * 4 * CG_NPART);
    float2 *keep = (float2 *)b;
    hipStream_t s = p->stream;
    if (reset) {
        hipLaunchKernelGGL(k_cg_reset, dim3(1), dim3(64), 0, s, scal);
        LAUNCHCHK();
    }
    const long n2 = (long)p->d.n * p->d.n;
    for (int c = 0; c < n_cycles; ++c) {
        // 1. gradient (sums in numO/numP), LLK, denominators
        p->shifts_in_grad = upd_pos;
        st = grad_pass(p, obj, probe, keep);
        p->shifts_in_grad = false;
        if (st) return st;
        {
        Timed tm(p, TC_OTHER);
        hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(SUM_THREADS), 0, s, p->red, (long)p->L.nred, 1,
                           scal + CG_LLK, 0);
        hipLaunchKernelGGL(k_max_partial, dim3(NPART), dim3(256), 0, s, p->denO, (long)no, p->denP, n2, p->part);
        // 2. inner products for beta, then the new direction
        hipLaunchKernelGGL(k_cg_dots, dim3(CG_NPART), dim3(256), 0, s, p->numO, g_o, (long)no, p->numP, g_p,
                           (long)np, upd, cpart);
        hipLaunchKernelGGL(k_cg_beta, dim3(1), dim3(256), 0, s, cpart, p->part, NPART, scal, hist ? hist + c : nullptr);
        hipLaunchKernelGGL(k_cg_direction, dim3(grid_for((long)std::max(no, np))), dim3(256), 0, s, p->numO, g_o, d_o,
                           (long)no, p->numP, g_p, d_p, (long)np, upd, scal);
        }
        // 3. line search along d, then the step
        st = ls_pass(p, obj, probe, (const float *)d_o, (const float *)d_p, scal + CG_L1, keep);
        if (st) return st;
        hipLaunchKernelGGL(k_cg_step, dim3(grid_for((long)std::max(no, np))), dim3(256), 0, s, (float2 *)obj, d_o,
                           (long)no, (float2 *)probe, d_p, (long)np, upd, scal);
        LAUNCHCHK();
        // positions: the shifts the gradient pass took at the cycle's start
        if (upd_pos) {
            st = move_positions(p);
            if (st) return st;
        }
    }
    return PTYCHO_OK;
}

// ------------------------------------------------- allocation-free LLK ---
// Scratch of ptycho_llk_noalloc: one static device array per GPU (held until
// the process ends), reached from host code through the address that
// hipGetSymbolAddress returns on that device, never through its name.
namespace {
__device__ __align__(256) unsigned char scratch[PTYCHO_NOALLOC_SCRATCH_BYTES];
std::mutex g_scratch_mu;
std::vector<void *> g_scratch_ptr;   // per device, null until looked up
}  // namespace

static int scratch_for_current_device(char **out) {
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if ((int)g_scratch_ptr.size() <= dev) g_scratch_ptr.resize(dev + 1, nullptr);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        HIPCHK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr) return fail(PTYCHO_E_HIP, "no device address for the static scratch");
        g_scratch_ptr[dev] = ptr;
    }
    *out = (char *)g_scratch_ptr[dev];
    return PTYCHO_OK;
}

// Layout of the static scratch for one call: flag and count, the frame
// tables, the reduction partials, then as many frames of stack scratch as
// fit.  S = 0 when not even one frame fits.
struct NoAllocLayout {
    int S, nstacks, maxb;
    size_t nred, off_flag, off_count, off_offs, off_order, off_red, off_scr, total;
};
static NoAllocLayout noalloc_layout(const ptycho_desc_t &d) {
    NoAllocLayout L{};
    const size_t J = (size_t)d.n_frames, N = (size_t)d.n, K = (size_t)d.n_modes;
    const size_t frame = sizeof(float2) * K * N * N;
    const int cb = col_cb(d.n);
    size_t o = 0;
    L.off_flag = o; o = up(o + sizeof(int));
    L.off_count = o; o = up(o + sizeof(double));
    L.off_offs = o; o = up(o + sizeof(int2) * J);
    L.off_order = o; o = up(o + sizeof(int) * J);
    // partials: one per column block of every stack; bounded by the
    // all-frames count, sized after S is known
    const size_t fixed = o;
    const size_t per_frame = frame + sizeof(double) * (N + cb - 1) / cb + sizeof(double);
    int S = 0;
    if (PTYCHO_NOALLOC_SCRATCH_BYTES > fixed + 2 * ALIGN)
        S = (int)std::min<size_t>(J, (PTYCHO_NOALLOC_SCRATCH_BYTES - fixed - 2 * ALIGN) / per_frame);
    L.S = S;
    if (S < 1) { L.total = SIZE_MAX; return L; }
    L.nstacks = (int)((J + S - 1) / S);
    L.maxb = (int)(((long)S * d.n + cb - 1) / cb);
    L.nred = (size_t)L.nstacks * L.maxb;
    L.off_red = o; o = up(o + sizeof(double) * L.nred);
    L.off_scr = o; o = up(o + frame * (size_t)S);
    L.total = o;
    return L;
}

extern "C" int ptycho_llk_noalloc(const ptycho_desc_t *d, const int32_t *offsets, const float *iobs,
                                  const uint8_t *mask, const float *obj, const float *probe, double *llk,
                                  void *stream) {
    int st = check_desc(d);
    if (st) return st;
    if (!offsets || !iobs || !obj || !probe || !llk) return fail(PTYCHO_E_INVALID, "null pointer");
    if (d->flags != 0) return fail(PTYCHO_E_INVALID, "the allocation-free LLK takes a far-field descriptor without flags");
    const NoAllocLayout L = noalloc_layout(*d);
    if (L.S < 1 || L.total > PTYCHO_NOALLOC_SCRATCH_BYTES)
        return fail(PTYCHO_E_WORKSPACE, "problem exceeds the allocation-free scratch (" +
                                             std::to_string(PTYCHO_NOALLOC_SCRATCH_BYTES >> 20) + " MiB)");
    const NPass *np = passes_for(d->n);
    if (!np) return PTYCHO_E_UNSUPPORTED;
    st = ensure_twiddles();
    if (st) return st;
    char *base = nullptr;
    st = scratch_for_current_device(&base);
    if (st) return st;
    hipStream_t s = (hipStream_t)stream;
    // a plan on the stack whose tables and scratch are carved from the
    // static array; the forward pass is the plan path's own
    ptycho_plan_s p{};
    p.d = *d;
    p.L.S = L.S;
    p.L.nstacks = L.nstacks;
    p.L.maxb = L.maxb;
    p.L.nred = L.nred;
    p.stream = s;
    p.iobs = iobs;
    p.mask = mask;
    p.offs = (int2 *)(base + L.off_offs);
    p.order = (int *)(base + L.off_order);
    p.scr = (float2 *)(base + L.off_scr);
    p.red = (double *)(base + L.off_red);
    int *flag = (int *)(base + L.off_flag);
    double *count = (double *)(base + L.off_count);
    const int J = d->n_frames;
    // every word the call reads is written first: the flag and partials are
    // cleared by fill kernels, the tables and count are written whole
    st = zero_async(flag, ALIGN, s);
    if (!st) st = zero_async(p.red, up(sizeof(double) * L.nred), s);
    if (st) return st;
    hipLaunchKernelGGL(k_frame_tables, dim3(grid_for(J)), dim3(256), 0, s, (const int *)offsets, J, d->n, d->obj_ny,
                       d->obj_nx, p.offs, p.order, flag);
    hipLaunchKernelGGL(k_count_good, dim3(1), dim3(256), 0, s, mask, d->n * d->n, (double)J, count);
    LAUNCHCHK();
    st = np->forward(&p, OP_LLK, obj, probe, nullptr, nullptr, nullptr, LLK_POISSON, nullptr);
    if (st) return st;
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(SUM_THREADS), 0, s, p.red, (long)L.nred, 1, llk, 0);
    hipLaunchKernelGGL(k_copy_scalar, dim3(1), dim3(1), 0, s, llk + 1, count);
    hipLaunchKernelGGL(k_nan_if_flagged, dim3(1), dim3(1), 0, s, llk, flag);
    LAUNCHCHK();
    return PTYCHO_OK;
}

// ------------------------------------------------------------ plain FFT ---
extern "C" int ptycho_fft2(int32_t n, int32_t count, float *data, int32_t dir, void *stream) {
    if (!supported_n(n)) return fail(PTYCHO_E_UNSUPPORTED, "unsupported frame size");
    if (count < 0 || (dir != -1 && dir != 1)) return fail(PTYCHO_E_INVALID, "bad count or direction");
    if (count == 0) return PTYCHO_OK;
    if (!data) return fail(PTYCHO_E_INVALID, "null data");
    int st = ensure_twiddles();
    if (st) return st;
    const NPass *np = passes_for(n);
    if (!np) return PTYCHO_E_UNSUPPORTED;
    return np->fft2(count, data, dir, (hipStream_t)stream);
}
