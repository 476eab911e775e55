// abi.cpp -- the extern "C" entry points of libsmi (declared in include/smi.h).
//
// Each entry point validates on the host (synchronous error codes), builds a plan, uploads
// the plan's small tables into the caller's workspace and enqueues the time loop on the
// caller's stream.  No device memory is allocated here.
#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "smi_internal.hpp"

using smi::Plan;
using smi::Views;

// ---------------------------------------------------------------- static workspace
// The workspace of smi_forward_static: a file-scope device array of SMI_STATIC_WS_BYTES.  Each
// GPU the library runs on holds its own copy until the process ends.  Host code never hands
// the array's name to a kernel or a copy (on the host it is only a stand-in symbol): the
// array's address on a device comes from hipGetSymbolAddress, taken once per device, with that
// device current, when the first context on it is created.
static __device__ __align__(256) unsigned char scratch[SMI_STATIC_WS_BYTES];

namespace {
constexpr int kMaxDevices = 64;

// A roctx range over one host phase of a call (plan and upload, autotuning, time loop, reverse
// loop), for timelines taken with a marker trace; without a profiler the push and pop return
// at once.
struct Range {
    explicit Range(const char *name) { roctxRangePushA(name); }
    ~Range() { roctxRangePop(); }
    Range(const Range &) = delete;
    Range &operator=(const Range &) = delete;
};
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Address of the static workspace on `dev` (the current device); looked up once per device.
hipError_t scratch_setup(int dev) {
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[dev]) return hipSuccess;
    void *p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e == hipSuccess && p) g_scratch_ptr[dev] = p;
    return e != hipSuccess ? e : (p ? hipSuccess : hipErrorInvalidSymbol);
}

void *scratch_of(int dev) {
    if (dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return g_scratch_ptr[dev];
}
}  // namespace

struct smi_ctx {
    int device = 0;
    std::string err;
    std::string scratch_err;   // why the static workspace is unavailable (empty: available)
    int opt_kernel = 0;
    int opt_graph = 0;
    int opt_chunk = 0;
    int opt_rev = 0;
    int opt_rev_group = 0;      // SMI_OPT_REV_GROUP: 0 by the cache budget, k: at most k shots
    int opt_fwd_group = 0;      // SMI_OPT_FWD_GROUP: the same for 2D forward passes
    int opt_xcd = 0;
    int opt_family = 1;
    void *last_ws = nullptr;
    size_t last_status_off = 0;
    double cnt[3] = {0, 0, 0};
    double bytes[2] = {0, 0};
    // kernel timing (SMI_OPT_TIMING): every opt_timing-th forward step of the batched sweep
    // is launched with device-stamped events; events[4 k .. 4 k + 4) belong to sample k
    int opt_timing = 0;
    // captured time loops (SMI_OPT_GRAPH), keyed by everything their launches bind
    std::vector<std::pair<std::string, hipGraphExec_t>> graphs;
    hipStream_t cap = nullptr;
    std::vector<hipEvent_t> events;
    std::vector<double> sample_bytes;   // [samples][3], as Plan::step_bytes
    std::vector<int> sample_nk;         // kernels of the sampled step (2, or 1 for the fused step)
    size_t nsample = 0;
    // reverse steps sampled by SMI_OPT_TIMING: events around every opt_timing-th reverse
    // iteration (rev_events[2 k], [2 k + 1]) and that step's algorithmic bytes
    std::vector<hipEvent_t> rev_events;
    std::vector<double> rev_sample_bytes;
    size_t nrev = 0;
    // shot groups (smi_set_shot_groups): offsets [ngroup + 1]; empty = one group of all shots
    std::vector<int> groups;
    // autotuner (SMI_OPT_AUTOTUNE): the kernel choice picked per plan shape, the reverse-form
    // samples of a first reverse call still to be read, and the text of the last pick
    int opt_autotune = 0;
    struct Pick {
        bool fwd = false, rev = false;     // forward kernels / 2D reverse form tuned
        int march = 0, run = 32, depth = 2, rev_form = 0, yp = 0, y3 = 0;
        bool xcd = false, ymap = false, step2d = false;
    };
    std::map<std::string, Pick> picks;
    struct RevTune {
        std::string key;
        std::vector<hipEvent_t> ev;        // [2 k], [2 k + 1] around sampled iteration k
        std::vector<int> form;             // its reverse form (1 or 2)
    };
    std::vector<RevTune> rev_tunes;
    std::vector<hipEvent_t> tune_events;
    std::string tune_report;
    ~smi_ctx() {
        for (hipEvent_t e : events) (void)hipEventDestroy(e);
        for (hipEvent_t e : rev_events) (void)hipEventDestroy(e);
        for (hipEvent_t e : tune_events) (void)hipEventDestroy(e);
        for (auto &r : rev_tunes)
            for (hipEvent_t e : r.ev) (void)hipEventDestroy(e);
        for (auto &g : graphs) (void)hipGraphExecDestroy(g.second);
        if (cap) (void)hipStreamDestroy(cap);
    }
};

struct smi_state {
    smi_ctx *ctx = nullptr;
    Plan plan;
    void *ws = nullptr;
    size_t ws_bytes = 0;
    const float *vp = nullptr, *rho = nullptr, *stf = nullptr;
    bool consumed = false;
};

namespace {

// The plan shape an autotuner pick holds for: geometry, batch, schedule and job kind.
std::string shape_key(const Plan &pl) {
    char b[256];
    snprintf(b, sizeof b, "%d %d %d %d %d %d %d %d %d %d %d %d", pl.nd, pl.N, pl.n[0], pl.n[1],
             pl.n[2], pl.g.nb, pl.nshot, pl.g.nt, pl.g.box, pl.g.dr, pl.g.freesurf, (int)pl.save);
    return b;
}

// Apply an autotuner pick (SMI_OPT_AUTOTUNE) for this plan shape over the kernel options:
// the forward kernels to a forward pass, the reverse form to a reverse pass.
void apply_pick(smi::StepCtx &c, const smi_ctx *ctx, const Plan &pl, bool forward) {
    if (!ctx->opt_autotune || c.plain) return;
    auto it = ctx->picks.find(shape_key(pl));
    if (it == ctx->picks.end()) return;
    const smi_ctx::Pick &p = it->second;
    if (forward && p.fwd) {
        c.march = p.march;
        c.xcd = p.xcd;
        c.ymap = p.ymap;
        c.step2d = p.step2d;
        c.run = p.run;
        c.depth = p.depth;
        c.yp = p.yp;
        c.zl = false;
        c.y3 = p.y3;
    }
    if (!forward && p.rev) c.rev = p.rev_form;
}

// Kernel choice of a step context from the context options.  Default: register-blocked half
// steps, 4 cells per lane with the XCD-contiguous order in 2D; in 3D the half steps marching
// along y for the forward and adjoint steps where they apply, and register-blocked kernels with
// 2 cells per lane for the reconstruction and elsewhere (the fastest measured on the
// configurations the library targets).
void configure(smi::StepCtx &c, const smi_ctx *ctx, const Plan &pl) {
    c.plain = ctx->opt_kernel == 1;
    c.march = 0;
    c.xcd = false;
    c.y3 = 0;
    c.zl = false;
    c.ymap = false;
    c.rev = ctx->opt_rev;
    c.step2d = false;
    c.run = 32;
    c.depth = 2;
    c.yp = 0;
    // 3D forward and adjoint half steps of options 0, 6 and 7: the y-marching kernels (4-column
    // tiles, 32 planes per workgroup) wherever they apply -- 8.5 % faster on the whole 3D RTM and
    // 15 % on the full-grid step than the register-blocked kernels, which remain option 3
    const int y3_default = pl.nd == 3 && smi::y3_available(pl) ? 432 : 0;
    if (ctx->opt_kernel == 0 || ctx->opt_kernel == 6 || ctx->opt_kernel == 7) {
        c.y3 = y3_default;
        // the register-blocked 3D kernels (the reconstruction, and every half step where the
        // y-marching ones do not apply) in the XCD-contiguous z-fastest order
        c.ymap = pl.nd == 3;
    }
    if (ctx->opt_kernel == 6) {
        // the fused marching 2D forward step (other passes and 3D: the kernels of 0)
        c.march = pl.nd == 2 ? 4 : 2;
        c.xcd = pl.nd == 2;
        c.step2d = smi::step2d_available(pl);
        c.run = ctx->opt_chunk % 100 == 64 ? 64 : 32;
        const int d = ctx->opt_chunk / 100;
        c.depth = d == 1 || d == 4 ? d : 2;
    } else if (ctx->opt_kernel == 8) {
        // the plane-tiled y-marching 3D half steps (2D: the kernels of 0)
        c.march = pl.nd == 2 ? 4 : 2;
        c.xcd = pl.nd == 2;
        // SMI_OPT_CHUNK = CY + 1000 form (0: 32, form 0 with 32 planes, the fastest measured)
        const int code = ctx->opt_chunk > 0 ? ctx->opt_chunk : 32;
        const int cy = code % 1000, form = code / 1000;
        c.yp = smi::yp_available(pl) ? 1000 * (form <= 2 ? form : 0) + (cy == 16 || cy == 64 ? cy : 32) : 0;
    } else if (ctx->opt_kernel == 7) {
        // the tiled fused 2D forward step (other passes and 3D: the kernels of 0)
        c.march = pl.nd == 2 ? 4 : 2;
        c.xcd = pl.nd == 2;
        c.step2d = smi::step2d_available(pl);
        c.run = ctx->opt_chunk == 64 ? 64 : 32;
        c.depth = 0;
    } else if (ctx->opt_kernel == 0) {
        c.march = pl.nd == 2 ? 4 : 2;
        c.xcd = pl.nd == 2;
    } else if (ctx->opt_kernel == 2) {
        c.march = ctx->opt_chunk % 100 == 8 ? 8 : 4;
        c.zl = ctx->opt_chunk >= 100;   // the tiled variant of the fused step
    } else if (ctx->opt_kernel == 3) {
        const int cm = ctx->opt_chunk % 100;
        c.march = cm == 2 || cm == 8 ? cm : 4;
        c.zl = ctx->opt_chunk >= 100;
        c.xcd = ctx->opt_xcd == 1;
        c.ymap = ctx->opt_xcd == 2 && pl.nd == 3;
    } else if (ctx->opt_kernel == 4) {
        c.xcd = ctx->opt_xcd != 0;
    } else if (ctx->opt_kernel == 5) {
        c.march = pl.nd == 2 ? 4 : 2;
        c.xcd = pl.nd == 2;
        c.y3 = smi::y3_available(pl) ? (ctx->opt_chunk > 0 ? ctx->opt_chunk : 432) : 0;
    }
}

smi_status fail(smi_ctx *c, smi_status st, const std::string &msg) {
    if (c) c->err = msg;
    return st;
}

smi_status hip_fail(smi_ctx *c, hipError_t e, const char *where) {
    std::string m = std::string(where) + ": " + hipGetErrorString(e);
    return fail(c, SMI_E_HIP, m);
}

#define HIPCHK(expr, where)                                   \
    do {                                                      \
        hipError_t e_ = (expr);                               \
        if (e_ != hipSuccess) return hip_fail(ctx, e_, where); \
    } while (0)

// ---------------------------------------------------------------- captured time loops

constexpr size_t kMaxGraphs = 8;
// state of one group of shots in a 2D forward or reverse pass: 7/8 of the 256 MB last-level cache
constexpr double kGroupBudget = 224.0 * 1024 * 1024;

struct Key {
    std::string b;
    template <class T> Key &put(const T &v) {
        b.append(reinterpret_cast<const char *>(&v), sizeof(T));
        return *this;
    }
    template <class T> Key &vec(const std::vector<T> &v) {   // FNV-1a of the contents
        uint64_t h = 1469598103934665603ull;
        const unsigned char *q = reinterpret_cast<const unsigned char *>(v.data());
        for (size_t i = 0; i < v.size() * sizeof(T); ++i) h = (h ^ q[i]) * 1099511628211ull;
        return put(h).put(v.size());
    }
};

// Everything a plan bakes into the launches of its time loop: geometry, boxes and kernel
// choice, and the point-operator layout that decides which launches exist and how wide their
// grids are (sources spread over several nodes or not, the taps per source, the nodes of the
// adjoint-source gather).
Key plan_key(char tag, const Plan &pl, const smi::StepCtx &c) {
    Key k;
    k.put(tag).put(pl.geom).put(pl.band).put(pl.nshot).put(pl.nrun).put(pl.nsave);
    k.put(pl.save).put(pl.g.nt).put(pl.g.dr).put(c.plain).put(c.march).put(c.xcd).put(c.zl).put(c.rev).put(c.ymap);
    k.put(c.y3).put(pl.chunk).put(c.step2d).put(c.run).put(c.depth).put(c.yp);
    k.vec(pl.fbox).vec(pl.abox).vec(pl.rbox).vec(pl.rec_off);
    k.put(pl.src_multi).vec(pl.src_toff).vec(pl.src_cell).vec(pl.inj_off);
    k.put(pl.inj_fused).put(pl.inj_zlo).put(pl.inj_nrow);
    return k;
}

// Enqueue the loop through a cached graph: captured on the context's own stream the first
// time a key is seen, instantiated, then launched on the caller's stream (after the work the
// call already enqueued there).  `enqueue(s)` must enqueue the loop on s.
template <class F>
smi_status graph_run(smi_ctx *ctx, const std::string &key, hipStream_t st, F enqueue) {
    size_t i = 0;
    while (i < ctx->graphs.size() && ctx->graphs[i].first != key) ++i;
    if (i == ctx->graphs.size()) {
        if (!ctx->cap) HIPCHK(hipStreamCreateWithFlags(&ctx->cap, hipStreamNonBlocking), "capture stream");
        HIPCHK(hipStreamBeginCapture(ctx->cap, hipStreamCaptureModeThreadLocal), "capture begin");
        smi_status s = enqueue(ctx->cap);
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(ctx->cap, &g);
        if (s != SMI_OK) {
            if (g) (void)hipGraphDestroy(g);
            return s;
        }
        if (e != hipSuccess) return hip_fail(ctx, e, "capture end");
        hipGraphExec_t x = nullptr;
        e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) return hip_fail(ctx, e, "graph instantiate");
        if (ctx->graphs.size() >= kMaxGraphs) {
            (void)hipGraphExecDestroy(ctx->graphs.front().second);
            ctx->graphs.erase(ctx->graphs.begin());
        }
        ctx->graphs.emplace_back(key, x);
        i = ctx->graphs.size() - 1;
    }
    HIPCHK(hipGraphLaunch(ctx->graphs[i].second, st), "graph launch");
    return SMI_OK;
}


// Model speed range: the grid's stated bounds, or a device reduction read back once.
smi_status speeds(smi_ctx *ctx, const smi_grid *g, const float *vp, void *ws, size_t ws_bytes,
                  hipStream_t st, double &vmin, double &vmax) {
    if (g->vpmin > 0 && g->vpmax > 0) {
        vmin = g->vpmin;
        vmax = g->vpmax;
        return SMI_OK;
    }
    if (!vp || !ws || ws_bytes < 64) return fail(ctx, SMI_E_ARG, "vp / workspace missing");
    unsigned init[2] = {0x7f7fffffu, 0u}, out[2];
    unsigned *d = (unsigned *)((char *)ws + 16);
    long long n = (long long)g->n1 * g->n2 * (g->ndim == 3 ? g->n3 : 1);
    HIPCHK(hipMemcpyAsync(d, init, sizeof init, hipMemcpyHostToDevice, st), "minmax init");
    HIPCHK(smi::launch_minmax(vp, n, d, st), "minmax");
    HIPCHK(hipMemcpyAsync(out, d, sizeof out, hipMemcpyDeviceToHost, st), "minmax read");
    HIPCHK(hipStreamSynchronize(st), "minmax sync");
    float lo, hi;
    std::memcpy(&lo, &out[0], 4);
    std::memcpy(&hi, &out[1], 4);
    if (out[0] == 0u || !(hi > 0)) return fail(ctx, SMI_E_NONFINITE, "vp has non-finite or non-positive values");
    vmin = lo;
    vmax = hi;
    return SMI_OK;
}

// Upload CPML profiles, box tables, receivers and sources; clear the status word.
smi_status upload(smi_ctx *ctx, const Plan &pl, const Views &w, hipStream_t st) {
    HIPCHK(hipMemsetAsync(w.status, 0, 64, st), "status clear");
    HIPCHK(hipMemcpyAsync((void *)w.bdesc, &pl.band, sizeof(pl.band), hipMemcpyHostToDevice, st),
           "band layout");
    for (int a = 0; a < pl.nd; ++a) {
        std::vector<float> ai, bi, ah, bh;
        smi::cpml_profiles(pl, a, ai, bi, ah, bh);
        size_t M = pl.M[a] * sizeof(float);
        HIPCHK(hipMemcpyAsync(w.cpml.a_i[a], ai.data(), M, hipMemcpyHostToDevice, st), "cpml");
        HIPCHK(hipMemcpyAsync(w.cpml.b_i[a], bi.data(), M, hipMemcpyHostToDevice, st), "cpml");
        HIPCHK(hipMemcpyAsync(w.cpml.a_h[a], ah.data(), M, hipMemcpyHostToDevice, st), "cpml");
        HIPCHK(hipMemcpyAsync(w.cpml.b_h[a], bh.data(), M, hipMemcpyHostToDevice, st), "cpml");
    }
    HIPCHK(hipMemcpyAsync(w.fbox, pl.fbox.data(), pl.fbox.size() * sizeof(int),
                          hipMemcpyHostToDevice, st), "fbox");
    if (pl.adjoint) {
        HIPCHK(hipMemcpyAsync(w.abox, pl.abox.data(), pl.abox.size() * sizeof(int),
                              hipMemcpyHostToDevice, st), "abox");
        HIPCHK(hipMemcpyAsync(w.rbox, pl.rbox.data(), pl.rbox.size() * sizeof(int),
                              hipMemcpyHostToDevice, st), "rbox");
    }
    int R = pl.rec_off[pl.nshot];
    if (R > 0) {
        std::vector<long long> obase(R);
        std::vector<int> shot(R), stride(R);
        for (int s = 0; s < pl.nshot; ++s)
            for (int r = pl.rec_off[s]; r < pl.rec_off[s + 1]; ++r) {
                obase[r] = (long long)pl.g.nt * pl.rec_off[s] + (r - pl.rec_off[s]);
                shot[r] = s;
                stride[r] = pl.rec_off[s + 1] - pl.rec_off[s];
            }
        HIPCHK(hipMemcpyAsync(w.recv.obase, obase.data(), R * sizeof(long long), hipMemcpyHostToDevice, st), "rec");
        HIPCHK(hipMemcpyAsync(w.recv.shot, shot.data(), R * sizeof(int), hipMemcpyHostToDevice, st), "rec");
        HIPCHK(hipMemcpyAsync(w.recv.stride, stride.data(), R * sizeof(int), hipMemcpyHostToDevice, st), "rec");
        HIPCHK(hipMemcpyAsync(w.recv.toff, pl.rec_toff.data(), pl.rec_toff.size() * sizeof(int),
                              hipMemcpyHostToDevice, st), "rec");
        HIPCHK(hipMemcpyAsync(w.recv.tcell, pl.rec_tcell.data(), pl.rec_tcell.size() * sizeof(long long),
                              hipMemcpyHostToDevice, st), "rec");
        HIPCHK(hipMemcpyAsync(w.recv.tw, pl.rec_tw.data(), pl.rec_tw.size() * sizeof(float),
                              hipMemcpyHostToDevice, st), "rec");
    }
    const size_t U = pl.inj_cell.size(), T = pl.inj_rec.size();
    if (U > 0) {
        HIPCHK(hipMemcpyAsync(w.inj.cell, pl.inj_cell.data(), U * sizeof(long long), hipMemcpyHostToDevice, st), "inj");
        HIPCHK(hipMemcpyAsync(w.inj.shot, pl.inj_shot.data(), U * sizeof(int), hipMemcpyHostToDevice, st), "inj");
        HIPCHK(hipMemcpyAsync(w.inj.off, pl.inj_off.data(), (U + 1) * sizeof(int), hipMemcpyHostToDevice, st), "inj");
        HIPCHK(hipMemcpyAsync(w.inj.rec, pl.inj_rec.data(), T * sizeof(int), hipMemcpyHostToDevice, st), "inj");
        HIPCHK(hipMemcpyAsync(w.inj.w, pl.inj_w.data(), T * sizeof(float), hipMemcpyHostToDevice, st), "inj");
    }
    if (w.injmap)
        HIPCHK(hipMemcpyAsync(w.injmap, pl.inj_map.data(), pl.inj_map.size() * sizeof(int),
                              hipMemcpyHostToDevice, st), "inj");
    HIPCHK(hipMemcpyAsync(w.src_cell, pl.src_cell.data(), pl.nshot * sizeof(long long),
                          hipMemcpyHostToDevice, st), "src");
    HIPCHK(hipMemcpyAsync(w.src_toff, pl.src_toff.data(), pl.src_toff.size() * sizeof(int),
                          hipMemcpyHostToDevice, st), "src");
    HIPCHK(hipMemcpyAsync(w.src_tcell, pl.src_tcell.data(), pl.src_tcell.size() * sizeof(long long),
                          hipMemcpyHostToDevice, st), "src");
    HIPCHK(hipMemcpyAsync(w.src_tw, pl.src_tw.data(), pl.src_tw.size() * sizeof(float),
                          hipMemcpyHostToDevice, st), "src");
    return SMI_OK;
}

size_t field_bytes(const Plan &pl) {
    return sizeof(float) * (size_t)pl.nshot * ((size_t)pl.P * (1 + pl.nd) +
           2 * (size_t)(pl.geom.psz[0] + pl.geom.psz[1] + pl.geom.psz[2]));
}

smi_status zero_fields(smi_ctx *ctx, const Plan &pl, const smi::Fields &f, hipStream_t st) {
    HIPCHK(hipMemsetAsync(f.p, 0, field_bytes(pl), st), "field clear");
    return SMI_OK;
}

// The shot ranges the results are reduced over: the context's groups, or all shots.
smi_status shot_groups(smi_ctx *ctx, int nshot, std::vector<int> &off) {
    if (ctx->groups.empty()) {
        off = {0, nshot};
        return SMI_OK;
    }
    if (ctx->groups.back() != nshot)
        return fail(ctx, SMI_E_ARG, "the shot groups cover " + std::to_string(ctx->groups.back()) +
                                        " shots, the call has " + std::to_string(nshot));
    off = ctx->groups;
    return SMI_OK;
}

smi_status check_snaps(smi_ctx *ctx, const smi_grid *g, const int *snap_it, int nsnap, float *snaps) {
    if (nsnap < 0) return fail(ctx, SMI_E_ARG, "nsnap < 0");
    if (nsnap > 0) {
        if (!snap_it || !snaps) return fail(ctx, SMI_E_ARG, "snapshot list or buffer missing");
        for (int k = 0; k < nsnap; ++k)
            if (snap_it[k] < 0 || snap_it[k] > g->nt) return fail(ctx, SMI_E_ARG, "snapshot level outside 0..nt");
    }
    return SMI_OK;
}

// ---------------------------------------------------------------- autotuner

// Forward candidates for a plan: kernel family, cells per lane, tile order, and the run width
// and look-ahead of the fused 2D step.  Every candidate gives the default's results (bitwise
// for the register-blocked kernels and the fused step, as the parity tests check).
struct Cand {
    int march;
    bool xcd, ymap, step2d;
    int run, depth;
    const char *name;
    int yp = 0, y3 = 0;
};

std::vector<Cand> fwd_candidates(const Plan &pl) {
    std::vector<Cand> v;
    if (pl.nd == 2) {
        v.push_back({4, true, false, false, 32, 2, "march4-xcd"});
        v.push_back({2, true, false, false, 32, 2, "march2-xcd"});
        v.push_back({8, true, false, false, 32, 2, "march8-xcd"});
        v.push_back({4, false, false, false, 32, 2, "march4-plain"});
        if (smi::step2d_available(pl)) {
            v.push_back({4, true, false, true, 32, 2, "fused-c32-d2"});
            v.push_back({4, true, false, true, 64, 2, "fused-c64-d2"});
            v.push_back({4, true, false, true, 32, 4, "fused-c32-d4"});
            v.push_back({4, true, false, true, 32, 0, "tile-32"});
            v.push_back({4, true, false, true, 64, 0, "tile-64"});
        }
    } else {
        v.push_back({2, false, false, false, 32, 2, "march2-plain"});
        v.push_back({4, false, false, false, 32, 2, "march4-plain"});
        v.push_back({2, true, false, false, 32, 2, "march2-xcd"});
        v.push_back({2, false, true, false, 32, 2, "march2-zfast"});
        if (smi::yp_available(pl)) {
            v.push_back({2, false, false, false, 32, 2, "yplane-2x8", 32});
        }
        if (smi::y3_available(pl)) v.push_back({2, false, false, false, 32, 2, "ymarch-4x32", 0, 432});
    }
    return v;
}

void set_cand(smi::StepCtx &c, const Cand &q) {
    c.march = q.march;
    c.xcd = q.xcd;
    c.ymap = q.ymap;
    c.step2d = q.step2d;
    c.run = q.run;
    c.depth = q.depth;
    c.yp = q.yp;
    c.zl = false;
    c.y3 = q.y3;
}

smi_status zero_fields(smi_ctx *ctx, const Plan &pl, const smi::Fields &f, hipStream_t st);

// Time every forward candidate on the same steps -- three windows of 8 consecutive steps at
// 30, 60 and 90 % of the schedule, so the boxes are those the call will run -- with events
// around each candidate's launches (gaps between dependent launches included), keep the
// fastest for this plan shape, and clear the fields the timing runs wrote.  Blocks until the
// timing runs are done (once per plan shape and context).
smi_status tune_forward(smi_ctx *ctx, const Plan &pl, const Views &w, smi::StepCtx &c,
                        hipStream_t st) {
    Range range("smi autotune forward");
    const std::vector<Cand> cands = fwd_candidates(pl);
    constexpr int K = 8;
    std::vector<int> steps;
    for (double f : {0.3, 0.6, 0.9}) {
        const int s0 = (int)(f * std::max(0, pl.nrun - K));
        for (int k = 0; k < K && s0 + k < pl.nrun; ++k) steps.push_back(s0 + k);
    }
    while (ctx->tune_events.size() < 2 * cands.size()) {
        hipEvent_t e;
        HIPCHK(hipEventCreate(&e), "tuning event");
        ctx->tune_events.push_back(e);
    }
    smi::StepCtx t = c;
    t.st = st;
    t.ev = nullptr;
    t.ext_it = -1;
    t.save_p_slot = t.save_v_slot = -1;
    for (size_t q = 0; q < cands.size(); ++q) {
        set_cand(t, cands[q]);
        HIPCHK(hipEventRecord(ctx->tune_events[2 * q], st), "tuning event");
        for (int it : steps)
            HIPCHK(t.step2d ? smi::fwd_step_2d(t, w.f, w.f2, it) : smi::fwd_step(t, it), "tuning step");
        HIPCHK(hipEventRecord(ctx->tune_events[2 * q + 1], st), "tuning event");
    }
    HIPCHK(hipEventSynchronize(ctx->tune_events[2 * cands.size() - 1]), "tuning sync");
    size_t best = 0;
    float best_ms = 0.f;
    std::string rep = "forward " + shape_key(pl) + ":";
    for (size_t q = 0; q < cands.size(); ++q) {
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, ctx->tune_events[2 * q], ctx->tune_events[2 * q + 1]), "tuning time");
        char b[96];
        snprintf(b, sizeof b, " %s %.1f us/step;", cands[q].name, 1e3 * ms / steps.size());
        rep += b;
        if (q == 0 || ms < best_ms) { best = q; best_ms = ms; }
    }
    rep += std::string(" pick ") + cands[best].name;
    smi_ctx::Pick &p = ctx->picks[shape_key(pl)];
    p.fwd = true;
    p.march = cands[best].march;
    p.xcd = cands[best].xcd;
    p.ymap = cands[best].ymap;
    p.step2d = cands[best].step2d;
    p.run = cands[best].run;
    p.depth = cands[best].depth;
    p.yp = cands[best].yp;
    p.y3 = cands[best].y3;
    ctx->tune_report = rep;
    set_cand(c, cands[best]);
    // the timing runs wrote both field sets (and receivers and bands the loop rewrites)
    smi_status s = zero_fields(ctx, pl, w.f, st);
    if (s == SMI_OK && pl.dbuf) s = zero_fields(ctx, pl, w.f2, st);
    return s;
}

// Read the reverse-form samples of an earlier reverse call on this plan shape (their events
// completed long ago) and keep the faster form.
smi_status read_rev_tune(smi_ctx *ctx, const std::string &key) {
    for (size_t i = 0; i < ctx->rev_tunes.size(); ++i) {
        smi_ctx::RevTune &r = ctx->rev_tunes[i];
        if (r.key != key) continue;
        double t[3] = {0, 0, 0};
        int n[3] = {0, 0, 0};
        for (size_t k = 0; k < r.form.size(); ++k) {
            HIPCHK(hipEventSynchronize(r.ev[2 * k + 1]), "tuning sync");
            float ms = 0.f;
            HIPCHK(hipEventElapsedTime(&ms, r.ev[2 * k], r.ev[2 * k + 1]), "tuning time");
            t[r.form[k]] += ms;
            ++n[r.form[k]];
        }
        smi_ctx::Pick &p = ctx->picks[key];
        p.rev = true;
        if (n[1] && n[2]) {
            const double a = t[1] / n[1], b = t[2] / n[2];
            p.rev_form = a <= b ? 1 : 2;
            char buf[160];
            snprintf(buf, sizeof buf, "reverse %s: two-launch %.1f us/step; five-launch %.1f us/step; pick %s",
                     key.c_str(), 1e3 * a, 1e3 * b, a <= b ? "two-launch" : "five-launch");
            ctx->tune_report = buf;
        }
        for (hipEvent_t e : r.ev) (void)hipEventDestroy(e);
        ctx->rev_tunes.erase(ctx->rev_tunes.begin() + i);
        return SMI_OK;
    }
    return SMI_OK;
}

// Alg. 2, forward loop: [save bands] -> v, p update with source -> record.
smi_status run_forward(smi_ctx *ctx, const Plan &pl, const Views &w, const float *vp,
                       const float *rho, const float *stf, float *dcal, const int *snap_it,
                       int nsnap, float *snaps, hipStream_t st) {
    Range range("smi forward");
    smi_status s = upload(ctx, pl, w, st);
    if (s != SMI_OK) return s;
    HIPCHK(smi::launch_model_prep(pl, w, vp, rho, st), "model prep");
    s = zero_fields(ctx, pl, w.f, st);
    if (s != SMI_OK) return s;
    smi::StepCtx c{&pl, &w, stf, st, false};
    configure(c, ctx, pl);
    apply_pick(c, ctx, pl, true);
    if (ctx->opt_autotune && !c.plain && !ctx->picks[shape_key(pl)].fwd) {
        s = tune_forward(ctx, pl, w, c, st);
        if (s != SMI_OK) return s;
    }
    for (int k = 0; k < nsnap; ++k)
        if (snap_it[k] == 0) HIPCHK(smi::snap(c, w.f, snaps, k, nsnap), "snap");
    const bool f2d = c.step2d;
    bool fused = f2d || (ctx->opt_kernel == 2 && pl.dbuf && pl.g.dr == 1 && smi::fused_fwd_available(pl));
    if (fused) {
        s = zero_fields(ctx, pl, w.f2, st);
        if (s != SMI_OK) return s;
    }
    const int nt = pl.g.nt, dr = pl.g.dr;
    const bool timed = ctx->opt_timing > 0 && !c.plain;
    const bool defer = !fused && smi::march_forward(c);
    const size_t state_bytes = sizeof(float) * (size_t)pl.nshot * (size_t)pl.P * (1 + pl.nd);
    // 2D, register-blocked kernels: the time loop runs once per group of shots whose fields stay
    // in the last-level cache between the launches of a step (one group when all of them fit);
    // every shot's arithmetic is the one of a single loop
    const std::vector<int> fg = pl.nd == 2 && !c.plain && !fused && c.march > 0
                                    ? smi::fwd_groups(pl, kGroupBudget, ctx->opt_fwd_group)
                                    : std::vector<int>{0, pl.nshot};
    // level nt of (p, v) of the current group: from src into dst (same layout, every shot)
    auto copy_state = [&](float *dst, const float *src, hipStream_t ls) -> hipError_t {
        if (c.s0 == 0 && smi::shot_end(c) == pl.nshot)
            return hipMemcpyAsync(dst, src, state_bytes, hipMemcpyDeviceToDevice, ls);
        const size_t n = (size_t)(smi::shot_end(c) - c.s0) * (size_t)pl.P;
        for (int k = 0; k <= pl.nd; ++k) {
            const size_t o = ((size_t)k * pl.nshot + c.s0) * (size_t)pl.P;
            const hipError_t e = hipMemcpyAsync(dst + o, src + o, sizeof(float) * n,
                                                hipMemcpyDeviceToDevice, ls);
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    };
    auto loop = [&](hipStream_t ls) -> smi_status {
    c.st = ls;
    for (size_t gi = 0; gi + 1 < fg.size(); ++gi) {
        c.s0 = fg[gi];
        c.s1 = fg[gi + 1];
        c.ext_it = -1;
        for (int it = 0; it < pl.nrun; ++it) {
            // fused steps alternate between the two buffers: level it lives in cur
            const smi::Fields &cur = fused && (it & 1) ? w.f2 : w.f;
            const smi::Fields &nxt = fused && !(it & 1) ? w.f2 : w.f;
            // saved levels: on the register-blocked path the p cells of level it ride on this
            // step's v launch and its v cells rode on the previous step's p launch
            c.save_p_slot = c.save_v_slot = -1;
            if (pl.save && it % dr == 0) {
                // the fused marching step reads level it from cur and carries the whole saved level
                if (f2d || (defer && it > 0)) c.save_p_slot = it / dr;
                else HIPCHK(smi::band_save(c, cur, it / dr), "band save");
            }
            if (pl.save && defer && (it + 1) % dr == 0 && it + 1 < pl.nrun) c.save_v_slot = (it + 1) / dr;
            if (timed && it % ctx->opt_timing == 0) {
                const size_t k = ctx->nsample;
                while (ctx->events.size() < 4 * (k + 1)) {
                    hipEvent_t e;
                    HIPCHK(hipEventCreate(&e), "timing event");
                    ctx->events.push_back(e);
                }
                double sb[3];
                smi::step_bytes_of(pl, it, c.s0, smi::shot_end(c), sb);
                // the fused step is one kernel: it carries the step's bytes as its "first" kernel
                const double row[3] = {sb[0], fused ? sb[0] : sb[1], fused ? 0.0 : sb[2]};
                ctx->sample_bytes.insert(ctx->sample_bytes.end(), row, row + 3);
                ctx->sample_nk.push_back(fused ? 1 : 2);
                ctx->nsample = k + 1;
                c.ev = &ctx->events[4 * k];
            }
            if (f2d) {
                // receivers of step it - 1 are sampled by this launch from cur (level it)
                HIPCHK(smi::fwd_step_2d(c, cur, nxt, it), "forward step");
                c.ev = nullptr;
                c.ext_it = -1;
                if (it < nt) HIPCHK(smi::src_taps(c, it, nxt.p, 1.f), "source");
                if (it < nt) {
                    c.ext_it = it;
                    c.ext_dcal = dcal;
                }
            } else if (fused) {
                HIPCHK(smi::fwd_step_fused(c, cur, nxt, it), "forward step");
                c.ev = nullptr;
                if (it < nt) HIPCHK(smi::src_taps(c, it, nxt.p, 1.f), "source");
                if (it < nt) HIPCHK(smi::extract(c, it, dcal, nxt.p), "extract");
            } else {
                // the register-blocked kernels sample the receivers of step it inside the v launch
                // of step it + 1 (the v update leaves p alone); the last one is sampled below
                HIPCHK(smi::fwd_step(c, it), "forward step");
                c.ev = nullptr;
                c.ext_it = -1;
                if (it < nt) HIPCHK(smi::src_taps(c, it, w.f.p, 1.f), "source");
                if (it < nt && defer) {
                    c.ext_it = it;
                    c.ext_dcal = dcal;
                } else if (it < nt) {
                    HIPCHK(smi::extract(c, it, dcal), "extract");
                }
            }
            for (int k = 0; k < nsnap; ++k)
                if (snap_it[k] == it + 1) HIPCHK(smi::snap(c, nxt, snaps, k, nsnap), "snap");
            if (w.fin && it + 1 == nt)   // level nt: the reverse pass starts from here
                HIPCHK(copy_state(w.fin, nxt.p, ls), "final copy");
        }
        if (c.ext_it >= 0) {
            // the last sampled step: level ext_it + 1 is in the second buffer after an odd step of
            // the fused steps
            const bool second = fused && ((c.ext_it + 1) & 1);
            HIPCHK(smi::extract(c, c.ext_it, dcal, second ? w.f2.p : w.f.p), "extract");
            c.ext_it = -1;
        }
        if (fused && (pl.nrun & 1)) {
            // the final level is in the second buffer; the reverse pass works on the first
            HIPCHK(hipMemcpyAsync(w.f.p, w.f2.p, field_bytes(pl), hipMemcpyDeviceToDevice, ls),
                   "final state copy");
        }
        if (pl.save && dr > 1) {
            HIPCHK(smi::band_save(c, w.f, pl.nsave - 1), "band save (last level)");
            HIPCHK(copy_state(w.f.p, w.fin, ls), "final restore");
        }
    }
    c.s0 = 0;
    c.s1 = -1;
    return SMI_OK;
    };
    if (ctx->opt_graph && !timed) {
        Key k = plan_key('F', pl, c);
        k.put(fused).put(w.status).put(stf).put(dcal).put(snaps).put(nsnap);
        for (int q = 0; q < nsnap; ++q) k.put(snap_it[q]);
        for (int v : fg) k.put(v);
        s = graph_run(ctx, k.b, st, loop);
    } else {
        s = loop(st);
    }
    c.st = st;
    if (s != SMI_OK) return s;
    ctx->cnt[0] = pl.cnt_fwd;
    ctx->cnt[1] = ctx->cnt[2] = 0;
    ctx->bytes[0] = pl.bytes_fwd;
    ctx->bytes[1] = 0;
    ctx->last_ws = (void *)w.status;
    return SMI_OK;
}

// Alg. 2, reverse loop: adjoint source -> reconstruction (+gradient) -> adjoint step (+image).
smi_status run_reverse(smi_ctx *ctx, smi_state *stt, const float *G, float *grad,
                       float *grad_rho, float *image, float *illum, float *image_norm,
                       const int *snap_it, int nsnap, float *snaps, hipStream_t st) {
    Range range("smi reverse");
    const Plan &pl = stt->plan;
    Views w = smi::views(pl, stt->ws);
    bool adj = G != nullptr;
    const int family = ctx->opt_family;
    // the density face sums are needed for the second gradient and for Vp at fixed Ip
    const bool want_r = adj && (grad_rho || (grad && family == 2));
    if (want_r && !pl.rho_acc)
        return fail(ctx, SMI_E_ARG, "this job keeps no density accumulators (use a gradient job)");
    bool want_g = adj && (grad || grad_rho), want_i = adj && (image || illum || image_norm);
    std::vector<int> grp;
    smi_status s = shot_groups(ctx, pl.nshot, grp);
    if (s != SMI_OK) return s;
    s = zero_fields(ctx, pl, w.q, st);
    if (s != SMI_OK) return s;
    HIPCHK(hipMemsetAsync(w.acc_g, 0, sizeof(float) * 3 * (size_t)pl.nshot * pl.I, st), "acc clear");
    if (want_r)
        HIPCHK(hipMemsetAsync(w.acc_r[0], 0, sizeof(float) * pl.nd * (size_t)pl.nshot * pl.P, st),
               "density sums clear");
    const std::string key = shape_key(pl);
    if (ctx->opt_autotune) {
        s = read_rev_tune(ctx, key);
        if (s != SMI_OK) return s;
    }
    smi::StepCtx c{&pl, &w, stt->stf, st, false};
    configure(c, ctx, pl);
    apply_pick(c, ctx, pl, false);
    for (int k = 0; k < nsnap; ++k)
        if (snap_it[k] == pl.g.nt) HIPCHK(smi::snap(c, w.f, snaps, k, nsnap), "snap");
    // 2D: the reverse loop runs once per group of shots, each group small enough that its
    // reverse state (source and adjoint fields, memory variables, accumulators) stays in the
    // last-level cache between its launches; every shot's arithmetic is the same as in one
    // loop over all shots, and the outputs are reduced per shot afterwards
    const std::vector<int> rg = c.plain ? std::vector<int>{0, pl.nshot}
                                        : smi::rev_groups(pl, kGroupBudget, ctx->opt_rev_group, want_r);
    const bool timed = ctx->opt_timing > 0;
    // 2D reverse form not yet tuned for this shape: sampled iterations of this call alternate
    // the two forms (bitwise the same results), timed by events read on the next call
    const bool rev_tune = ctx->opt_autotune && pl.nd == 2 && !c.plain && c.march == 4 && !c.zl &&
                          !ctx->picks[key].rev && pl.g.nt >= 64;
    smi_ctx::RevTune rt;
    rt.key = key;
    const int base_rev = c.rev;
    auto loop = [&](hipStream_t ls) -> smi_status {
        c.st = ls;
        for (size_t gi = 0; gi + 1 < rg.size(); ++gi) {
            c.s0 = rg[gi];
            c.s1 = rg[gi + 1];
            // the adjoint sources of this level were added by the previous reverse step
            bool injected = false;
            for (int it = pl.g.nt - 1; it >= 0; --it) {
                // sampled reverse step: the device stamps an event before its first launch and
                // after its last
                hipEvent_t *ev = nullptr;
                if (timed && it % ctx->opt_timing == 0) {
                    const size_t k = ctx->nrev;
                    while (ctx->rev_events.size() < 2 * (k + 1)) {
                        hipEvent_t e;
                        HIPCHK(hipEventCreate(&e), "timing event");
                        ctx->rev_events.push_back(e);
                    }
                    double q[4];
                    smi::rev_iter_bytes(pl, it, c.s0, c.s1, q);
                    ctx->rev_sample_bytes.push_back(q[0] + (want_g ? q[1] : 0.0) +
                                                    (want_i && (image || image_norm) ? q[2] : 0.0) +
                                                    (want_i && (illum || image_norm) ? q[3] : 0.0));
                    ctx->nrev = k + 1;
                    ev = &ctx->rev_events[2 * k];
                    HIPCHK(hipEventRecord(ev[0], ls), "timing event");
                }
                if (adj && !injected) HIPCHK(smi::adj_inject(c, it, G), "adjoint source");
                HIPCHK(smi::src_taps(c, it, w.f.p, -1.f), "source removal");
                if (rev_tune && it % 16 == 7) {
                    hipEvent_t e0, e1;
                    HIPCHK(hipEventCreate(&e0), "tuning event");
                    HIPCHK(hipEventCreate(&e1), "tuning event");
                    rt.ev.push_back(e0);
                    rt.ev.push_back(e1);
                    rt.form.push_back(rt.form.size() % 2 ? 2 : 1);
                    c.rev = rt.form.back();
                    HIPCHK(hipEventRecord(e0, ls), "tuning event");
                    HIPCHK(smi::rev_step(c, it, want_g, want_i, adj ? G : nullptr, &injected),
                           "reverse step");
                    HIPCHK(hipEventRecord(e1, ls), "tuning event");
                    c.rev = base_rev;
                } else {
                    HIPCHK(smi::rev_step(c, it, want_g, want_i, adj ? G : nullptr, &injected),
                           "reverse step");
                }
                if (want_r) HIPCHK(smi::rho_faces(c, it), "density faces");
                if (ev) HIPCHK(hipEventRecord(ev[1], ls), "timing event");
                for (int k = 0; k < nsnap; ++k)
                    if (snap_it[k] == it) HIPCHK(smi::snap(c, w.f, snaps, k, nsnap), "snap");
            }
        }
        c.s0 = 0;
        c.s1 = -1;
        return SMI_OK;
    };
    if (ctx->opt_graph && !timed && !rev_tune) {
        Key k = plan_key('R', pl, c);
        k.put(stt->ws).put(stt->stf).put(G).put(snaps).put(nsnap).put(adj).put(want_g);
        k.put(want_i).put(want_r);
        for (int q = 0; q < nsnap; ++q) k.put(snap_it[q]);
        for (int v : rg) k.put(v);
        s = graph_run(ctx, k.b, st, loop);
    } else {
        s = loop(st);
    }
    c.st = st;
    if (rev_tune && !rt.form.empty()) ctx->rev_tunes.push_back(rt);
    else for (hipEvent_t e : rt.ev) (void)hipEventDestroy(e);
    if (s != SMI_OK) return s;
    // one output array per shot group, each the fixed-order sum over its own shots
    const size_t ng = grp.size() - 1;
    for (size_t k = 0; k < ng; ++k) {
        const size_t o = k * (size_t)pl.I;
        auto at = [&](float *p) { return p ? p + o : nullptr; };
        HIPCHK(smi::finalize(c, stt->vp, want_g && !want_r ? at(grad) : nullptr,
                             want_i ? at(image) : nullptr, want_i ? at(illum) : nullptr,
                             want_i ? at(image_norm) : nullptr, grp[k], grp[k + 1]), "finalize");
        if (want_r)
            HIPCHK(smi::finalize_family(c, stt->vp, stt->rho, family, at(grad), at(grad_rho),
                                        grp[k], grp[k + 1]), "finalize");
    }
    if (!adj) {
        size_t I = sizeof(float) * pl.I * ng;
        if (grad) HIPCHK(hipMemsetAsync(grad, 0, I, st), "grad clear");
        if (grad_rho) HIPCHK(hipMemsetAsync(grad_rho, 0, I, st), "grad_rho clear");
        if (image) HIPCHK(hipMemsetAsync(image, 0, I, st), "image clear");
        if (illum) HIPCHK(hipMemsetAsync(illum, 0, I, st), "illum clear");
        if (image_norm) HIPCHK(hipMemsetAsync(image_norm, 0, I, st), "image_norm clear");
    }
    ctx->cnt[1] = adj ? pl.cnt_adj : 0;
    ctx->cnt[2] = pl.cnt_rec;
    ctx->bytes[1] = pl.bytes_rev;
    return SMI_OK;
}

smi_status forward_common(smi_ctx *ctx, const smi_grid *grid, const smi_acq *acq,
                          smi_job job, const float *vp, const float *rho, const float *stf,
                          float *dcal, const int *snap_it, int nsnap, float *snaps, void *ws,
                          size_t ws_bytes, hipStream_t st, std::unique_ptr<smi_state> &out) {
    if (!grid || !acq) return fail(ctx, SMI_E_ARG, "grid / acq is NULL");
    if (!vp || !rho || !stf || !dcal) return fail(ctx, SMI_E_ARG, "vp, rho, stf and dcal are required");
    if (!ws) return fail(ctx, SMI_E_WORKSPACE, "workspace is NULL");
    smi_status s = check_snaps(ctx, grid, snap_it, nsnap, snaps);
    if (s != SMI_OK) return s;
    double vmin = 0, vmax = 0;
    s = speeds(ctx, grid, vp, ws, ws_bytes, st, vmin, vmax);
    if (s != SMI_OK) return s;
    auto stt = std::make_unique<smi_state>();
    s = smi::make_plan(grid, acq, job, vmin, vmax, stt->plan, ctx->err);
    if (s != SMI_OK) return s;
    if (ws_bytes < stt->plan.bytes) {
        char b[200];
        snprintf(b, sizeof b, "workspace has %zu bytes, %zu needed", ws_bytes, stt->plan.bytes);
        return fail(ctx, SMI_E_WORKSPACE, b);
    }
    stt->plan.chunk = ctx->opt_chunk;
    Views w = smi::views(stt->plan, ws);
    s = run_forward(ctx, stt->plan, w, vp, rho, stf, dcal, snap_it, nsnap, snaps, st);
    if (s != SMI_OK) return s;
    stt->ctx = ctx;
    stt->ws = ws;
    stt->ws_bytes = ws_bytes;
    stt->vp = vp;
    stt->rho = rho;
    stt->stf = stf;
    out = std::move(stt);
    return SMI_OK;
}

}  // namespace

extern "C" {

smi_status smi_ctx_create(int hip_device, smi_ctx **out) {
    if (!out) return SMI_E_ARG;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || hip_device < 0 || hip_device >= n) return SMI_E_HIP;
    if (hipSetDevice(hip_device) != hipSuccess) return SMI_E_HIP;
    smi_ctx *c = new smi_ctx();
    c->device = hip_device;
    // set-up of the static workspace on this device (a failure only disables smi_forward_static)
    const hipError_t e = scratch_setup(hip_device);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        c->scratch_err = std::string("static workspace: hipGetSymbolAddress: ") + hipGetErrorString(e);
    }
    *out = c;
    return SMI_OK;
}

void smi_ctx_destroy(smi_ctx *ctx) { delete ctx; }

const char *smi_last_error(const smi_ctx *ctx) { return ctx ? ctx->err.c_str() : "no context"; }

smi_status smi_set_option(smi_ctx *ctx, int option, int value) {
    if (!ctx) return SMI_E_ARG;
    if (option == SMI_OPT_KERNEL && value >= 0 && value <= 8) { ctx->opt_kernel = value; return SMI_OK; }
    if (option == SMI_OPT_GRAPH && (value == 0 || value == 1)) { ctx->opt_graph = value; return SMI_OK; }
    if (option == SMI_OPT_CHUNK && value >= 0 && value <= 9999) { ctx->opt_chunk = value; return SMI_OK; }
    if (option == SMI_OPT_REVERSE && value >= 0 && value <= 2) { ctx->opt_rev = value; return SMI_OK; }
    if (option == SMI_OPT_REV_GROUP && value >= 0) { ctx->opt_rev_group = value; return SMI_OK; }
    if (option == SMI_OPT_FWD_GROUP && value >= 0) { ctx->opt_fwd_group = value; return SMI_OK; }
    if (option == SMI_OPT_TILEMAP && value >= 0 && value <= 2) { ctx->opt_xcd = value; return SMI_OK; }
    if (option == SMI_OPT_FAMILY && (value == 1 || value == 2)) { ctx->opt_family = value; return SMI_OK; }
    if (option == SMI_OPT_AUTOTUNE && (value == 0 || value == 1 || value == 2)) {
        if (value == 2) {   // forget the picks
            ctx->picks.clear();
            value = ctx->opt_autotune;
        }
        ctx->opt_autotune = value;
        return SMI_OK;
    }
    if (option == SMI_OPT_TIMING && value >= 0) {
        ctx->opt_timing = value;
        ctx->nsample = 0;
        ctx->sample_bytes.clear();
        ctx->sample_nk.clear();
        ctx->nrev = 0;
        ctx->rev_sample_bytes.clear();
        return SMI_OK;
    }
    return fail(ctx, SMI_E_ARG, "unknown option or value");
}

smi_status smi_set_shot_groups(smi_ctx *ctx, int ngroup, const int *shot_off) {
    if (!ctx) return SMI_E_ARG;
    if (ngroup == 0) {
        ctx->groups.clear();
        return SMI_OK;
    }
    if (ngroup < 0 || !shot_off || shot_off[0] != 0)
        return fail(ctx, SMI_E_ARG, "shot groups: ngroup > 0 and shot_off[0] = 0 required");
    for (int k = 0; k < ngroup; ++k)
        if (shot_off[k + 1] <= shot_off[k]) return fail(ctx, SMI_E_ARG, "shot groups must not be empty");
    ctx->groups.assign(shot_off, shot_off + ngroup + 1);
    return SMI_OK;
}

smi_status smi_check(const smi_ctx *ctx, const smi_grid *grid, double vp_min, double vp_max) {
    std::string err;
    smi_status s = smi::check_grid(grid, vp_min, vp_max, err);
    if (ctx) const_cast<smi_ctx *>(ctx)->err = err;
    return s;
}

smi_status smi_workspace_bytes(const smi_ctx *ctx, const smi_grid *grid, const smi_acq *acq,
                               smi_job job, size_t *bytes) {
    smi_ctx *c = const_cast<smi_ctx *>(ctx);
    if (!grid || !acq || !bytes) return fail(c, SMI_E_ARG, "NULL argument");
    if (job < SMI_JOB_FORWARD || job > SMI_JOB_BORN) return fail(c, SMI_E_ARG, "bad job");
    // the layout does not depend on the speeds; use a range that passes the checks
    smi_grid g = *grid;
    double vmin = grid->vpmin > 0 ? grid->vpmin : 0, vmax = grid->vpmax > 0 ? grid->vpmax : 0;
    Plan pl;
    std::string err;
    if (!(vmin > 0 && vmax > 0)) {
        vmax = 1e-3 / g.dt;   // tiny CFL number
        vmin = vmax;
        g.fm = 1e-9;          // no dispersion limit
    }
    smi_status s = smi::make_plan(&g, acq, job, vmin, vmax, pl, err);
    if (c) c->err = err;
    if (s != SMI_OK) return s;
    *bytes = pl.bytes;
    return SMI_OK;
}

smi_status smi_forward(smi_ctx *ctx, const smi_grid *grid, const smi_acq *acq, const float *vp,
                       const float *rho, const float *stf, float *dcal, smi_state **state_out,
                       const int *snap_it, int nsnap, float *snaps, void *ws, size_t ws_bytes,
                       void *hip_stream) {
    if (!ctx) return SMI_E_ARG;
    std::unique_ptr<smi_state> stt;
    smi_status s = forward_common(ctx, grid, acq, state_out ? SMI_JOB_FORWARD_SAVE : SMI_JOB_FORWARD,
                                  vp, rho, stf, dcal, snap_it, nsnap, snaps, ws, ws_bytes,
                                  (hipStream_t)hip_stream, stt);
    if (s != SMI_OK) return s;
    if (state_out) *state_out = stt.release();
    return SMI_OK;
}

smi_status smi_forward_static(smi_ctx *ctx, const smi_grid *grid, const smi_acq *acq,
                              const float *vp, const float *rho, const float *stf, float *dcal,
                              void *hip_stream) {
    if (!ctx) return SMI_E_ARG;
    if (!grid || !acq) return fail(ctx, SMI_E_ARG, "grid / acq is NULL");
    void *ws = scratch_of(ctx->device);
    if (!ws || !ctx->scratch_err.empty())
        return fail(ctx, SMI_E_HIP, ctx->scratch_err.empty() ? "static workspace unavailable" : ctx->scratch_err);
    size_t need = 0;
    smi_status s = smi_workspace_bytes(ctx, grid, acq, SMI_JOB_FORWARD, &need);
    if (s != SMI_OK) return s;
    if (need > (size_t)SMI_STATIC_WS_BYTES) {
        char b[200];
        snprintf(b, sizeof b, "this job needs a %zu-byte workspace; the static workspace holds %zu",
                 need, (size_t)SMI_STATIC_WS_BYTES);
        return fail(ctx, SMI_E_WORKSPACE, b);
    }
    // nothing that creates runtime objects: no graph capture, no timing events
    const int graph = ctx->opt_graph, timing = ctx->opt_timing, tune = ctx->opt_autotune;
    ctx->opt_graph = 0;
    ctx->opt_timing = 0;
    ctx->opt_autotune = 0;
    std::unique_ptr<smi_state> stt;
    s = forward_common(ctx, grid, acq, SMI_JOB_FORWARD, vp, rho, stf, dcal, nullptr, 0, nullptr,
                       ws, (size_t)SMI_STATIC_WS_BYTES, (hipStream_t)hip_stream, stt);
    ctx->opt_graph = graph;
    ctx->opt_timing = timing;
    ctx->opt_autotune = tune;
    return s;
}

const char *smi_tuning_report(const smi_ctx *ctx) { return ctx ? ctx->tune_report.c_str() : ""; }

smi_status smi_adjoint_reconstruct(smi_ctx *ctx, smi_state *state, const float *adj_src,
                                   float *grad_vp, float *grad_rho, float *image, float *illum,
                                   float *image_norm, const int *snap_it, int nsnap, float *snaps,
                                   void *hip_stream) {
    if (!ctx) return SMI_E_ARG;
    if (!state || state->consumed || !state->plan.save)
        return fail(ctx, SMI_E_STATE, "state missing, already consumed, or saved without boundaries");
    if (state->ctx != ctx) return fail(ctx, SMI_E_STATE, "state belongs to another context");
    smi_status s = check_snaps(ctx, &state->plan.g, snap_it, nsnap, snaps);
    if (s != SMI_OK) return s;
    s = run_reverse(ctx, state, adj_src, grad_vp, grad_rho, image, illum, image_norm, snap_it,
                    nsnap, snaps, (hipStream_t)hip_stream);
    if (s != SMI_OK) return s;
    state->consumed = true;
    return SMI_OK;
}

smi_status smi_rtm_image(smi_ctx *ctx, const smi_grid *grid, const smi_acq *acq, const float *vp,
                         const float *rho, const float *stf, const float *dobs, float *image,
                         float *illum, float *image_norm, void *ws, size_t ws_bytes,
                         void *hip_stream) {
    if (!ctx) return SMI_E_ARG;
    if (!dobs) return fail(ctx, SMI_E_ARG, "dobs is NULL");
    hipStream_t st = (hipStream_t)hip_stream;
    // the internal dcal buffer sits inside ws; plan once to find it
    double vmin = 0, vmax = 0;
    smi_status s = speeds(ctx, grid, vp, ws, ws_bytes, st, vmin, vmax);
    if (s != SMI_OK) return s;
    smi_grid g = *grid;
    g.vpmin = vmin;
    g.vpmax = vmax;
    Plan pl;
    s = smi::make_plan(&g, acq, SMI_JOB_RTM, vmin, vmax, pl, ctx->err);
    if (s != SMI_OK) return s;
    if (!ws || ws_bytes < pl.bytes) return fail(ctx, SMI_E_WORKSPACE, "workspace too small");
    Views w = smi::views(pl, ws);
    std::unique_ptr<smi_state> stt;
    s = forward_common(ctx, &g, acq, SMI_JOB_RTM, vp, rho, stf, w.dcal, nullptr, 0, nullptr, ws,
                       ws_bytes, st, stt);
    if (s != SMI_OK) return s;
    smi::StepCtx c{&stt->plan, &w, stf, st, false};
    configure(c, ctx, stt->plan);
    HIPCHK(smi::scale_copy(c, dobs, w.G, (float)g.dt), "rtm source");
    return run_reverse(ctx, stt.get(), w.G, nullptr, nullptr, image, illum, image_norm, nullptr, 0,
                       nullptr, st);
}

smi_status smi_fwi_grad(smi_ctx *ctx, const smi_grid *grid, const smi_acq *acq, const float *vp,
                        const float *rho, const float *stf, const float *dobs, float *grad_vp,
                        float *grad_rho, double *misfit, float *dcal_out, void *ws,
                        size_t ws_bytes, void *hip_stream) {
    if (!ctx) return SMI_E_ARG;
    if (!dobs || (!grad_vp && !grad_rho))
        return fail(ctx, SMI_E_ARG, "dobs and at least one of grad_vp, grad_rho are required");
    hipStream_t st = (hipStream_t)hip_stream;
    double vmin = 0, vmax = 0;
    smi_status s = speeds(ctx, grid, vp, ws, ws_bytes, st, vmin, vmax);
    if (s != SMI_OK) return s;
    smi_grid g = *grid;
    g.vpmin = vmin;
    g.vpmax = vmax;
    Plan pl;
    s = smi::make_plan(&g, acq, SMI_JOB_GRAD, vmin, vmax, pl, ctx->err);
    if (s != SMI_OK) return s;
    if (!ws || ws_bytes < pl.bytes) return fail(ctx, SMI_E_WORKSPACE, "workspace too small");
    Views w = smi::views(pl, ws);
    float *dcal = dcal_out ? dcal_out : w.dcal;
    std::unique_ptr<smi_state> stt;
    s = forward_common(ctx, &g, acq, SMI_JOB_GRAD, vp, rho, stf, dcal, nullptr, 0, nullptr, ws,
                       ws_bytes, st, stt);
    if (s != SMI_OK) return s;
    smi::StepCtx c{&stt->plan, &w, stf, st, false};
    configure(c, ctx, stt->plan);
    std::vector<int> grp;
    s = shot_groups(ctx, stt->plan.nshot, grp);
    if (s != SMI_OK) return s;
    for (size_t k = 0; k + 1 < grp.size(); ++k)
        HIPCHK(smi::residual(c, dcal, dobs, w.G, misfit ? misfit + k : nullptr, grp[k], grp[k + 1]),
               "residual");
    return run_reverse(ctx, stt.get(), w.G, grad_vp, grad_rho, nullptr, nullptr, nullptr, nullptr,
                       0, nullptr, st);
}

void smi_state_destroy(smi_state *state) { delete state; }

smi_status smi_poll_status(smi_ctx *ctx, void *hip_stream) {
    if (!ctx) return SMI_E_ARG;
    hipStream_t st = (hipStream_t)hip_stream;
    HIPCHK(hipStreamSynchronize(st), "sync");
    if (!ctx->last_ws) return SMI_OK;
    unsigned word = 0;
    HIPCHK(hipMemcpy(&word, ctx->last_ws, sizeof word, hipMemcpyDeviceToHost), "status read");
    unsigned zero = 0;
    HIPCHK(hipMemcpy(ctx->last_ws, &zero, sizeof zero, hipMemcpyHostToDevice), "status clear");
    if (word & 1u) return fail(ctx, SMI_E_NONFINITE, "model has non-finite, non-positive or out-of-range values");
    if (word & 2u) return fail(ctx, SMI_E_NONFINITE, "wavefield became non-finite");
    return SMI_OK;
}

smi_status smi_last_counts(const smi_ctx *ctx, double *fwd, double *adj, double *rec) {
    if (!ctx) return SMI_E_ARG;
    if (fwd) *fwd = ctx->cnt[0];
    if (adj) *adj = ctx->cnt[1];
    if (rec) *rec = ctx->cnt[2];
    return SMI_OK;
}

smi_status smi_born(smi_ctx *ctx, const smi_grid *grid, const smi_acq *acq, const float *vp,
                    const float *rho, const float *stf, const float *dkappa, float *ddata,
                    void *ws, size_t ws_bytes, void *hip_stream) {
    if (!ctx) return SMI_E_ARG;
    if (!grid || !acq) return fail(ctx, SMI_E_ARG, "grid / acq is NULL");
    if (!vp || !rho || !stf || !dkappa || !ddata)
        return fail(ctx, SMI_E_ARG, "vp, rho, stf, dkappa and ddata are required");
    if (!ws) return fail(ctx, SMI_E_WORKSPACE, "workspace is NULL");
    hipStream_t st = (hipStream_t)hip_stream;
    double vmin = 0, vmax = 0;
    smi_status s = speeds(ctx, grid, vp, ws, ws_bytes, st, vmin, vmax);
    if (s != SMI_OK) return s;
    Plan pl;
    s = smi::make_plan(grid, acq, SMI_JOB_BORN, vmin, vmax, pl, ctx->err);
    if (s != SMI_OK) return s;
    if (ws_bytes < pl.bytes) return fail(ctx, SMI_E_WORKSPACE, "workspace too small");
    Views w = smi::views(pl, ws);
    s = upload(ctx, pl, w, st);
    if (s != SMI_OK) return s;
    HIPCHK(smi::launch_model_prep(pl, w, vp, rho, st), "model prep");
    s = zero_fields(ctx, pl, w.f, st);
    if (s == SMI_OK) s = zero_fields(ctx, pl, w.q, st);
    if (s != SMI_OK) return s;
    smi::StepCtx c{&pl, &w, stf, st, false};
    configure(c, ctx, pl);
    c.plain = false;
    for (int it = 0; it < pl.g.nt; ++it) {
        HIPCHK(smi::fwd_step(c, it), "background step");
        HIPCHK(smi::src_taps(c, it, w.f.p, 1.f), "source");
        HIPCHK(smi::born_step(c, it, dkappa), "perturbation step");
        HIPCHK(smi::extract(c, it, ddata, w.q.p), "extract");
    }
    ctx->cnt[0] = 2 * pl.cnt_fwd;
    ctx->cnt[1] = ctx->cnt[2] = 0;
    ctx->bytes[0] = 2 * pl.bytes_fwd;
    ctx->bytes[1] = 0;
    ctx->last_ws = (void *)w.status;
    return SMI_OK;
}

smi_status smi_laplacian(smi_ctx *ctx, const smi_grid *grid, const float *in, float *out,
                         void *hip_stream) {
    if (!ctx) return SMI_E_ARG;
    if (!grid || !in || !out) return fail(ctx, SMI_E_ARG, "grid, in and out are required");
    if (in == out) return fail(ctx, SMI_E_ARG, "in and out must not alias");
    if ((grid->ndim != 2 && grid->ndim != 3) || grid->n1 < 1 || grid->n2 < 1 ||
        (grid->ndim == 3 && grid->n3 < 1) || !(grid->d1 > 0) || !(grid->d2 > 0) ||
        (grid->ndim == 3 && !(grid->d3 > 0)))
        return fail(ctx, SMI_E_ARG, "ndim must be 2 or 3 with positive sizes and spacings");
    HIPCHK(smi::launch_laplacian(grid, in, out, (hipStream_t)hip_stream), "laplacian");
    return SMI_OK;
}

smi_status smi_kernel_timing(smi_ctx *ctx, int which, double *avg_ms, double *avg_bytes,
                             int *nsamples) {
    if (!ctx || which < 0 || which > 3) return fail(ctx, SMI_E_ARG, "which must be 0, 1, 2 or 3");
    double ms = 0, by = 0;
    if (which == 3) {
        for (size_t k = 0; k < ctx->nrev; ++k) {
            hipError_t e = hipEventSynchronize(ctx->rev_events[2 * k + 1]);
            float t = 0.f;
            if (e == hipSuccess) e = hipEventElapsedTime(&t, ctx->rev_events[2 * k], ctx->rev_events[2 * k + 1]);
            if (e != hipSuccess) return hip_fail(ctx, e, "kernel timing");
            ms += t;
            by += ctx->rev_sample_bytes[k];
        }
        const double n = (double)ctx->nrev;
        if (avg_ms) *avg_ms = n > 0 ? ms / n : 0.0;
        if (avg_bytes) *avg_bytes = n > 0 ? by / n : 0.0;
        if (nsamples) *nsamples = (int)ctx->nrev;
        return SMI_OK;
    }
    for (size_t k = 0; k < ctx->nsample; ++k) {
        const bool one = ctx->sample_nk[k] == 1;
        if (one && which == 2) continue;          // a fused step has no second kernel
        hipEvent_t a = ctx->events[4 * k + (which == 2 ? 2 : 0)];
        hipEvent_t b = ctx->events[4 * k + (which == 1 || one ? 1 : 3)];
        hipError_t e = hipEventSynchronize(b);
        float t = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&t, a, b);
        if (e != hipSuccess) return hip_fail(ctx, e, "kernel timing");
        ms += t;
        by += ctx->sample_bytes[3 * k + which];
    }
    const double n = (double)ctx->nsample;
    if (avg_ms) *avg_ms = n > 0 ? ms / n : 0.0;
    if (avg_bytes) *avg_bytes = n > 0 ? by / n : 0.0;
    if (nsamples) *nsamples = (int)ctx->nsample;
    return SMI_OK;
}

smi_status smi_last_bytes(const smi_ctx *ctx, double *fwd_bytes, double *rev_bytes) {
    if (!ctx) return SMI_E_ARG;
    if (fwd_bytes) *fwd_bytes = ctx->bytes[0];
    if (rev_bytes) *rev_bytes = ctx->bytes[1];
    return SMI_OK;
}

}  // extern "C"
