// Host side of the C ABI declared in include/mt.h: validation, table
// building (cumulative counts, inverse-CDF guide, z-slab grid, float4 field),
// launch dispatch, hipGraph cache for the persistent form and the autotuner.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <limits>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "mt_internal.h"

// Workspace of mt_propagate_noalloc: a file-scope device array, so that the
// call allocates nothing.  Each device the library runs on holds its own copy
// until the process ends.
static __device__ __align__(256) unsigned char scratch[MT_NOALLOC_SCRATCH_BYTES];

namespace {

using mt::Tables;

thread_local std::string g_err;

int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define MT_HIP(call)                                                                     \
    do {                                                                                 \
        hipError_t e_ = (call);                                                          \
        if (e_ != hipSuccess)                                                            \
            return fail(MT_ERR_HIP, "%s failed: %s", #call, hipGetErrorString(e_));      \
    } while (0)

// A device buffer owned by the library.
struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    // Grow to at least n bytes (contents not preserved).
    int ensure(size_t n) {
        if (n <= bytes && p) return MT_OK;
        release();
        if (n == 0) n = 16;
        if (hipMalloc(&p, n) != hipSuccess) {
            (void)hipGetLastError();
            return fail(MT_ERR_OOM, "device allocation of %zu bytes failed", n);
        }
        bytes = n;
        return MT_OK;
    }
    int upload(const void *src, size_t n) {
        int rc = ensure(n);
        if (rc) return rc;
        if (n && hipMemcpy(p, src, n, hipMemcpyHostToDevice) != hipSuccess)
            return fail(MT_ERR_HIP, "hipMemcpy of %zu bytes failed", n);
        return MT_OK;
    }
};

struct GraphEntry {
    std::vector<unsigned char> key;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

struct TuneEntry {
    std::vector<unsigned char> key;
    int block = 0, compact = 0;
};

struct State {
    std::mutex mu;
    int device = -1;
    bool hist_loaded = false, geom_loaded = false;
    int n_mat = 0, n_pbin = 0;
    int64_t version = 0;  // bumped on every table change
    DevBuf cdf, guide, totals, edges2, alias, blk, grid, nodes;
    DevBuf box4, material, bfield, magnet, slab_z, slab_mask;
    DevBuf map;
    DevBuf queue, partial, scratch, gs_lane, lists;
    Tables T{};
    int max_material = -1;
    hipStream_t cap_stream = nullptr;
    std::vector<GraphEntry> graphs;
    std::vector<TuneEntry> tuned;
    int cu_count = 0;
    // tuning switches (mt_set_option); none changes a result bit
    int opt_guide_bits = 0;          // 0: automatic
    int opt_adjoint_block = 64;
    int opt_adjoint_lds_history = 0;
};

State g;

// Device address of the workspace array `scratch` on each device (looked up
// once per device; the array's name is no device address in host code).
// Layout: the persistent form's work counter at byte 0, the tally partial
// sums from byte kNoallocCounterBytes.
constexpr size_t kNoallocCounterBytes = 256;
constexpr int kMaxDevices = 64;
void *noalloc_addr[kMaxDevices] = {};

int ensure_device() {
    if (g.device < 0) {
        int d = 0;
        if (hipGetDevice(&d) != hipSuccess) return fail(MT_ERR_HIP, "no HIP device is available");
        g.device = d;
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, d) == hipSuccess) g.cu_count = prop.multiProcessorCount;
        if (g.cu_count <= 0) g.cu_count = 256;
    }
    return MT_OK;
}

void drop_graphs() {
    for (auto &e : g.graphs) {
        if (e.exec) (void)hipGraphExecDestroy(e.exec);
        if (e.graph) (void)hipGraphDestroy(e.graph);
    }
    g.graphs.clear();
}

// Captured graphs hold the addresses of the workspace buffers (the
// persistent queue and the tally partials) baked into
// their kernel nodes, and their cache key does not: a graph whose workspace
// has been reallocated since its capture must never be replayed.  Growing a
// buffer frees the old one (hipFree waits for the device), then every cached
// graph is dropped.
struct WorkspaceAddr {
    void *queue, *partial, *lists;
};

WorkspaceAddr workspace_addr() { return {g.queue.p, g.partial.p, g.lists.p}; }

void drop_graphs_if_moved(const WorkspaceAddr &before) {
    if (before.queue != g.queue.p || before.partial != g.partial.p || before.lists != g.lists.p)
        drop_graphs();
}

void tables_changed() {
    ++g.version;
    drop_graphs();
    g.tuned.clear();
}

// LDS layout of the staged tables (depends on histogram and geometry sizes).
void relayout() {
    mt::LdsLayout L{};
    int off = 0;
    auto take = [&](int bytes, int align) {
        off = (off + align - 1) / align * align;
        const int o = off;
        off += bytes;
        return o;
    };
    const int P = g.T.hist.n_pbin, nb = g.T.geom.n_box, ns = g.T.geom.n_slab;
    const int np = g.T.geom.n_poly;
    const int nh = g.T.hist.n_mat * P;
    L.off_e2 = take(8 * (P + 1), 16);
    L.off_tot = take(4 * nh, 16);
    L.off_box4 = take(np > 0 ? 0 : 32 * nb, 16);
    L.off_blk = take(8 * mt::kBlockRec * np, 16);
    L.off_grid = take(np > 0 ? 8 * g.T.geom.gx * g.T.geom.gy * g.T.geom.gz : 0, 16);
    L.off_bf = take(16 * nb, 16);
    L.off_mat = take(4 * nb, 16);
    L.off_mag = take(4 * nb, 16);
    L.off_slabz = take(8 * (ns + 1), 16);
    L.off_slabm = take(8 * ns, 16);
    L.bytes = (off + 15) / 16 * 16;
    g.T.lds = L;
}

std::vector<unsigned char> make_key(const void *a, size_t na, const void *b = nullptr,
                                    size_t nb = 0) {
    std::vector<unsigned char> k(na + nb + sizeof(int64_t));
    std::memcpy(k.data(), a, na);
    if (nb) std::memcpy(k.data() + na, b, nb);
    std::memcpy(k.data() + na + nb, &g.version, sizeof(int64_t));
    return k;
}

// Validated, device-side description of one propagate call.
struct Call {
    mt::DevRun R{};
    mt::DevIO io{};
    int block = 256;
    int compact = 128;
    int n_variants = 1;
    int64_t n = 0, lanes = 0;
};

int validate(const mt_params *p, int64_t n, const mt_muons *in, const mt_muons *out,
             const mt_result *res, bool backward, Call &c) {
    if (!g.hist_loaded || !g.geom_loaded)
        return fail(MT_ERR_NOT_LOADED, "histograms and geometry must be loaded before propagating");
    if (!p) return fail(MT_ERR_INVALID_ARG, "params is NULL");
    if (n < 0) return fail(MT_ERR_INVALID_ARG, "n = %lld is negative", (long long)n);
    if (p->n_variants < 1) return fail(MT_ERR_INVALID_ARG, "n_variants must be >= 1");
    if (n > 0 && p->n_variants > std::numeric_limits<int64_t>::max() / n)
        return fail(MT_ERR_INVALID_ARG, "n_variants * n overflows");
    if (!(p->step_m > 0.0) || !std::isfinite(p->step_m))
        return fail(MT_ERR_INVALID_ARG, "step_m must be finite and > 0");
    if (p->max_steps < 0) return fail(MT_ERR_INVALID_ARG, "max_steps must be >= 0");
    if (!(p->p_min >= 0.0) || !std::isfinite(p->p_min))
        return fail(MT_ERR_INVALID_ARG, "p_min must be finite and >= 0");
    if (p->mode != MT_MODE_PLAIN && p->mode != MT_MODE_PERSISTENT &&
        p->mode != MT_MODE_VARIANT_WAVES)
        return fail(MT_ERR_INVALID_ARG, "unknown mode %d", p->mode);
    if (p->mode == MT_MODE_VARIANT_WAVES && p->n_trace > 0 && p->trace_steps > 0)
        return fail(MT_ERR_INVALID_ARG, "MT_MODE_VARIANT_WAVES does not record traces");
    if (p->block != 0 && (p->block < 64 || p->block > 1024 || p->block % 64 != 0))
        return fail(MT_ERR_INVALID_ARG, "block must be a multiple of 64 in [64, 1024]");
    if (p->compact_every < 0) return fail(MT_ERR_INVALID_ARG, "compact_every must be >= 0");
    if (p->sampler != MT_SAMPLER_CDF && p->sampler != MT_SAMPLER_ALIAS)
        return fail(MT_ERR_INVALID_ARG, "unknown sampler %d", p->sampler);
    if (p->interp != MT_INTERP_TRILINEAR && p->interp != MT_INTERP_NEAREST)
        return fail(MT_ERR_INVALID_ARG, "unknown interp %d", p->interp);
    if (p->stage_field != 0 && p->stage_field != 1)
        return fail(MT_ERR_INVALID_ARG, "stage_field must be 0 or 1");
    if (p->ckpt_every != 0 && (p->interp != MT_INTERP_TRILINEAR || p->stage_field != 0))
        return fail(MT_ERR_INVALID_ARG, "the differentiable form (ckpt_every) supports the "
                                        "held trilinear field only");
    if (g.T.geom.n_poly > 0 && (p->ckpt_every != 0 || p->stage_field != 0))
        return fail(MT_ERR_INVALID_ARG, "convex-block geometry supports neither the "
                                        "differentiable form nor stage_field = 1");
    if (p->ckpt_every != 0 && p->ckpt_every != mt::kCkptEvery)
        return fail(MT_ERR_INVALID_ARG, "ckpt_every must be 0 or %d", mt::kCkptEvery);
    if (p->ckpt_every != 0) {
        if (!p->ckpt || !p->tape)
            return fail(MT_ERR_INVALID_ARG, "checkpointing needs both ckpt and tape buffers");
        if (p->mode != MT_MODE_PLAIN)
            return fail(MT_ERR_INVALID_ARG, "checkpointing is only supported in MT_MODE_PLAIN");
    }
    if (backward && p->ckpt_every == 0)
        return fail(MT_ERR_INVALID_ARG, "the backward pass needs the checkpointed forward's "
                                        "ckpt_every, ckpt and tape");
    if (p->n_trace < 0 || p->trace_steps < 0)
        return fail(MT_ERR_INVALID_ARG, "n_trace and trace_steps must be >= 0");
    if (p->n_trace > 0 && p->trace_steps > 0 && !p->trace)
        return fail(MT_ERR_INVALID_ARG, "trace buffer is NULL");
    if (p->scales && g.T.geom.n_mag == 0)
        return fail(MT_ERR_SHAPE, "scales given but the geometry has no magnets");
    if (p->tally && !(p->r_scale > 0.0))
        return fail(MT_ERR_INVALID_ARG, "tally needs r_scale > 0");
    if (g.max_material >= g.n_mat)
        return fail(MT_ERR_SHAPE, "geometry uses material %d but histograms hold %d materials",
                    g.max_material, g.n_mat);
    if (n > 0) {
        if (!in || !in->x || !in->y || !in->z || !in->px || !in->py || !in->pz || !in->q)
            return fail(MT_ERR_INVALID_ARG, "input muon pointers must be non-NULL");
        if (!res || !res->status || !res->n_steps || !res->volume)
            return fail(MT_ERR_INVALID_ARG, "result pointers must be non-NULL");
        if (!backward && (!out || !out->x || !out->y || !out->z || !out->px || !out->py ||
                          !out->pz))
            return fail(MT_ERR_INVALID_ARG, "output muon pointers must be non-NULL");
    }
    c.n = n;
    c.n_variants = p->n_variants;
    c.lanes = n * p->n_variants;
    c.block = p->block ? p->block : 256;
    c.compact = p->compact_every ? p->compact_every : 128;
    mt::DevRun &R = c.R;
    R.h = p->step_m;
    R.sampler = p->sampler;
    R.interp = p->interp;
    R.stage_field = p->stage_field;
    // lanes sharing a random stream in the variant-wave form: the largest
    // power of two dividing n_variants, at most one wavefront
    R.share_shift = 0;
    while (R.share_shift < 6 && p->n_variants % (2 << R.share_shift) == 0) ++R.share_shift;
    R.pmin2 = p->p_min * p->p_min;
    R.max_steps = p->max_steps;
    R.key0 = (uint32_t)p->seed;
    R.key1 = (uint32_t)(p->seed >> 32);
    R.n = n;
    R.lanes = c.lanes;
    R.scales = p->scales;
    R.ckpt = p->ckpt_every ? p->ckpt : nullptr;
    R.tape = p->ckpt_every ? p->tape : nullptr;
    R.trace = p->trace;
    R.n_trace = (p->trace && p->trace_steps > 0) ? p->n_trace : 0;
    R.trace_steps = p->trace_steps;
    mt::DevIO &io = c.io;
    if (n > 0) {
        io.x = in->x; io.y = in->y; io.z = in->z;
        io.px = in->px; io.py = in->py; io.pz = in->pz; io.q = in->q;
        if (out) {
            io.ox = out->x; io.oy = out->y; io.oz = out->z;
            io.opx = out->px; io.opy = out->py; io.opz = out->pz;
        }
        io.status = res->status; io.n_steps = res->n_steps; io.volume = res->volume;
    }
    return MT_OK;
}

int n_part_blocks(int64_t n) {
    int64_t nb = (n + 4095) / 4096;
    return (int)std::max<int64_t>(1, std::min<int64_t>(nb, 256));
}

// Passes of the compacting form: steps per pass S (compact_every, at least
// (max_steps + 1) / kMaxPasses) and their number.  Passes 0 .. P-2 end at
// (p + 1) S <= max_steps, the last one runs to the step cap.
constexpr int kMaxPasses = 64;

void pass_plan(int max_steps, int compact, int *S, int *P) {
    const int64_t span = (int64_t)max_steps + 1;
    int64_t st = std::max<int64_t>(compact, (span + kMaxPasses - 1) / kMaxPasses);
    *S = (int)std::min<int64_t>(st, span);
    *P = (int)((span + *S - 1) / *S);
}

// Enqueue transport (+ tallies) on stream s.  `counters` holds kMaxPasses
// 64-bit survivor counts, one per pass of the compacting form (cleared by a
// kernel here, never by a memset node in a captured graph); `lists` the two
// lists of survivor slots (lanes int64 each), or nullptr: then the
// compacting form runs the whole step range as one pass.
int enqueue_ws(const mt_params *p, const Call &c, hipStream_t s, unsigned long long *counters,
               char *lists, double *partial) {
    if (p->mode == MT_MODE_PERSISTENT) {
        int S = 0, P = 1;
        pass_plan(p->max_steps, lists ? c.compact : p->max_steps + 1, &S, &P);
        if (P > 1)
            MT_HIP(mt::launch_queue_reset(counters, reinterpret_cast<double *>(counters), P, s));
        for (int pp = 0; pp < P; ++pp) {
            mt::PassArgs a{};
            a.k_begin = pp * S;
            a.max_steps = p->max_steps;
            mt::DevRun r = c.R;                 // the pass ends at its own step cap
            if (pp < P - 1) r.max_steps = (pp + 1) * S;
            a.n_in = pp == 0 ? nullptr : counters + pp - 1;
            a.n_out = counters + pp;
            if (P > 1) {
                int64_t *l = reinterpret_cast<int64_t *>(lists);
                if (pp > 0) a.in = l + ((pp - 1) & 1) * c.lanes;
                a.out = l + (pp & 1) * c.lanes;
            }
            MT_HIP(mt::launch_pass(g.T, r, c.io, c.block, a, s));
        }
    } else if (p->mode == MT_MODE_VARIANT_WAVES) {
        MT_HIP(mt::launch_variant_waves(g.T, c.R, c.io, c.block, s));
    } else {
        MT_HIP(mt::launch_plain(g.T, c.R, c.io, c.block, s));
    }
    if (p->tally) {
        const int nb = n_part_blocks(c.n);
        MT_HIP(mt::launch_tally(c.io, c.n, c.n_variants, p->z_det, p->r_ap, p->r_scale, partial,
                                nb, p->tally, s));
    }
    return MT_OK;
}

int enqueue(const mt_params *p, const Call &c, hipStream_t s) {
    int S = 0, P = 1;
    if (p->mode == MT_MODE_PERSISTENT) pass_plan(p->max_steps, c.compact, &S, &P);
    return enqueue_ws(p, c, s, reinterpret_cast<unsigned long long *>(g.queue.p),
                      P > 1 ? reinterpret_cast<char *>(g.lists.p) : nullptr,
                      reinterpret_cast<double *>(g.partial.p));
}

int prepare_workspace(const mt_params *p, const Call &c) {
    int rc = g.queue.ensure(kMaxPasses * sizeof(unsigned long long));
    if (rc) return rc;
    if (p->mode == MT_MODE_PERSISTENT) {
        int S = 0, P = 1;
        pass_plan(p->max_steps, c.compact, &S, &P);
        if (P > 1 && (rc = g.lists.ensure(2 * (size_t)c.lanes * sizeof(int64_t)))) return rc;
    }
    if (p->tally) {
        rc = g.partial.ensure((size_t)n_part_blocks(c.n) * c.n_variants * 3 * sizeof(double));
        if (rc) return rc;
    }
    return MT_OK;
}

const TuneEntry *find_tuned(const std::vector<unsigned char> &key) {
    for (auto &t : g.tuned)
        if (t.key == key) return &t;
    return nullptr;
}

std::vector<unsigned char> tune_key(const mt_params *p, int64_t n) {
    struct K {
        int64_t n;
        int32_t nv, max_steps, has_map, mode;
        double step, pmin;
        int32_t sampler, interp, stage_field, blocks;   // the kernel variant
    } k;
    std::memset(&k, 0, sizeof(k));
    k.n = n;
    k.nv = p->n_variants;
    k.max_steps = p->max_steps;
    k.has_map = g.T.field.map != nullptr;
    k.mode = p->mode;
    k.step = p->step_m;
    k.pmin = p->p_min;
    k.sampler = p->sampler;
    k.interp = p->interp;
    k.stage_field = p->stage_field;
    k.blocks = g.T.geom.n_poly > 0;
    return make_key(&k, sizeof(k));
}

int propagate_impl(const mt_params *p, int64_t n, const mt_muons *in, mt_muons *out,
                   mt_result *res, void *hip_stream, int force_block, int force_compact,
                   bool allow_graph) {
    Call c;
    int rc = validate(p, n, in, out, res, false, c);
    if (rc) return rc;
    hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
    const WorkspaceAddr ws = workspace_addr();
    if (c.lanes == 0) {
        if (p->tally) {
            rc = g.queue.ensure(sizeof(unsigned long long));
            drop_graphs_if_moved(ws);
            if (rc) return rc;
            MT_HIP(mt::launch_queue_reset(reinterpret_cast<unsigned long long *>(g.queue.p),
                                          p->tally, (int64_t)p->n_variants * 3, s));
        }
        return MT_OK;
    }
    if (p->mode != MT_MODE_PLAIN && p->block == 0 && p->compact_every == 0) {
        if (const TuneEntry *t = find_tuned(tune_key(p, n))) {
            c.block = t->block;
            c.compact = t->compact;
        }
    }
    if (force_block) c.block = force_block;
    if (force_compact) c.compact = force_compact;
    rc = prepare_workspace(p, c);
    drop_graphs_if_moved(ws);
    if (rc) return rc;
    if (allow_graph && p->use_graph && p->mode != MT_MODE_PLAIN) {
        struct K {
            mt_params p;
            int64_t n;
            mt_muons in, out;
            mt_result res;
            int block, compact;
        } k;
        std::memset(&k, 0, sizeof(k));
        k.p = *p;
        k.n = n;
        k.in = *in;
        k.out = *out;
        k.res = *res;
        k.block = c.block;
        k.compact = c.compact;
        std::vector<unsigned char> key = make_key(&k, sizeof(k));
        GraphEntry *hit = nullptr;
        for (auto &e : g.graphs)
            if (e.key == key) hit = &e;
        if (!hit) {
            if (!g.cap_stream) MT_HIP(hipStreamCreateWithFlags(&g.cap_stream, hipStreamNonBlocking));
            if (g.graphs.size() >= 8) {
                GraphEntry &old = g.graphs.front();
                if (old.exec) (void)hipGraphExecDestroy(old.exec);
                if (old.graph) (void)hipGraphDestroy(old.graph);
                g.graphs.erase(g.graphs.begin());
            }
            GraphEntry e;
            e.key = key;
            MT_HIP(hipStreamBeginCapture(g.cap_stream, hipStreamCaptureModeThreadLocal));
            int erc = enqueue(p, c, g.cap_stream);
            hipGraph_t graph = nullptr;
            hipError_t ec = hipStreamEndCapture(g.cap_stream, &graph);
            if (erc) {
                if (graph) (void)hipGraphDestroy(graph);
                return erc;
            }
            if (ec != hipSuccess)
                return fail(MT_ERR_HIP, "hipStreamEndCapture failed: %s", hipGetErrorString(ec));
            e.graph = graph;
            MT_HIP(hipGraphInstantiate(&e.exec, graph, nullptr, nullptr, 0));
            g.graphs.push_back(e);
            hit = &g.graphs.back();
        }
        MT_HIP(hipGraphLaunch(hit->exec, s));
        return MT_OK;
    }
    return enqueue(p, c, s);
}

}  // namespace

extern "C" {

// Walker alias table of one histogram (the Prob/Alias tables of the paper's
// alias method), in exact integer arithmetic.  Column c starts with weight
// K * count[c] against a capacity of T = total; LIFO worklists of the
// columns under capacity ("under") and at or over it ("over"), each filled
// in ascending order, are paired off: the top "under" column keeps its
// weight as its threshold and takes the top "over" column as its alias,
// which loses the difference to T and moves to "under" once below T.
// Columns still "over" at the end hold exactly T and alias themselves.
// Entry c of the result is (x_split, alias): the draw keeps cell c when the
// 24-bit threshold word x is below x_split = ceil(threshold * 2^24 / T),
// which is the same as floor(x * T / 2^24) < threshold.
static void alias_table(const uint32_t *count, int64_t K, uint64_t T, uint2 *out) {
    std::vector<uint64_t> wt((size_t)K);
    std::vector<int32_t> under, over;
    under.reserve((size_t)K);
    over.reserve((size_t)K);
    for (int64_t c = 0; c < K; ++c) {
        wt[(size_t)c] = (uint64_t)K * count[c];
        (wt[(size_t)c] < T ? under : over).push_back((int32_t)c);
    }
    auto split_of = [T](uint64_t thr) { return (uint32_t)(((thr << 24) + T - 1) / T); };
    while (!under.empty() && !over.empty()) {
        const int32_t u = under.back();
        under.pop_back();
        const int32_t o = over.back();
        out[u] = make_uint2(split_of(wt[(size_t)u]), (uint32_t)o);
        wt[(size_t)o] -= T - wt[(size_t)u];
        if (wt[(size_t)o] < T) {
            over.pop_back();
            under.push_back(o);
        }
    }
    for (int32_t o : over) out[o] = make_uint2(1u << 24, (uint32_t)o);
}

int mt_load_histograms(int32_t n_mat, int32_t n_pbin, const double *p_edges, int32_t n_loss,
                       double loss_lo, double loss_hi, int32_t n_scat, double scat_lo,
                       double scat_hi, const uint32_t *counts) {
    return mt_load_histograms_ex(n_mat, n_pbin, p_edges, n_loss, loss_lo, loss_hi, n_scat,
                                 scat_lo, scat_hi, counts, 0);
}

int mt_optimal_edges(const double *p_probe, const double *phi, int32_t n_probe, double eps,
                     double *edges, int32_t max_edges, int32_t *n_edges) {
    if (!p_probe || !phi || !edges || !n_edges)
        return fail(MT_ERR_INVALID_ARG, "pointers must be non-NULL");
    if (n_probe < 2) return fail(MT_ERR_INVALID_ARG, "need at least two probe momenta");
    if (!(eps >= 0.0) || !std::isfinite(eps))
        return fail(MT_ERR_INVALID_ARG, "eps must be finite and >= 0");
    for (int32_t j = 0; j < n_probe; ++j) {
        if (!std::isfinite(p_probe[j]) || !std::isfinite(phi[j]))
            return fail(MT_ERR_INVALID_ARG, "probe %d: values must be finite", j);
        if (j > 0 && !(p_probe[j] > p_probe[j - 1]))
            return fail(MT_ERR_INVALID_ARG, "probe momenta must be strictly ascending");
    }
    int32_t count = 0;
    auto put = [&](double v) {
        if (count >= max_edges) return false;
        edges[count++] = v;
        return true;
    };
    if (!put(p_probe[0])) return fail(MT_ERR_LIMIT, "max_edges = %d is too small", max_edges);
    int32_t start = 0;
    while (start < n_probe - 1) {
        const double ref = phi[start];
        int32_t next = start + 1;
        while (next < n_probe - 1 && std::fabs(phi[next] - ref) <= eps) ++next;
        if (!put(p_probe[next])) return fail(MT_ERR_LIMIT, "max_edges = %d is too small", max_edges);
        start = next;
    }
    *n_edges = count;
    return MT_OK;
}

int mt_load_histograms_ex(int32_t n_mat, int32_t n_pbin, const double *p_edges, int32_t n_loss,
                          double loss_lo, double loss_hi, int32_t n_scat, double scat_lo,
                          double scat_hi, const uint32_t *counts, int32_t axes) {
    std::lock_guard<std::mutex> lk(g.mu);
    int rc = MT_OK;
    if (axes & ~(MT_AXIS_LOG_LOSS | MT_AXIS_LOG_SCAT))
        return fail(MT_ERR_INVALID_ARG, "unknown axis flags %d", axes);
    const bool log_l = (axes & MT_AXIS_LOG_LOSS) != 0, log_s = (axes & MT_AXIS_LOG_SCAT) != 0;
    if ((log_l && !(loss_lo > 0.0)) || (log_s && !(scat_lo > 0.0)))
        return fail(MT_ERR_INVALID_ARG, "a logarithmic axis needs lo > 0");
    if (n_mat < 1 || n_pbin < 1 || n_loss < 1 || n_scat < 1)
        return fail(MT_ERR_INVALID_ARG, "n_mat, n_pbin, n_loss and n_scat must be >= 1");
    if (!p_edges || !counts) return fail(MT_ERR_INVALID_ARG, "p_edges and counts must be non-NULL");
    if (n_pbin > MT_MAX_PBINS)
        return fail(MT_ERR_LIMIT, "n_pbin = %d exceeds %d", n_pbin, MT_MAX_PBINS);
    const int64_t K = (int64_t)n_loss * n_scat;
    if (K > MT_MAX_CELLS)
        return fail(MT_ERR_LIMIT, "n_loss * n_scat = %lld exceeds %d", (long long)K, MT_MAX_CELLS);
    if (!(loss_hi > loss_lo) || !(scat_hi > scat_lo) || !std::isfinite(loss_lo) ||
        !std::isfinite(loss_hi) || !std::isfinite(scat_lo) || !std::isfinite(scat_hi))
        return fail(MT_ERR_INVALID_ARG, "axis ranges must be finite with hi > lo");
    for (int i = 0; i <= n_pbin; ++i) {
        if (!std::isfinite(p_edges[i]) || !(p_edges[i] > 0.0))
            return fail(MT_ERR_INVALID_ARG, "p_edges[%d] must be finite and > 0", i);
        if (i > 0 && !(p_edges[i] > p_edges[i - 1]))
            return fail(MT_ERR_INVALID_ARG, "p_edges must be strictly ascending (index %d)", i);
    }
    const int64_t nh = (int64_t)n_mat * n_pbin;
    if (nh > MT_MAX_HISTS)
        return fail(MT_ERR_LIMIT, "n_mat * n_pbin = %lld exceeds %d", (long long)nh, MT_MAX_HISTS);
    // Guide resolution: about one guide entry per cell, at most 2^16.
    int gbits = 1;
    while (gbits < 16 && ((int64_t)1 << gbits) < K) ++gbits;
    if (gbits > 1) --gbits;
    if (g.opt_guide_bits > 0) gbits = g.opt_guide_bits;
    const int64_t G = (int64_t)1 << gbits;
    std::vector<uint32_t> cdf((size_t)(nh * K)), totals((size_t)nh);
    std::vector<uint2> guide((size_t)(nh * G));
    std::vector<uint2> alias((size_t)(nh * K));
    for (int64_t h = 0; h < nh; ++h) {
        uint64_t acc = 0;
        const uint32_t *src = counts + h * K;
        uint32_t *C = cdf.data() + h * K;
        for (int64_t c = 0; c < K; ++c) {
            acc += src[c];
            if (acc > 0xFFFFFFFFull)
                return fail(MT_ERR_EMPTY_HIST, "histogram %lld: total count does not fit in 32 bits",
                            (long long)h);
            C[c] = (uint32_t)acc;
        }
        if (acc == 0)
            return fail(MT_ERR_EMPTY_HIST, "histogram %lld (material %lld, bin %lld) is empty",
                        (long long)h, (long long)(h / n_pbin), (long long)(h % n_pbin));
        const uint64_t T = acc;
        totals[(size_t)h] = (uint32_t)T;
        auto cell_of = [&](uint32_t t) {
            return (uint32_t)(std::upper_bound(C, C + K, t) - C);
        };
        uint2 *Gd = guide.data() + h * G;
        for (int64_t gi = 0; gi < G; ++gi) {
            const uint64_t w_lo = (uint64_t)gi << (32 - gbits);
            const uint64_t w_hi = (((uint64_t)gi + 1) << (32 - gbits)) - 1;
            const uint32_t lo = cell_of((uint32_t)((w_lo * T) >> 32));
            const uint32_t hi = cell_of((uint32_t)((w_hi * T) >> 32));
            Gd[gi] = make_uint2(lo | (hi << 16), C[lo]);
        }
        alias_table(src, K, T, alias.data() + h * K);
    }
    std::vector<double> e2((size_t)n_pbin + 1);
    for (int i = 0; i <= n_pbin; ++i) e2[i] = p_edges[i] * p_edges[i];
    if ((rc = ensure_device())) return rc;
    if ((rc = g.cdf.upload(cdf.data(), cdf.size() * 4))) return rc;
    if ((rc = g.guide.upload(guide.data(), guide.size() * sizeof(uint2)))) return rc;
    if ((rc = g.totals.upload(totals.data(), totals.size() * 4))) return rc;
    if ((rc = g.edges2.upload(e2.data(), e2.size() * 8))) return rc;
    if ((rc = g.alias.upload(alias.data(), alias.size() * sizeof(uint2)))) return rc;
    mt::DevHist &H = g.T.hist;
    H.cdf = reinterpret_cast<const uint32_t *>(g.cdf.p);
    H.guide = reinterpret_cast<const uint2 *>(g.guide.p);
    H.totals = reinterpret_cast<const uint32_t *>(g.totals.p);
    H.edges2 = reinterpret_cast<const double *>(g.edges2.p);
    H.alias = reinterpret_cast<const uint2 *>(g.alias.p);
    H.n_mat = n_mat;
    H.n_pbin = n_pbin;
    H.n_loss = n_loss;
    H.n_scat = n_scat;
    H.n_cells = (int32_t)K;
    H.gbits = gbits;
    H.nscat_magic = 0xFFFFFFFFu / (uint32_t)n_scat;
    // axis origin and bin width in the axis' own units (log10 on a log axis)
    const double l0 = log_l ? std::log10(loss_lo) : loss_lo, l1 = log_l ? std::log10(loss_hi) : loss_hi;
    const double s0 = log_s ? std::log10(scat_lo) : scat_lo, s1 = log_s ? std::log10(scat_hi) : scat_hi;
    H.loss_lo = (float)l0;
    H.loss_w = (float)((l1 - l0) / n_loss);
    H.scat_lo = (float)s0;
    H.scat_w = (float)((s1 - s0) / n_scat);
    H.log_loss = log_l ? 1 : 0;
    H.log_scat = log_s ? 1 : 0;
    g.n_mat = n_mat;
    g.n_pbin = n_pbin;
    g.hist_loaded = true;
    relayout();
    tables_changed();
    return MT_OK;
}

int mt_load_geometry(int32_t n_box, const double *box, const int32_t *material, const float *b_box,
                     const int32_t *magnet, int32_t n_mag, const double *world) {
    std::lock_guard<std::mutex> lk(g.mu);
    int rc = MT_OK;
    if (n_box < 0 || n_box > MT_MAX_BOXES)
        return fail(n_box < 0 ? MT_ERR_INVALID_ARG : MT_ERR_LIMIT, "n_box = %d not in [0, %d]",
                    n_box, MT_MAX_BOXES);
    if (n_mag < 0 || n_mag > MT_MAX_MAGNETS)
        return fail(n_mag < 0 ? MT_ERR_INVALID_ARG : MT_ERR_LIMIT, "n_mag = %d not in [0, %d]",
                    n_mag, MT_MAX_MAGNETS);
    if (!world) return fail(MT_ERR_INVALID_ARG, "world must be non-NULL");
    if (n_box > 0 && (!box || !material))
        return fail(MT_ERR_INVALID_ARG, "box and material must be non-NULL");
    for (int a = 0; a < 3; ++a)
        if (std::isnan(world[a])) return fail(MT_ERR_INVALID_ARG, "world[%d] is NaN", a);
    std::vector<double> box4((size_t)4 * n_box);
    std::vector<float4> bf((size_t)n_box);
    std::vector<int32_t> mat((size_t)n_box), mag((size_t)n_box);
    std::vector<double> zs;
    int max_mat = -1;
    for (int b = 0; b < n_box; ++b) {
        const double *bx = box + 6 * b;
        for (int a = 0; a < 3; ++a)
            if (!std::isfinite(bx[2 * a]) || !std::isfinite(bx[2 * a + 1]) || !(bx[2 * a] < bx[2 * a + 1]))
                return fail(MT_ERR_INVALID_ARG, "box %d: bounds must be finite with lo < hi", b);
        box4[4 * b + 0] = bx[0];
        box4[4 * b + 1] = bx[1];
        box4[4 * b + 2] = bx[2];
        box4[4 * b + 3] = bx[3];
        zs.push_back(bx[4]);
        zs.push_back(bx[5]);
        if (material[b] < -1) return fail(MT_ERR_INVALID_ARG, "material[%d] < -1", b);
        mat[b] = material[b];
        max_mat = std::max(max_mat, material[b]);
        const int m = magnet ? magnet[b] : -1;
        if (m < -1 || m >= n_mag)
            return fail(MT_ERR_INVALID_ARG, "magnet[%d] = %d not in [-1, n_mag)", b, m);
        mag[b] = m;
        bf[b] = b_box ? make_float4(b_box[3 * b], b_box[3 * b + 1], b_box[3 * b + 2], 0.f)
                      : make_float4(0.f, 0.f, 0.f, 0.f);
    }
    bool disjoint = true;
    for (int a = 0; a < n_box && disjoint; ++a)
        for (int b = a + 1; b < n_box && disjoint; ++b) {
            bool overlap = true;
            for (int ax = 0; ax < 3; ++ax)
                overlap = overlap && box[6 * a + 2 * ax] < box[6 * b + 2 * ax + 1] &&
                          box[6 * b + 2 * ax] < box[6 * a + 2 * ax + 1];
            if (overlap) disjoint = false;
        }
    std::sort(zs.begin(), zs.end());
    zs.erase(std::unique(zs.begin(), zs.end()), zs.end());
    std::vector<double> slab_z;
    slab_z.push_back(-std::numeric_limits<double>::infinity());
    for (double z : zs) slab_z.push_back(z);
    slab_z.push_back(std::numeric_limits<double>::infinity());
    const int n_slab = (int)slab_z.size() - 1;
    std::vector<uint64_t> mask((size_t)n_slab, 0ull);
    for (int s = 0; s < n_slab; ++s)
        for (int b = 0; b < n_box; ++b)
            if (box[6 * b + 4] <= slab_z[s] && slab_z[s + 1] <= box[6 * b + 5])
                mask[s] |= 1ull << b;
    if ((rc = ensure_device())) return rc;
    if ((rc = g.box4.upload(box4.data(), box4.size() * 8))) return rc;
    if ((rc = g.bfield.upload(bf.data(), bf.size() * 16))) return rc;
    if ((rc = g.material.upload(mat.data(), mat.size() * 4))) return rc;
    if ((rc = g.magnet.upload(mag.data(), mag.size() * 4))) return rc;
    if ((rc = g.slab_z.upload(slab_z.data(), slab_z.size() * 8))) return rc;
    if ((rc = g.slab_mask.upload(mask.data(), mask.size() * 8))) return rc;
    mt::DevGeom &G = g.T.geom;
    G.n_box = n_box;
    G.n_poly = 0;
    G.n_slab = n_slab;
    G.n_mag = n_mag;
    G.disjoint = disjoint ? 1 : 0;
    G.box4 = reinterpret_cast<const double *>(g.box4.p);
    G.material = reinterpret_cast<const int32_t *>(g.material.p);
    G.bfield = reinterpret_cast<const float4 *>(g.bfield.p);
    G.magnet = reinterpret_cast<const int32_t *>(g.magnet.p);
    G.slab_z = reinterpret_cast<const double *>(g.slab_z.p);
    G.slab_mask = reinterpret_cast<const uint64_t *>(g.slab_mask.p);
    G.x_max = world[0];
    G.y_max = world[1];
    G.z_max = world[2];
    g.max_material = max_mat;
    g.geom_loaded = true;
    relayout();
    tables_changed();
    return MT_OK;
}

// Convex blocks (Section "Simulation", item 1).  Each block is stored as
// kBlockRec doubles: z_lo, z_hi, 1 / (z_hi - z_lo), m (below), the quad at
// z_lo as (x, y) x 4, and the per-vertex change (top - bottom) x 4, so that
// the slice at height z is bottom + t (top - bottom), t = (z - z_lo) / (z_hi -
// z_lo).
//
// m = sigma tau lets a lane keep the block it found at the previous step:
// a point whose edge products S_i of block b's slice all satisfy
// sigma S_i > tau (sigma = +-1 the vertex order) is inside b and, when m is
// not 0, inside no block of lower index, so the lookup's answer is b
// without testing the others.  m is not 0 only if every lower-index block
// whose z range meets b's lies, over the common z range, on the outer side
// of one edge line of b up to tau / 2: then any point of it has
// sigma S_i <= tau for that edge (S_i is affine in the point at fixed z, so
// its largest value over a slice is at a vertex, and quadratic in z along a
// vertex, so its largest value over the z range is at an end or at the
// stationary point).  tau = 1e-9 L^2 (L the largest extent of the blocks)
// is far above the rounding of S_i and far below any distance that matters.
// A uniform grid over the blocks' bounding box lists, per cell, the blocks
// whose bounding box (grown by a small margin) meets the cell: the spatial
// hashing that prunes candidates before the sign test.
static double cross_z(const double *a, const double *b, const double *c) {
    return (b[0] - a[0]) * (c[1] - b[1]) - (b[1] - a[1]) * (c[0] - b[0]);
}

// +1 / -1: strictly convex quad listed counter-clockwise / clockwise; 0: not convex.
static int quad_orientation(const double q[8]) {
    int sgn = 0;
    for (int i = 0; i < 4; ++i) {
        const double c = cross_z(q + 2 * i, q + 2 * ((i + 1) % 4), q + 2 * ((i + 2) % 4));
        const int si = c > 0.0 ? 1 : (c < 0.0 ? -1 : 0);
        if (si == 0 || (sgn != 0 && si != sgn)) return 0;
        sgn = si;
    }
    return sgn;
}

// Edge product S_i of the slice at height z of the block with record r at
// the point (px, py), in the kernel's formula.
static double block_edge_product(const double *r, int i, double px, double py, double z) {
    const double t = (z - r[0]) * r[2];
    const int j = (i + 1) & 3;
    const double vix = t * r[12 + 2 * i] + r[4 + 2 * i], viy = t * r[13 + 2 * i] + r[5 + 2 * i];
    const double vjx = t * r[12 + 2 * j] + r[4 + 2 * j], vjy = t * r[13 + 2 * j] + r[5 + 2 * j];
    return (vjx - vix) * (py - viy) - (vjy - viy) * (px - vix);
}

// Largest value over [z0, z1] of sigma S_i of block rb at vertex k of block ra.
static double max_edge_product_on_vertex(const double *rb, int i, double sigma, const double *ra,
                                         int k, double z0, double z1) {
    auto f = [&](double z) {
        const double ta = (z - ra[0]) * ra[2];
        const double px = ta * ra[12 + 2 * k] + ra[4 + 2 * k];
        const double py = ta * ra[13 + 2 * k] + ra[5 + 2 * k];
        return sigma * block_edge_product(rb, i, px, py, z);
    };
    const double fa = f(z0), fm = f(0.5 * (z0 + z1)), fb = f(z1);
    double best = std::max(fa, std::max(fm, fb));
    // quadratic through the three samples: f = fm + b u + a u^2, u in [-1, 1]
    const double a = 0.5 * (fa + fb) - fm, b = 0.5 * (fb - fa);
    if (a < 0.0) {
        const double u = -b / (2.0 * a);
        if (u > -1.0 && u < 1.0) best = std::max(best, fm + b * u + a * u * u);
    }
    return best;
}

int mt_load_blocks(int32_t n, const double *block, const int32_t *material, const float *b_box,
                   const int32_t *magnet, int32_t n_mag, const double *world) {
    std::lock_guard<std::mutex> lk(g.mu);
    int rc = MT_OK;
    if (n < 1 || n > MT_MAX_BOXES)
        return fail(n < 1 ? MT_ERR_INVALID_ARG : MT_ERR_LIMIT, "n = %d not in [1, %d]", n,
                    MT_MAX_BOXES);
    if (n_mag < 0 || n_mag > MT_MAX_MAGNETS)
        return fail(n_mag < 0 ? MT_ERR_INVALID_ARG : MT_ERR_LIMIT, "n_mag = %d not in [0, %d]",
                    n_mag, MT_MAX_MAGNETS);
    if (!block || !material || !world)
        return fail(MT_ERR_INVALID_ARG, "block, material and world must be non-NULL");
    for (int a = 0; a < 3; ++a)
        if (std::isnan(world[a])) return fail(MT_ERR_INVALID_ARG, "world[%d] is NaN", a);
    std::vector<double> rec((size_t)mt::kBlockRec * n);
    std::vector<float4> bf((size_t)n);
    std::vector<int32_t> mat((size_t)n), mag((size_t)n);
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    std::vector<double> bb((size_t)6 * n);
    int max_mat = -1;
    for (int b = 0; b < n; ++b) {
        const double *p = block + 18 * b;
        for (int i = 0; i < 18; ++i)
            if (!std::isfinite(p[i]))
                return fail(MT_ERR_INVALID_ARG, "block %d: coordinates must be finite", b);
        if (!(p[0] < p[1])) return fail(MT_ERR_INVALID_ARG, "block %d: z_lo must be < z_hi", b);
        double mid[8];
        for (int i = 0; i < 8; ++i) mid[i] = 0.5 * (p[2 + i] + p[10 + i]);
        const int o0 = quad_orientation(p + 2), o1 = quad_orientation(p + 10);
        if (o0 == 0 || o1 != o0 || quad_orientation(mid) != o0)
            return fail(MT_ERR_INVALID_ARG, "block %d: end quads must be strictly convex with the "
                                            "same vertex order", b);
        double *r = rec.data() + (size_t)mt::kBlockRec * b;
        r[0] = p[0];
        r[1] = p[1];
        r[2] = 1.0 / (p[1] - p[0]);
        r[3] = 0.0;
        for (int i = 0; i < 8; ++i) {
            r[4 + i] = p[2 + i];
            r[12 + i] = p[10 + i] - p[2 + i];
        }
        double *q = bb.data() + 6 * b;
        q[0] = q[2] = INFINITY;
        q[1] = q[3] = -INFINITY;
        for (int i = 0; i < 8; ++i) {
            const double x = (i < 4 ? p[2 + 2 * i] : p[10 + 2 * (i - 4)]);
            const double y = (i < 4 ? p[3 + 2 * i] : p[11 + 2 * (i - 4)]);
            q[0] = std::min(q[0], x);
            q[1] = std::max(q[1], x);
            q[2] = std::min(q[2], y);
            q[3] = std::max(q[3], y);
        }
        q[4] = p[0];
        q[5] = p[1];
        for (int a = 0; a < 3; ++a) {
            lo[a] = std::min(lo[a], q[2 * a]);
            hi[a] = std::max(hi[a], q[2 * a + 1]);
        }
        if (material[b] < -1) return fail(MT_ERR_INVALID_ARG, "material[%d] < -1", b);
        mat[b] = material[b];
        max_mat = std::max(max_mat, material[b]);
        const int m = magnet ? magnet[b] : -1;
        if (m < -1 || m >= n_mag)
            return fail(MT_ERR_INVALID_ARG, "magnet[%d] = %d not in [-1, n_mag)", b, m);
        mag[b] = m;
        bf[b] = b_box ? make_float4(b_box[3 * b], b_box[3 * b + 1], b_box[3 * b + 2], 0.f)
                      : make_float4(0.f, 0.f, 0.f, 0.f);
    }
    // m of every block (see above): lower-index blocks separated by an edge line
    {
        double L = 0.0;
        for (int a = 0; a < 3; ++a) L = std::max(L, hi[a] - lo[a]);
        const double tau = 1e-9 * L * L;
        for (int b = 0; b < n; ++b) {
            double *rb = rec.data() + (size_t)mt::kBlockRec * b;
            const double sigma = (double)quad_orientation(block + 18 * b + 2);
            bool ok = true;
            for (int a = 0; a < b && ok; ++a) {
                const double *ra = rec.data() + (size_t)mt::kBlockRec * a;
                const double z0 = std::max(ra[0], rb[0]), z1 = std::min(ra[1], rb[1]);
                if (!(z0 < z1)) continue;            // half-open z ranges that do not meet
                bool sep = false;
                for (int i = 0; i < 4 && !sep; ++i) {
                    double worst = -INFINITY;
                    for (int k = 0; k < 4; ++k)
                        worst = std::max(worst, max_edge_product_on_vertex(rb, i, sigma, ra, k,
                                                                           z0, z1));
                    sep = worst <= 0.5 * tau;
                }
                ok = sep;
            }
            rb[3] = ok ? sigma * tau : 0.0;
        }
    }
    // Grid: about kGridCells roughly cubic cells over the bounding box grown by
    // a margin far above the rounding of a cell index.
    double ext[3], eps = 0.0;
    for (int a = 0; a < 3; ++a) eps = std::max(eps, hi[a] - lo[a]);
    eps = 1e-6 * (1.0 + eps);
    for (int a = 0; a < 3; ++a) {
        lo[a] -= eps;
        hi[a] += eps;
        ext[a] = hi[a] - lo[a];
    }
    const double cell = std::cbrt(ext[0] * ext[1] * ext[2] / (double)mt::kGridCells);
    int dims[3];
    for (int a = 0; a < 3; ++a) dims[a] = (int)std::max(1.0, std::min(256.0, std::floor(ext[a] / cell)));
    while ((int64_t)dims[0] * dims[1] * dims[2] > mt::kGridCells) {
        int a = 0;
        for (int c = 1; c < 3; ++c)
            if (ext[c] / dims[c] < ext[a] / dims[a]) a = c;
        --dims[a];
    }
    const int G = dims[0] * dims[1] * dims[2];
    std::vector<uint64_t> grid((size_t)G, 0ull);
    for (int b = 0; b < n; ++b) {
        const double *q = bb.data() + 6 * b;
        int c0[3], c1[3];
        for (int a = 0; a < 3; ++a) {
            const double w = ext[a] / dims[a];
            c0[a] = std::max(0, (int)std::floor((q[2 * a] - eps - lo[a]) / w));
            c1[a] = std::min(dims[a] - 1, (int)std::floor((q[2 * a + 1] + eps - lo[a]) / w));
        }
        for (int k = c0[2]; k <= c1[2]; ++k)
            for (int j = c0[1]; j <= c1[1]; ++j)
                for (int i = c0[0]; i <= c1[0]; ++i)
                    grid[((size_t)k * dims[1] + j) * dims[0] + i] |= 1ull << b;
    }
    if ((rc = ensure_device())) return rc;
    if ((rc = g.blk.upload(rec.data(), rec.size() * 8))) return rc;
    if ((rc = g.grid.upload(grid.data(), grid.size() * 8))) return rc;
    if ((rc = g.bfield.upload(bf.data(), bf.size() * 16))) return rc;
    if ((rc = g.material.upload(mat.data(), mat.size() * 4))) return rc;
    if ((rc = g.magnet.upload(mag.data(), mag.size() * 4))) return rc;
    mt::DevGeom &G_ = g.T.geom;
    G_.n_box = n;
    G_.n_poly = n;
    G_.n_slab = 0;
    G_.n_mag = n_mag;
    G_.disjoint = 0;
    G_.box4 = nullptr;
    G_.slab_z = nullptr;
    G_.slab_mask = nullptr;
    G_.poly = reinterpret_cast<const double *>(g.blk.p);
    G_.grid = reinterpret_cast<const uint64_t *>(g.grid.p);
    G_.gx = dims[0];
    G_.gy = dims[1];
    G_.gz = dims[2];
    for (int a = 0; a < 3; ++a) {
        G_.g0[a] = lo[a];
        G_.ginv[a] = (double)dims[a] / ext[a];
    }
    G_.material = reinterpret_cast<const int32_t *>(g.material.p);
    G_.bfield = reinterpret_cast<const float4 *>(g.bfield.p);
    G_.magnet = reinterpret_cast<const int32_t *>(g.magnet.p);
    G_.x_max = world[0];
    G_.y_max = world[1];
    G_.z_max = world[2];
    g.max_material = max_mat;
    g.geom_loaded = true;
    relayout();
    tables_changed();
    return MT_OK;
}

int mt_load_field(int32_t nx, int32_t ny, int32_t nz, const double *lo, const double *hi,
                  const float *b) {
    std::lock_guard<std::mutex> lk(g.mu);
    int rc = MT_OK;
    if (!b) {
        g.map.release();
        g.nodes.release();
        g.T.field = mt::DevField{};
        tables_changed();
        return MT_OK;
    }
    if (nx < 2 || ny < 2 || nz < 2) return fail(MT_ERR_INVALID_ARG, "nx, ny, nz must be >= 2");
    if (!lo || !hi) return fail(MT_ERR_INVALID_ARG, "lo and hi must be non-NULL");
    for (int a = 0; a < 3; ++a)
        if (!std::isfinite(lo[a]) || !std::isfinite(hi[a]) || !(hi[a] > lo[a]))
            return fail(MT_ERR_INVALID_ARG, "field bounds must be finite with hi > lo (axis %d)", a);
    // Cell-major copy: every cell's trilinear interpolant in one 128-byte
    // record, as the coefficients k0..k7 of
    //   k0 + k1 fx + k2 fy + k3 fz + k4 fx fy + k5 fx fz + k6 fy fz + k7 fx fy fz
    // in the fractional coordinates of the cell (formed in FP64 from the 8
    // corner values, then rounded), so a lookup touches one cache line
    // instead of four and evaluates 7 FMAs per component.
    const size_t cx = (size_t)nx - 1, cy = (size_t)ny - 1, cz = (size_t)nz - 1;
    const size_t cells = cx * cy * cz;
    if ((size_t)nx * ny * nz > 0x7FFFFFFFull)
        return fail(MT_ERR_LIMIT, "the field map has %zu nodes, more than 2^31 - 1",
                    (size_t)nx * ny * nz);
    if ((size_t)nx >= (1u << 24) || (size_t)ny * nz >= (1u << 24))
        return fail(MT_ERR_LIMIT, "the field map needs nx < 2^24 and ny nz < 2^24 (cell and "
                                  "node indices are formed with 24-bit products)");
    for (size_t i = 0; i < 3 * (size_t)nx * ny * nz; ++i)
        if (!std::isfinite(b[i]))
            return fail(MT_ERR_INVALID_ARG, "field map value %zu (node %zu, component %zu) is "
                                            "not finite", i, i / 3, i % 3);
    std::vector<float4> m;
    try {
        m.resize(cells * 8);
    } catch (const std::bad_alloc &) {
        return fail(MT_ERR_OOM, "host memory for %zu field-map cells", cells);
    }
    for (size_t k = 0; k < cz; ++k)
        for (size_t j = 0; j < cy; ++j)
            for (size_t i = 0; i < cx; ++i) {
                float4 *rec = m.data() + ((k * cy + j) * cx + i) * 8;
                float kc[8][3];
                for (int a = 0; a < 3; ++a) {
                    // corner values C[c], c = dx + 2 dy + 4 dz
                    double C[8];
                    for (int c = 0; c < 8; ++c) {
                        const size_t node = ((k + (c >> 2)) * (size_t)ny + (j + ((c >> 1) & 1))) *
                                                nx + (i + (c & 1));
                        C[c] = (double)b[3 * node + a];
                    }
                    const double q[8] = {
                        C[0],
                        C[1] - C[0],
                        C[2] - C[0],
                        C[4] - C[0],
                        C[3] - C[1] - C[2] + C[0],
                        C[5] - C[1] - C[4] + C[0],
                        C[6] - C[2] - C[4] + C[0],
                        C[7] - C[3] - C[5] - C[6] + C[1] + C[2] + C[4] - C[0]};
                    for (int c = 0; c < 8; ++c) {
                        kc[c][a] = (float)q[c];
                        if (!std::isfinite(kc[c][a]))
                            return fail(MT_ERR_INVALID_ARG,
                                        "field map cell (%zu, %zu, %zu): an interpolation "
                                        "coefficient overflows single precision", i, j, k);
                    }
                }
                for (int c = 0; c < 8; ++c) rec[c] = make_float4(kc[c][0], kc[c][1], kc[c][2], 0.f);
            }
    // Node-major copy for the nearest-node lookup (one value per lookup).
    std::vector<float4> nd;
    try {
        nd.resize((size_t)nx * ny * nz);
    } catch (const std::bad_alloc &) {
        return fail(MT_ERR_OOM, "host memory for %zu field-map nodes", nd.size());
    }
    for (size_t i = 0; i < nd.size(); ++i)
        nd[i] = make_float4(b[3 * i], b[3 * i + 1], b[3 * i + 2], 0.f);
    if ((rc = ensure_device())) return rc;
    if ((rc = g.map.upload(m.data(), m.size() * sizeof(float4)))) return rc;
    if ((rc = g.nodes.upload(nd.data(), nd.size() * sizeof(float4)))) return rc;
    mt::DevField &F = g.T.field;
    F.map = reinterpret_cast<const float4 *>(g.map.p);
    F.nodes = reinterpret_cast<const float4 *>(g.nodes.p);
    F.nx = nx;
    F.ny = ny;
    F.nz = nz;
    const int n[3] = {nx, ny, nz};
    for (int a = 0; a < 3; ++a) {
        F.lo[a] = lo[a];
        F.inv_d[a] = (double)(n[a] - 1) / (hi[a] - lo[a]);
        F.umax[a] = (double)(n[a] - 1);
        F.off[a] = -lo[a] * F.inv_d[a];
    }
    tables_changed();
    return MT_OK;
}

int mt_propagate(const mt_params *params, int64_t n, const mt_muons *in, mt_muons *out,
                 mt_result *res, void *hip_stream) {
    std::lock_guard<std::mutex> lk(g.mu);
    return propagate_impl(params, n, in, out, res, hip_stream, 0, 0, true);
}

int mt_propagate_noalloc(const mt_params *params, int64_t n, const mt_muons *in, mt_muons *out,
                         mt_result *res, void *hip_stream) {
    std::lock_guard<std::mutex> lk(g.mu);
    Call c;
    int rc = validate(params, n, in, out, res, false, c);
    if (rc) return rc;
    if (params->use_graph)
        return fail(MT_ERR_INVALID_ARG, "mt_propagate_noalloc captures no graph: use_graph "
                                        "must be 0");
    if (params->ckpt_every != 0)
        return fail(MT_ERR_INVALID_ARG, "mt_propagate_noalloc does not checkpoint");
    const size_t need =
        kNoallocCounterBytes +
        (params->tally ? (size_t)n_part_blocks(c.n) * c.n_variants * 3 * sizeof(double) : 0);
    if (need > sizeof(scratch))
        return fail(MT_ERR_LIMIT, "the tally partial sums need %zu bytes of workspace, more than "
                                  "the %zu of MT_NOALLOC_SCRATCH_BYTES", need, sizeof(scratch));
    int dev = -1;
    MT_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices)
        return fail(MT_ERR_LIMIT, "device index %d beyond %d", dev, kMaxDevices);
    if (!noalloc_addr[dev]) {       // once per device, with that device current
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(MT_ERR_HIP, "hipGetSymbolAddress of the workspace failed: %s",
                        hipGetErrorString(e));
        noalloc_addr[dev] = ptr;
    }
    char *ws = reinterpret_cast<char *>(noalloc_addr[dev]);
    unsigned long long *queue = reinterpret_cast<unsigned long long *>(ws);
    double *partial = reinterpret_cast<double *>(ws + kNoallocCounterBytes);
    hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
    if (c.lanes == 0) {
        if (params->tally)
            MT_HIP(mt::launch_queue_reset(queue, params->tally, (int64_t)params->n_variants * 3,
                                          s));
        return MT_OK;
    }
    // block as given (0: default); no autotuner lookup; the persistent form
    // runs as one pass (its survivor lists would need 112 bytes per lane)
    return enqueue_ws(params, c, s, queue, nullptr, partial);
}

int mt_propagate_backward(const mt_params *params, int64_t n, const mt_muons *in,
                          const mt_result *res, const double *g_out, double *g_in,
                          double *g_scales, void *hip_stream) {
    std::lock_guard<std::mutex> lk(g.mu);
    Call c;
    int rc = validate(params, n, in, nullptr, res, true, c);
    if (rc) return rc;
    if (params->mode != MT_MODE_PLAIN)
        return fail(MT_ERR_INVALID_ARG, "the backward pass follows a MT_MODE_PLAIN forward");
    if (c.lanes > 0 && (!g_out || !g_in))
        return fail(MT_ERR_INVALID_ARG, "g_out and g_in must be non-NULL");
    hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
    const int n_mag = g.T.geom.n_mag;
    const WorkspaceAddr ws = workspace_addr();
    if (c.lanes == 0) {
        if (g_scales && n_mag > 0) {
            rc = g.queue.ensure(8);
            drop_graphs_if_moved(ws);
            if (rc) return rc;
            MT_HIP(mt::launch_queue_reset(reinterpret_cast<unsigned long long *>(g.queue.p),
                                          g_scales, (int64_t)params->n_variants * n_mag, s));
        }
        return MT_OK;
    }
    if ((rc = g.scratch.ensure((size_t)mt::adjoint_scratch_bytes(g.T, c.lanes)))) return rc;
    if ((rc = g.gs_lane.ensure((size_t)std::max(1, n_mag) * c.lanes * sizeof(double)))) return rc;
    MT_HIP(mt::launch_adjoint(g.T, c.R, c.io, g_out, g_in,
                              reinterpret_cast<double *>(g.gs_lane.p), g.scratch.p,
                              g.opt_adjoint_block, g.opt_adjoint_lds_history != 0, s));
    if (g_scales && n_mag > 0) {
        const int nb = n_part_blocks(c.n);
        rc = g.partial.ensure((size_t)nb * c.n_variants * n_mag * sizeof(double));
        drop_graphs_if_moved(ws);
        if (rc) return rc;
        MT_HIP(mt::launch_column_sums(reinterpret_cast<const double *>(g.gs_lane.p), n_mag, c.n,
                                      c.n_variants, reinterpret_cast<double *>(g.partial.p), nb,
                                      g_scales, s));
    }
    return MT_OK;
}

int mt_autotune(const mt_params *params, int64_t n, const mt_muons *in, mt_muons *out,
                mt_result *res, void *hip_stream, int32_t *best_block, int32_t *best_compact,
                float *best_ms) {
    std::lock_guard<std::mutex> lk(g.mu);
    if (!params) return fail(MT_ERR_INVALID_ARG, "params is NULL");
    if (params->mode != MT_MODE_PERSISTENT && params->mode != MT_MODE_VARIANT_WAVES)
        return fail(MT_ERR_INVALID_ARG, "the autotuner tunes MT_MODE_PERSISTENT and "
                                        "MT_MODE_VARIANT_WAVES launches");
    hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
    const int blocks[] = {64, 128, 256, 512};
    const bool waves = params->mode == MT_MODE_VARIANT_WAVES;   // no pass length to tune
    const std::vector<int> compacts =
        waves ? std::vector<int>{16} : std::vector<int>{32, 64, 128, 256, 512, 1 << 30};
    hipEvent_t e0, e1;
    MT_HIP(hipEventCreate(&e0));
    MT_HIP(hipEventCreate(&e1));
    float best = std::numeric_limits<float>::infinity();
    int bb = 256, bc = 16;
    mt_params p = *params;
    p.tally = nullptr;
    p.use_graph = 0;
    int rc = MT_OK;
    for (int b : blocks) {
        for (int cpt : compacts) {
            rc = propagate_impl(&p, n, in, out, res, hip_stream, b, cpt, false);   // warm-up
            if (rc) break;
            if (hipEventRecord(e0, s) != hipSuccess) { rc = fail(MT_ERR_HIP, "hipEventRecord failed"); break; }
            const int reps = 2;
            for (int r = 0; r < reps && !rc; ++r)
                rc = propagate_impl(&p, n, in, out, res, hip_stream, b, cpt, false);
            if (rc) break;
            if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
                rc = fail(MT_ERR_HIP, "event timing failed");
                break;
            }
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            ms /= reps;
            if (ms < best) {
                best = ms;
                bb = b;
                bc = cpt;
            }
        }
        if (rc) break;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    std::vector<unsigned char> key = tune_key(params, n);
    bool found = false;
    for (auto &t : g.tuned)
        if (t.key == key) {
            t.block = bb;
            t.compact = bc;
            found = true;
        }
    if (!found) g.tuned.push_back(TuneEntry{key, bb, bc});
    drop_graphs();
    if (best_block) *best_block = bb;
    if (best_compact) *best_compact = waves ? 0 : bc;
    if (best_ms) *best_ms = best;
    return MT_OK;
}

int mt_set_option(int32_t option, int64_t value) {
    std::lock_guard<std::mutex> lk(g.mu);
    switch (option) {
    case MT_OPT_GUIDE_BITS:
        if (value < 0 || value > 16)
            return fail(MT_ERR_INVALID_ARG, "MT_OPT_GUIDE_BITS must be 0 (automatic) or 1..16");
        g.opt_guide_bits = (int)value;
        return MT_OK;
    case MT_OPT_ADJOINT_BLOCK:
        if (value < 64 || value > 256 || value % 64)
            return fail(MT_ERR_INVALID_ARG, "MT_OPT_ADJOINT_BLOCK must be 64, 128, 192 or 256");
        g.opt_adjoint_block = (int)value;
        return MT_OK;
    case MT_OPT_ADJOINT_LDS_HISTORY:
        if (value != 0 && value != 1)
            return fail(MT_ERR_INVALID_ARG, "MT_OPT_ADJOINT_LDS_HISTORY must be 0 or 1");
        g.opt_adjoint_lds_history = (int)value;
        return MT_OK;
    default:
        return fail(MT_ERR_INVALID_ARG, "unknown option %d", option);
    }
}

const char *mt_last_error(void) { return g_err.c_str(); }

void mt_release(void) {
    std::lock_guard<std::mutex> lk(g.mu);
    drop_graphs();
    for (DevBuf *b : {&g.cdf, &g.guide, &g.totals, &g.edges2, &g.alias, &g.blk, &g.grid, &g.nodes, &g.box4, &g.material, &g.bfield,
                      &g.magnet, &g.slab_z, &g.slab_mask, &g.map, &g.queue, &g.partial,
                      &g.scratch, &g.gs_lane, &g.lists})
        b->release();
    if (g.cap_stream) {
        (void)hipStreamDestroy(g.cap_stream);
        g.cap_stream = nullptr;
    }
    g.T = Tables{};
    g.hist_loaded = g.geom_loaded = false;
    g.n_mat = g.n_pbin = 0;
    g.max_material = -1;
    g.tuned.clear();
    g.opt_guide_bits = 0;
    g.opt_adjoint_block = 64;
    g.opt_adjoint_lds_history = 0;
    ++g.version;
}

int mt_device_info(int32_t *info) {
    std::lock_guard<std::mutex> lk(g.mu);
    if (!info) return fail(MT_ERR_INVALID_ARG, "info is NULL");
    int rc = ensure_device();
    if (rc) return rc;
    hipDeviceProp_t prop;
    MT_HIP(hipGetDeviceProperties(&prop, g.device));
    info[0] = prop.multiProcessorCount;
    info[1] = 8;
    info[2] = (int32_t)prop.sharedMemPerBlock;
    info[3] = prop.warpSize;
    return MT_OK;
}

}  // extern "C"
