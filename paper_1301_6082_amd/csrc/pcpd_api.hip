// pcpd_api.hip -- host runtime behind include/pcpd.h: argument validation,
// thresholds, buffer ownership, tiling, phase planning and the C ABI.
// Everything numeric runs in the kernels of sweep.hip; this file only plans
// and enqueues.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/pcpd.h"
#include "pcpd_internal.h"

using pcpd::Counts;
using pcpd::DenChunk;
using pcpd::LatDesc;
using pcpd::PersistLaunch;
using pcpd::PersistState;
using pcpd::PhaseShape;
using pcpd::TileDeps;
using pcpd::TileDesc;

static_assert(sizeof(pcpd_counts) == sizeof(Counts), "count layout");

struct pcpd_ctx {
    int32_t n = 2;          // tuple size
    uint32_t B = 64;
    uint32_t planes = 1;
    uint32_t seed = 0;
    uint32_t n_inst = 0;
    std::vector<uint64_t> L;         // per instance
    std::vector<uint64_t> inst_base; // word offset of instance i's first plane
    uint64_t total_words = 0;        // planes * sum L
    uint32_t nlat = 0;               // n_inst * planes
    bool connected = false;          // connected multispin layout (pcpd_config.layout)
    bool wide = false;               // four decorrelation bits (pcpd_config.mask_bits)

    hipStream_t stream = nullptr;
    uint64_t *buf[2] = {nullptr, nullptr};
    int cur = 0;                     // index of the copy holding the current lattice
    bool owns_buf = false;

    LatDesc *d_lats = nullptr;
    TileDesc *d_tiles = nullptr;
    uint32_t ntiles = 0;
    TileDeps *d_deps = nullptr;      // per tile, for persistent launches
    uint32_t *d_done = nullptr;      // [ntiles] completion flags of a persistent launch
    PersistState *d_pstate = nullptr;
    uint32_t *h_abort = nullptr;     // pinned copy of d_pstate->abort after each batch
    DenChunk *d_chunks = nullptr;
    uint32_t nchunks = 0;
    Counts *d_counts = nullptr;      // [count_slots][nlat]
    uint32_t count_slots = 0;
    Counts *h_counts = nullptr;      // pinned mirror of d_counts

    std::vector<LatDesc> lats;       // host copy of d_lats
    PhaseShape shape{};
    uint32_t phase_max = 64;

    uint64_t t = 0;
    bool broken = false;
    hipError_t last_error = hipSuccess;  // the HIP status behind the last PCPD_EDEVICE / ENOMEM

    bool profiling = false;
    std::vector<hipEvent_t> events;  // pairs (start, stop) per profiled launch
    size_t events_used = 0;

    uint64_t *d_clock = nullptr;     // substep index at the start of the next enqueued batch
    uint32_t options = 0;            // PCPD_OPT_* flags
    hipStream_t cap_stream = nullptr;  // private stream used only to capture graphs
    struct GraphEntry;
    std::vector<GraphEntry *> graphs;  // cached executable graphs, oldest first
};

// One step of a batch: sweep `steps` Monte Carlo steps, then record the
// counts into slot `slot` (if >= 0).
struct BatchOp {
    uint64_t steps;
    int32_t slot;
    bool operator==(const BatchOp &o) const { return steps == o.steps && slot == o.slot; }
};

// A captured batch. It is valid for any starting time (the kernels read the
// device clock) but only for the same buffers, parity, tiles and slots.
struct pcpd_ctx::GraphEntry {
    std::vector<BatchOp> ops;
    int cur_in = 0, cur_out = 0;
    hipGraphExec_t exec = nullptr;
};

namespace {

constexpr uint32_t kDenChunkWords = 8192;
// Polls of one dependency wait in a persistent launch before it gives up
// (about a second; a correct schedule waits at most a few item durations).
constexpr uint32_t kPersistSpinLimit = 1u << 20;
constexpr size_t kMaxGraphs = 16;

// K = rint(q * 2^(32+m)): the integer threshold of a probability-q decision
// with m decorrelation bits. ldexp is exact and rint rounds half to even.
uint64_t rate_threshold(double q, uint32_t m) {
    return static_cast<uint64_t>(std::rint(std::ldexp(q, 32 + static_cast<int>(m))));
}

// m of a configuration (0 means the default, 2).
uint32_t mask_bits_of(const pcpd_config *cfg) { return cfg->mask_bits ? cfg->mask_bits : 2u; }

bool rate_ok(double q) { return std::isfinite(q) && q >= 0.0 && q <= 1.0; }

// check_init: also check the start kind and its host words (pcpd_init);
// pcpd_run_noalloc takes its start from device memory and ignores them.
int validate(const pcpd_config *cfg, const pcpd_instance *inst, uint32_t n_inst,
             bool check_init = true) {
    if (!cfg || !inst || n_inst == 0) return PCPD_EINVAL;
    if (cfg->model < 1 || cfg->model > 4) return PCPD_EINVAL;
    if (cfg->layout != PCPD_LAYOUT_CLASSICAL && cfg->layout != PCPD_LAYOUT_CONNECTED)
        return PCPD_EINVAL;
    if (mask_bits_of(cfg) != 2u && mask_bits_of(cfg) != 4u) return PCPD_EINVAL;
    const uint32_t n = static_cast<uint32_t>(cfg->model);
    if (cfg->B < n + 2 || cfg->planes == 0 || cfg->planes >= (1u << 29)) return PCPD_EINVAL;
    uint64_t total = 0;
    for (uint32_t i = 0; i < n_inst; ++i) {
        const pcpd_instance &in = inst[i];
        if (!rate_ok(in.p) || !rate_ok(in.d)) return PCPD_EINVAL;
        if (in.L < cfg->B || in.L % cfg->B != 0) return PCPD_EINVAL;
        if (in.L / cfg->B >= (1ull << 32)) return PCPD_EINVAL;
        if (check_init && (in.init < PCPD_INIT_FULL || in.init > PCPD_INIT_HOST)) return PCPD_EINVAL;
        if (check_init && in.init == PCPD_INIT_HOST && !in.host_words) return PCPD_EINVAL;
        const uint64_t words = in.L * cfg->planes;
        if (words / cfg->planes != in.L || total + words < total) return PCPD_EINVAL;
        total += words;
    }
    if (total > (1ull << 58)) return PCPD_EINVAL;
    return PCPD_OK;
}

// Shape for `cols` LDS columns; hb halo blocks are needed for phase_max
// substeps: an attempt reaches n+1 sites, so S substeps need (n+1)*S sites.
bool make_shape(uint32_t n, uint32_t B, uint32_t cols, uint32_t phase_max, uint32_t teams,
                PhaseShape *out) {
    if (cols == 0 || phase_max == 0) return false;
    if (teams != 2 && teams != 4) return false;
    const uint64_t reach = static_cast<uint64_t>(n + 1) * phase_max;
    const uint64_t hb = (reach + B - 1) / B;
    if (cols <= 2 * hb) return false;
    if (cols > 256) return false;
    const uint32_t ldw = (cols + 3u) | 1u;  // three spare columns, odd pitch
    if (pcpd::phase_lds_bytes(B, ldw, phase_max) > pcpd::kMaxLdsBytes) return false;
    const uint32_t threads = teams * ((cols + 63u) / 64u * 64u);  // one lane per block per team
    if (threads > 1024) return false;
    out->cols = cols;
    out->threads = threads;
    out->ldw = ldw;
    out->hb = static_cast<uint32_t>(hb);
    out->teams = teams;
    return true;
}

// Teams per tile of the default shape: four lanes per block column, each
// applying every fourth substep (measured on one GPU against two teams: +2.5%
// on 16 x 4 rings of 2^20 PCPD sites, +2.6% on 512 batched rings, equal on
// 8 TCPD rings of 2^18).
constexpr uint32_t kDefaultTeams = 4;

// Default shape: phases of two Monte Carlo steps (at most 128 substeps) and
// the widest tile of at most 128 blocks that lets two workgroups share a CU
// (half the LDS each), so that one workgroup's barriers and tile copies
// overlap the other's arithmetic; failing that, any tile that fits.
bool default_shape(uint32_t n, uint32_t B, PhaseShape *shape, uint32_t *phase_max) {
    uint32_t pm = std::max<uint32_t>(1, std::min<uint32_t>(2 * B, 128));
    for (; pm >= 1; pm = pm / 2) {
        for (uint32_t lds_cap : {pcpd::kMaxLdsBytes / 2, pcpd::kMaxLdsBytes}) {
            for (uint32_t cols = 128; cols >= 1; --cols) {
                if (make_shape(n, B, cols, pm, kDefaultTeams, shape) &&
                    pcpd::phase_lds_bytes(B, shape->ldw, pm) <= lds_cap) {
                    *phase_max = pm;
                    return true;
                }
            }
        }
        if (pm == 1) break;
    }
    return false;
}

int fail(pcpd_ctx *ctx, hipError_t e) {
    if (e == hipSuccess) return PCPD_OK;
    if (ctx) {
        ctx->broken = true;
        ctx->last_error = e;
    }
    return (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) ? PCPD_ENOMEM
                                                                       : PCPD_EDEVICE;
}

void drop_graphs(pcpd_ctx *ctx);

// Wait for the context's stream; a persistent launch that gave up a wait
// (its abort word, copied to the host after each batch) is a device error.
hipError_t sync_checked(pcpd_ctx *ctx) {
    hipError_t e = hipStreamSynchronize(ctx->stream);
    if (e == hipSuccess && ctx->h_abort && *ctx->h_abort) e = hipErrorLaunchTimeOut;
    return e;
}

// Tiles of a shape over a set of rings: each ring cut into runs of at most
// cols - 2*hb interior blocks.
std::vector<TileDesc> plan_tiles(const std::vector<LatDesc> &lats, const PhaseShape &shape) {
    std::vector<TileDesc> tiles;
    const uint32_t kmax = shape.cols - 2 * shape.hb;
    for (uint32_t l = 0; l < lats.size(); ++l) {
        const uint32_t nb = lats[l].nblocks;
        for (uint32_t k0 = 0; k0 < nb; k0 += kmax) {
            TileDesc td{};
            td.lat = l;
            td.k0 = k0;
            td.kint = std::min(kmax, nb - k0);
            tiles.push_back(td);
        }
    }
    return tiles;
}

// Dependencies of each tile in a persistent launch (TileDeps): going back
// from a tile, the fewest preceding tiles of its ring whose interiors cover
// the hb halo blocks (lo), and likewise forward (hi). plan_tiles emits the
// tiles of a ring consecutively.
std::vector<TileDeps> plan_deps(const std::vector<TileDesc> &tiles, uint32_t hb) {
    std::vector<TileDeps> deps(tiles.size());
    size_t r0 = 0;
    while (r0 < tiles.size()) {
        size_t r1 = r0;
        while (r1 < tiles.size() && tiles[r1].lat == tiles[r0].lat) ++r1;
        const uint32_t cnt = static_cast<uint32_t>(r1 - r0);
        for (uint32_t i = 0; i < cnt; ++i) {
            uint32_t lo = 0, hi = 0;
            for (uint32_t covered = 0; covered < hb && lo < cnt; ++lo)
                covered += tiles[r0 + (i + cnt - 1 - lo) % cnt].kint;
            for (uint32_t covered = 0; covered < hb && hi < cnt; ++hi)
                covered += tiles[r0 + (i + 1 + hi) % cnt].kint;
            TileDeps d{};
            d.first = static_cast<uint32_t>(r0);
            d.count = cnt;
            d.local = i;
            if (lo + hi + 1 >= cnt) lo = hi = cnt;  // the whole ring
            d.lohi = std::min<uint32_t>(lo, 0xFFFF) | (std::min<uint32_t>(hi, 0xFFFF) << 16);
            deps[r0 + i] = d;
        }
        r0 = r1;
    }
    return deps;
}

// Chunks of the density reduction: every ring cut into runs of kDenChunkWords.
std::vector<DenChunk> plan_chunks(const std::vector<LatDesc> &lats) {
    std::vector<DenChunk> chunks;
    for (uint32_t l = 0; l < lats.size(); ++l) {
        for (uint64_t w0 = 0; w0 < lats[l].L; w0 += kDenChunkWords) {
            DenChunk c{};
            c.lat = l;
            c.w0 = w0;
            c.nw = static_cast<uint32_t>(std::min<uint64_t>(kDenChunkWords, lats[l].L - w0));
            chunks.push_back(c);
        }
    }
    return chunks;
}

// Ring descriptors of validated instances, instance-major then plane-major,
// concatenated from word 0; *total_words receives planes * sum L.
std::vector<LatDesc> plan_lats(const pcpd_config *cfg, const pcpd_instance *inst, uint32_t n_inst,
                               uint64_t *total_words) {
    std::vector<LatDesc> lats;
    uint64_t base = 0;
    for (uint32_t i = 0; i < n_inst; ++i) {
        const uint32_t m = mask_bits_of(cfg);
        const uint64_t kd = rate_threshold(inst[i].d, m), kp = rate_threshold(inst[i].p, m);
        for (uint32_t q = 0; q < cfg->planes; ++q) {
            LatDesc ld{};
            ld.base = base + q * inst[i].L;
            ld.L = inst[i].L;
            ld.nblocks = static_cast<uint32_t>(inst[i].L / cfg->B);
            ld.plane = q;
            ld.key0 = cfg->seed;
            ld.key1 = inst[i].stream_id;
            ld.kd_hi = static_cast<uint32_t>(kd >> 32);
            ld.kd_lo = static_cast<uint32_t>(kd);
            ld.kp_hi = static_cast<uint32_t>(kp >> 32);
            ld.kp_lo = static_cast<uint32_t>(kp);
            ld.connected = cfg->layout == PCPD_LAYOUT_CONNECTED ? 1u : 0u;
            ld.mbits = m;
            lats.push_back(ld);
        }
        base += inst[i].L * cfg->planes;
    }
    *total_words = base;
    return lats;
}

hipError_t build_tiles(pcpd_ctx *ctx) {
    drop_graphs(ctx);  // captured launches refer to the old tile table
    const std::vector<TileDesc> tiles = plan_tiles(ctx->lats, ctx->shape);
    if (ctx->d_tiles) {
        hipError_t e = hipFree(ctx->d_tiles);
        ctx->d_tiles = nullptr;
        if (e != hipSuccess) return e;
    }
    hipError_t e = hipMalloc(&ctx->d_tiles, tiles.size() * sizeof(TileDesc));
    if (e != hipSuccess) return e;
    e = hipMemcpy(ctx->d_tiles, tiles.data(), tiles.size() * sizeof(TileDesc),
                  hipMemcpyHostToDevice);
    if (e != hipSuccess) return e;
    ctx->ntiles = static_cast<uint32_t>(tiles.size());
    // dependencies and completion flags of persistent launches
    const std::vector<TileDeps> deps = plan_deps(tiles, ctx->shape.hb);
    if (ctx->d_deps) (void)hipFree(ctx->d_deps);
    if (ctx->d_done) (void)hipFree(ctx->d_done);
    ctx->d_deps = nullptr;
    ctx->d_done = nullptr;
    if ((e = hipMalloc(&ctx->d_deps, deps.size() * sizeof(TileDeps))) != hipSuccess) return e;
    if ((e = hipMalloc(&ctx->d_done, deps.size() * sizeof(uint32_t))) != hipSuccess) return e;
    return hipMemcpy(ctx->d_deps, deps.data(), deps.size() * sizeof(TileDeps),
                     hipMemcpyHostToDevice);
}

hipError_t ensure_count_slots(pcpd_ctx *ctx, uint32_t slots) {
    if (slots <= ctx->count_slots) return hipSuccess;
    drop_graphs(ctx);  // captured density launches refer to the old slots
    if (ctx->d_counts) {
        hipError_t e = hipStreamSynchronize(ctx->stream);
        if (e != hipSuccess) return e;
        (void)hipFree(ctx->d_counts);
        (void)hipHostFree(ctx->h_counts);
        ctx->d_counts = nullptr;
        ctx->h_counts = nullptr;
        ctx->count_slots = 0;
    }
    const size_t bytes = static_cast<size_t>(slots) * ctx->nlat * sizeof(Counts);
    hipError_t e = hipMalloc(&ctx->d_counts, bytes);
    if (e != hipSuccess) return e;
    e = hipHostMalloc(&ctx->h_counts, bytes, hipHostMallocDefault);
    if (e != hipSuccess) return e;
    ctx->count_slots = slots;
    return hipSuccess;
}

// A (start, stop) event pair from the context's pool.
hipError_t next_event_pair(pcpd_ctx *ctx, hipEvent_t **pair) {
    while (ctx->events.size() < ctx->events_used + 2) {
        hipEvent_t e;
        hipError_t err = hipEventCreate(&e);
        if (err != hipSuccess) return err;
        ctx->events.push_back(e);
    }
    *pair = &ctx->events[ctx->events_used];
    ctx->events_used += 2;
    return hipSuccess;
}

void drop_graphs(pcpd_ctx *ctx) {
    for (auto *g : ctx->graphs) {
        if (g->exec) (void)hipGraphExecDestroy(g->exec);
        delete g;
    }
    ctx->graphs.clear();
}

// Enqueue a batch on `stream`: phases of at most phase_max substeps reading
// the device clock plus their offset in the batch, density records into their
// slots, and one clock advance at the end. Returns the index of the copy that
// holds the lattice afterwards.
hipError_t enqueue_ops(pcpd_ctx *ctx, const std::vector<BatchOp> &ops, hipStream_t stream,
                       bool profile, int *cur_out) {
    int cur = ctx->cur;
    uint64_t rel = 0;
    // shapes whose tile fills the whole LDS leave no room for the persistent
    // kernel's own words and run one launch per phase
    const bool persistent =
        (ctx->options & PCPD_OPT_PERSISTENT) && ctx->d_pstate &&
        pcpd::phase_lds_bytes(ctx->B, ctx->shape.ldw, ctx->phase_max) + pcpd::kPersistStaticLds <=
            pcpd::kMaxLdsBytes;
    PhaseShape shape = ctx->shape;
    shape.skip_empty = (ctx->options & PCPD_OPT_SKIP_EMPTY) ? 1u : 0u;
    shape.general = (shape.skip_empty || ctx->connected || ctx->wide) ? 1u : 0u;
    for (const BatchOp &op : ops) {
        const uint64_t end = rel + op.steps * ctx->B;
        if (persistent && end > rel) {
            // every phase of this stretch in one launch
            const uint64_t sub = end - rel;
            const uint64_t nph = (sub + ctx->phase_max - 1) / ctx->phase_max;
            PersistLaunch a{};
            a.buf0 = ctx->buf[cur];
            a.buf1 = ctx->buf[cur ^ 1];
            a.lats = ctx->d_lats;
            a.tiles = ctx->d_tiles;
            a.deps = ctx->d_deps;
            a.ntiles = ctx->ntiles;
            a.nphases = static_cast<uint32_t>(nph);
            a.clock = ctx->d_clock;
            a.s_off = rel;
            a.S = ctx->phase_max;
            a.S_last = static_cast<uint32_t>(sub - (nph - 1) * ctx->phase_max);
            a.B = ctx->B;
            a.state = ctx->d_pstate;
            a.done = ctx->d_done;
            a.spin_limit = kPersistSpinLimit;
            if (nph >= (1ull << 32) / std::max<uint32_t>(ctx->ntiles, 1)) return hipErrorInvalidValue;
            hipEvent_t *ev = nullptr;
            if (profile) {
                hipError_t e = next_event_pair(ctx, &ev);
                if (e == hipSuccess) e = hipEventRecord(ev[0], stream);
                if (e != hipSuccess) return e;
            }
            hipError_t e = pcpd::launch_persist(ctx->n, a, shape, stream);
            if (e == hipSuccess && ev) e = hipEventRecord(ev[1], stream);
            if (e == hipSuccess)
                e = hipMemcpyAsync(ctx->h_abort, &ctx->d_pstate->abort, sizeof(uint32_t),
                                   hipMemcpyDeviceToHost, stream);
            if (e != hipSuccess) return e;
            if (nph & 1) cur ^= 1;
            rel = end;
        }
        while (rel < end) {
            const uint32_t S = static_cast<uint32_t>(std::min<uint64_t>(ctx->phase_max, end - rel));
            hipEvent_t *ev = nullptr;
            if (profile) {
                hipError_t e = next_event_pair(ctx, &ev);
                if (e == hipSuccess) e = hipEventRecord(ev[0], stream);
                if (e != hipSuccess) return e;
            }
            hipError_t e = pcpd::launch_phase(ctx->n, ctx->buf[cur], ctx->buf[cur ^ 1], ctx->d_lats,
                                              ctx->d_tiles, ctx->ntiles, ctx->d_clock, rel, S,
                                              ctx->B, shape, stream);
            if (e == hipSuccess && ev) e = hipEventRecord(ev[1], stream);
            if (e != hipSuccess) return e;
            cur ^= 1;
            rel += S;
        }
        if (op.slot >= 0) {
            hipError_t e = pcpd::launch_density(
                ctx->buf[cur], ctx->d_lats, ctx->d_chunks, ctx->nchunks,
                ctx->d_counts + static_cast<size_t>(op.slot) * ctx->nlat, ctx->nlat, stream);
            if (e != hipSuccess) return e;
        }
    }
    if (rel) {
        hipError_t e = pcpd::launch_advance_clock(ctx->d_clock, rel, stream);
        if (e != hipSuccess) return e;
    }
    *cur_out = cur;
    return hipSuccess;
}

// Capture a batch into an executable graph on the private capture stream.
hipError_t capture_ops(pcpd_ctx *ctx, const std::vector<BatchOp> &ops,
                       pcpd_ctx::GraphEntry **out) {
    hipError_t e = hipSuccess;
    if (!ctx->cap_stream) {
        e = hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking);
        if (e != hipSuccess) return e;
    }
    e = hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    int cur_out = 0;
    hipError_t e_enq = enqueue_ops(ctx, ops, ctx->cap_stream, false, &cur_out);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(ctx->cap_stream, &graph);
    if (e_enq != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return e_enq;
    }
    if (e != hipSuccess) return e;
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return e;
    auto *g = new (std::nothrow) pcpd_ctx::GraphEntry();
    if (!g) {
        (void)hipGraphExecDestroy(exec);
        return hipErrorOutOfMemory;
    }
    g->ops = ops;
    g->cur_in = ctx->cur;
    g->cur_out = cur_out;
    g->exec = exec;
    if (ctx->graphs.size() >= kMaxGraphs) {
        (void)hipGraphExecDestroy(ctx->graphs.front()->exec);
        delete ctx->graphs.front();
        ctx->graphs.erase(ctx->graphs.begin());
    }
    ctx->graphs.push_back(g);
    *out = g;
    return hipSuccess;
}

// Phase launches per captured graph. A run of 10^6 Monte Carlo steps is
// 10^5..10^6 launches; one graph of them all exhausts the runtime, so long
// batches are cut into segments of a fixed number of steps, each replayed
// from one cached graph.
constexpr uint64_t kLaunchesPerGraph = 256;

// Run a batch. With graphs on (and not profiling), every whole segment of
// `seg` steps without a record replays the cached graph of that segment
// (captured on first use), and the rest of each op (fewer steps, and its
// density record) is launched directly; otherwise everything is launched
// directly.
hipError_t execute_ops(pcpd_ctx *ctx, const std::vector<BatchOp> &ops) {
    if (!(ctx->options & PCPD_OPT_GRAPH) || ctx->profiling) {
        int cur = ctx->cur;
        uint64_t steps = 0;
        for (const BatchOp &op : ops) steps += op.steps;
        hipError_t e = enqueue_ops(ctx, ops, ctx->stream, ctx->profiling, &cur);
        if (e != hipSuccess) return e;
        ctx->cur = cur;
        ctx->t += steps;
        return hipSuccess;
    }
    const uint64_t seg = std::max<uint64_t>(1, kLaunchesPerGraph * ctx->phase_max / ctx->B);
    for (const BatchOp &op : ops) {
        uint64_t left = op.steps;
        while (left >= seg) {
            const std::vector<BatchOp> one{BatchOp{seg, -1}};
            pcpd_ctx::GraphEntry *g = nullptr;
            for (auto *c : ctx->graphs)
                if (c->cur_in == ctx->cur && c->ops == one) g = c;
            if (!g) {
                hipError_t e = capture_ops(ctx, one, &g);
                if (e != hipSuccess) return e;
            }
            hipError_t e = hipGraphLaunch(g->exec, ctx->stream);
            if (e != hipSuccess) return e;
            ctx->cur = g->cur_out;
            ctx->t += seg;
            left -= seg;
        }
        if (left || op.slot >= 0) {
            int cur = ctx->cur;
            hipError_t e = enqueue_ops(ctx, {BatchOp{left, op.slot}}, ctx->stream, false, &cur);
            if (e != hipSuccess) return e;
            ctx->cur = cur;
            ctx->t += left;
        }
    }
    return hipSuccess;
}

void release(pcpd_ctx *ctx) {
    if (!ctx) return;
    if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
    if (ctx->owns_buf && ctx->buf[0]) (void)hipFree(ctx->buf[0]);
    if (ctx->d_lats) (void)hipFree(ctx->d_lats);
    if (ctx->d_tiles) (void)hipFree(ctx->d_tiles);
    if (ctx->d_deps) (void)hipFree(ctx->d_deps);
    if (ctx->d_done) (void)hipFree(ctx->d_done);
    if (ctx->d_pstate) (void)hipFree(ctx->d_pstate);
    if (ctx->h_abort) (void)hipHostFree(ctx->h_abort);
    if (ctx->d_chunks) (void)hipFree(ctx->d_chunks);
    if (ctx->d_counts) (void)hipFree(ctx->d_counts);
    if (ctx->h_counts) (void)hipHostFree(ctx->h_counts);
    for (hipEvent_t e : ctx->events) (void)hipEventDestroy(e);
    drop_graphs(ctx);
    if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
    if (ctx->d_clock) (void)hipFree(ctx->d_clock);
    delete ctx;
}

bool overflow_steps(uint64_t t, uint64_t steps, uint32_t B) {
    if (t + steps < t) return true;
    const uint64_t T = t + steps;
    return T > UINT64_MAX / B;
}

// Shapes the autotuner tries, and its process-wide cache keyed by what the
// best shape depends on: model, block width and the sizes of the rings.
using TuneKey = std::vector<uint64_t>;

TuneKey tune_key(const pcpd_ctx *ctx) {
    TuneKey k{static_cast<uint64_t>(ctx->n), ctx->B, ctx->nlat};
    uint64_t total = 0, nbmax = 0, nbmin = UINT64_MAX;
    for (const LatDesc &ld : ctx->lats) {
        total += ld.nblocks;
        nbmax = std::max<uint64_t>(nbmax, ld.nblocks);
        nbmin = std::min<uint64_t>(nbmin, ld.nblocks);
    }
    k.push_back(total);
    k.push_back(nbmax);
    k.push_back(nbmin);
    return k;
}

std::map<TuneKey, std::pair<PhaseShape, uint32_t>> &tune_cache() {
    static std::map<TuneKey, std::pair<PhaseShape, uint32_t>> cache;
    return cache;
}

// On-disk tuning cache: when the environment variable PCPD_TUNE_CACHE names a
// file, pcpd_autotune first looks the context up there (by GPU architecture
// and the key above) and appends what it measures otherwise. One entry per
// line: arch, the key's six numbers, then tile columns, phase length, teams.
// An entry may also be written by hand to force a shape; every shape gives
// the same results, and an entry the library cannot build is ignored.
std::string device_arch() {
    int dev = 0;
    hipDeviceProp_t prop{};
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) {
        (void)hipGetLastError();
        return "unknown";
    }
    std::string a(prop.gcnArchName);
    const size_t colon = a.find(':');
    return colon == std::string::npos ? a : a.substr(0, colon);
}

bool disk_lookup(const char *path, const std::string &arch, const TuneKey &key, uint32_t n,
                 uint32_t B, PhaseShape *shape, uint32_t *pm) {
    FILE *f = std::fopen(path, "r");
    if (!f) return false;
    char line[512];
    bool found = false;
    while (std::fgets(line, sizeof line, f)) {
        char a[128];
        unsigned long long k[6];
        unsigned cols, phase, teams;
        if (std::sscanf(line, "%127s %llu %llu %llu %llu %llu %llu %u %u %u", a, &k[0], &k[1], &k[2],
                        &k[3], &k[4], &k[5], &cols, &phase, &teams) != 10)
            continue;
        if (arch != a || key.size() != 6) continue;
        bool same = true;
        for (int i = 0; i < 6; ++i) same = same && key[i] == k[i];
        PhaseShape sh{};
        if (same && make_shape(n, B, cols, phase, teams, &sh)) {
            *shape = sh;
            *pm = phase;
            found = true;  // the last matching entry wins
        }
    }
    std::fclose(f);
    return found;
}

void disk_append(const char *path, const std::string &arch, const TuneKey &key,
                 const PhaseShape &shape, uint32_t pm) {
    FILE *f = std::fopen(path, "a");
    if (!f) return;
    std::fprintf(f, "%s", arch.c_str());
    for (uint64_t v : key) std::fprintf(f, " %llu", static_cast<unsigned long long>(v));
    std::fprintf(f, " %u %u %u\n", shape.cols, pm, shape.teams);
    std::fclose(f);
}

// Time one phase launch of each candidate shape on the context's own lattice:
// it reads the current copy and writes the spare one, so the state is left
// untouched. Cost = kernel time per interior window-substep.
hipError_t search_shape(pcpd_ctx *ctx, uint32_t reps, PhaseShape *best, uint32_t *best_pm) {
    hipError_t e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) return e;
    uint64_t interior = 0;
    for (const LatDesc &ld : ctx->lats) interior += ld.nblocks;
    hipEvent_t ev[2];
    if ((e = hipEventCreate(&ev[0])) != hipSuccess) return e;
    if ((e = hipEventCreate(&ev[1])) != hipSuccess) {
        (void)hipEventDestroy(ev[0]);
        return e;
    }
    const PhaseShape keep_shape = ctx->shape;
    const uint32_t keep_pm = ctx->phase_max;
    double best_cost = 0.0;
    bool found = false;
    const uint32_t cols_list[] = {32, 48, 64, 96, 128, 160, 192, 256};
    const uint32_t B = ctx->B;
    const uint32_t pm_list[] = {B / 2, B, 2 * B, 3 * B, 4 * B};
    for (uint32_t cols : cols_list) {
        for (uint32_t pm : pm_list) {
          for (uint32_t teams : {2u, 4u}) {
            PhaseShape sh{};
            if (pm == 0 || pm > 512 ||
                !make_shape(static_cast<uint32_t>(ctx->n), B, cols, pm, teams, &sh))
                continue;
            ctx->shape = sh;
            // time the kernel copy the context's runs will use
            sh.skip_empty = (ctx->options & PCPD_OPT_SKIP_EMPTY) ? 1u : 0u;
            sh.general = (sh.skip_empty || ctx->connected || ctx->wide) ? 1u : 0u;
            ctx->phase_max = pm;
            if ((e = build_tiles(ctx)) != hipSuccess) break;
            float ms = 0.0f;
            for (uint32_t r = 0; r <= reps && e == hipSuccess; ++r) {
                if (r == 1) e = hipEventRecord(ev[0], ctx->stream);
                if (e == hipSuccess)
                    e = pcpd::launch_phase(ctx->n, ctx->buf[ctx->cur], ctx->buf[ctx->cur ^ 1],
                                           ctx->d_lats, ctx->d_tiles, ctx->ntiles, ctx->d_clock, 0,
                                           pm, B, sh, ctx->stream);
            }
            if (e == hipSuccess) e = hipEventRecord(ev[1], ctx->stream);
            if (e == hipSuccess) e = hipEventSynchronize(ev[1]);
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, ev[0], ev[1]);
            if (e != hipSuccess) break;
            const double cost = ms / (static_cast<double>(reps) * interior * pm);
            if (!found || cost < best_cost) {
                best_cost = cost;
                *best = sh;
                *best_pm = pm;
                found = true;
            }
          }
          if (e != hipSuccess) break;
        }
        if (e != hipSuccess) break;
    }
    (void)hipEventDestroy(ev[0]);
    (void)hipEventDestroy(ev[1]);
    ctx->shape = keep_shape;
    ctx->phase_max = keep_pm;
    if (e == hipSuccess && !found) e = hipErrorInvalidValue;
    if (e == hipSuccess) e = build_tiles(ctx);
    return e;
}

// ---- workspace of pcpd_run_noalloc -------------------------------------
//
// One fixed region per device, in the code object's data: the spare lattice
// copy the phases alternate with, the ring, tile and density-chunk tables,
// the count records and the device clock. Each region starts 256-byte aligned.
constexpr uint64_t kNaWords = PCPD_NOALLOC_MAX_WORDS;
constexpr uint64_t kNaRings = PCPD_NOALLOC_MAX_RINGS;
constexpr uint64_t kNaRecords = PCPD_NOALLOC_MAX_RECORDS;
constexpr uint64_t kNaTiles = 65536;
constexpr uint64_t kNaChunks = 8192;
constexpr size_t align256(size_t x) { return (x + 255) / 256 * 256; }
constexpr size_t kNaOffLats = align256(kNaWords * sizeof(uint64_t));
constexpr size_t kNaOffTiles = kNaOffLats + align256(kNaRings * sizeof(LatDesc));
constexpr size_t kNaOffChunks = kNaOffTiles + align256(kNaTiles * sizeof(TileDesc));
constexpr size_t kNaOffCounts = kNaOffChunks + align256(kNaChunks * sizeof(DenChunk));
constexpr size_t kNaOffClock = kNaOffCounts + align256(kNaRecords * sizeof(Counts));
constexpr size_t kNaBytes = kNaOffClock + 256;

}  // namespace

// The workspace itself. In host code this name stands for the variable but is
// not its device address: host code uses only the address that
// hipGetSymbolAddress returns for the current device (noalloc_workspace).
static __device__ __align__(256) unsigned char scratch[kNaBytes];

namespace {

constexpr int kNaMaxDevices = 64;
std::mutex na_mu;
unsigned char *na_ptr[kNaMaxDevices] = {};

// Device address of the current device's copy of the workspace, looked up on
// the first call on that device (with it current) and kept.
hipError_t noalloc_workspace(unsigned char **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kNaMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(na_mu);
    if (!na_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        na_ptr[dev] = static_cast<unsigned char *>(p);
    }
    *out = na_ptr[dev];
    return hipSuccess;
}

}  // namespace

extern "C" {

int pcpd_lattice_bytes(const pcpd_config *cfg, const pcpd_instance *inst, uint32_t n_inst,
                       size_t *bytes_out) {
    int v = validate(cfg, inst, n_inst);
    if (v != PCPD_OK) return v;
    if (!bytes_out) return PCPD_EINVAL;
    uint64_t total = 0;
    for (uint32_t i = 0; i < n_inst; ++i) total += inst[i].L * cfg->planes;
    *bytes_out = static_cast<size_t>(2 * total * sizeof(uint64_t));
    return PCPD_OK;
}

int pcpd_init(pcpd_ctx **out, const pcpd_config *cfg, const pcpd_instance *inst,
              uint32_t n_inst, uint64_t t0, const pcpd_device *dev) {
    if (!out) return PCPD_EINVAL;
    int v = validate(cfg, inst, n_inst);
    if (v != PCPD_OK) return v;
    if (overflow_steps(t0, 0, cfg->B)) return PCPD_EOVERFLOW;
    size_t need = 0;
    pcpd_lattice_bytes(cfg, inst, n_inst, &need);
    if (dev && dev->dev_buf) {
        if (dev->dev_buf_bytes < need) return PCPD_EINVAL;
        if (reinterpret_cast<uintptr_t>(dev->dev_buf) % 256 != 0) return PCPD_EINVAL;
    }
    PhaseShape shape{};
    uint32_t pmax = 0;
    if (!default_shape(static_cast<uint32_t>(cfg->model), cfg->B, &shape, &pmax))
        return PCPD_EINVAL;

    pcpd_ctx *ctx = new (std::nothrow) pcpd_ctx();
    if (!ctx) return PCPD_ENOMEM;
    ctx->n = cfg->model;
    ctx->connected = cfg->layout == PCPD_LAYOUT_CONNECTED;
    ctx->wide = mask_bits_of(cfg) == 4u;
    ctx->B = cfg->B;
    ctx->planes = cfg->planes;
    ctx->seed = cfg->seed;
    ctx->n_inst = n_inst;
    ctx->nlat = n_inst * cfg->planes;
    ctx->t = t0;
    ctx->shape = shape;
    ctx->phase_max = pmax;
    ctx->stream = dev ? static_cast<hipStream_t>(dev->hip_stream) : nullptr;

    ctx->lats = plan_lats(cfg, inst, n_inst, &ctx->total_words);
    for (uint32_t i = 0; i < n_inst; ++i) {
        ctx->L.push_back(inst[i].L);
        ctx->inst_base.push_back(ctx->lats[i * cfg->planes].base);
    }

    hipError_t e = hipSuccess;
    if (dev && dev->dev_buf) {
        ctx->buf[0] = static_cast<uint64_t *>(dev->dev_buf);
        ctx->owns_buf = false;
    } else {
        void *p = nullptr;
        e = hipMalloc(&p, need);
        if (e != hipSuccess) {
            release(ctx);
            return fail(nullptr, e);
        }
        ctx->buf[0] = static_cast<uint64_t *>(p);
        ctx->owns_buf = true;
    }
    ctx->buf[1] = ctx->buf[0] + ctx->total_words;

    const std::vector<DenChunk> chunks = plan_chunks(ctx->lats);
    ctx->nchunks = static_cast<uint32_t>(chunks.size());

    if ((e = hipMalloc(&ctx->d_lats, ctx->lats.size() * sizeof(LatDesc))) != hipSuccess ||
        (e = hipMemcpy(ctx->d_lats, ctx->lats.data(), ctx->lats.size() * sizeof(LatDesc),
                       hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMalloc(&ctx->d_chunks, chunks.size() * sizeof(DenChunk))) != hipSuccess ||
        (e = hipMemcpy(ctx->d_chunks, chunks.data(), chunks.size() * sizeof(DenChunk),
                       hipMemcpyHostToDevice)) != hipSuccess ||
        (e = build_tiles(ctx)) != hipSuccess || (e = ensure_count_slots(ctx, 1)) != hipSuccess ||
        (e = hipMalloc(&ctx->d_clock, sizeof(uint64_t))) != hipSuccess ||
        (e = hipMalloc(&ctx->d_pstate, sizeof(PersistState))) != hipSuccess ||
        (e = hipHostMalloc(&ctx->h_abort, sizeof(uint32_t), hipHostMallocDefault)) != hipSuccess) {
        release(ctx);
        return fail(nullptr, e);
    }
    *ctx->h_abort = 0;
    const uint64_t sub0 = t0 * cfg->B;
    e = hipMemcpy(ctx->d_clock, &sub0, sizeof(uint64_t), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        release(ctx);
        return fail(nullptr, e);
    }

    // initial lattice into copy 0
    for (uint32_t i = 0; i < n_inst && e == hipSuccess; ++i) {
        uint64_t *dst = ctx->buf[0] + ctx->inst_base[i];
        const uint64_t words = inst[i].L * cfg->planes;
        if (inst[i].init == PCPD_INIT_HOST)
            e = hipMemcpyAsync(dst, inst[i].host_words, words * sizeof(uint64_t),
                               hipMemcpyHostToDevice, ctx->stream);
        else
            e = pcpd::launch_fill(dst, words, inst[i].init == PCPD_INIT_FULL ? ~0ull : 0ull,
                                  ctx->stream);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) {
        release(ctx);
        return fail(nullptr, e);
    }
    ctx->cur = 0;
    *out = ctx;
    return PCPD_OK;
}

int pcpd_sweep(pcpd_ctx *ctx, uint64_t n_steps) {
    if (!ctx) return PCPD_EINVAL;
    if (ctx->broken) return PCPD_ESTATE;
    if (overflow_steps(ctx->t, n_steps, ctx->B)) return PCPD_EOVERFLOW;
    if (n_steps == 0) return PCPD_OK;
    return fail(ctx, execute_ops(ctx, {BatchOp{n_steps, -1}}));
}

int pcpd_density(pcpd_ctx *ctx, pcpd_counts *out) {
    if (!ctx || !out) return PCPD_EINVAL;
    if (ctx->broken) return PCPD_ESTATE;
    hipError_t e = execute_ops(ctx, {BatchOp{0, 0}});
    if (e == hipSuccess)
        e = hipMemcpyAsync(ctx->h_counts, ctx->d_counts, ctx->nlat * sizeof(Counts),
                           hipMemcpyDeviceToHost, ctx->stream);
    if (e == hipSuccess) e = sync_checked(ctx);
    if (e != hipSuccess) return fail(ctx, e);
    std::memcpy(out, ctx->h_counts, ctx->nlat * sizeof(Counts));
    return PCPD_OK;
}

int pcpd_run(pcpd_ctx *ctx, const uint64_t *times, uint32_t n_times, pcpd_counts *out) {
    if (!ctx || (!times && n_times) || (!out && n_times)) return PCPD_EINVAL;
    if (ctx->broken) return PCPD_ESTATE;
    for (uint32_t r = 0; r < n_times; ++r) {
        if (times[r] < ctx->t || (r > 0 && times[r] <= times[r - 1])) return PCPD_EINVAL;
    }
    if (n_times && overflow_steps(times[n_times - 1], 0, ctx->B)) return PCPD_EOVERFLOW;
    hipError_t e = ensure_count_slots(ctx, n_times);
    std::vector<BatchOp> ops;
    uint64_t at = ctx->t;
    for (uint32_t r = 0; r < n_times; ++r) {
        ops.push_back(BatchOp{times[r] - at, static_cast<int32_t>(r)});
        at = times[r];
    }
    if (e == hipSuccess && n_times) e = execute_ops(ctx, ops);
    if (e == hipSuccess && n_times)
        e = hipMemcpyAsync(ctx->h_counts, ctx->d_counts,
                           static_cast<size_t>(n_times) * ctx->nlat * sizeof(Counts),
                           hipMemcpyDeviceToHost, ctx->stream);
    if (e == hipSuccess) e = sync_checked(ctx);
    if (e != hipSuccess) return fail(ctx, e);
    if (n_times)
        std::memcpy(out, ctx->h_counts, static_cast<size_t>(n_times) * ctx->nlat * sizeof(Counts));
    return PCPD_OK;
}

int pcpd_get_lattice(pcpd_ctx *ctx, uint32_t inst, uint64_t *host_words) {
    if (!ctx || !host_words || inst >= ctx->n_inst) return PCPD_EINVAL;
    if (ctx->broken) return PCPD_ESTATE;
    const size_t bytes = ctx->L[inst] * ctx->planes * sizeof(uint64_t);
    hipError_t e = hipMemcpyAsync(host_words, ctx->buf[ctx->cur] + ctx->inst_base[inst], bytes,
                                  hipMemcpyDeviceToHost, ctx->stream);
    if (e == hipSuccess) e = sync_checked(ctx);
    return fail(ctx, e);
}

int pcpd_set_lattice(pcpd_ctx *ctx, uint32_t inst, const uint64_t *host_words) {
    if (!ctx || !host_words || inst >= ctx->n_inst) return PCPD_EINVAL;
    if (ctx->broken) return PCPD_ESTATE;
    const size_t bytes = ctx->L[inst] * ctx->planes * sizeof(uint64_t);
    hipError_t e = hipMemcpyAsync(ctx->buf[ctx->cur] + ctx->inst_base[inst], host_words, bytes,
                                  hipMemcpyHostToDevice, ctx->stream);
    if (e == hipSuccess) e = sync_checked(ctx);
    return fail(ctx, e);
}

int pcpd_time(pcpd_ctx *ctx, uint64_t *t_out) {
    if (!ctx || !t_out) return PCPD_EINVAL;
    *t_out = ctx->t;
    return PCPD_OK;
}

int pcpd_sync(pcpd_ctx *ctx) {
    if (!ctx) return PCPD_EINVAL;
    if (ctx->broken) return PCPD_ESTATE;
    return fail(ctx, sync_checked(ctx));
}

int pcpd_set_tuning(pcpd_ctx *ctx, const pcpd_tuning *tuning) {
    if (!ctx || !tuning) return PCPD_EINVAL;
    if (ctx->broken) return PCPD_ESTATE;
    PhaseShape shape{};
    uint32_t pmax = ctx->phase_max;
    if (tuning->tile_cols == 0 && tuning->phase_max == 0 && tuning->teams == 0) {
        if (!default_shape(static_cast<uint32_t>(ctx->n), ctx->B, &shape, &pmax))
            return PCPD_EINVAL;
    } else {
        pmax = tuning->phase_max ? tuning->phase_max : ctx->phase_max;
        const uint32_t cols = tuning->tile_cols ? tuning->tile_cols : ctx->shape.cols;
        const uint32_t teams = tuning->teams ? tuning->teams : ctx->shape.teams;
        if (!make_shape(static_cast<uint32_t>(ctx->n), ctx->B, cols, pmax, teams, &shape))
            return PCPD_EINVAL;
    }
    // tiles in flight must not see their table change
    hipError_t e = sync_checked(ctx);
    if (e != hipSuccess) return fail(ctx, e);
    ctx->shape = shape;
    ctx->phase_max = pmax;
    return fail(ctx, build_tiles(ctx));
}

int pcpd_get_tuning(pcpd_ctx *ctx, pcpd_tuning *tuning) {
    if (!ctx || !tuning) return PCPD_EINVAL;
    tuning->tile_cols = ctx->shape.cols;
    tuning->phase_max = ctx->phase_max;
    tuning->teams = ctx->shape.teams;
    return PCPD_OK;
}

int pcpd_set_options(pcpd_ctx *ctx, uint32_t options) {
    constexpr uint32_t known = PCPD_OPT_GRAPH | PCPD_OPT_PERSISTENT | PCPD_OPT_SKIP_EMPTY;
    if (!ctx || (options & ~known)) return PCPD_EINVAL;
    if (ctx->broken) return PCPD_ESTATE;
    if (options != ctx->options) {
        // captured graphs hold the launches of the old options
        hipError_t e = sync_checked(ctx);
        if (e != hipSuccess) return fail(ctx, e);
        drop_graphs(ctx);
    }
    ctx->options = options;
    return PCPD_OK;
}

int pcpd_autotune(pcpd_ctx *ctx, uint32_t reps, pcpd_tuning *chosen) {
    if (!ctx) return PCPD_EINVAL;
    if (ctx->broken) return PCPD_ESTATE;
    if (reps == 0) reps = 3;
    TuneKey key = tune_key(ctx);
    PhaseShape best{};
    uint32_t best_pm = 0;
    const char *path = std::getenv("PCPD_TUNE_CACHE");
    const std::string arch = path ? device_arch() : std::string();
    auto hit = tune_cache().find(key);
    if (path && *path &&
        disk_lookup(path, arch, key, static_cast<uint32_t>(ctx->n), ctx->B, &best, &best_pm)) {
        tune_cache()[key] = {best, best_pm};
    } else if (hit != tune_cache().end()) {
        best = hit->second.first;
        best_pm = hit->second.second;
    } else {
        hipError_t e = search_shape(ctx, reps, &best, &best_pm);
        if (e != hipSuccess) return fail(ctx, e);
        tune_cache()[key] = {best, best_pm};
        if (path && *path) disk_append(path, arch, key, best, best_pm);
    }
    hipError_t e = sync_checked(ctx);
    if (e != hipSuccess) return fail(ctx, e);
    ctx->shape = best;
    ctx->phase_max = best_pm;
    e = build_tiles(ctx);
    if (e != hipSuccess) return fail(ctx, e);
    if (chosen) {
        chosen->tile_cols = best.cols;
        chosen->phase_max = best_pm;
        chosen->teams = best.teams;
    }
    return PCPD_OK;
}

int pcpd_profile(pcpd_ctx *ctx, int enable) {
    if (!ctx) return PCPD_EINVAL;
    if (ctx->broken) return PCPD_ESTATE;
    ctx->profiling = enable != 0;
    return PCPD_OK;
}

int pcpd_profile_read(pcpd_ctx *ctx, double *kernel_ms, uint64_t *launches) {
    if (!ctx || !kernel_ms || !launches) return PCPD_EINVAL;
    if (ctx->broken) return PCPD_ESTATE;
    hipError_t e = sync_checked(ctx);
    if (e != hipSuccess) return fail(ctx, e);
    double total = 0.0;
    for (size_t i = 0; i + 1 < ctx->events_used; i += 2) {
        float ms = 0.0f;
        e = hipEventElapsedTime(&ms, ctx->events[i], ctx->events[i + 1]);
        if (e != hipSuccess) return fail(ctx, e);
        total += ms;
    }
    *kernel_ms = total;
    *launches = ctx->events_used / 2;
    ctx->events_used = 0;
    return PCPD_OK;
}

int pcpd_free(pcpd_ctx *ctx) {
    if (!ctx) return PCPD_EINVAL;
    release(ctx);
    return PCPD_OK;
}

int pcpd_run_noalloc(const pcpd_config *cfg, const pcpd_instance *inst, uint32_t n_inst,
                     uint64_t t0, uint64_t *dev_lattice, const uint64_t *times, uint32_t n_times,
                     pcpd_counts *out, void *hip_stream) {
    int v = validate(cfg, inst, n_inst, /*check_init=*/false);
    if (v != PCPD_OK) return v;
    if (!dev_lattice || (!times && n_times) || (!out && n_times)) return PCPD_EINVAL;
    if (reinterpret_cast<uintptr_t>(dev_lattice) % sizeof(uint64_t) != 0) return PCPD_EINVAL;
    for (uint32_t r = 0; r < n_times; ++r)
        if (times[r] < t0 || (r > 0 && times[r] <= times[r - 1])) return PCPD_EINVAL;
    if (overflow_steps(t0, 0, cfg->B)) return PCPD_EOVERFLOW;
    if (n_times && overflow_steps(times[n_times - 1], 0, cfg->B)) return PCPD_EOVERFLOW;
    PhaseShape shape{};
    uint32_t pmax = 0;
    if (!default_shape(static_cast<uint32_t>(cfg->model), cfg->B, &shape, &pmax))
        return PCPD_EINVAL;
    uint64_t total = 0;
    const std::vector<LatDesc> lats = plan_lats(cfg, inst, n_inst, &total);
    if (total > kNaWords || lats.size() > kNaRings) return PCPD_ELIMIT;
    if (static_cast<uint64_t>(n_times) * lats.size() > kNaRecords) return PCPD_ELIMIT;
    const std::vector<TileDesc> tiles = plan_tiles(lats, shape);
    const std::vector<DenChunk> chunks = plan_chunks(lats);
    if (tiles.size() > kNaTiles || chunks.size() > kNaChunks) return PCPD_ELIMIT;
    if (n_times == 0) return PCPD_OK;

    unsigned char *ws = nullptr;
    hipError_t e = noalloc_workspace(&ws);
    if (e != hipSuccess) return fail(nullptr, e);
    const hipStream_t stream = static_cast<hipStream_t>(hip_stream);

    // A context whose two lattice copies are the caller's words and the
    // workspace's spare copy, and whose tables live in the workspace. It
    // owns nothing and is never released.
    pcpd_ctx c;
    c.n = cfg->model;
    c.B = cfg->B;
    c.planes = cfg->planes;
    c.n_inst = n_inst;
    c.nlat = static_cast<uint32_t>(lats.size());
    c.total_words = total;
    c.stream = stream;
    c.buf[0] = dev_lattice;
    c.buf[1] = reinterpret_cast<uint64_t *>(ws);
    c.cur = 0;
    c.d_lats = reinterpret_cast<LatDesc *>(ws + kNaOffLats);
    c.d_tiles = reinterpret_cast<TileDesc *>(ws + kNaOffTiles);
    c.ntiles = static_cast<uint32_t>(tiles.size());
    c.d_chunks = reinterpret_cast<DenChunk *>(ws + kNaOffChunks);
    c.nchunks = static_cast<uint32_t>(chunks.size());
    c.d_counts = reinterpret_cast<Counts *>(ws + kNaOffCounts);
    c.count_slots = n_times;
    c.d_clock = reinterpret_cast<uint64_t *>(ws + kNaOffClock);
    c.shape = shape;
    c.phase_max = pmax;
    c.connected = cfg->layout == PCPD_LAYOUT_CONNECTED;
    c.wide = mask_bits_of(cfg) == 4u;

    // The host tables are read by the copies before this call returns (it
    // synchronises below). Every count record is cleared by a kernel before
    // it is summed into, and the clock is written here, so nothing left in
    // the workspace by an earlier call is read.
    if ((e = hipMemcpyAsync(c.d_lats, lats.data(), lats.size() * sizeof(LatDesc),
                            hipMemcpyHostToDevice, stream)) != hipSuccess ||
        (e = hipMemcpyAsync(c.d_tiles, tiles.data(), tiles.size() * sizeof(TileDesc),
                            hipMemcpyHostToDevice, stream)) != hipSuccess ||
        (e = hipMemcpyAsync(c.d_chunks, chunks.data(), chunks.size() * sizeof(DenChunk),
                            hipMemcpyHostToDevice, stream)) != hipSuccess ||
        (e = pcpd::launch_fill(c.d_clock, 1, t0 * cfg->B, stream)) != hipSuccess) {
        (void)hipStreamSynchronize(stream);
        return fail(nullptr, e);
    }
    std::vector<BatchOp> ops;
    uint64_t at = t0;
    for (uint32_t r = 0; r < n_times; ++r) {
        ops.push_back(BatchOp{times[r] - at, static_cast<int32_t>(r)});
        at = times[r];
    }
    int cur = 0;
    e = enqueue_ops(&c, ops, stream, false, &cur);
    if (e == hipSuccess && cur != 0)  // the last phase wrote the spare copy
        e = hipMemcpyAsync(dev_lattice, c.buf[1], total * sizeof(uint64_t),
                           hipMemcpyDeviceToDevice, stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(out, c.d_counts, static_cast<size_t>(n_times) * c.nlat * sizeof(Counts),
                           hipMemcpyDeviceToHost, stream);
    const hipError_t es = hipStreamSynchronize(stream);
    if (e == hipSuccess) e = es;
    return fail(nullptr, e);
}

const char *pcpd_device_error(pcpd_ctx *ctx) {
    if (!ctx) return "no context";
    if (ctx->last_error == hipErrorLaunchTimeOut && ctx->h_abort && *ctx->h_abort)
        return "a persistent launch stopped: a dependency wait exceeded its bound";
    return ctx->last_error == hipSuccess ? "none" : hipGetErrorString(ctx->last_error);
}

const char *pcpd_strerror(int status) {
    switch (status) {
        case PCPD_OK: return "success";
        case PCPD_EINVAL: return "invalid argument";
        case PCPD_ENOMEM: return "out of memory";
        case PCPD_EDEVICE: return "device error";
        case PCPD_ESTATE: return "context unusable after an earlier device error";
        case PCPD_EOVERFLOW: return "substep counter overflow";
        case PCPD_ELIMIT: return "exceeds the fixed workspace of the allocation-free run";
        default: return "unknown status";
    }
}

}  // extern "C"
