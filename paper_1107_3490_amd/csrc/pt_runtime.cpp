// pt_runtime.cpp -- host side of libpt.so: validation, workspace layout,
// uploads, hipGraph replay of sweeps, read-back of state and observables.
// The C ABI is declared (with its contract) in include/pt.h.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <tuple>
#include <vector>

#include "pt.h"
#include "pt_internal.hpp"

namespace {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define PT_HIP(call)                                                                         \
    do {                                                                                     \
        hipError_t e_ = (call);                                                              \
        if (e_ != hipSuccess)                                                                \
            return fail(PT_EHIP, "%s failed: %s", #call, hipGetErrorString(e_));             \
    } while (0)

constexpr int kMaxBeads = 2048;      // 4 wavefronts x 64 lanes x 8 beads per lane
constexpr double kSentinel = 1.0e30; // x coordinate of padding beads (far from everything)
constexpr int kFlowMinSlots = 1024;  // bead slots per replica from which AUTO picks the task flow
constexpr int kSchedFlags = PT_SCHED_FULL_ENERGY | PT_SCHED_FP64_ON_ACCEPT;  // or-ed into a schedule

// Mapping of a chain of n beads: beads per lane (a power of two <= 8) and
// wavefronts per replica (1, 2 or 4), the smallest that cover n.
void mapping(int n, int *bpl, int *wpr) {
    int b = 1;
    while (b < 8 && 64 * b < n) b <<= 1;
    int w = 1;
    while (64 * w * b < n) w <<= 1;
    *bpl = b;
    *wpr = w;
}

// Position of bead j in the swizzled layout of a (B, W) chain.
int swizzle(int j, int B, int W) { return (j % B) * 64 * W + j / B; }

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// Offsets of every device array inside the caller's workspace.
struct Layout {
    int n_chains = 0, total = 0;
    std::vector<int> bpl, wpr;        // per chain
    std::vector<char> lane;           // per chain: one lane per replica
    std::vector<char> pack;           // per chain: replicas per wavefront (1, 2 or 4)
    std::vector<int64_t> coord_off;   // per conformation (doubles)
    std::vector<int64_t> word_off;    // per slot
    int64_t coord_total = 0, words_total = 0;
    size_t o_slot_chain, o_slot_index, o_slot_gid, o_beta, o_perm, o_acc, o_counts, o_word_off;
    size_t o_coord_off, o_e_run, o_b_run, o_coords, o_slot_of, o_done, o_dec, o_err;
    size_t o_chain_n, o_chain_slots, o_chain_slot0, o_chain_sid, o_chain_bpl;
    size_t o_te, o_lists, o_tmp, o_alog, o_elog, o_series, o_dig;
    size_t o_flow_ready, o_flow_arr, o_flow_task;
    size_t bytes = 0;
    int64_t log_cap = 0, series_cap = 0;
    int lists_len = 0;
};

int validate(const pt_model *m, const pt_config *c) {
    if (m == nullptr || c == nullptr) return fail(PT_EINVAL, "model and config must be non-NULL");
    const double v[7] = {m->epsilon, m->sigma, m->r_cut, m->fene_k, m->fene_R, m->fene_r0, m->step_edge};
    const char *nm[7] = {"epsilon", "sigma", "r_cut", "fene_k", "fene_R", "fene_r0", "step_edge"};
    for (int i = 0; i < 7; ++i)
        if (!(isfinite(v[i]) && v[i] > 0.0)) return fail(PT_EINVAL, "model.%s must be finite and > 0", nm[i]);
    if (!(m->fene_R < m->fene_r0)) return fail(PT_EINVAL, "model.fene_R must be below fene_r0");
    if (c->n_chains < 1) return fail(PT_EINVAL, "n_chains must be >= 1");
    if (!c->n_beads || !c->n_slots || !c->beta || !c->coords)
        return fail(PT_EINVAL, "n_beads, n_slots, beta and coords must be non-NULL");
    if (c->precision != PT_FP64 && c->precision != PT_MIXED) return fail(PT_EINVAL, "precision must be PT_FP64 or PT_MIXED");
    if (c->exchange_every < 0) return fail(PT_EINVAL, "exchange_every must be >= 0");
    if (c->series_capacity < 0 || c->log_capacity < 0) return fail(PT_EINVAL, "capacities must be >= 0");
    const int sched = c->schedule & ~kSchedFlags;
    if (sched < PT_SCHED_AUTO || sched > PT_SCHED_FLOW)
        return fail(PT_EINVAL, "schedule must be PT_SCHED_AUTO, PT_SCHED_PER_SWEEP, PT_SCHED_PERSISTENT or "
                               "PT_SCHED_FLOW, optionally with PT_SCHED_FULL_ENERGY and PT_SCHED_FP64_ON_ACCEPT");
    int64_t total = 0;
    for (int ch = 0; ch < c->n_chains; ++ch) {
        if (c->n_beads[ch] < 2) return fail(PT_EINVAL, "chain %d: n_beads must be >= 2", ch);
        if (c->mapping != nullptr && c->mapping[ch] != 0) {
            const int code = c->mapping[ch], B = (code >> 4) & 15, W = code & 15;
            const bool okb = B == 1 || B == 2 || B == 4 || B == 8, okw = W == 1 || W == 2 || W == 4;
            const int flags = code & ~0xFF;
            if (!okb || !okw || (flags != 0 && flags != PT_MAP_LANE && flags != PT_MAP_PACK2 && flags != PT_MAP_PACK4))
                return fail(PT_EINVAL, "chain %d: mapping %d is not 16*B + W with B in {1,2,4,8}, W in {1,2,4} "
                                       "(optionally + one of PT_MAP_LANE, PT_MAP_PACK2, PT_MAP_PACK4)", ch, code);
            if ((code & PT_MAP_LANE) != 0 && c->precision != PT_FP64)
                return fail(PT_EUNSUPPORTED, "chain %d: mapping PT_MAP_LANE runs the FP64 order only", ch);
            if ((flags == PT_MAP_PACK2 || flags == PT_MAP_PACK4) && !(W == 1 && (B == 1 || B == 2)))
                return fail(PT_EUNSUPPORTED, "chain %d: PT_MAP_PACK2 / PT_MAP_PACK4 take the layouts B = 1 or 2, "
                                             "W = 1 (N <= 128)", ch);
            if (64 * W * B < c->n_beads[ch])
                return fail(PT_EINVAL, "chain %d: mapping B=%d W=%d holds %d < %d beads", ch, B, W, 64 * W * B, c->n_beads[ch]);
        }
        if (c->n_beads[ch] > kMaxBeads) return fail(PT_EUNSUPPORTED, "chain %d: %d beads exceeds %d", ch, c->n_beads[ch], kMaxBeads);
        if (c->n_slots[ch] < 1) return fail(PT_EINVAL, "chain %d: n_slots must be >= 1", ch);
        total += c->n_slots[ch];
    }
    if (total > (1 << 24)) return fail(PT_EUNSUPPORTED, "too many slots (%lld)", (long long)total);
    for (int64_t g = 0; g < total; ++g)
        if (!(isfinite(c->beta[g]) && c->beta[g] >= 0.0)) return fail(PT_EINVAL, "beta[%lld] must be finite and >= 0", (long long)g);
    return PT_OK;
}

// Constants in the fixed expressions of include/pt.h, plus the mixed-path bound.
pt::Consts make_consts(const pt_model *m, double resync_rel) {
    pt::Consts k;
    k.sig2 = m->sigma * m->sigma;
    k.rc2 = m->r_cut * m->r_cut;
    k.four_eps = 4.0 * m->epsilon;
    {
        const double s2 = k.sig2 / k.rc2;
        const double s6 = (s2 * s2) * s2;
        k.e_rc = k.four_eps * (s6 * (s6 - 1.0));
    }
    k.fene_cf = ((-0.5 * m->fene_k) * m->fene_R) * m->fene_R;
    k.r0 = m->fene_r0;
    k.R = m->fene_R;
    k.edge = m->step_edge;
    k.sig2_f = (float)k.sig2;
    k.rc2_f = (float)k.rc2;
    k.four_eps_f = (float)k.four_eps;
    k.e_rc_f = (float)k.e_rc;
    // kappa of the FP32 term bound (derivation next to lj32 in pt_device.hpp).
    const double s2c = k.sig2 / k.rc2;
    const double s6c = s2c * s2c * s2c;
    const double brc = s6c * (1.0 + s6c);
    const double c_erc = 3.0 * fabs(k.e_rc) / (k.four_eps * brc);
    const double slope = (3.0 * k.four_eps / k.rc2) * fabs(2.0 * s6c * s6c - s6c);  // |dE/dr^2| at rc
    const double c_win = slope * 6.0 * k.rc2 * (1.0 + 0x1p-4) / (k.four_eps * brc);
    // + 24: the FP32 pair sums (pairwise trees of depth <= 11).
    const double kappa = std::max(128.0, ceil(1.25 * (62.0 + c_erc + c_win))) + 24.0;
    k.kbound = kappa * 0x1p-24 * k.four_eps * (1.0 + 0x1p-8);
    k.neg_floor = (m->epsilon + fabs(k.e_rc)) * (1.0 + 0x1p-30);
    k.resync_rel = resync_rel;
    return k;
}

// A sweep ends with an FP64-order energy when the running energy's bound has
// passed this fraction of max(1, |E|): 2^-30 (< 1e-9) where the running energy
// adds FP64-order differences only (PT_FP64, or PT_MIXED with
// PT_SCHED_FP64_ON_ACCEPT), 2^-6 where it adds FP32 sums.  The bound only sets
// the width of the exchange test's band (an exchange inside it is decided on
// FP64-order energies), so this is a trade between full energies at the end of
// sweeps and in-band exchanges: against 2^-10, 2^-6 took N = 2000 x 4096 from
// 22.3 to 19.7 ms per sweep (re-synchronisations 30% -> 7% of replica-sweeps,
// in-band exchanges 0.14% -> 0.7% of attempts) and the smaller workloads 2-4%.
double resync_threshold(const pt_config *c) {
    const bool fp32_sums = c->precision == PT_MIXED && (c->schedule & PT_SCHED_FP64_ON_ACCEPT) == 0;
    return fp32_sums ? 0x1p-6 : 0x1p-30;
}

Layout plan(const pt_config *c) {
    Layout L;
    L.n_chains = c->n_chains;
    int64_t total = 0;
    for (int ch = 0; ch < c->n_chains; ++ch) total += c->n_slots[ch];
    L.total = (int)total;
    L.bpl.resize(c->n_chains);
    L.wpr.resize(c->n_chains);
    L.lane.assign(c->n_chains, 0);
    L.pack.assign(c->n_chains, 1);
    L.coord_off.resize(total);
    L.word_off.resize(total);
    int g = 0;
    for (int ch = 0; ch < c->n_chains; ++ch) {
        if (c->mapping != nullptr && c->mapping[ch] != 0) {
            L.bpl[ch] = (c->mapping[ch] >> 4) & 15;
            L.wpr[ch] = c->mapping[ch] & 15;
            L.lane[ch] = (c->mapping[ch] & PT_MAP_LANE) != 0;
            L.pack[ch] = (c->mapping[ch] & PT_MAP_PACK4) ? 4 : (c->mapping[ch] & PT_MAP_PACK2) ? 2 : 1;
        } else {
            mapping(c->n_beads[ch], &L.bpl[ch], &L.wpr[ch]);
        }
        for (int s = 0; s < c->n_slots[ch]; ++s, ++g) {
            L.coord_off[g] = L.coord_total;
            L.word_off[g] = L.words_total;
            L.coord_total += 3 * 64 * L.wpr[ch] * L.bpl[ch];
            L.words_total += (c->n_beads[ch] + 63) / 64;
        }
    }
    L.log_cap = c->log_capacity;
    L.series_cap = c->series_capacity;
    // lists: per class slot lists (total) + chain lists (n_chains) + the
    // conformation lists of the persistent launches (total) + the slot lists
    // of the packed classes (total, each chain padded by at most 3)
    L.lists_len = 3 * L.total + 4 * L.n_chains;
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t r = o; o = align256(o + bytes); return r; };
    const size_t S = (size_t)L.total, C = (size_t)L.n_chains;
    L.o_slot_chain = take(4 * S);
    L.o_slot_index = take(4 * S);
    L.o_slot_gid = take(4 * S);
    L.o_beta = take(8 * S);
    L.o_perm = take(4 * S);
    L.o_acc = take(8 * 5 * S);
    L.o_counts = take(8 * pt::PT_NCOUNTS * S);
    L.o_word_off = take(8 * S);
    L.o_coord_off = take(8 * S);
    L.o_e_run = take(8 * S);
    L.o_b_run = take(8 * S);
    L.o_coords = take(8 * (size_t)L.coord_total);
    L.o_slot_of = take(4 * S);
    L.o_done = take(8 * S);
    L.o_dec = take(8 * S);
    L.o_err = take(16);
    L.o_chain_n = take(4 * C);
    L.o_chain_slots = take(4 * C);
    L.o_chain_slot0 = take(4 * C);
    L.o_chain_sid = take(4 * C);
    L.o_chain_bpl = take(4 * C);
    L.o_te = take(16);
    L.o_dig = take(16 * S);
    L.o_flow_ready = take(8 * S);
    L.o_flow_arr = take(8 * S);
    L.o_flow_task = take(16);
    L.o_lists = take(4 * (size_t)L.lists_len);
    L.o_tmp = take(16 * S);
    L.o_alog = take(8 * (size_t)L.words_total * (size_t)L.log_cap);
    L.o_elog = take(S * (size_t)L.log_cap);
    L.o_series = take(8 * 3 * S * (size_t)L.series_cap);
    L.bytes = o;
    return L;
}

// Same expression as the kernels' FENE argument (r^2 -> y); used for the
// domain check of the starting bonds.
double fene_y(const pt::Consts &k, const double *a, const double *b) {
    const double dx = b[0] - a[0], dy = b[1] - a[1], dz = b[2] - a[2];
    const double r2 = fma(dz, dz, fma(dy, dy, dx * dx));
    const double x = (sqrt(r2) - k.r0) / k.R;
    return fma(-x, x, 1.0);
}

}  // namespace

struct Class {
    int bpl = 0, wpr = 0;
    bool lane = false;        // one lane per replica (FP64 order, per-sweep launches)
    int pack = 1;             // replicas per wavefront (2, 4: per-sweep launches of k_sweep_pack)
    bool persistent = false;  // whole sweeps run by a persistent launch (of its run group)
    bool flow = false;        // whole sweeps run by one task-flow launch (slots do not all fit)
    bool whole() const { return persistent || flow; }
    int n_slots = 0, n_chains = 0, max_pairs = 0;
    int32_t *d_slots = nullptr;   // slot (= starting conformation) list
    int32_t *d_chains = nullptr;  // chain list
    int32_t *d_pack = nullptr;    // packed classes: slot list, each chain padded to a multiple of pack with -1
    int n_pack_blocks = 0;
    int64_t resident = 0;         // task flow: blocks the device holds at once
};

// Persistent classes of one wavefront count W that run in one launch (every
// block resident at once); blocks take their chain's B at run time.
struct RunGroup {
    int wpr = 0, max_bpl = 0, n = 0;
    bool dense = false;         // the register-capped build (more blocks per compute unit)
    int32_t *d_list = nullptr;  // conformations, longest chains first
};

struct pt_handle {
    pt_model model;
    pt::Consts k;
    Layout L;
    pt::Tables T;
    hipStream_t stream = nullptr;
    hipStream_t cap_stream = nullptr;
    char *ws = nullptr;
    bool mixed = false;
    std::vector<Class> classes;
    std::vector<RunGroup> groups;
    std::vector<int32_t> n_beads, n_slots;
    int exchange_every = 1;
    int64_t t_host = 0, e_host = 0;  // counters as enqueued
    hipGraphExec_t graph1 = nullptr, graph16 = nullptr;
    // Graphs of the persistent and task-flow launches of n sweeps, by n.
    std::vector<std::pair<int64_t, hipGraphExec_t>> whole_graphs;
    double *d_tmp = nullptr;
    uint64_t seed = 0;
    bool failed = false;  // a persistent or task-flow run timed out; only pt_set_state recovers
};

namespace {

hipError_t launch_class_sweep(const pt_handle *h, const Class &c, hipStream_t s) {
    if (c.lane) return pt::launch_sweep_lane(c.bpl, c.wpr, h->T, c.d_slots, c.n_slots, s);
    if (c.pack > 1) return pt::launch_sweep_pack(c.bpl, c.pack, h->mixed, h->T, c.d_pack, c.n_pack_blocks, s);
    return pt::launch_sweep(c.bpl, c.wpr, h->mixed, h->T, c.d_slots, c.n_slots, s);
}

int enqueue_sweep(pt_handle *h, hipStream_t s) {
    for (const Class &c : h->classes) {
        if (c.whole()) continue;
        hipError_t e = launch_class_sweep(h, c, s);
        if (e != hipSuccess) return fail(PT_EHIP, "sweep launch failed: %s", hipGetErrorString(e));
    }
    for (const Class &c : h->classes) {
        if (c.whole()) continue;
        hipError_t e = pt::launch_exchange(c.bpl, c.wpr, h->T, c.d_chains, c.n_chains, c.max_pairs, 0, s);
        if (e != hipSuccess) return fail(PT_EHIP, "exchange launch failed: %s", hipGetErrorString(e));
    }
    hipError_t e = pt::launch_advance(h->T, 0, s);
    if (e != hipSuccess) return fail(PT_EHIP, "advance launch failed: %s", hipGetErrorString(e));
    return PT_OK;
}

int capture(pt_handle *h, int sweeps, hipGraphExec_t *out) {
    hipGraph_t graph = nullptr;
    PT_HIP(hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal));
    int rc = PT_OK;
    for (int i = 0; i < sweeps && rc == PT_OK; ++i) rc = enqueue_sweep(h, h->cap_stream);
    hipError_t e = hipStreamEndCapture(h->cap_stream, &graph);
    if (rc != PT_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return rc;
    }
    if (e != hipSuccess) return fail(PT_EHIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
    e = hipGraphInstantiate(out, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return fail(PT_EHIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
    return PT_OK;
}

void advance_host(pt_handle *h, int64_t sweeps) {
    for (int64_t i = 0; i < sweeps; ++i) {
        if (h->exchange_every > 0 && (h->t_host + 1) % h->exchange_every == 0) h->e_host += 1;
        h->t_host += 1;
    }
}

}  // namespace

PT_API size_t pt_workspace_bytes(const pt_model *model, const pt_config *config) {
    if (validate(model, config) != PT_OK) return 0;
    return plan(config).bytes;
}

PT_API int pt_init(const pt_model *model, const pt_config *cfg, void *d_workspace, size_t ws_bytes,
                   void *hip_stream, pt_handle **out) {
    if (out == nullptr) return fail(PT_EINVAL, "out must be non-NULL");
    *out = nullptr;
    int rc = validate(model, cfg);
    if (rc != PT_OK) return rc;
    Layout L = plan(cfg);
    if (d_workspace == nullptr || ws_bytes < L.bytes)
        return fail(PT_ENOMEM, "workspace of %zu bytes is smaller than the %zu needed", ws_bytes, L.bytes);
    if (((uintptr_t)d_workspace & 255) != 0) return fail(PT_EINVAL, "workspace must be 256-byte aligned");
    const pt::Consts k = make_consts(model, resync_threshold(cfg));

    // Host-side checks and swizzled coordinates.
    const int S = L.total, C = L.n_chains;
    std::vector<int32_t> slot_chain(S), slot_index(S), perm(S);
    std::vector<uint32_t> slot_gid(S), chain_sid(C);
    std::vector<int32_t> chain_n(C), chain_slots(C), chain_slot0(C);
    std::vector<double> coords((size_t)L.coord_total);
    {
        int g = 0;
        int64_t src = 0;
        for (int ch = 0; ch < C; ++ch) {
            const int n = cfg->n_beads[ch], B = L.bpl[ch], W = L.wpr[ch], NP = 64 * W * B;
            chain_n[ch] = n;
            chain_slots[ch] = cfg->n_slots[ch];
            chain_slot0[ch] = g;
            chain_sid[ch] = cfg->stream_chain ? cfg->stream_chain[ch] : (uint32_t)ch;
            const uint32_t sid0 = cfg->stream_slot0 ? cfg->stream_slot0[ch] : (uint32_t)g;
            for (int s = 0; s < cfg->n_slots[ch]; ++s, ++g) {
                slot_chain[g] = ch;
                slot_index[g] = s;
                slot_gid[g] = sid0 + (uint32_t)s;
                perm[g] = g;
                const double *xyz = cfg->coords + src;
                for (int j = 0; j < 3 * n; ++j)
                    if (!isfinite(xyz[j])) return fail(PT_EINVAL, "slot %d: non-finite coordinate", g);
                for (int j = 0; j + 1 < n; ++j)
                    if (!(fene_y(k, xyz + 3 * j, xyz + 3 * (j + 1)) > 0.0))
                        return fail(PT_EDOMAIN, "slot %d: bond (%d,%d) at or beyond r0 +- R", g, j, j + 1);
                double *dst = coords.data() + L.coord_off[g];
                for (int j = 0; j < NP; ++j) {
                    const int p = swizzle(j, B, W);
                    dst[p] = (j < n) ? xyz[3 * j] : kSentinel;
                    dst[NP + p] = (j < n) ? xyz[3 * j + 1] : 0.0;
                    dst[2 * NP + p] = (j < n) ? xyz[3 * j + 2] : 0.0;
                }
                src += 3 * (int64_t)n;
            }
        }
    }

    pt_handle *h = new (std::nothrow) pt_handle();
    if (h == nullptr) return fail(PT_ENOMEM, "host allocation failed");
    h->model = *model;
    h->k = k;
    h->L = L;
    h->stream = (hipStream_t)hip_stream;
    h->ws = (char *)d_workspace;
    h->mixed = cfg->precision == PT_MIXED;
    h->exchange_every = cfg->exchange_every;
    h->seed = cfg->seed;
    h->n_beads.assign(cfg->n_beads, cfg->n_beads + C);
    h->n_slots.assign(cfg->n_slots, cfg->n_slots + C);
    char *w = h->ws;
    pt::Tables &T = h->T;
    T.slot_chain = (const int32_t *)(w + L.o_slot_chain);
    T.slot_index = (const int32_t *)(w + L.o_slot_index);
    T.slot_gid = (const uint32_t *)(w + L.o_slot_gid);
    T.beta = (const double *)(w + L.o_beta);
    T.perm = (int32_t *)(w + L.o_perm);
    T.acc = (double *)(w + L.o_acc);
    T.counts = (int64_t *)(w + L.o_counts);
    T.word_off = (const int64_t *)(w + L.o_word_off);
    T.coords = (double *)(w + L.o_coords);
    T.coord_off = (const int64_t *)(w + L.o_coord_off);
    T.e_run = (double *)(w + L.o_e_run);
    T.b_run = (double *)(w + L.o_b_run);
    T.chain_n = (const int32_t *)(w + L.o_chain_n);
    T.chain_slots = (const int32_t *)(w + L.o_chain_slots);
    T.chain_slot0 = (const int32_t *)(w + L.o_chain_slot0);
    T.chain_sid = (const uint32_t *)(w + L.o_chain_sid);
    T.chain_bpl = (const int32_t *)(w + L.o_chain_bpl);
    T.te = (int64_t *)(w + L.o_te);
    T.slot_of = (int32_t *)(w + L.o_slot_of);
    T.done = (int64_t *)(w + L.o_done);
    T.dec = (int64_t *)(w + L.o_dec);
    T.err = (int32_t *)(w + L.o_err);
    T.dig = (uint64_t *)(w + L.o_dig);
    T.flow_ready = (int64_t *)(w + L.o_flow_ready);
    T.flow_arr = (int64_t *)(w + L.o_flow_arr);
    T.flow_task = (int64_t *)(w + L.o_flow_task);
    T.accept_log = L.log_cap > 0 ? (uint64_t *)(w + L.o_alog) : nullptr;
    T.log_cap = L.log_cap;
    T.words_total = L.words_total;
    T.exch_log = L.log_cap > 0 ? (uint8_t *)(w + L.o_elog) : nullptr;
    T.series = L.series_cap > 0 ? (double *)(w + L.o_series) : nullptr;
    T.series_cap = L.series_cap;
    T.total_slots = S;
    T.exchange_every = cfg->exchange_every;
    T.spin_limit = 1u << 24;
    T.guard_scale = 1.0;
    T.full_energy = (cfg->schedule & PT_SCHED_FULL_ENERGY) != 0 ? 1 : 0;
    T.fp64_on_accept = (cfg->schedule & PT_SCHED_FP64_ON_ACCEPT) != 0 ? 1 : 0;
    T.seed = cfg->seed;
    T.k = k;
    h->d_tmp = (double *)(w + L.o_tmp);

    // Classes by (beads per lane, wavefronts per replica, one lane per replica).
    std::map<std::tuple<int, int, int, int>, std::vector<int>> cls_chains;
    for (int ch = 0; ch < C; ++ch) cls_chains[{L.bpl[ch], L.wpr[ch], (int)L.lane[ch], (int)L.pack[ch]}].push_back(ch);
    std::vector<int32_t> lists;
    lists.reserve(L.lists_len);
    std::vector<std::vector<int>> class_chains;
    for (auto &kv : cls_chains) {
        Class cl;
        cl.bpl = std::get<0>(kv.first);
        cl.wpr = std::get<1>(kv.first);
        cl.lane = std::get<2>(kv.first) != 0;
        cl.pack = std::get<3>(kv.first);
        const size_t slot_at = lists.size();
        for (int ch : kv.second)
            for (int s = 0; s < cfg->n_slots[ch]; ++s) lists.push_back(chain_slot0[ch] + s);
        cl.n_slots = (int)(lists.size() - slot_at);
        const size_t chain_at = lists.size();
        for (int ch : kv.second) {
            lists.push_back(ch);
            cl.max_pairs = std::max(cl.max_pairs, cfg->n_slots[ch] / 2);
        }
        cl.n_chains = (int)kv.second.size();
        cl.d_slots = (int32_t *)(w + L.o_lists) + slot_at;
        cl.d_chains = (int32_t *)(w + L.o_lists) + chain_at;
        if (cl.pack > 1) {
            const size_t pack_at = lists.size();
            for (int ch : kv.second) {
                const int ns = cfg->n_slots[ch], padded = (ns + cl.pack - 1) / cl.pack * cl.pack;
                for (int s = 0; s < padded; ++s) lists.push_back(s < ns ? chain_slot0[ch] + s : -1);
            }
            cl.d_pack = (int32_t *)(w + L.o_lists) + pack_at;
            cl.n_pack_blocks = (int)((lists.size() - pack_at) / cl.pack);
        }
        h->classes.push_back(cl);
        class_chains.push_back(kv.second);
    }
    auto fin = [&](int code) {
        if (code != PT_OK) pt_destroy(h);
        return code;
    };

    // Persistent launches: the classes of one wavefront count W whose
    // replicas fit on the device at once share one launch (a run group), the
    // widest bead count per lane first, as long as the group still fits; a
    // class that does not fit alone takes the task flow when its tasks are
    // long (a sweep of 1024 or more bead slots: shorter tasks pay more for
    // their device-scope fences and flags than one launch per sweep does),
    // else one launch per sweep.  PT_SCHED_FLOW: the task flow for all.
    const int sched = cfg->schedule & ~kSchedFlags;
    if (sched != PT_SCHED_PER_SWEEP) {
        std::vector<int> order;
        for (int i = 0; i < (int)h->classes.size(); ++i)
            if (!h->classes[i].lane && h->classes[i].pack == 1) order.push_back(i);
        std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
            const Class &x = h->classes[a], &y = h->classes[b];
            return x.wpr != y.wpr ? x.wpr < y.wpr : x.bpl > y.bpl;
        });
        std::vector<char> placed(h->classes.size(), 0);
        if (sched != PT_SCHED_FLOW) {
            for (size_t a = 0; a < order.size(); ++a) {
                const int lead = order[a];
                if (placed[lead]) continue;
                const Class &cl = h->classes[lead];
                // The build without a register cap when the group fits with it,
                // else the capped one with room for more blocks.
                int64_t cap_free = 0, cap = 0;
                hipError_t e0 = pt::run_capacity(cl.wpr, h->mixed, cl.bpl, false, &cap_free);
                if (e0 == hipSuccess) e0 = pt::run_capacity(cl.wpr, h->mixed, cl.bpl, true, &cap);
                if (e0 != hipSuccess) return fin(fail(PT_EHIP, "occupancy query failed: %s", hipGetErrorString(e0)));
                cap = std::max(cap, cap_free);
                if (cl.n_slots > cap) continue;
                std::vector<int> members = {lead};
                int64_t count = cl.n_slots;
                for (size_t b = a + 1; b < order.size(); ++b) {
                    const Class &o = h->classes[order[b]];
                    if (placed[order[b]] || o.wpr != cl.wpr || count + o.n_slots > cap) continue;
                    members.push_back(order[b]);
                    count += o.n_slots;
                }
                // Conformation q starts in slot q: the group's list holds the
                // starting slots of its chains, longest chains first.
                std::vector<int> chains;
                for (int m : members) {
                    placed[m] = 1;
                    h->classes[m].persistent = true;
                    chains.insert(chains.end(), class_chains[m].begin(), class_chains[m].end());
                }
                std::stable_sort(chains.begin(), chains.end(),
                                 [&](int x, int y) { return cfg->n_beads[x] > cfg->n_beads[y]; });
                RunGroup rg;
                rg.wpr = cl.wpr;
                rg.max_bpl = cl.bpl;
                rg.n = (int)count;
                rg.dense = count > cap_free;
                rg.d_list = (int32_t *)(w + L.o_lists) + lists.size();
                for (int ch : chains)
                    for (int s = 0; s < cfg->n_slots[ch]; ++s) lists.push_back(chain_slot0[ch] + s);
                h->groups.push_back(rg);
            }
        }
        for (Class &cl : h->classes) {
            cl.flow = !cl.lane && cl.pack == 1 && !cl.persistent &&
                      (sched == PT_SCHED_FLOW || 64 * cl.wpr * cl.bpl >= kFlowMinSlots);
            if (cl.flow) {
                hipError_t e0 = pt::flow_capacity(cl.bpl, cl.wpr, h->mixed, &cl.resident);
                if (e0 != hipSuccess) return fin(fail(PT_EHIP, "occupancy query failed: %s", hipGetErrorString(e0)));
            }
        }
    }

    std::vector<int64_t> te = {0, 0};
    std::vector<int32_t> chain_bpl(L.bpl.begin(), L.bpl.end());
#define PT_UP(off, vec) \
    if (!(vec).empty()) { \
        hipError_t e_ = hipMemcpyAsync(w + (off), (vec).data(), sizeof((vec)[0]) * (vec).size(), hipMemcpyHostToDevice, h->stream); \
        if (e_ != hipSuccess) return fin(fail(PT_EHIP, "upload failed: %s", hipGetErrorString(e_))); }
    std::vector<double> beta(cfg->beta, cfg->beta + S);
    PT_UP(L.o_slot_chain, slot_chain);
    PT_UP(L.o_slot_index, slot_index);
    PT_UP(L.o_slot_gid, slot_gid);
    PT_UP(L.o_beta, beta);
    PT_UP(L.o_perm, perm);
    PT_UP(L.o_word_off, L.word_off);
    PT_UP(L.o_coord_off, L.coord_off);
    PT_UP(L.o_coords, coords);
    PT_UP(L.o_chain_n, chain_n);
    PT_UP(L.o_chain_slots, chain_slots);
    PT_UP(L.o_chain_slot0, chain_slot0);
    PT_UP(L.o_chain_sid, chain_sid);
    PT_UP(L.o_chain_bpl, chain_bpl);
    PT_UP(L.o_te, te);
    PT_UP(L.o_lists, lists);
    PT_UP(L.o_slot_of, perm);
#undef PT_UP
    hipError_t e = hipMemsetAsync(w + L.o_acc, 0, 8 * 5 * (size_t)S, h->stream);
    if (e == hipSuccess) e = hipMemsetAsync(w + L.o_done, 0, 8 * (size_t)S, h->stream);
    if (e == hipSuccess) e = hipMemsetAsync(w + L.o_dec, 0, 8 * (size_t)S, h->stream);
    if (e == hipSuccess) e = hipMemsetAsync(w + L.o_err, 0, 16, h->stream);
    if (e == hipSuccess) e = hipMemsetAsync(w + L.o_dig, 0, 16 * (size_t)S, h->stream);
    if (e == hipSuccess) e = hipMemsetAsync(w + L.o_flow_ready, 0, 8 * (size_t)S, h->stream);
    if (e == hipSuccess) e = hipMemsetAsync(w + L.o_flow_arr, 0, 8 * (size_t)S, h->stream);
    if (e == hipSuccess) e = hipMemsetAsync(w + L.o_flow_task, 0, 16, h->stream);
    if (e == hipSuccess) e = hipMemsetAsync(w + L.o_counts, 0, 8 * pt::PT_NCOUNTS * (size_t)S, h->stream);
    if (e == hipSuccess && L.log_cap > 0) e = hipMemsetAsync(w + L.o_elog, 0xFF, (size_t)S * L.log_cap, h->stream);
    if (e == hipSuccess && L.log_cap > 0) e = hipMemsetAsync(w + L.o_alog, 0, 8 * (size_t)L.words_total * L.log_cap, h->stream);
    if (e != hipSuccess) return fin(fail(PT_EHIP, "hipMemsetAsync: %s", hipGetErrorString(e)));
    // Starting energies in the FP64 order; their bounds seed the running bounds.
    for (const Class &cl : h->classes) {
        e = pt::launch_energy(cl.bpl, cl.wpr, T, cl.d_slots, cl.n_slots, T.e_run, T.b_run, h->stream);
        if (e != hipSuccess) return fin(fail(PT_EHIP, "energy launch failed: %s", hipGetErrorString(e)));
    }
    e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return fin(fail(PT_EHIP, "initialisation failed: %s", hipGetErrorString(e)));
    e = hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking);
    if (e != hipSuccess) return fin(fail(PT_EHIP, "hipStreamCreate: %s", hipGetErrorString(e)));
    *out = h;
    return PT_OK;
}

// Persistent run groups and task-flow classes: one launch each covers all n
// sweeps, exchanges included; they start at the device's run counters.  With
// ev, brackets every launch with an event pair.
int enqueue_persistent(pt_handle *h, int64_t n, hipStream_t s, std::vector<hipEvent_t> *ev, size_t *k) {
    for (const RunGroup &g : h->groups) {
        if (ev) PT_HIP(hipEventRecord((*ev)[2 * *k], s));
        hipError_t e = pt::launch_run(g.wpr, h->mixed, g.dense, h->T, g.d_list, g.n, g.max_bpl, n, s);
        if (e != hipSuccess) return fail(PT_EHIP, "persistent launch failed: %s", hipGetErrorString(e));
        if (ev) PT_HIP(hipEventRecord((*ev)[2 * *k + 1], s));
        if (k) ++*k;
    }
    for (const Class &c : h->classes) {
        if (!c.flow) continue;
        if (ev) PT_HIP(hipEventRecord((*ev)[2 * *k], s));
        hipError_t e = pt::launch_flow(c.bpl, c.wpr, h->mixed, h->T, c.d_slots, c.n_slots, n, c.resident, s);
        if (e != hipSuccess) return fail(PT_EHIP, "task-flow launch failed: %s", hipGetErrorString(e));
        if (ev) PT_HIP(hipEventRecord((*ev)[2 * *k + 1], s));
        if (k) ++*k;
    }
    return PT_OK;
}

bool any_per_sweep(const pt_handle *h) {
    for (const Class &c : h->classes)
        if (!c.whole()) return true;
    return false;
}

bool any_whole(const pt_handle *h) {
    for (const Class &c : h->classes)
        if (c.whole()) return true;
    return false;
}

void drop_graphs(pt_handle *h) {
    if (h->graph1) (void)hipGraphExecDestroy(h->graph1);
    if (h->graph16) (void)hipGraphExecDestroy(h->graph16);
    h->graph1 = h->graph16 = nullptr;
    for (auto &x : h->whole_graphs) (void)hipGraphExecDestroy(x.second);
    h->whole_graphs.clear();
}

// The graph of the persistent and task-flow launches of n sweeps (and of the
// counter update when no class runs one launch per sweep), captured on first
// use and kept for the last few sweep counts: every replay starts from the
// run counters in device memory, so one graph serves every call with that n.
int whole_graph(pt_handle *h, int64_t n, hipGraphExec_t *out) {
    for (auto &x : h->whole_graphs)
        if (x.first == n) {
            *out = x.second;
            return PT_OK;
        }
    hipGraph_t graph = nullptr;
    PT_HIP(hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal));
    int rc = enqueue_persistent(h, n, h->cap_stream, nullptr, nullptr);
    if (rc == PT_OK && !any_per_sweep(h)) {
        hipError_t e = pt::launch_advance_n(h->T, n, h->cap_stream);
        if (e != hipSuccess) rc = fail(PT_EHIP, "counter update failed: %s", hipGetErrorString(e));
    }
    hipError_t e = hipStreamEndCapture(h->cap_stream, &graph);
    if (rc != PT_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return rc;
    }
    if (e != hipSuccess) return fail(PT_EHIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
    hipGraphExec_t ex = nullptr;
    e = hipGraphInstantiate(&ex, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return fail(PT_EHIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
    constexpr size_t kKeep = 4;
    if (h->whole_graphs.size() >= kKeep) {
        // The stream may still replay the oldest graph: destroy it after that.
        PT_HIP(hipStreamSynchronize(h->stream));
        (void)hipGraphExecDestroy(h->whole_graphs.front().second);
        h->whole_graphs.erase(h->whole_graphs.begin());
    }
    h->whole_graphs.push_back({n, ex});
    *out = ex;
    return PT_OK;
}

PT_API int pt_sweep(pt_handle *h, int64_t n) {
    if (h == nullptr) return fail(PT_EINVAL, "NULL handle");
    if (h->failed) return fail(PT_ESTATE, "the handle failed earlier; restore a state with pt_set_state");
    if (n < 0) return fail(PT_EINVAL, "n_sweeps must be >= 0");
    if (n == 0) return PT_OK;
    int rc = PT_OK;
    if (any_whole(h)) {
        hipGraphExec_t g = nullptr;
        rc = whole_graph(h, n, &g);
        if (rc != PT_OK) return rc;
        PT_HIP(hipGraphLaunch(g, h->stream));
    }
    if (any_per_sweep(h)) {
        if (n >= 16 && h->graph16 == nullptr) {
            rc = capture(h, 16, &h->graph16);
            if (rc != PT_OK) return rc;
        }
        if (h->graph1 == nullptr) {
            rc = capture(h, 1, &h->graph1);
            if (rc != PT_OK) return rc;
        }
        int64_t left = n;
        while (left >= 16) {
            PT_HIP(hipGraphLaunch(h->graph16, h->stream));
            left -= 16;
        }
        while (left > 0) {
            PT_HIP(hipGraphLaunch(h->graph1, h->stream));
            left -= 1;
        }
    }
    advance_host(h, n);
    return PT_OK;
}

PT_API int pt_exchange(pt_handle *h) {
    if (h == nullptr) return fail(PT_EINVAL, "NULL handle");
    if (h->failed) return fail(PT_ESTATE, "the handle failed earlier; restore a state with pt_set_state");
    for (const Class &c : h->classes) {
        hipError_t e = pt::launch_exchange(c.bpl, c.wpr, h->T, c.d_chains, c.n_chains, c.max_pairs, 1, h->stream);
        if (e != hipSuccess) return fail(PT_EHIP, "exchange launch failed: %s", hipGetErrorString(e));
    }
    hipError_t e = pt::launch_advance(h->T, 1, h->stream);
    if (e != hipSuccess) return fail(PT_EHIP, "advance launch failed: %s", hipGetErrorString(e));
    h->e_host += 1;
    return PT_OK;
}

PT_API int pt_time_sweeps(pt_handle *h, int64_t n, double *sweep_ms, double *total_ms, int64_t *launches) {
    if (h == nullptr) return fail(PT_EINVAL, "NULL handle");
    if (h->failed) return fail(PT_ESTATE, "the handle failed earlier; restore a state with pt_set_state");
    if (n < 0) return fail(PT_EINVAL, "n_sweeps must be >= 0");
    size_t per = 0, pers = h->groups.size();
    for (const Class &c : h->classes) {
        if (c.flow) pers += 1;
        if (!c.whole()) per += 1;
    }
    const size_t nev = pers + (size_t)n * per;
    std::vector<hipEvent_t> ev(2 * nev + 2, nullptr);
    for (auto &x : ev) PT_HIP(hipEventCreate(&x));
    int rc = PT_OK;
    PT_HIP(hipEventRecord(ev[2 * nev], h->stream));
    size_t k = 0;
    if (n > 0) rc = enqueue_persistent(h, n, h->stream, &ev, &k);
    for (int64_t i = 0; i < n && rc == PT_OK && per > 0; ++i) {
        for (const Class &c : h->classes) {
            if (c.whole()) continue;
            PT_HIP(hipEventRecord(ev[2 * k], h->stream));
            hipError_t e = launch_class_sweep(h, c, h->stream);
            if (e != hipSuccess) { rc = fail(PT_EHIP, "sweep launch failed: %s", hipGetErrorString(e)); break; }
            PT_HIP(hipEventRecord(ev[2 * k + 1], h->stream));
            ++k;
        }
        for (const Class &c : h->classes) {
            if (c.whole() || rc != PT_OK) continue;
            hipError_t e = pt::launch_exchange(c.bpl, c.wpr, h->T, c.d_chains, c.n_chains, c.max_pairs, 0, h->stream);
            if (e != hipSuccess) rc = fail(PT_EHIP, "exchange launch failed: %s", hipGetErrorString(e));
        }
        if (rc == PT_OK) {
            hipError_t e = pt::launch_advance(h->T, 0, h->stream);
            if (e != hipSuccess) rc = fail(PT_EHIP, "advance launch failed: %s", hipGetErrorString(e));
        }
    }
    if (rc == PT_OK && n > 0) {
        if (per == 0) {
            hipError_t e = pt::launch_advance_n(h->T, n, h->stream);
            if (e != hipSuccess) rc = fail(PT_EHIP, "counter update failed: %s", hipGetErrorString(e));
        }
        advance_host(h, n);
    }
    PT_HIP(hipEventRecord(ev[2 * nev + 1], h->stream));
    PT_HIP(hipEventSynchronize(ev[2 * nev + 1]));
    if (rc == PT_OK) {
        double acc = 0.0;
        for (size_t i = 0; i < k; ++i) {
            float ms = 0.f;
            PT_HIP(hipEventElapsedTime(&ms, ev[2 * i], ev[2 * i + 1]));
            acc += ms;
        }
        float tot = 0.f;
        PT_HIP(hipEventElapsedTime(&tot, ev[2 * nev], ev[2 * nev + 1]));
        if (sweep_ms) *sweep_ms = acc;
        if (total_ms) *total_ms = tot;
        if (launches) *launches = (int64_t)k;
    }
    for (auto &x : ev) (void)hipEventDestroy(x);
    return rc;
}

// Reports a persistent run whose blocks stopped waiting for each other.
int check_err(pt_handle *h) {
    int32_t err = 0;
    PT_HIP(hipMemcpyAsync(&err, h->ws + h->L.o_err, 4, hipMemcpyDeviceToHost, h->stream));
    PT_HIP(hipStreamSynchronize(h->stream));
    if (err != 0) {
        h->failed = true;
        return fail(PT_EHIP, "a persistent or task-flow run timed out waiting for an exchange partner");
    }
    return PT_OK;
}

PT_API int pt_energy(pt_handle *h, double *h_e) {
    if (h == nullptr || h_e == nullptr) return fail(PT_EINVAL, "NULL argument");
    for (const Class &c : h->classes) {
        hipError_t e = pt::launch_energy(c.bpl, c.wpr, h->T, c.d_slots, c.n_slots, h->d_tmp, nullptr, h->stream);
        if (e != hipSuccess) return fail(PT_EHIP, "energy launch failed: %s", hipGetErrorString(e));
    }
    PT_HIP(hipMemcpyAsync(h_e, h->d_tmp, 8 * (size_t)h->L.total, hipMemcpyDeviceToHost, h->stream));
    PT_HIP(hipStreamSynchronize(h->stream));
    return check_err(h);
}

PT_API int pt_energy_method(pt_handle *h, int32_t method, double *h_e, double *h_b, double *kernel_ms) {
    if (h == nullptr || h_e == nullptr) return fail(PT_EINVAL, "NULL argument");
    if (method != PT_ENERGY_FP64_ORDER && method != PT_ENERGY_PAIR_PER_THREAD)
        return fail(PT_EINVAL, "unknown energy method %d", method);
    const size_t S = (size_t)h->L.total;
    double *d_e = h->d_tmp, *d_b = h->d_tmp + S;
    hipEvent_t ev[2] = {nullptr, nullptr};
    PT_HIP(hipEventCreate(&ev[0]));
    PT_HIP(hipEventCreate(&ev[1]));
    int rc = PT_OK;
    PT_HIP(hipEventRecord(ev[0], h->stream));
    for (const Class &c : h->classes) {
        hipError_t e = method == PT_ENERGY_FP64_ORDER
                           ? pt::launch_energy(c.bpl, c.wpr, h->T, c.d_slots, c.n_slots, d_e, nullptr, h->stream)
                           : pt::launch_energy_pairs(c.bpl, c.wpr, h->T, c.d_slots, c.n_slots, d_e, d_b, h->stream);
        if (e != hipSuccess) {
            rc = fail(PT_EHIP, "energy launch failed: %s", hipGetErrorString(e));
            break;
        }
    }
    PT_HIP(hipEventRecord(ev[1], h->stream));
    if (rc == PT_OK) {
        PT_HIP(hipMemcpyAsync(h_e, d_e, 8 * S, hipMemcpyDeviceToHost, h->stream));
        if (h_b && method == PT_ENERGY_PAIR_PER_THREAD)
            PT_HIP(hipMemcpyAsync(h_b, d_b, 8 * S, hipMemcpyDeviceToHost, h->stream));
        PT_HIP(hipStreamSynchronize(h->stream));
        float ms = 0.f;
        PT_HIP(hipEventElapsedTime(&ms, ev[0], ev[1]));
        if (kernel_ms) *kernel_ms = ms;
        if (h_b && method == PT_ENERGY_FP64_ORDER) {
            // The a-priori bound of the FP64 order, as the kernels compute it.
            for (int c = 0, g = 0; c < h->L.n_chains; ++c) {
                const int n = h->n_beads[c];
                const int lg = 32 - __builtin_clz((unsigned)(n - 1));
                const double pairs = 0.5 * (double)n * (double)(n - 1);
                for (int s = 0; s < h->n_slots[c]; ++s, ++g)
                    h_b[g] = 0x1p-51 * (double)(2 * lg + 4) * (fabs(h_e[g]) + 2.0 * pairs * h->k.neg_floor);
            }
        }
    }
    (void)hipEventDestroy(ev[0]);
    (void)hipEventDestroy(ev[1]);
    if (rc != PT_OK) return rc;
    return check_err(h);
}

PT_API int pt_observables(pt_handle *h, double *acc, int64_t *counts, int32_t *perm, int64_t *te) {
    if (h == nullptr) return fail(PT_EINVAL, "NULL handle");
    const size_t S = (size_t)h->L.total;
    if (acc) PT_HIP(hipMemcpyAsync(acc, h->ws + h->L.o_acc, 8 * 5 * S, hipMemcpyDeviceToHost, h->stream));
    if (counts) PT_HIP(hipMemcpyAsync(counts, h->ws + h->L.o_counts, 8 * pt::PT_NCOUNTS * S, hipMemcpyDeviceToHost, h->stream));
    if (perm) PT_HIP(hipMemcpyAsync(perm, h->ws + h->L.o_perm, 4 * S, hipMemcpyDeviceToHost, h->stream));
    if (te) PT_HIP(hipMemcpyAsync(te, h->ws + h->L.o_te, 16, hipMemcpyDeviceToHost, h->stream));
    PT_HIP(hipStreamSynchronize(h->stream));
    return check_err(h);
}

PT_API int pt_reset_observables(pt_handle *h) {
    if (h == nullptr) return fail(PT_EINVAL, "NULL handle");
    PT_HIP(hipMemsetAsync(h->ws + h->L.o_acc, 0, 8 * 5 * (size_t)h->L.total, h->stream));
    return PT_OK;
}

PT_API int pt_get_coords(pt_handle *h, double *out) {
    if (h == nullptr || out == nullptr) return fail(PT_EINVAL, "NULL argument");
    std::vector<double> sw((size_t)h->L.coord_total);
    PT_HIP(hipMemcpyAsync(sw.data(), h->ws + h->L.o_coords, 8 * sw.size(), hipMemcpyDeviceToHost, h->stream));
    PT_HIP(hipStreamSynchronize(h->stream));
    int g = 0;
    int64_t dst = 0;
    for (int ch = 0; ch < h->L.n_chains; ++ch) {
        const int n = h->n_beads[ch], B = h->L.bpl[ch], W = h->L.wpr[ch], NP = 64 * W * B;
        for (int s = 0; s < h->n_slots[ch]; ++s, ++g) {
            const double *src = sw.data() + h->L.coord_off[g];
            for (int j = 0; j < n; ++j) {
                const int p = swizzle(j, B, W);
                out[dst + 3 * j] = src[p];
                out[dst + 3 * j + 1] = src[NP + p];
                out[dst + 3 * j + 2] = src[2 * NP + p];
            }
            dst += 3 * (int64_t)n;
        }
    }
    return PT_OK;
}

PT_API int pt_get_running(pt_handle *h, double *he, double *hb) {
    if (h == nullptr) return fail(PT_EINVAL, "NULL handle");
    const size_t S = (size_t)h->L.total;
    if (he) PT_HIP(hipMemcpyAsync(he, h->ws + h->L.o_e_run, 8 * S, hipMemcpyDeviceToHost, h->stream));
    if (hb) PT_HIP(hipMemcpyAsync(hb, h->ws + h->L.o_b_run, 8 * S, hipMemcpyDeviceToHost, h->stream));
    PT_HIP(hipStreamSynchronize(h->stream));
    return PT_OK;
}

PT_API int pt_get_series(pt_handle *h, double *out, int64_t *rows) {
    if (h == nullptr) return fail(PT_EINVAL, "NULL handle");
    const int64_t r = std::min<int64_t>(h->t_host, h->L.series_cap);
    if (rows) *rows = r;
    if (out && r > 0)
        PT_HIP(hipMemcpyAsync(out, h->ws + h->L.o_series, 8 * 3 * (size_t)h->L.total * r, hipMemcpyDeviceToHost, h->stream));
    PT_HIP(hipStreamSynchronize(h->stream));
    return PT_OK;
}

PT_API int pt_get_logs(pt_handle *h, uint64_t *alog, int64_t *arows, uint8_t *elog, int64_t *erows) {
    if (h == nullptr) return fail(PT_EINVAL, "NULL handle");
    const int64_t ra = std::min<int64_t>(h->t_host, h->L.log_cap);
    const int64_t re = std::min<int64_t>(h->e_host, h->L.log_cap);
    if (arows) *arows = ra;
    if (erows) *erows = re;
    if (alog && ra > 0)
        PT_HIP(hipMemcpyAsync(alog, h->ws + h->L.o_alog, 8 * (size_t)h->L.words_total * ra, hipMemcpyDeviceToHost, h->stream));
    if (elog && re > 0)
        PT_HIP(hipMemcpyAsync(elog, h->ws + h->L.o_elog, (size_t)h->L.total * re, hipMemcpyDeviceToHost, h->stream));
    PT_HIP(hipStreamSynchronize(h->stream));
    return PT_OK;
}

PT_API int pt_get_mapping(pt_handle *h, int32_t *bpl, int32_t *wpr, int32_t *persistent) {
    if (h == nullptr) return fail(PT_EINVAL, "NULL handle");
    for (int c = 0; c < h->L.n_chains; ++c) {
        if (bpl) bpl[c] = h->L.bpl[c];
        if (wpr) wpr[c] = h->L.wpr[c];
        if (persistent) {
            persistent[c] = 0;
            for (const Class &cl : h->classes)
                if (cl.bpl == h->L.bpl[c] && cl.wpr == h->L.wpr[c] && cl.lane == (h->L.lane[c] != 0) &&
                    cl.pack == h->L.pack[c])
                    persistent[c] = cl.persistent ? 1 : cl.flow ? 2 : 0;
        }
    }
    return PT_OK;
}

// Arguments of a pt_selftest call: validation and the sizes (doubles) of its
// input, second input and output arrays.
static int selftest_args(const pt_model *model, int op, const double *hx, const double *hout, int64_t n, size_t *nin,
                  size_t *ny, size_t *nout) {
    if (model == nullptr || hx == nullptr || hout == nullptr || n < 0) return fail(PT_EINVAL, "bad argument");
    if (op < 0 || op > 9) return fail(PT_EINVAL, "unknown op %d", op);
    if ((op == 7 || op == 8) && n % 64 != 0) return fail(PT_EINVAL, "op %d needs n a multiple of 64", op);
    if (op == 9) {
        for (int64_t i = 0; i < n; ++i) {
            const double nb = hx[i * pt::kMoveItem + 3 * 512], kk = hx[i * pt::kMoveItem + 3 * 512 + 1];
            if (!(nb >= 2 && nb <= 512 && nb == (int)nb && kk >= 0 && kk < nb && kk == (int)kk))
                return fail(PT_EINVAL, "op 9 item %lld: N in [2, 512] and 0 <= k < N, integers", (long long)i);
        }
    }
    *nin = (op == 6) ? 4 * (size_t)n : (op == 9) ? (size_t)pt::kMoveItem * n : (size_t)n;
    *ny = (op == 6) ? 2 : (op == 9) ? 1 : (size_t)n;
    *nout = (op == 5 || op == 9) ? 2 * (size_t)n : (op == 6) ? 4 * (size_t)n : (size_t)n;
    return PT_OK;
}

PT_API int pt_selftest(const pt_model *model, int op, const double *hx, const double *hy, double *hout, int64_t n) {
    size_t nin = 0, ny = 0, nout = 0;
    const int rc = selftest_args(model, op, hx, hout, n, &nin, &ny, &nout);
    if (rc != PT_OK || n == 0) return rc;
    const pt::Consts k = make_consts(model, 0x1p-10);
    double *dx = nullptr, *dy = nullptr, *dout = nullptr;
    std::vector<double> zeros;
    if (hy == nullptr) {
        zeros.assign(ny, 0.0);
        hy = zeros.data();
    }
    PT_HIP(hipMalloc(&dx, 8 * nin));
    hipError_t e = hipMalloc(&dy, 8 * ny);
    if (e == hipSuccess) e = hipMalloc(&dout, 8 * nout);
    if (e == hipSuccess) e = hipMemcpy(dx, hx, 8 * nin, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(dy, hy, 8 * ny, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = pt::launch_selftest(k, op, dx, dy, dout, n, nullptr);
    if (e == hipSuccess) e = hipMemcpy(hout, dout, 8 * nout, hipMemcpyDeviceToHost);
    (void)hipFree(dx);
    (void)hipFree(dy);
    (void)hipFree(dout);
    if (e != hipSuccess) return fail(PT_EHIP, "selftest failed: %s", hipGetErrorString(e));
    return PT_OK;
}

// ------------------------------------------------- no-allocation variant --
// Staging of pt_selftest_noalloc: a file-scope device array instead of
// hipMalloc'd buffers.  Every GPU the library runs on holds its own copy
// until the process ends.  In host code the array's name is not a device
// address: host code uses only the address hipGetSymbolAddress gives for the
// current device (kept per device below), never the name itself.
constexpr size_t kScratchDoubles = (size_t)1 << 21;  // 16 MiB per device
static __device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static double *g_scratch_ptr[kMaxDevices];

// Device address of the current device's scratch array, looked up on the
// first call on that device.
static int scratch_base(double **out) {
    int dev = 0;
    PT_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(PT_EINVAL, "device %d beyond the %d supported", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[dev] == nullptr) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || p == nullptr)
            return fail(PT_EHIP, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
        g_scratch_ptr[dev] = (double *)p;
    }
    *out = g_scratch_ptr[dev];
    return PT_OK;
}

PT_API int pt_selftest_noalloc(const pt_model *model, int op, const double *hx, const double *hy, double *hout,
                               int64_t n) {
    size_t nin = 0, ny = 0, nout = 0;
    int rc = selftest_args(model, op, hx, hout, n, &nin, &ny, &nout);
    if (rc != PT_OK || n == 0) return rc;
    // Only ops 1, 5 and 6 read the second input.
    const size_t ny_used = (op == 1 || op == 5 || op == 6) ? ny : 0;
    if (nin + ny_used + nout > kScratchDoubles)
        return fail(PT_EINVAL, "op %d with n = %lld needs %zu doubles of staging; the no-allocation buffer holds %zu",
                    op, (long long)n, nin + ny_used + nout, kScratchDoubles);
    double *base = nullptr;
    rc = scratch_base(&base);
    if (rc != PT_OK) return rc;
    double *dx = base, *dy = base + nin, *dout = base + nin + ny_used;
    const pt::Consts k = make_consts(model, 0x1p-10);
    PT_HIP(hipMemcpy(dx, hx, 8 * nin, hipMemcpyHostToDevice));
    if (ny_used > 0) {
        // The array keeps the previous call's contents: a missing second
        // input is cleared to zeros, as pt_selftest takes it.
        if (hy != nullptr) PT_HIP(hipMemcpy(dy, hy, 8 * ny_used, hipMemcpyHostToDevice));
        else PT_HIP(hipMemset(dy, 0, 8 * ny_used));
    }
    PT_HIP(pt::launch_selftest(k, op, dx, ny_used > 0 ? dy : nullptr, dout, n, nullptr));
    PT_HIP(hipMemcpy(hout, dout, 8 * nout, hipMemcpyDeviceToHost));
    return PT_OK;
}

PT_API void pt_destroy(pt_handle *h) {
    if (h == nullptr) return;
    // Work enqueued on the caller's stream may still replay the handle's
    // graphs: wait for it before they go.
    (void)hipStreamSynchronize(h->stream);
    drop_graphs(h);
    if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
    delete h;
}

PT_API const char *pt_last_error(void) { return g_err.c_str(); }

// ------------------------------------------------------------ state I/O --
namespace {

constexpr uint64_t kStateMagic = 0x3145544154535450ull;  // "PTSTATE1"

struct StateHeader {
    uint64_t magic;
    int32_t n_chains, precision;
    int64_t total, coord_doubles, t, e;
    uint64_t seed;
};

size_t state_bytes(const pt_handle *h) {
    const size_t C = (size_t)h->L.n_chains, S = (size_t)h->L.total;
    size_t cd = 0;
    for (size_t c = 0; c < C; ++c) cd += 3 * (size_t)h->n_beads[c] * (size_t)h->n_slots[c];
    return sizeof(StateHeader) + 8 * C + 8 * ((4 * S + 7) / 8) + 8 * cd + 8 * S * (2 + 5 + pt::PT_NCOUNTS + 2);
}

}  // namespace

PT_API size_t pt_state_bytes(pt_handle *h) {
    if (h == nullptr) {
        fail(PT_EINVAL, "NULL handle");
        return 0;
    }
    return state_bytes(h);
}

PT_API int pt_get_digests(pt_handle *h, uint64_t *h_dig) {
    if (h == nullptr || h_dig == nullptr) return fail(PT_EINVAL, "NULL argument");
    PT_HIP(hipMemcpyAsync(h_dig, h->ws + h->L.o_dig, 16 * (size_t)h->L.total, hipMemcpyDeviceToHost, h->stream));
    PT_HIP(hipStreamSynchronize(h->stream));
    return PT_OK;
}

PT_API int pt_get_state(pt_handle *h, void *buf, size_t bytes) {
    if (h == nullptr || buf == nullptr) return fail(PT_EINVAL, "NULL argument");
    const size_t need = state_bytes(h);
    if (bytes < need) return fail(PT_ENOMEM, "state buffer of %zu bytes is smaller than the %zu needed", bytes, need);
    const int C = h->L.n_chains, S = h->L.total;
    char *p = (char *)buf;
    std::memset(p, 0, need);
    StateHeader hd{};
    hd.magic = kStateMagic;
    hd.n_chains = C;
    hd.precision = h->mixed ? PT_MIXED : PT_FP64;
    hd.total = S;
    hd.t = h->t_host;
    hd.e = h->e_host;
    hd.seed = h->seed;
    size_t cd = 0;
    for (int c = 0; c < C; ++c) cd += 3 * (size_t)h->n_beads[c] * (size_t)h->n_slots[c];
    hd.coord_doubles = (int64_t)cd;
    std::memcpy(p, &hd, sizeof hd);
    p += sizeof hd;
    std::memcpy(p, h->n_beads.data(), 4 * (size_t)C);
    std::memcpy(p + 4 * (size_t)C, h->n_slots.data(), 4 * (size_t)C);
    p += 8 * (size_t)C;
    int32_t *perm = (int32_t *)p;
    p += 8 * ((4 * (size_t)S + 7) / 8);
    double *coords = (double *)p;
    p += 8 * cd;
    double *e_run = (double *)p, *b_run = e_run + S, *acc = b_run + S;
    int64_t *counts = (int64_t *)(acc + 5 * (size_t)S);
    uint64_t *dig = (uint64_t *)(counts + pt::PT_NCOUNTS * (size_t)S);
    int rc = pt_observables(h, acc, counts, perm, nullptr);
    if (rc == PT_OK) rc = pt_get_running(h, e_run, b_run);
    if (rc == PT_OK) rc = pt_get_coords(h, coords);
    if (rc == PT_OK) rc = pt_get_digests(h, dig);
    return rc;
}

PT_API int pt_set_state(pt_handle *h, const void *buf, size_t bytes) {
    if (h == nullptr || buf == nullptr) return fail(PT_EINVAL, "NULL argument");
    const size_t need = state_bytes(h);
    if (bytes < need) return fail(PT_EINVAL, "state of %zu bytes is shorter than the %zu this handle needs", bytes, need);
    const int C = h->L.n_chains, S = h->L.total;
    const char *p = (const char *)buf;
    StateHeader hd;
    std::memcpy(&hd, p, sizeof hd);
    if (hd.magic != kStateMagic) return fail(PT_EINVAL, "not a saved state");
    if (hd.n_chains != C || hd.total != S || hd.seed != h->seed)
        return fail(PT_EINVAL, "the state belongs to another batch (chains, slots or seed differ)");
    if (hd.t < 0 || hd.e < 0) return fail(PT_EINVAL, "negative run counters in the state");
    p += sizeof hd;
    const int32_t *nb = (const int32_t *)p, *ns = nb + C;
    for (int c = 0; c < C; ++c)
        if (nb[c] != h->n_beads[c] || ns[c] != h->n_slots[c])
            return fail(PT_EINVAL, "chain %d: beads or slots differ from this handle's", c);
    p += 8 * (size_t)C;
    const int32_t *perm = (const int32_t *)p;
    p += 8 * ((4 * (size_t)S + 7) / 8);
    const double *coords = (const double *)p;
    p += 8 * (size_t)hd.coord_doubles;
    const double *e_run = (const double *)p, *b_run = e_run + S, *acc = b_run + S;
    const int64_t *counts = (const int64_t *)(acc + 5 * (size_t)S);
    const uint64_t *dig = (const uint64_t *)(counts + pt::PT_NCOUNTS * (size_t)S);
    // Permutation within each chain's slots; coordinates finite with intact bonds.
    std::vector<int32_t> slot_of(S, -1);
    std::vector<double> swz((size_t)h->L.coord_total);
    {
        int g = 0;
        int64_t src = 0;
        for (int c = 0; c < C; ++c) {
            const int n = h->n_beads[c], B = h->L.bpl[c], W = h->L.wpr[c], NP = 64 * W * B;
            const int g0 = g;
            for (int s = 0; s < h->n_slots[c]; ++s, ++g) {
                const int q = perm[g];
                if (q < g0 || q >= g0 + h->n_slots[c] || slot_of[q] >= 0)
                    return fail(PT_EINVAL, "slot %d: the permutation is not one of chain %d's slots", g, c);
                slot_of[q] = g;
                const double *xyz = coords + src;  // conformation g (started in slot g)
                for (int j = 0; j < 3 * n; ++j)
                    if (!isfinite(xyz[j])) return fail(PT_EINVAL, "conformation %d: non-finite coordinate", g);
                for (int j = 0; j + 1 < n; ++j)
                    if (!(fene_y(h->k, xyz + 3 * j, xyz + 3 * (j + 1)) > 0.0))
                        return fail(PT_EDOMAIN, "conformation %d: bond (%d,%d) at or beyond r0 +- R", g, j, j + 1);
                double *dst = swz.data() + h->L.coord_off[g];
                for (int j = 0; j < NP; ++j) {
                    const int pp = swizzle(j, B, W);
                    dst[pp] = (j < n) ? xyz[3 * j] : kSentinel;
                    dst[NP + pp] = (j < n) ? xyz[3 * j + 1] : 0.0;
                    dst[2 * NP + pp] = (j < n) ? xyz[3 * j + 2] : 0.0;
                }
                src += 3 * (int64_t)n;
            }
        }
    }
    char *w = h->ws;
    const int64_t te[2] = {hd.t, hd.e};
    auto up = [&](size_t off, const void *src, size_t n) {
        return hipMemcpyAsync(w + off, src, n, hipMemcpyHostToDevice, h->stream);
    };
    hipError_t e = up(h->L.o_coords, swz.data(), 8 * swz.size());
    if (e == hipSuccess) e = up(h->L.o_perm, perm, 4 * (size_t)S);
    if (e == hipSuccess) e = up(h->L.o_slot_of, slot_of.data(), 4 * (size_t)S);
    if (e == hipSuccess) e = up(h->L.o_e_run, e_run, 8 * (size_t)S);
    if (e == hipSuccess) e = up(h->L.o_b_run, b_run, 8 * (size_t)S);
    if (e == hipSuccess) e = up(h->L.o_acc, acc, 8 * 5 * (size_t)S);
    if (e == hipSuccess) e = up(h->L.o_counts, counts, 8 * pt::PT_NCOUNTS * (size_t)S);
    if (e == hipSuccess) e = up(h->L.o_dig, dig, 16 * (size_t)S);
    if (e == hipSuccess) e = up(h->L.o_te, te, 16);
    // Pair flags of the persistent schedule are keyed by sweep index, the task
    // flow's by sweep index and arrival count: clear them.
    if (e == hipSuccess) e = hipMemsetAsync(w + h->L.o_done, 0, 8 * (size_t)S, h->stream);
    if (e == hipSuccess) e = hipMemsetAsync(w + h->L.o_flow_ready, 0, 8 * (size_t)S, h->stream);
    if (e == hipSuccess) e = hipMemsetAsync(w + h->L.o_flow_arr, 0, 8 * (size_t)S, h->stream);
    if (e == hipSuccess) e = hipMemsetAsync(w + h->L.o_dec, 0, 8 * (size_t)S, h->stream);
    if (e == hipSuccess) e = hipMemsetAsync(w + h->L.o_err, 0, 16, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return fail(PT_EHIP, "state upload failed: %s", hipGetErrorString(e));
    h->t_host = hd.t;
    h->e_host = hd.e;
    h->failed = false;
    return PT_OK;
}

// -------------------------------------------------------------- autotune --
// A timing of trial_sweeps sweeps; one that comes within 3% of the best so
// far (best_ms > 0) is taken twice more and the fastest kept: close candidates
// can differ by 1-2%, about the spread of one timing.
static int time_close(pt_handle *h, int64_t trial_sweeps, double best_ms, double *ms) {
    for (int rep = 0; rep < 3; ++rep) {
        double m = 0.0;
        const int r = pt_time_sweeps(h, trial_sweeps, nullptr, &m, nullptr);
        if (r != PT_OK) return r;
        if (rep == 0 || m < *ms) *ms = m;
        if (best_ms > 0.0 && *ms > 1.03 * best_ms) break;
    }
    return PT_OK;
}

PT_API int pt_autotune(const pt_model *model, const pt_config *cfg, int32_t trial_sweeps, void *hip_stream,
                       int32_t *out) {
    int rc = validate(model, cfg);
    if (rc != PT_OK) return rc;
    if (out == nullptr || trial_sweeps < 1) return fail(PT_EINVAL, "mapping_out must be non-NULL and trial_sweeps >= 1");
    const int C = cfg->n_chains;
    // Offsets of each chain's slots and coordinates in the caller's arrays.
    std::vector<int64_t> slot0(C + 1, 0), coord0(C + 1, 0);
    for (int c = 0; c < C; ++c) {
        slot0[c + 1] = slot0[c] + cfg->n_slots[c];
        coord0[c + 1] = coord0[c] + 3 * (int64_t)cfg->n_beads[c] * cfg->n_slots[c];
    }
    std::map<int, std::vector<int>> by_n;
    for (int c = 0; c < C; ++c) by_n[cfg->n_beads[c]].push_back(c);
    std::map<int, std::vector<std::pair<int, double>>> timed;  // length -> (code, ms)
    for (auto &kv : by_n) {
        const int n = kv.first;
        const std::vector<int> &chains = kv.second;
        std::vector<int> cand;
        for (int W : {1, 2, 4})
            for (int B : {1, 2, 4, 8}) {
                const int np = 64 * W * B;
                if (np >= n && np < std::max(65, 4 * n)) cand.push_back(16 * B + W);
            }
        // Short chains can share a wavefront, two or four replicas of 32 or 16 lanes.
        for (int B : {1, 2})
            if (64 * B >= n && 64 * B < std::max(65, 4 * n))
                for (int f : {PT_MAP_PACK2, PT_MAP_PACK4}) cand.push_back(f | (16 * B + 1));
        // The FP64 order can also run one lane per replica (in the default layout).
        if (cfg->precision == PT_FP64) {
            int b = 0, w = 0;
            mapping(n, &b, &w);
            cand.push_back(PT_MAP_LANE | (16 * b + w));
        }
        int best = 0;
        if (cand.size() == 1) {
            best = cand[0];
        } else {
            // The chains of this length as a batch of their own.
            std::vector<int32_t> nb, ns, mp;
            std::vector<uint32_t> sc, s0;
            std::vector<double> beta, xyz;
            for (int c : chains) {
                nb.push_back(cfg->n_beads[c]);
                ns.push_back(cfg->n_slots[c]);
                sc.push_back(cfg->stream_chain ? cfg->stream_chain[c] : (uint32_t)c);
                s0.push_back(cfg->stream_slot0 ? cfg->stream_slot0[c] : (uint32_t)slot0[c]);
                beta.insert(beta.end(), cfg->beta + slot0[c], cfg->beta + slot0[c + 1]);
                xyz.insert(xyz.end(), cfg->coords + coord0[c], cfg->coords + coord0[c + 1]);
            }
            pt_config t = *cfg;
            t.n_chains = (int32_t)chains.size();
            t.n_beads = nb.data();
            t.n_slots = ns.data();
            t.beta = beta.data();
            t.coords = xyz.data();
            t.stream_chain = sc.data();
            t.stream_slot0 = s0.data();
            t.series_capacity = 0;
            t.log_capacity = 0;
            double best_ms = 0.0;
            for (int code : cand) {
                mp.assign(chains.size(), code);
                t.mapping = mp.data();
                const size_t bytes = plan(&t).bytes;
                void *ws = nullptr;
                if (hipMalloc(&ws, bytes) != hipSuccess) return fail(PT_ENOMEM, "autotune: no room for %zu bytes", bytes);
                pt_handle *h = nullptr;
                rc = pt_init(model, &t, ws, bytes, hip_stream, &h);
                double ms = 0.0;
                if (rc == PT_OK) rc = pt_sweep(h, std::min<int64_t>(trial_sweeps, 4));
                if (rc == PT_OK) rc = time_close(h, trial_sweeps, best == 0 ? 0.0 : best_ms, &ms);
                if (h) pt_destroy(h);
                (void)hipFree(ws);
                if (rc != PT_OK) return rc;
                timed[n].push_back({code, ms});
                if (best == 0 || ms < best_ms) {
                    best = code;
                    best_ms = ms;
                }
            }
        }
        for (int c : chains) out[c] = best;
    }
    // Persistent classes of one wavefront count share a launch, but launches
    // of different wavefront counts run one after another, so a batch split
    // over several counts adds their times.  Candidates for the whole batch:
    // the per-length choices above, and for each wavefront count W every
    // length on its fastest timed mapping with W (or the smallest bead count
    // that holds it at W); the fastest batch wins.
    if ((cfg->schedule & ~kSchedFlags) != PT_SCHED_PER_SWEEP) {
        pt_config t = *cfg;
        t.series_capacity = 0;
        t.log_capacity = 0;
        auto time_batch = [&](const std::vector<int32_t> &m, double *ms) -> int {
            t.mapping = m.data();
            const size_t bytes = plan(&t).bytes;
            void *ws = nullptr;
            if (hipMalloc(&ws, bytes) != hipSuccess) return fail(PT_ENOMEM, "autotune: no room for %zu bytes", bytes);
            pt_handle *h = nullptr;
            int r = pt_init(model, &t, ws, bytes, hip_stream, &h);
            if (r == PT_OK) r = pt_sweep(h, std::min<int64_t>(trial_sweeps, 4));
            if (r == PT_OK) r = time_close(h, trial_sweeps, *ms, ms);
            if (h) pt_destroy(h);
            (void)hipFree(ws);
            return r;
        };
        std::vector<std::vector<int32_t>> cands = {std::vector<int32_t>(out, out + C)};
        for (int W : {1, 2, 4}) {
            std::vector<int32_t> m(C, 0);
            bool ok = true, differs = false;
            for (int c = 0; c < C && ok; ++c) {
                const int n = cfg->n_beads[c];
                int code = 0;
                double best_ms = 0.0;
                for (const auto &x : timed[n])
                    if ((x.first & ~0xFF) == 0 && (x.first & 15) == W && (code == 0 || x.second < best_ms)) {
                        code = x.first;
                        best_ms = x.second;
                    }
                if (code == 0) {
                    int b = 1;
                    while (b < 8 && 64 * W * b < n) b <<= 1;
                    if (64 * W * b < n) ok = false;
                    code = 16 * b + W;
                }
                m[c] = code;
                differs = differs || code != out[c];
            }
            if (ok && differs) cands.push_back(m);
        }
        if (cands.size() > 1) {
            size_t best = 0;
            double best_ms = 0.0;
            for (size_t i = 0; i < cands.size(); ++i) {
                double ms = best_ms;  // in: the best so far (0: none); out: this candidate's
                rc = time_batch(cands[i], &ms);
                if (rc != PT_OK) return rc;
                if (i == 0 || ms < best_ms) {
                    best = i;
                    best_ms = ms;
                }
            }
            std::copy(cands[best].begin(), cands[best].end(), out);
        }
    }
    return PT_OK;
}

PT_API int pt_set_spin_limit(pt_handle *h, uint32_t polls) {
    if (h == nullptr || polls < 1) return fail(PT_EINVAL, "NULL handle or zero polls");
    // Graphs hold the kernel arguments of their capture: capture them anew.
    PT_HIP(hipStreamSynchronize(h->stream));
    drop_graphs(h);
    h->T.spin_limit = polls;
    return PT_OK;
}

PT_API int pt_set_guard_scale(pt_handle *h, double factor) {
    if (h == nullptr || !(isfinite(factor) && factor >= 1.0))
        return fail(PT_EINVAL, "NULL handle, or a guard scale that is not a finite number >= 1");
    PT_HIP(hipStreamSynchronize(h->stream));
    drop_graphs(h);
    h->T.guard_scale = factor;
    return PT_OK;
}
