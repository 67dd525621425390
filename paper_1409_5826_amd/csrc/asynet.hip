// Host side of the asynet C ABI: descriptor validation, incidence layouts,
// device upload, launch configuration, graph replay and autotuning.  See
// include/asynet.h for the contract of every entry point.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "asynet.h"
#include "integrate_kernels.h"
#include "stratified_kernel.h"

using namespace asynet;

namespace {

thread_local std::string g_last_error;

asy_status fail(asy_status st, const std::string &msg)
{
    g_last_error = msg;
    return st;
}

#define HIP_TRY(expr)                                                                    \
    do {                                                                                 \
        hipError_t e_ = (expr);                                                          \
        if (e_ != hipSuccess)                                                            \
            return fail(e_ == hipErrorOutOfMemory ? ASY_ENOMEM : ASY_EDEVICE,            \
                        std::string(#expr) + ": " + hipGetErrorString(e_));              \
    } while (0)

// Layout of variant 1 for one choice of waves per zone.
struct StratLayout {
    int W = 0, lanes = 0, K = 0, C_needed = 0, C = 0, SPL = 0;
    void *dev = nullptr;
    StratNetwork sn{};
    bool ok = false;
};

// Captured launch sequence for repeated identical calls.
struct GraphCache {
    hipGraphExec_t exec = nullptr;
    std::vector<uint8_t> key;
};

}  // namespace

struct asy_network {
    int32_t n_species = 0;
    int32_t n_reactions = 0;
    int32_t n_destruction = 0;
    int32_t rate_form = ASY_RATES_PER_ZONE;
    int device = 0;
    int n_cu = 0;
    size_t lds_per_group_max = 0;
    void *dev_block = nullptr;  // network structure (variant 0) and the zone queue
    int32_t *queue = nullptr;
    DevNetwork dn{};
    StratLayout strat[3];       // variant 1 with W = 1, 2, 4
    double *rate_buf = nullptr; // Arrhenius rates of one call, [zones][reactions]
    size_t rate_buf_zones = 0;
    float *key_buf = nullptr;   // scheduling keys of one call, [zones]
    int32_t *order_buf = nullptr; // scheduling order of one call, [zones]
    size_t order_buf_zones = 0;
    asy_launch launch{};
    hipStream_t capture_stream = nullptr;
    GraphCache graph;
};

namespace {

// ---- variant 1 kernel instances -----------------------------------------------------------

using StratKernel = void (*)(StratNetwork, DevOptions, ZoneArgs, const double *, const int32_t *);

struct StratInstance {
    int W, SPL, C;
    StratKernel fn;
};

#define ASY_STRAT(W_, SPL_, C_) {W_, SPL_, C_, integrate_strat_kernel<W_, SPL_, C_>}
const StratInstance kStratInstances[] = {
    ASY_STRAT(1, 1, 16), ASY_STRAT(1, 1, 32), ASY_STRAT(1, 2, 32), ASY_STRAT(1, 2, 64),
    ASY_STRAT(1, 3, 64), ASY_STRAT(1, 3, 104), ASY_STRAT(1, 3, 112), ASY_STRAT(1, 4, 64),
    ASY_STRAT(2, 1, 32), ASY_STRAT(2, 2, 48), ASY_STRAT(2, 2, 64), ASY_STRAT(2, 2, 72),
    ASY_STRAT(2, 2, 80), ASY_STRAT(2, 3, 64), ASY_STRAT(2, 3, 96), ASY_STRAT(2, 3, 136),
    ASY_STRAT(4, 1, 32), ASY_STRAT(4, 1, 48), ASY_STRAT(4, 1, 56), ASY_STRAT(4, 1, 64),
    ASY_STRAT(4, 2, 48), ASY_STRAT(4, 2, 64), ASY_STRAT(4, 2, 80), ASY_STRAT(4, 2, 96),
};
#undef ASY_STRAT

const StratInstance *find_strat_instance(int W, int SPL, int C_needed)
{
    const StratInstance *best = nullptr;
    for (const auto &in : kStratInstances)
        if (in.W == W && in.SPL == SPL && in.C >= C_needed && (!best || in.C < best->C))
            best = &in;
    return best;
}

int w_index(int W) { return W == 1 ? 0 : (W == 2 ? 1 : 2); }

// Rows of the network: row i (< N) sums the creation flux of species i, row
// N + i its depletion rate; terms in ascending reaction index.  A term is
// (rx, x, y) with x, y LDS cells of Y (cell N holds 1.0).
struct Term {
    int32_t rx, x, y;
};

std::vector<std::vector<Term>> network_rows(int N, int R, const int32_t *r0, const int32_t *r1,
                                            const int32_t *pr)
{
    std::vector<std::vector<Term>> rows(2 * (size_t)N);
    for (int j = 0; j < R; ++j) {  // ascending j keeps every row in reaction order
        const int a = r0[j], b = r1[j], c = pr[j];
        rows[c].push_back({j, a, b >= 0 ? b : N});
        rows[N + a].push_back({j, b >= 0 ? b : N, N});
        if (b >= 0)
            rows[N + b].push_back({j, a, N});
    }
    return rows;
}

// Deal the rows out in strata of 64*W lanes, longest rows first.  Leaves
// L.ok false when no compiled instance can hold the layout.
void build_strat(asy_network *net, int W, const std::vector<std::vector<Term>> &rows)
{
    StratLayout &L = net->strat[w_index(W)];
    L = StratLayout{};
    const int N = net->n_species;
    const int lanes = 64 * W;
    std::vector<int> order(rows.size());
    for (size_t r = 0; r < rows.size(); ++r)
        order[r] = (int)r;
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return rows[a].size() > rows[b].size(); });
    const int K = (int)((rows.size() + lanes - 1) / lanes);
    std::vector<int32_t> strat_end(K);
    int slot = 0;
    for (int k = 0; k < K; ++k) {
        size_t len = 1;  // every stratum closes at a slot, even when all its rows are empty
        for (int l = 0; l < lanes; ++l) {
            const size_t r = (size_t)k * lanes + l;
            if (r < order.size())
                len = std::max(len, rows[order[r]].size());
        }
        slot += (int)((len + 3) / 4 * 4);  // strata end on multiples of 4 slots
        strat_end[k] = slot;
    }
    if ((N + 1) * 8 > 65535)
        return;  // byte offsets of Y cells must fit 16 bits
    L.W = W;
    L.lanes = lanes;
    L.K = K;
    L.C_needed = slot;
    L.SPL = (N + lanes - 1) / lanes;
    const StratInstance *inst = find_strat_instance(W, L.SPL, L.C_needed);
    if (!inst || L.C_needed > 256)
        return;  // end_mask holds at most 64 blocks of 4 slots
    const int C = inst->C;
    L.C = C;
    // descriptors hold byte offsets of the two Y cells (cell N = 1.0)
    const uint32_t one = (uint32_t)N * 8u;
    std::vector<uint32_t> desc((size_t)C * lanes, one | (one << 16));
    std::vector<int32_t> rx((size_t)C * lanes, -1);
    std::vector<int32_t> dst((size_t)K * lanes, 2 * N);
    int start = 0;
    for (int k = 0; k < K; ++k) {
        for (int l = 0; l < lanes; ++l) {
            const size_t r = (size_t)k * lanes + l;
            if (r >= order.size())
                continue;
            const int row = order[r];
            dst[(size_t)k * lanes + l] = row;
            const auto &terms = rows[row];
            for (size_t e = 0; e < terms.size(); ++e) {
                const size_t at = (size_t)(start + (int)e) * lanes + l;
                desc[at] = (uint32_t)terms[e].x * 8u | ((uint32_t)terms[e].y * 8u << 16);
                rx[at] = terms[e].rx;
            }
        }
        start = strat_end[k];
    }
    size_t off = 0;
    auto carve = [&](size_t bytes) {
        size_t o = off;
        off += (bytes + 255) / 256 * 256;
        return o;
    };
    const size_t o_desc = carve(desc.size() * 4), o_rx = carve(rx.size() * 4);
    const size_t o_end = carve(strat_end.size() * 4), o_dst = carve(dst.size() * 4);
    if (hipMalloc(&L.dev, off) != hipSuccess) {
        L.dev = nullptr;
        return;
    }
    char *base = static_cast<char *>(L.dev);
    hipError_t e = hipSuccess;
    auto put = [&](size_t o, const void *src, size_t bytes) {
        if (e == hipSuccess)
            e = hipMemcpy(base + o, src, bytes, hipMemcpyHostToDevice);
    };
    put(o_desc, desc.data(), desc.size() * 4);
    put(o_rx, rx.data(), rx.size() * 4);
    put(o_end, strat_end.data(), strat_end.size() * 4);
    put(o_dst, dst.data(), dst.size() * 4);
    if (e != hipSuccess)
        return;
    L.sn.n_species = N;
    L.sn.n_reactions = net->n_reactions;
    L.sn.n_strata = K;
    L.sn.n_slots = L.C_needed;
    L.sn.end_mask = 0;
    for (int k = 0; k < K; ++k)
        L.sn.end_mask |= 1ull << (strat_end[k] / 4 - 1);
    L.sn.desc = reinterpret_cast<const uint32_t *>(base + o_desc);
    L.sn.rx = reinterpret_cast<const int32_t *>(base + o_rx);
    L.sn.strat_end = reinterpret_cast<const int32_t *>(base + o_end);
    L.sn.strat_dst = reinterpret_cast<const int32_t *>(base + o_dst);
    L.ok = true;
}

size_t lds_bytes_variant0(const asy_network *net)
{
    return sizeof(double) * ((size_t)net->n_reactions + 2 * (size_t)net->n_species);
}

size_t lds_bytes_variant1(const asy_network *net, int zones_per_group)
{
    return sizeof(double) * (size_t)strat_zone_cells(net->n_species) * zones_per_group;
}

asy_status validate_launch(const asy_network *net, const asy_launch *c)
{
    if (c->zone_order != 0 && c->zone_order != 1)
        return fail(ASY_EINVAL, "asy_launch.zone_order must be 0 or 1");
    if (c->zone_order == 1 && c->variant != 1)
        return fail(ASY_EINVAL, "asy_launch.zone_order 1 needs variant 1");
    if (c->groups_per_cu < 0 || c->groups_per_cu > 32)
        return fail(ASY_EINVAL, "asy_launch.groups_per_cu must be in [0, 32]");
    if (c->use_graph != 0 && c->use_graph != 1)
        return fail(ASY_EINVAL, "asy_launch.use_graph must be 0 or 1");
    if (c->variant == 0) {
        if (c->threads_per_zone != 64 && c->threads_per_zone != 128 &&
            c->threads_per_zone != 256 && c->threads_per_zone != 512)
            return fail(ASY_EINVAL, "variant 0: threads_per_zone must be 64, 128, 256 or 512");
        if (c->zones_per_group != 1)
            return fail(ASY_EINVAL, "variant 0: zones_per_group must be 1");
        if (lds_bytes_variant0(net) > net->lds_per_group_max)
            return fail(ASY_ENOTSUP, "variant 0: network too large for the LDS of one workgroup");
        return ASY_OK;
    }
    if (c->variant == 1) {
        const int W = c->threads_per_zone / 64;
        if (c->threads_per_zone % 64 || (W != 1 && W != 2 && W != 4))
            return fail(ASY_EINVAL, "variant 1: threads_per_zone must be 64, 128 or 256");
        if (c->zones_per_group != 1)
            return fail(ASY_EINVAL, "variant 1: zones_per_group must be 1");
        if (!net->strat[w_index(W)].ok)
            return fail(ASY_ENOTSUP, "variant 1 has no kernel instance for this network with " +
                                         std::to_string(c->threads_per_zone) + " threads per zone");
        if (lds_bytes_variant1(net, c->zones_per_group) > net->lds_per_group_max)
            return fail(ASY_ENOTSUP, "variant 1: zones do not fit the LDS of one workgroup");
        return ASY_OK;
    }
    return fail(ASY_EINVAL, "asy_launch.variant must be 0 or 1");
}

template <int NT, bool ARR>
hipError_t launch_variant0(asy_network *net, const DevOptions &o, const ZoneArgs &za, int grid,
                           hipStream_t s)
{
    hipLaunchKernelGGL((integrate_group_kernel<NT, ARR>), dim3(grid), dim3(NT),
                       lds_bytes_variant0(net), s, net->dn, o, za);
    return hipGetLastError();
}

// Queue every kernel of one call on stream s (no allocation, no host sync, so
// the sequence can be captured into a graph).
hipError_t launch_all(asy_network *net, const asy_launch &c, const DevOptions &o,
                      const ZoneArgs &za, hipStream_t s)
{
    hipLaunchKernelGGL(reset_queue_kernel, dim3(1), dim3(64), 0, s, za.queue);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    if (c.variant == 1) {
        const int W = c.threads_per_zone / 64;
        const StratLayout &L = net->strat[w_index(W)];
        const double *rates = za.k_zone;
        if (net->rate_form == ASY_RATES_ARRHENIUS) {
            const size_t total = (size_t)za.n_zones * net->n_reactions;
            const int blocks = (int)std::min<size_t>((total + 255) / 256, (size_t)net->n_cu * 16);
            hipLaunchKernelGGL(rates_arrhenius_kernel, dim3(blocks), dim3(256), 0, s, za.n_zones,
                               net->n_reactions, net->dn.A, net->dn.E, za.T, net->rate_buf);
            e = hipGetLastError();
            if (e != hipSuccess)
                return e;
            rates = net->rate_buf;
        }
        const int32_t *order = nullptr;
        if (c.zone_order == 1) {
            const int kb = (int)std::min<size_t>(((size_t)za.n_zones * kWave + 255) / 256,
                                                 (size_t)net->n_cu * 16);
            hipLaunchKernelGGL(zone_cost_kernel, dim3(kb), dim3(256), 0, s, za.n_zones,
                               net->n_reactions, rates, net->key_buf);
            e = hipGetLastError();
            if (e != hipSuccess)
                return e;
            const int ob = (za.n_zones + kOrderChunk - 1) / kOrderChunk;
            hipLaunchKernelGGL(zone_order_kernel, dim3(ob), dim3(1024), 0, s, za.n_zones,
                               net->key_buf, net->order_buf);
            e = hipGetLastError();
            if (e != hipSuccess)
                return e;
            order = net->order_buf;
        }
        const StratInstance *inst = find_strat_instance(W, L.SPL, L.C);
        const int zpg = c.zones_per_group;
        int grid = (za.n_zones + zpg - 1) / zpg;
        if (c.groups_per_cu > 0)
            grid = std::min(grid, c.groups_per_cu * net->n_cu);
        hipLaunchKernelGGL(inst->fn, dim3(grid), dim3(c.threads_per_zone * zpg),
                           lds_bytes_variant1(net, zpg), s, L.sn, o, za, rates, order);
        return hipGetLastError();
    }
    int grid = za.n_zones;
    if (c.groups_per_cu > 0)
        grid = std::min(grid, c.groups_per_cu * net->n_cu);
    const bool arr = net->rate_form == ASY_RATES_ARRHENIUS;
    switch (c.threads_per_zone) {
    case 64:
        return arr ? launch_variant0<64, true>(net, o, za, grid, s)
                   : launch_variant0<64, false>(net, o, za, grid, s);
    case 128:
        return arr ? launch_variant0<128, true>(net, o, za, grid, s)
                   : launch_variant0<128, false>(net, o, za, grid, s);
    case 256:
        return arr ? launch_variant0<256, true>(net, o, za, grid, s)
                   : launch_variant0<256, false>(net, o, za, grid, s);
    default:
        return arr ? launch_variant0<512, true>(net, o, za, grid, s)
                   : launch_variant0<512, false>(net, o, za, grid, s);
    }
}

asy_status validate_options(const asy_options *o)
{
    auto pos = [](double v) { return std::isfinite(v) && v > 0.0; };
    if (!(o->kappa > 0.0) || std::isnan(o->kappa))
        return fail(ASY_EINVAL, "kappa must be > 0 (may be +inf)");
    if (!pos(o->tol) || !pos(o->y_floor) || !pos(o->safety))
        return fail(ASY_EINVAL, "tol, y_floor and safety must be finite and > 0");
    if (!(std::isfinite(o->grow_max) && o->grow_max >= 1.0))
        return fail(ASY_EINVAL, "grow_max must be finite and >= 1");
    if (!(std::isfinite(o->shrink_min) && o->shrink_min > 0.0 && o->shrink_min < 1.0))
        return fail(ASY_EINVAL, "shrink_min must be in (0, 1)");
    if (!(std::isfinite(o->dt_min) && o->dt_min >= 0.0))
        return fail(ASY_EINVAL, "dt_min must be finite and >= 0");
    if (o->max_steps < 0)
        return fail(ASY_EINVAL, "max_steps must be >= 0");
    if (o->controller != ASY_CTRL_PLAIN && o->controller != ASY_CTRL_LEARNED)
        return fail(ASY_EINVAL, "unknown controller");
    if (o->controller == ASY_CTRL_LEARNED)
        return fail(ASY_ENOTSUP, "learned controller not available in this build");
    if (o->reserved != 0)
        return fail(ASY_EINVAL, "asy_options.reserved must be 0");
    return ASY_OK;
}

// Make the per-call device tables (Arrhenius rates, scheduling keys and
// order) large enough for n_zones.  Synchronizes the stream before replacing
// tables a queued call may still read, and drops a captured graph that holds
// their old addresses.
asy_status ensure_call_bufs(asy_network *net, const asy_launch &c, int32_t n_zones, hipStream_t s)
{
    const bool need_rates = c.variant == 1 && net->rate_form == ASY_RATES_ARRHENIUS &&
                            net->rate_buf_zones < (size_t)n_zones;
    const bool need_order = c.variant == 1 && c.zone_order == 1 &&
                            net->order_buf_zones < (size_t)n_zones;
    if (!need_rates && !need_order)
        return ASY_OK;
    HIP_TRY(hipStreamSynchronize(s));
    if (net->graph.exec) {
        HIP_TRY(hipGraphExecDestroy(net->graph.exec));
        net->graph.exec = nullptr;
        net->graph.key.clear();
    }
    if (need_rates) {
        if (net->rate_buf)
            HIP_TRY(hipFree(net->rate_buf));
        net->rate_buf = nullptr;
        net->rate_buf_zones = 0;
        HIP_TRY(hipMalloc(&net->rate_buf, sizeof(double) * (size_t)n_zones * net->n_reactions));
        net->rate_buf_zones = (size_t)n_zones;
    }
    if (need_order) {
        if (net->key_buf)
            HIP_TRY(hipFree(net->key_buf));
        if (net->order_buf)
            HIP_TRY(hipFree(net->order_buf));
        net->key_buf = nullptr;
        net->order_buf = nullptr;
        net->order_buf_zones = 0;
        HIP_TRY(hipMalloc(&net->key_buf, sizeof(float) * (size_t)n_zones));
        HIP_TRY(hipMalloc(&net->order_buf, sizeof(int32_t) * (size_t)n_zones));
        net->order_buf_zones = (size_t)n_zones;
    }
    return ASY_OK;
}

template <typename T>
void append_bytes(std::vector<uint8_t> &key, const T &v)
{
    const uint8_t *p = reinterpret_cast<const uint8_t *>(&v);
    key.insert(key.end(), p, p + sizeof(T));
}

// Queue one call, replaying a captured graph when the launch is identical to
// the previous one (same configuration, options, sizes and buffers).
asy_status enqueue(asy_network *net, const asy_launch &c, const DevOptions &o, const ZoneArgs &za,
                   hipStream_t s)
{
    if (!c.use_graph) {
        HIP_TRY(launch_all(net, c, o, za, s));
        return ASY_OK;
    }
    std::vector<uint8_t> key;
    append_bytes(key, c);
    append_bytes(key, o);
    append_bytes(key, za);
    if (net->graph.exec == nullptr || key != net->graph.key) {
        if (net->graph.exec) {
            HIP_TRY(hipGraphExecDestroy(net->graph.exec));
            net->graph.exec = nullptr;
            net->graph.key.clear();
        }
        if (!net->capture_stream)
            HIP_TRY(hipStreamCreateWithFlags(&net->capture_stream, hipStreamNonBlocking));
        HIP_TRY(hipStreamBeginCapture(net->capture_stream, hipStreamCaptureModeThreadLocal));
        hipError_t le = launch_all(net, c, o, za, net->capture_stream);
        hipGraph_t graph = nullptr;
        hipError_t ee = hipStreamEndCapture(net->capture_stream, &graph);
        if (le != hipSuccess || ee != hipSuccess) {
            if (graph)
                (void)hipGraphDestroy(graph);
            return fail(ASY_EDEVICE, std::string("graph capture: ") +
                                         hipGetErrorString(le != hipSuccess ? le : ee));
        }
        hipError_t ie = hipGraphInstantiate(&net->graph.exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (ie != hipSuccess) {
            net->graph.exec = nullptr;
            return fail(ASY_EDEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(ie));
        }
        net->graph.key = key;
    }
    HIP_TRY(hipGraphLaunch(net->graph.exec, s));
    return ASY_OK;
}

DevOptions to_dev(const asy_options &o)
{
    return DevOptions{o.kappa, o.tol, o.y_floor, o.grow_max, o.safety, o.shrink_min, o.dt_min,
                      o.max_steps};
}

}  // namespace

extern "C" {

void asy_options_default(asy_options *o)
{
    if (!o)
        return;
    o->kappa = 1.0;
    o->tol = 0.01;
    o->y_floor = 1e-10;
    o->grow_max = 2.0;
    o->safety = 0.9;
    o->shrink_min = 0.1;
    o->dt_min = 1e-20;
    o->max_steps = 10000000;
    o->controller = ASY_CTRL_PLAIN;
    o->reserved = 0;
}

const char *asy_last_error(void) { return g_last_error.c_str(); }

const char *asy_version(void) { return "asynet 0.2 (gfx950)"; }

asy_status asy_network_create(const asy_network_desc *d, asy_network **out)
{
    g_last_error.clear();
    if (!d || !out)
        return fail(ASY_EINVAL, "desc and out must be non-NULL");
    const int32_t N = d->n_species, R = d->n_reactions;
    if (N < 1 || R < 1)
        return fail(ASY_EINVAL, "n_species and n_reactions must be >= 1");
    if (N > 32000 || R > (1 << 24))
        return fail(ASY_EINVAL, "network too large (n_species <= 32000, n_reactions <= 2^24)");
    if (!d->reactant0 || !d->reactant1 || !d->product)
        return fail(ASY_EINVAL, "reactant0, reactant1 and product must be non-NULL");
    if (d->rate_form == ASY_RATES_ARRHENIUS) {
        if (!d->A || !d->E)
            return fail(ASY_EINVAL, "Arrhenius rates need A and E");
    } else if (d->rate_form == ASY_RATES_PER_ZONE) {
        if (d->A || d->E)
            return fail(ASY_EINVAL, "per-zone rates take no A or E");
    } else {
        return fail(ASY_EINVAL, "unknown rate_form");
    }
    int32_t n_two = 0;
    for (int32_t j = 0; j < R; ++j) {
        const int32_t a = d->reactant0[j], b = d->reactant1[j], c = d->product[j];
        if (a < 0 || a >= N || c < 0 || c >= N || b < -1 || b >= N)
            return fail(ASY_EINVAL, "species index out of range in reaction " + std::to_string(j));
        if (a == b)
            return fail(ASY_EINVAL, "identical reactants in reaction " + std::to_string(j));
        if (c == a || c == b)
            return fail(ASY_EINVAL, "product equals a reactant in reaction " + std::to_string(j));
        if (d->weight) {
            const int64_t wa = d->weight[a], wb = b >= 0 ? d->weight[b] : 0, wc = d->weight[c];
            if (wc != wa + wb)
                return fail(ASY_EINVAL, "reaction " + std::to_string(j) + " does not conserve weight");
        }
        if (d->rate_form == ASY_RATES_ARRHENIUS) {
            if (!std::isfinite(d->A[j]) || !(d->A[j] > 0.0) || !std::isfinite(d->E[j]))
                return fail(ASY_EINVAL, "invalid Arrhenius parameters in reaction " + std::to_string(j));
        }
        n_two += b >= 0;
    }
    const int32_t D = R + n_two;

    // variant 0 layout: species-major rows, ascending reaction index within each row
    std::vector<int32_t> prod_ptr(N + 1, 0), dest_ptr(N + 1, 0);
    for (int32_t j = 0; j < R; ++j) {
        prod_ptr[d->product[j] + 1]++;
        dest_ptr[d->reactant0[j] + 1]++;
        if (d->reactant1[j] >= 0)
            dest_ptr[d->reactant1[j] + 1]++;
    }
    for (int32_t i = 0; i < N; ++i) {
        prod_ptr[i + 1] += prod_ptr[i];
        dest_ptr[i + 1] += dest_ptr[i];
    }
    std::vector<int32_t> prod_rx(R), prod_a(R), prod_b(R), dest_rx(D), dest_o(D);
    {
        std::vector<int32_t> pf(prod_ptr.begin(), prod_ptr.end() - 1);
        std::vector<int32_t> df(dest_ptr.begin(), dest_ptr.end() - 1);
        for (int32_t j = 0; j < R; ++j) {
            const int32_t a = d->reactant0[j], b = d->reactant1[j], c = d->product[j];
            int32_t e = pf[c]++;
            prod_rx[e] = j;
            prod_a[e] = a;
            prod_b[e] = b;
            e = df[a]++;
            dest_rx[e] = j;
            dest_o[e] = b;
            if (b >= 0) {
                e = df[b]++;
                dest_rx[e] = j;
                dest_o[e] = a;
            }
        }
    }

    // device: require gfx950 before allocating anything
    int dev = 0;
    hipError_t he = hipGetDevice(&dev);
    if (he != hipSuccess)
        return fail(ASY_EDEVICE, std::string("no HIP device: ") + hipGetErrorString(he));
    hipDeviceProp_t prop;
    he = hipGetDeviceProperties(&prop, dev);
    if (he != hipSuccess)
        return fail(ASY_EDEVICE, std::string("hipGetDeviceProperties: ") + hipGetErrorString(he));
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(ASY_EDEVICE, std::string("device is ") + prop.gcnArchName +
                                     "; this library is built for gfx950 only");

    auto *net = new asy_network();
    net->n_species = N;
    net->n_reactions = R;
    net->n_destruction = D;
    net->rate_form = d->rate_form;
    net->device = dev;
    net->n_cu = prop.multiProcessorCount;
    net->lds_per_group_max = prop.sharedMemPerBlock;

    size_t off = 0;
    auto carve = [&](size_t bytes) {
        size_t o = off;
        off += (bytes + 255) / 256 * 256;
        return o;
    };
    const size_t o_queue = carve(256);
    const size_t o_pp = carve(sizeof(int32_t) * (N + 1));
    const size_t o_prx = carve(sizeof(int32_t) * R);
    const size_t o_pa = carve(sizeof(int32_t) * R);
    const size_t o_pb = carve(sizeof(int32_t) * R);
    const size_t o_dp = carve(sizeof(int32_t) * (N + 1));
    const size_t o_drx = carve(sizeof(int32_t) * D);
    const size_t o_do = carve(sizeof(int32_t) * D);
    const bool arr = d->rate_form == ASY_RATES_ARRHENIUS;
    const size_t o_A = arr ? carve(sizeof(double) * R) : 0;
    const size_t o_E = arr ? carve(sizeof(double) * R) : 0;
    he = hipMalloc(&net->dev_block, off);
    if (he != hipSuccess) {
        delete net;
        return fail(ASY_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(he));
    }
    char *base = static_cast<char *>(net->dev_block);
    hipError_t ce = hipSuccess;
    auto put = [&](size_t o, const void *src, size_t bytes) {
        if (ce == hipSuccess)
            ce = hipMemcpy(base + o, src, bytes, hipMemcpyHostToDevice);
    };
    if (ce == hipSuccess)
        ce = hipMemset(base + o_queue, 0, 256);
    put(o_pp, prod_ptr.data(), sizeof(int32_t) * (N + 1));
    put(o_prx, prod_rx.data(), sizeof(int32_t) * R);
    put(o_pa, prod_a.data(), sizeof(int32_t) * R);
    put(o_pb, prod_b.data(), sizeof(int32_t) * R);
    put(o_dp, dest_ptr.data(), sizeof(int32_t) * (N + 1));
    put(o_drx, dest_rx.data(), sizeof(int32_t) * D);
    put(o_do, dest_o.data(), sizeof(int32_t) * D);
    if (arr) {
        put(o_A, d->A, sizeof(double) * R);
        put(o_E, d->E, sizeof(double) * R);
    }
    if (ce != hipSuccess) {
        asy_network_destroy(net);
        return fail(ASY_EDEVICE, std::string("upload: ") + hipGetErrorString(ce));
    }
    net->queue = reinterpret_cast<int32_t *>(base + o_queue);
    DevNetwork &dn = net->dn;
    dn.n_species = N;
    dn.n_reactions = R;
    dn.prod_ptr = reinterpret_cast<const int32_t *>(base + o_pp);
    dn.prod_rx = reinterpret_cast<const int32_t *>(base + o_prx);
    dn.prod_a = reinterpret_cast<const int32_t *>(base + o_pa);
    dn.prod_b = reinterpret_cast<const int32_t *>(base + o_pb);
    dn.dest_ptr = reinterpret_cast<const int32_t *>(base + o_dp);
    dn.dest_rx = reinterpret_cast<const int32_t *>(base + o_drx);
    dn.dest_o = reinterpret_cast<const int32_t *>(base + o_do);
    dn.A = arr ? reinterpret_cast<const double *>(base + o_A) : nullptr;
    dn.E = arr ? reinterpret_cast<const double *>(base + o_E) : nullptr;

    // variant 1 layouts
    {
        const auto rows = network_rows(N, R, d->reactant0, d->reactant1, d->product);
        for (int W : {1, 2, 4})
            build_strat(net, W, rows);
    }
    // default launch: variant 1 with the fewest waves per zone whose rates fit
    // in 80 slots per lane (two waves per SIMD), else the fewest waves with
    // any instance, else the generic variant 0 (asy_autotune measures instead)
    asy_launch c{};
    c.variant = 0;
    c.threads_per_zone = N <= 64 ? 64 : (N <= 128 ? 128 : 256);
    c.zones_per_group = 1;
    for (int pass = 0; pass < 2 && c.variant == 0; ++pass) {
        for (int W : {1, 2, 4}) {
            const StratLayout &L = net->strat[w_index(W)];
            if (L.ok && (pass == 1 || L.C <= 80)) {
                c.variant = 1;
                c.threads_per_zone = 64 * W;
                c.zone_order = 1;
                break;
            }
        }
    }
    net->launch = c;
    if (validate_launch(net, &net->launch) != ASY_OK) {
        asy_network_destroy(net);
        return fail(ASY_ENOTSUP, "network too large for the LDS of one workgroup");
    }
    *out = net;
    return ASY_OK;
}

void asy_network_destroy(asy_network *net)
{
    if (!net)
        return;
    (void)hipDeviceSynchronize();
    if (net->graph.exec)
        (void)hipGraphExecDestroy(net->graph.exec);
    if (net->capture_stream)
        (void)hipStreamDestroy(net->capture_stream);
    if (net->dev_block)
        (void)hipFree(net->dev_block);
    for (auto &L : net->strat)
        if (L.dev)
            (void)hipFree(L.dev);
    if (net->rate_buf)
        (void)hipFree(net->rate_buf);
    if (net->key_buf)
        (void)hipFree(net->key_buf);
    if (net->order_buf)
        (void)hipFree(net->order_buf);
    delete net;
}

asy_status asy_get_launch(const asy_network *net, asy_launch *cfg)
{
    if (!net || !cfg)
        return fail(ASY_EINVAL, "net and cfg must be non-NULL");
    *cfg = net->launch;
    return ASY_OK;
}

asy_status asy_set_launch(asy_network *net, const asy_launch *cfg)
{
    if (!net || !cfg)
        return fail(ASY_EINVAL, "net and cfg must be non-NULL");
    asy_status st = validate_launch(net, cfg);
    if (st != ASY_OK)
        return st;
    net->launch = *cfg;
    return ASY_OK;
}

asy_status asy_integrate_batch(asy_network *net, const asy_options *opts, int32_t n_zones,
                               double *Y, const double *T, const double *k_zone,
                               const double *t_end, double *dt, int64_t *n_accepted,
                               int64_t *n_rejected, int32_t *zone_status, void *stream)
{
    g_last_error.clear();
    if (!net)
        return fail(ASY_EINVAL, "net must be non-NULL");
    asy_options o;
    asy_options_default(&o);
    if (opts)
        o = *opts;
    asy_status st = validate_options(&o);
    if (st != ASY_OK)
        return st;
    if (n_zones < 0)
        return fail(ASY_EINVAL, "n_zones must be >= 0");
    if (n_zones == 0)
        return ASY_OK;
    if (!Y || !t_end || !dt || !n_accepted || !n_rejected || !zone_status)
        return fail(ASY_EINVAL, "Y, t_end, dt, n_accepted, n_rejected, zone_status must be non-NULL");
    if (net->rate_form == ASY_RATES_ARRHENIUS) {
        if (!T || k_zone)
            return fail(ASY_EINVAL, "Arrhenius networks take T and no k_zone");
    } else if (!k_zone || T) {
        return fail(ASY_EINVAL, "per-zone-rate networks take k_zone and no T");
    }
    ZoneArgs za{n_zones, Y, T, k_zone, t_end, dt, n_accepted, n_rejected, zone_status, net->queue};
    hipStream_t s = static_cast<hipStream_t>(stream);
    HIP_TRY(hipSetDevice(net->device));
    st = ensure_call_bufs(net, net->launch, n_zones, s);
    if (st != ASY_OK)
        return st;
    return enqueue(net, net->launch, to_dev(o), za, s);
}

asy_status asy_autotune(asy_network *net, const asy_options *opts, int32_t sample_zones,
                        const double *Y, const double *T, const double *k_zone,
                        const double *t_end, const double *dt, asy_launch *best)
{
    g_last_error.clear();
    if (!net)
        return fail(ASY_EINVAL, "net must be non-NULL");
    asy_options o;
    asy_options_default(&o);
    if (opts)
        o = *opts;
    asy_status st = validate_options(&o);
    if (st != ASY_OK)
        return st;
    if (sample_zones < 1)
        return fail(ASY_EINVAL, "sample_zones must be >= 1");
    if (!Y || !t_end || !dt)
        return fail(ASY_EINVAL, "Y, t_end and dt must be non-NULL");
    if (net->rate_form == ASY_RATES_ARRHENIUS ? (!T || k_zone) : (!k_zone || T))
        return fail(ASY_EINVAL, "rate arguments do not match the network's rate form");
    HIP_TRY(hipSetDevice(net->device));
    const int Z = sample_zones;
    const size_t nY = (size_t)Z * net->n_species;
    // private copies: the integration works in place
    double *wY = nullptr, *wdt = nullptr;
    int64_t *wacc = nullptr, *wrej = nullptr;
    int32_t *wst = nullptr;
    auto cleanup = [&]() {
        (void)hipFree(wY);
        (void)hipFree(wdt);
        (void)hipFree(wacc);
        (void)hipFree(wrej);
        (void)hipFree(wst);
    };
    if (hipMalloc(&wY, nY * 8) != hipSuccess || hipMalloc(&wdt, (size_t)Z * 8) != hipSuccess ||
        hipMalloc(&wacc, (size_t)Z * 8) != hipSuccess || hipMalloc(&wrej, (size_t)Z * 8) != hipSuccess ||
        hipMalloc(&wst, (size_t)Z * 4) != hipSuccess) {
        cleanup();
        return fail(ASY_ENOMEM, "autotune: allocation of the sample copies failed");
    }
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        cleanup();
        return fail(ASY_EDEVICE, "autotune: hipEventCreate failed");
    }
    std::vector<asy_launch> cands;
    for (int W : {1, 2, 4}) {
        if (!net->strat[w_index(W)].ok)
            continue;
        asy_launch c{1, 64 * W, 1, 0, net->launch.use_graph, 0};
        if (validate_launch(net, &c) == ASY_OK)
            cands.push_back(c);
    }
    for (int nt : {128, 256}) {
        asy_launch c{0, nt, 1, 0, net->launch.use_graph, 0};
        if (validate_launch(net, &c) == ASY_OK)
            cands.push_back(c);
    }
    g_last_error.clear();
    const asy_launch saved = net->launch;
    float best_ms = 0.0f;
    asy_launch best_c = saved;
    ZoneArgs za{Z, wY, T, k_zone, t_end, wdt, wacc, wrej, wst, net->queue};
    asy_status result = ASY_OK;
    for (const asy_launch &c : cands) {
        net->launch = c;
        st = ensure_call_bufs(net, c, Z, nullptr);
        float ms = 0.0f;
        for (int rep = 0; rep < 2 && st == ASY_OK; ++rep) {  // first run warms up
            if (hipMemcpy(wY, Y, nY * 8, hipMemcpyDeviceToDevice) != hipSuccess ||
                hipMemcpy(wdt, dt, (size_t)Z * 8, hipMemcpyDeviceToDevice) != hipSuccess ||
                hipEventRecord(e0, nullptr) != hipSuccess ||
                launch_all(net, c, to_dev(o), za, nullptr) != hipSuccess ||
                hipEventRecord(e1, nullptr) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
                st = fail(ASY_EDEVICE, "autotune: a candidate launch failed");
        }
        if (st != ASY_OK) {
            result = st;
            break;
        }
        if (best_ms == 0.0f || ms < best_ms) {
            best_ms = ms;
            best_c = c;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    cleanup();
    net->launch = (result == ASY_OK) ? best_c : saved;
    if (best)
        *best = net->launch;
    return result;
}

}  // extern "C"
