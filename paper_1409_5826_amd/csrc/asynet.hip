// Host side of the asynet C ABI: descriptor validation, incidence layouts,
// device upload, launch configuration, graph replay and autotuning.  See
// include/asynet.h for the contract of every entry point.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cfloat>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "asynet.h"
#include "integrate_kernels.h"
#include "lds_layout.h"
#include "lds_probe.h"
#include "mlp_kernels.h"
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
    int W = 0, lanes = 0, C_needed = 0, C = 0, SPL = 0;
    int n_split = 0;      // rows summed in chunks
    int64_t gather_cycles_before = 0, gather_cycles_after = 0;  // modelled, per zone-step
    uint32_t one_waves = 0;  // waves whose terms all have 1.0 as second factor
    int f1 = 0;           // leading slots whose terms all have 1.0 as second factor
    int C2 = 0;           // balanced layout: slots of the two-factor waves (0: all C)
    bool ok32 = false;    // the single-precision tables exist
    StratNetwork sn32{};  // the same layout with descriptors for float cells
    void *dev = nullptr;
    StratNetwork sn{};
    bool ok = false;
};

// Captured launch sequence for repeated identical calls.
struct GraphCache {
    hipGraphExec_t exec = nullptr;
    std::vector<uint8_t> key;
};

// Scratch of asy_integrate_batch_noalloc, one copy per device for the life of
// the process (64 MiB): the zone counter (256 B), the scheduling keys and order
// of at most kNoAllocMaxZones zones, then the Arrhenius rate table [zones]
// [reactions] (FP64), which bounds the zones of an Arrhenius network's call to
// kScratchRateBytes / (8 n_reactions).  Host code never touches the array by
// name (the name is a host-side stand-in); it uses the device address resolved
// by scratch_setup.
constexpr int32_t kNoAllocMaxZones = 1 << 18;
constexpr size_t kScratchKeyOff = 256;
constexpr size_t kScratchOrderOff = kScratchKeyOff + sizeof(float) * (size_t)kNoAllocMaxZones;
constexpr size_t kScratchRateOff = kScratchOrderOff + sizeof(int32_t) * (size_t)kNoAllocMaxZones;
constexpr size_t kScratchBytes = (size_t)64 << 20;
constexpr size_t kScratchRateBytes = kScratchBytes - kScratchRateOff;
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char *g_scratch_ptr[kMaxDevices] = {};  // device address of `scratch` on each device

}  // namespace

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

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
    StratLayout strat_bal[3];   // balanced variant-1 layouts of the plain kernels (if built)
    double *rate_buf = nullptr; // Arrhenius rates of one call, [zones][reactions]
    size_t rate_buf_zones = 0;
    float *key_buf = nullptr;   // scheduling keys of one call, [zones]
    int32_t *order_buf = nullptr; // scheduling order of one call, [zones]
    size_t order_buf_zones = 0;
    void *sched_block = nullptr;  // asy_integrate_schedule: before-abundances and step counters
    size_t sched_zones = 0;
    asy_launch launch{};
    hipStream_t capture_stream = nullptr;
    GraphCache graph;
    // learned controller: weights arranged for in-kernel inference (asy_set_mlp)
    void *mlp_block = nullptr;
    MlpDevice mlp{};
    bool has_mlp = false;
    const double *pow2 = nullptr;  // device [32]: 2^(b/32), in dev_block
};

struct asy_mlp {
    int32_t batch_max = 0;  // rounded up to a multiple of 32
    int device = 0;
    void *block = nullptr;
    float *p = nullptr, *g = nullptr, *m = nullptr, *v = nullptr;  // [kMlpParams]
    float *b3pad = nullptr;                                         // [16]
    uint16_t *W1b = nullptr, *W2b = nullptr, *W3b = nullptr;
    uint16_t *w1s = nullptr, *w2s = nullptr, *w3s = nullptr;
    uint16_t *xb = nullptr, *h1b = nullptr, *h2b = nullptr, *g_ob = nullptr, *g_a2b = nullptr,
             *g_a1b = nullptr;
    float *a1 = nullptr, *a2 = nullptr, *out16 = nullptr, *o = nullptr, *g_o = nullptr,
          *g_a2 = nullptr, *g_a1 = nullptr;
    float *colsum = nullptr;  // [kColsumBlocks][4][128] partial column sums
    int64_t t = 0;  // Adam steps taken
    bool bf16_current = false;  // W1b, W2b, W3b hold the masters' BF16 copies
};

namespace {

// ---- variant 1 kernel instances -----------------------------------------------------------

using StratKernel = void (*)(StratNetwork, DevOptions, ZoneArgs, const double *, const int32_t *,
                             LearnArgs);

// mode: 0 plain controller, 1 plain with trace, 2 learned, 3 learned with trace,
//       4 plain controller in single precision
// CR: slots whose rates the instance keeps in registers (the rest in LDS)
// F1: leading slots the instance runs as one-factor terms on every wave (0: none)
// C2: slots the waves with two-factor terms run (0: all C, like the other waves)
struct StratInstance {
    int W, SPL, C, CR, mode;
    StratKernel fn;
    int F1 = 0;
    int C2 = 0;
};

#define ASY_STRAT(W_, SPL_, C_)                                                                 \
    {W_, SPL_, C_, C_, 0, integrate_strat_kernel<W_, SPL_, C_, strat_gather_ahead<C_>(), false, false>}
#define ASY_STRAT_CR(W_, SPL_, C_, CR_)                                                         \
    {W_, SPL_, C_, CR_, 0, integrate_strat_kernel<W_, SPL_, C_, strat_gather_ahead<CR_>(), false,    \
                                                false, double, CR_>}
#define ASY_STRAT_F32(W_, SPL_, C_)                                                             \
    {W_, SPL_, C_, C_, 4, integrate_strat_kernel<W_, SPL_, C_, strat_gather_ahead<C_, float>(), false, \
                                               false, float>}
#define ASY_STRAT_F1(W_, SPL_, C_, CR_, F1_)                                                    \
    {W_, SPL_, C_, CR_, 0, integrate_strat_kernel<W_, SPL_, C_, strat_gather_ahead<CR_>(), false,    \
                                                false, double, CR_, F1_>, F1_}
#define ASY_STRAT_F32_F1(W_, SPL_, C_, F1_)                                                     \
    {W_, SPL_, C_, C_, 4, integrate_strat_kernel<W_, SPL_, C_, strat_gather_ahead<C_, float>(), false, \
                                               false, float, C_, F1_>, F1_}
#define ASY_STRAT_SPLIT(W_, SPL_, C_, CR_, F1_, C2_)                                            \
    {W_, SPL_, C_, CR_, 0, integrate_strat_kernel<W_, SPL_, C_, strat_gather_ahead<CR_>(), false,    \
                                                false, double, CR_, F1_, C2_>, F1_, C2_}
#define ASY_STRAT_F32_SPLIT(W_, SPL_, C_, CR_, C2_)                                             \
    {W_, SPL_, C_, CR_, 4, integrate_strat_kernel<W_, SPL_, C_, strat_gather_ahead<CR_, float>(),   \
                                                false, false, float, CR_, 0, C2_>, 0, C2_}
#define ASY_STRAT_LEARN(W_, SPL_, C_)                                                           \
    {W_, SPL_, C_, C_, 1, integrate_strat_kernel<W_, SPL_, C_, 2, false, true>},                \
    {W_, SPL_, C_, C_, 2, integrate_strat_kernel<W_, SPL_, C_, 2, true, false>},                \
    {W_, SPL_, C_, C_, 3, integrate_strat_kernel<W_, SPL_, C_, 2, true, true>}
const StratInstance kStratInstances[] = {
    ASY_STRAT(1, 1, 16), ASY_STRAT(1, 1, 32), ASY_STRAT(1, 2, 32), ASY_STRAT(1, 2, 48),
    ASY_STRAT(1, 3, 48), ASY_STRAT(1, 3, 64), ASY_STRAT(1, 3, 80), ASY_STRAT(1, 3, 96),
    ASY_STRAT(2, 1, 16), ASY_STRAT(2, 1, 32), ASY_STRAT(2, 2, 32), ASY_STRAT(2, 2, 40),
    ASY_STRAT(2, 2, 48), ASY_STRAT(2, 2, 64), ASY_STRAT(2, 3, 64), ASY_STRAT(2, 3, 96),
    ASY_STRAT(2, 3, 104), ASY_STRAT(2, 3, 112),
    ASY_STRAT(4, 1, 16), ASY_STRAT(4, 1, 32), ASY_STRAT(4, 1, 40), ASY_STRAT(4, 1, 48),
    ASY_STRAT(4, 2, 48), ASY_STRAT_CR(4, 2, 56, 40), ASY_STRAT(4, 2, 64), ASY_STRAT(4, 2, 80),
    ASY_STRAT_LEARN(1, 1, 16), ASY_STRAT_LEARN(2, 2, 40), ASY_STRAT_LEARN(2, 2, 48),
    ASY_STRAT_F32(1, 1, 16), ASY_STRAT_F32(1, 1, 32), ASY_STRAT_F32(1, 2, 32), ASY_STRAT_F32(1, 2, 48),
    ASY_STRAT_F32(1, 3, 48), ASY_STRAT_F32(1, 3, 64), ASY_STRAT_F32(1, 3, 80), ASY_STRAT_F32(1, 3, 96),
    ASY_STRAT_F32(2, 1, 16), ASY_STRAT_F32(2, 1, 32), ASY_STRAT_F32(2, 2, 32), ASY_STRAT_F32(2, 2, 40),
    ASY_STRAT_F32(2, 2, 48), ASY_STRAT_F32(2, 2, 64), ASY_STRAT_F32(2, 3, 64), ASY_STRAT_F32(2, 3, 96),
    ASY_STRAT_F32(2, 3, 104), ASY_STRAT_F32(2, 3, 112),
    ASY_STRAT_F32(4, 1, 16), ASY_STRAT_F32(4, 1, 32), ASY_STRAT_F32(4, 1, 40), ASY_STRAT_F32(4, 1, 48),
    ASY_STRAT_F32(4, 2, 48), ASY_STRAT_F32(4, 2, 56), ASY_STRAT_F32(4, 2, 64), ASY_STRAT_F32(4, 2, 80),
    ASY_STRAT_F1(2, 2, 40, 40, 8), ASY_STRAT_F32_F1(2, 2, 40, 8),
    ASY_STRAT_F1(4, 2, 56, 40, 16), ASY_STRAT_F32_F1(4, 2, 56, 16),
    ASY_STRAT_SPLIT(2, 2, 44, 40, 0, 32), ASY_STRAT_F32_SPLIT(2, 2, 44, 40, 32),
};
#undef ASY_STRAT
#undef ASY_STRAT_CR
#undef ASY_STRAT_F1
#undef ASY_STRAT_F32
#undef ASY_STRAT_F32_F1
#undef ASY_STRAT_SPLIT
#undef ASY_STRAT_F32_SPLIT
#undef ASY_STRAT_LEARN

// The instance for a layout: the smallest C that holds C_needed slots, and of those the one
// with the most leading one-factor slots the layout allows (f1_max, from build_strat); c2 > 0
// asks for an instance whose two-factor waves stop at slot c2 (a balanced layout).
const StratInstance *find_strat_instance(int W, int SPL, int C_needed, int mode = 0,
                                         int f1_max = 0, int c2 = 0)
{
    const StratInstance *best = nullptr;
    for (const auto &in : kStratInstances)
        if (in.W == W && in.SPL == SPL && in.mode == mode && in.C >= C_needed &&
            in.F1 <= f1_max && in.C2 == c2 &&
            (!best || in.C < best->C || (in.C == best->C && in.F1 > best->F1)))
            best = &in;
    return best;
}

int w_index(int W) { return W == 1 ? 0 : (W == 2 ? 1 : 2); }

// Variant 1's tables hold absolute LDS addresses, valid because its kernels
// declare no static LDS, so their dynamic LDS starts at address 0.  Checked
// once per process on the kernels' attributes.
asy_status check_strat_lds_base()
{
    static const bool good = [] {  // initialised once, thread-safe
        for (const auto &in : kStratInstances) {
            hipFuncAttributes a{};
            if (hipFuncGetAttributes(&a, reinterpret_cast<const void *>(in.fn)) != hipSuccess ||
                a.sharedSizeBytes != 0)
                return false;
        }
        return true;
    }();
    return good ? ASY_OK : fail(ASY_EDEVICE, "variant 1 kernels must not use static LDS");
}

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

// Term descriptors are stored block-major: the 4 slots of block b of lane l are
// consecutive, so a lane fetches a block's descriptors with one 16-byte load.
size_t desc_index(int slot, int lane, int lanes)
{
    return ((size_t)(slot / 4) * lanes + lane) * 4 + slot % 4;
}

constexpr int kSplitAboveDefault = 64;  // rows with more terms are summed in chunks
constexpr int64_t kLayoutIters = 100000;  // annealing moves per layout (~0.4 s for 150 species)

// Pack the rows onto 64*W lanes: every row padded to a multiple of 4 terms
// (at least 4, so that an empty row still writes its 0.0), longest first,
// each onto the lane with the least work so far (lowest lane on ties); the
// slot count C is the smallest compiled one that holds this packing.  Within
// that C, a second packing frees whole waves of second gathers when it can
// (below).  Then the bank-aware placement (lds_layout.h) picks the Y cells,
// the lanes' order within each wave and the rows' order within each lane.
// Row sums take the cells after Y in lane order (lane 0's rows first, each
// lane's in its slot order); split rows' totals follow.  Leaves L.ok false
// when no compiled instance can hold the layout.
// bal: build the balanced layout of that instance instead (into strat_bal): the
// two-factor rows packed into the first C2 slots of as few lanes as a cap allows,
// the one-factor rows into the rest (C2 slots on the lanes of waves with two-factor
// rows, C on the others), so the two kinds of wave get about equal work.
void build_strat(asy_network *net, int W, const std::vector<std::vector<Term>> &rows_in,
                 int split_above, const StratInstance *bal = nullptr)
{
    const int chunk = std::max(4, split_above / 2 / 4 * 4);  // terms per chunk of a split row
    StratLayout &L = bal ? net->strat_bal[w_index(W)] : net->strat[w_index(W)];
    L = StratLayout{};
    const int N = net->n_species;
    const int lanes = 64 * W;
    if (N * 8 > 0x7fff)
        return;  // the byte address of Y[y] fits the 15 bits below the row-end bit
    // Rows of more than split_above terms (by default hub species: far longer than the lanes'
    // average work) are split into chunks of `chunk` consecutive terms; every chunk is a row of
    // its own, and the kernel adds a split row's chunk sums in chunk order.  The rule does not
    // depend on the launch, so every launch configuration computes the same sums.
    std::vector<std::vector<Term>> rows = rows_in;
    std::vector<std::vector<int>> split_chunks;  // per split row: its packed rows, in chunk order
    std::vector<int> split_of(rows.size(), -1);  // original row -> split index
    {
        const size_t n_rows = rows.size();
        for (size_t r = 0; r < n_rows; ++r) {
            const size_t len = rows[r].size();
            if (len <= (size_t)split_above)
                continue;
            std::vector<Term> whole = std::move(rows[r]);
            split_of[r] = (int)split_chunks.size();
            split_chunks.emplace_back();
            for (size_t b = 0; b < len; b += chunk) {
                std::vector<Term> part(whole.begin() + b,
                                       whole.begin() + std::min(len, b + (size_t)chunk));
                if (b == 0) {
                    rows[r] = std::move(part);
                    split_chunks.back().push_back((int)r);
                } else {
                    split_chunks.back().push_back((int)rows.size());
                    rows.push_back(std::move(part));
                }
            }
        }
    }
    const int n_split = (int)split_chunks.size();
    auto padded = [&](size_t r) { return (int)std::max<size_t>(4, (rows[r].size() + 3) / 4 * 4); };
    std::vector<int> order(rows.size());
    for (size_t r = 0; r < rows.size(); ++r)
        order[r] = (int)r;
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return padded(a) > padded(b); });
    std::vector<int> load(lanes, 0);
    std::vector<std::vector<int>> lane_rows(lanes);
    for (int r : order) {
        const int l = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        lane_rows[l].push_back(r);
        load[l] += padded(r);
    }
    const int C_needed = std::max(4, *std::max_element(load.begin(), load.end()));
    L.W = W;
    L.lanes = lanes;
    L.C_needed = C_needed;
    L.SPL = (N + lanes - 1) / lanes;
    const StratInstance *inst = bal ? bal : find_strat_instance(W, L.SPL, C_needed);
    if (!inst || inst->SPL != L.SPL || inst->W != W)
        return;
    const int C = inst->C;
    L.C = C;
    L.C2 = bal ? bal->C2 : 0;
    // Rows whose second factors are all the 1.0 cell (depletion rows, creation rows of
    // one-body reactions only) need no second gather and no multiply by 1.0 (exact).  A wave
    // whose lanes hold only such rows runs a slot phase without either, so pack the other
    // rows onto as few lanes as a cap allows (first fit, longest first: they fill the first
    // waves), then the rest by least load, within the same C.  Keep the smallest cap that
    // frees the most waves; with none freed, keep the plain packing.
    std::vector<char> one_factor(rows.size());
    for (size_t r = 0; r < rows.size(); ++r)
        one_factor[r] = std::all_of(rows[r].begin(), rows[r].end(),
                                    [&](const Term &t) { return t.y == N; });
    std::vector<int> lane_start(lanes, 0);  // first slot of the lane's rows (padding before)
    {
        std::vector<int> other, ones;
        for (int r : order)
            (one_factor[r] ? ones : other).push_back(r);
        int best_free = 0;
        std::vector<std::vector<int>> best_rows;
        std::vector<int> best_load;
        const int cap0 = other.empty() ? 4 : padded(other.front());
        if (bal) {
            // the smallest cap whose first-fit packing leaves a wave free of two-factor rows
            // and lets the one-factor rows fit (each onto the lane with the most room left)
            const int C2 = bal->C2;
            bool done = false;
            for (int cap = cap0; cap <= C2 && !done; cap += 4) {
                std::vector<int> tload(lanes, 0);
                std::vector<std::vector<int>> lr(lanes), lone(lanes);
                bool ok = true;
                int used = 0;
                for (int r : other) {
                    int l = 0;
                    while (l < lanes && tload[l] + padded(r) > cap)
                        ++l;
                    if (l == lanes) {
                        ok = false;
                        break;
                    }
                    tload[l] += padded(r);
                    lr[l].push_back(r);
                    used = std::max(used, l + 1);
                }
                const int two_waves = (used + 63) / 64;
                if (!ok || two_waves >= W)
                    continue;
                std::vector<int> room(lanes);
                for (int l = 0; l < lanes; ++l)
                    room[l] = l < 64 * two_waves ? C2 : C;
                for (int r : ones) {
                    int l = 0;
                    for (int m = 1; m < lanes; ++m)
                        if (room[m] - tload[m] > room[l] - tload[l])
                            l = m;
                    if (tload[l] + padded(r) > room[l]) {
                        ok = false;
                        break;
                    }
                    tload[l] += padded(r);
                    lone[l].push_back(r);
                }
                if (!ok)
                    continue;
                for (int l = 0; l < lanes; ++l) {
                    lane_rows[l] = lone[l];
                    lane_rows[l].insert(lane_rows[l].end(), lr[l].begin(), lr[l].end());
                    lane_start[l] = room[l] - tload[l];
                }
                done = true;
            }
            if (!done)
                return;
        }
        for (int cap = cap0; cap <= C && best_free < W && !bal; cap += 4) {
            std::vector<int> tload(lanes, 0);
            std::vector<std::vector<int>> lr(lanes), lone(lanes);
            bool ok = true;
            int used = 0;  // lanes holding other rows: 0 .. used-1
            for (int r : other) {
                int l = 0;
                while (l < lanes && tload[l] + padded(r) > cap)
                    ++l;
                if (l == lanes) {
                    ok = false;
                    break;
                }
                tload[l] += padded(r);
                lr[l].push_back(r);
                used = std::max(used, l + 1);
            }
            const int free_waves = ok ? W - (used + 63) / 64 : 0;
            if (free_waves <= best_free)
                continue;
            for (int r : ones) {
                const int l = (int)(std::min_element(tload.begin(), tload.end()) - tload.begin());
                if (tload[l] + padded(r) > C) {
                    ok = false;
                    break;
                }
                tload[l] += padded(r);
                lone[l].push_back(r);
            }
            if (!ok)
                continue;
            best_free = free_waves;
            best_rows.assign(lanes, {});
            for (int l = 0; l < lanes; ++l) {
                best_rows[l] = lone[l];
                best_rows[l].insert(best_rows[l].end(), lr[l].begin(), lr[l].end());
            }
            best_load = tload;
        }
        if (best_free > 0) {
            lane_rows = best_rows;
            for (int l = 0; l < lanes; ++l)
                lane_start[l] = C - best_load[l];
        }
    }
    // bank-aware placement: which Y cell holds which species, which physical lane holds
    // which column, the order of rows within a column
    std::vector<int> cell_of(N + 1);
    {
        LayoutProblem lp;
        lp.n_species = N;
        lp.lanes = lanes;
        lp.slots = C;
        lp.rows.resize(rows.size());
        lp.padded.resize(rows.size());
        for (size_t r = 0; r < rows.size(); ++r) {
            for (const Term &t : rows[r])
                lp.rows[r].push_back({t.x, t.y});
            lp.padded[r] = padded(r);
        }
        lp.lane_rows = lane_rows;
        lp.lane_start = lane_start;
        // a lane's one-factor rows stay ahead of its other rows, which keeps the other rows in
        // the lane's last slots (the leading one-factor slots below)
        lp.row_class.assign(rows.size(), 0);
        for (size_t r = 0; r < rows.size(); ++r)
            lp.row_class[r] = one_factor[r] ? 0 : 1;
        const LayoutResult lr = optimise_gather_layout(lp, kLayoutIters, 0x5eed0001ull + W);
        lane_rows = lr.lane_rows;
        lane_start = lr.lane_start;
        for (int i = 0; i < N; ++i)
            cell_of[i] = lr.cell_of_species[i];
        cell_of[N] = N;
        L.gather_cycles_before = lr.cycles_before;
        L.gather_cycles_after = lr.cycles_after;
    }
    std::vector<int32_t> cell_species(N);
    for (int i = 0; i < N; ++i)
        cell_species[cell_of[i]] = i;
    // cells: Y (species i in cell cell_of[i], ONE in cell N), then the packed rows' sums in
    // lane order, then the totals of split rows
    const int n_packed = (int)rows.size();
    std::vector<int> cell(rows.size());
    std::vector<int> lane_first(lanes);
    {
        int next = N + 1;
        for (int l = 0; l < lanes; ++l) {
            lane_first[l] = next;
            for (int row : lane_rows[l])
                cell[row] = next++;
        }
    }
    const int n_cells = N + 1 + n_packed + n_split;
    if ((size_t)n_cells * 8 > 0x10000)
        return;  // cell addresses fit 16 bits
    auto total_cell = [&](int orig) {
        return split_of[orig] >= 0 ? N + 1 + n_packed + split_of[orig] : cell[orig];
    };
    L.n_split = n_split;
    // tables for cells of `bytes` bytes: [0] double, [1] float
    std::vector<uint32_t> desc[2], lane_out[2], species_out[2], split_src[2];
    std::vector<int32_t> rx((size_t)C * lanes, -1), split_first(1, 0);
    for (const auto &ch : split_chunks)
        split_first.push_back(split_first.back() + (int32_t)ch.size());
    for (int p = 0; p < 2; ++p) {
        const uint32_t B = p == 0 ? 8u : 4u;
        // padding terms read ONE twice and carry a zero rate
        const uint32_t one = (uint32_t)N * B;
        desc[p].assign((size_t)C * lanes, one | (one << 16));
        for (int l = 0; l < lanes; ++l) {
            int start = lane_start[l];
            for (int row : lane_rows[l]) {
                const auto &terms = rows[row];
                for (size_t e = 0; e < terms.size(); ++e) {
                    const int slot = start + (int)e;
                    desc[p][desc_index(slot, l, lanes)] = (uint32_t)cell_of[terms[e].x] * B |
                                                          ((uint32_t)cell_of[terms[e].y] * B << 16);
                    if (p == 0)
                        rx[(size_t)slot * lanes + l] = terms[e].rx;
                }
                start += padded(row);
                const int blk = start / 4 - 1;  // the row ends in this block
                desc[p][desc_index(4 * blk, l, lanes)] |= 0x80000000u;
            }
            lane_out[p].push_back((uint32_t)lane_first[l] * B);
        }
        for (int c = 0; c < N; ++c) {  // by Y cell
            const int i = cell_species[c];
            species_out[p].push_back((uint32_t)total_cell(i) * B |
                                     ((uint32_t)total_cell(N + i) * B << 16));
        }
        for (int q = 0; q < n_split; ++q)
            for (int r : split_chunks[q])
                split_src[p].push_back((uint32_t)cell[r] * B);
        if (n_split == 0)
            split_src[p].push_back(0);
    }
    // bit w: every term of wave w has the 1.0 cell as second factor
    uint32_t one_waves = 0;
    for (int w = 0; w < W; ++w) {
        bool all = true;
        for (int s = 0; s < C && all; ++s)
            for (int l = 64 * w; l < 64 * w + 64 && all; ++l)
                all = ((desc[0][desc_index(s, l, lanes)] >> 16) & 0x7fffu) == (uint32_t)N * 8u;
        if (all)
            one_waves |= 1u << w;
    }
    L.one_waves = one_waves;
    if (bal) {  // the waves with two-factor terms hold nothing past slot C2
        const uint32_t pad = (uint32_t)N * 8u | ((uint32_t)N * 8u << 16);
        for (int l = 0; l < lanes; ++l)
            if (!((one_waves >> (l / 64)) & 1u))
                for (int s = L.C2; s < C; ++s)
                    if (desc[0][desc_index(s, l, lanes)] != pad || rx[(size_t)s * lanes + l] != -1)
                        return;
    }
    // leading slots in which no lane holds a term with a second factor other than 1.0 (whole
    // blocks); instances with that many one-factor slots or fewer can run the layout
    int f1 = C;
    for (int l = 0; l < lanes; ++l)
        for (int s = 0; s < f1; ++s)
            if (((desc[0][desc_index(s, l, lanes)] >> 16) & 0x7fffu) != (uint32_t)N * 8u) {
                f1 = s / 4 * 4;
                break;
            }
    L.f1 = f1;
    size_t off = 0;
    auto carve = [&](size_t bytes) {
        size_t o = off;
        off += (bytes + 255) / 256 * 256;
        return o;
    };
    size_t o_desc[2], o_lane[2], o_spec[2], o_ssrc[2];
    for (int p = 0; p < 2; ++p) {
        o_desc[p] = carve(desc[p].size() * 4);
        o_lane[p] = carve(lane_out[p].size() * 4);
        o_spec[p] = carve(species_out[p].size() * 4);
        o_ssrc[p] = carve(split_src[p].size() * 4);
    }
    const size_t o_rx = carve(rx.size() * 4);
    const size_t o_cspec = carve(cell_species.size() * 4);
    const size_t o_sfirst = carve(split_first.size() * 4);
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
    for (int p = 0; p < 2; ++p) {
        put(o_desc[p], desc[p].data(), desc[p].size() * 4);
        put(o_lane[p], lane_out[p].data(), lane_out[p].size() * 4);
        put(o_spec[p], species_out[p].data(), species_out[p].size() * 4);
        put(o_ssrc[p], split_src[p].data(), split_src[p].size() * 4);
    }
    put(o_rx, rx.data(), rx.size() * 4);
    put(o_cspec, cell_species.data(), cell_species.size() * 4);
    put(o_sfirst, split_first.data(), split_first.size() * 4);
    if (e != hipSuccess)
        return;
    for (int p = 0; p < 2; ++p) {
        StratNetwork &sn = p == 0 ? L.sn : L.sn32;
        const int B = p == 0 ? 8 : 4;
        sn.n_species = N;
        sn.n_reactions = net->n_reactions;
        sn.n_slots = C_needed;
        sn.xch = (n_cells * B + 255) / 256 * 256;
        sn.tab = sn.xch + kStratXchBytes;
        // rates of the slots the plain instance does not keep in registers
        const StratInstance *pi = find_strat_instance(W, L.SPL, L.C, p == 0 ? 0 : 4, L.f1, L.C2);
        const int spill_slots = pi ? pi->C - pi->CR : 0;
        sn.rlds = sn.tab + ((L.SPL * lanes + n_split + 1 + split_first.back()) * 4 + 15) / 16 * 16;
        sn.feat = sn.rlds + spill_slots * lanes * B;
        sn.one_waves = one_waves;
        // a lane's second and later Y cells start at the first one-factor wave
        sn.rot = one_waves ? (lanes - 64 * __builtin_ctz(one_waves)) % lanes : 0;
        sn.desc = reinterpret_cast<const uint32_t *>(base + o_desc[p]);
        sn.rx = reinterpret_cast<const int32_t *>(base + o_rx);
        sn.cell_species = reinterpret_cast<const int32_t *>(base + o_cspec);
        sn.lane_out = reinterpret_cast<const uint32_t *>(base + o_lane[p]);
        sn.species_out = reinterpret_cast<const uint32_t *>(base + o_spec[p]);
        sn.n_split = n_split;
        sn.n_chunks = split_first.back();
        sn.split_dst = (uint32_t)(N + 1 + n_packed) * B;
        sn.split_first = reinterpret_cast<const int32_t *>(base + o_sfirst);
        sn.split_src = reinterpret_cast<const uint32_t *>(base + o_ssrc[p]);
    }
    L.ok32 = true;
    L.ok = true;
}

size_t lds_bytes_variant0(const asy_network *net)
{
    return sizeof(double) * ((size_t)net->n_reactions + 2 * (size_t)net->n_species);
}

// LDS of one workgroup of variant 1: mode 4 (single precision) has float cells;
// modes 1-3 (traces, learned controller) add the network's input and hidden layers.
// Modelled cost of the slower kind of wave of a layout per step, in units of a one-factor slot:
// a two-factor slot costs 1.45 (second gather and product; measured per-slot phase times of the
// two kinds of wave, 93 and 65 cycles), a rate read from LDS (slots >= CR) 0.3.
double modeled_wave_cost(const StratLayout &L, const StratInstance &in)
{
    const int all = (1 << L.W) - 1;
    const int c2 = in.C2 > 0 ? in.C2 : in.C;
    auto lds_rates = [&](int slots) { return 0.3 * std::max(0, slots - in.CR); };
    double cost = 0.0;
    if ((int)L.one_waves != all)  // waves with two-factor terms
        cost = std::max(cost, in.F1 + 1.45 * (c2 - in.F1) + lds_rates(c2));
    if (L.one_waves)              // one-factor waves
        cost = std::max(cost, in.C + lds_rates(in.C));
    return cost;
}

// The layout a kernel family runs with W waves per zone: the balanced layout for the plain
// controller (double or single precision) where it was built and an instance exists, else the
// default layout, which every family can run.
const StratLayout &layout_for(const asy_network *net, int W, int mode)
{
    const StratLayout &B = net->strat_bal[w_index(W)];
    if ((mode == 0 || mode == 4) && B.ok && (mode == 0 || B.ok32) &&
        find_strat_instance(W, B.SPL, B.C, mode, B.f1, B.C2))
        return B;
    return net->strat[w_index(W)];
}

size_t lds_bytes_variant1(const asy_network *net, int W, int mode)
{
    const StratLayout &L = layout_for(net, W, mode);
    const bool features = mode >= 1 && mode <= 3;
    return strat_lds_bytes(mode == 4 ? L.sn32.feat : L.sn.feat, features);
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
        if (std::max(lds_bytes_variant1(net, W, 0), lds_bytes_variant1(net, W, 1)) >
            net->lds_per_group_max)
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

// Resolve the device address of `scratch` on device dev, which must be
// current; once per device (later calls return the cached address).
asy_status scratch_setup(int dev, char **out)
{
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (dev < 0 || dev >= kMaxDevices)
        return fail(ASY_ENOTSUP, "device index beyond the scratch table");
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(ASY_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") +
                                         hipGetErrorString(e));
        g_scratch_ptr[dev] = static_cast<char *>(ptr);
    }
    if (out)
        *out = g_scratch_ptr[dev];
    return ASY_OK;
}

// Per-call device scratch: the Arrhenius rates [zones][reactions] of variant 1,
// the scheduling keys and the longest-first order [zones] (the zone counter
// travels in ZoneArgs::queue).
struct CallBufs {
    double *rates;
    float *key;
    int32_t *order;
};

CallBufs net_bufs(const asy_network *net)
{
    return CallBufs{net->rate_buf, net->key_buf, net->order_buf};
}

// Queue every kernel of one call on stream s (no allocation, no host sync, so
// the sequence can be captured into a graph).
hipError_t launch_all(asy_network *net, const asy_launch &c, const DevOptions &o,
                      const ZoneArgs &za, const CallBufs &cb, hipStream_t s, int mode = 0,
                      LearnArgs la = LearnArgs{})
{
    hipLaunchKernelGGL(reset_queue_kernel, dim3(1), dim3(64), 0, s, za.queue);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    if (c.variant == 1) {
        const int W = c.threads_per_zone / 64;
        const StratLayout &L = layout_for(net, W, mode);
        const double *rates = za.k_zone;
        if (net->rate_form == ASY_RATES_ARRHENIUS) {
            const size_t total = (size_t)za.n_zones * net->n_reactions;
            const int blocks = (int)std::min<size_t>((total + 255) / 256, (size_t)net->n_cu * 16);
            hipLaunchKernelGGL(rates_arrhenius_kernel, dim3(blocks), dim3(256), 0, s, za.n_zones,
                               net->n_reactions, net->dn.A, net->dn.E, za.T, cb.rates);
            e = hipGetLastError();
            if (e != hipSuccess)
                return e;
            rates = cb.rates;
        }
        const int32_t *order = nullptr;
        if (c.zone_order == 1) {
            const int kb = (int)std::min<size_t>(((size_t)za.n_zones * kWave + 255) / 256,
                                                 (size_t)net->n_cu * 16);
            hipLaunchKernelGGL(zone_cost_kernel, dim3(kb), dim3(256), 0, s, za.n_zones,
                               net->n_reactions, rates, cb.key);
            e = hipGetLastError();
            if (e != hipSuccess)
                return e;
            const int ob = (za.n_zones + kOrderChunk - 1) / kOrderChunk;
            hipLaunchKernelGGL(zone_order_kernel, dim3(ob), dim3(1024), 0, s, za.n_zones, cb.key,
                               cb.order);
            e = hipGetLastError();
            if (e != hipSuccess)
                return e;
            order = cb.order;
        }
        const StratInstance *inst = find_strat_instance(W, L.SPL, L.C, mode, L.f1, L.C2);
        if (!inst)
            return hipErrorInvalidDeviceFunction;
        if (mode >= 1 && mode <= 3)
            la.pow2 = net->pow2;
        if (mode >= 2)
            la.mlp = net->mlp;
        const int zpg = c.zones_per_group;
        int grid = (za.n_zones + zpg - 1) / zpg;
        if (c.groups_per_cu > 0)
            grid = std::min(grid, c.groups_per_cu * net->n_cu);
        hipLaunchKernelGGL(inst->fn, dim3(grid), dim3(c.threads_per_zone * zpg),
                           lds_bytes_variant1(net, W, mode), s, mode == 4 ? L.sn32 : L.sn, o, za,
                           rates, order, la);
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
    if (o->precision != ASY_PREC_F64 && o->precision != ASY_PREC_F32)
        return fail(ASY_EINVAL, "unknown precision");
    // single precision rounds y_floor to float: below the smallest normal float it would
    // lose digits or become 0 (a species at 0 that gains anything then gives r = inf)
    if (o->precision == ASY_PREC_F32 && !(o->y_floor >= (double)FLT_MIN))
        return fail(ASY_EINVAL, "single precision needs y_floor >= FLT_MIN (1.17549435e-38)");
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
                   hipStream_t s, int mode = 0, const LearnArgs &la = LearnArgs{})
{
    if (!c.use_graph) {
        HIP_TRY(launch_all(net, c, o, za, net_bufs(net), s, mode, la));
        return ASY_OK;
    }
    std::vector<uint8_t> key;
    append_bytes(key, c);
    append_bytes(key, o);
    append_bytes(key, za);
    append_bytes(key, mode);
    append_bytes(key, la);
    append_bytes(key, net->mlp);
    if (net->graph.exec == nullptr || key != net->graph.key) {
        if (net->graph.exec) {
            HIP_TRY(hipGraphExecDestroy(net->graph.exec));
            net->graph.exec = nullptr;
            net->graph.key.clear();
        }
        if (!net->capture_stream)
            HIP_TRY(hipStreamCreateWithFlags(&net->capture_stream, hipStreamNonBlocking));
        HIP_TRY(hipStreamBeginCapture(net->capture_stream, hipStreamCaptureModeThreadLocal));
        hipError_t le = launch_all(net, c, o, za, net_bufs(net), net->capture_stream, mode, la);
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

// ---- learned step proposer: host side --------------------------------------------------------

template <bool TA, bool TB>
hipError_t launch_gemm(int M, int N, int K, const uint16_t *A, int lda, const uint16_t *B, int ldb,
                       float *C32, uint16_t *Cb, int ldc, const float *bias, const float *pre,
                       int epi, int n_store, hipStream_t s)
{
    const int tiles = (M / 16) * (N / 16);
    hipLaunchKernelGGL((gemm_bf16_kernel<TA, TB>), dim3((tiles + 3) / 4), dim3(256), 0, s, M, N, K,
                       A, lda, B, ldb, C32, Cb, ldc, bias, pre, epi, n_store);
    return hipGetLastError();
}

int mlp_pad(int n) { return (n + 31) / 32 * 32; }

// Forward pass on n samples (rows padded to a multiple of 32 with zeros).
hipError_t mlp_forward_pass(asy_mlp *m, int n, const float *x, hipStream_t s)
{
    const int B = mlp_pad(n);
    if (!m->bf16_current) {  // after new parameters; a training step's Adam keeps them current
        hipLaunchKernelGGL(mlp_cast_weights_kernel, dim3(64), dim3(256), 0, s, m->p, m->W1b, m->W2b,
                           m->W3b);
        m->bf16_current = true;
    }
    hipLaunchKernelGGL(mlp_pack_input_kernel, dim3(64), dim3(256), 0, s, n, B, x, m->xb);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    e = launch_gemm<false, false>(B, kMlpHid, kMlpInPad, m->xb, kMlpInPad, m->W1b, kMlpHid, m->a1,
                                  m->h1b, kMlpHid, m->p + kOffB1, nullptr, kEpiForward, kMlpHid, s);
    if (e != hipSuccess)
        return e;
    e = launch_gemm<false, false>(B, kMlpHid, kMlpHid, m->h1b, kMlpHid, m->W2b, kMlpHid, m->a2,
                                  m->h2b, kMlpHid, m->p + kOffB2, nullptr, kEpiForward, kMlpHid, s);
    if (e != hipSuccess)
        return e;
    return launch_gemm<false, false>(B, 16, kMlpHid, m->h2b, kMlpHid, m->W3b, 16, m->out16, nullptr,
                                     16, m->b3pad, nullptr, kEpiStore, 16, s);
}

// Forward, loss and gradient into m->g.
// With sums_in_adam the gradients of b1, b2, W3 and b3 are left in the column-sum partials
// (m->colsum) for the Adam kernel, which adds them itself.
hipError_t mlp_gradient_pass(asy_mlp *m, int n, const float *x, const float *y, float *loss,
                             hipStream_t s, bool sums_in_adam = false)
{
    const int B = mlp_pad(n);
    hipError_t e = mlp_forward_pass(m, n, x, s);
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(mlp_loss_kernel, dim3(1), dim3(1024), 0, s, n, B, m->out16, y, m->o, m->g_o,
                       m->g_ob, loss);
    hipLaunchKernelGGL(mlp_out_grad_kernel, dim3(64), dim3(256), 0, s, B, m->g_ob, m->W3b, m->a2,
                       m->g_a2, m->g_a2b);
    e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    // g_a1 = (g_a2b W2b^T) [a1 > 0]
    e = launch_gemm<false, true>(B, kMlpHid, kMlpHid, m->g_a2b, kMlpHid, m->W2b, kMlpHid, m->g_a1,
                                 m->g_a1b, kMlpHid, nullptr, m->a1, kEpiReluGrad, kMlpHid, s);
    if (e != hipSuccess)
        return e;
    // dW2 = h1b^T g_a2b, dW1 = xb^T g_a1b (the batch split over the waves of a tile)
    hipLaunchKernelGGL(gemm_bf16_wgrad_kernel, dim3((kMlpHid / 16) * (kMlpHid / 16)), dim3(256), 0,
                       s, kMlpHid, kMlpHid, B, m->h1b, kMlpHid, m->g_a2b, kMlpHid, m->g + kOffW2,
                       kMlpHid);
    hipLaunchKernelGGL(gemm_bf16_wgrad_kernel, dim3((kMlpInPad / 16) * (kMlpHid / 16)), dim3(256),
                       0, s, kMlpInPad, kMlpHid, B, m->xb, kMlpInPad, m->g_a1b, kMlpHid,
                       m->g + kOffW1, kMlpHid);
    e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    // bias gradients and the output layer's weight gradient: column sums over the batch
    const int rows_per = (B + kColsumBlocks - 1) / kColsumBlocks;
    hipLaunchKernelGGL(mlp_colsum_part_kernel, dim3(kColsumBlocks), dim3(kColsumGroups * kMlpHid),
                       0, s, B, rows_per, m->g_a1, m->g_a2, m->g_o, m->h2b, m->g_ob, m->colsum);
    if (!sums_in_adam)
        hipLaunchKernelGGL(mlp_colsum_final_kernel, dim3(1), dim3(kMlpHid), 0, s, kColsumBlocks,
                           m->colsum, m->g);
    return hipGetLastError();
}

asy_status mlp_check(const asy_mlp *m, int32_t n, const void *x)
{
    if (!m)
        return fail(ASY_EINVAL, "mlp must be non-NULL");
    if (n < 1 || n > m->batch_max)
        return fail(ASY_EINVAL, "n must be in [1, batch_max]");
    if (!x)
        return fail(ASY_EINVAL, "x must be non-NULL");
    return ASY_OK;
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
    o->precision = ASY_PREC_F64;
}

const char *asy_last_error(void) { return g_last_error.c_str(); }

const char *asy_version(void) { return "asynet 0.2 (gfx950)"; }

asy_status asy_probe_lds_bandwidth(int32_t width_bytes, double *bytes_per_second)
{
    g_last_error.clear();
    if (!bytes_per_second || (width_bytes != 8 && width_bytes != 16))
        return fail(ASY_EINVAL, "width_bytes must be 8 or 16 and bytes_per_second non-NULL");
    int dev = 0, n_cu = 0;
    HIP_TRY(hipGetDevice(&dev));
    HIP_TRY(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev));
    const int blocks = n_cu * 16;
    const int passes = width_bytes == 16 ? 4000 : 8000;
    uint32_t *sink = nullptr;
    HIP_TRY(hipMalloc(&sink, sizeof(uint32_t) * (size_t)blocks * kProbeThreads));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    auto cleanup = [&]() {
        if (e0)
            (void)hipEventDestroy(e0);
        if (e1)
            (void)hipEventDestroy(e1);
        (void)hipFree(sink);
    };
    auto launch = [&]() {
        if (width_bytes == 16)
            lds_read_probe_kernel<uint4><<<blocks, kProbeThreads, 0, nullptr>>>(passes, sink);
        else
            lds_read_probe_kernel<uint2><<<blocks, kProbeThreads, 0, nullptr>>>(passes, sink);
    };
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess)
        e = hipEventCreate(&e1);
    const int reps = 5;
    if (e == hipSuccess) {
        launch();  // warm-up
        e = hipEventRecord(e0, nullptr);
    }
    for (int r = 0; r < reps && e == hipSuccess; ++r) {
        launch();
        e = hipGetLastError();
    }
    if (e == hipSuccess)
        e = hipEventRecord(e1, nullptr);
    if (e == hipSuccess)
        e = hipEventSynchronize(e1);
    float ms = 0.0f;
    if (e == hipSuccess)
        e = hipEventElapsedTime(&ms, e0, e1);
    cleanup();
    if (e != hipSuccess)
        return fail(ASY_EDEVICE, std::string("LDS probe: ") + hipGetErrorString(e));
    const double bytes = (double)reps * blocks * kProbeThreads * (double)passes * kProbeUnroll *
                         width_bytes;
    *bytes_per_second = bytes / (ms * 1e-3);
    return ASY_OK;
}

asy_status asy_network_create(const asy_network_desc *d, asy_network **out)
{
    g_last_error.clear();
    if (!d || !out)
        return fail(ASY_EINVAL, "desc and out must be non-NULL");
    const int32_t N = d->n_species, R = d->n_reactions;
    if (N < 1 || R < 1)
        return fail(ASY_EINVAL, "n_species and n_reactions must be >= 1");
    if (d->split_above < 0 || (d->split_above > 0 && d->split_above < 8))
        return fail(ASY_EINVAL, "split_above must be 0 or >= 8");
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

    if (check_strat_lds_base() != ASY_OK)
        return ASY_EDEVICE;
    if (scratch_setup(dev, nullptr) != ASY_OK)  // device dev is current here
        return ASY_EDEVICE;

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
    const size_t o_pow2 = carve(sizeof(double) * 32);
    double pow2_tab[32];  // 2^(b/32): steps h 2^(q/32) of learned proposals and trace labels
    for (int b = 0; b < 32; ++b)
        pow2_tab[b] = std::exp2(b / 32.0);
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
    put(o_pow2, pow2_tab, sizeof(pow2_tab));
    if (ce != hipSuccess) {
        asy_network_destroy(net);
        return fail(ASY_EDEVICE, std::string("upload: ") + hipGetErrorString(ce));
    }
    net->queue = reinterpret_cast<int32_t *>(base + o_queue);
    net->pow2 = reinterpret_cast<const double *>(base + o_pow2);
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
        const int split_above = d->split_above > 0 ? d->split_above : kSplitAboveDefault;
        for (int W : {1, 2, 4}) {
            build_strat(net, W, rows, split_above);
            // a balanced layout for the plain kernels where the default one frees a wave of
            // second gathers and an instance for it exists (the first that packs)
            const StratLayout &L = net->strat[w_index(W)];
            if (!L.ok || !L.one_waves)
                continue;
            const StratInstance *din = find_strat_instance(W, L.SPL, L.C, 0, L.f1);
            if (!din)
                continue;
            for (const auto &in : kStratInstances)
                if (in.mode == 0 && in.C2 > 0 && in.W == W && in.SPL == L.SPL) {
                    build_strat(net, W, rows, split_above, &in);
                    StratLayout &B = net->strat_bal[w_index(W)];
                    const StratInstance *bin =
                        B.ok ? find_strat_instance(W, B.SPL, B.C, 0, B.f1, B.C2) : nullptr;
                    // kept only where the model expects it to be faster than the default layout
                    if (bin && modeled_wave_cost(B, *bin) < modeled_wave_cost(L, *din))
                        break;
                    if (B.dev)
                        (void)hipFree(B.dev);
                    B = StratLayout{};
                }
        }
    }
    // default launch: variant 1 with the least slot work per zone step (slots
    // per lane x waves), slots beyond 64 per lane weighted 1.25 for the
    // occupancy their rate registers cost, fewest waves on ties; else the
    // generic variant 0 (asy_autotune measures instead)
    asy_launch c{};
    c.variant = 0;
    c.threads_per_zone = N <= 64 ? 64 : (N <= 128 ? 128 : 256);
    c.zones_per_group = 1;
    {
        double best = 0.0;
        for (int W : {1, 2, 4}) {
            const StratLayout &L = net->strat[w_index(W)];
            if (!L.ok)
                continue;
            const double cost = (double)L.C * W * (L.C > 64 ? 1.25 : 1.0);
            if (c.variant == 0 || cost < best) {
                best = cost;
                c.variant = 1;
                c.threads_per_zone = 64 * W;
                c.zone_order = 1;
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
    for (auto &L : net->strat_bal)
        if (L.dev)
            (void)hipFree(L.dev);
    if (net->mlp_block)
        (void)hipFree(net->mlp_block);
    if (net->sched_block)
        (void)hipFree(net->sched_block);
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

asy_status asy_network_layout_info(const asy_network *net, int32_t threads_per_zone,
                                   asy_layout_info *info)
{
    if (!net || !info)
        return fail(ASY_EINVAL, "net and info must be non-NULL");
    if (threads_per_zone != 64 && threads_per_zone != 128 && threads_per_zone != 256)
        return fail(ASY_EINVAL, "threads_per_zone must be 64, 128 or 256");
    const StratLayout &L = layout_for(net, threads_per_zone / 64, 0);
    *info = asy_layout_info{};
    if (!L.ok)
        return ASY_OK;
    info->available = 1;
    info->slots = L.C;
    info->slots_used = L.C_needed;
    info->species_per_lane = L.SPL;
    info->split_rows = L.n_split;
    info->one_factor_waves = L.one_waves;
    info->gather_cycles_packed = L.gather_cycles_before;
    info->gather_cycles_placed = L.gather_cycles_after;
    info->one_factor_slots = L.f1;
    const StratInstance *in = find_strat_instance(L.W, L.SPL, L.C, 0, L.f1, L.C2);
    info->one_factor_slots_run = in ? in->F1 : 0;
    info->two_factor_wave_slots = L.C2 > 0 ? L.C2 : L.C;
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

namespace {

// Shared argument checks and launch of asy_integrate_batch and asy_integrate_batch_trace.
// Kernel family of a call: 0 plain, 1 plain + trace, 2 learned, 3 learned + trace, 4 plain in
// single precision; ASY_ENOTSUP / ASY_ESTATE when the network or launch cannot run it.
asy_status resolve_mode(const asy_network *net, const asy_options &o, bool trace, int *mode_out)
{
    const bool learned = o.controller == ASY_CTRL_LEARNED;
    int mode = (learned ? 2 : 0) + (trace ? 1 : 0);
    if (o.precision == ASY_PREC_F32) {
        if (mode != 0)
            return fail(ASY_ENOTSUP, "single precision supports the plain controller without trace");
        if (net->launch.variant != 1)
            return fail(ASY_ENOTSUP, "single precision needs launch variant 1");
        const StratLayout &L = layout_for(net, net->launch.threads_per_zone / 64, 4);
        if (!L.ok32 || !find_strat_instance(L.W, L.SPL, L.C, 4, L.f1, L.C2))
            return fail(ASY_ENOTSUP, "no single-precision kernel instance for this network and "
                                     "launch configuration");
        mode = 4;
    }
    if (mode != 0 && mode != 4) {
        if (net->n_species > ASY_MLP_N_IN - 4)
            return fail(ASY_ENOTSUP, "learned controller and trace take at most 162 species");
        if (learned && !net->has_mlp)
            return fail(ASY_ESTATE, "the learned controller needs asy_set_mlp first");
        if (net->launch.variant != 1)
            return fail(ASY_ENOTSUP, "learned controller and trace need launch variant 1");
        const StratLayout &L = net->strat[w_index(net->launch.threads_per_zone / 64)];
        if (!find_strat_instance(L.W, L.SPL, L.C, mode))
            return fail(ASY_ENOTSUP, "no learned/trace kernel instance for this network and "
                                     "launch configuration");
    }
    *mode_out = mode;
    return ASY_OK;
}

// Most zones asy_integrate_batch_noalloc takes on this network (-1 before a network exists):
// the keys and order hold kNoAllocMaxZones, the rate table (Arrhenius networks)
// kScratchRateBytes / (8 n_reactions).
int64_t noalloc_max_zones(const asy_network *net)
{
    if (!net)
        return -1;
    int64_t limit = kNoAllocMaxZones;
    if (net->rate_form == ASY_RATES_ARRHENIUS)
        limit = std::min<int64_t>(limit, (int64_t)(kScratchRateBytes / (8 * (size_t)net->n_reactions)));
    return limit;
}

asy_status integrate_common(asy_network *net, const asy_options *opts, int32_t n_zones, double *Y,
                            const double *T, const double *k_zone, const double *t_end, double *dt,
                            int64_t *n_accepted, int64_t *n_rejected, int32_t *zone_status,
                            void *stream, bool trace, LearnArgs la, bool noalloc = false)
{
    g_last_error.clear();
    asy_options o;
    asy_options_default(&o);
    if (opts)
        o = *opts;
    asy_status st = validate_options(&o);
    if (st != ASY_OK)
        return st;
    if (!net)
        return fail(ASY_EINVAL, "net must be non-NULL");
    if (n_zones < 0)
        return fail(ASY_EINVAL, "n_zones must be >= 0");
    if (noalloc) {
        const int64_t limit = noalloc_max_zones(net);
        if (limit >= 0 && n_zones > limit)
            return fail(ASY_EINVAL, "asy_integrate_batch_noalloc takes at most " +
                                        std::to_string(limit) + " zones for this network");
    }
    if (trace && (!la.trace || !la.count || la.capacity < 0 || la.capacity > INT32_MAX ||
                  la.stride < 1 || la.trace_zones < 0))
        return fail(ASY_EINVAL, "trace needs buffers, 0 <= capacity < 2^31, stride >= 1, "
                                "trace_zones >= 0");
    int mode = 0;
    st = resolve_mode(net, o, trace, &mode);
    if (st != ASY_OK)
        return st;
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
    if (noalloc) {
        // the counter, keys and order in this device's static scratch; no graph (instantiating
        // one allocates).  The counter is cleared by a kernel at the start of the launch; keys
        // and order are rewritten for every zone of the call.
        char *sp = nullptr;
        st = scratch_setup(net->device, &sp);
        if (st != ASY_OK)
            return st;
        za.queue = reinterpret_cast<int32_t *>(sp);
        const CallBufs cb{reinterpret_cast<double *>(sp + kScratchRateOff),
                          reinterpret_cast<float *>(sp + kScratchKeyOff),
                          reinterpret_cast<int32_t *>(sp + kScratchOrderOff)};
        HIP_TRY(launch_all(net, net->launch, to_dev(o), za, cb, s, mode, la));
        return ASY_OK;
    }
    st = ensure_call_bufs(net, net->launch, n_zones, s);
    if (st != ASY_OK)
        return st;
    return enqueue(net, net->launch, to_dev(o), za, s, mode, la);
}

}  // namespace

asy_status asy_integrate_batch(asy_network *net, const asy_options *opts, int32_t n_zones,
                               double *Y, const double *T, const double *k_zone,
                               const double *t_end, double *dt, int64_t *n_accepted,
                               int64_t *n_rejected, int32_t *zone_status, void *stream)
{
    return integrate_common(net, opts, n_zones, Y, T, k_zone, t_end, dt, n_accepted, n_rejected,
                            zone_status, stream, false, LearnArgs{});
}

asy_status asy_integrate_batch_noalloc(asy_network *net, const asy_options *opts, int32_t n_zones,
                                       double *Y, const double *T, const double *k_zone,
                                       const double *t_end, double *dt, int64_t *n_accepted,
                                       int64_t *n_rejected, int32_t *zone_status, void *stream)
{
    return integrate_common(net, opts, n_zones, Y, T, k_zone, t_end, dt, n_accepted, n_rejected,
                            zone_status, stream, false, LearnArgs{}, true);
}

asy_status asy_integrate_batch_trace(asy_network *net, const asy_options *opts, int32_t n_zones,
                                     double *Y, const double *T, const double *k_zone,
                                     const double *t_end, double *dt, int64_t *n_accepted,
                                     int64_t *n_rejected, int32_t *zone_status, float *trace,
                                     int64_t capacity, unsigned long long *count, int32_t stride,
                                     int32_t trace_zones, void *stream)
{
    LearnArgs la{};
    la.trace = trace;
    la.capacity = capacity;
    la.count = count;
    la.stride = stride;
    la.trace_zones = trace_zones;
    return integrate_common(net, opts, n_zones, Y, T, k_zone, t_end, dt, n_accepted, n_rejected,
                            zone_status, stream, true, la);
}

asy_status asy_integrate_schedule(asy_network *net, const asy_options *opts, int32_t n_zones,
                                  int32_t n_steps, double *Y, const double *T, const double *k_zone,
                                  const double *dt_hydro, double *dt, const double *q,
                                  double *energy, int64_t *n_accepted, int64_t *n_rejected,
                                  int32_t *zone_status, void *stream)
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
    if (n_zones < 0 || n_steps < 1)
        return fail(ASY_EINVAL, "n_zones must be >= 0 and n_steps >= 1");
    if (energy && !q)
        return fail(ASY_EINVAL, "the energy release needs q");
    int mode = 0;
    st = resolve_mode(net, o, false, &mode);
    if (st != ASY_OK)
        return st;
    if (n_zones == 0)
        return ASY_OK;
    if (!Y || !dt_hydro || !dt || !n_accepted || !n_rejected || !zone_status)
        return fail(ASY_EINVAL,
                    "Y, dt_hydro, dt, n_accepted, n_rejected, zone_status must be non-NULL");
    if (net->rate_form == ASY_RATES_ARRHENIUS) {
        if (!T || k_zone)
            return fail(ASY_EINVAL, "Arrhenius networks take T and no k_zone");
    } else if (!k_zone || T) {
        return fail(ASY_EINVAL, "per-zone-rate networks take k_zone and no T");
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    HIP_TRY(hipSetDevice(net->device));
    st = ensure_call_bufs(net, net->launch, n_zones, s);
    if (st != ASY_OK)
        return st;
    // per-step counters and the abundances before the step (grow-only scratch)
    const size_t nY = (size_t)n_zones * net->n_species;
    if (net->sched_zones < (size_t)n_zones) {
        HIP_TRY(hipStreamSynchronize(s));
        (void)hipFree(net->sched_block);
        net->sched_block = nullptr;
        net->sched_zones = 0;
        HIP_TRY(hipMalloc(&net->sched_block, (size_t)n_zones * (8 + 8 + 4 + 8 * net->n_species)));
        net->sched_zones = (size_t)n_zones;
    }
    char *b = static_cast<char *>(net->sched_block);
    double *before = reinterpret_cast<double *>(b);
    int64_t *acc_s = reinterpret_cast<int64_t *>(b + nY * 8);
    int64_t *rej_s = acc_s + n_zones;
    int32_t *st_s = reinterpret_cast<int32_t *>(rej_s + n_zones);
    const DevOptions dev = to_dev(o);
    const int blocks = std::max(1, std::min((n_zones + 255) / 256, net->n_cu * 4));
    for (int32_t step = 0; step < n_steps; ++step) {
        if (energy)
            HIP_TRY(hipMemcpyAsync(before, Y, nY * 8, hipMemcpyDeviceToDevice, s));
        ZoneArgs za{n_zones, Y, T ? T + (size_t)step * n_zones : nullptr, k_zone,
                    dt_hydro + (size_t)step * n_zones, dt, acc_s, rej_s, st_s, net->queue};
        HIP_TRY(launch_all(net, net->launch, dev, za, net_bufs(net), s, mode));
        hipLaunchKernelGGL(schedule_step_kernel, dim3(blocks), dim3(256), 0, s, n_zones,
                           net->n_species, step == 0 ? 1 : 0, acc_s, rej_s, st_s, n_accepted,
                           n_rejected, zone_status, Y, before, q,
                           energy ? energy + (size_t)step * n_zones : nullptr);
        HIP_TRY(hipGetLastError());
    }
    return ASY_OK;
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
    // candidates: variant 1 for each W with both zone orders, and variant 0 (double only);
    // the plain controller is timed whatever opts->controller says
    const int mode = o.precision == ASY_PREC_F32 ? 4 : 0;
    std::vector<asy_launch> cands;
    for (int W : {1, 2, 4}) {
        const StratLayout &L = layout_for(net, W, mode);
        if (!L.ok || (mode == 4 && (!L.ok32 || !find_strat_instance(W, L.SPL, L.C, 4, L.f1, L.C2))))
            continue;
        for (int zo : {1, 0}) {
            asy_launch c{1, 64 * W, 1, 0, 0, zo};
            if (validate_launch(net, &c) == ASY_OK)
                cands.push_back(c);
        }
    }
    for (int nt : {128, 256}) {
        asy_launch c{0, nt, 1, 0, 0, 0};
        if (mode == 0 && validate_launch(net, &c) == ASY_OK)
            cands.push_back(c);
    }
    g_last_error.clear();
    const asy_launch saved = net->launch;
    float best_ms = 0.0f;
    asy_launch best_c = saved;
    ZoneArgs za{Z, wY, T, k_zone, t_end, wdt, wacc, wrej, wst, net->queue};
    asy_status result = ASY_OK;
    // time one candidate: the first run warms up (and captures the graph of a graph launch),
    // the second is timed; calls go through enqueue like asy_integrate_batch
    auto time_candidate = [&](const asy_launch &c, float *ms) {
        net->launch = c;
        asy_status cst = ensure_call_bufs(net, c, Z, nullptr);
        for (int rep = 0; rep < 2 && cst == ASY_OK; ++rep) {
            if (hipMemcpy(wY, Y, nY * 8, hipMemcpyDeviceToDevice) != hipSuccess ||
                hipMemcpy(wdt, dt, (size_t)Z * 8, hipMemcpyDeviceToDevice) != hipSuccess ||
                hipEventRecord(e0, nullptr) != hipSuccess)
                return fail(ASY_EDEVICE, "autotune: a candidate launch failed");
            cst = enqueue(net, c, to_dev(o), za, nullptr, mode);
            if (cst != ASY_OK)
                return cst;
            if (hipEventRecord(e1, nullptr) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                hipEventElapsedTime(ms, e0, e1) != hipSuccess)
                return fail(ASY_EDEVICE, "autotune: a candidate launch failed");
        }
        return cst;
    };
    auto consider = [&](const asy_launch &c) {
        float ms = 0.0f;
        asy_status cst = time_candidate(c, &ms);
        if (cst == ASY_OK && (best_ms == 0.0f || ms < best_ms)) {
            best_ms = ms;
            best_c = c;
        }
        return cst;
    };
    for (const asy_launch &c : cands) {
        result = consider(c);
        if (result != ASY_OK)
            break;
    }
    // then, for the best kernel: persistent grids of 1..8 workgroups per compute unit, and
    // graph replay of each grid
    if (result == ASY_OK && !cands.empty()) {
        const asy_launch base = best_c;
        for (int gpc : {0, 1, 2, 3, 4, 6, 8}) {
            for (int graph : {0, 1}) {
                asy_launch c = base;
                c.groups_per_cu = gpc;
                c.use_graph = graph;
                if ((gpc == base.groups_per_cu && graph == base.use_graph) ||
                    validate_launch(net, &c) != ASY_OK)
                    continue;
                result = consider(c);
                if (result != ASY_OK)
                    break;
            }
            if (result != ASY_OK)
                break;
        }
    }
    g_last_error.clear();
    if (net->graph.exec) {  // the graph of the sample copies is of no use to later calls
        (void)hipGraphExecDestroy(net->graph.exec);
        net->graph.exec = nullptr;
        net->graph.key.clear();
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    cleanup();
    net->launch = (result == ASY_OK) ? best_c : saved;
    if (best)
        *best = net->launch;
    return result;
}

asy_status asy_mlp_create(int32_t batch_max, asy_mlp **out)
{
    g_last_error.clear();
    if (!out || batch_max < 1 || batch_max > (1 << 20))
        return fail(ASY_EINVAL, "batch_max must be in [1, 2^20] and out non-NULL");
    auto *m = new asy_mlp();
    m->batch_max = batch_max;
    const size_t B = (size_t)mlp_pad(batch_max);
    HIP_TRY(hipGetDevice(&m->device));
    size_t off = 0;
    auto carve = [&](size_t bytes) {
        size_t o = off;
        off += (bytes + 255) / 256 * 256;
        return o;
    };
    const size_t P = kMlpParams;
    const size_t o_p = carve(P * 4), o_g = carve(P * 4), o_m = carve(P * 4), o_v = carve(P * 4);
    const size_t o_b3 = carve(16 * 4);
    const size_t o_W1 = carve(kMlpInPad * kMlpHid * 2), o_W2 = carve(kMlpHid * kMlpHid * 2);
    const size_t o_W3 = carve(kMlpHid * 16 * 2);
    const size_t o_s1 = carve(8 * 6 * 64 * 8 * 2), o_s2 = carve(8 * 4 * 64 * 8 * 2);
    const size_t o_s3 = carve(4 * 64 * 8 * 2);
    const size_t o_xb = carve(B * kMlpInPad * 2), o_h1 = carve(B * kMlpHid * 2);
    const size_t o_h2 = carve(B * kMlpHid * 2), o_gob = carve(B * 2), o_ga2b = carve(B * kMlpHid * 2);
    const size_t o_ga1b = carve(B * kMlpHid * 2);
    const size_t o_a1 = carve(B * kMlpHid * 4), o_a2 = carve(B * kMlpHid * 4), o_o16 = carve(B * 16 * 4);
    const size_t o_o = carve(B * 4), o_go = carve(B * 4), o_ga2 = carve(B * kMlpHid * 4);
    const size_t o_ga1 = carve(B * kMlpHid * 4);
    const size_t o_cs = carve((size_t)kColsumBlocks * 4 * kMlpHid * 4);
    hipError_t e = hipMalloc(&m->block, off);
    if (e != hipSuccess) {
        delete m;
        return fail(ASY_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
    }
    char *b = static_cast<char *>(m->block);
    e = hipMemset(b, 0, off);
    if (e != hipSuccess) {
        asy_mlp_destroy(m);
        return fail(ASY_EDEVICE, std::string("hipMemset: ") + hipGetErrorString(e));
    }
    auto F = [&](size_t o) { return reinterpret_cast<float *>(b + o); };
    auto H = [&](size_t o) { return reinterpret_cast<uint16_t *>(b + o); };
    m->p = F(o_p); m->g = F(o_g); m->m = F(o_m); m->v = F(o_v); m->b3pad = F(o_b3);
    m->W1b = H(o_W1); m->W2b = H(o_W2); m->W3b = H(o_W3);
    m->w1s = H(o_s1); m->w2s = H(o_s2); m->w3s = H(o_s3);
    m->xb = H(o_xb); m->h1b = H(o_h1); m->h2b = H(o_h2); m->g_ob = H(o_gob); m->g_a2b = H(o_ga2b);
    m->g_a1b = H(o_ga1b);
    m->a1 = F(o_a1); m->a2 = F(o_a2); m->out16 = F(o_o16); m->o = F(o_o); m->g_o = F(o_go);
    m->g_a2 = F(o_ga2); m->g_a1 = F(o_ga1);
    m->colsum = F(o_cs);
    *out = m;
    return ASY_OK;
}

void asy_mlp_destroy(asy_mlp *m)
{
    if (!m)
        return;
    (void)hipDeviceSynchronize();
    if (m->block)
        (void)hipFree(m->block);
    delete m;
}

asy_status asy_mlp_set_params(asy_mlp *m, const float *params)
{
    g_last_error.clear();
    if (!m || !params)
        return fail(ASY_EINVAL, "mlp and params must be non-NULL");
    HIP_TRY(hipMemcpy(m->p, params, kMlpParams * 4, hipMemcpyHostToDevice));
    float b3pad[16] = {params[kOffB3]};
    HIP_TRY(hipMemcpy(m->b3pad, b3pad, sizeof(b3pad), hipMemcpyHostToDevice));
    HIP_TRY(hipMemset(m->m, 0, kMlpParams * 4));
    HIP_TRY(hipMemset(m->v, 0, kMlpParams * 4));
    m->t = 0;
    m->bf16_current = false;
    return ASY_OK;
}

asy_status asy_mlp_get_params(const asy_mlp *m, float *params)
{
    g_last_error.clear();
    if (!m || !params)
        return fail(ASY_EINVAL, "mlp and params must be non-NULL");
    HIP_TRY(hipMemcpy(params, m->p, kMlpParams * 4, hipMemcpyDeviceToHost));
    return ASY_OK;
}

asy_status asy_mlp_forward(asy_mlp *m, int32_t n, const float *x, float *o, void *stream)
{
    g_last_error.clear();
    asy_status st = mlp_check(m, n, x);
    if (st != ASY_OK)
        return st;
    if (!o)
        return fail(ASY_EINVAL, "o must be non-NULL");
    hipStream_t s = static_cast<hipStream_t>(stream);
    HIP_TRY(mlp_forward_pass(m, n, x, s));
    hipLaunchKernelGGL(mlp_loss_kernel, dim3(1), dim3(1024), 0, s, n, n, m->out16, nullptr, o,
                       nullptr, nullptr, nullptr);
    HIP_TRY(hipGetLastError());
    return ASY_OK;
}

asy_status asy_mlp_gradient(asy_mlp *m, int32_t n, const float *x, const float *y, float *loss,
                            float *grad, void *stream)
{
    g_last_error.clear();
    asy_status st = mlp_check(m, n, x);
    if (st != ASY_OK)
        return st;
    if (!y || !grad)
        return fail(ASY_EINVAL, "y and grad must be non-NULL");
    hipStream_t s = static_cast<hipStream_t>(stream);
    HIP_TRY(mlp_gradient_pass(m, n, x, y, loss, s));
    HIP_TRY(hipMemcpyAsync(grad, m->g, kMlpParams * 4, hipMemcpyDeviceToDevice, s));
    return ASY_OK;
}

asy_status asy_mlp_train_step(asy_mlp *m, int32_t n, const float *x, const float *y, float lr,
                              float *loss, void *stream)
{
    g_last_error.clear();
    asy_status st = mlp_check(m, n, x);
    if (st != ASY_OK)
        return st;
    if (!y || !(lr > 0.0f) || !std::isfinite(lr))
        return fail(ASY_EINVAL, "y must be non-NULL and lr finite and > 0");
    hipStream_t s = static_cast<hipStream_t>(stream);
    HIP_TRY(mlp_gradient_pass(m, n, x, y, loss, s, true));
    m->t += 1;
    const double beta1 = 0.9, beta2 = 0.999;
    const float c1 = (float)(1.0 - std::pow(beta1, (double)m->t));
    const float c2 = (float)(1.0 - std::pow(beta2, (double)m->t));
    // one thread per parameter
    hipLaunchKernelGGL(mlp_adam_kernel, dim3((kMlpParams + 255) / 256), dim3(256), 0, s, m->p, m->g,
                       m->colsum, kColsumBlocks, m->m, m->v, m->W1b, m->W2b, m->W3b, lr,
                       (float)beta1, (float)beta2, 1e-8f, c1, c2);
    HIP_TRY(hipGetLastError());
    return ASY_OK;
}

asy_status asy_mlp_train_epoch(asy_mlp *m, int32_t n_batches, int32_t batch, const float *x,
                               const float *y, float lr, float *losses, void *stream)
{
    g_last_error.clear();
    if (n_batches < 0)
        return fail(ASY_EINVAL, "n_batches must be >= 0");
    asy_status st = mlp_check(m, batch, x);
    if (st != ASY_OK)
        return st;
    if (!y || !(lr > 0.0f) || !std::isfinite(lr))
        return fail(ASY_EINVAL, "y must be non-NULL and lr finite and > 0");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const double beta1 = 0.9, beta2 = 0.999;
    for (int32_t b = 0; b < n_batches; ++b) {
        const size_t first = (size_t)b * (size_t)batch;
        HIP_TRY(mlp_gradient_pass(m, batch, x + first * kMlpIn, y + first,
                                  losses ? losses + b : nullptr, s, true));
        m->t += 1;
        const float c1 = (float)(1.0 - std::pow(beta1, (double)m->t));
        const float c2 = (float)(1.0 - std::pow(beta2, (double)m->t));
        hipLaunchKernelGGL(mlp_adam_kernel, dim3((kMlpParams + 255) / 256), dim3(256), 0, s, m->p,
                           m->g, m->colsum, kColsumBlocks, m->m, m->v, m->W1b, m->W2b, m->W3b, lr,
                           (float)beta1, (float)beta2, 1e-8f, c1, c2);
        HIP_TRY(hipGetLastError());
    }
    return ASY_OK;
}

asy_status asy_mlp_infer(asy_mlp *m, int32_t n, const float *x, float *o, void *stream)
{
    g_last_error.clear();
    asy_status st = mlp_check(m, n, x);
    if (st != ASY_OK)
        return st;
    if (!o)
        return fail(ASY_EINVAL, "o must be non-NULL");
    hipStream_t s = static_cast<hipStream_t>(stream);
    float b3 = 0.0f;
    HIP_TRY(hipStreamSynchronize(s));
    HIP_TRY(hipMemcpy(&b3, m->p + kOffB3, 4, hipMemcpyDeviceToHost));
    hipLaunchKernelGGL(mlp_swizzle_kernel, dim3(64), dim3(256), 0, s, m->p, m->w1s, m->w2s, m->w3s);
    HIP_TRY(hipGetLastError());
    MlpDevice w{m->w1s, m->w2s, m->w3s, m->p + kOffB1, m->p + kOffB2, b3};
    hipLaunchKernelGGL(mlp_infer_batch_kernel, dim3(std::min(n, 4096)), dim3(64), 0, s, n, x, w, o);
    HIP_TRY(hipGetLastError());
    return ASY_OK;
}

asy_status asy_set_mlp(asy_network *net, const asy_mlp *m)
{
    g_last_error.clear();
    if (!net || !m)
        return fail(ASY_EINVAL, "net and mlp must be non-NULL");
    if (net->n_species > ASY_MLP_N_IN - 4)
        return fail(ASY_ENOTSUP, "the learned controller takes at most 162 species");
    HIP_TRY(hipSetDevice(net->device));
    if (!net->mlp_block) {
        const size_t bytes = (8 * 6 + 8 * 4 + 4) * 64 * 8 * 2 + 2 * kMlpHid * 4;
        HIP_TRY(hipMalloc(&net->mlp_block, bytes));
    }
    uint16_t *w = static_cast<uint16_t *>(net->mlp_block);
    uint16_t *w1s = w, *w2s = w1s + 8 * 6 * 64 * 8, *w3s = w2s + 8 * 4 * 64 * 8;
    float *bias = reinterpret_cast<float *>(w3s + 4 * 64 * 8);
    HIP_TRY(hipDeviceSynchronize());
    hipLaunchKernelGGL(mlp_swizzle_kernel, dim3(64), dim3(256), 0, nullptr, m->p, w1s, w2s, w3s);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpy(bias, m->p + kOffB1, kMlpHid * 4, hipMemcpyDeviceToDevice));
    HIP_TRY(hipMemcpy(bias + kMlpHid, m->p + kOffB2, kMlpHid * 4, hipMemcpyDeviceToDevice));
    float b3 = 0.0f;
    HIP_TRY(hipMemcpy(&b3, m->p + kOffB3, 4, hipMemcpyDeviceToHost));
    HIP_TRY(hipDeviceSynchronize());
    net->mlp = MlpDevice{w1s, w2s, w3s, bias, bias + kMlpHid, b3};
    net->has_mlp = true;
    return ASY_OK;
}

}  // extern "C"
