// Variant 1 of the integrator: packed rows, rates in registers.
//
// The creation flux F+_i and the depletion rate k_i of Eq. (eq1.1) are sums
// over the reactions that create or destroy species i.  Each such sum is a
// "row" of terms, every term of the form (k_j * Y[x]) * Y[y]:
//   creation of i by j:          x = first reactant, y = second reactant (or ONE)
//   depletion of i by j:         x = the other reactant (or ONE),  y = ONE
// where ONE is an extra LDS cell holding 1.0, so a one-body flux is
// (k_j * Y_a) * 1.0 and a one-body depletion rate is (k_j * 1.0) * 1.0 --
// products by 1.0 are exact, and every row is summed from +0.0 in ascending
// reaction index, exactly as the plain definition does.
//
// The host pads every row to a multiple of 4 terms with zero-rate terms
// (adding +0.0 leaves a sum unchanged) and packs the 2N rows onto the 64*W
// lanes of a zone's workgroup, longest first, each onto the lane with the
// least work so far -- or, where that frees whole waves, the rows with a
// second factor other than ONE first-fit onto the first lanes, so that the
// remaining waves hold only terms (k_j * Y[x]) * 1.0 and run a copy of the
// slot phase without the second gather and the product by 1.0 (exact).  A
// lane's column is its padding, then its rows back to back, so a row ends at
// the end of a block of 4 slots, at a different block on each lane.  The sums land in the LDS cells after Y in lane order -- lane l's k-th
// row in cell lane_out[l] + k -- so a lane needs only one bit per block, set
// in the first descriptor of the block where one of its rows ends, and a
// running cell address (a block-wide mask of the blocks where some lane ends a
// row would skip the test elsewhere, but the compiler keeps it as one scalar
// register pair per block, which spills scalars at 44 slots and more, and at
// these sizes nearly every block ends a row on some lane).  Each species' update reads
// its two sums through a per-species pair of cell addresses.
// The zone's rates are loaded once into registers (slot s of the lane holds
// the rate of its term s), so per step the only random LDS traffic is the
// abundance gathers.  The term descriptors stream from global memory in
// slot-major order and stay in the L1/L2 caches for all zones.
//
// The kernel keeps all of its LDS in the dynamic allocation (it declares no
// static LDS), which therefore starts at LDS address 0: descriptors and cell
// tables hold absolute LDS byte addresses, and a gather is one mask or
// bit-field extract of a descriptor.  Which Y cell holds which species, which
// lane holds which column and the order of rows within a column are chosen on
// the host to spread each gather over the LDS banks (lds_layout.h); a lane
// updates the species in its Y cells, whatever they are.
#pragma once

#include "integrate_kernels.h"
#include "mlp_kernels.h"

namespace asynet {

struct StratNetwork {
    int32_t n_species;
    int32_t n_reactions;
    int32_t n_slots;           // slots used (<= compile-time C)
    int32_t xch;               // LDS byte address of the exchange area (after the zone's cells)
    int32_t tab;               // LDS byte address of species_out (lane-major: the entry of
                               // the lane's m-th Y cell at zl * SPL + m), split_first, split_src
    int32_t rlds;              // LDS byte address of the rates of slots >= CR (instances that
                               // keep only CR slots' rates in registers): [C - CR][lanes] of T
    int32_t feat;              // LDS byte address of the learned controller's input and layers
    int32_t rot;               // rotation of the lanes' second and later Y cells
    uint32_t one_waves;        // bit w: every term of wave w has the 1.0 cell as second factor
                               // (no second gathers, no multiplies by 1.0)
    const uint32_t *desc;      // [C/4][lanes][4]: LDS byte address of Y[x] | that of Y[y] << 16,
                               // bit 31 set in slot 4b when the lane ends a row in block b;
                               // a lane's 4 descriptors of a block are one 16-byte load
    const int32_t *rx;         // [C][lanes]: reaction of the term, -1 for padding
    const uint32_t *lane_out;  // [lanes]: LDS byte address of the lane's first row sum
    const int32_t *cell_species;  // [N]: species held by Y cell c (cell N holds 1.0)
    const uint32_t *species_out;  // [N]: by Y cell c, address of F+ | address of k << 16
    // rows longer than a chunk are summed in chunks; split row q adds the sums at
    // split_src[split_first[q] .. split_first[q+1]-1], in that order, into the cell at
    // split_dst + q * sizeof(cell)
    int32_t n_split;
    int32_t n_chunks;
    uint32_t split_dst;
    const int32_t *split_first;   // [n_split + 1]
    const uint32_t *split_src;    // [n_chunks]
};

// LDS of a zone's workgroup after its cells: the exchange area (cross-wave
// reductions, the zone ticket), copies of the cell tables, and (learned
// controller and traces) the network input and hidden layers.
constexpr int kStratXchBytes = 128;
constexpr int kStratFeatBytes = (kMlpInPad + 2 * kMlpHid) * 4;

__host__ __device__ inline size_t strat_lds_bytes(int feat, bool features)
{
    return (size_t)feat + (features ? kStratFeatBytes : 0);
}

// Loads and stores at absolute LDS byte addresses.
template <typename T>
__device__ inline T lds_ld(uint32_t a)
{
    return *reinterpret_cast<const __attribute__((address_space(3))) T *>((size_t)a);
}
template <typename T>
__device__ inline void lds_st(uint32_t a, T v)
{
    *reinterpret_cast<__attribute__((address_space(3))) T *>((size_t)a) = v;
}

// Arrhenius rates of every zone, k[z][j] = A_j exp(-E_j / T_z), once per call.
// A non-finite T gives NaN rates and T <= 0 gives -1, which the integrator's
// input checks turn into the zone statuses NONFINITE and BAD_INPUT.
__global__ void __launch_bounds__(256)
rates_arrhenius_kernel(int32_t n_zones, int32_t n_reactions, const double *A, const double *E,
                       const double *T, double *k)
{
    const size_t total = (size_t)n_zones * n_reactions;
    for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (size_t)gridDim.x * blockDim.x) {
        const int z = (int)(idx / n_reactions);
        const int j = (int)(idx - (size_t)z * n_reactions);
        const double Tz = T[z];
        double kj;
        if (!isfinite(Tz))
            kj = NAN;
        else if (!(Tz > 0.0))
            kj = -1.0;
        else
            kj = A[j] * rate_exp(-E[j] / Tz);
        k[idx] = kj;
    }
}

// Scheduling key of each zone: the sum of its rate constants (for Arrhenius
// rates it grows with T, and step counts grow with it).  One wave per zone.
// Non-finite or negative sums (zones that fail their input checks) get key 0.
__global__ void __launch_bounds__(256)
zone_cost_kernel(int32_t n_zones, int32_t n_reactions, const double *rates, float *key)
{
    const int wave = (blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const int lane = threadIdx.x % kWave;
    const int n_waves = gridDim.x * blockDim.x / kWave;
    for (int z = wave; z < n_zones; z += n_waves) {
        const double *kz = rates + (size_t)z * n_reactions;
        double s = 0.0;
        for (int j = lane; j < n_reactions; j += kWave)
            s += kz[j];
        for (int off = kWave / 2; off > 0; off >>= 1)
            s += __shfl_xor(s, off, kWave);
        if (lane == 0)
            key[z] = (isfinite(s) && s > 0.0) ? (float)s : 0.0f;
    }
}

// Longest-first scheduling order: each workgroup sorts one chunk of up to
// kOrderChunk zones by descending key (bitonic sort in LDS on key bits | zone
// index; keys are non-negative floats, whose bit patterns order like the
// values) and writes the chunk's zone indices in that order.
constexpr int kOrderChunk = 16384;

__global__ void __launch_bounds__(1024)
zone_order_kernel(int32_t n_zones, const float *key, int32_t *order)
{
    __shared__ unsigned long long v[kOrderChunk];
    const int base = blockIdx.x * kOrderChunk;
    const int n = min(kOrderChunk, n_zones - base);
    int pow2 = 1;
    while (pow2 < n)
        pow2 <<= 1;
    for (int i = threadIdx.x; i < pow2; i += blockDim.x) {
        unsigned long long e = 0;  // padding sorts last (key 0, descending order)
        if (i < n) {
            const unsigned int kb = __float_as_uint(key[base + i]);
            // descending key, then ascending zone index: sort ascending on (~key, index)
            e = ((unsigned long long)(~kb) << 32) | (unsigned int)(base + i);
        } else {
            e = ~0ull;
        }
        v[i] = e;
    }
    __syncthreads();
    for (int size = 2; size <= pow2; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int i = threadIdx.x; i < pow2; i += blockDim.x) {
                const int j = i ^ stride;
                if (j > i) {
                    const bool up = (i & size) == 0;
                    const unsigned long long a = v[i], b = v[j];
                    if ((a > b) == up) {
                        v[i] = b;
                        v[j] = a;
                    }
                }
            }
            __syncthreads();
        }
    }
    for (int i = threadIdx.x; i < n; i += blockDim.x)
        order[base + i] = (int32_t)(v[i] & 0xffffffffu);
}

// Learned controller and trace output of variant 1.
//  Trace record (kTraceRec floats) per sampled state n (after the n-th accepted step):
//   [0, 166) features of the state, [166] training label (the largest accepted step of a
//   grid around the last step, see boundary_label below), [167] 32 q of the learned
//   proposal made from the state (NaN for the plain controller), [168] zone, [169] n.
constexpr int kTraceRec = 170;

struct LearnArgs {
    MlpDevice mlp;
    const double *pow2;  // [32]: 2^(b/32) (learned proposals, trace labels)
    float *trace;        // [capacity][kTraceRec] or nullptr
    int64_t capacity;
    unsigned long long *count;  // records taken (may exceed capacity)
    int32_t stride;      // record every stride-th accepted state
    int32_t trace_zones; // only zones below this index record
};

template <bool B>
struct BoolTag {
    static constexpr bool value = B;
};

template <int W>
__device__ inline void zone_sync()
{
    if constexpr (W == 1) {
        // one wave: LDS operations of a wave complete in order; this only keeps
        // the compiler from moving LDS accesses across the phase boundary
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    } else {
        __syncthreads();
    }
}

// A workgroup of W waves integrates one zone at a time.
// Waves per SIMD (the register budget the compiler gets): the zone's rates
// take C registers per 4 bytes of T, the pipelines, addresses and update the
// rest.  Occupancy outweighs some spilling at up to 40 slots (3 waves in
// double, 4 in float) and up to 56 slots in float (3 waves), as measured on
// the 150- and 365-species workloads; otherwise the budget leaves about 128
// (double) or 96 (float) registers beside the rates.
template <int C, typename T = double>
constexpr int strat_waves_per_eu()
{
    if (sizeof(T) == 8 && C <= 40)
        return 3;
    if (sizeof(T) == 4 && C <= 40)
        return 4;
    if (sizeof(T) == 4 && C <= 56)
        return 3;
    constexpr int regs = C * (int)(sizeof(T) / 4) + (sizeof(T) == 8 ? 128 : 96);
    return 512 / regs < 1 ? 1 : (512 / regs > 8 ? 8 : 512 / regs);
}

// Abundance-gather distance in blocks: 1 where the budget above is tight in
// double precision, else 2.
template <int C, typename T = double>
constexpr int strat_gather_ahead()
{
    return (sizeof(T) == 8 && C <= 40) ? 1 : 2;
}

// CR: the slots whose rates live in registers (the rest are read from LDS every step, one
// conflict-free read per slot: lanes read consecutive cells), which lets a network that needs
// many slots keep the register budget -- and occupancy -- of CR slots.
// F1: leading slots that hold only terms with the 1.0 cell as second factor on every lane (the
// host packs a lane's rows with such terms first and verifies the layout), so the waves that do
// run two-factor terms skip the second gather and the product by 1.0 there too (exact).
// C2: slots of the waves that hold two-factor terms; their lanes' rows all end by slot C2 (the
// host packs them so), and they stop there, while the one-factor waves run all C slots -- the
// two kinds of wave get about equal work per step.
template <int W, int SPL, int C, int GA = 2, bool LEARNED = false, bool TRACE = false,
          typename T = double, int CR = C, int F1 = 0, int C2 = C>
__global__ void __attribute__((amdgpu_flat_work_group_size(64 * W, 64 * W),
                               amdgpu_waves_per_eu(strat_waves_per_eu<CR, T>())))
integrate_strat_kernel(StratNetwork sn, DevOptions o, ZoneArgs za, const double *rates,
                       const int32_t *order, LearnArgs la)
{
    constexpr bool FEATURES = LEARNED || TRACE;
    static_assert(!FEATURES || sizeof(T) == 8, "learned controller and trace in double only");
    static_assert(C % 4 == 0, "slots come in blocks of 4");
    static_assert(CR % 4 == 0 && CR <= C, "register-held rates cover whole blocks");
    static_assert(F1 % 4 == 0 && F1 <= C, "one-factor slots cover whole blocks");
    static_assert(C2 % 4 == 0 && F1 <= C2 && C2 <= C, "two-factor waves run whole blocks");
    static_assert(W <= 4, "the exchange area holds 4 waves");
    constexpr int LANES = 64 * W;
    extern __shared__ double lds[];

    const int N = sn.n_species;
    const int R = sn.n_reactions;
    const int tid = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid / kWave);  // uniform: scalar addresses
    const int lane = tid % kWave;
    const int zl = tid;  // lane within the zone
    T *Y = reinterpret_cast<T *>(lds);
    char *xb = reinterpret_cast<char *>(lds) + sn.xch;
    double *xw_r = reinterpret_cast<double *>(xb);        // [W]
    double *xw_sum = reinterpret_cast<double *>(xb + 32); // [W]
    int *xw_flag = reinterpret_cast<int *>(xb + 64);      // [W]
    int &xw_zone = *reinterpret_cast<int *>(xb + 80);
    float &xw_o = *reinterpret_cast<float *>(xb + 84);
    float *feat = reinterpret_cast<float *>(reinterpret_cast<char *>(lds) + sn.feat);
    float *hs = feat + kMlpInPad;  // [2 * kMlpHid]
    // Y cells of the lane: zl, then m * lanes + ((zl + rot) mod lanes) for m > 0, so that the
    // cells past the first lanes-many go first to the one-factor waves (measured faster)
    auto cell_at = [&](int m) {
        return m == 0 ? zl : m * LANES + ((zl + sn.rot) & (LANES - 1));
    };
    // the lane's first row-sum cell; its species' F+ / k cells, read from LDS where
    // needed (held in registers across the step loop they would spill), lane-major
    // so that one read fetches all of a lane's entries
    const uint32_t wbase = sn.lane_out[zl];
    uint32_t *tab_species = reinterpret_cast<uint32_t *>(reinterpret_cast<char *>(lds) + sn.tab);
    int32_t *tab_first = reinterpret_cast<int32_t *>(tab_species + SPL * LANES);
    uint32_t *tab_src = reinterpret_cast<uint32_t *>(tab_first + sn.n_split + 1);
#pragma unroll
    for (int m = 0; m < SPL; ++m) {
        const int i = cell_at(m);
        tab_species[zl * SPL + m] = i < N ? sn.species_out[i] : 0u;
    }
    if (sn.n_split > 0) {
        for (int q = zl; q <= sn.n_split; q += LANES)
            tab_first[q] = sn.split_first[q];
        for (int c = zl; c < sn.n_chunks; c += LANES)
            tab_src[c] = sn.split_src[c];
    }

    for (;;) {
        // ---- next zone: a wave-wide atomic, lane 0's ticket broadcast by a cross-lane read
        int z;
        if constexpr (W == 1) {
            int ticket = atomicAdd(za.queue, lane == 0 ? 1 : 0);
            z = __shfl(ticket, 0, kWave);
        } else {
            if (wave == 0) {
                int ticket = atomicAdd(za.queue, lane == 0 ? 1 : 0);
                ticket = __shfl(ticket, 0, kWave);
                if (lane == 0)
                    xw_zone = ticket;
            }
            __syncthreads();
            z = __builtin_amdgcn_readfirstlane(xw_zone);
            __syncthreads();
        }
        if (z >= za.n_zones)
            break;
        if (order)  // tickets walk the zones in the scheduling order
            z = __builtin_amdgcn_readfirstlane(order[z]);

        // ---- load the zone: rates into registers (evaluated once per interval), Y into LDS
        const double t_end = za.t_end[z];
        const double dt0 = za.dt[z];
        int flag = 0;  // bit 0: non-finite input, bit 1: out-of-domain input
        // rates: gathered once per zone from the [zone][reaction] table (the
        // per-zone input, or the table the Arrhenius rate kernel filled)
        T kr[CR];
        const uint32_t rl_lane = (uint32_t)sn.rlds + (uint32_t)zl * (uint32_t)sizeof(T);
        {
            const double *kz = rates + (size_t)z * R;
#pragma unroll
            for (int s = 0; s < C; ++s) {
                const int j = sn.rx[s * LANES + zl];
                double kj = 0.0;
                if (j >= 0) {
                    kj = kz[j];
                    if (!isfinite(kj))
                        flag |= 1;
                    else if (kj < 0.0)
                        flag |= 2;
                }
                if (s < CR)
                    kr[s] = (T)kj;
                else
                    lds_st<T>(rl_lane + (uint32_t)((s - CR) * LANES * (int)sizeof(T)), (T)kj);
            }
        }
        const double *Yz = za.Y + (size_t)z * N;
#pragma unroll
        for (int m = 0; m < SPL; ++m) {
            const int i = cell_at(m);  // Y cell
            if (i < N) {
                const double y = Yz[sn.cell_species[i]];
                Y[i] = (T)y;
                if (!isfinite(y))
                    flag |= 1;
                else if (y < 0.0)
                    flag |= 2;
            }
        }
        if (zl == 0)
            Y[N] = (T)1.0;
        if (!isfinite(t_end) || !isfinite(dt0))
            flag |= 1;
        else if (t_end < 0.0 || !(dt0 > 0.0))
            flag |= 2;
        flag = wave_or(flag);
        if constexpr (W > 1) {
            if (lane == 0)
                xw_flag[wave] = flag;
            __syncthreads();
            flag = 0;
#pragma unroll
            for (int w = 0; w < W; ++w)
                flag |= xw_flag[w];
        }
        zone_sync<W>();
        if (flag) {
            if (zl == 0) {
                za.status[z] = (flag & 1) ? kZoneNonfinite : kZoneBadInput;
                za.n_acc[z] = 0;
                za.n_rej[z] = 0;
            }
            zone_sync<W>();
            continue;  // Y and dt stay as given
        }

        // ---- integrate over [0, t_end]
        double t = 0.0, step = dt0;
        int64_t nacc = 0, nrej = 0;
        int32_t status = kZoneOk;
        double plain_step = dt0;   // learned: the plain proposal to fall back to
        bool mlp_attempt = false;  // learned: the current attempt uses the network's proposal
        if constexpr (FEATURES) {
            for (int c = zl; c < kMlpInPad; c += 64 * W)
                feat[c] = 0.0f;
        }
        // every term of this wave has the 1.0 cell as second factor (a uniform value)
        const bool one_wave = (sn.one_waves >> __builtin_amdgcn_readfirstlane(wave)) & 1u;
        constexpr int NB = C / 4;
        // descriptor prefetch distance, in blocks of 4 slots (measured: 4 blocks is 1 % faster than
        // 3 up to 44 slots, 16 % slower at 56 slots, where the descriptors in flight cost occupancy)
        constexpr int kDescAhead = C <= 44 ? 4 : 3;
        constexpr int kGatherAhead = GA; // abundance-gather distance, in blocks
        uint32_t dq[C];
        // The descriptors are read through a buffer resource: the lane's byte offset is one
        // register for the whole zone and a block's offset is a scalar, so a load costs no
        // vector address arithmetic (a 64-bit pointer per block costs two adds per load).
        const __amdgpu_buffer_rsrc_t dsc_rsrc = __builtin_amdgcn_make_buffer_rsrc(
            const_cast<uint32_t *>(sn.desc), (short)0, C * LANES * 4, 0x00020000);
        const int dsc_lane = zl * 16;
        int dsc_base = 0;
        // the descriptors of block b (one 16-byte load per lane)
        auto load_block = [&](int b) {
            const auto v = __builtin_amdgcn_raw_buffer_load_b128(dsc_rsrc, dsc_lane,
                                                                 dsc_base + b * LANES * 16, 0);
            dq[4 * b] = v[0];
            dq[4 * b + 1] = v[1];
            dq[4 * b + 2] = v[2];
            dq[4 * b + 3] = v[3];
        };
        {
            // opaque offset: the descriptor loads stay inside the step loop
            // instead of being hoisted into registers for the whole zone
            asm volatile("" : "+s"(dsc_base));
#pragma unroll
            for (int b = 0; b < kDescAhead && b < NB; ++b)
                load_block(b);
        }
        for (;;) {
            if (t >= t_end) {
                status = kZoneOk;
                break;
            }
            if (nacc + nrej >= o.max_steps) {
                status = kZoneMaxSteps;
                break;
            }
            const bool clipped = step >= t_end - t;
            const double h = clipped ? t_end - t : step;

            // Creation fluxes and depletion rates: the lane's packed rows.
            // Rows end on multiples of 4 slots; a lane's test at the end of a
            // block is the sign of the block's first descriptor.
            // Software pipeline: while block b is summed, the gathers of blocks
            // up to b+kGatherAhead and the descriptors of block b+kDescAhead are
            // in flight; the first kDescAhead blocks' descriptors of a step are
            // loaded during the previous step's update.
            // one copy of the slot phase per kind of wave: where every second factor is
            // the 1.0 cell, no second gathers and no products by 1.0 (exact)
            auto slot_phase = [&](auto one_tag) {
                constexpr bool ONE = decltype(one_tag)::value;
                constexpr int NBP = ONE ? NB : C2 / 4;  // blocks this kind of wave runs
                T gx[C], gy[C], kl[C];
                // slot s's rate: a register, or (s >= CR) an LDS read issued with its gathers
                auto rate_of = [&](int s) -> T { return s < CR ? kr[s < CR ? s : 0] : kl[s]; };
                auto gather = [&](int s) {
                    gx[s] = lds_ld<T>(dq[s] & 0xffffu);
                    if (!ONE && s >= F1)  // s is a constant of the unrolled loops
                        gy[s] = lds_ld<T>((dq[s] >> 16) & 0x7fffu);
                    if (s >= CR)
                        kl[s] = lds_ld<T>(rl_lane + (uint32_t)((s - CR) * LANES * (int)sizeof(T)));
                };
#pragma unroll
                for (int s = 0; s < 4 * kGatherAhead && s < 4 * NBP; ++s)
                    gather(s);
                T acc = (T)0.0;
                uint32_t wp = wbase;
#pragma unroll
                for (int b = 0; b < NBP; ++b) {
                    if (b + kDescAhead < NBP)
                        load_block(b + kDescAhead);
#pragma unroll
                    for (int s = 4 * (b + kGatherAhead); s < 4 * (b + kGatherAhead + 1) && s < 4 * NBP;
                         ++s)
                        gather(s);
#pragma unroll
                    for (int s = 4 * b; s < 4 * b + 4; ++s) {
                        if (ONE || s < F1)  // second factor 1.0: the product by 1.0 is exact
                            acc = acc + rate_of(s) * gx[s];
                        else
                            acc = acc + (rate_of(s) * gx[s]) * gy[s];
                    }
                    if ((int32_t)dq[4 * b] < 0) {
                        lds_st<T>(wp, acc);
                        wp += sizeof(T);
                        acc = (T)0.0;
                    }
                }
            };
            if (one_wave)
                slot_phase(BoolTag<true>{});
            else
                slot_phase(BoolTag<false>{});
            // descriptors of the first blocks of the next step
            {
                dsc_base = 0;
                asm volatile("" : "+s"(dsc_base));
#pragma unroll
                for (int b = 0; b < kDescAhead && b < NB; ++b)
                    load_block(b);
            }
            zone_sync<W>();
            if (sn.n_split > 0) {
                // split rows: their chunk sums, added in chunk order
                for (int q = zl; q < sn.n_split; q += LANES) {
                    const int f = tab_first[q], l = tab_first[q + 1];
                    T sum = lds_ld<T>(tab_src[f]);
                    int c = f + 1;
                    for (; c + 4 <= l; c += 4) {  // four loads in flight, added in order
                        const T v0 = lds_ld<T>(tab_src[c]), v1 = lds_ld<T>(tab_src[c + 1]);
                        const T v2 = lds_ld<T>(tab_src[c + 2]), v3 = lds_ld<T>(tab_src[c + 3]);
                        sum = sum + v0;
                        sum = sum + v1;
                        sum = sum + v2;
                        sum = sum + v3;
                    }
                    for (; c < l; ++c)
                        sum = sum + lds_ld<T>(tab_src[c]);
                    lds_st<T>(sn.split_dst + (uint32_t)(q * sizeof(T)), sum);
                }
                zone_sync<W>();
            }

            // kappa-switched update of the lane's species and the change measure
            T yn[SPL];
            T rloc = (T)0.0;
            bool bad = false;
            const T hT = (T)h, kappaT = (T)o.kappa, floorT = (T)o.y_floor;
            // the lane's sums, read together (entries past N read Y[0] and go unused)
            T fpv[SPL], kdv[SPL];
            {
                uint32_t spv[SPL];
#pragma unroll
                for (int m = 0; m < SPL; ++m)
                    spv[m] = tab_species[zl * SPL + m];
#pragma unroll
                for (int m = 0; m < SPL; ++m) {
                    fpv[m] = lds_ld<T>(spv[m] & 0xffffu);
                    kdv[m] = lds_ld<T>(spv[m] >> 16);
                }
            }
#pragma unroll
            for (int m = 0; m < SPL; ++m) {
                const int i = cell_at(m);
                yn[m] = (T)0.0;
                if (i < N) {
                    const T fp = fpv[m];
                    const T kd = kdv[m];
                    const T y = Y[i];
                    const T kh = kd * hT;
                    T v;
                    if (kh < kappaT)
                        v = y + hT * (fp - kd * y);          // forward Euler
                    else
                        v = (y + hT * fp) / ((T)1.0 + kh);   // asymptotic form
                    yn[m] = v;
                    if (!isfinite(v))
                        bad = true;
                    else
                        rloc = fmax(rloc, fabs(v - y) / fmax(y, floorT));
                }
            }
            if (bad)
                rloc = (T)INFINITY;
            double r = (double)wave_max_nonneg_dpp(rloc);
            if constexpr (W > 1) {
                if (lane == 0)
                    xw_r[wave] = r;
                __syncthreads();
                r = xw_r[0];
#pragma unroll
                for (int w = 1; w < W; ++w)
                    r = fmax(r, xw_r[w]);
            }
            if (r <= o.tol) {
#pragma unroll
                for (int m = 0; m < SPL; ++m) {
                    const int i = cell_at(m);
                    if (i < N)
                        Y[i] = yn[m];
                }
                ++nacc;
                t = clipped ? t_end : t + h;
                if (!clipped) {
                    const double g = (r == 0.0) ? o.grow_max : fmin(o.grow_max, o.safety * o.tol / r);
                    step = h * g;
                }
                mlp_attempt = false;
                if constexpr (FEATURES) {
                    const bool propose = !clipped && t < t_end;
                    const bool record = TRACE && propose && z < la.trace_zones &&
                                        (nacc % la.stride) == 0;
                    if ((LEARNED && propose) || record) {
                        // features of the accepted state (depletion rates of this step)
                        double kmax = 0.0, ksum = 0.0;
#pragma unroll
                        for (int m = 0; m < SPL; ++m) {
                            const int i = cell_at(m);
                            if (i < N) {
                                const double y = yn[m];
                                feat[sn.cell_species[i]] =
                                    (float)(fmax(log10(fmax(y, 1e-300)), -30.0) / 30.0);
                                const double kh = lds_ld<double>(tab_species[zl * SPL + m] >> 16) * h;
                                kmax = fmax(kmax, kh);
                                ksum += kh;
                            }
                        }
                        kmax = wave_max_nonneg_dpp(kmax);
                        ksum = wave_sum_dpp(ksum);
                        if constexpr (W > 1) {
                            zone_sync<W>();
                            if (lane == 0) {
                                xw_r[wave] = kmax;
                                xw_sum[wave] = ksum;
                            }
                            __syncthreads();
                            kmax = xw_r[0];
                            ksum = xw_sum[0];
#pragma unroll
                            for (int w = 1; w < W; ++w) {
                                kmax = fmax(kmax, xw_r[w]);
                                ksum += xw_sum[w];
                            }
                        }
                        if (zl == 0) {
                            feat[N] = (float)(log10(fmax(kmax, 1e-300)) / 10.0);
                            feat[N + 1] = (float)(log10(fmax(ksum / N, 1e-300)) / 10.0);
                            feat[N + 2] = (float)(log10(h) / 10.0);
                            feat[N + 3] = (float)(log10(o.tol) / 10.0);
                        }
                        zone_sync<W>();
                        int q32 = 0;
                        if constexpr (LEARNED) {
                            if (propose) {
                                const float ov = mlp_infer_group<W>(
                                    la.mlp, feat, hs, hs + kMlpHid, &xw_o, lane, wave,
                                    [] { zone_sync<W>(); });
                                const double oc = fmin(fmax((double)ov, -3.0), 3.0);
                                q32 = (int)rint(32.0 * oc);
                                const int qa = (q32 >= 0) ? q32 / 32 : -((31 - q32) / 32);
                                const int qb = q32 - 32 * qa;
                                plain_step = step;
                                step = ldexp(h * la.pow2[qb], qa);
                                mlp_attempt = true;
                            }
                        }
                        if (record) {
                            // slot of the record; -1 once the buffer is full (capacity < 2^31)
                            int slot = -1;
                            if (zl == 0) {
                                const unsigned long long c = atomicAdd(la.count, 1ull);
                                slot = (c < (unsigned long long)la.capacity) ? (int)c : -1;
                            }
                            slot = __shfl(slot, 0, kWave);
                            if constexpr (W > 1) {
                                if (tid == 0)
                                    xw_zone = slot;
                                __syncthreads();
                                slot = __builtin_amdgcn_readfirstlane(xw_zone);
                            }
                            if (slot >= 0) {
                                float *rec = la.trace + (int64_t)slot * kTraceRec;
                                for (int c = zl; c < kMlpIn; c += 64 * W)
                                    rec[c] = feat[c];
                                if (zl == 0) {
                                    rec[167] = LEARNED ? (float)q32 : NAN;
                                    rec[168] = (float)z;
                                    rec[169] = (float)nacc;
                                }
                            }
                            zone_sync<W>();
                            if constexpr (TRACE) {
                                if (slot >= 0) {
                                    // Training label of the accepted state the step h reached (trace output):
                                    // log2 of safety times the largest step of the grid h 2^(q/32), q = -96..96,
                                    // whose attempt from the state the controller would accept, over h; NaN if no
                                    // step of the grid is accepted.  Bisection on q, taking acceptance as monotone
                                    // in the step: the state's sums once, then only the update and change measure
                                    // per trial step.  Nothing of the zone changes.
                                    auto boundary_label = [&](double hb) {
                                        // the sums of the accepted state (the same phase as a step's)
                                        if (one_wave)
                                            slot_phase(BoolTag<true>{});
                                        else
                                            slot_phase(BoolTag<false>{});
                                        // descriptors of the first blocks of the next step
                                        {
                                            dsc_base = 0;
                                            asm volatile("" : "+s"(dsc_base));
#pragma unroll
                                            for (int b = 0; b < kDescAhead && b < NB; ++b)
                                                load_block(b);
                                        }
                                        zone_sync<W>();
                                        if (sn.n_split > 0) {
                                            // split rows: their chunk sums, added in chunk order
                                            for (int q = zl; q < sn.n_split; q += LANES) {
                                                const int f = tab_first[q], l = tab_first[q + 1];
                                                T sum = lds_ld<T>(tab_src[f]);
                                                int c = f + 1;
                                                for (; c + 4 <= l; c += 4) {  // four loads in flight, added in order
                                                    const T v0 = lds_ld<T>(tab_src[c]), v1 = lds_ld<T>(tab_src[c + 1]);
                                                    const T v2 = lds_ld<T>(tab_src[c + 2]), v3 = lds_ld<T>(tab_src[c + 3]);
                                                    sum = sum + v0;
                                                    sum = sum + v1;
                                                    sum = sum + v2;
                                                    sum = sum + v3;
                                                }
                                                for (; c < l; ++c)
                                                    sum = sum + lds_ld<T>(tab_src[c]);
                                                lds_st<T>(sn.split_dst + (uint32_t)(q * sizeof(T)), sum);
                                            }
                                            zone_sync<W>();
                                        }

                                        auto trial_r = [&](double hp) {
                                            T rl = (T)0.0;
                                            bool nonfinite = false;
                                            const T hT = (T)hp, kappaT = (T)o.kappa, floorT = (T)o.y_floor;
#pragma unroll
                                            for (int m = 0; m < SPL; ++m) {
                                                const int i = cell_at(m);
                                                if (i < N) {
                                                    const uint32_t sp = tab_species[zl * SPL + m];
                                                    const T fp = lds_ld<T>(sp & 0xffffu), kd = lds_ld<T>(sp >> 16);
                                                    const T y = Y[i];
                                                    const T kh = kd * hT;
                                                    const T v = kh < kappaT ? y + hT * (fp - kd * y)
                                                                            : (y + hT * fp) / ((T)1.0 + kh);
                                                    if (!isfinite(v))
                                                        nonfinite = true;
                                                    else
                                                        rl = fmax(rl, fabs(v - y) / fmax(y, floorT));
                                                }
                                            }
                                            if (nonfinite)
                                                rl = (T)INFINITY;
                                            double r = (double)wave_max_nonneg_dpp(rl);
                                            if constexpr (W > 1) {
                                                zone_sync<W>();  // the previous trial's exchange has been read
                                                if (lane == 0)
                                                    xw_r[wave] = r;
                                                __syncthreads();
                                                r = xw_r[0];
#pragma unroll
                                                for (int w = 1; w < W; ++w)
                                                    r = fmax(r, xw_r[w]);
                                            }
                                            return r;
                                        };
                                        int lo = -97, hi = 97;
                                        while (hi - lo > 1) {
                                            const int mid = lo + (hi - lo) / 2;
                                            const int qa = (mid >= 0) ? mid / 32 : -((31 - mid) / 32);  // floor(mid / 32)
                                            const int qb = mid - 32 * qa;
                                            if (trial_r(ldexp(hb * la.pow2[qb], qa)) <= o.tol)
                                                lo = mid;
                                            else
                                                hi = mid;
                                        }
                                        zone_sync<W>();
                                        return lo == -97 ? NAN : (float)(log2(o.safety) + lo / 32.0);
                                    };
                                    const float lab = boundary_label(h);
                                    if (zl == 0)
                                        la.trace[(int64_t)slot * kTraceRec + 166] = lab;
                                }
                            }
                        }
                        zone_sync<W>();
                    }
                }
            } else {
                ++nrej;
                if (mlp_attempt) {
                    // the network's proposal failed: continue with the plain rule
                    mlp_attempt = false;
                    step = plain_step;
                } else {
                    const double s = isinf(r) ? o.shrink_min : fmax(o.shrink_min, o.safety * o.tol / r);
                    step = h * s;
                }
                if (step < o.dt_min) {
                    status = kZoneDtUnderflow;
                    break;
                }
            }
            zone_sync<W>();
        }
        zone_sync<W>();
        double *Yo = za.Y + (size_t)z * N;
#pragma unroll
        for (int m = 0; m < SPL; ++m) {
            const int i = cell_at(m);
            if (i < N)
                Yo[sn.cell_species[i]] = (double)Y[i];
        }
        if (zl == 0) {
            za.dt[z] = step;
            za.n_acc[z] = nacc;
            za.n_rej[z] = nrej;
            za.status[z] = status;
        }
        // convergent point between the lane-0 stores and the next zone fetch
        zone_sync<W>();
    }
}

}  // namespace asynet
