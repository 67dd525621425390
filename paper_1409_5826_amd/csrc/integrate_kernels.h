// Device code of the batched explicit asymptotic integrator (gfx950).
//
// One zone is one independent network instance (its own abundances, rates,
// interval and step).  A workgroup integrates one zone at a time, keeping the
// zone's rates and abundances in LDS for the whole interval, and pulls the
// next zone from a device-wide counter when it is done, so zones with uneven
// step counts balance across the chip (the paper launches one block per
// network and leaves load balance open, section "Multiple Parallel Networks
// and Thread Occupancy").
//
// Arithmetic is FP64 and the file is compiled with -ffp-contract=off: every
// product and sum rounds as written, and each creation/depletion sum takes its
// terms in ascending reaction index, so a zone's result does not depend on
// the launch configuration.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace asynet {

constexpr int kWave = 64;

enum ZoneStatus : int32_t {
    kZoneOk = 0,
    kZoneMaxSteps = 1,
    kZoneDtUnderflow = 2,
    kZoneNonfinite = 3,
    kZoneBadInput = 4,
};

// Species-major incidence of a network, built on the host.
//  production row of species i:  entries [prod_ptr[i], prod_ptr[i+1]), ascending reaction
//    index, each entry = (reaction j, reactant0[j], reactant1[j] or -1)
//  destruction row of species i: entries [dest_ptr[i], dest_ptr[i+1]), ascending reaction
//    index, each entry = (reaction j, the other reactant of j or -1)
struct DevNetwork {
    int32_t n_species;
    int32_t n_reactions;
    const int32_t *prod_ptr;
    const int32_t *prod_rx;
    const int32_t *prod_a;
    const int32_t *prod_b;
    const int32_t *dest_ptr;
    const int32_t *dest_rx;
    const int32_t *dest_o;
    const double *A;  // Arrhenius prefactors or nullptr
    const double *E;  // Arrhenius activation energies or nullptr
};

struct DevOptions {
    double kappa, tol, y_floor, grow_max, safety, shrink_min, dt_min;
    int64_t max_steps;
};

struct ZoneArgs {
    int32_t n_zones;
    double *Y;
    const double *T;
    const double *k_zone;
    const double *t_end;
    double *dt;
    int64_t *n_acc;
    int64_t *n_rej;
    int32_t *status;
    int32_t *queue;  // zone counter, zero at launch
};

// exp(x) of the Arrhenius factor k = A exp(-E/T), by a fixed algorithm (not the
// device library's exp, whose last bit can differ from other implementations; over
// thousands of steps such a difference can move an accept/reject decision):
// Cody and Waite's reduction x = n ln2 + r, n = rint(x / ln2), with ln2 split into a
// 33-bit head (n * head is exact for |n| < 2^20) and a tail; the Taylor polynomial of
// exp(r) to degree 13 in Horner form, coefficients 1/k! (each a correctly rounded
// division); then 2^n exactly.  Compiled without fused multiply-add.
__host__ __device__ inline double rate_exp(double x)
{
    constexpr double kLn2Hi = 0x1.62e42fefp-1, kLn2Lo = 0x1.473de6af278edp-34;
    constexpr double kInvLn2 = 0x1.71547652b82fep+0;
    if (isnan(x))
        return x;
    if (x > 709.782712893384)
        return INFINITY;
    if (x < -745.2)
        return 0.0;
    const double n = rint(x * kInvLn2);
    const double r = (x - n * kLn2Hi) - n * kLn2Lo;
    constexpr double f2 = 2.0, f3 = 6.0, f4 = 24.0, f5 = 120.0, f6 = 720.0, f7 = 5040.0,
                     f8 = 40320.0, f9 = 362880.0, f10 = 3628800.0, f11 = 39916800.0,
                     f12 = 479001600.0, f13 = 6227020800.0;
    double p = 1.0 / f13;
    p = p * r + 1.0 / f12;
    p = p * r + 1.0 / f11;
    p = p * r + 1.0 / f10;
    p = p * r + 1.0 / f9;
    p = p * r + 1.0 / f8;
    p = p * r + 1.0 / f7;
    p = p * r + 1.0 / f6;
    p = p * r + 1.0 / f5;
    p = p * r + 1.0 / f4;
    p = p * r + 1.0 / f3;
    p = p * r + 1.0 / f2;
    p = p * r + 1.0;
    p = p * r + 1.0;
    return ldexp(p, (int)n);
}

__device__ inline double wave_max(double v)
{
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1)
        v = fmax(v, __shfl_xor(v, off, kWave));
    return v;
}

// Maximum over the 64 lanes of a wave through DPP lane moves (no LDS round
// trips): row_shr 1, 2, 4, 8 leave each row's maximum in its lane 15,
// row_bcast15 and row_bcast31 carry it across rows into lane 63, which is
// read back as a uniform value.  Lanes without a DPP source keep their own
// value, the identity of max.
#define ASY_DPP_MAX_STEP(v, ctrl, rmask)                                                       \
    do {                                                                                       \
        const int lo_ = __builtin_amdgcn_update_dpp(__double2loint(v), __double2loint(v),      \
                                                    ctrl, rmask, 0xf, false);                  \
        const int hi_ = __builtin_amdgcn_update_dpp(__double2hiint(v), __double2hiint(v),      \
                                                    ctrl, rmask, 0xf, false);                  \
        v = fmax(v, __hiloint2double(hi_, lo_));                                               \
    } while (0)

__device__ inline double wave_max_dpp(double v)
{
    ASY_DPP_MAX_STEP(v, 0x111, 0xf);  // row_shr:1
    ASY_DPP_MAX_STEP(v, 0x112, 0xf);  // row_shr:2
    ASY_DPP_MAX_STEP(v, 0x114, 0xf);  // row_shr:4
    ASY_DPP_MAX_STEP(v, 0x118, 0xf);  // row_shr:8
    ASY_DPP_MAX_STEP(v, 0x142, 0xa);  // row_bcast:15 into rows 1 and 3
    ASY_DPP_MAX_STEP(v, 0x143, 0xc);  // row_bcast:31 into rows 2 and 3
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), 63);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 63);
    return __hiloint2double(hi, lo);
}

// Maximum of non-negative values (the change measure, depletion rates): lanes
// without a DPP source read 0, harmless for the maximum, and every row takes
// part in the row broadcasts, so no lane keeps an old value and the moves need
// no copies.
#define ASY_DPP_MAX0_STEP(v, ctrl)                                                              \
    do {                                                                                       \
        const int lo_ = __builtin_amdgcn_mov_dpp(__double2loint(v), ctrl, 0xf, 0xf, true);     \
        const int hi_ = __builtin_amdgcn_mov_dpp(__double2hiint(v), ctrl, 0xf, 0xf, true);     \
        v = fmax(v, __hiloint2double(hi_, lo_));                                               \
    } while (0)

__device__ inline double wave_max_nonneg_dpp(double v)
{
    ASY_DPP_MAX0_STEP(v, 0x111);  // row_shr:1
    ASY_DPP_MAX0_STEP(v, 0x112);  // row_shr:2
    ASY_DPP_MAX0_STEP(v, 0x114);  // row_shr:4
    ASY_DPP_MAX0_STEP(v, 0x118);  // row_shr:8
    ASY_DPP_MAX0_STEP(v, 0x142);  // row_bcast:15
    ASY_DPP_MAX0_STEP(v, 0x143);  // row_bcast:31
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), 63);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 63);
    return __hiloint2double(hi, lo);
}

__device__ inline float wave_max_nonneg_dpp(float v)
{
#define ASY_DPP_MAX0_STEP_F32(ctrl)                                                             \
    v = fmaxf(v, __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), ctrl, 0xf, 0xf, true)))
    ASY_DPP_MAX0_STEP_F32(0x111);
    ASY_DPP_MAX0_STEP_F32(0x112);
    ASY_DPP_MAX0_STEP_F32(0x114);
    ASY_DPP_MAX0_STEP_F32(0x118);
    ASY_DPP_MAX0_STEP_F32(0x142);
    ASY_DPP_MAX0_STEP_F32(0x143);
#undef ASY_DPP_MAX0_STEP_F32
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}

// The same for float.
__device__ inline float wave_max_dpp(float v)
{
#define ASY_DPP_MAX_STEP_F32(ctrl, rmask)                                                       \
    v = fmaxf(v, __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(v), __float_as_int(v), \
                                                            ctrl, rmask, 0xf, false)))
    ASY_DPP_MAX_STEP_F32(0x111, 0xf);
    ASY_DPP_MAX_STEP_F32(0x112, 0xf);
    ASY_DPP_MAX_STEP_F32(0x114, 0xf);
    ASY_DPP_MAX_STEP_F32(0x118, 0xf);
    ASY_DPP_MAX_STEP_F32(0x142, 0xa);
    ASY_DPP_MAX_STEP_F32(0x143, 0xc);
#undef ASY_DPP_MAX_STEP_F32
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}

#define ASY_DPP_SUM_STEP(v, ctrl, rmask)                                                       \
    do {                                                                                       \
        const int lo_ = __builtin_amdgcn_update_dpp(0, __double2loint(v), ctrl, rmask, 0xf, false); \
        const int hi_ = __builtin_amdgcn_update_dpp(0, __double2hiint(v), ctrl, rmask, 0xf, false); \
        v = v + __hiloint2double(hi_, lo_);                                                    \
    } while (0)

// Sum over the 64 lanes of a wave through DPP lane moves (lanes without a
// source add +0.0).  The order of the additions is fixed.
__device__ inline double wave_sum_dpp(double v)
{
    ASY_DPP_SUM_STEP(v, 0x111, 0xf);
    ASY_DPP_SUM_STEP(v, 0x112, 0xf);
    ASY_DPP_SUM_STEP(v, 0x114, 0xf);
    ASY_DPP_SUM_STEP(v, 0x118, 0xf);
    ASY_DPP_SUM_STEP(v, 0x142, 0xa);
    ASY_DPP_SUM_STEP(v, 0x143, 0xc);
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), 63);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 63);
    return __hiloint2double(hi, lo);
}

__device__ inline int wave_or(int v)
{
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1)
        v |= __shfl_xor(v, off, kWave);
    return v;
}

__global__ void reset_queue_kernel(int32_t *queue)
{
    if (threadIdx.x == 0 && blockIdx.x == 0)
        queue[0] = 0;
}

// Variant 0: one zone per workgroup, species strided over the workgroup's
// threads.  Dynamic LDS: k[R], Y[N], Yn[N] (FP64).
template <int NTHREADS, bool ARRHENIUS>
__global__ void __launch_bounds__(NTHREADS)
integrate_group_kernel(DevNetwork net, DevOptions o, ZoneArgs za)
{
    constexpr int NWAVES = NTHREADS / kWave;
    extern __shared__ double lds[];
    __shared__ double wave_r[NWAVES];
    __shared__ int wave_flag[NWAVES];
    __shared__ int zone_slot;

    const int N = net.n_species;
    const int R = net.n_reactions;
    double *k = lds;
    double *Y = k + R;
    double *Yn = Y + N;
    const int tid = threadIdx.x;
    const int wave = tid / kWave;
    const int lane = tid % kWave;

    for (;;) {
        // Fetch the next zone.  Wave 0 takes a ticket with a wave-wide atomic
        // (lane 0 adds 1, the others 0) and broadcasts lane 0's ticket with a
        // cross-lane read, so every lane leaves this block with the same z and
        // no lane-divergent branch sits at the head of the loop.
        if (wave == 0) {
            int ticket = atomicAdd(za.queue, lane == 0 ? 1 : 0);
            ticket = __shfl(ticket, 0, kWave);
            if (lane == 0)
                zone_slot = ticket;
        }
        __syncthreads();
        const int z = __builtin_amdgcn_readfirstlane(zone_slot);
        __syncthreads();
        if (z >= za.n_zones)
            break;

        // ---- load the zone: rates (evaluated once per interval), abundances, checks
        const double t_end = za.t_end[z];
        const double dt0 = za.dt[z];
        int flag = 0;  // bit 0: non-finite input, bit 1: out-of-domain input
        if (ARRHENIUS) {
            const double T = za.T[z];
            if (!isfinite(T))
                flag |= 1;
            else if (!(T > 0.0))
                flag |= 2;
            for (int j = tid; j < R; j += NTHREADS) {
                double kj = net.A[j] * rate_exp(-net.E[j] / T);
                k[j] = kj;
                if (!isfinite(kj))
                    flag |= 1;
            }
        } else {
            const double *kz = za.k_zone + (size_t)z * R;
            for (int j = tid; j < R; j += NTHREADS) {
                double kj = kz[j];
                k[j] = kj;
                if (!isfinite(kj))
                    flag |= 1;
                else if (kj < 0.0)
                    flag |= 2;
            }
        }
        const double *Yz = za.Y + (size_t)z * N;
        for (int i = tid; i < N; i += NTHREADS) {
            double y = Yz[i];
            Y[i] = y;
            if (!isfinite(y))
                flag |= 1;
            else if (y < 0.0)
                flag |= 2;
        }
        if (!isfinite(t_end) || !isfinite(dt0))
            flag |= 1;
        else if (t_end < 0.0 || !(dt0 > 0.0))
            flag |= 2;
        flag = wave_or(flag);
        if (lane == 0)
            wave_flag[wave] = flag;
        __syncthreads();
        flag = 0;
#pragma unroll
        for (int w = 0; w < NWAVES; ++w)
            flag |= wave_flag[w];
        if (flag) {
            if (tid == 0) {
                za.status[z] = (flag & 1) ? kZoneNonfinite : kZoneBadInput;
                za.n_acc[z] = 0;
                za.n_rej[z] = 0;
            }
            __syncthreads();  // keeps the lane-0 block off the loop back edge
            continue;         // Y and dt stay as given
        }

        // ---- integrate over [0, t_end]
        double t = 0.0, step = dt0;
        int64_t nacc = 0, nrej = 0;
        int32_t status = kZoneOk;
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
            double rloc = 0.0;
            bool bad = false;
            for (int i = tid; i < N; i += NTHREADS) {
                // creation flux F+_i: fluxes of the reactions producing i
                double fp = 0.0;
                const int pe = net.prod_ptr[i + 1];
                for (int e = net.prod_ptr[i]; e < pe; ++e) {
                    const int b = net.prod_b[e];
                    double f = k[net.prod_rx[e]] * Y[net.prod_a[e]];
                    if (b >= 0)
                        f = f * Y[b];
                    fp = fp + f;
                }
                // depletion rate k_i: F-_i / Y_i summed from the reactions destroying i
                double kd = 0.0;
                const int de = net.dest_ptr[i + 1];
                for (int e = net.dest_ptr[i]; e < de; ++e) {
                    const int oth = net.dest_o[e];
                    const double kj = k[net.dest_rx[e]];
                    kd = kd + (oth >= 0 ? kj * Y[oth] : kj);
                }
                const double y = Y[i];
                const double kh = kd * h;
                double yn;
                if (kh < o.kappa)
                    yn = y + h * (fp - kd * y);    // forward Euler
                else
                    yn = (y + h * fp) / (1.0 + kh); // asymptotic form
                Yn[i] = yn;
                if (!isfinite(yn))
                    bad = true;
                else
                    rloc = fmax(rloc, fabs(yn - y) / fmax(y, o.y_floor));
            }
            if (bad)
                rloc = INFINITY;
            rloc = wave_max(rloc);
            if (lane == 0)
                wave_r[wave] = rloc;
            __syncthreads();
            double r = wave_r[0];
#pragma unroll
            for (int w = 1; w < NWAVES; ++w)
                r = fmax(r, wave_r[w]);
            if (r <= o.tol) {
                for (int i = tid; i < N; i += NTHREADS)
                    Y[i] = Yn[i];
                ++nacc;
                t = clipped ? t_end : t + h;
                if (!clipped) {
                    const double g = (r == 0.0) ? o.grow_max : fmin(o.grow_max, o.safety * o.tol / r);
                    step = h * g;
                }
            } else {
                ++nrej;
                const double s = isinf(r) ? o.shrink_min : fmax(o.shrink_min, o.safety * o.tol / r);
                step = h * s;
                if (step < o.dt_min) {
                    status = kZoneDtUnderflow;
                    break;
                }
            }
            __syncthreads();
        }
        __syncthreads();
        double *Yo = za.Y + (size_t)z * N;
        for (int i = tid; i < N; i += NTHREADS)
            Yo[i] = Y[i];
        if (tid == 0) {
            za.dt[z] = step;
            za.n_acc[z] = nacc;
            za.n_rej[z] = nrej;
            za.status[z] = status;
        }
        // A convergent point between the lane-0 stores above and the zone
        // fetch at the loop head: without it the compiler may thread the
        // lane-0 condition across the back edge and let the other lanes
        // re-read a stale zone index.
        __syncthreads();
    }
}

// One hydro step of a schedule, after the integration: add the step's counters to the
// totals (set them on the first step), keep the first non-OK status, and the energy
// released, sum_i q_i (Y_i - before_i) in ascending species order (one thread per zone).
__global__ void __launch_bounds__(256)
schedule_step_kernel(int32_t n_zones, int32_t n_species, int first, const int64_t *acc_s,
                     const int64_t *rej_s, const int32_t *st_s, int64_t *n_acc, int64_t *n_rej,
                     int32_t *status, const double *Y, const double *before, const double *q,
                     double *energy)
{
    for (int z = blockIdx.x * blockDim.x + threadIdx.x; z < n_zones; z += gridDim.x * blockDim.x) {
        n_acc[z] = (first ? 0 : n_acc[z]) + acc_s[z];
        n_rej[z] = (first ? 0 : n_rej[z]) + rej_s[z];
        status[z] = (first || status[z] == kZoneOk) ? st_s[z] : status[z];
        if (energy) {
            const double *y = Y + (size_t)z * n_species;
            const double *y0 = before + (size_t)z * n_species;
            double e = 0.0;
            for (int i = 0; i < n_species; ++i)
                e += q[i] * (y[i] - y0[i]);
            energy[z] = e;
        }
    }
}

}  // namespace asynet
