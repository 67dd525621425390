// Host side of the asynet C ABI: descriptor validation, species-major
// incidence build, device upload, launch configuration, graph replay and
// autotuning.  See include/asynet.h for the contract of every entry point.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "asynet.h"
#include "integrate_kernels.h"

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

}  // namespace

struct asy_network {
    int32_t n_species = 0;
    int32_t n_reactions = 0;
    int32_t n_destruction = 0;
    int32_t rate_form = ASY_RATES_PER_ZONE;
    int device = 0;
    int n_cu = 0;
    size_t lds_per_group_max = 0;
    // device arrays (one allocation, carved)
    void *dev_block = nullptr;
    int32_t *queue = nullptr;
    DevNetwork dn{};
    asy_launch launch{};
    // host copies of the structure (for validation of launches and autotuning)
    std::vector<int32_t> prod_ptr, dest_ptr;
    // graph replay cache
    hipStream_t capture_stream = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    std::vector<uint8_t> graph_key;
};

namespace {

size_t lds_bytes_variant0(const asy_network *net)
{
    return sizeof(double) * ((size_t)net->n_reactions + 2 * (size_t)net->n_species);
}

asy_status validate_launch(const asy_network *net, const asy_launch *c)
{
    if (c->reserved != 0)
        return fail(ASY_EINVAL, "asy_launch.reserved must be 0");
    if (c->variant != 0)
        return fail(ASY_EINVAL, "asy_launch.variant must be 0");
    if (c->threads_per_zone != 64 && c->threads_per_zone != 128 && c->threads_per_zone != 256 &&
        c->threads_per_zone != 512)
        return fail(ASY_EINVAL, "asy_launch.threads_per_zone must be 64, 128, 256 or 512");
    if (c->zones_per_group != 1)
        return fail(ASY_EINVAL, "asy_launch.zones_per_group must be 1 for variant 0");
    if (c->groups_per_cu < 0 || c->groups_per_cu > 32)
        return fail(ASY_EINVAL, "asy_launch.groups_per_cu must be in [0, 32]");
    if (c->use_graph != 0 && c->use_graph != 1)
        return fail(ASY_EINVAL, "asy_launch.use_graph must be 0 or 1");
    if (lds_bytes_variant0(net) > net->lds_per_group_max)
        return fail(ASY_ENOTSUP, "network too large for the LDS of one workgroup");
    return ASY_OK;
}

template <int NT, bool ARR>
hipError_t launch_variant0(asy_network *net, const DevOptions &o, const ZoneArgs &za, int grid,
                           hipStream_t s)
{
    hipLaunchKernelGGL((integrate_group_kernel<NT, ARR>), dim3(grid), dim3(NT),
                       lds_bytes_variant0(net), s, net->dn, o, za);
    return hipGetLastError();
}

hipError_t launch_all(asy_network *net, const asy_launch &c, const DevOptions &o,
                      const ZoneArgs &za, hipStream_t s)
{
    hipLaunchKernelGGL(reset_queue_kernel, dim3(1), dim3(64), 0, s, za.queue);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
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

const char *asy_version(void) { return "asynet 0.1 (gfx950)"; }

asy_status asy_network_create(const asy_network_desc *d, asy_network **out)
{
    g_last_error.clear();
    if (!d || !out)
        return fail(ASY_EINVAL, "desc and out must be non-NULL");
    const int32_t N = d->n_species, R = d->n_reactions;
    if (N < 1 || R < 1)
        return fail(ASY_EINVAL, "n_species and n_reactions must be >= 1");
    if (N > 32767 || R > (1 << 24))
        return fail(ASY_EINVAL, "network too large (n_species <= 32767, n_reactions <= 2^24)");
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

    // species-major incidence, ascending reaction index within each row
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
        for (int32_t j = 0; j < R; ++j) {  // ascending j keeps each row sorted
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

    // device: check for a gfx950 device before allocating
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
    net->prod_ptr = prod_ptr;
    net->dest_ptr = dest_ptr;

    // one device allocation, 256-byte aligned pieces
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
    auto put = [&](size_t o, const void *src, size_t bytes) {
        return hipMemcpy(base + o, src, bytes, hipMemcpyHostToDevice);
    };
    hipError_t ce = hipSuccess;
    auto chk = [&](hipError_t e) {
        if (ce == hipSuccess)
            ce = e;
    };
    chk(hipMemset(base + o_queue, 0, 256));
    chk(put(o_pp, prod_ptr.data(), sizeof(int32_t) * (N + 1)));
    chk(put(o_prx, prod_rx.data(), sizeof(int32_t) * R));
    chk(put(o_pa, prod_a.data(), sizeof(int32_t) * R));
    chk(put(o_pb, prod_b.data(), sizeof(int32_t) * R));
    chk(put(o_dp, dest_ptr.data(), sizeof(int32_t) * (N + 1)));
    chk(put(o_drx, dest_rx.data(), sizeof(int32_t) * D));
    chk(put(o_do, dest_o.data(), sizeof(int32_t) * D));
    if (arr) {
        chk(put(o_A, d->A, sizeof(double) * R));
        chk(put(o_E, d->E, sizeof(double) * R));
    }
    if (ce != hipSuccess) {
        (void)hipFree(net->dev_block);
        delete net;
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

    net->launch.variant = 0;
    net->launch.threads_per_zone = N <= 64 ? 64 : (N <= 128 ? 128 : 256);
    net->launch.zones_per_group = 1;
    net->launch.groups_per_cu = 0;
    net->launch.use_graph = 0;
    net->launch.reserved = 0;
    if (validate_launch(net, &net->launch) != ASY_OK) {
        (void)hipFree(net->dev_block);
        delete net;
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
    if (net->graph_exec)
        (void)hipGraphExecDestroy(net->graph_exec);
    if (net->capture_stream)
        (void)hipStreamDestroy(net->capture_stream);
    if (net->dev_block)
        (void)hipFree(net->dev_block);
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
    DevOptions dop{o.kappa, o.tol, o.y_floor, o.grow_max, o.safety, o.shrink_min, o.dt_min,
                   o.max_steps};
    ZoneArgs za{n_zones, Y, T, k_zone, t_end, dt, n_accepted, n_rejected, zone_status, net->queue};
    hipStream_t s = static_cast<hipStream_t>(stream);
    HIP_TRY(hipSetDevice(net->device));
    HIP_TRY(launch_all(net, net->launch, dop, za, s));
    return ASY_OK;
}

asy_status asy_autotune(asy_network *net, const asy_options *opts, int32_t sample_zones,
                        const double *Y, const double *T, const double *k_zone,
                        const double *t_end, const double *dt, asy_launch *best)
{
    (void)opts; (void)sample_zones; (void)Y; (void)T; (void)k_zone; (void)t_end; (void)dt;
    if (!net)
        return fail(ASY_EINVAL, "net must be non-NULL");
    if (best)
        *best = net->launch;
    return fail(ASY_ENOTSUP, "autotuning not available in this build");
}

}  // extern "C"
