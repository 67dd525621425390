/*
 * asynet: batched explicit asymptotic integration of stiff kinetic networks
 * on AMD Instinct MI355X (gfx950).
 *
 * The method is the algebraically stabilized explicit integrator of Brock,
 * Belt, Billings and Guidry, "Explicit Integration with GPU Acceleration for
 * Large Kinetic Networks" (arXiv:1409.5826):
 *
 *   dY_i/dt = F+_i - F-_i = F+_i - k_i Y_i                      Eq. (eq1.1)
 *
 * advanced per species either by forward Euler (k_i dt < kappa) or by the
 * asymptotic form (section "Algebraic Stabilization of Solutions Using
 * Asymptotic Approximations", Eq. (asySophia)):
 *
 *   Y_i <- (Y_i + dt F+_i) / (1 + k_i dt)                        (k_i dt >= kappa)
 *
 * with kappa = 1 and an adaptive network timestep.  Many independent networks
 * ("zones", one per hydrodynamic zone) share one reaction structure and are
 * integrated together (section "Multiple Parallel Networks and Thread
 * Occupancy").  Rates are constant over one integration because temperature
 * and density are frozen over a hydro step (section "GPU Virtues and the
 * Explicit Approach", footnote on rates).
 *
 * Conventions for every entry point:
 *  - Arguments documented "host" are host pointers, read during the call and
 *    owned by the caller.  Arguments documented "device" are device pointers
 *    on the current HIP device, owned by the caller, which must keep them
 *    valid until the work queued on the given stream has finished.
 *  - A negative asy_status reports an API or device error; asy_last_error()
 *    then returns a message (thread-local).  On an argument error nothing is
 *    modified and nothing is queued.
 *  - Per-zone numerical outcomes are written to zone_status; the call still
 *    returns ASY_OK.
 *  - A network handle owns device memory and a work queue.  Calls on one
 *    handle must be ordered on one stream; use one handle per concurrent
 *    stream.  Handles are not thread-safe.
 */
#ifndef ASYNET_H
#define ASYNET_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct asy_network asy_network; /* opaque; owned by the library */

typedef enum {
    ASY_OK = 0,
    ASY_EINVAL = -1,  /* invalid argument or descriptor */
    ASY_ENOMEM = -2,  /* device or host allocation failed */
    ASY_EDEVICE = -3, /* HIP runtime error, or no usable gfx950 device */
    ASY_ENOTSUP = -4, /* valid request the library does not support */
    ASY_ESTATE = -5   /* call out of order (e.g. learned controller before asy_set_mlp) */
} asy_status;

/* Per-zone outcome. */
enum {
    ASY_ZONE_OK = 0,           /* reached t_end */
    ASY_ZONE_MAX_STEPS = 1,    /* attempted-step budget exhausted before t_end */
    ASY_ZONE_DT_UNDERFLOW = 2, /* a rejection asked for a step below dt_min */
    ASY_ZONE_NONFINITE = 3,    /* an input of the zone (Y, rate, T, t_end, dt) is not finite */
    ASY_ZONE_BAD_INPUT = 4     /* negative Y or rate, T <= 0, t_end < 0 or dt <= 0 */
};

/* Rate forms. */
enum {
    ASY_RATES_PER_ZONE = 0, /* constant k[z][j] supplied per zone and reaction */
    ASY_RATES_ARRHENIUS = 1 /* k_j = A_j exp(-E_j / T_z), evaluated once per call */
};

/* Step-size controllers. */
enum {
    ASY_CTRL_PLAIN = 0,  /* dY/Y-limited rule below */
    ASY_CTRL_LEARNED = 1 /* MLP proposal with fallback to the plain rule */
};

/*
 * Reaction structure (section "Implementation of Realistic Kinetic Networks").
 * Reaction j destroys reactant0[j] (and reactant1[j] for a two-body
 * reaction; -1 marks a one-body reaction) and creates product[j], with flux
 * f_j = k_j Y_a (Y_b).  All arrays are host arrays of length n_reactions
 * (weight: n_species), copied during asy_network_create.
 */
typedef struct {
    int32_t n_species;        /* N >= 1 */
    int32_t n_reactions;      /* R >= 1 */
    const int32_t *reactant0; /* [R] species index in [0, N) */
    const int32_t *reactant1; /* [R] species index in [0, N), distinct from reactant0, or -1 */
    const int32_t *product;   /* [R] species index, distinct from the reactants */
    const int32_t *weight;    /* [N] conserved integer weights (mass numbers, Eq. 5.35); NULL skips the check */
    int32_t rate_form;        /* ASY_RATES_PER_ZONE or ASY_RATES_ARRHENIUS */
    const double *A;          /* [R] Arrhenius prefactors (> 0, finite); NULL for per-zone rates */
    const double *E;          /* [R] activation energies in units of T (finite); NULL for per-zone rates */
    int32_t split_above;      /* rows (creation or depletion sums of one species) with more terms are
                                 summed in chunks of split_above / 2 terms (rounded down to a multiple
                                 of 4) on separate lanes, the chunk sums added in order: 0 = 64.
                                 Splitting changes the order of the additions of such rows (results
                                 differ by rounding, independent of the launch) */
} asy_network_desc;

/*
 * Integration options.  The paper fixes kappa = 1 and leaves the timestep
 * controller unspecified; the controller of this library is, per zone:
 *   r = max_i |Yn_i - Y_i| / max(Y_i, y_floor)   (+inf if any Yn_i is not finite)
 *   accept iff r <= tol;
 *   after an accepted, unclipped step h: dt = h * min(grow_max, safety*tol/r);
 *   after a rejection:                   dt = h * max(shrink_min, safety*tol/r),
 *                                        and dt < dt_min ends the zone;
 *   the last step is clipped to land on t_end and leaves dt unchanged.
 */
typedef struct {
    double kappa;      /* stiffness switch; 1.0 */
    double tol;        /* relative-change bound; 0.01 */
    double y_floor;    /* abundance floor of the change measure; 1e-10 (>= FLT_MIN, the
                          smallest normal float, with ASY_PREC_F32; else ASY_EINVAL) */
    double grow_max;   /* 2.0 */
    double safety;     /* 0.9 */
    double shrink_min; /* 0.1 */
    double dt_min;     /* 1e-20 */
    int64_t max_steps; /* attempted steps per zone; 10,000,000 */
    int32_t controller;/* ASY_CTRL_PLAIN */
    int32_t precision; /* ASY_PREC_F64 */
} asy_options;

/*
 * Arithmetic of the integration (the paper compares single- and double-
 * precision integration, section "Performance for a Single Network").
 * ASY_PREC_F32: abundances, rates, fluxes, sums, the update and the change
 * measure in float, rounded from the double inputs once per zone and widened
 * back on output; time, the step size and its rule stay double.  Launch
 * variant 1 and the plain controller only (ASY_ENOTSUP otherwise, also for
 * asy_integrate_batch_trace).
 */
enum { ASY_PREC_F64 = 0, ASY_PREC_F32 = 1 };

/* Launch configuration of the integrator kernel (see asy_autotune). */
typedef struct {
    int32_t variant;          /* kernel variant: 0 = one zone per workgroup */
    int32_t threads_per_zone; /* threads cooperating on one zone (multiple of 64) */
    int32_t zones_per_group;  /* zones resident in one workgroup */
    int32_t groups_per_cu;    /* persistent workgroups launched per compute unit; 0 = one per zone */
    int32_t use_graph;        /* 1: replay a captured hipGraph for repeated identical calls */
    int32_t zone_order;       /* 0: zones start in index order; 1: longest first, by the sum of
                                 their rate constants (variant 1 only).  Scheduling only: the
                                 results do not depend on it */
} asy_launch;

/* Fill *o with the defaults listed above.  o: host, non-NULL. */
void asy_options_default(asy_options *o);

/*
 * Validate a reaction structure and upload it to the current HIP device (the
 * paper's one-time setup copy of rate-library parameters, section
 * "Implementing the Explicit Asymptotic Algorithm on a CPU-GPU System").
 * Rejects with ASY_EINVAL: sizes < 1, an index out of range, reactant0 ==
 * reactant1, a product equal to a reactant, a reaction that breaks
 * weight conservation (when weight != NULL), a missing or extra Arrhenius
 * array, a non-finite or non-positive A, a non-finite E.  Validation runs
 * on the host before any device call.  *out receives the handle on success
 * and is left untouched otherwise.  ASY_EDEVICE: no gfx950 device, or a
 * device call failed.  Creation also lays out variant 1 for 1, 2 and 4
 * waves per zone (row packing and a bank-aware placement of the gathers,
 * a seeded search of about 0.4 s of host time per layout at 150 species);
 * the plain controller's results do not depend on the layout, only its
 * speed does (the learned controller's features sum over species in lane
 * order, so its proposals may differ in the last bits between layouts).
 */
asy_status asy_network_create(const asy_network_desc *desc, asy_network **out);

/* Release a handle and its device memory after synchronizing the device.  NULL is a no-op. */
void asy_network_destroy(asy_network *net);

/*
 * Integrate n_zones independent zones from t = 0 to t_end[z] with constant
 * rates (one hydro step of the operator-split scheme, section
 * "Operator-Split Integration Timesteps"; the per-zone inputs and outputs
 * are the paper's copy-in and copy-out lists of section "Implementing the
 * Explicit Asymptotic Algorithm on a CPU-GPU System").
 *
 *  Y           device [n_zones][N] FP64, row-major; in: Y(0), out: the last
 *              accepted state (unchanged for a zone that fails its input checks)
 *  T           device [n_zones] FP64 temperatures for ASY_RATES_ARRHENIUS, else NULL
 *  k_zone      device [n_zones][R] FP64 rates for ASY_RATES_PER_ZONE, else NULL
 *  t_end       device [n_zones] FP64 interval lengths (>= 0)
 *  dt          device [n_zones] FP64; in: trial step (> 0), out: next trial step
 *  n_accepted  device [n_zones] int64, out
 *  n_rejected  device [n_zones] int64, out
 *  zone_status device [n_zones] int32, out (ASY_ZONE_*)
 *  opts        host; NULL means defaults
 *  stream      hipStream_t to queue the work on (NULL = the null stream);
 *              the call returns after queuing; outputs are valid once the
 *              stream has been synchronized
 *
 * n_zones == 0 queues nothing and returns ASY_OK.  The arithmetic is FP64
 * without fused multiply-add contraction, and every creation/depletion sum
 * takes its terms in ascending reaction index, so results do not depend on
 * the launch configuration.
 */
asy_status asy_integrate_batch(asy_network *net, const asy_options *opts, int32_t n_zones,
                               double *Y, const double *T, const double *k_zone,
                               const double *t_end, double *dt, int64_t *n_accepted,
                               int64_t *n_rejected, int32_t *zone_status, void *stream);

/*
 * asy_integrate_batch_noalloc: asy_integrate_batch for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments, results and errors as
 * asy_integrate_batch, bit for bit, except:
 *  - n_zones must not exceed 262144, nor, for an Arrhenius network, 65011456 /
 *    (8 n_reactions) (5066 zones at 1604 reactions); ASY_EINVAL otherwise,
 *    nothing queued;
 *  - the call allocates nothing: its scratch (the zone counter; with zone_order
 *    1 the scheduling keys and order; for Arrhenius networks the table of the
 *    call's rates) is a 64 MiB static device array that every device the
 *    library runs on holds until the process ends; the counter is cleared by a
 *    kernel at the start of each call, keys, order and rates are rewritten for
 *    every zone of the call;
 *  - the launch configuration's graph replay is not used.
 * All calls on one device share that device's array: calls that overlap in
 * time on one device (several streams or threads, any handles) race and
 * give wrong results.  Order them on one stream.
 */
asy_status asy_integrate_batch_noalloc(asy_network *net, const asy_options *opts, int32_t n_zones,
                                       double *Y, const double *T, const double *k_zone,
                                       const double *t_end, double *dt, int64_t *n_accepted,
                                       int64_t *n_rejected, int32_t *zone_status, void *stream);

/* Current launch configuration of a handle.  cfg: host, out. */
asy_status asy_get_launch(const asy_network *net, asy_launch *cfg);

/* Layout of variant 1 for one choice of threads per zone (host information). */
typedef struct {
    int32_t available;          /* 1 if variant 1 can run with this many threads per zone */
    int32_t slots;              /* compiled slots per lane (C) */
    int32_t slots_used;         /* slots per lane the packing needs */
    int32_t species_per_lane;   /* Y cells per lane in the update */
    int32_t split_rows;         /* rows summed in chunks (split_above) */
    uint32_t one_factor_waves;  /* bit w: every term of wave w has 1.0 as second factor, so the
                                   wave skips the second gathers and the products by 1.0 */
    int64_t gather_cycles_packed;  /* modelled LDS cycles of one zone-step's gathers (the gfx950
                                      bank rules) in packing order ... */
    int64_t gather_cycles_placed;  /* ... and after the bank-aware placement */
    int32_t one_factor_slots;      /* leading slots in which every lane's terms have 1.0 as second
                                      factor (whole blocks of 4) */
    int32_t one_factor_slots_run;  /* of those, the slots the double-precision plain kernel runs
                                      without the second gather on every wave */
    int32_t two_factor_wave_slots; /* slots the waves with two-factor terms run (= slots unless
                                      the layout is balanced: those waves stop earlier and the
                                      one-factor waves carry more slots) */
} asy_layout_info;

/*
 * The variant-1 layout the plain double-precision kernel runs for
 * threads_per_zone (64, 128 or 256; ASY_EINVAL otherwise): the balanced layout
 * where one was built, else the default one.  Host only, no device call.
 * info: host, out; available = 0 (and the rest zero) when no compiled instance
 * holds it.
 */
asy_status asy_network_layout_info(const asy_network *net, int32_t threads_per_zone,
                                   asy_layout_info *info);

/*
 * Set the launch configuration (validated against the device limits and the
 * network's LDS footprint; ASY_EINVAL if it cannot run).  The results of
 * asy_integrate_batch do not depend on it, only the speed does.
 */
asy_status asy_set_launch(asy_network *net, const asy_launch *cfg);

/*
 * Time candidate launch configurations on copies of the first sample_zones
 * zones of the given batch (same arguments as asy_integrate_batch, left
 * unmodified; every array must hold at least sample_zones zones, which the
 * library cannot check) and keep the fastest: first variant 1 with 1, 2 and 4
 * waves per zone and both zone orders, and variant 0 with 128 and 256 threads
 * (double precision only), one workgroup per zone without graph; then, for the
 * fastest of those, persistent grids of 1, 2, 3, 4, 6 and 8 workgroups per
 * compute unit and graph replay, each grid with and without.  Candidates run in
 * opts->precision with the plain controller, each timed on its second run.
 * Synchronous.  best: host, out, may be NULL.
 */
asy_status asy_autotune(asy_network *net, const asy_options *opts, int32_t sample_zones,
                        const double *Y, const double *T, const double *k_zone,
                        const double *t_end, const double *dt, asy_launch *best);

/*
 * ---- Learned step proposer ---------------------------------------------------------------
 * A 166 -> 128 -> 128 -> 1 ReLU perceptron that maps features of a zone's
 * accepted state to o, the predicted log2 of the ratio of the next accepted
 * step to the last one (no counterpart in the paper: it only replaces how the
 * next trial step of the adaptive network timestep is proposed).  Weights are
 * FP32 masters; every product runs on the matrix cores with BF16 operands and
 * FP32 accumulation.  Parameters travel as one FP32 vector of
 * ASY_MLP_N_PARAMS values: W1 [192][128] (input-major; rows 166..191 multiply
 * zero padding), b1 [128], W2 [128][128], b2 [128], W3 [128], b3 [1].
 * Features of a state (ASY_MLP_N_IN values): x[i] = max(log10 Y_i, -30)/30
 * for i < n_species (Y_i <= 0 gives -1), then log10 of the largest and of the
 * mean of k_i*h, log10 h, log10 tol (each /10, arguments floored at 1e-300),
 * zero up to ASY_MLP_N_IN; k_i are the depletion rates of the last accepted
 * step h.  Requires n_species <= ASY_MLP_N_IN - 4.
 */
#define ASY_MLP_N_IN 166
#define ASY_MLP_N_PARAMS 41345

typedef struct asy_mlp asy_mlp; /* opaque training context; owned by the library */

/* Create a context for batches of up to batch_max samples; parameters start at zero. */
asy_status asy_mlp_create(int32_t batch_max, asy_mlp **out);
void       asy_mlp_destroy(asy_mlp *m); /* NULL is a no-op */

/* Copy parameters in (host [ASY_MLP_N_PARAMS]; resets the Adam state) or out. */
asy_status asy_mlp_set_params(asy_mlp *m, const float *params);
asy_status asy_mlp_get_params(const asy_mlp *m, float *params);

/* o[b] for x [n][ASY_MLP_N_IN] (device FP32); o device [n]; n <= batch_max. */
asy_status asy_mlp_forward(asy_mlp *m, int32_t n, const float *x, float *o, void *stream);

/* Loss (device [1]) and gradient (device [ASY_MLP_N_PARAMS]) of mean (o - y)^2. */
asy_status asy_mlp_gradient(asy_mlp *m, int32_t n, const float *x, const float *y, float *loss,
                            float *grad, void *stream);

/*
 * One Adam step (beta 0.9 / 0.999, eps 1e-8, learning rate lr) on the batch
 * (x, y); loss (device [1], may be NULL) receives the batch loss before the update.
 */
asy_status asy_mlp_train_step(asy_mlp *m, int32_t n, const float *x, const float *y, float lr,
                              float *loss, void *stream);

/*
 * n_batches Adam steps in a row, step b on the samples [b batch, (b + 1) batch) of
 * x (device [n_batches batch][ASY_MLP_N_IN]) and y (device [n_batches batch]); the
 * same results as n_batches calls of asy_mlp_train_step, without the host's
 * round trip per step.  losses (device [n_batches], may be NULL) receives each
 * step's batch loss before its update.  1 <= batch <= batch_max, n_batches >= 0.
 */
asy_status asy_mlp_train_epoch(asy_mlp *m, int32_t n_batches, int32_t batch, const float *x,
                               const float *y, float lr, float *losses, void *stream);

/*
 * Batched inference through the same routine the integrator runs per zone
 * (one wave per sample, weights arranged for the matrix cores); o device [n].
 */
asy_status asy_mlp_infer(asy_mlp *m, int32_t n, const float *x, float *o, void *stream);

/* Give a network the current parameters of m for ASY_CTRL_LEARNED (a copy is kept). */
asy_status asy_set_mlp(asy_network *net, const asy_mlp *m);

/*
 * With opts->controller == ASY_CTRL_LEARNED, asy_integrate_batch proposes the
 * step after every accepted, unclipped step h as h * 2^(q/32), where
 * q = rint(32 clamp(o, -3, 3)) and o is the network's output for the accepted
 * state; if that attempt is rejected the zone falls back to the plain
 * proposal, and after any further rejection to the plain shrink rule, until a
 * step is accepted.  Requires asy_set_mlp (else ASY_ESTATE) and launch variant 1
 * with a learned kernel instance (else ASY_ENOTSUP).
 *
 * asy_integrate_batch_trace: asy_integrate_batch that also writes training
 * records, one per sampled accepted state of zones z < trace_zones (every
 * stride-th accepted step), ASY_TRACE_REC floats each, into trace (device
 * [capacity][ASY_TRACE_REC]): [0, 166) the state's features, [166] the
 * training label log2(safety * h_b / h), where h_b is the largest step of the
 * grid h 2^(q/32), q = -96..96, from which the controller would accept the
 * attempt, found by bisection on q assuming acceptance is monotone in the step
 * (the state's sums once, then one trial update per bisection step; nothing
 * of the zone changes; NaN when no step of the grid is accepted), [167] 32 q
 * of the learned proposal (NaN with the plain controller), [168] zone index,
 * [169] accepted-step index.
 * count (device, in/out) counts records taken; those beyond capacity are
 * dropped.  capacity < 2^31.  Record order is not deterministic.
 */
#define ASY_TRACE_REC 170
asy_status asy_integrate_batch_trace(asy_network *net, const asy_options *opts, int32_t n_zones,
                                     double *Y, const double *T, const double *k_zone,
                                     const double *t_end, double *dt, int64_t *n_accepted,
                                     int64_t *n_rejected, int32_t *zone_status, float *trace,
                                     int64_t capacity, unsigned long long *count, int32_t stride,
                                     int32_t trace_zones, void *stream);

/*
 * asy_probe_lds_bandwidth: measures the LDS read bandwidth of the current
 * device, summed over all compute units, in bytes per second.  Every lane
 * reads width_bytes (8 or 16) per LDS instruction at conflict-free addresses.
 * The integrator keeps each zone's state in LDS for the whole integration
 * (section "Implementing the Explicit Asymptotic Algorithm on a CPU-GPU
 * System"), so this is the bandwidth its roofline is priced against.
 * Synchronous (runs on the null stream); allocates and frees a small sink
 * buffer.  ASY_EINVAL for another width or a NULL output.
 */
asy_status asy_probe_lds_bandwidth(int32_t width_bytes, double *bytes_per_second);

/*
 * asy_integrate_schedule: n_steps consecutive hydro steps of the operator-split
 * scheme (section "Operator-Split Integration Timesteps"), queued on stream
 * without host synchronisation.  In step s every zone z is integrated over
 * dt_hydro[s][z] (device [n_steps][n_zones]) with the temperature T[s][z]
 * (device [n_steps][n_zones], Arrhenius networks) or its constant rates k_zone
 * (device [n_zones][n_reactions]), starting from the abundances and the trial
 * step the previous step left in Y and dt (in/out, as asy_integrate_batch).
 * The copy-out of the section "Implementing the Explicit Asymptotic Algorithm
 * on a CPU-GPU System" lists the energy released by the integration; with q
 * (device [n_species], energy per unit abundance of each species) it is
 *   energy[s][z] = sum_i q_i (Y_i after step s - Y_i before step s),
 * summed in ascending species index (energy: device [n_steps][n_zones], or
 * NULL; q may then be NULL).  n_accepted / n_rejected (device [n_zones], out)
 * sum over the steps; zone_status holds each zone's first non-OK status, else
 * ASY_ZONE_OK.  Later steps still integrate a zone after a failed step, from
 * what that step left.  Options and launch as asy_integrate_batch (no trace);
 * the launch configuration's graph replay is not used.  ASY_EINVAL for
 * n_steps < 1, energy without q, or missing arrays.
 */
asy_status asy_integrate_schedule(asy_network *net, const asy_options *opts, int32_t n_zones,
                                  int32_t n_steps, double *Y, const double *T, const double *k_zone,
                                  const double *dt_hydro, double *dt, const double *q,
                                  double *energy, int64_t *n_accepted, int64_t *n_rejected,
                                  int32_t *zone_status, void *stream);

/* Message of the last failed call on this thread ("" if none). */
const char *asy_last_error(void);

/* Library version string. */
const char *asy_version(void);

#ifdef __cplusplus
}
#endif

#endif /* ASYNET_H */
