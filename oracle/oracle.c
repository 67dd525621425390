/*
 * CPU oracle for the explicit asymptotic integration of kinetic networks.
 *
 * TEST INFRASTRUCTURE ONLY.  The test suite, the smoke check and the CPU
 * baseline leg of the benchmark load this library; the product path never
 * does.  It shares no code, header or table with the HIP library: it takes
 * the network and the zones as plain arrays and computes everything itself.
 *
 * Plain and slow on purpose: every quantity follows its definition in the
 * paper (Brock, Belt, Billings, Guidry, "Explicit Integration with GPU
 * Acceleration for Large Kinetic Networks", arXiv:1409.5826), in FP64, with
 * no blocking and no reordering.  Build with -ffp-contract=off so that no
 * multiply-add is fused: every expression rounds exactly as written.
 *
 * Readings where the paper is silent (the timestep controller, the tie at
 * k*dt == kappa, the clipping at the end of the interval) are the ones listed
 * in the design notes of this repository; each is marked "reading" below.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* per-zone outcome codes */
enum { ORC_ZONE_OK = 0, ORC_ZONE_MAX_STEPS = 1, ORC_ZONE_DT_UNDERFLOW = 2,
       ORC_ZONE_NONFINITE = 3, ORC_ZONE_BAD_INPUT = 4 };

typedef struct {
    double kappa;      /* stiffness switch, kappa = 1 in the paper */
    double tol;        /* bound on max_i |dY_i| / max(Y_i, y_floor) */
    double y_floor;    /* abundance floor of the relative-change measure */
    double grow_max;   /* largest growth factor of dt after an accepted step */
    double safety;     /* safety factor on tol / r */
    double shrink_min; /* smallest shrink factor of dt after a rejected step */
    double dt_min;     /* a rejection that asks for a smaller dt ends the zone */
    int64_t max_steps; /* attempted-step budget per zone */
} orc_options;

/*
 * Rate constants of the Arrhenius form used by the synthetic workloads:
 * k_j = A_j * exp(-E_j / T).  The paper evaluates rates once per network
 * integration because temperature and density are frozen over a hydro step
 * (section "GPU Virtues and the Explicit Approach", its footnote on rates).
 */
void orc_rates_arrhenius(int32_t n_reactions, const double *A, const double *E,
                         double T, double *k)
{
    for (int32_t j = 0; j < n_reactions; ++j)
        k[j] = A[j] * exp(-E[j] / T);
}

/*
 * Creation flux F+_i and effective depletion rate k_i of Eq. (eq1.1):
 *   dY_i/dt = F+_i - F-_i,   F-_i = k_i Y_i.
 * Reaction j with reactants a_j (and b_j for a two-body reaction) and product
 * c_j carries the flux f_j = k_j Y_a (Y_b).  It adds f_j to F+ of c_j, and it
 * depletes each reactant: the depletion rate of a_j gains k_j Y_b (k_j alone
 * for a one-body reaction) and that of b_j gains k_j Y_a, so that
 * k_i Y_i sums exactly the fluxes that destroy species i.
 *
 * Each sum starts from +0.0 and takes its terms in ascending reaction index.
 */
void orc_rhs(int32_t n_species, int32_t n_reactions, const int32_t *a, const int32_t *b,
             const int32_t *c, const double *k, const double *Y, double *Fp, double *kd)
{
    for (int32_t i = 0; i < n_species; ++i) {
        Fp[i] = 0.0;
        kd[i] = 0.0;
    }
    for (int32_t j = 0; j < n_reactions; ++j) {
        double f;
        if (b[j] < 0) {
            f = k[j] * Y[a[j]];
            kd[a[j]] += k[j];
        } else {
            f = (k[j] * Y[a[j]]) * Y[b[j]];
            kd[a[j]] += k[j] * Y[b[j]];
            kd[b[j]] += k[j] * Y[a[j]];
        }
        Fp[c[j]] += f;
    }
}

/*
 * One update of every species over a step of length h (section "Algebraic
 * Stabilization ... Asymptotic Approximations"):
 *   k_i h <  kappa : forward Euler on Eq. (eq1.1), Y + h (F+ - k Y);
 *   k_i h >= kappa : the asymptotic form Eq. (asySophia), (Y + h F+) / (1 + k h).
 * branch[i] (optional) receives 1 for the asymptotic form, 0 for Euler.
 */
void orc_update(int32_t n_species, const double *Y, const double *Fp, const double *kd,
                double h, double kappa, double *Yn, int32_t *branch)
{
    for (int32_t i = 0; i < n_species; ++i) {
        double kh = kd[i] * h;
        if (kh < kappa) {
            Yn[i] = Y[i] + h * (Fp[i] - kd[i] * Y[i]);
            if (branch) branch[i] = 0;
        } else {
            Yn[i] = (Y[i] + h * Fp[i]) / (1.0 + kh);
            if (branch) branch[i] = 1;
        }
    }
}

/*
 * Relative change that the controller bounds (reading: the paper names an
 * adaptive network timestep but gives no rule; the dY/Y limit is used):
 *   r = max_i |Yn_i - Y_i| / max(Y_i, y_floor),   r = +inf if any Yn_i is not finite.
 */
double orc_change(int32_t n_species, const double *Y, const double *Yn, double y_floor)
{
    double r = 0.0;
    for (int32_t i = 0; i < n_species; ++i) {
        if (!isfinite(Yn[i]))
            return INFINITY;
        double q = fabs(Yn[i] - Y[i]) / fmax(Y[i], y_floor);
        if (q > r)
            r = q;
    }
    return r;
}

typedef struct {
    int64_t capacity; /* entries available in the arrays below */
    int64_t count;    /* attempts recorded (may exceed capacity; extra ones are dropped) */
    double *h;        /* attempted step */
    double *r;        /* relative change of the attempt */
    int32_t *accepted;
} orc_trace;

/*
 * Integrate one zone from t = 0 to t_end with constant rates k.
 * Y holds Y(0) on entry and the last accepted state on exit; *dt holds the
 * trial step on entry and the next trial step on exit (the paper's "final
 * kinetic network integration timestep", section "Implementing the Explicit
 * Asymptotic Algorithm on a CPU-GPU System").  Returns the zone status.
 */
int32_t orc_integrate_zone(int32_t n_species, int32_t n_reactions, const int32_t *a,
                           const int32_t *b, const int32_t *c, const double *k, double *Y,
                           double t_end, double *dt, const orc_options *o, int64_t *n_acc_out,
                           int64_t *n_rej_out, orc_trace *tr)
{
    int64_t n_acc = 0, n_rej = 0;
    *n_acc_out = 0;
    *n_rej_out = 0;
    for (int32_t j = 0; j < n_reactions; ++j)
        if (!isfinite(k[j]))
            return ORC_ZONE_NONFINITE;
    for (int32_t i = 0; i < n_species; ++i)
        if (!isfinite(Y[i]))
            return ORC_ZONE_NONFINITE;
    if (!isfinite(t_end) || !isfinite(*dt))
        return ORC_ZONE_NONFINITE;
    for (int32_t j = 0; j < n_reactions; ++j)
        if (k[j] < 0.0)
            return ORC_ZONE_BAD_INPUT;
    for (int32_t i = 0; i < n_species; ++i)
        if (Y[i] < 0.0)
            return ORC_ZONE_BAD_INPUT;
    if (t_end < 0.0 || !(*dt > 0.0))
        return ORC_ZONE_BAD_INPUT;

    double *Fp = malloc(sizeof(double) * (size_t)n_species);
    double *kd = malloc(sizeof(double) * (size_t)n_species);
    double *Yn = malloc(sizeof(double) * (size_t)n_species);
    double t = 0.0, step = *dt;
    int32_t status = ORC_ZONE_OK;
    for (;;) {
        if (t >= t_end) {
            status = ORC_ZONE_OK;
            break;
        }
        if (n_acc + n_rej >= o->max_steps) {
            status = ORC_ZONE_MAX_STEPS;
            break;
        }
        /* reading: the last step is clipped to land exactly on t_end */
        int clipped = step >= t_end - t;
        double h = clipped ? t_end - t : step;
        orc_rhs(n_species, n_reactions, a, b, c, k, Y, Fp, kd);
        orc_update(n_species, Y, Fp, kd, h, o->kappa, Yn, NULL);
        double r = orc_change(n_species, Y, Yn, o->y_floor);
        int accept = r <= o->tol;
        if (tr) {
            if (tr->count < tr->capacity) {
                tr->h[tr->count] = h;
                tr->r[tr->count] = r;
                tr->accepted[tr->count] = accept;
            }
            tr->count++;
        }
        if (accept) {
            memcpy(Y, Yn, sizeof(double) * (size_t)n_species);
            n_acc++;
            t = clipped ? t_end : t + h;
            /* reading: a clipped last step keeps the unclipped proposal as the
               trial step handed back for the next interval */
            if (!clipped) {
                double g = (r == 0.0) ? o->grow_max : fmin(o->grow_max, o->safety * o->tol / r);
                step = h * g;
            }
        } else {
            n_rej++;
            double s = isinf(r) ? o->shrink_min : fmax(o->shrink_min, o->safety * o->tol / r);
            step = h * s;
            if (step < o->dt_min) {
                status = ORC_ZONE_DT_UNDERFLOW;
                break;
            }
        }
    }
    free(Fp);
    free(kd);
    free(Yn);
    *dt = step;
    *n_acc_out = n_acc;
    *n_rej_out = n_rej;
    return status;
}

/*
 * A batch of independent zones sharing one network (the paper's many
 * concurrent networks, section "Multiple Parallel Networks and Thread
 * Occupancy").  Exactly one of T (Arrhenius, with A and E) and k_zone
 * ([Z][R] constant rates) is given.  Zones run in parallel over n_threads
 * OpenMP threads (<= 0: the runtime's default); the result of a zone does
 * not depend on the thread count.
 */
void orc_integrate_batch(int32_t n_species, int32_t n_reactions, const int32_t *a,
                         const int32_t *b, const int32_t *c, const double *A, const double *E,
                         int32_t n_zones, double *Y, const double *T, const double *k_zone,
                         const double *t_end, double *dt, int64_t *n_acc, int64_t *n_rej,
                         int32_t *status, const orc_options *o, int32_t n_threads)
{
#ifdef _OPENMP
    int nt = n_threads > 0 ? n_threads : omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 1) num_threads(nt)
#endif
    for (int32_t z = 0; z < n_zones; ++z) {
        double *k = malloc(sizeof(double) * (size_t)n_reactions);
        if (k_zone) {
            memcpy(k, k_zone + (size_t)z * n_reactions, sizeof(double) * (size_t)n_reactions);
        } else if (!isfinite(T[z])) {
            for (int32_t j = 0; j < n_reactions; ++j) k[j] = NAN;
        } else if (!(T[z] > 0.0)) {
            for (int32_t j = 0; j < n_reactions; ++j) k[j] = -1.0;
        } else {
            orc_rates_arrhenius(n_reactions, A, E, T[z], k);
        }
        status[z] = orc_integrate_zone(n_species, n_reactions, a, b, c, k,
                                       Y + (size_t)z * n_species, t_end[z], dt + z, o,
                                       n_acc + z, n_rej + z, NULL);
        free(k);
    }
}

int32_t orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
