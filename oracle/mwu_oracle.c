/*
 * Plain single-threaded FP64 reference implementation of the multiplicative
 * weight update (MWU) solver for positive LPs with step-size search.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle that the GPU library is
 * checked against.  Only the test suite, the smoke check and the CPU baseline
 * leg of the benchmark may load it; the GPU library never calls into it and
 * shares no code, header or table with it.
 *
 * Everything is written for clarity, not speed: matrices are explicit CSR with
 * explicit values, every vector is double, every sum runs in index order.
 *
 * Paper: Ju, Yesil, Sun, Chekuri, Solomonik, "Efficient Parallel
 * Implementation of the Multiplicative Weight Update Method for Graph-based
 * Linear Programs" (arXiv 2307.03307).
 *   - smooth max / min and their gradients: Section 2.2
 *   - Algorithm 1 (parameters, initial point, direction): Section 2.2
 *   - embedding of pure packing/covering objectives and the search over M:
 *     end of Section 2.2
 *   - Algorithm 2 (MWU with step-size search): Section 4
 *   - potential differences Phi, Psi and the bang-for-buck test: Section 4.1
 *   - Algorithm 3 (exponential then binary step search): Section 4.2
 *   - densest subgraph dual with D fixed and searched: Section 3
 *
 * Readings taken where the paper is silent or garbled (each is also listed in
 * the design notes of the repository):
 *   R1  binary search runs while (ub - lb) > eps*lb  (the prose of 4.2; the
 *       algorithm box prints (1-eps)).
 *   R2  the early return of Algorithm 3 tests min(z + alpha*dz) >= 1.
 *   R3  a probe stops FEASIBLE when min(z) >= 1, INFEASIBLE when max(d) = 0
 *       or when alpha < 1, MAX_ITER after max_iter iterations.
 *   R4  T(1) failing is reported as alpha < 1 directly (the bisection of
 *       [1/2, 1] could only end below 1).
 *   R5  step scale s = 1 when one side has exactly one row, else 1/2.
 *   R6  satisfied covering rows are never dropped (Section 6.2 says so).
 *   R7  natural logarithm in eta = 10 ln(m) / eps.
 *   R8  Phi and Psi are evaluated in cancellation-free forms (below) that are
 *       exact identities of the Section 4.1 definitions.
 *   R9  outer search over M (or D): geometric bisection of a search bracket
 *       that moves to every probed value (feasible: upper end, infeasible:
 *       lower end), kept apart from the certified bracket on OPT, which only
 *       certificates move.  It stops when the certified bracket is within
 *       1+eps, when the search bracket is within 1+eps/16, or at the probe cap.
 *       Only certificates move the certified bracket (rescaled feasible
 *       points, weak-duality bounds, infeasible verdicts); a probe that hits
 *       the iteration cap moves only the search bracket (as if infeasible).
 *       The result is certified exactly when the final bracket is within
 *       1+eps.  When the search bracket closes first, the probes continue at
 *       half the tolerance (a feasible probe then overshoots its M by about
 *       eps/2 instead of eps) from the certified bracket, at most twice.
 *   R19 warm start (ORC_STEP_BIN_WARM; the setting of the Bin column of
 *       Table 2, which starts each search at the previous step): the search
 *       of an iteration starts at the step the probe accepted last (1 in a
 *       probe's first iteration).  If T holds there, the search goes on
 *       exactly as Algorithm 3 from that value (doubling with the early
 *       return, then the bisection).  If T fails there, the value is halved
 *       until T holds (a halving below 1 evaluates 1 instead, and a failing
 *       T(1) ends the probe as in R4); the first value where T holds is
 *       returned at once when it satisfies every covering row (R2), and
 *       otherwise the bracket [it, the last failing value] is bisected as in
 *       R1.
 *   R20 Newton step search (ORC_STEP_NEWTON; Section 4.2): Newton's method on
 *       g(alpha) = Phi(alpha)/Psi(alpha) - 1 with g' = (Psi Phi' - Phi Psi') /
 *       Psi^2, where Psi' and Phi' are the averages of P d and C d under the
 *       weights of the moved point (the paper's formulas, the denominator of
 *       Psi' read with Px in place of its printed Pd).  It starts at the step
 *       the probe accepted last; in a probe's first iteration Algorithm 3
 *       from 1 gives the step (the exponential search).  Each Newton step
 *       evaluates the test at its alpha (one evaluation).  A value where the
 *       test holds and every covering row is met (or alpha = 2^50) is
 *       returned at once (R2); a failing test at 1 ends the probe (R4).  The
 *       values tested bracket the largest admissible step between lo (the
 *       largest that passed, 0 before one has) and hi (the smallest that
 *       failed, infinite before one has); once hi <= (1 + eps) lo, lo is the
 *       step, as in Algorithm 3.  Newton's method converges only near its
 *       root, which a start far from it is not, so a Newton iterate outside
 *       (lo, hi), or none (Psi = 0, g' >= 0, a value that is not finite), is
 *       replaced by a safeguard step: 2 alpha while hi is infinite, hi/2
 *       while lo is 0, else sqrt(lo hi).  Every iterate is clamped to
 *       [1, 2^50].  Newton stops at alpha_k when its correction |g/g'| is at
 *       most eps alpha_k (returning alpha_k if the test holds there), or
 *       after 8 evaluations.  From the alpha it stopped at, the values
 *       alpha (1-eps)^p, p = 1, 2, ..., each the previous one times (1 - eps)
 *       and at least 1, are tested in turn; the first where the test holds is
 *       the step, one at or below lo gives lo (it holds there), and a failing
 *       test at 1 ends the probe as in R4.
 *   R22 dropping satisfied covering rows (ORC_FLAG_DROP; the line
 *       C <- {c_i : c_i^T x < 1} of Algorithms 1 and 2, which the paper's own
 *       runs leave out): every iteration works on the covering rows with
 *       z_i < 1 only -- smin, its gradient u (0 on the other rows), h, Phi,
 *       and the early return and the stop test over those rows, with eta
 *       still from the full m.  z only grows, so a row once left out stays
 *       out, and the set is that of the algorithm from the end of the first
 *       iteration on; a row already satisfied at the start is left out of
 *       the first iteration too (the set is a function of the current point
 *       alone).  The probe stops FEASIBLE when no row is left.
 *   R23 mixed optimization (orc_solve_mixed_opt; the last sentence of
 *       Section 2.2): the objective of max/min c^T x s.t. P x <= 1, C x >= 1
 *       is embedded as the row (1/M) c^T x >= 1 (covering side, maximizing)
 *       or <= 1 (packing side, minimizing) and M is searched geometrically;
 *       infeasible probes bound OPT exactly, feasible ones give points with
 *       C x >= 1 and P x within Algorithm 2's 1 + eps of 1 (the violation is
 *       reported); when minimizing, M grows fourfold until a probe is
 *       feasible.
 *   R21 probe-to-probe reuse (the reuse argument of the outer searches): a
 *       probe after the first starts from its predecessor's iterate scaled so
 *       that its largest packing row, under the new probe's scale, is eps --
 *       the level the Algorithm 1 point starts from -- and a warm-started
 *       search begins its first iteration at the predecessor's last step.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int64_t rows, cols;
    const int64_t *ptr;   /* rows+1 */
    const int32_t *idx;   /* column of each nonzero */
    const double *val;    /* value of each nonzero */
} orc_mat;

enum { ORC_RUNNING = 0, ORC_FEASIBLE = 1, ORC_INFEASIBLE = 2, ORC_MAX_ITER = 3 };
enum { ORC_STEP_STD = 0, ORC_STEP_BIN = 1, ORC_STEP_BIN_WARM = 2, ORC_STEP_NEWTON = 3 };
/* flags of the outer searches: probe-to-probe reuse (R21), dropping satisfied covering rows (R22) */
enum { ORC_FLAG_REUSE = 1, ORC_FLAG_DROP = 2 };
enum { ORC_OK = 0, ORC_ERR_ARG = -1, ORC_ERR_UNBOUNDED = -2, ORC_ERR_OOM = -3 };

/* Threshold below which 1 + sum(u*expm1(-b)) is taken as too cancelled and the
 * shifted form of Phi is used instead (R8). */
#define ORC_PHI_LOG1P_MIN 0.5
/* Largest eta*alpha*dy for which the expm1 form of Psi is used (R8). */
#define ORC_PSI_EXPM1_MAX 700.0
/* Times the probe tolerance may be halved when the search bracket closes
 * without a certified (1+eps) bracket (R9). */
#define ORC_MAX_HALVINGS 2
/* Cap of the exponential phase of Algorithm 3. */
#define ORC_ALPHA_CAP 1125899906842624.0 /* 2^50 */
/* Most evaluations of the Newton iteration before its back-off (R20). */
#define ORC_NEWTON_STEPS 8

/* ------------------------------------------------------------------ basics */

/* y = s * A x  (definition of a sparse matrix-vector product) */
void orc_matvec(const orc_mat *A, double s, const double *x, double *y)
{
    for (int64_t r = 0; r < A->rows; ++r) {
        double acc = 0.0;
        for (int64_t k = A->ptr[r]; k < A->ptr[r + 1]; ++k)
            acc += A->val[k] * x[A->idx[k]];
        y[r] = s * acc;
    }
}

/* g = s * A^T w  (scatter over the rows of A) */
void orc_matvec_t(const orc_mat *A, double s, const double *w, double *g)
{
    for (int64_t c = 0; c < A->cols; ++c) g[c] = 0.0;
    for (int64_t r = 0; r < A->rows; ++r)
        for (int64_t k = A->ptr[r]; k < A->ptr[r + 1]; ++k)
            g[A->idx[k]] += A->val[k] * w[r];
    for (int64_t c = 0; c < A->cols; ++c) g[c] *= s;
}

/* smax_eta(y) = (1/eta) log sum exp(eta*y_i), evaluated with the max shift;
 * grad (nullable) receives exp(eta*y)/<1, exp(eta*y)>  (Section 2.2). */
double orc_smax(const double *y, int64_t m, double eta, double *grad)
{
    double ymax = -INFINITY;
    for (int64_t i = 0; i < m; ++i) if (y[i] > ymax) ymax = y[i];
    double sum = 0.0;
    for (int64_t i = 0; i < m; ++i) sum += exp(eta * (y[i] - ymax));
    if (grad) for (int64_t i = 0; i < m; ++i) grad[i] = exp(eta * (y[i] - ymax)) / sum;
    return ymax + log(sum) / eta;
}

/* smin_eta(z) = -(1/eta) log sum exp(-eta*z_j); grad = exp(-eta*z)/<1, exp(-eta*z)> */
double orc_smin(const double *z, int64_t m, double eta, double *grad)
{
    double zmin = INFINITY;
    for (int64_t j = 0; j < m; ++j) if (z[j] < zmin) zmin = z[j];
    double sum = 0.0;
    for (int64_t j = 0; j < m; ++j) sum += exp(-eta * (z[j] - zmin));
    if (grad) for (int64_t j = 0; j < m; ++j) grad[j] = exp(-eta * (z[j] - zmin)) / sum;
    return zmin - log(sum) / eta;
}

/* Smoothed potential of Section 4.1 at x: smax_eta(sP P x) - smin_eta(sC C x),
 * the quantity whose decrease the step test of Algorithm 3 certifies.  grad
 * (nullable, length P->cols) receives its gradient
 * sP P^T grad smax(sP P x) - sC C^T grad smin(sC C x), the g - h of
 * Algorithm 2 (chain rule through the two linear maps). */
double orc_potential(const orc_mat *P, double sP, const orc_mat *C, double sC, double eta,
                     const double *x, double *grad)
{
    int64_t n = P->cols;
    double *y = malloc((size_t)P->rows * sizeof(double));
    double *z = malloc((size_t)C->rows * sizeof(double));
    double *w = malloc((size_t)P->rows * sizeof(double));
    double *u = malloc((size_t)C->rows * sizeof(double));
    double *gh = malloc((size_t)n * sizeof(double));
    double val = NAN;
    if (!y || !z || !w || !u || !gh) goto out;
    orc_matvec(P, sP, x, y);
    orc_matvec(C, sC, x, z);
    val = orc_smax(y, P->rows, eta, w) - orc_smin(z, C->rows, eta, u);
    if (grad) {
        orc_matvec_t(P, sP, w, grad);
        orc_matvec_t(C, sC, u, gh);
        for (int64_t i = 0; i < n; ++i) grad[i] -= gh[i];
    }
out:
    free(y); free(z); free(w); free(u); free(gh);
    return val;
}

/* Psi(alpha) = smax(y + alpha*dy) - smax(y)   (Section 4.1).
 * With w = grad smax(y) and a_i = eta*alpha*dy_i >= 0 this is exactly
 *   eta*Psi = log sum_i w_i e^{a_i} = log1p(sum_i w_i expm1(a_i)),
 * and, when some a_i is large, eta*Psi = eta*(max y' - L) + log sum exp(eta*(y'_i - max y'))
 * with y' = y + alpha*dy and L = smax(y). */
double orc_psi(const double *y, const double *dy, const double *w, int64_t m,
               double eta, double L, double alpha)
{
    double ea = eta * alpha;
    double amax = 0.0;
    for (int64_t i = 0; i < m; ++i) if (ea * dy[i] > amax) amax = ea * dy[i];
    if (amax <= ORC_PSI_EXPM1_MAX) {
        double s = 0.0;
        for (int64_t i = 0; i < m; ++i) s += w[i] * expm1(ea * dy[i]);
        return log1p(s) / eta;
    }
    double ymx = -INFINITY;
    for (int64_t i = 0; i < m; ++i) {
        double yp = y[i] + alpha * dy[i];
        if (yp > ymx) ymx = yp;
    }
    double s = 0.0;
    for (int64_t i = 0; i < m; ++i) s += exp(eta * (y[i] + alpha * dy[i] - ymx));
    return (ymx - L) + log(s) / eta;
}

/* Phi(alpha) = smin(z + alpha*dz) - smin(z)   (Section 4.1).
 * With u = grad smin(z) and b_j = eta*alpha*dz_j >= 0:
 *   eta*Phi = -log sum_j u_j e^{-b_j} = -log1p(sum_j u_j expm1(-b_j)),
 * and, when that sum is close to -1, eta*Phi = eta*(min z' - L) - log sum exp(-eta*(z'_j - min z')).
 * zmin_out (nullable) receives min_j (z_j + alpha*dz_j). */
double orc_phi(const double *z, const double *dz, const double *u, int64_t m,
               double eta, double L, double alpha, double *zmin_out)
{
    double ea = eta * alpha;
    double zpm = INFINITY;
    for (int64_t j = 0; j < m; ++j) {
        double zp = z[j] + alpha * dz[j];
        if (zp < zpm) zpm = zp;
    }
    if (zmin_out) *zmin_out = zpm;
    double s = 0.0;
    for (int64_t j = 0; j < m; ++j) s += u[j] * expm1(-ea * dz[j]);
    if (1.0 + s >= ORC_PHI_LOG1P_MIN) return -log1p(s) / eta;
    double t = 0.0;
    for (int64_t j = 0; j < m; ++j) t += exp(-eta * (z[j] + alpha * dz[j] - zpm));
    return (zpm - L) - log(t) / eta;
}

/* ------------------------------------------------------------------ state */

typedef struct {
    const orc_mat *P, *C;
    double sP, sC;              /* uniform scale applied to every value of P, C */
    int64_t n, mP, mC;
    double eta, eps, step;      /* step = s/eta in the direction formula */
    double *x, *y, *z, *d, *dy, *dz, *w, *u, *g, *h;
    double LP, LC;              /* smax(y), smin(z) of the current point */
    /* the covering rows the iteration works on (R22): all of them, or with
     * drop set the rows with z < 1, gathered into za, dza, ua (na rows) */
    int drop;
    int64_t na;
    int64_t *ai;                /* their row indices */
    double *za, *dza, *ua;
} orc_state;

typedef struct {
    int32_t status;
    int64_t iterations;
    int64_t evaluations;        /* number of T(alpha) evaluations */
    double pack_bound;          /* min over iterations of 1/min_i g_i   */
    double cover_bound;         /* max over iterations of 1/max_i h_i   */
    double last_alpha;
    double max_violation;       /* max{0, max(Px)-1, 1-min(Cx)} at exit */
} orc_probe_result;

typedef struct {
    double psi, phi, zmin_new;
    int pass;
} orc_eval;

static orc_eval evaluate(orc_state *st, double alpha)
{
    orc_eval e;
    e.psi = orc_psi(st->y, st->dy, st->w, st->mP, st->eta, st->LP, alpha);
    e.phi = orc_phi(st->za, st->dza, st->ua, st->na, st->eta, st->LC, alpha, &e.zmin_new);
    /* bang-for-buck: f = Phi/Psi >= 1, i.e. Phi >= Psi (Psi >= 0) */
    e.pass = (e.phi >= e.psi);
    return e;
}

/* Bisection of [lb, ub] (T holds at lb, fails at ub) until (ub-lb) <= eps*lb
 * (R1); returns lb. */
static double bisect(orc_state *st, double lb, double ub, int64_t *evals)
{
    while (ub - lb > st->eps * lb) {
        double beta = (lb + ub) / 2.0;
        orc_eval eb = evaluate(st, beta);
        ++*evals;
        if (eb.pass) lb = beta; else ub = beta;
    }
    return lb;
}

/* Algorithm 3 from alpha = start (start = 1: the algorithm as printed):
 * doubling while T holds, with the early return (R2), then the bisection of
 * [alpha, 2 alpha].  When T fails at start > 1 the search halves downward
 * (R19).  Returns a value < 1 when T(1) fails (R4). */
static double step_search_from(orc_state *st, double start, int64_t *evals)
{
    double alpha = start;
    orc_eval e = evaluate(st, alpha);
    ++*evals;
    if (!e.pass) {
        if (!(start > 1.0)) return 0.5;
        double ub = start;
        for (;;) {                                    /* downward (R19) */
            double b = ub / 2.0;
            if (b < 1.0) b = 1.0;
            orc_eval eb = evaluate(st, b);
            ++*evals;
            if (eb.pass) {
                if (eb.zmin_new >= 1.0) return b;
                return bisect(st, b, ub, evals);
            }
            if (b <= 1.0) return 0.5;
            ub = b;
        }
    }
    for (;;) {
        if (e.zmin_new >= 1.0) return alpha;          /* early return (R2) */
        if (alpha >= ORC_ALPHA_CAP) return alpha;
        double next = 2.0 * alpha;
        orc_eval en = evaluate(st, next);
        ++*evals;
        if (!en.pass) break;
        alpha = next;
        e = en;
    }
    return bisect(st, alpha, 2.0 * alpha, evals);
}

/* Psi'(alpha) and Phi'(alpha) (Section 4.2): the averages of dy and dz under
 * the weights of the moved rows y' = y + alpha dy, z' = z + alpha dz, each
 * formed with the shift of its largest weight so that no term overflows or
 * all underflow.  A single row gives its own dy or dz. */
static void derivatives(const orc_state *st, double alpha, double *dpsi, double *dphi)
{
    if (st->mP == 1) *dpsi = st->dy[0];
    else {
        double ymx = -INFINITY, num = 0.0, den = 0.0;
        for (int64_t i = 0; i < st->mP; ++i) {
            double yp = st->y[i] + alpha * st->dy[i];
            if (yp > ymx) ymx = yp;
        }
        for (int64_t i = 0; i < st->mP; ++i) {
            double t = exp(st->eta * (st->y[i] + alpha * st->dy[i] - ymx));
            num += st->dy[i] * t;
            den += t;
        }
        *dpsi = num / den;
    }
    if (st->mC == 1) *dphi = st->dz[0];
    else {
        double zmn = INFINITY, num = 0.0, den = 0.0;
        for (int64_t j = 0; j < st->mC; ++j) {
            double zp = st->z[j] + alpha * st->dz[j];
            if (zp < zmn) zmn = zp;
        }
        for (int64_t j = 0; j < st->mC; ++j) {
            double t = exp(-st->eta * (st->z[j] + alpha * st->dz[j] - zmn));
            num += st->dz[j] * t;
            den += t;
        }
        *dphi = num / den;
    }
}

/* Newton's method for the step (R20), from `start` (>= 1): Newton steps on
 * g = Phi/Psi - 1 kept inside the bracket of the values tested so far, each
 * one evaluation of the test, then the (1-eps)^p back-off from the alpha it
 * stopped at.  Returns a value < 1 when the test fails at 1. */
static double step_search_newton(orc_state *st, double start, int64_t *evals)
{
    double a = start < 1.0 ? 1.0 : start;
    double lo = 0.0, hi = INFINITY;        /* largest passing, smallest failing alpha tested */
    orc_eval e;
    for (int k = 0;; ++k) {
        e = evaluate(st, a);
        ++*evals;
        if (e.pass) {
            if (e.zmin_new >= 1.0 || a >= ORC_ALPHA_CAP) return a;     /* (R2) */
            lo = a;
        } else {
            if (!(a > 1.0)) return 0.5;                                /* T(1) fails (R4) */
            hi = a;
        }
        if (hi <= (1.0 + st->eps) * lo) return lo;                     /* bracket of Algorithm 3 */
        if (k + 1 >= ORC_NEWTON_STEPS) break;
        double next = NAN;
        if (e.psi > 0.0) {
            double dpsi, dphi;
            derivatives(st, a, &dpsi, &dphi);
            double g = e.phi / e.psi - 1.0;
            double gp = (e.psi * dphi - e.phi * dpsi) / (e.psi * e.psi);
            if (gp < 0.0 && isfinite(g)) {
                double corr = g / gp;
                if (fabs(corr) <= st->eps * a) {                       /* converged at a */
                    if (e.pass) return a;
                    break;
                }
                next = a - corr;
            }
        }
        if (!(next > lo && next < hi)) {                               /* safeguard step */
            if (hi == INFINITY) next = 2.0 * a;
            else if (lo == 0.0) next = hi / 2.0;
            else next = sqrt(lo * hi);
        }
        if (next < 1.0) next = 1.0;
        if (next > ORC_ALPHA_CAP) next = ORC_ALPHA_CAP;
        a = next;
    }
    if (e.pass) return a;
    double b = a;
    for (;;) {                                                      /* (1-eps)^p back-off */
        b *= 1.0 - st->eps;
        if (b <= lo) return lo;
        if (b < 1.0) b = 1.0;
        orc_eval eb = evaluate(st, b);
        ++*evals;
        if (eb.pass) return b;
        if (!(b > 1.0)) return 0.5;                                 /* T(1) fails (R4) */
    }
}

/* Algorithm 3: exponential search from alpha = 1, then binary search on
 * [alpha/2, alpha] until (ub-lb) <= eps*lb; returns lb.  Returns a value < 1
 * when T(1) fails (R4). */
static double step_search(orc_state *st, int64_t *evals)
{
    return step_search_from(st, 1.0, evals);
}

static double col_max_P(const orc_state *st, double *colmax)
{
    for (int64_t i = 0; i < st->n; ++i) colmax[i] = 0.0;
    for (int64_t r = 0; r < st->mP; ++r)
        for (int64_t k = st->P->ptr[r]; k < st->P->ptr[r + 1]; ++k) {
            double v = st->sP * st->P->val[k];
            if (v > colmax[st->P->idx[k]]) colmax[st->P->idx[k]] = v;
        }
    double mn = INFINITY;
    for (int64_t i = 0; i < st->n; ++i) if (colmax[i] < mn) mn = colmax[i];
    return mn;
}

/* Gradients and direction at the current x (Algorithm 2 lines for g, h, d):
 *   w = grad smax(y), u = grad smin(z), g = P^T w, h = C^T u,
 *   d_i = (s/eta) max{0, 1 - g_i/h_i} x_i  (d_i = 0 when h_i = 0),
 * then dy = P d and dz = C d.  Returns max(d). */
static double direction(orc_state *st)
{
    st->LP = orc_smax(st->y, st->mP, st->eta, st->w);
    if (st->drop) {                 /* (R22) smin and u over the rows with z < 1 */
        st->na = 0;
        for (int64_t j = 0; j < st->mC; ++j)
            if (st->z[j] < 1.0) { st->ai[st->na] = j; st->za[st->na] = st->z[j]; ++st->na; }
        st->LC = orc_smin(st->za, st->na, st->eta, st->ua);
        for (int64_t j = 0; j < st->mC; ++j) st->u[j] = 0.0;
        for (int64_t k = 0; k < st->na; ++k) st->u[st->ai[k]] = st->ua[k];
    } else {
        st->LC = orc_smin(st->z, st->mC, st->eta, st->u);
    }
    orc_matvec_t(st->P, st->sP, st->w, st->g);
    orc_matvec_t(st->C, st->sC, st->u, st->h);
    double dmax = 0.0;
    for (int64_t i = 0; i < st->n; ++i) {
        double di = 0.0;
        if (st->h[i] > 0.0) {
            double r = 1.0 - st->g[i] / st->h[i];
            di = st->step * (r > 0.0 ? r : 0.0) * st->x[i];
        }
        st->d[i] = di;
        if (di > dmax) dmax = di;
    }
    orc_matvec(st->P, st->sP, st->d, st->dy);
    orc_matvec(st->C, st->sC, st->d, st->dz);
    if (st->drop)
        for (int64_t k = 0; k < st->na; ++k) st->dza[k] = st->dz[st->ai[k]];
    return dmax;
}

static void state_free(orc_state *st)
{
    free(st->y); free(st->z); free(st->d); free(st->dy); free(st->dz);
    free(st->w); free(st->u); free(st->g); free(st->h);
    if (st->drop) { free(st->ai); free(st->za); free(st->dza); free(st->ua); }
}

static int state_init(orc_state *st, const orc_mat *P, double sP, const orc_mat *C,
                      double sC, double eps, double *x, int drop)
{
    memset(st, 0, sizeof(*st));
    if (!P || !C || P->cols != C->cols || P->rows < 1 || C->rows < 1 || !(eps > 0.0 && eps < 1.0))
        return ORC_ERR_ARG;
    st->P = P; st->C = C; st->sP = sP; st->sC = sC;
    st->n = P->cols; st->mP = P->rows; st->mC = C->rows; st->eps = eps;
    st->x = x;
    /* Algorithm 1: eta = 10 ln(m)/eps with m = m_P + m_C (R7) */
    st->eta = 10.0 * log((double)(st->mP + st->mC)) / eps;
    /* (R5) factor-2 step when one side is a single row (end of Section 2.2) */
    double s = (st->mP == 1 || st->mC == 1) ? 1.0 : 0.5;
    st->step = s / st->eta;
    st->y = calloc((size_t)st->mP, sizeof(double));
    st->z = calloc((size_t)st->mC, sizeof(double));
    st->dy = calloc((size_t)st->mP, sizeof(double));
    st->dz = calloc((size_t)st->mC, sizeof(double));
    st->w = calloc((size_t)st->mP, sizeof(double));
    st->u = calloc((size_t)st->mC, sizeof(double));
    st->d = calloc((size_t)st->n, sizeof(double));
    st->g = calloc((size_t)st->n, sizeof(double));
    st->h = calloc((size_t)st->n, sizeof(double));
    if (!st->y || !st->z || !st->dy || !st->dz || !st->w || !st->u || !st->d || !st->g || !st->h) {
        state_free(st);
        return ORC_ERR_OOM;
    }
    st->drop = drop != 0;
    st->na = st->mC;
    if (st->drop) {
        st->ai = calloc((size_t)st->mC, sizeof(int64_t));
        st->za = calloc((size_t)st->mC, sizeof(double));
        st->dza = calloc((size_t)st->mC, sizeof(double));
        st->ua = calloc((size_t)st->mC, sizeof(double));
        if (!st->ai || !st->za || !st->dza || !st->ua) { state_free(st); return ORC_ERR_OOM; }
    } else {
        st->za = st->z; st->dza = st->dz; st->ua = st->u;
    }
    return ORC_OK;
}

/* Algorithm 1 initial point x_i = eps / (n * max_j P_ji). */
int orc_initial_point(const orc_mat *P, double sP, double eps, double *x)
{
    double *cm = calloc((size_t)P->cols, sizeof(double));
    if (!cm) return ORC_ERR_OOM;
    orc_state tmp;
    memset(&tmp, 0, sizeof tmp);
    tmp.P = P; tmp.sP = sP; tmp.n = P->cols; tmp.mP = P->rows;
    double mn = col_max_P(&tmp, cm);
    if (!(mn > 0.0)) { free(cm); return ORC_ERR_UNBOUNDED; }
    for (int64_t i = 0; i < P->cols; ++i) x[i] = eps / ((double)P->cols * cm[i]);
    free(cm);
    return ORC_OK;
}

/*
 * One feasibility probe: Algorithm 2 with the step rule of Algorithm 3
 * (step_rule = ORC_STEP_BIN) or the standard step alpha = 1 (ORC_STEP_STD).
 *
 * x: in/out, length n.  If x0_given is 0 it is overwritten with the
 * Algorithm 1 initial point.  forced_alpha (nullable, n_forced entries)
 * replaces the step search for the first n_forced iterations: the decision
 * replay mode used to compare trajectories.  alpha_trace (nullable, trace_cap
 * entries) receives the accepted steps.
 */
int orc_probe_from(const orc_mat *P, double sP, const orc_mat *C, double sC, double eps,
                   int32_t max_iter, int32_t step_rule, int32_t x0_given, double *x,
                   const double *forced_alpha, int64_t n_forced,
                   double *alpha_trace, int64_t trace_cap, double start_alpha, int32_t drop,
                   orc_probe_result *res);

int orc_probe(const orc_mat *P, double sP, const orc_mat *C, double sC, double eps,
              int32_t max_iter, int32_t step_rule, int32_t x0_given, double *x,
              const double *forced_alpha, int64_t n_forced,
              double *alpha_trace, int64_t trace_cap, orc_probe_result *res)
{
    return orc_probe_from(P, sP, C, sC, eps, max_iter, step_rule, x0_given, x, forced_alpha, n_forced,
                          alpha_trace, trace_cap, 0.0, 0, res);
}

/* As orc_probe; with the warm-started search (ORC_STEP_BIN_WARM) the first
 * iteration's search starts at start_alpha when it exceeds 1 (the last step
 * of a previous probe, R21) instead of at 1, and with drop set the
 * iterations leave the satisfied covering rows out (R22). */
int orc_probe_from(const orc_mat *P, double sP, const orc_mat *C, double sC, double eps,
                   int32_t max_iter, int32_t step_rule, int32_t x0_given, double *x,
                   const double *forced_alpha, int64_t n_forced,
                   double *alpha_trace, int64_t trace_cap, double start_alpha, int32_t drop,
                   orc_probe_result *res)
{
    orc_state st;
    int rc = state_init(&st, P, sP, C, sC, eps, x, drop);
    if (rc) return rc;
    memset(res, 0, sizeof(*res));
    res->pack_bound = INFINITY;
    res->cover_bound = 0.0;
    if (!x0_given) {
        rc = orc_initial_point(P, sP, eps, x);
        if (rc) { state_free(&st); return rc; }
    }
    orc_matvec(P, sP, x, st.y);            /* y = P x, z = C x */
    orc_matvec(C, sC, x, st.z);
    res->status = ORC_MAX_ITER;
    double warm = start_alpha;   /* where a warm-started search begins */
    int64_t t;
    for (t = 0; t < max_iter; ++t) {
        double zmin = INFINITY;
        for (int64_t j = 0; j < st.mC; ++j) if (st.z[j] < zmin) zmin = st.z[j];
        if (zmin >= 1.0) { res->status = ORC_FEASIBLE; break; }      /* (R3) */
        double dmax = direction(&st);
        {   /* weak-duality bounds from the current weights */
            double gmin = INFINITY, hmax = 0.0;
            for (int64_t i = 0; i < st.n; ++i) {
                if (st.g[i] < gmin) gmin = st.g[i];
                if (st.h[i] > hmax) hmax = st.h[i];
            }
            if (gmin > 0.0 && 1.0 / gmin < res->pack_bound) res->pack_bound = 1.0 / gmin;
            if (hmax > 0.0 && 1.0 / hmax > res->cover_bound) res->cover_bound = 1.0 / hmax;
        }
        if (dmax == 0.0) { res->status = ORC_INFEASIBLE; break; }
        double alpha;
        if (forced_alpha && t < n_forced) alpha = forced_alpha[t];
        else if (step_rule == ORC_STEP_STD) alpha = 1.0;
        else if (step_rule == ORC_STEP_BIN_WARM && warm > 1.0)
            alpha = step_search_from(&st, warm, &res->evaluations);   /* (R19) */
        else if (step_rule == ORC_STEP_NEWTON && warm >= 1.0)
            alpha = step_search_newton(&st, warm, &res->evaluations);   /* (R20) */
        else alpha = step_search(&st, &res->evaluations);
        if (alpha < 1.0) { res->status = ORC_INFEASIBLE; break; }
        if (alpha_trace && t < trace_cap) alpha_trace[t] = alpha;
        res->last_alpha = alpha;
        warm = alpha;
        for (int64_t i = 0; i < st.n; ++i) x[i] += alpha * st.d[i];
        for (int64_t r = 0; r < st.mP; ++r) st.y[r] += alpha * st.dy[r];
        for (int64_t r = 0; r < st.mC; ++r) st.z[r] += alpha * st.dz[r];
    }
    res->iterations = t;
    {
        double ymax = -INFINITY, zmin = INFINITY;
        for (int64_t r = 0; r < st.mP; ++r) if (st.y[r] > ymax) ymax = st.y[r];
        for (int64_t r = 0; r < st.mC; ++r) if (st.z[r] < zmin) zmin = st.z[r];
        double v = 0.0;
        if (ymax - 1.0 > v) v = ymax - 1.0;
        if (1.0 - zmin > v) v = 1.0 - zmin;
        res->max_violation = v;
    }
    state_free(&st);
    return ORC_OK;
}

/*
 * Quantities of one iteration at a given point, for per-pass comparison:
 * y = Px, z = Cx, w, u, g, h, d, dy, dz, and (Psi, Phi, min z') at each of
 * the n_alpha step sizes.  Every output pointer is nullable.  drop: leave
 * the satisfied covering rows out (R22); eta_override > 0 replaces eta.
 */
int orc_iteration_terms(const orc_mat *P, double sP, const orc_mat *C, double sC,
                        double eps, const double *x_in,
                        double *y, double *z, double *w, double *u, double *g, double *h,
                        double *d, double *dy, double *dz, double *LP, double *LC,
                        const double *alphas, int64_t n_alpha,
                        double *psi, double *phi, double *zmin_new, int32_t drop, double eta_override)
{
    orc_state st;
    double *x = malloc((size_t)P->cols * sizeof(double));
    if (!x) return ORC_ERR_OOM;
    memcpy(x, x_in, (size_t)P->cols * sizeof(double));
    int rc = state_init(&st, P, sP, C, sC, eps, x, drop);
    if (rc) { free(x); return rc; }
    if (eta_override > 0.0) {       /* the eta of a larger row set (checks of R22) */
        st.step *= st.eta / eta_override;
        st.eta = eta_override;
    }
    orc_matvec(P, sP, x, st.y);
    orc_matvec(C, sC, x, st.z);
    direction(&st);
#define OUT(dst, src, len) if (dst) memcpy(dst, src, (size_t)(len) * sizeof(double))
    OUT(y, st.y, st.mP); OUT(z, st.z, st.mC); OUT(w, st.w, st.mP); OUT(u, st.u, st.mC);
    OUT(g, st.g, st.n); OUT(h, st.h, st.n); OUT(d, st.d, st.n);
    OUT(dy, st.dy, st.mP); OUT(dz, st.dz, st.mC);
#undef OUT
    if (LP) *LP = st.LP;
    if (LC) *LC = st.LC;
    for (int64_t k = 0; k < n_alpha; ++k) {
        orc_eval e = evaluate(&st, alphas[k]);
        if (psi) psi[k] = e.psi;
        if (phi) phi[k] = e.phi;
        if (zmin_new) zmin_new[k] = e.zmin_new;
    }
    state_free(&st);
    free(x);
    return ORC_OK;
}

/* Eta used by a probe with m_P + m_C rows (Algorithm 1). */
double orc_eta(int64_t rows_total, double eps) { return 10.0 * log((double)rows_total) / eps; }

/* ------------------------------------------------------------ outer search */

/* Start of the next probe when probes reuse their predecessor's point (R21):
 * the previous iterate x scaled so that its largest packing row under the
 * next probe's P (values scaled by sP) is eps -- the level the Algorithm 1
 * point starts from (P x0 <= eps).  Returns 0 when x has no positive
 * packing row (the caller then takes the Algorithm 1 point). */
int orc_reuse_start(const orc_mat *P, double sP, double eps, double *x)
{
    double *y = malloc((size_t)P->rows * sizeof(double));
    if (!y) return 0;
    orc_matvec(P, sP, x, y);
    double ymax = 0.0;
    for (int64_t j = 0; j < P->rows; ++j) if (y[j] > ymax) ymax = y[j];
    free(y);
    if (!(ymax > 0.0) || !isfinite(ymax)) return 0;
    double th = eps / ymax;
    for (int64_t i = 0; i < P->cols; ++i) x[i] *= th;
    return 1;
}

typedef struct {
    int32_t status;            /* 0 certified, 1 uncertified, <0 error */
    double objective;          /* value of the returned feasible solution */
    double lower, upper;       /* final bracket on OPT */
    int64_t probes, total_iterations, final_probe_iterations, evaluations;
} orc_solve_result;

/* C = (1/M) 1^T as an explicit single row over n columns. */
typedef struct { int64_t ptr[2]; int32_t *idx; double *val; orc_mat m; } ones_row;

static int ones_row_make(ones_row *o, int64_t n)
{
    o->idx = malloc((size_t)n * sizeof(int32_t));
    o->val = malloc((size_t)n * sizeof(double));
    if (!o->idx || !o->val) { free(o->idx); free(o->val); return ORC_ERR_OOM; }
    for (int64_t i = 0; i < n; ++i) { o->idx[i] = (int32_t)i; o->val[i] = 1.0; }
    o->ptr[0] = 0; o->ptr[1] = n;
    o->m.rows = 1; o->m.cols = n; o->m.ptr = o->ptr; o->m.idx = o->idx; o->m.val = o->val;
    return ORC_OK;
}

static void ones_row_free(ones_row *o) { free(o->idx); free(o->val); }

/*
 * Pure packing  max 1^T x  s.t.  P x <= 1, x >= 0  (P already normalized).
 * The objective is embedded as the covering row (1/M) 1^T x >= 1 and M is
 * searched geometrically (end of Section 2.2).  Bracket: lo from feasible
 * rescaled points x/max(Px); hi from infeasible probes and from the weak
 * duality bound 1/min_i (P^T w)_i of every iteration.  Stops at
 * hi <= (1+eps) lo.
 */
int orc_solve_packing(const orc_mat *P, double eps, int32_t max_iter, int32_t max_probes,
                      int32_t step_rule, int32_t flags, double *x_best, orc_solve_result *r)
{
    double last = 0.0;   /* the previous probe's last step (R21) */
    int64_t n = P->cols;
    memset(r, 0, sizeof(*r));
    ones_row one;
    int rc = ones_row_make(&one, n);
    if (rc) return rc;
    double *x = malloc((size_t)n * sizeof(double));
    double *y = malloc((size_t)P->rows * sizeof(double));
    double *cm = calloc((size_t)n, sizeof(double));
    if (!x || !y || !cm) { rc = ORC_ERR_OOM; goto done; }
    /* upper bound: sum_i max_{j: P_ji > 0} 1/P_ji */
    for (int64_t i = 0; i < n; ++i) cm[i] = INFINITY;
    for (int64_t rr = 0; rr < P->rows; ++rr)
        for (int64_t k = P->ptr[rr]; k < P->ptr[rr + 1]; ++k)
            if (P->val[k] > 0.0 && P->val[k] < cm[P->idx[k]]) cm[P->idx[k]] = P->val[k];
    double hi = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        if (!isfinite(cm[i])) { rc = ORC_ERR_UNBOUNDED; goto done; }
        hi += 1.0 / cm[i];
    }
    /* lower bound: rescaled Algorithm 1 start */
    rc = orc_initial_point(P, 1.0, eps, x);
    if (rc) goto done;
    orc_matvec(P, 1.0, x, y);
    double ymax = 0.0, sx = 0.0;
    for (int64_t j = 0; j < P->rows; ++j) if (y[j] > ymax) ymax = y[j];
    for (int64_t i = 0; i < n; ++i) sx += x[i];
    double lo = sx / ymax;
    for (int64_t i = 0; i < n; ++i) x_best[i] = x[i] / ymax;
    double slo = lo, shi = hi;   /* search bracket for M (R9) */
    double ep = eps;             /* probe tolerance (R9) */
    int halvings = 0;
    while (r->probes < max_probes && hi > (1.0 + eps) * lo) {
        if (!(shi > (1.0 + eps / 16.0) * slo)) {
            if (halvings == ORC_MAX_HALVINGS) break;
            halvings++;
            ep *= 0.5;
            slo = lo;
            shi = hi;
            continue;
        }
        double M = sqrt(slo * shi);
        orc_probe_result pr;
        {
            const int warm = (flags & ORC_FLAG_REUSE) && r->probes > 0 && orc_reuse_start(P, 1.0, ep, x);
            rc = orc_probe_from(P, 1.0, &one.m, 1.0 / M, ep, max_iter, step_rule, warm, x,
                                NULL, 0, NULL, 0, warm ? last : 0.0, (flags & ORC_FLAG_DROP) != 0, &pr);
        }
        if (rc) goto done;
        last = pr.last_alpha;
        r->probes++;
        r->total_iterations += pr.iterations;
        r->final_probe_iterations = pr.iterations;
        r->evaluations += pr.evaluations;
        if (pr.pack_bound < hi) hi = pr.pack_bound;
        if (pr.status == ORC_FEASIBLE) {
            orc_matvec(P, 1.0, x, y);
            ymax = 0.0; sx = 0.0;
            for (int64_t j = 0; j < P->rows; ++j) if (y[j] > ymax) ymax = y[j];
            for (int64_t i = 0; i < n; ++i) sx += x[i];
            if (sx / ymax > lo) {
                lo = sx / ymax;
                for (int64_t i = 0; i < n; ++i) x_best[i] = x[i] / ymax;
            }
            slo = M;
        } else {
            if (pr.status == ORC_INFEASIBLE && M < hi) hi = M;
            shi = M;
        }
        if (lo > slo) slo = lo;
        if (hi < shi) shi = hi;
    }
    r->lower = lo; r->upper = hi; r->objective = lo;
    r->status = (hi <= (1.0 + eps) * lo) ? 0 : 1;
done:
    free(x); free(y); free(cm);
    ones_row_free(&one);
    return rc;
}

/*
 * Pure covering  min 1^T x  s.t.  C x >= 1, x >= 0  (C normalized, no empty
 * rows or columns).  The objective is the packing row (1/M) 1^T x <= 1.
 * Bracket: hi from feasible rescaled points x/min(Cx) and from the trivially
 * feasible x_i = max_{j: C_ji>0} 1/(C_ji nnz_j); lo from infeasible probes and
 * from the weak duality bound 1/max_i (C^T u)_i of every iteration (uniform u
 * gives the starting lo).
 */
int orc_solve_covering(const orc_mat *C, double eps, int32_t max_iter, int32_t max_probes,
                       int32_t step_rule, int32_t flags, double *x_best, orc_solve_result *r)
{
    double last = 0.0;   /* the previous probe's last step (R21) */
    int64_t n = C->cols;
    memset(r, 0, sizeof(*r));
    ones_row one;
    int rc = ones_row_make(&one, n);
    if (rc) return rc;
    double *x = malloc((size_t)n * sizeof(double));
    double *z = malloc((size_t)C->rows * sizeof(double));
    double *cs = calloc((size_t)n, sizeof(double));
    if (!x || !z || !cs) { rc = ORC_ERR_OOM; goto done; }
    /* lo at uniform u: 1 / max_i (C^T 1/m)_i */
    for (int64_t j = 0; j < C->rows; ++j)
        for (int64_t k = C->ptr[j]; k < C->ptr[j + 1]; ++k) cs[C->idx[k]] += C->val[k];
    double csmax = 0.0;
    for (int64_t i = 0; i < n; ++i) if (cs[i] > csmax) csmax = cs[i];
    if (!(csmax > 0.0)) { rc = ORC_ERR_ARG; goto done; }
    double lo = (double)C->rows / csmax;
    /* hi from a trivially feasible point */
    for (int64_t i = 0; i < n; ++i) x[i] = 0.0;
    for (int64_t j = 0; j < C->rows; ++j) {
        int64_t nnz = C->ptr[j + 1] - C->ptr[j];
        if (nnz == 0) { rc = ORC_ERR_ARG; goto done; }
        for (int64_t k = C->ptr[j]; k < C->ptr[j + 1]; ++k) {
            double v = 1.0 / (C->val[k] * (double)nnz);
            if (v > x[C->idx[k]]) x[C->idx[k]] = v;
        }
    }
    double hi = 0.0;
    for (int64_t i = 0; i < n; ++i) { hi += x[i]; x_best[i] = x[i]; }
    double slo = lo, shi = hi;   /* search bracket for M (R9) */
    double ep = eps;             /* probe tolerance (R9) */
    int halvings = 0;
    while (r->probes < max_probes && hi > (1.0 + eps) * lo) {
        if (!(shi > (1.0 + eps / 16.0) * slo)) {
            if (halvings == ORC_MAX_HALVINGS) break;
            halvings++;
            ep *= 0.5;
            slo = lo;
            shi = hi;
            continue;
        }
        double M = sqrt(slo * shi);
        orc_probe_result pr;
        {
            const int warm = (flags & ORC_FLAG_REUSE) && r->probes > 0 && orc_reuse_start(&one.m, 1.0 / M, ep, x);
            rc = orc_probe_from(&one.m, 1.0 / M, C, 1.0, ep, max_iter, step_rule, warm, x,
                                NULL, 0, NULL, 0, warm ? last : 0.0, (flags & ORC_FLAG_DROP) != 0, &pr);
        }
        if (rc) goto done;
        last = pr.last_alpha;
        r->probes++;
        r->total_iterations += pr.iterations;
        r->final_probe_iterations = pr.iterations;
        r->evaluations += pr.evaluations;
        if (pr.cover_bound > lo) lo = pr.cover_bound;
        if (pr.status == ORC_FEASIBLE) {
            orc_matvec(C, 1.0, x, z);
            double zmin = INFINITY, sx = 0.0;
            for (int64_t j = 0; j < C->rows; ++j) if (z[j] < zmin) zmin = z[j];
            for (int64_t i = 0; i < n; ++i) sx += x[i];
            if (sx / zmin < hi) {
                hi = sx / zmin;
                for (int64_t i = 0; i < n; ++i) x_best[i] = x[i] / zmin;
            }
            shi = M;
        } else {
            if (pr.status == ORC_INFEASIBLE && M > lo) lo = M;
            slo = M;
        }
        if (lo > slo) slo = lo;
        if (hi < shi) shi = hi;
    }
    r->lower = lo; r->upper = hi; r->objective = hi;
    r->status = (hi <= (1.0 + eps) * lo) ? 0 : 1;
done:
    free(x); free(z); free(cs);
    ones_row_free(&one);
    return rc;
}

/* ------------------------------------------------ mixed optimization (R23) */

/*
 * maximize (maximize = 1) or minimize (maximize = 0) c^T x
 *   s.t.  P x <= 1,  C x >= 1,  x >= 0      (rows already normalized by b)
 * The objective is embedded as one more row, (1/M) c^T x >= 1 on the
 * covering side (maximization) or (1/M) c^T x <= 1 on the packing side
 * (minimization), and M is searched geometrically (end of Section 2.2).
 * An infeasible probe at M proves OPT < M (maximization) or OPT > M
 * (minimization); a feasible probe returns x with C x >= 1, the objective
 * row met, and every packing row (the objective row too when minimizing)
 * at most max(Px), which Algorithm 2 keeps within about 1 + eps of 1.
 * Bracket: [largest feasible M, smallest infeasible M] when
 * maximizing (the upper end starts at sum_i c_i / max_j P_ji, which bounds
 * OPT), [largest infeasible M, smallest feasible M] when minimizing (the
 * lower end starts at the uniform dual bound m_C min_i c_i / (1^T C)_i of
 * the covering rows, and the probes grow M fourfold until one is feasible).
 * x_best is the point of the best feasible probe; r->objective its c^T x;
 * *violation its max{0, max(Px) - 1} over those packing rows.  The probes
 * start from the Algorithm 1 point (probe reuse is not applied here).
 */
int orc_solve_mixed_opt(const orc_mat *P, const orc_mat *C, const double *c, int32_t maximize, double eps,
                        int32_t max_iter, int32_t max_probes, int32_t step_rule, int32_t flags,
                        double *x_best, double *violation, orc_solve_result *r)
{
    const int64_t n = P->cols;
    memset(r, 0, sizeof(*r));
    *violation = 0.0;
    if (C->cols != n || P->rows < 1 || C->rows < 1) return ORC_ERR_ARG;
    for (int64_t i = 0; i < n; ++i) if (!(c[i] > 0.0) || !isfinite(c[i])) return ORC_ERR_ARG;
    /* the side that receives the objective row, as a copy with one more row */
    const orc_mat *S = maximize ? C : P;
    const int64_t nnz = S->ptr[S->rows];
    int64_t *ptr = malloc((size_t)(S->rows + 2) * sizeof(int64_t));
    int32_t *idx = malloc((size_t)(nnz + n) * sizeof(int32_t));
    double *val = malloc((size_t)(nnz + n) * sizeof(double));
    double *x = malloc((size_t)n * sizeof(double));
    double *y = malloc((size_t)(P->rows + 1) * sizeof(double));
    double *cm = calloc((size_t)n, sizeof(double));
    double *cs = calloc((size_t)n, sizeof(double));
    int rc = ORC_OK;
    if (!ptr || !idx || !val || !x || !y || !cm || !cs) { rc = ORC_ERR_OOM; goto done; }
    memcpy(ptr, S->ptr, (size_t)(S->rows + 1) * sizeof(int64_t));
    memcpy(idx, S->idx, (size_t)nnz * sizeof(int32_t));
    memcpy(val, S->val, (size_t)nnz * sizeof(double));
    for (int64_t i = 0; i < n; ++i) idx[nnz + i] = (int32_t)i;
    ptr[S->rows + 1] = nnz + n;
    orc_mat A = {S->rows + 1, n, ptr, idx, val};
    const orc_mat *Pp = maximize ? P : &A, *Cp = maximize ? &A : C;
    /* starting brackets */
    double lo, hi, slo, shi;
    if (maximize) {
        for (int64_t j = 0; j < P->rows; ++j)
            for (int64_t k = P->ptr[j]; k < P->ptr[j + 1]; ++k)
                if (P->val[k] > cm[P->idx[k]]) cm[P->idx[k]] = P->val[k];
        hi = 0.0;
        for (int64_t i = 0; i < n; ++i) {
            if (!(cm[i] > 0.0)) { rc = ORC_ERR_UNBOUNDED; goto done; }
            hi += c[i] / cm[i];
        }
        lo = 0.0;
        shi = hi;
        slo = hi / 1048576.0;
    } else {
        for (int64_t j = 0; j < C->rows; ++j)
            for (int64_t k = C->ptr[j]; k < C->ptr[j + 1]; ++k) cs[C->idx[k]] += C->val[k];
        double t = INFINITY;
        for (int64_t i = 0; i < n; ++i) if (cs[i] > 0.0 && c[i] / cs[i] < t) t = c[i] / cs[i];
        if (!isfinite(t)) { rc = ORC_ERR_ARG; goto done; }
        lo = (double)C->rows * t;
        hi = INFINITY;
        /* the value of the covering-feasible point x_i = max_{j: C_ji>0} 1/(C_ji nnz_j) */
        for (int64_t i = 0; i < n; ++i) x[i] = 0.0;
        for (int64_t j = 0; j < C->rows; ++j) {
            const double nz = (double)(C->ptr[j + 1] - C->ptr[j]);
            for (int64_t k = C->ptr[j]; k < C->ptr[j + 1]; ++k) {
                const double v = 1.0 / (C->val[k] * nz);
                if (v > x[C->idx[k]]) x[C->idx[k]] = v;
            }
        }
        double cx = 0.0;
        for (int64_t i = 0; i < n; ++i) cx += c[i] * x[i];
        slo = lo;
        shi = cx > 2.0 * lo ? cx : 2.0 * lo;
    }
    int have = 0;
    while (r->probes < max_probes && !(hi <= (1.0 + eps) * lo)) {
        /* minimization before any feasible probe: probe the top of the bracket */
        const int grow = !maximize && !have;
        if (!grow && !(shi > (1.0 + eps / 16.0) * slo)) break;
        const double M = grow ? shi : sqrt(slo * shi);
        for (int64_t i = 0; i < n; ++i) val[nnz + i] = c[i] / M;
        orc_probe_result pr;
        /* every probe starts from the Algorithm 1 point (no reuse here) */
        rc = orc_probe_from(Pp, 1.0, Cp, 1.0, eps, max_iter, step_rule, 0, x, NULL, 0, NULL, 0,
                            0.0, (flags & ORC_FLAG_DROP) != 0, &pr);
        if (rc) goto done;
        r->probes++;
        r->total_iterations += pr.iterations;
        r->final_probe_iterations = pr.iterations;
        r->evaluations += pr.evaluations;
        const int feasible = pr.status == ORC_FEASIBLE;
        if (feasible) {
            double cx = 0.0, ym = 0.0;
            for (int64_t i = 0; i < n; ++i) cx += c[i] * x[i];
            orc_matvec(Pp, 1.0, x, y);      /* the packing rows with the objective row if there */
            for (int64_t j = 0; j < Pp->rows; ++j) if (y[j] > ym) ym = y[j];
            const int better = !have || (maximize ? M > lo : M < hi);
            if (better) {
                memcpy(x_best, x, (size_t)n * sizeof(double));
                r->objective = cx;
                *violation = ym > 1.0 ? ym - 1.0 : 0.0;
                have = 1;
            }
            if (maximize) { if (M > lo) lo = M; slo = M; }
            else { if (M < hi) hi = M; shi = M; }
        } else {
            if (maximize) {
                if (pr.status == ORC_INFEASIBLE && M < hi) hi = M;
                shi = M;
            } else {
                if (pr.status == ORC_INFEASIBLE && M > lo) lo = M;
                slo = M;
                if (grow) shi = 4.0 * M;
            }
        }
        if (slo < lo) slo = lo;
        if (shi > hi) shi = hi;
    }
    r->lower = lo;
    r->upper = hi;
    r->status = (have && hi <= (1.0 + eps) * lo) ? 0 : 1;
done:
    free(ptr); free(idx); free(val); free(x); free(y); free(cm); free(cs);
    return rc;
}

/* ------------------------------------------------------ densest subgraph */

typedef struct { double key; int32_t id; } keyed;

static int keyed_desc(const void *a, const void *b)
{
    const keyed *p = a, *q = b;
    if (p->key > q->key) return -1;
    if (p->key < q->key) return 1;
    return (p->id > q->id) - (p->id < q->id);
}

/* Largest density |E(S)|/|S| over the prefixes S of the vertices sorted by
 * score (descending, ties to the smaller id): a level-set rounding whose every
 * candidate is a real subgraph, hence a lower bound on the densest density. */
double orc_level_set_density(int64_t nv, int64_t ne, const int32_t *eu, const int32_t *ev,
                             const double *score)
{
    keyed *k = malloc((size_t)nv * sizeof(keyed));
    int64_t *rank = malloc((size_t)nv * sizeof(int64_t));
    int64_t *cnt = calloc((size_t)nv + 1, sizeof(int64_t));
    double best = 0.0;
    if (!k || !rank || !cnt) goto out;
    for (int64_t i = 0; i < nv; ++i) { k[i].key = score[i]; k[i].id = (int32_t)i; }
    qsort(k, (size_t)nv, sizeof(keyed), keyed_desc);
    for (int64_t i = 0; i < nv; ++i) rank[k[i].id] = i;
    for (int64_t e = 0; e < ne; ++e) {
        int64_t a = rank[eu[e]], b = rank[ev[e]];
        cnt[(a > b ? a : b) + 1]++;
    }
    int64_t acc = 0;
    for (int64_t s = 1; s <= nv; ++s) {
        acc += cnt[s];
        double dens = (double)acc / (double)s;
        if (dens > best) best = dens;
    }
out:
    free(k); free(rank); free(cnt);
    return best;
}

/*
 * Densest subgraph through the dual of Charikar's LP with D fixed (Section 3):
 * find z in R^{2m} with W z >= 1, O z <= D 1, z >= 0, and search D.
 * O (n x 2m) and W (m x 2m) are passed explicitly; eu/ev is the edge list the
 * level-set rounding uses.  hi: feasible probes give D' = max(O z/min(Wz)); the
 * start z = 1/2 gives Delta/2.  lo: infeasible probes, the whole graph's
 * density, and level sets of the final vertex loads of every probe.
 */
int orc_solve_densest(const orc_mat *O, const orc_mat *W, const int32_t *eu, const int32_t *ev,
                      double eps, int32_t max_iter, int32_t max_probes, int32_t step_rule,
                      int32_t flags, double *z_best, orc_solve_result *r)
{
    double last = 0.0;   /* the previous probe's last step (R21) */
    int64_t n = O->cols, nv = O->rows, ne = W->rows;
    memset(r, 0, sizeof(*r));
    double *z = malloc((size_t)n * sizeof(double));
    double *load = malloc((size_t)nv * sizeof(double));
    double *cov = malloc((size_t)ne * sizeof(double));
    int rc = ORC_OK;
    if (!z || !load || !cov) { rc = ORC_ERR_OOM; goto done; }
    for (int64_t i = 0; i < n; ++i) { z[i] = 0.5; z_best[i] = 0.5; }
    orc_matvec(O, 1.0, z, load);
    double hi = 0.0;
    for (int64_t v = 0; v < nv; ++v) if (load[v] > hi) hi = load[v];
    double lo = (double)ne / (double)nv;
    double slo = lo, shi = hi;   /* search bracket for D (R9) */
    double ep = eps;             /* probe tolerance (R9) */
    int halvings = 0;
    while (r->probes < max_probes && hi > (1.0 + eps) * lo) {
        if (!(shi > (1.0 + eps / 16.0) * slo)) {
            if (halvings == ORC_MAX_HALVINGS) break;
            halvings++;
            ep *= 0.5;
            slo = lo;
            shi = hi;
            continue;
        }
        double D = sqrt(slo * shi);
        orc_probe_result pr;
        {
            const int warm = (flags & ORC_FLAG_REUSE) && r->probes > 0 && orc_reuse_start(O, 1.0 / D, ep, z);
            rc = orc_probe_from(O, 1.0 / D, W, 1.0, ep, max_iter, step_rule, warm, z,
                                NULL, 0, NULL, 0, warm ? last : 0.0, (flags & ORC_FLAG_DROP) != 0, &pr);
        }
        if (rc) goto done;
        last = pr.last_alpha;
        r->probes++;
        r->total_iterations += pr.iterations;
        r->final_probe_iterations = pr.iterations;
        r->evaluations += pr.evaluations;
        orc_matvec(O, 1.0, z, load);
        double lsd = orc_level_set_density(nv, ne, eu, ev, load);
        if (lsd > lo) lo = lsd;
        if (pr.status == ORC_FEASIBLE) {
            orc_matvec(W, 1.0, z, cov);
            double cmin = INFINITY, lmax = 0.0;
            for (int64_t e = 0; e < ne; ++e) if (cov[e] < cmin) cmin = cov[e];
            for (int64_t v = 0; v < nv; ++v) if (load[v] > lmax) lmax = load[v];
            if (lmax / cmin < hi) {
                hi = lmax / cmin;
                for (int64_t i = 0; i < n; ++i) z_best[i] = z[i] / cmin;
            }
            shi = D;
        } else {
            if (pr.status == ORC_INFEASIBLE && D > lo) lo = D;
            slo = D;
        }
        if (lo > slo) slo = lo;
        if (hi < shi) shi = hi;
    }
    r->lower = lo; r->upper = hi; r->objective = hi;
    r->status = (hi <= (1.0 + eps) * lo) ? 0 : 1;
done:
    free(z); free(load); free(cov);
    return rc;
}

/*
 * Algorithm 3 on given vectors (w = grad smax(y), u = grad smin(z), L_P =
 * smax(y), L_C = smin(z)), for testing the search on its own, started at
 * `start` (1: the algorithm as printed; above 1: the warm start of R19).
 * Returns the accepted alpha (< 1 means T(1) failed) and the number of T
 * evaluations.
 */
double orc_step_search_terms_from(const double *y, const double *dy, const double *w, int64_t mP,
                                  double LP, const double *z, const double *dz, const double *u,
                                  int64_t mC, double LC, double eta, double eps, double start,
                                  int64_t *evals)
{
    orc_state st;
    memset(&st, 0, sizeof st);
    st.y = (double *)y; st.dy = (double *)dy; st.w = (double *)w; st.mP = mP; st.LP = LP;
    st.z = (double *)z; st.dz = (double *)dz; st.u = (double *)u; st.mC = mC; st.LC = LC;
    st.za = st.z; st.dza = st.dz; st.ua = st.u; st.na = mC;
    st.eta = eta; st.eps = eps;
    *evals = 0;
    return step_search_from(&st, start, evals);
}

/* The Newton search of R20 from `start` on given vectors, and the two
 * derivatives it uses at alpha (testing the search on its own). */
double orc_newton_search_terms(const double *y, const double *dy, const double *w, int64_t mP,
                               double LP, const double *z, const double *dz, const double *u,
                               int64_t mC, double LC, double eta, double eps, double start,
                               int64_t *evals)
{
    orc_state st;
    memset(&st, 0, sizeof st);
    st.y = (double *)y; st.dy = (double *)dy; st.w = (double *)w; st.mP = mP; st.LP = LP;
    st.z = (double *)z; st.dz = (double *)dz; st.u = (double *)u; st.mC = mC; st.LC = LC;
    st.za = st.z; st.dza = st.dz; st.ua = st.u; st.na = mC;
    st.eta = eta; st.eps = eps;
    *evals = 0;
    return step_search_newton(&st, start, evals);
}

void orc_step_derivatives(const double *y, const double *dy, int64_t mP, const double *z,
                          const double *dz, int64_t mC, double eta, double alpha, double *dpsi,
                          double *dphi)
{
    orc_state st;
    memset(&st, 0, sizeof st);
    st.y = (double *)y; st.dy = (double *)dy; st.mP = mP;
    st.z = (double *)z; st.dz = (double *)dz; st.mC = mC;
    st.eta = eta;
    derivatives(&st, alpha, dpsi, dphi);
}

/* The search from alpha = 1 (Algorithm 3 as printed). */
double orc_step_search_terms(const double *y, const double *dy, const double *w, int64_t mP,
                             double LP, const double *z, const double *dz, const double *u,
                             int64_t mC, double LC, double eta, double eps, int64_t *evals)
{
    return orc_step_search_terms_from(y, dy, w, mP, LP, z, dz, u, mC, LC, eta, eps, 1.0, evals);
}
