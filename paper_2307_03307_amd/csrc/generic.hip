// Generic MWU engine for explicit CSR constraint sides (gfx950).
//
// One iteration of Algorithm 2 (Section 4) is split into passes:
//   row pass     y += a dy, z += a dz; weights w = exp(eta (y - L_P)),
//                u = exp(-eta (z - L_C)) and their sums (smax/smin gradients,
//                Section 2.2); exact LSE totals L_P, L_C.
//   column pass  x += a d; g = P^T w, h = C^T u (transpose products over a
//                column structure); d_i = (s/eta) max(0, 1 - g_i/h_i) x_i.
//   forward pass dy = P d, dz = C d.
//   search pass  Psi/Phi of up to KC candidate steps (Section 4.1) and the
//                device-side replay of Algorithm 3.
// Each pass is a wide kernel that stores one reduction record per workgroup
// plus a one-workgroup finisher that folds the records, completes segments
// longer than a tile, and advances the state machine.  Rows of P come first
// in the concatenated row space, then rows of C.  A side equal to the single
// objective row (1/M) 1^T (end of Section 2.2) is kept as a scalar.
#include "device_common.h"

namespace mwu {

// ------------------------------------------------------------------ epilogues

// Column epilogue: commit the pending step, form g, h and the direction.
template <class T>
struct ColEpi {
    GenericDev<T> gd;
    double sP, sC, invSw, invSu, step, qmin;
    int onesP, onesC;
    T a;
    MWU_DEV void load(const Ctl *c)
    {
        sP = c->sP; sC = c->sC; invSw = c->invSw; invSu = c->invSu; step = c->step; qmin = c->qmin;
        onesP = c->onesP; onesC = c->onesC; a = (T)c->alpha;
    }
    // v: [sum d | min g | max d | max h]
    MWU_DEV void operator()(int i, Pair<T> acc, double *v) const
    {
        const double g = onesP ? sP : sP * (double)acc.g * invSw;
        const double h = onesC ? sC : sC * (double)acc.h * invSu;
        const T x = gd.x[i] + a * gd.d[i];
        gd.x[i] = x;
        double di = 0.0;
        if (h > 0.0) {
            const double q = 1.0 - g / h;
            if (q > qmin) di = step * q * (double)x;
        }
        const T dt = (T)di;
        gd.d[i] = dt;
        v[0] += (double)dt;
        v[1] = fmin(v[1], g);
        v[2] = fmax(v[2], (double)dt);
        v[3] = fmax(v[3], h);
        if (gd.g_dbg) { gd.g_dbg[i] = g; gd.h_dbg[i] = h; }
        if (gd.grad) gd.grad[gd.cmap ? gd.cmap[i] : i] = gd.grad_scale * (g - h);
    }
};

// Row epilogue of a forward product: vout[r] = s * acc; v: [min C rows | max P rows].
template <class T>
struct FwdEpi {
    T *vout;
    double sP, sC;
    int mPc;
    MWU_DEV void operator()(int r, T acc, double *v) const
    {
        const double s = r < mPc ? sP : sC;
        const T o = (T)(s * (double)acc);
        vout[r] = o;
        if (r < mPc) v[1] = fmax(v[1], (double)o);
        else v[0] = fmin(v[0], (double)o);
    }
};

// Row epilogue of the FP64 statistics: v: [min C rows | max P rows].
struct StatEpi {
    double sP, sC;
    int mPc;
    MWU_DEV void operator()(int r, double acc, double *v) const
    {
        if (r < mPc) v[1] = fmax(v[1], sP * acc);
        else v[0] = fmin(v[0], sC * acc);
    }
};

// ------------------------------------------------------------------ kernels

template <class T>
__global__ __launch_bounds__(BLOCK) void k_init_x(GenericDev<T> gd, Ctl *ctl, int have_x0,
                                                   const double *src, double *part)
{
    __shared__ double s_wave[4];
    __shared__ double s_rec[QMAX];
    const double eps = ctl->eps, sP = ctl->sP;
    const int onesP = ctl->onesP;
    double v[1] = {0.0};
    const int stride = gridDim.x * BLOCK;
    for (int i = blockIdx.x * BLOCK + threadIdx.x; i < gd.n; i += stride) {
        T x;
        if (src) {
            x = (T)src[gd.cmap ? gd.cmap[i] : i];
            gd.x[i] = x;
        } else if (!have_x0) {
            // Algorithm 1: x_i = eps / (n max_j P_ji)
            const double cm = onesP ? sP : sP * gd.colmaxP[i];
            x = (T)(eps / ((double)gd.n * cm));
            gd.x[i] = x;
        } else {
            x = gd.x[i];
        }
        gd.d[i] = T(0);
        v[0] += (double)x;
    }
    for (int r = blockIdx.x * BLOCK + threadIdx.x; r < gd.mR; r += stride) gd.dyz[r] = T(0);
    const Red red{1, 0, 0};
    block_combine<1>(v, red, 0, s_wave, s_rec);
    store_record(s_rec, 1, part);
}

__global__ __launch_bounds__(BLOCK) void k_init_x_fin(Ctl *ctl, const double *part, int G)
{
    __shared__ double s_wave[4];
    __shared__ double s_rec[QMAX];
    const Red red{1, 0, 0};
    fold_records<1>(part, G, red, 0, s_wave, s_rec);
    if (threadIdx.x == 0) finish_sumx(ctl, s_rec[0]);
}

template <class T>
__global__ __launch_bounds__(BLOCK) void k_row(GenericDev<T> gd, Ctl *ctl, double *part)
{
    __shared__ double s_wave[4 * 4];
    __shared__ double s_rec[QMAX];
    if (ctl->phase != PH_ROW) return;
    const double alpha = ctl->alpha, eta = ctl->eta, LP = ctl->LP, LC = ctl->LC;
    const T a = (T)alpha;
    double v[4] = {0.0, 0.0, INFINITY, -INFINITY};   // sum w | sum u | min z | max y
    const int stride = gridDim.x * BLOCK;
    for (int r = blockIdx.x * BLOCK + threadIdx.x; r < gd.mR; r += stride) {
        const T y = gd.yz[r] + a * gd.dyz[r];
        gd.yz[r] = y;
        if (r < gd.mPc) {
            const T w = exp_arg(eta * ((double)y - LP), T(0));
            gd.wu[r] = w;
            v[0] += (double)w;
            v[3] = fmax(v[3], (double)y);
        } else {
            const T u = row_met(ctl, (double)y) ? T(0) : exp_arg(-eta * ((double)y - LC), T(0));
            gd.wu[r] = u;
            v[1] += (double)u;
            v[2] = fmin(v[2], (double)y);
        }
    }
    const Red red{2, 1, 1};
    block_combine<4>(v, red, 0, s_wave, s_rec);
    store_record(s_rec, 4, part);
}

__global__ __launch_bounds__(BLOCK) void k_row_fin(Ctl *ctl, const double *part, int G)
{
    __shared__ double s_wave[4 * 4];
    __shared__ double s_rec[QMAX];
    if (ctl->phase != PH_ROW) return;
    const Red red{2, 1, 1};
    fold_records<4>(part, G, red, 0, s_wave, s_rec);
    on_ctl(ctl, [&](Ctl *c) { finish_row(c, s_rec); });
}

template <class T>
__global__ __launch_bounds__(BLOCK) void k_col(GenericDev<T> gd, Ctl *ctl, double *part)
{
    __shared__ Pair<T> s_acc[TILE_LDS];
    __shared__ int32_t s_ptr[TILE_NZ + 1];
    __shared__ int32_t s_tseg[BLOCK];
    __shared__ Pair<T> s_tacc[BLOCK];
    __shared__ double s_wave[4 * 4];
    __shared__ double s_rec[QMAX];
    const int ph = ctl->phase;
    if (ph != PH_COL && ph != PH_COMMIT) return;
    if (ph == PH_COMMIT) {
        const T a = (T)ctl->alpha;
        for (int i = blockIdx.x * BLOCK + threadIdx.x; i < gd.n; i += gridDim.x * BLOCK)
            gd.x[i] = gd.x[i] + a * gd.d[i];
        return;
    }
    ColEpi<T> ep;
    ep.gd = gd;
    ep.load(ctl);
    const int mPc = gd.mPc;
    double v[4] = {0.0, INFINITY, -INFINITY, -INFINITY};   // sum d | min g | max d | max h
    auto elem = [&](int k) -> Pair<T> {
        const int r = gd.crow[k];
        const T val = (gd.cval ? gd.cval[k] : T(1)) * gd.wu[r];
        Pair<T> p;
        p.g = r < mPc ? val : T(0);
        p.h = r < mPc ? T(0) : val;
        return p;
    };
    auto epi = [&](int i, Pair<T> acc) { ep(i, acc, v); };
    for (int t = blockIdx.x; t < gd.nctiles; t += gridDim.x) {
        const Tile tl = gd.ctiles[t];
        if (tl.lid < 0) seg_tile<Pair<T>>(tl, gd.cptr, elem, epi, s_acc, s_ptr, s_tseg, s_tacc);
        else chunk_tile<Pair<T>>(tl, elem, s_tacc, (Pair<T> *)gd.clpart, gd.clong.lfirst);
    }
    const Red red{1, 1, 2};
    block_combine<4>(v, red, 0, s_wave, s_rec);
    store_record(s_rec, 4, part);
}

template <class T>
__global__ __launch_bounds__(BLOCK) void k_col_fin(GenericDev<T> gd, Ctl *ctl, const double *part, int G)
{
    __shared__ double s_wave[4 * 4];
    __shared__ double s_rec[QMAX];
    __shared__ double s_lng[QMAX];
    const int ph = ctl->phase;
    if (ph != PH_COL && ph != PH_COMMIT) return;
    if (ph == PH_COMMIT) {
        if (threadIdx.x == 0 && !held(ctl)) { ctl->alpha = 0.0; ctl->phase = PH_DONE; }
        return;
    }
    ColEpi<T> ep;
    ep.gd = gd;
    ep.load(ctl);
    const Red red{1, 1, 2};
    double v[4] = {0.0, INFINITY, -INFINITY, -INFINITY};
    for (int l = threadIdx.x; l < gd.clong.nlong; l += BLOCK)
        ep(gd.clong.lseg[l], long_sum<Pair<T>>(l, (const Pair<T> *)gd.clpart, gd.clong.lfirst,
                                               gd.clong.lcount), v);
    block_combine<4>(v, red, 0, s_wave, s_lng);
    fold_records<4>(part, G, red, 0, s_wave, s_rec);
    on_ctl(ctl, [&](Ctl *c) {
        for (int q = 0; q < 4; ++q) s_rec[q] = red_op(s_rec[q], s_lng[q], q, red);
        finish_col(c, s_rec);
    });
}

// Forward product vout = (scaled rows) * vin.  INIT: y = Px, z = Cx at the
// probe start (no phase check); otherwise dy = Pd, dz = Cd.
template <class T, bool INIT>
__global__ __launch_bounds__(BLOCK) void k_fwd(GenericDev<T> gd, Ctl *ctl, const T *vin, T *vout,
                                                double *part)
{
    __shared__ T s_acc[TILE_LDS];
    __shared__ int32_t s_ptr[TILE_NZ + 1];
    __shared__ int32_t s_tseg[BLOCK];
    __shared__ T s_tacc[BLOCK];
    __shared__ double s_wave[4 * 2];
    __shared__ double s_rec[QMAX];
    if (!INIT && ctl->phase != PH_FWD) return;
    FwdEpi<T> ep{vout, ctl->sP, ctl->sC, gd.mPc};
    double v[2] = {INFINITY, -INFINITY};   // min over C rows | max over P rows
    auto elem = [&](int k) -> T { return (gd.rval ? gd.rval[k] : T(1)) * vin[gd.rcol[k]]; };
    auto epi = [&](int r, T acc) { ep(r, acc, v); };
    for (int t = blockIdx.x; t < gd.nrtiles; t += gridDim.x) {
        const Tile tl = gd.rtiles[t];
        if (tl.lid < 0) seg_tile<T>(tl, gd.rptr, elem, epi, s_acc, s_ptr, s_tseg, s_tacc);
        else chunk_tile<T>(tl, elem, s_tacc, gd.rlpart, gd.rlong.lfirst);
    }
    const Red red{0, 1, 1};
    block_combine<2>(v, red, 0, s_wave, s_rec);
    store_record(s_rec, 2, part);
}

template <class T, bool INIT>
__global__ __launch_bounds__(BLOCK) void k_fwd_fin(GenericDev<T> gd, Ctl *ctl, T *vout,
                                                    const double *part, int G)
{
    __shared__ double s_wave[4 * 2];
    __shared__ double s_rec[QMAX];
    __shared__ double s_lng[QMAX];
    if (!INIT && ctl->phase != PH_FWD) return;
    FwdEpi<T> ep{vout, ctl->sP, ctl->sC, gd.mPc};
    const Red red{0, 1, 1};
    double v[2] = {INFINITY, -INFINITY};
    for (int l = threadIdx.x; l < gd.rlong.nlong; l += BLOCK)
        ep(gd.rlong.lseg[l], long_sum<T>(l, gd.rlpart, gd.rlong.lfirst, gd.rlong.lcount), v);
    block_combine<2>(v, red, 0, s_wave, s_lng);
    fold_records<2>(part, G, red, 0, s_wave, s_rec);
    on_ctl(ctl, [&](Ctl *c) {
        for (int q = 0; q < 2; ++q) s_rec[q] = red_op(s_rec[q], s_lng[q], q, red);
        if (INIT) {
            finish_init_fwd(c, s_rec);
        } else if (!held(c)) {
            c->dymax = s_rec[1];
            begin_search(c, gd.forced);
        }
    });
}

// Certificate statistics of the current x in FP64 whatever the storage type:
// max over packing rows and min over covering rows of (scaled) A x, formed from
// the double coefficients (rval64, nullable = all ones).
template <class T>
__global__ __launch_bounds__(BLOCK) void k_stats(GenericDev<T> gd, Ctl *ctl, const double *rval64,
                                                  double *part)
{
    __shared__ double s_acc[TILE_LDS];
    __shared__ int32_t s_ptr[TILE_NZ + 1];
    __shared__ int32_t s_tseg[BLOCK];
    __shared__ double s_tacc[BLOCK];
    __shared__ double s_wave[4 * 2];
    __shared__ double s_rec[QMAX];
    StatEpi ep{ctl->sP, ctl->sC, gd.mPc};
    double v[2] = {INFINITY, -INFINITY};
    auto elem = [&](int k) -> double { return (rval64 ? rval64[k] : 1.0) * (double)gd.x[gd.rcol[k]]; };
    auto epi = [&](int r, double acc) { ep(r, acc, v); };
    for (int t = blockIdx.x; t < gd.nrtiles; t += gridDim.x) {
        const Tile tl = gd.rtiles[t];
        if (tl.lid < 0) seg_tile<double>(tl, gd.rptr, elem, epi, s_acc, s_ptr, s_tseg, s_tacc);
        else chunk_tile<double>(tl, elem, s_tacc, gd.rlpart64, gd.rlong.lfirst);
    }
    const Red red{0, 1, 1};
    block_combine<2>(v, red, 0, s_wave, s_rec);
    store_record(s_rec, 2, part);
}

template <class T>
__global__ __launch_bounds__(BLOCK) void k_stats_fin(GenericDev<T> gd, Ctl *ctl, const double *part, int G)
{
    __shared__ double s_wave[4 * 2];
    __shared__ double s_rec[QMAX];
    __shared__ double s_lng[QMAX];
    StatEpi ep{ctl->sP, ctl->sC, gd.mPc};
    const Red red{0, 1, 1};
    double v[2] = {INFINITY, -INFINITY};
    for (int l = threadIdx.x; l < gd.rlong.nlong; l += BLOCK)
        ep(gd.rlong.lseg[l], long_sum<double>(l, gd.rlpart64, gd.rlong.lfirst, gd.rlong.lcount), v);
    block_combine<2>(v, red, 0, s_wave, s_lng);
    fold_records<2>(part, G, red, 0, s_wave, s_rec);
    if (threadIdx.x == 0) {
        for (int q = 0; q < 2; ++q) s_rec[q] = red_op(s_rec[q], s_lng[q], q, red);
        ctl->zmin = ctl->onesC ? ctl->sC * ctl->sumx : s_rec[0];
        ctl->ymax = ctl->onesP ? ctl->sP * ctl->sumx : s_rec[1];
    }
}

// Candidate sums of one search pass over the stored rows (KIND fixed per
// launch): packing s1P[k] = sum_i w_i expm1(eta a_k dy_i); covering sums and
// minima as in cov_terms.  Leaves [s1P | s1C | s2C | zmin] in s_rec.
template <class T, int KIND>
__device__ void search_rows(const GenericDev<T> &gd, const Ctl *ctl, double *s_wave, double *s_rec)
{
    const double eta = ctl->eta;
    const int stride = gridDim.x * BLOCK;
    const int r0 = blockIdx.x * BLOCK + threadIdx.x;
    const int mPc = gd.mPc, mR = gd.mR;
    const int nc = ctl->ncand;
    const double *cand = ctl->cand;
    const double a0 = ctl->cand[0], ga0 = ctl->ga0, dymax = ctl->dymax;
    const uint32_t shm = shifted_mask(ctl);
    const double gdel = ctl->gdelta;
    const bool deriv = ctl->skind == SK_NEWTON;
    {
        double s1[KC];
#pragma unroll
        for (int k = 0; k < KC; ++k) s1[k] = 0.0;
        for (int r = r0; r < mPc; r += stride)
            pack_terms<T, KIND>(nc, cand, a0, ga0, gdel, eta, gd.wu[r], gd.dyz[r], dymax, shm, s1, deriv);
        const Red redp{KC, 0, 0};
        block_combine<KC>(s1, redp, 0, s_wave, s_rec);
    }
    {
        CovAcc<T> ca;
        ca.init(pass_minima<KIND>());
        for (int r = mPc + r0; r < mR; r += stride)
            cov_terms<T, KIND>(nc, cand, a0, ga0, gdel, eta, gd.wu[r], gd.yz[r], gd.dyz[r], ca.acc, ca.zmn,
                               deriv);
        ca.combine(s_wave, s_rec + KC);
    }
}

// Search pass over the stored rows: for each candidate step, the sums that
// give Psi and Phi (Section 4.1) plus min(z + a dz) (Algorithm 3 early return).
template <class T>
__global__ __launch_bounds__(BLOCK) void k_search(GenericDev<T> gd, Ctl *ctl, double *part)
{
    __shared__ double s_wave[4 * 3 * KC];
    __shared__ double s_rec[QMAX];
    if (ctl->phase != PH_SEARCH) return;
    const int kind = ctl->skind;
    const double eta = ctl->eta;
    const int stride = gridDim.x * BLOCK;
    const int r0 = blockIdx.x * BLOCK + threadIdx.x;
    const int mPc = gd.mPc, mR = gd.mR;
    if (kind == SK_REFINE) {
        const double a = ctl->ref_alpha;
        if (ctl->ref_valid == 0) {
            double v[2] = {INFINITY, -INFINITY};   // min z' | max eta*y'
            for (int r = r0; r < mR; r += stride) {
                const double yp = (double)gd.yz[r] + a * (double)gd.dyz[r];
                if (r < mPc) v[1] = fmax(v[1], eta * yp);
                else if (!row_met(ctl, (double)gd.yz[r])) v[0] = fmin(v[0], yp);
            }
            const Red red{0, 1, 1};
            block_combine<2>(v, red, 0, s_wave, s_rec);
            store_record_qmajor(s_rec, 2, part);
        } else {                  // [sumP | sumC | sumP' | sumC']
            const double pm = ctl->rfPm, zm = ctl->rfZmin;
            double v[4] = {0.0, 0.0, 0.0, 0.0};
            for (int r = r0; r < mR; r += stride) {
                const double dv = (double)gd.dyz[r];
                const double yp = (double)gd.yz[r] + a * dv;
                if (r < mPc) {
                    const double t = exp(eta * yp - pm);
                    v[0] += t;
                    v[2] += dv * t;
                } else if (!row_met(ctl, (double)gd.yz[r])) {
                    const double t = exp(-eta * (yp - zm));
                    v[1] += t;
                    v[3] += dv * t;
                }
            }
            const Red red{4, 0, 0};
            block_combine<4>(v, red, 0, s_wave, s_rec);
            store_record_qmajor(s_rec, 4, part);
        }
        return;
    }
    switch (kind) {
    case SK_EXP: search_rows<T, SK_EXP>(gd, ctl, s_wave, s_rec); break;
    case SK_GRID: search_rows<T, SK_GRID>(gd, ctl, s_wave, s_rec); break;
    case SK_COMBO: search_rows<T, SK_COMBO>(gd, ctl, s_wave, s_rec); break;
    default: search_rows<T, SK_LIST>(gd, ctl, s_wave, s_rec); break;
    }
    store_record_qmajor(s_rec, 4 * KC, part);
}

__global__ __launch_bounds__(BLOCK) void k_search_fin(Ctl *ctl, const double *part, int G)
{
    __shared__ double s_wave[4 * 4 * KC];
    __shared__ double s_rec[QMAX];
    if (ctl->phase != PH_SEARCH) return;
    // the search records are stored entry-major (G is the search grid)
    if (ctl->skind == SK_REFINE) {
        if (ctl->ref_valid == 0) fold_records_qmajor<2>(part, G, Red{0, 1, 1}, s_wave, s_rec);
        else fold_records_qmajor<4>(part, G, Red{4, 0, 0}, s_wave, s_rec);
    } else {
        const Red red{3 * KC, KC, 0};
        fold_records_qmajor<4 * KC>(part, G, red, s_wave, s_rec);
    }
    // every candidate of a grid or list pass is evaluated at once, one per
    // lane, before the sequential replay
    auto pre = [&](Ctl *c) {
        if (c->skind != SK_REFINE && !c->hold) pre_eval_search(c, s_rec);
    };
    on_ctl_all(ctl, pre, [&](Ctl *c) { finish_search(c, s_rec, c->skind != SK_REFINE); });
}

template <class T>
__global__ void k_widen(const T *src, double *dst, int64_t n)
{
    for (int64_t i = blockIdx.x * (int64_t)BLOCK + threadIdx.x; i < n; i += (int64_t)gridDim.x * BLOCK)
        dst[i] = (double)src[i];
}

template <class T>
__global__ void k_narrow(const double *src, T *dst, int64_t n)
{
    for (int64_t i = blockIdx.x * (int64_t)BLOCK + threadIdx.x; i < n; i += (int64_t)gridDim.x * BLOCK)
        dst[i] = (T)src[i];
}

__global__ void k_set_phase(Ctl *ctl, int phase) { ctl->phase = phase; }

template <class T>
__global__ void k_scale(T *v, int64_t n, int64_t stride, double th)
{
    for (int64_t i = blockIdx.x * (int64_t)BLOCK + threadIdx.x; i < n; i += (int64_t)gridDim.x * BLOCK)
        v[i * stride] = (T)(th * (double)v[i * stride]);
}

// Continue a probe after a direction formed in evaluation mode (the probe
// API): the checks of Algorithm 2 that evaluation mode skipped (covered,
// iteration cap, zero direction), then the step search of this iteration,
// exactly as the finishers of an uninterrupted iteration would start it.
__global__ void k_resume_search(Ctl *c, const double *forced)
{
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    c->eval_mode = 0;
    c->hold = 0;
    c->ev_cached = 0;
    c->alpha = 0.0;
    if (c->zmin >= 1.0) { c->status = ST_FEASIBLE; c->phase = PH_DONE; return; }
    if (c->iter >= c->max_iter) { c->status = ST_MAX_ITER; c->phase = PH_DONE; return; }
    if (!(c->dmax > 0.0)) { c->status = ST_INFEASIBLE; c->phase = PH_DONE; return; }
    begin_search(c, forced);
}

__global__ void k_potential_finish(const double *g, const double *h, int n, double scale,
                                   double *out, const int32_t *map, const Ctl *ctl, double *val)
{
    for (int i = blockIdx.x * BLOCK + threadIdx.x; i < n; i += gridDim.x * BLOCK)
        out[map ? map[i] : i] = scale * (g[i] - h[i]);
    if (val && blockIdx.x == 0 && threadIdx.x == 0) *val = ctl->LP - ctl->LC;
}

// ------------------------------------------------------------------ launchers

static inline int grid_for(int64_t items)
{
    int64_t g = (items + BLOCK - 1) / BLOCK;
    if (g < 1) g = 1;
    if (g > GRID_MAX) g = GRID_MAX;
    return (int)g;
}

#define LAUNCH(kernel, grid, ...) hipLaunchKernelGGL(kernel, dim3(grid), dim3(BLOCK), 0, st, __VA_ARGS__)

template <class T>
static void init_sum(const GenericDev<T> &g, Ctl *ctl, const Launch &L, hipStream_t st, int have_x0,
                     const double *src)
{
    LAUNCH(k_init_x<T>, L.grid_elem_cols, g, ctl, have_x0, src, L.partials);
    LAUNCH(k_init_x_fin, 1, ctl, (const double *)L.partials, L.grid_elem_cols);
}

template <class T>
static void fwd_init(const GenericDev<T> &g, Ctl *ctl, const Launch &L, hipStream_t st)
{
    LAUNCH((k_fwd<T, true>), L.grid_rtile, g, ctl, (const T *)g.x, g.yz, L.partials);
    LAUNCH((k_fwd_fin<T, true>), 1, g, ctl, g.yz, (const double *)L.partials, L.grid_rtile);
}

template <class T>
void generic_init(const GenericDev<T> &g, Ctl *ctl, const Launch &L, hipStream_t st, bool have_x0)
{
    init_sum(g, ctl, L, st, have_x0 ? 1 : 0, nullptr);
    fwd_init(g, ctl, L, st);
}

template <class T>
void generic_load_x(const GenericDev<T> &g, Ctl *ctl, const Launch &L, hipStream_t st,
                    const double *x_dev)
{
    init_sum(g, ctl, L, st, 1, x_dev);
    fwd_init(g, ctl, L, st);
}

template <class T>
void generic_stats(const GenericDev<T> &g, Ctl *ctl, const Launch &L, hipStream_t st,
                   const double *rval64)
{
    init_sum(g, ctl, L, st, 1, nullptr);
    LAUNCH(k_stats<T>, L.grid_rtile, g, ctl, rval64, L.partials);
    LAUNCH(k_stats_fin<T>, 1, g, ctl, (const double *)L.partials, L.grid_rtile);
}

template <class T>
void generic_row(const GenericDev<T> &g, Ctl *ctl, const Launch &L, hipStream_t st)
{
    LAUNCH(k_row<T>, L.grid_elem_rows, g, ctl, L.partials);
    LAUNCH(k_row_fin, 1, ctl, (const double *)L.partials, L.grid_elem_rows);
}

template <class T>
void generic_col(const GenericDev<T> &g, Ctl *ctl, const Launch &L, hipStream_t st)
{
    LAUNCH(k_col<T>, L.grid_ctile, g, ctl, L.partials);
    LAUNCH(k_col_fin<T>, 1, g, ctl, (const double *)L.partials, L.grid_ctile);
}

template <class T>
void generic_fwd(const GenericDev<T> &g, Ctl *ctl, const Launch &L, hipStream_t st)
{
    LAUNCH((k_fwd<T, false>), L.grid_rtile, g, ctl, (const T *)g.d, g.dyz, L.partials);
    LAUNCH((k_fwd_fin<T, false>), 1, g, ctl, g.dyz, (const double *)L.partials, L.grid_rtile);
}

template <class T>
void generic_search(const GenericDev<T> &g, Ctl *ctl, const Launch &L, hipStream_t st)
{
    LAUNCH(k_search<T>, L.grid_search, g, ctl, L.partials);
    LAUNCH(k_search_fin, 1, ctl, (const double *)L.partials, L.grid_search);
}

// One iteration slot with a single search launch: most iterations finish
// their step search in the combined first pass; one that needs more passes
// takes them in the following slots, whose other passes see the search phase
// and return at once.
template <class T>
void generic_iteration(const GenericDev<T> &g, Ctl *ctl, const Launch &L, hipStream_t st)
{
    generic_row(g, ctl, L, st);
    generic_col(g, ctl, L, st);
    generic_fwd(g, ctl, L, st);
    generic_search(g, ctl, L, st);
}

void potential_finish(const double *g_dbg, const double *h_dbg, int n, double scale, double *out,
                      const int32_t *map, const Ctl *ctl, double *val, hipStream_t st)
{
    LAUNCH(k_potential_finish, grid_for(n), g_dbg, h_dbg, n, scale, out, map, ctl, val);
}

template <class T>
void widen(const T *src, double *dst, int64_t n, hipStream_t st)
{
    LAUNCH(k_widen<T>, grid_for(n), src, dst, n);
}

template <class T>
void narrow(const double *src, T *dst, int64_t n, hipStream_t st)
{
    LAUNCH(k_narrow<T>, grid_for(n), src, dst, n);
}

void set_phase(Ctl *ctl, int phase, hipStream_t st)
{
    hipLaunchKernelGGL(k_set_phase, dim3(1), dim3(1), 0, st, ctl, phase);
}

template <class T>
void scale_vec(T *v, int64_t n, int64_t stride, double th, hipStream_t st)
{
    LAUNCH(k_scale<T>, grid_for(n), v, n, stride, th);
}
template <class T>
__global__ void k_set_row(T *rval, double *rval64, int64_t k0, int64_t n, T *cval, const int32_t *pos, double v,
                          double *colmax, const double *base)
{
    for (int64_t j = blockIdx.x * (int64_t)BLOCK + threadIdx.x; j < n; j += (int64_t)gridDim.x * BLOCK) {
        rval[k0 + j] = (T)v;
        rval64[k0 + j] = v;
        cval[pos[j]] = (T)v;
        if (colmax) colmax[j] = fmax(base[j], v);
    }
}

template <class T>
void generic_set_row(T *rval, double *rval64, int64_t k0, int64_t n, T *cval, const int32_t *pos, double v,
                     double *colmax, const double *base, hipStream_t st)
{
    LAUNCH(k_set_row<T>, grid_for(n), rval, rval64, k0, n, cval, pos, v, colmax, base);
}
template void generic_set_row<float>(float *, double *, int64_t, int64_t, float *, const int32_t *, double,
                                     double *, const double *, hipStream_t);
template void generic_set_row<double>(double *, double *, int64_t, int64_t, double *, const int32_t *, double,
                                      double *, const double *, hipStream_t);

template void scale_vec<float>(float *, int64_t, int64_t, double, hipStream_t);
template void scale_vec<double>(double *, int64_t, int64_t, double, hipStream_t);

void resume_search(Ctl *ctl, const double *forced, hipStream_t st)
{
    hipLaunchKernelGGL(k_resume_search, dim3(1), dim3(64), 0, st, ctl, forced);
}

// The main kernel of one pass alone (no finisher): timing of held passes.
template <class T>
void generic_main(const GenericDev<T> &g, Ctl *ctl, const Launch &L, hipStream_t st, int which)
{
    switch (which) {
    case 0: LAUNCH(k_row<T>, L.grid_elem_rows, g, ctl, L.partials); break;
    case 1: LAUNCH(k_col<T>, L.grid_ctile, g, ctl, L.partials); break;
    case 2: LAUNCH((k_fwd<T, false>), L.grid_rtile, g, ctl, (const T *)g.d, g.dyz, L.partials); break;
    default: LAUNCH(k_search<T>, L.grid_search, g, ctl, L.partials); break;
    }
}

// Workgroups per CU of the persistent tile kernels and the search kernel.
template <class T>
void generic_occupancy(int *per_cu_fwd, int *per_cu_col, int *per_cu_search)
{
    int a = 0, b = 0, c = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&a, k_fwd<T, false>, BLOCK, 0) != hipSuccess) a = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, k_col<T>, BLOCK, 0) != hipSuccess) b = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&c, k_search<T>, BLOCK, 0) != hipSuccess) c = 0;
    *per_cu_fwd = a > 0 ? a : 1;
    *per_cu_col = b > 0 ? b : 1;
    *per_cu_search = c > 0 ? c : 1;
}

#define MWU_INSTANTIATE(T)                                                                      \
    template void generic_occupancy<T>(int *, int *, int *);                                   \
    template void generic_main<T>(const GenericDev<T> &, Ctl *, const Launch &, hipStream_t, int); \
    template void generic_init<T>(const GenericDev<T> &, Ctl *, const Launch &, hipStream_t,    \
                                  bool);                                                        \
    template void generic_load_x<T>(const GenericDev<T> &, Ctl *, const Launch &, hipStream_t,  \
                                    const double *);                                            \
    template void generic_row<T>(const GenericDev<T> &, Ctl *, const Launch &, hipStream_t);    \
    template void generic_stats<T>(const GenericDev<T> &, Ctl *, const Launch &, hipStream_t,   \
                                   const double *);                                             \
    template void generic_col<T>(const GenericDev<T> &, Ctl *, const Launch &, hipStream_t);    \
    template void generic_fwd<T>(const GenericDev<T> &, Ctl *, const Launch &, hipStream_t);    \
    template void generic_search<T>(const GenericDev<T> &, Ctl *, const Launch &, hipStream_t); \
    template void generic_iteration<T>(const GenericDev<T> &, Ctl *, const Launch &,            \
                                       hipStream_t);                                            \
    template void widen<T>(const T *, double *, int64_t, hipStream_t);                          \
    template void narrow<T>(const double *, T *, int64_t, hipStream_t);

MWU_INSTANTIATE(float)
MWU_INSTANTIATE(double)

}  // namespace mwu
