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
// Rows of P come first in the concatenated row space, then rows of C.  A side
// equal to the single objective row (1/M) 1^T (end of Section 2.2) is kept as
// a scalar in the control block.
#include "device_common.h"

namespace mwu {

// ------------------------------------------------------------------ finishers

MWU_DEV void finish_row(Ctl *c, const double *rec)
{
    // rec: [sum w | sum u | min z | max y]
    if (held(c)) return;
    const double a = c->alpha;
    bool bad = false;
    if (c->onesP) {
        c->y1 += a * c->dy1;
        c->LP = c->y1;
        c->invSw = 1.0;
        c->ymax = c->y1;
    } else {
        const double sw = rec[0];
        bad |= !(sw > 0.0) || !isfinite(sw);
        c->LP += log(sw) / c->eta;
        c->invSw = 1.0 / sw;
        c->ymax = rec[3];
    }
    if (c->onesC) {
        c->z1 += a * c->dz1;
        c->LC = c->z1;
        c->invSu = 1.0;
        c->zmin = c->z1;
    } else {
        const double su = rec[1];
        bad |= !(su > 0.0) || !isfinite(su);
        c->LC -= log(su) / c->eta;
        c->invSu = 1.0 / su;
        c->zmin = rec[2];
    }
    if (c->eval_mode) { c->phase = PH_COL; return; }
    if (bad) { c->status = ST_NUMERIC; c->phase = PH_COMMIT; return; }
    if (c->zmin >= 1.0) { c->status = ST_FEASIBLE; c->phase = PH_COMMIT; }
    else if (c->iter >= c->max_iter) { c->status = ST_MAX_ITER; c->phase = PH_COMMIT; }
    else c->phase = PH_COL;
}

MWU_DEV void finish_col(Ctl *c, const double *rec)
{
    // rec: [sum d | min g | max d | max h]
    if (held(c)) return;
    c->alpha = 0.0;
    c->dsum = rec[0];
    c->gmin = rec[1];
    c->dmax = rec[2];
    c->hmax = rec[3];
    if (c->gmin > 0.0 && 1.0 / c->gmin < c->pack_bound) c->pack_bound = 1.0 / c->gmin;
    if (c->hmax > 0.0 && 1.0 / c->hmax > c->cover_bound) c->cover_bound = 1.0 / c->hmax;
    c->dy1 = c->onesP ? c->sP * c->dsum : 0.0;
    c->dz1 = c->onesC ? c->sC * c->dsum : 0.0;
    if (c->eval_mode) { c->phase = PH_FWD; return; }
    if (!(c->dmax > 0.0)) { c->status = ST_INFEASIBLE; c->phase = PH_DONE; return; }
    c->phase = PH_FWD;
}

MWU_DEV void finish_init_fwd(Ctl *c, const double *rec)
{
    // rec: [min z | max y]
    c->zmin = c->onesC ? c->z1 : rec[0];
    c->ymax = c->onesP ? c->y1 : rec[1];
    c->LP = c->ymax;        // first shifts; the row pass turns them into exact LSE totals
    c->LC = c->zmin;
    c->alpha = 0.0;
    c->status = ST_RUNNING;
    c->phase = PH_ROW;
}

// ------------------------------------------------------------------ kernels

template <class T>
__global__ __launch_bounds__(BLOCK) void k_init_x(GenericDev<T> gd, Ctl *ctl, int have_x0,
                                                   double *part, double *gpart, unsigned *tick)
{
    __shared__ double s_wave[4];
    __shared__ double s_rec[QMAX];
    const double eps = ctl->eps, sP = ctl->sP;
    const int onesP = ctl->onesP;
    double v[1] = {0.0};
    const int stride = gridDim.x * BLOCK;
    for (int i = blockIdx.x * BLOCK + threadIdx.x; i < gd.n; i += stride) {
        T x;
        if (!have_x0) {
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
    Red red{1, 0, 0};
    block_combine<1>(v, red, 0, s_wave, s_rec);
    if (grid_reduce(s_rec, red, part, gpart, tick) && threadIdx.x == 0) {
        ctl->sumx = s_rec[0];
        ctl->y1 = ctl->sP * s_rec[0];
        ctl->z1 = ctl->sC * s_rec[0];
        ctl->dy1 = 0.0;
        ctl->dz1 = 0.0;
    }
}

template <class T>
__global__ __launch_bounds__(BLOCK) void k_load_x(GenericDev<T> gd, Ctl *ctl, const double *src,
                                                   double *part, double *gpart, unsigned *tick)
{
    __shared__ double s_wave[4];
    __shared__ double s_rec[QMAX];
    double v[1] = {0.0};
    const int stride = gridDim.x * BLOCK;
    for (int i = blockIdx.x * BLOCK + threadIdx.x; i < gd.n; i += stride) {
        const T x = (T)src[i];
        gd.x[i] = x;
        gd.d[i] = T(0);
        v[0] += (double)x;
    }
    for (int r = blockIdx.x * BLOCK + threadIdx.x; r < gd.mR; r += stride) gd.dyz[r] = T(0);
    Red red{1, 0, 0};
    block_combine<1>(v, red, 0, s_wave, s_rec);
    if (grid_reduce(s_rec, red, part, gpart, tick) && threadIdx.x == 0) {
        ctl->sumx = s_rec[0];
        ctl->y1 = ctl->sP * s_rec[0];
        ctl->z1 = ctl->sC * s_rec[0];
        ctl->dy1 = 0.0;
        ctl->dz1 = 0.0;
    }
}

template <class T>
__global__ __launch_bounds__(BLOCK) void k_row(GenericDev<T> gd, Ctl *ctl, double *part,
                                                double *gpart, unsigned *tick)
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
            const T w = exp_t((T)(eta * ((double)y - LP)));
            gd.wu[r] = w;
            v[0] += (double)w;
            v[3] = fmax(v[3], (double)y);
        } else {
            const T u = exp_t((T)(-eta * ((double)y - LC)));
            gd.wu[r] = u;
            v[1] += (double)u;
            v[2] = fmin(v[2], (double)y);
        }
    }
    const Red red{2, 1, 1};
    block_combine<4>(v, red, 0, s_wave, s_rec);
    if (grid_reduce(s_rec, red, part, gpart, tick) && threadIdx.x == 0) finish_row(ctl, s_rec);
}

template <class T>
__global__ __launch_bounds__(BLOCK) void k_col(GenericDev<T> gd, Ctl *ctl, double *part,
                                                double *gpart, unsigned *tick)
{
    __shared__ Pair<T> s_acc[TILE_LDS];
    __shared__ int32_t s_ptr[TILE_NZ + 1];
    __shared__ int32_t s_tseg[BLOCK];
    __shared__ Pair<T> s_tacc[BLOCK];
    __shared__ double s_wave[4 * 4];
    __shared__ double s_rec[QMAX];
    const int ph = ctl->phase;
    if (ph != PH_COL && ph != PH_COMMIT) return;
    const double alpha = ctl->alpha;
    const T a = (T)alpha;
    const int stride = gridDim.x * BLOCK;
    if (ph == PH_COMMIT) {
        for (int i = blockIdx.x * BLOCK + threadIdx.x; i < gd.n; i += stride)
            gd.x[i] = gd.x[i] + a * gd.d[i];
        double v[1] = {0.0};
        const Red red{1, 0, 0};
        block_combine<1>(v, red, 0, s_wave, s_rec);
        if (grid_reduce(s_rec, red, part, gpart, tick) && threadIdx.x == 0) {
            ctl->alpha = 0.0;
            ctl->phase = PH_DONE;
        }
        return;
    }
    const double sP = ctl->sP, sC = ctl->sC, invSw = ctl->invSw, invSu = ctl->invSu;
    const double step = ctl->step;
    const int onesP = ctl->onesP, onesC = ctl->onesC;
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
    auto epi = [&](int i, Pair<T> acc) {
        const double g = onesP ? sP : sP * (double)acc.g * invSw;
        const double h = onesC ? sC : sC * (double)acc.h * invSu;
        const T x = gd.x[i] + a * gd.d[i];
        gd.x[i] = x;
        double di = 0.0;
        if (h > 0.0) {
            const double q = 1.0 - g / h;
            if (q > 0.0) di = step * q * (double)x;
        }
        const T dt = (T)di;
        gd.d[i] = dt;
        v[0] += (double)dt;
        v[1] = fmin(v[1], g);
        v[2] = fmax(v[2], (double)dt);
        v[3] = fmax(v[3], h);
        if (gd.g_dbg) { gd.g_dbg[i] = g; gd.h_dbg[i] = h; }
    };
    for (int t = blockIdx.x; t < gd.nctiles; t += gridDim.x) {
        const Tile tl = gd.ctiles[t];
        if (tl.lid < 0) seg_tile<Pair<T>>(tl, gd.cptr, elem, epi, s_acc, s_ptr, s_tseg, s_tacc);
        else chunk_tile<Pair<T>>(tl, elem, epi, s_tacc, (Pair<T> *)gd.clpart, gd.clfirst,
                                 gd.clcount, gd.cltick);
    }
    const Red red{1, 1, 2};
    block_combine<4>(v, red, 0, s_wave, s_rec);
    if (grid_reduce(s_rec, red, part, gpart, tick) && threadIdx.x == 0) finish_col(ctl, s_rec);
}

// Forward product vout = (scaled rows) * vin.  INIT: y = Px, z = Cx at the
// probe start (no phase check); otherwise dy = Pd, dz = Cd and the search setup.
template <class T, bool INIT>
__global__ __launch_bounds__(BLOCK) void k_fwd(GenericDev<T> gd, Ctl *ctl, const T *vin, T *vout,
                                                double *part, double *gpart, unsigned *tick)
{
    __shared__ T s_acc[TILE_LDS];
    __shared__ int32_t s_ptr[TILE_NZ + 1];
    __shared__ int32_t s_tseg[BLOCK];
    __shared__ T s_tacc[BLOCK];
    __shared__ double s_wave[4 * 2];
    __shared__ double s_rec[QMAX];
    if (!INIT && ctl->phase != PH_FWD) return;
    const double sP = ctl->sP, sC = ctl->sC;
    const int mPc = gd.mPc;
    double v[2] = {INFINITY, -INFINITY};   // min over C rows | max over P rows
    auto elem = [&](int k) -> T { return (gd.rval ? gd.rval[k] : T(1)) * vin[gd.rcol[k]]; };
    auto epi = [&](int r, T acc) {
        const double s = r < mPc ? sP : sC;
        const T o = (T)(s * (double)acc);
        vout[r] = o;
        if (r < mPc) v[1] = fmax(v[1], (double)o);
        else v[0] = fmin(v[0], (double)o);
    };
    for (int t = blockIdx.x; t < gd.nrtiles; t += gridDim.x) {
        const Tile tl = gd.rtiles[t];
        if (tl.lid < 0) seg_tile<T>(tl, gd.rptr, elem, epi, s_acc, s_ptr, s_tseg, s_tacc);
        else chunk_tile<T>(tl, elem, epi, s_tacc, (T *)gd.rlpart, gd.rlfirst, gd.rlcount, gd.rltick);
    }
    const Red red{0, 1, 1};
    block_combine<2>(v, red, 0, s_wave, s_rec);
    if (grid_reduce(s_rec, red, part, gpart, tick) && threadIdx.x == 0) {
        if (INIT) {
            finish_init_fwd(ctl, s_rec);
        } else if (!held(ctl)) {
            ctl->dymax = s_rec[1];
            begin_search(ctl, gd.forced);
        }
    }
}

// Certificate statistics of the current x in FP64 whatever the storage type:
// max over packing rows and min over covering rows of (scaled) A x, formed from
// the double coefficients (rval64, nullable = all ones).
template <class T>
__global__ __launch_bounds__(BLOCK) void k_stats(GenericDev<T> gd, Ctl *ctl, const double *rval64,
                                                  double *part, double *gpart, unsigned *tick)
{
    __shared__ double s_acc[TILE_LDS];
    __shared__ int32_t s_ptr[TILE_NZ + 1];
    __shared__ int32_t s_tseg[BLOCK];
    __shared__ double s_tacc[BLOCK];
    __shared__ double s_wave[4 * 2];
    __shared__ double s_rec[QMAX];
    const double sP = ctl->sP, sC = ctl->sC;
    const int mPc = gd.mPc;
    double v[2] = {INFINITY, -INFINITY};
    auto elem = [&](int k) -> double { return (rval64 ? rval64[k] : 1.0) * (double)gd.x[gd.rcol[k]]; };
    auto epi = [&](int r, double acc) {
        if (r < mPc) v[1] = fmax(v[1], sP * acc);
        else v[0] = fmin(v[0], sC * acc);
    };
    for (int t = blockIdx.x; t < gd.nrtiles; t += gridDim.x) {
        const Tile tl = gd.rtiles[t];
        if (tl.lid < 0) seg_tile<double>(tl, gd.rptr, elem, epi, s_acc, s_ptr, s_tseg, s_tacc);
        else chunk_tile<double>(tl, elem, epi, s_tacc, (double *)gd.rlpart64, gd.rlfirst, gd.rlcount,
                                gd.rltick);
    }
    const Red red{0, 1, 1};
    block_combine<2>(v, red, 0, s_wave, s_rec);
    if (grid_reduce(s_rec, red, part, gpart, tick) && threadIdx.x == 0) {
        ctl->zmin = ctl->onesC ? ctl->sC * ctl->sumx : s_rec[0];
        ctl->ymax = ctl->onesP ? ctl->sP * ctl->sumx : s_rec[1];
    }
}

// Search pass over the stored rows: for each candidate step, the sums that
// give Psi and Phi (Section 4.1) plus min(z + a dz) (Algorithm 3 early return).
template <class T>
__global__ __launch_bounds__(BLOCK) void k_search(GenericDev<T> gd, Ctl *ctl, double *part,
                                                   double *gpart, unsigned *tick)
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
                else v[0] = fmin(v[0], yp);
            }
            const Red red{0, 1, 1};
            block_combine<2>(v, red, 0, s_wave, s_rec);
            if (grid_reduce(s_rec, red, part, gpart, tick) && threadIdx.x == 0)
                finish_search(ctl, s_rec);
        } else {
            const double pm = ctl->rfPm, zm = ctl->rfZmin;
            double v[2] = {0.0, 0.0};
            for (int r = r0; r < mR; r += stride) {
                const double yp = (double)gd.yz[r] + a * (double)gd.dyz[r];
                if (r < mPc) v[0] += exp(eta * yp - pm);
                else v[1] += exp(-eta * (yp - zm));
            }
            const Red red{2, 0, 0};
            block_combine<2>(v, red, 0, s_wave, s_rec);
            if (grid_reduce(s_rec, red, part, gpart, tick) && threadIdx.x == 0)
                finish_search(ctl, s_rec);
        }
        return;
    }
    const int nc = ctl->ncand;
    double cd[KC];
#pragma unroll
    for (int k = 0; k < KC; ++k) cd[k] = ctl->cand[k];
    const double gdel = ctl->gdelta;
    // ---- packing rows: s1P[k] = sum_i w_i expm1(eta a_k dy_i)
    {
        double s1[KC];
#pragma unroll
        for (int k = 0; k < KC; ++k) s1[k] = 0.0;
        for (int r = r0; r < mPc; r += stride) {
            const T w = gd.wu[r], dy = gd.dyz[r];
            if (!(w > T(0)) || !(dy > T(0))) continue;
            if (kind == SK_EXP) {
                T m = expm1_t((T)(eta * cd[0] * (double)dy));
#pragma unroll
                for (int k = 0; k < KC; ++k) {
                    s1[k] += (double)(w * m);
                    m = m * (m + T(2));                    // expm1(2x) = expm1(x)(expm1(x)+2)
                }
            } else if (kind == SK_GRID) {
                T m = expm1_t((T)(eta * cd[0] * (double)dy));
                const T mr = expm1_t((T)(eta * gdel * (double)dy));
#pragma unroll
                for (int k = 0; k < KC; ++k) {
                    s1[k] += (double)(w * m);
                    m = m + mr + m * mr;                   // expm1(x+y) from expm1(x), expm1(y)
                }
            } else {
                for (int k = 0; k < nc; ++k)
                    s1[k] += (double)(w * expm1_t((T)(eta * cd[k] * (double)dy)));
            }
        }
        const Red redp{KC, 0, 0};
        block_combine<KC>(s1, redp, 0, s_wave, s_rec);
    }
    // ---- covering rows: s1C[k] = sum_j u_j expm1(-b_jk), s2C[k] = sum_j u_j e^{-b_jk},
    //      zmin[k] = min_j z_j + a_k dz_j, with b_jk = eta a_k dz_j
    {
        double acc[3 * KC];
#pragma unroll
        for (int k = 0; k < KC; ++k) { acc[k] = 0.0; acc[KC + k] = 0.0; acc[2 * KC + k] = INFINITY; }
        for (int r = mPc + r0; r < mR; r += stride)
            cov_row_terms<T>(kind, nc, cd, gdel, eta, gd.wu[r], gd.yz[r], gd.dyz[r], acc);
        const Red redc{3 * KC, KC, 0};
        block_combine<3 * KC>(acc, redc, KC, s_wave, s_rec + KC);
    }
    const Red red{3 * KC, KC, 0};
    if (grid_reduce(s_rec, red, part, gpart, tick) && threadIdx.x == 0) finish_search(ctl, s_rec);
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

__global__ void k_potential_finish(const double *g, const double *h, int n, double scale,
                                   double *out, const Ctl *ctl, double *val)
{
    for (int i = blockIdx.x * BLOCK + threadIdx.x; i < n; i += gridDim.x * BLOCK)
        out[i] = scale * (g[i] - h[i]);
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

template <class T>
void generic_init(const GenericDev<T> &g, Ctl *ctl, const Launch &L, hipStream_t st, bool have_x0)
{
    hipLaunchKernelGGL(k_init_x<T>, dim3(L.grid_elem_cols), dim3(BLOCK), 0, st, g, ctl,
                       have_x0 ? 1 : 0, L.partials, L.gpart, L.tickets);
    hipLaunchKernelGGL((k_fwd<T, true>), dim3(L.grid_rtile), dim3(BLOCK), 0, st, g, ctl,
                       (const T *)g.x, g.yz, L.partials, L.gpart, L.tickets);
}

template <class T>
void generic_load_x(const GenericDev<T> &g, Ctl *ctl, const Launch &L, hipStream_t st,
                    const double *x_dev)
{
    hipLaunchKernelGGL(k_load_x<T>, dim3(L.grid_elem_cols), dim3(BLOCK), 0, st, g, ctl, x_dev,
                       L.partials, L.gpart, L.tickets);
    hipLaunchKernelGGL((k_fwd<T, true>), dim3(L.grid_rtile), dim3(BLOCK), 0, st, g, ctl,
                       (const T *)g.x, g.yz, L.partials, L.gpart, L.tickets);
}

template <class T>
void generic_stats(const GenericDev<T> &g, Ctl *ctl, const Launch &L, hipStream_t st,
                   const double *rval64)
{
    hipLaunchKernelGGL(k_init_x<T>, dim3(L.grid_elem_cols), dim3(BLOCK), 0, st, g, ctl, 1,
                       L.partials, L.gpart, L.tickets);
    hipLaunchKernelGGL(k_stats<T>, dim3(L.grid_rtile), dim3(BLOCK), 0, st, g, ctl, rval64,
                       L.partials, L.gpart, L.tickets);
}

template <class T>
void generic_row(const GenericDev<T> &g, Ctl *ctl, const Launch &L, hipStream_t st)
{
    hipLaunchKernelGGL(k_row<T>, dim3(L.grid_elem_rows), dim3(BLOCK), 0, st, g, ctl, L.partials,
                       L.gpart, L.tickets);
}

template <class T>
void generic_col(const GenericDev<T> &g, Ctl *ctl, const Launch &L, hipStream_t st)
{
    hipLaunchKernelGGL(k_col<T>, dim3(L.grid_ctile), dim3(BLOCK), 0, st, g, ctl, L.partials,
                       L.gpart, L.tickets);
}

template <class T>
void generic_fwd(const GenericDev<T> &g, Ctl *ctl, const Launch &L, hipStream_t st)
{
    hipLaunchKernelGGL((k_fwd<T, false>), dim3(L.grid_rtile), dim3(BLOCK), 0, st, g, ctl,
                       (const T *)g.d, g.dyz, L.partials, L.gpart, L.tickets);
}

template <class T>
void generic_search(const GenericDev<T> &g, Ctl *ctl, const Launch &L, hipStream_t st)
{
    hipLaunchKernelGGL(k_search<T>, dim3(L.grid_elem_rows), dim3(BLOCK), 0, st, g, ctl, L.partials,
                       L.gpart, L.tickets);
}

template <class T>
void generic_iteration(const GenericDev<T> &g, Ctl *ctl, const Launch &L, hipStream_t st)
{
    generic_row(g, ctl, L, st);
    generic_col(g, ctl, L, st);
    generic_fwd(g, ctl, L, st);
    generic_search(g, ctl, L, st);
    generic_search(g, ctl, L, st);
}

void potential_finish(const double *g_dbg, const double *h_dbg, int n, double scale, double *out,
                      const Ctl *ctl, double *val, hipStream_t st)
{
    hipLaunchKernelGGL(k_potential_finish, dim3(grid_for(n)), dim3(BLOCK), 0, st, g_dbg, h_dbg, n,
                       scale, out, ctl, val);
}

template <class T>
void widen(const T *src, double *dst, int64_t n, hipStream_t st)
{
    hipLaunchKernelGGL(k_widen<T>, dim3(grid_for(n)), dim3(BLOCK), 0, st, src, dst, n);
}

template <class T>
void narrow(const double *src, T *dst, int64_t n, hipStream_t st)
{
    hipLaunchKernelGGL(k_narrow<T>, dim3(grid_for(n)), dim3(BLOCK), 0, st, src, dst, n);
}

void set_phase(Ctl *ctl, int phase, hipStream_t st)
{
    hipLaunchKernelGGL(k_set_phase, dim3(1), dim3(1), 0, st, ctl, phase);
}

#define MWU_INSTANTIATE(T)                                                                      \
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
