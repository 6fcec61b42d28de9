// Fused densest-subgraph program (gfx950): the dual of Charikar's LP with D
// fixed (Section 3), W z >= 1, (1/D) O z <= 1, z >= 0, run through Algorithm 2
// with the step search of Algorithm 3 (Section 4).
//
// Variables are the edge ends (the caller's z_{2e} and z_{2e+1}; internally
// the first and second end of edge e in degree order, stored as two arrays).
// Every variable lies in exactly one packing row (its
// vertex) and one covering row (its edge), so the transpose products need no
// index structure: g_i = w_{v(i)} / (D sum w), h_i = u_{e(i)} / sum u.  The
// vertex rows are segmented sums over each vertex's variables (nnz-balanced
// tiles with LDS staging); the edge rows are pairs.
//
// The direction compares g_i with h_i.  In FP32 both weights of a variable
// whose edge is well covered and whose vertex is lightly loaded underflow, so
// the chosen form forms the ratio in the log domain from y_v and z_e:
// g_i / h_i = exp(eta (y_v - L_P) + eta (z_e - L_C) + ln(sP / sC)), with L_P and
// L_C the LSE totals of the current point, and q = 1 - g_i / h_i by an FP64
// expm1.  FP64 keeps the plain ratio of the stored weights, as the definition
// reads.  In both forms x, d, y, z, Pd, Cd, the weights as the row pass forms
// them and their LSE totals are FP64: with single-weight rows and steps up to
// ~1e5, a relative perturbation of 1e-7 in any of them (FP32 storage, an FP32
// expm1, totals summed from FP32-rounded weights) grows to 1e-5..1e-2 in the
// objective of a probe.  Only the stored weights that the step search reads
// and the search terms are T.
#include <algorithm>

#include "device_common.h"

namespace mwu {

#define DLAUNCH(kernel, grid, ...) hipLaunchKernelGGL(kernel, dim3(grid), dim3(BLOCK), 0, st, __VA_ARGS__)

// ------------------------------------------------------------------ init

template <class T>
__global__ __launch_bounds__(BLOCK) void dn_init_x(DnDev<T> dd, Ctl *ctl, int have_x0, const double *src,
                                                    double *part)
{
    __shared__ double s_wave[4];
    __shared__ double s_rec[QMAX];
    const double eps = ctl->eps, sP = ctl->sP;
    double v[1] = {0.0};
    for (int i = blockIdx.x * BLOCK + threadIdx.x; i < dd.n; i += gridDim.x * BLOCK) {
        double x;
        if (src) {
            x = src[dd.cpos[i]];   // caller order -> internal
            dd.x[i] = x;
        } else if (!have_x0) {
            x = eps / ((double)dd.n * sP);   // Algorithm 1: eps / (n max_j P_ji), P_ji = sP
            dd.x[i] = x;
        } else {
            x = dd.x[i];
        }
        dd.d[i] = 0.0;
        v[0] += x;
    }
    const Red red{1, 0, 0};
    block_combine<1>(v, red, 0, s_wave, s_rec);
    store_record(s_rec, 1, part);
}

__global__ __launch_bounds__(BLOCK) void dn_init_x_fin(Ctl *ctl, const double *part, int G)
{
    __shared__ double s_wave[4];
    __shared__ double s_rec[QMAX];
    const Red red{1, 0, 0};
    fold_records<1>(part, G, red, 0, s_wave, s_rec);
    if (threadIdx.x == 0) finish_sumx(ctl, s_rec[0]);
}

// ------------------------------------------------------------------ forward products

// Vertex rows: INIT y = sP O x (clears dy), else dy = sP O d.  Record [max].
template <class T, bool INIT>
__global__ __launch_bounds__(BLOCK) void dn_fwd_v(DnDev<T> dd, Ctl *ctl, double *part)
{
    __shared__ double s_acc[TILE_LDS];
    __shared__ int32_t s_ptr[TILE_NZ + 1];
    __shared__ double s_tacc[BLOCK / 64];
    __shared__ double s_wave[4];
    __shared__ double s_rec[QMAX];
    if (!INIT && ctl->phase != PH_FWD) return;
    const double *src = INIT ? dd.x : dd.d;
    const double sP = ctl->sP;
    double v[1] = {-INFINITY};
    auto elem = [&](int k) -> double { return src[dd.vvar[k]]; };
    auto epi = [&](int r, double acc) {
        acc = sP * acc;
        if (INIT) { dd.y[r] = acc; dd.dy[r] = 0.0; }
        else dd.dy[r] = acc;
        v[0] = fmax(v[0], acc);
    };
    for (int t = blockIdx.x; t < dd.nvtiles; t += gridDim.x) {
        const Tile tl = dd.vtiles[t];
        if (tl.lid < 0) seg_tile<double>(tl, dd.vptr, elem, epi, s_acc, s_ptr, nullptr, nullptr);
        else chunk_tile<double>(tl, elem, s_tacc, dd.lpart, dd.vlong.lfirst);
    }
    const Red red{0, 0, 1};
    block_combine<1>(v, red, 0, s_wave, s_rec);
    store_record(s_rec, 1, part);
}

// Long vertex rows (more variables than one tile) from the chunk partials of
// dn_fwd_v, one wave per long row, chunks summed lane-strided and folded in a
// fixed order; INIT also forms the edge rows z = sC (x_first + x_second) (clearing
// dz; in an iteration the column pass writes Cd).  Record [min z | max over
// the long rows] (INIT) or [max over the long rows].
template <class T, bool INIT>
__global__ __launch_bounds__(BLOCK) void dn_fwd_e(DnDev<T> dd, Ctl *ctl, double *part)
{
    __shared__ double s_wave[4 * 2];
    __shared__ double s_rec[QMAX];
    if (!INIT && ctl->phase != PH_FWD) return;
    const double sP = ctl->sP;
    double mn = INFINITY, mx = -INFINITY;
    if (INIT) {
        const double sC = ctl->sC;
        for (int e = blockIdx.x * BLOCK + threadIdx.x; e < dd.ne; e += gridDim.x * BLOCK) {
            const double val = sC * (dd.x[e] + dd.x[dd.ne + e]);
            dd.z[e] = val;
            dd.dz[e] = 0.0;
            mn = fmin(mn, val);
        }
    }
    const int lane = threadIdx.x & 63;
    const int nwaves = gridDim.x * (BLOCK / 64);
    for (int l = blockIdx.x * (BLOCK / 64) + (threadIdx.x >> 6); l < dd.vlong.nlong; l += nwaves) {
        const int f = dd.vlong.lfirst[l], c = dd.vlong.lcount[l];
        double acc = 0.0;
        for (int i = lane; i < c; i += 64) acc += dd.lpart[f + i];
#pragma unroll
        for (int m = 32; m > 0; m >>= 1) acc += __shfl_xor(acc, m);
        acc = sP * acc;
        if (lane == 0) {
            const int r = dd.vlong.lseg[l];
            if (INIT) { dd.y[r] = acc; dd.dy[r] = 0.0; }
            else dd.dy[r] = acc;
        }
        mx = fmax(mx, acc);
    }
    if (INIT) {
        double v[2] = {mn, mx};
        const Red red{0, 1, 1};
        block_combine<2>(v, red, 0, s_wave, s_rec);
        store_record(s_rec, 2, part);
    } else {
        double v[1] = {mx};
        const Red red{0, 0, 1};
        block_combine<1>(v, red, 0, s_wave, s_rec);
        store_record(s_rec, 1, part);
    }
}

template <class T, bool INIT>
__global__ __launch_bounds__(BLOCK) void dn_fwd_fin(DnDev<T> dd, Ctl *ctl, const double *pv, int Gv,
                                                     const double *pe, int Ge)
{
    __shared__ double s_wave[4 * 2];
    __shared__ double s_a[QMAX], s_b[QMAX];
    if (!INIT && ctl->phase != PH_FWD) return;
    const Red rmax{0, 0, 1};
    fold_records<1>(pv, Gv, rmax, 0, s_wave, s_a);
    if (INIT) {
        const Red rlast{0, 1, 1};
        fold_records<2>(pe, Ge, rlast, 0, s_wave, s_b);
    } else {
        fold_records<1>(pe, Ge, rmax, 0, s_wave, s_b);
    }
    on_ctl(ctl, [&](Ctl *c) {
        // [min over C rows | max over P rows]
        double rec[2] = {INIT ? s_b[0] : 0.0, fmax(s_a[0], INIT ? s_b[1] : s_b[0])};
        if (INIT) {
            finish_init_fwd(c, rec);
        } else if (!held(c)) {
            c->dymax = rec[1];
            begin_search(c, dd.forced);
        }
    });
}

// ------------------------------------------------------------------ row pass

// y += a dy, w = exp(eta (y - L_P)) over vertices; z += a dz, u = exp(-eta (z
// - L_C)) over edges.  Record [sum w | sum u | min z | max y].  The weights
// are formed and summed in FP64 in both forms (the LSE totals they give enter
// every log-domain ratio of the direction) and stored in T for the search.
template <class T>
__global__ __launch_bounds__(BLOCK) void dn_row(DnDev<T> dd, Ctl *ctl, double *part)
{
    __shared__ double s_wave[4 * 4];
    __shared__ double s_rec[QMAX];
    if (ctl->phase != PH_ROW) return;
    const double a = ctl->alpha;
    const double eta = ctl->eta, LP = ctl->LP, LC = ctl->LC;
    double v[4] = {0.0, 0.0, INFINITY, -INFINITY};
    const int stride = gridDim.x * BLOCK;
    for (int r = blockIdx.x * BLOCK + threadIdx.x; r < dd.nv; r += stride) {
        const double y = dd.y[r] + a * dd.dy[r];
        dd.y[r] = y;
        const double w = exp(eta * (y - LP));
        dd.w[r] = (T)w;
        v[0] += w;
        v[3] = fmax(v[3], y);
    }
    for (int e = blockIdx.x * BLOCK + threadIdx.x; e < dd.ne; e += stride) {
        const double z = dd.z[e] + a * dd.dz[e];
        dd.z[e] = z;
        const double u = row_met(ctl, z) ? 0.0 : exp(-eta * (z - LC));
        dd.u[e] = (T)u;
        v[1] += u;
        v[2] = fmin(v[2], z);
    }
    const Red red{2, 1, 1};
    block_combine<4>(v, red, 0, s_wave, s_rec);
    store_record(s_rec, 4, part);
}

__global__ __launch_bounds__(BLOCK) void dn_row_fin(Ctl *ctl, const double *part, int G)
{
    __shared__ double s_wave[4 * 4];
    __shared__ double s_rec[QMAX];
    if (ctl->phase != PH_ROW) return;
    const Red red{2, 1, 1};
    fold_records<4>(part, G, red, 0, s_wave, s_rec);
    on_ctl(ctl, [&](Ctl *c) { finish_row(c, s_rec); });
}

// ------------------------------------------------------------------ column pass

// Commit x += a d, then g, h and the direction of every variable, and the
// edge rows of the direction Cd = sC (d_first + d_second).  One thread per
// edge takes its two variables (coalesced in both halves of x and d).  Record
// [sum d | min g | max d | max h].  In PH_COMMIT only the commit.
template <class T>
__global__ __launch_bounds__(BLOCK) void dn_col(DnDev<T> dd, Ctl *ctl, double *part)
{
    __shared__ double s_wave[4 * 4];
    __shared__ double s_rec[QMAX];
    const int ph = ctl->phase;
    if (ph != PH_COL && ph != PH_COMMIT) return;
    const double a = ctl->alpha;
    const int stride = gridDim.x * BLOCK;
    const int ne = dd.ne;
    if (ph == PH_COMMIT) {
        for (int e = blockIdx.x * BLOCK + threadIdx.x; e < ne; e += stride) {
            dd.x[e] = dd.x[e] + a * dd.d[e];
            dd.x[ne + e] = dd.x[ne + e] + a * dd.d[ne + e];
        }
        return;
    }
    const double sP = ctl->sP, sC = ctl->sC, invSw = ctl->invSw, invSu = ctl->invSu;
    const double step = ctl->step, qmin = ctl->qmin, eta = ctl->eta, LP = ctl->LP, LC = ctl->LC;
    // after the row pass L_P and L_C are the exact LSE totals: the normalized
    // weights are exp(eta (y - L_P)) and exp(-eta (z - L_C))
    const double lnK = log(sP / sC);
    // g and h from the stored weights: the FP64 direction and the
    // certificates; the FP32 direction needs only y and z, and the densest
    // outer search uses no weak-duality bound, so FP32 skips them unless they
    // are being recorded
    const bool need_gh = sizeof(T) == 8 || dd.g_dbg != nullptr || dd.grad != nullptr;
    double v[4] = {0.0, INFINITY, -INFINITY, -INFINITY};
    for (int e = blockIdx.x * BLOCK + threadIdx.x; e < dd.ne; e += stride) {
        const int ru = dd.eu[e], rv = dd.ev[e];
        const double xs[2] = {dd.x[e] + a * dd.d[e], dd.x[ne + e] + a * dd.d[ne + e]};
        const double h = need_gh ? sC * (double)dd.u[e] * invSu : -INFINITY;
        const double ze = sizeof(T) == 4 ? dd.z[e] : 0.0;
        const bool met = sizeof(T) == 4 && row_met(ctl, ze);   // FP64: u = 0 gives h = 0
        double ds[2];
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const int r = k ? rv : ru;
            const double g = need_gh ? sP * (double)dd.w[r] * invSw : INFINITY;
            double q;
            if (sizeof(T) == 4) {
                // log-domain ratio: no underflow of the FP32 weights, and
                // q = 1 - g/h = -expm1(ln(g/h)) without cancellation near g = h
                const double lr = eta * (dd.y[r] - LP) + eta * (ze - LC) + lnK;
                q = met ? 0.0 : -expm1(fmin(lr, 80.0));
            } else {
                q = h > 0.0 ? 1.0 - g / h : 0.0;
            }
            const double di = q > qmin ? step * q * xs[k] : 0.0;
            ds[k] = di;
            v[0] += di;
            v[1] = fmin(v[1], g);
            v[2] = fmax(v[2], di);
            if (dd.g_dbg) { dd.g_dbg[k * ne + e] = g; dd.h_dbg[k * ne + e] = h; }
            if (dd.grad) dd.grad[dd.cpos[k * ne + e]] = dd.grad_scale * (g - h);   // caller order
        }
        v[3] = fmax(v[3], h);
        dd.x[e] = xs[0];
        dd.x[ne + e] = xs[1];
        dd.d[e] = ds[0];
        dd.d[ne + e] = ds[1];
        dd.dz[e] = sC * (ds[0] + ds[1]);
    }
    const Red red{1, 1, 2};
    block_combine<4>(v, red, 0, s_wave, s_rec);
    store_record(s_rec, 4, part);
}

__global__ __launch_bounds__(BLOCK) void dn_col_fin(Ctl *ctl, const double *part, int G)
{
    __shared__ double s_wave[4 * 4];
    __shared__ double s_rec[QMAX];
    const int ph = ctl->phase;
    if (ph != PH_COL && ph != PH_COMMIT) return;
    if (ph == PH_COMMIT) {
        if (threadIdx.x == 0 && !held(ctl)) { ctl->alpha = 0.0; ctl->phase = PH_DONE; }
        return;
    }
    const Red red{1, 1, 2};
    fold_records<4>(part, G, red, 0, s_wave, s_rec);
    on_ctl(ctl, [&](Ctl *c) { finish_col(c, s_rec); });
}

// ------------------------------------------------------------------ step search

template <class T, int KIND>
__device__ void dn_search_rows(const DnDev<T> &dd, const Ctl *ctl, double *s_wave, double *s_rec)
{
    const double eta = ctl->eta;
    const int stride = gridDim.x * BLOCK;
    const int r0 = blockIdx.x * BLOCK + threadIdx.x;
    const int nc = ctl->ncand;
    const double *cand = ctl->cand;
    const double a0 = ctl->cand[0], ga0 = ctl->ga0, gdel = ctl->gdelta, dymax = ctl->dymax;
    const uint32_t shm = shifted_mask(ctl);
    const bool deriv = ctl->skind == SK_NEWTON;
    {
        double s1[KC];
#pragma unroll
        for (int k = 0; k < KC; ++k) s1[k] = 0.0;
        // In FP32 storage the max-shifted packing terms are formed from y in
        // FP64 (lw = eta (y - L) for the L the stored w was formed with: the
        // row pass has since moved L by log(sum w) / eta).
        constexpr bool SH64 = sizeof(T) == 4;
        const double LP = ctl->LP, lsw = -log(ctl->invSw);
        for (int r = r0; r < dd.nv; r += stride) {
            const double dy64 = dd.dy[r];
            const double lw = SH64 && shm ? eta * (dd.y[r] - LP) + lsw : 0.0;
            pack_terms<T, KIND, SH64>(nc, cand, a0, ga0, gdel, eta, dd.w[r], (T)dy64, dymax, shm, s1, deriv, lw,
                                      dy64);
        }
        const Red redp{KC, 0, 0};
        block_combine<KC>(s1, redp, 0, s_wave, s_rec);
    }
    {
        CovAcc<T, double> ca;
        ca.init(pass_minima<KIND>());
        for (int e = r0; e < dd.ne; e += stride)
            cov_terms<T, KIND, double>(nc, cand, a0, ga0, gdel, eta, dd.u[e], dd.z[e], (T)dd.dz[e], ca.acc,
                                       ca.zmn, deriv);
        ca.combine(s_wave, s_rec + KC);
    }
}

template <class T>
__global__ __launch_bounds__(BLOCK) void dn_search(DnDev<T> dd, Ctl *ctl, double *part)
{
    __shared__ double s_wave[4 * 3 * KC];
    __shared__ double s_rec[QMAX];
    if (ctl->phase != PH_SEARCH) return;
    const int kind = ctl->skind;
    if (kind == SK_REFINE) {
        const double a = ctl->ref_alpha, eta = ctl->eta;
        const int stride = gridDim.x * BLOCK;
        const int r0 = blockIdx.x * BLOCK + threadIdx.x;
        if (ctl->ref_valid == 0) {   // [min z' | max eta y']
            double v[2] = {INFINITY, -INFINITY};
            for (int r = r0; r < dd.nv; r += stride) v[1] = fmax(v[1], eta * (dd.y[r] + a * dd.dy[r]));
            for (int e = r0; e < dd.ne; e += stride)
                if (!row_met(ctl, dd.z[e])) v[0] = fmin(v[0], dd.z[e] + a * dd.dz[e]);
            const Red red{0, 1, 1};
            block_combine<2>(v, red, 0, s_wave, s_rec);
            store_record_qmajor(s_rec, 2, part);
        } else {                     // [sum over packing rows | over covering rows | their derivative sums]
            const double pm = ctl->rfPm, zm = ctl->rfZmin;
            double v[4] = {0.0, 0.0, 0.0, 0.0};
            for (int r = r0; r < dd.nv; r += stride) {
                const double t = exp(eta * (dd.y[r] + a * dd.dy[r]) - pm);
                v[0] += t;
                v[2] += dd.dy[r] * t;
            }
            for (int e = r0; e < dd.ne; e += stride) {
                if (row_met(ctl, dd.z[e])) continue;
                const double t = exp(-eta * ((dd.z[e] + a * dd.dz[e]) - zm));
                v[1] += t;
                v[3] += dd.dz[e] * t;
            }
            const Red red{4, 0, 0};
            block_combine<4>(v, red, 0, s_wave, s_rec);
            store_record_qmajor(s_rec, 4, part);
        }
        return;
    }
    switch (kind) {
    case SK_EXP: dn_search_rows<T, SK_EXP>(dd, ctl, s_wave, s_rec); break;
    case SK_GRID: dn_search_rows<T, SK_GRID>(dd, ctl, s_wave, s_rec); break;
    case SK_COMBO: dn_search_rows<T, SK_COMBO>(dd, ctl, s_wave, s_rec); break;
    default: dn_search_rows<T, SK_LIST>(dd, ctl, s_wave, s_rec); break;
    }
    store_record_qmajor(s_rec, 4 * KC, part);
}

__global__ __launch_bounds__(BLOCK) void dn_search_fin(Ctl *ctl, const double *part, int G)
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

// ------------------------------------------------------------------ FP64 statistics

template <class T>
__global__ __launch_bounds__(BLOCK) void dn_stats_v(DnDev<T> dd, double *part)
{
    __shared__ double s_acc[TILE_LDS];
    __shared__ int32_t s_ptr[TILE_NZ + 1];
    __shared__ double s_tacc[BLOCK / 64];
    __shared__ double s_wave[4];
    __shared__ double s_rec[QMAX];
    double v[1] = {-INFINITY};
    auto elem = [&](int k) -> double { return dd.x[dd.vvar[k]]; };
    auto epi = [&](int, double acc) { v[0] = fmax(v[0], acc); };
    for (int t = blockIdx.x; t < dd.nvtiles; t += gridDim.x) {
        const Tile tl = dd.vtiles[t];
        if (tl.lid < 0) seg_tile<double>(tl, dd.vptr, elem, epi, s_acc, s_ptr, nullptr, nullptr);
        else chunk_tile<double>(tl, elem, s_tacc, dd.lpart64, dd.vlong.lfirst);
    }
    const Red red{0, 0, 1};
    block_combine<1>(v, red, 0, s_wave, s_rec);
    store_record(s_rec, 1, part);
}

template <class T>
__global__ __launch_bounds__(BLOCK) void dn_stats_e(DnDev<T> dd, double *part)
{
    __shared__ double s_wave[4];
    __shared__ double s_rec[QMAX];
    double v[1] = {INFINITY};
    for (int e = blockIdx.x * BLOCK + threadIdx.x; e < dd.ne; e += gridDim.x * BLOCK)
        v[0] = fmin(v[0], dd.x[e] + dd.x[dd.ne + e]);
    const Red red{0, 1, 0};
    block_combine<1>(v, red, 0, s_wave, s_rec);
    store_record(s_rec, 1, part);
}

template <class T>
__global__ __launch_bounds__(BLOCK) void dn_stats_fin(DnDev<T> dd, Ctl *ctl, const double *pv, int Gv,
                                                       const double *pe, int Ge)
{
    __shared__ double s_wave[4];
    __shared__ double s_a[QMAX], s_b[QMAX], s_l[QMAX];
    double lv[1] = {-INFINITY};
    for (int l = threadIdx.x; l < dd.vlong.nlong; l += BLOCK)
        lv[0] = fmax(lv[0], long_sum<double>(l, dd.lpart64, dd.vlong.lfirst, dd.vlong.lcount));
    const Red rmax{0, 0, 1}, rmin{0, 1, 0};
    block_combine<1>(lv, rmax, 0, s_wave, s_l);
    fold_records<1>(pv, Gv, rmax, 0, s_wave, s_a);
    fold_records<1>(pe, Ge, rmin, 0, s_wave, s_b);
    if (threadIdx.x == 0) {
        ctl->ymax = ctl->sP * fmax(s_a[0], s_l[0]);
        ctl->zmin = ctl->sC * s_b[0];
    }
}

// ------------------------------------------------------------------ level sets

// For the level-set rounding of the outer search: back[v] = number of
// neighbours of v ranked before v (rank by descending load).  The edges of the
// top-k vertices are then the prefix sums of back in rank order.  One wave per
// vertex, no atomics.
template <class T>
__global__ __launch_bounds__(BLOCK) void dn_backcount(DnDev<T> dd, const int32_t *rank, int32_t *back)
{
    const int lane = threadIdx.x & 63;
    const int wave = (blockIdx.x * BLOCK + threadIdx.x) >> 6;
    const int nwaves = (gridDim.x * BLOCK) >> 6;
    for (int v = wave; v < dd.nv; v += nwaves) {
        const int rv = rank[v];
        int c = 0;
        for (int q = dd.vptr[v] + lane; q < dd.vptr[v + 1]; q += 64) {
            const int var = dd.vvar[q];
            const bool second = var >= dd.ne;
            const int e = second ? var - dd.ne : var;
            const int w = second ? dd.eu[e] : dd.ev[e];   // the other end of the edge
            c += rank[w] < rv;
        }
#pragma unroll
        for (int m = 32; m > 0; m >>= 1) c += __shfl_xor(c, m);
        if (lane == 0) back[v] = c;
    }
}

template <class T>
void dn_backcounts(const DnDev<T> &dd, const int32_t *rank, int32_t *back, hipStream_t st)
{
    const int grid = std::max(1, std::min(GRID_MAX * 4, (dd.nv + 3) / 4));
    DLAUNCH(dn_backcount<T>, grid, dd, rank, back);
}

// Internal variables -> the caller's order: dst[cpos[p]] = src[p] (a
// permutation: every destination written once).
__global__ __launch_bounds__(BLOCK) void dn_to_caller_k(const double *src, const int32_t *cpos, double *dst, int n)
{
    for (int p = blockIdx.x * BLOCK + threadIdx.x; p < n; p += gridDim.x * BLOCK) dst[cpos[p]] = src[p];
}

void dn_to_caller(const double *src, const int32_t *cpos, double *dst, int64_t n, hipStream_t st)
{
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>((n + BLOCK - 1) / BLOCK, 4 * GRID_MAX));
    DLAUNCH(dn_to_caller_k, grid, src, cpos, dst, (int)n);
}

// ------------------------------------------------------------------ launchers

template <class T>
void dn_init(const DnDev<T> &dd, Ctl *ctl, const DnLaunch &L, hipStream_t st, bool have_x0, const double *src)
{
    DLAUNCH(dn_init_x<T>, L.grid_n, dd, ctl, have_x0 ? 1 : 0, src, L.partials);
    DLAUNCH(dn_init_x_fin, 1, ctl, (const double *)L.partials, L.grid_n);
    DLAUNCH((dn_fwd_v<T, true>), L.grid_vt, dd, ctl, L.partials);
    DLAUNCH((dn_fwd_e<T, true>), L.grid_e, dd, ctl, L.partials2);
    DLAUNCH((dn_fwd_fin<T, true>), 1, dd, ctl, (const double *)L.partials, L.grid_vt,
            (const double *)L.partials2, L.grid_e);
}

template <class T>
void dn_row_pass(const DnDev<T> &dd, Ctl *ctl, const DnLaunch &L, hipStream_t st)
{
    DLAUNCH(dn_row<T>, L.grid_r, dd, ctl, L.partials);
    DLAUNCH(dn_row_fin, 1, ctl, (const double *)L.partials, L.grid_r);
}

template <class T>
void dn_col_pass(const DnDev<T> &dd, Ctl *ctl, const DnLaunch &L, hipStream_t st)
{
    DLAUNCH(dn_col<T>, L.grid_n, dd, ctl, L.partials);
    DLAUNCH(dn_col_fin, 1, ctl, (const double *)L.partials, L.grid_n);
}

template <class T>
void dn_fwd_pass(const DnDev<T> &dd, Ctl *ctl, const DnLaunch &L, hipStream_t st)
{
    DLAUNCH((dn_fwd_v<T, false>), L.grid_vt, dd, ctl, L.partials);
    DLAUNCH((dn_fwd_e<T, false>), L.grid_e, dd, ctl, L.partials2);
    DLAUNCH((dn_fwd_fin<T, false>), 1, dd, ctl, (const double *)L.partials, L.grid_vt,
            (const double *)L.partials2, L.grid_e);
}

template <class T>
void dn_search_pass(const DnDev<T> &dd, Ctl *ctl, const DnLaunch &L, hipStream_t st)
{
    DLAUNCH(dn_search<T>, L.grid_s, dd, ctl, L.partials);
    DLAUNCH(dn_search_fin, 1, ctl, (const double *)L.partials, L.grid_s);
}

// One iteration slot with a single search launch: most iterations finish
// their step search in the combined first pass; one that needs more passes
// takes them in the following slots, whose other passes see the search phase
// and return at once.
template <class T>
void dn_iteration(const DnDev<T> &dd, Ctl *ctl, const DnLaunch &L, hipStream_t st)
{
    dn_row_pass<T>(dd, ctl, L, st);
    dn_col_pass<T>(dd, ctl, L, st);
    dn_fwd_pass<T>(dd, ctl, L, st);
    dn_search_pass<T>(dd, ctl, L, st);
}

template <class T>
void dn_stats(const DnDev<T> &dd, Ctl *ctl, const DnLaunch &L, hipStream_t st)
{
    DLAUNCH(dn_init_x<T>, L.grid_n, dd, ctl, 1, (const double *)nullptr, L.partials);
    DLAUNCH(dn_init_x_fin, 1, ctl, (const double *)L.partials, L.grid_n);
    DLAUNCH(dn_stats_v<T>, L.grid_vt, dd, L.partials);
    DLAUNCH(dn_stats_e<T>, L.grid_e, dd, L.partials2);
    DLAUNCH(dn_stats_fin<T>, 1, dd, ctl, (const double *)L.partials, L.grid_vt, (const double *)L.partials2,
            L.grid_e);
}

template <class T>
void dn_main(const DnDev<T> &dd, Ctl *ctl, const DnLaunch &L, hipStream_t st, int which)
{
    switch (which) {
    case 0: DLAUNCH(dn_row<T>, L.grid_r, dd, ctl, L.partials); break;
    case 1: DLAUNCH(dn_col<T>, L.grid_n, dd, ctl, L.partials); break;
    case 2: DLAUNCH((dn_fwd_v<T, false>), L.grid_vt, dd, ctl, L.partials); break;
    default: DLAUNCH(dn_search<T>, L.grid_s, dd, ctl, L.partials); break;
    }
}

template <class T>
void dn_occupancy(int *per_cu_vt, int *per_cu_search)
{
    int a = 0, b = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&a, dn_fwd_v<T, false>, BLOCK, 0) != hipSuccess) a = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, dn_search<T>, BLOCK, 0) != hipSuccess) b = 0;
    *per_cu_vt = a > 0 ? a : 1;
    *per_cu_search = b > 0 ? b : 1;
}

#define MWU_DN_INSTANTIATE(T)                                                                          \
    template void dn_init<T>(const DnDev<T> &, Ctl *, const DnLaunch &, hipStream_t, bool, const double *); \
    template void dn_row_pass<T>(const DnDev<T> &, Ctl *, const DnLaunch &, hipStream_t);              \
    template void dn_col_pass<T>(const DnDev<T> &, Ctl *, const DnLaunch &, hipStream_t);              \
    template void dn_fwd_pass<T>(const DnDev<T> &, Ctl *, const DnLaunch &, hipStream_t);              \
    template void dn_search_pass<T>(const DnDev<T> &, Ctl *, const DnLaunch &, hipStream_t);           \
    template void dn_iteration<T>(const DnDev<T> &, Ctl *, const DnLaunch &, hipStream_t);             \
    template void dn_stats<T>(const DnDev<T> &, Ctl *, const DnLaunch &, hipStream_t);                 \
    template void dn_main<T>(const DnDev<T> &, Ctl *, const DnLaunch &, hipStream_t, int);             \
    template void dn_occupancy<T>(int *, int *);                                                      \
    template void dn_backcounts<T>(const DnDev<T> &, const int32_t *, int32_t *, hipStream_t);

MWU_DN_INSTANTIATE(float)
MWU_DN_INSTANTIATE(double)

}  // namespace mwu
