// Fused vertex-cover program (gfx950): min 1^T x s.t. M^T x >= 1 (Section 3),
// run as the mixed problem with the objective row (1/M) 1^T x <= 1 (end of
// Section 2.2) and Algorithm 2 / Algorithm 3 (Section 4).
//
// The covering rows are the edges: z_e = x_u + x_v, dz_e = d_u + d_v and the
// weights u_e = exp(-eta (z_e - L)) are recomputed from the vertex vectors in
// every pass instead of being stored, so a pass reads only the adjacency
// indices from HBM (the vertex vectors stay in the caches).  Per iteration:
//   commit  (vertices) x += a d for the step accepted last;
//   pass A  (full adjacency, one segment per vertex) h_v = sum_{w ~ v} u_vw,
//           min z, sum u: the transpose product C^T u fused with the weights
//           and the LSE totals;
//   pass B  (vertices) direction d_v = (1/eta) max(0, 1 - g/h_v) x_v with
//           g = 1/M, sum d (= M * Pd);
//   search  (edge list, one visit per edge) the K-candidate sums of Phi,
//           with the forward product C d formed on the fly.
#include <algorithm>

#include "device_common.h"

#define HIP_CHECK_OCC(call) do { if ((call) != hipSuccess) { a = b = 0; } } while (0)

namespace mwu {

// Multi-segment tile where each term depends on its segment: stage(k) and
// the segment values segval(s) are staged through LDS with coalesced loads
// (all gathers of the tile in flight at once), then each thread walks ITEMS
// consecutive nonzeros, accumulating term(segment value, staged value), and
// epi(seg, sum) is called once per segment.  Segments crossing thread
// boundaries are completed through seg_carry.
static_assert(TILE_NZ <= 32767, "tile row starts are staged in 16 bits");

template <class S, class Acc, class StageF, class SegF, class TermF, class EpiF>
MWU_DEV void seg_tile_rows(const Tile &tl, const int32_t *__restrict__ ptr, StageF &stage, SegF &segval,
                           TermF &term, EpiF &epi, S *s_val, S *s_seg, int16_t *s_ptr)
{
    const int tid = threadIdx.x;
    const int S_ = tl.s1 - tl.s0;
    const int base = tl.k0;
    const int N = tl.k1 - tl.k0;
    for (int i = tid; i < S_; i += BLOCK) s_ptr[i] = (int16_t)(ptr[tl.s0 + i] - base);
    if (tid == 0) s_ptr[S_] = (int16_t)N;   // = ptr[s1] - base in a full layout; packed tiles end early
    for (int i = tid; i < S_; i += BLOCK) s_seg[i] = segval(tl.s0 + i);
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
        const int k = j * BLOCK + tid;
        if (k < N) s_val[pad_idx(k)] = stage(base + k);
    }
    __syncthreads();
    const int a = tid * ITEMS;
    const int b = min(a + ITEMS, N);
    int pend = -1, tseg = -1;
    Acc pacc = acc_zero<Acc>(), tacc = acc_zero<Acc>();
    if (a < N) {
        int lo = 0, hi = S_;   // s_ptr[lo] <= a < s_ptr[hi]
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (s_ptr[mid] <= a) lo = mid; else hi = mid;
        }
        int s = lo;
        bool started = (s_ptr[s] == a);
        int end = s_ptr[s + 1];
        S sv = s_seg[s];
        Acc acc = acc_zero<Acc>();
        for (int k = a; k < b; ++k) {
            if (k >= end) {
                if (started) epi(tl.s0 + s, acc);
                else { pend = s; pacc = acc; }
                do { ++s; end = s_ptr[s + 1]; } while (k >= end);   // empty segments: separate pass
                started = true;
                acc = acc_zero<Acc>();
                sv = s_seg[s];
            }
            acc += term(sv, s_val[pad_idx(k)]);
        }
        if (end <= b) {
            if (started) epi(tl.s0 + s, acc);
            else { pend = s; pacc = acc; }
        } else {
            tseg = s;
            tacc = acc;
        }
    }
    Acc tot = seg_carry<Acc>(tseg, tacc, pend);
    if (pend >= 0) {
        tot += pacc;
        epi(tl.s0 + pend, tot);
    }
    for (int s = tid; s < S_; s += BLOCK)
        if (s_ptr[s] == s_ptr[s + 1]) epi(tl.s0 + s, acc_zero<Acc>());
    __syncthreads();
}

// Visit every edge of the list (eu, ew, ne) once: visit(x_d of u, x_d of w,
// e).  Grid-stride over the list, U edges per step so that their gathers are
// in flight together (fewer in FP64, where the search accumulators take twice
// the registers).
template <class T, class VisitF>
MWU_DEV void for_edge_list(const VcDev<T> &vd, const int32_t *__restrict__ eu, const int32_t *__restrict__ ew,
                           int ne, VisitF &visit)
{
    constexpr int U = sizeof(T) == 4 ? 3 : 2;
    const int stride = gridDim.x * BLOCK;
    int e = blockIdx.x * BLOCK + threadIdx.x;
    for (; e + (U - 1) * stride < ne; e += U * stride) {
        int iu[U], iw[U];
#pragma unroll
        for (int j = 0; j < U; ++j) { iu[j] = eu[e + j * stride]; iw[j] = ew[e + j * stride]; }
        XD<T> pu[U], pw[U];
#pragma unroll
        for (int j = 0; j < U; ++j) { pu[j] = vd.xd[iu[j]]; pw[j] = vd.xd[iw[j]]; }
#pragma unroll
        for (int j = 0; j < U; ++j) visit(pu[j], pw[j], e + j * stride);
    }
    for (; e < ne; e += stride) visit(vd.xd[eu[e]], vd.xd[ew[e]], e);
}

// Every edge of the graph.
template <class T, class VisitF>
MWU_DEV void for_edges(const VcDev<T> &vd, VisitF &visit)
{
    for_edge_list<T>(vd, vd.eu, vd.ew, vd.ne, visit);
}

// ------------------------------------------------------------------ finishers

MWU_DEV void finish_vc_start(Ctl *c, const double *rec)
{
    // rec: [- | min z]
    c->zmin = rec[1];
    c->ymax = c->y1;
    c->LP = c->y1;
    c->LC = c->zmin;        // first shift; pass A makes it the exact smin
    c->alpha = 0.0;
    c->status = ST_RUNNING;
    c->phase = PH_ROW;
}

MWU_DEV void finish_vcA(Ctl *c, const double *rec)
{
    // rec: [sum_v h_v (= 2 sum_e u_e) | min z]
    if (held(c)) return;
    const double a = c->alpha;
    c->y1 += a * c->dy1;
    c->LP = c->y1;
    c->ymax = c->y1;
    c->invSw = 1.0;
    const double su = 0.5 * rec[0];
    c->zmin = rec[1];
    // every edge met and left out (dropped rows): no weights, the probe ends
    const bool all_met = c->drop && c->zmin >= 1.0;
    const bool bad = !all_met && (!(su > 0.0) || !isfinite(su));
    c->LCw = c->LC;
    if (!all_met) {
        c->LC = c->LCw - log(su) / c->eta;
        c->invSu = 1.0 / su;
    }
    if (c->eval_mode) { c->phase = PH_COL; return; }
    if (bad) { c->status = ST_NUMERIC; c->phase = PH_COMMIT; return; }
    if (c->zmin >= 1.0) { c->status = ST_FEASIBLE; c->phase = PH_COMMIT; }
    else if (c->iter >= c->max_iter) { c->status = ST_MAX_ITER; c->phase = PH_COMMIT; }
    else c->phase = PH_COL;
}

MWU_DEV void finish_vcB(Ctl *c, const double *rec, const double *forced)
{
    // rec: [sum d | max d | max h]
    if (held(c)) return;
    c->alpha = 0.0;
    c->dsum = rec[0];
    c->dmax = rec[1];
    c->hmax = rec[2];
    c->gmin = c->sP;
    const double cf = 1.0 - c->qmin;   // margin for the rounding of h
    if (c->hmax > 0.0 && cf / c->hmax > c->cover_bound) c->cover_bound = cf / c->hmax;
    if (1.0 / c->sP < c->pack_bound) c->pack_bound = 1.0 / c->sP;
    c->dy1 = c->sP * c->dsum;
    c->dz1 = 0.0;
    c->dymax = 0.0;
    if (!c->eval_mode && !(c->dmax > 0.0)) { c->status = ST_INFEASIBLE; c->phase = PH_DONE; return; }
    begin_search(c, forced);
}

// ------------------------------------------------------------------ kernels

template <class T>
__global__ __launch_bounds__(BLOCK) void vc_init_x(VcDev<T> vd, Ctl *ctl, int have_x0, double *part)
{
    __shared__ double s_wave[4];
    __shared__ double s_rec[QMAX];
    const double eps = ctl->eps, sP = ctl->sP;
    double v[1] = {0.0};
    for (int i = blockIdx.x * BLOCK + threadIdx.x; i < vd.nv; i += gridDim.x * BLOCK) {
        XD<T> p = vd.xd[i];
        if (!have_x0) p.x = (T)(eps / ((double)vd.nv * sP));   // Algorithm 1 with P = (1/M) 1^T
        p.d = T(0);
        vd.xd[i] = p;
        vd.xs[i] = p.x;
        v[0] += (double)p.x;
    }
    const Red red{1, 0, 0};
    block_combine<1>(v, red, 0, s_wave, s_rec);
    store_record(s_rec, 1, part);
}

__global__ __launch_bounds__(BLOCK) void vc_init_x_fin(Ctl *ctl, const double *part, int G)
{
    __shared__ double s_wave[4];
    __shared__ double s_rec[QMAX];
    const Red red{1, 0, 0};
    fold_records<1>(part, G, red, 0, s_wave, s_rec);
    if (threadIdx.x == 0) {
        ctl->sumx = s_rec[0];
        ctl->y1 = ctl->sP * s_rec[0];
        ctl->dy1 = 0.0;
    }
}

// min over edges of x_u + x_w in FP64: the first LSE shift of a probe, and the
// min(Cx) certificate of the outer search.
template <class T>
__global__ __launch_bounds__(BLOCK) void vc_minz(VcDev<T> vd, Ctl *ctl, double *part)
{
    __shared__ double s_wave[4];
    __shared__ double s_rec[QMAX];
    double v[1] = {INFINITY};
    auto visit = [&](XD<T> pu, XD<T> pw, int) { v[0] = fmin(v[0], (double)pu.x + (double)pw.x); };
    for_edges<T>(vd, visit);
    const Red red{0, 1, 0};
    block_combine<1>(v, red, 0, s_wave, s_rec);
    store_record(s_rec, 1, part);
}

__global__ __launch_bounds__(BLOCK) void vc_minz_fin(Ctl *ctl, const double *part, int G)
{
    __shared__ double s_wave[4];
    __shared__ double s_rec[QMAX];
    const Red red{0, 1, 0};
    fold_records<1>(part, G, red, 0, s_wave, s_rec);
    if (threadIdx.x == 0) {
        double r[2] = {0.0, s_rec[0]};
        finish_vc_start(ctl, r);
    }
}

// x += a d for the step accepted by the last search (a no-op outside PH_ROW).
template <class T>
__global__ __launch_bounds__(BLOCK) void vc_commit_k(VcDev<T> vd, Ctl *ctl)
{
    if (ctl->phase != PH_ROW) return;
    const T a = (T)ctl->alpha;
    for (int i = blockIdx.x * BLOCK + threadIdx.x; i < vd.nv; i += gridDim.x * BLOCK) {
        XD<T> p = vd.xd[i];
        p.x = p.x + a * p.d;
        vd.xd[i] = p;
        vd.xs[i] = p.x;
    }
}

template <class T>
__global__ __launch_bounds__(BLOCK) void vc_passA_k(VcDev<T> vd, Ctl *ctl, double *part)
{
    __shared__ T s_val[TILE_LDS];
    __shared__ T s_seg[TILE_NZ];
    // row starts within the tile (at most TILE_NZ) in 16 bits: with them the
    // pass fits 7 workgroups per CU instead of 6
    __shared__ int16_t s_ptr[TILE_NZ + 1];
    __shared__ T s_tacc[BLOCK / 64];
    __shared__ double s_wave[4 * 2];
    __shared__ double s_rec[QMAX];
    if (ctl->phase != PH_ROW) return;
    const double eta = ctl->eta, Lw = ctl->LC;
    double v[2] = {0.0, INFINITY};   // sum h | min z
    // Sparse: the active neighbours concatenated over all tiles (ccol, cst),
    // visited by work items that merge runs of tiles; left-out neighbours
    // have negligible weight (skip_exponent) and never hold the minimum, which
    // an active row always does (eta (min z - Lw) stays below ln m).
    const bool sparse = act_rows_valid(ctl, Lw);
    const int32_t *__restrict__ fc = sparse ? vd.ccol : vd.fcol;
    const int32_t *__restrict__ fp = sparse ? vd.cst : vd.fptr;
    const Tile *__restrict__ tiles = sparse ? vd.items : vd.ftiles;
    const int ntiles = sparse ? ctl->act_nitems : vd.nftiles;
    auto stage = [&](int k) -> T { return vd.xs[fc[k]]; };
    auto segval = [&](int u) -> T { return vd.xs[u]; };
    auto term = [&](T xu, T xw) -> T {
        const double z = (double)xu + (double)xw;
        v[1] = fmin(v[1], z);
        return row_met(ctl, z) ? T(0) : exp_arg(-eta * (z - Lw), T(0));
    };
    auto epi = [&](int u, T acc) {
        vd.h[u] = acc;
        v[0] += (double)acc;
    };
    for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const Tile tl = tiles[t];
        if (tl.lid < 0) {
            seg_tile_rows<T, T>(tl, fp, stage, segval, term, epi, s_val, s_seg, s_ptr);
        } else {
            const T xu = segval(tl.s0);
            auto elem = [&](int k) -> T { return term(xu, stage(k)); };
            const T tot = chunk_tile<T>(tl, elem, s_tacc, vd.flpart, vd.flong.lfirst);
            v[0] += (double)tot;   // nonzero in thread 0 only
        }
    }
    const Red red{1, 1, 0};
    block_combine<2>(v, red, 0, s_wave, s_rec);
    store_record(s_rec, 2, part);
}

// with_long: the finisher also completes the long rows (when they are few;
// more of them pass B completes).
template <class T>
__global__ __launch_bounds__(BLOCK) void vc_passA_fin(VcDev<T> vd, Ctl *ctl, const double *part, int G,
                                                      int with_long)
{
    __shared__ double s_wave[4 * 2];
    __shared__ double s_rec[QMAX];
    __shared__ uint64_t s_ctl[CTL_WORDS];
    Ctl *c = ctl_stage(ctl, s_ctl);
    if (c->phase != PH_ROW) return;
    if (with_long)
        for (int l = threadIdx.x; l < vd.flong.nlong; l += BLOCK)
            vd.h[vd.flong.lseg[l]] = long_sum<T>(l, vd.flpart, vd.flong.lfirst, vd.flong.lcount);
    const Red red{1, 1, 0};
    fold_records<2>(part, G, red, 0, s_wave, s_rec);
    if (threadIdx.x == 0) finish_vcA(c, s_rec);
    ctl_write_back(ctl, s_ctl);
}

template <class T>
__global__ __launch_bounds__(BLOCK) void vc_passB_k(VcDev<T> vd, Ctl *ctl, double *part)
{
    __shared__ double s_wave[4 * 3];
    __shared__ double s_rec[QMAX];
    const int ph = ctl->phase;
    if (ph != PH_COL && ph != PH_COMMIT) return;
    if (ph == PH_COMMIT) return;   // x was committed before pass A
    const double invSu = ctl->invSu, g = ctl->sP, step = ctl->step, qmin = ctl->qmin;
    double v[3] = {0.0, -INFINITY, -INFINITY};   // sum d | max d | max h
    for (int i = blockIdx.x * BLOCK + threadIdx.x; i < vd.nv; i += gridDim.x * BLOCK) {
        XD<T> p = vd.xd[i];
        T hr;
        if (i < vd.nlong_b) {   // a long row (vertex i is long row i): its chunk partials, in order
            hr = long_sum<T>(i, vd.flpart, vd.flong.lfirst, vd.flong.lcount);
            vd.h[i] = hr;
        } else {
            hr = vd.h[i];
        }
        const double h = (double)hr * invSu;
        double di = 0.0;
        if (h > 0.0) {
            const double q = 1.0 - g / h;
            if (q > qmin) di = step * q * (double)p.x;
        }
        p.d = (T)di;
        v[0] += (double)p.d;
        v[1] = fmax(v[1], (double)p.d);
        v[2] = fmax(v[2], h);
        if (vd.h_dbg) vd.h_dbg[i] = h;
        vd.xd[i] = p;
    }
    const Red red{1, 0, 2};
    block_combine<3>(v, red, 0, s_wave, s_rec);
    store_record(s_rec, 3, part);
}

template <class T>
__global__ __launch_bounds__(BLOCK) void vc_passB_fin(VcDev<T> vd, Ctl *ctl, const double *part, int G)
{
    __shared__ double s_wave[4 * 3];
    __shared__ double s_rec[QMAX];
    __shared__ uint64_t s_ctl[CTL_WORDS];
    Ctl *c = ctl_stage(ctl, s_ctl);
    const int ph = c->phase;
    if (ph != PH_COL && ph != PH_COMMIT) return;
    if (ph == PH_COMMIT) {
        if (threadIdx.x == 0 && !held(c)) { c->alpha = 0.0; c->phase = PH_DONE; }
        ctl_write_back(ctl, s_ctl);
        return;
    }
    const Red red{1, 0, 2};
    fold_records<3>(part, G, red, 0, s_wave, s_rec);
    if (threadIdx.x == 0) finish_vcB(c, s_rec, vd.forced);
    ctl_write_back(ctl, s_ctl);
}

// K-candidate covering sums of one search pass over the edge list (KIND fixed
// per launch): [s1C | s2C | zmin] in s_rec.
template <class T, int KIND>
__device__ void vc_search_edges(const VcDev<T> &vd, const Ctl *ctl, double *s_wave, double *s_rec)
{
    const int nc = ctl->ncand;
    const double *cand = ctl->cand;
    const double eta = ctl->eta, a0 = ctl->cand[0], ga0 = ctl->ga0;
    const double gdel = ctl->gdelta, Lw = ctl->LCw;
    const bool deriv = ctl->skind == SK_NEWTON;
    CovAcc<T> ca;
    ca.init(pass_minima<KIND>());
    auto visit = [&](XD<T> pu, XD<T> pw, int) {
        const double zd = (double)pu.x + (double)pw.x;
        const T z = (T)zd;
        const T dz = pu.d + pw.d;
        const T u = row_met(ctl, zd) ? T(0) : exp_arg(-eta * (zd - Lw), T(0));
        cov_terms<T, KIND>(nc, cand, a0, ga0, gdel, eta, u, z, dz, ca.acc, ca.zmn, deriv);
    };
    if (act_valid(ctl, Lw)) for_edge_list<T>(vd, vd.aeu, vd.aew, ctl->act_ne, visit);
    else for_edges<T>(vd, visit);
    ca.template combine_compact<KIND>(s_wave, s_rec);
}

template <class T>
__device__ __forceinline__ void vc_search_body(const VcDev<T> &vd, Ctl *ctl, double *part)
{
    __shared__ double s_wave[4 * 3 * KC];
    __shared__ double s_rec[QMAX];
    if (ctl->phase != PH_SEARCH) return;
    const int kind = ctl->skind;
    if (kind == SK_REFINE) {
        const double eta = ctl->eta;
        const double a = ctl->ref_alpha;
        const bool second = ctl->ref_valid != 0;
        const double zm = ctl->rfZmin;
        // pass 2: [sum | derivative sum | -]; pass 1: [- | - | min z']
        double v[3] = {0.0, 0.0, INFINITY};
        auto visit = [&](XD<T> pu, XD<T> pw, int) {
            const double dzp = (double)pu.d + (double)pw.d;
            if (row_met(ctl, (double)pu.x + (double)pw.x)) return;
            const double zp = ((double)pu.x + (double)pw.x) + a * dzp;
            if (second) {
                const double t = exp(-eta * (zp - zm));
                v[0] += t;
                v[1] += dzp * t;
            } else {
                v[2] = fmin(v[2], zp);
            }
        };
        for_edges<T>(vd, visit);
        const Red red{2, 1, 0};
        block_combine<3>(v, red, 0, s_wave, s_rec);
        store_record(s_rec, 3, part);
        return;
    }
    // compact records of the covering sums only (no packing rows)
    switch (kind) {
    case SK_EXP:
        vc_search_edges<T, SK_EXP>(vd, ctl, s_wave, s_rec);
        store_record_qmajor(s_rec, cov_record_q<SK_EXP>(), part);
        break;
    case SK_GRID:
        vc_search_edges<T, SK_GRID>(vd, ctl, s_wave, s_rec);
        store_record_qmajor(s_rec, cov_record_q<SK_GRID>(), part);
        break;
    case SK_COMBO:
        vc_search_edges<T, SK_COMBO>(vd, ctl, s_wave, s_rec);
        store_record_qmajor(s_rec, cov_record_q<SK_COMBO>(), part);
        break;
    default:
        vc_search_edges<T, SK_LIST>(vd, ctl, s_wave, s_rec);
        store_record_qmajor(s_rec, cov_record_q<SK_LIST>(), part);
        break;
    }
}

// The FP32 search fits four waves per SIMD without spills (the combined pass
// holds 54 accumulators); ask the compiler to keep it there.
template <class T> __global__ void vc_search_k(VcDev<T> vd, Ctl *ctl, double *part);
template <>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(4)))
void vc_search_k<float>(VcDev<float> vd, Ctl *ctl, double *part) { vc_search_body<float>(vd, ctl, part); }
template <>
__global__ __launch_bounds__(BLOCK)
void vc_search_k<double>(VcDev<double> vd, Ctl *ctl, double *part) { vc_search_body<double>(vd, ctl, part); }

// part: the records of the search kernel (G of them, one per workgroup),
// folded here in one stage (each thread folds whole records, the loads of a
// record in flight together).
__global__ __launch_bounds__(BLOCK) void vc_search_fin(Ctl *ctl, const double *part, int G)
{
    __shared__ double s_wave[4 * 3 * KC];
    __shared__ double s_rec[QMAX];
    __shared__ double s_tmp[QMAX];
    __shared__ uint64_t s_ctl[CTL_WORDS];
    Ctl *c = ctl_stage(ctl, s_ctl);
    if (c->phase != PH_SEARCH) return;
    const int kind = c->skind;
    if (kind == SK_REFINE) {
        const Red red{2, 1, 0};
        fold_records<3>(part, G, red, 0, s_wave, s_rec);
        if (threadIdx.x == 0) {
            // finish_search expects pass 1 [min z' | max eta*y'], pass 2
            // [sumP | sumC | sumP' | sumC'] (no packing rows: Psi = a dy1)
            double r[4];
            if (c->ref_valid == 0) { r[0] = s_rec[2]; r[1] = -INFINITY; r[2] = r[3] = 0.0; }
            else { r[0] = 1.0; r[1] = s_rec[0]; r[2] = 0.0; r[3] = s_rec[1]; }
            finish_search(c, r);
        }
        ctl_write_back(ctl, s_ctl);
        return;
    }
    switch (kind) {
    case SK_EXP: fold_cov_compact<SK_EXP>(part, G, s_wave, s_tmp, s_rec + KC); break;
    case SK_GRID: fold_cov_compact<SK_GRID>(part, G, s_wave, s_tmp, s_rec + KC); break;
    case SK_COMBO: fold_cov_compact<SK_COMBO>(part, G, s_wave, s_tmp, s_rec + KC); break;
    default: fold_cov_compact<SK_LIST>(part, G, s_wave, s_tmp, s_rec + KC); break;
    }
    if (threadIdx.x < KC) s_rec[threadIdx.x] = 0.0;     // no packing rows: Psi = a * dy1
    if (threadIdx.x == 0) c->pass_sparse = act_valid(c, c->LCw);   // as the search kernel decided
    __syncthreads();
    if (!c->hold) pre_eval_search(c, s_rec);
    __syncthreads();
    if (threadIdx.x == 0) finish_search(c, s_rec, true);
    ctl_write_back(ctl, s_ctl);
}

template <class T>
__global__ __launch_bounds__(BLOCK) void vc_export_k(VcDev<T> vd, int which, double *out)
{
    if (which < 2) {
        for (int i = blockIdx.x * BLOCK + threadIdx.x; i < vd.nv; i += gridDim.x * BLOCK)
            out[i] = (double)(which == 0 ? vd.xd[i].x : vd.xd[i].d);
        return;
    }
    auto visit = [&](XD<T> pu, XD<T> pw, int e) {
        out[e] = which == 2 ? (double)(pu.x + pw.x) : (double)(pu.d + pw.d);
    };
    for_edges<T>(vd, visit);
}

template <class T>
__global__ void vc_import_k(VcDev<T> vd, const double *src)
{
    for (int i = blockIdx.x * BLOCK + threadIdx.x; i < vd.nv; i += gridDim.x * BLOCK) {
        XD<T> p;
        p.x = (T)src[i];
        p.d = T(0);
        vd.xd[i] = p;
        vd.xs[i] = p.x;
    }
}

// ------------------------------------------------------------------ active lists
// Built between graph launches against the current weight shift L = LC with
// margin mu: a covering row (edge) is left out when eta (z_e - L) exceeds the
// skip exponent plus mu, z_e from the committed x (z only grows, so this
// stays true while the shift drifts by less than mu / eta).

template <class T>
MWU_DEV bool left_out(double z, double eta, double L, double mu, bool drop)
{
    return eta * (z - L) > skip_exponent<T>() + mu || (drop && z >= 1.0);
}

// Pack the active neighbours of each tile of the full adjacency at the start
// of the tile's range (fcol_pk, in order), with the packed start of each row
// of a multi-row tile (fptr_pk) and the active count of every tile (tile_na).
template <class T>
__global__ __launch_bounds__(BLOCK) void vc_pack_k(VcDev<T> vd, const Ctl *ctl, double mu)
{
    __shared__ int32_t s_ptr[TILE_NZ + 1];
    __shared__ int32_t s_cnt[BLOCK / 64];
    const double eta = ctl->eta, L = ctl->LC;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int t = blockIdx.x; t < vd.nftiles; t += gridDim.x) {
        const Tile tl = vd.ftiles[t];
        const bool chunk = tl.lid >= 0;     // a piece of one long row
        const int S_ = tl.s1 - tl.s0;
        const int N = tl.k1 - tl.k0;
        if (!chunk) {
            for (int i = threadIdx.x; i < S_; i += BLOCK) s_ptr[i] = vd.fptr[tl.s0 + i] - tl.k0;
            if (threadIdx.x == 0) s_ptr[S_] = N;
        }
        __syncthreads();
        const double xrow = (double)vd.xs[tl.s0];
        int base = 0;
        for (int c0 = 0; c0 < N; c0 += BLOCK) {
            const int k = c0 + threadIdx.x;
            bool keep = false, first = false;
            int col = 0, lo = 0;
            if (k < N) {
                col = vd.fcol[tl.k0 + k];
                double zr = xrow;
                if (!chunk) {
                    int hi = S_;   // s_ptr[lo] <= k < s_ptr[hi]
                    while (hi - lo > 1) {
                        const int mid = (lo + hi) >> 1;
                        if (s_ptr[mid] <= k) lo = mid; else hi = mid;
                    }
                    zr = (double)vd.xs[tl.s0 + lo];
                    first = s_ptr[lo] == k;
                }
                keep = !left_out<T>(zr + (double)vd.xs[col], eta, L, mu, ctl->drop != 0);
            }
            const unsigned long long m = __ballot(keep);
            if (lane == 0) s_cnt[wv] = __popcll(m);
            __syncthreads();
            int off = 0, total = 0;
            for (int q = 0; q < BLOCK / 64; ++q) {
                if (q < wv) off += s_cnt[q];
                total += s_cnt[q];
            }
            const int rank = base + off + __popcll(m & ((1ull << lane) - 1ull));   // active before k
            if (keep) vd.fcol_pk[tl.k0 + rank] = col;
            if (first) vd.fptr_pk[tl.s0 + lo] = tl.k0 + rank;
            base += total;
            __syncthreads();
        }
        if (threadIdx.x == 0) vd.tile_na[t] = base;
    }
}

// Exclusive prefix of src[0..n) into dst[0..n] (dst[n] = total) by one
// workgroup, in batches of PER x BLOCK elements: each thread loads and sums
// PER consecutive elements, one scan over the thread totals places them, and
// each thread writes its elements' prefixes (two barriers per batch).
template <int PER>
MWU_DEV void block_exclusive_scan(const int32_t *src, int n, int32_t *dst)
{
    __shared__ int32_t s_w[BLOCK / 64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    int run = 0;
    for (int base = 0; base < n; base += PER * BLOCK) {
        const int i0 = base + threadIdx.x * PER;
        int32_t v[PER];
        int tsum = 0;
#pragma unroll
        for (int r = 0; r < PER; ++r) {
            v[r] = i0 + r < n ? src[i0 + r] : 0;
            tsum += v[r];
        }
        int x = tsum;                                       // inclusive scan in the wave
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const int y = __shfl_up(x, d);
            if (lane >= d) x += y;
        }
        if (lane == 63) s_w[wv] = x;
        __syncthreads();
        int off = run, tot = 0;
        for (int w = 0; w < BLOCK / 64; ++w) {
            if (w < wv) off += s_w[w];
            tot += s_w[w];
        }
        int p = off + x - tsum;
#pragma unroll
        for (int r = 0; r < PER; ++r) {
            if (i0 + r < n) dst[i0 + r] = p;
            p += v[r];
        }
        run += tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) dst[n] = run;
}

constexpr int ITEM_SCAN_PER = 16;

// Tile offsets goff of the concatenated packed neighbours (exclusive prefix
// of tile_na).
__global__ __launch_bounds__(BLOCK) void vc_goff_k(const int32_t *tile_na, int nt, int32_t *goff)
{
    block_exclusive_scan<ITEM_SCAN_PER>(tile_na, nt, goff);
}

// Work items of the packed pass: tile t joins the largest aligned run of 2^l
// tiles (l <= 6) that holds at most TILE_NZ rows and TILE_NZ active
// neighbours in total, so a run fits one tile's LDS staging; chunk tiles of
// long rows never join a run (tile_rows, the static exclusive prefix of rows
// per tile, counts them as TILE_NZ + 1 rows).  head[t] = 1 when tile t
// starts its run; run[t] = the run's length.
MWU_DEV int run_level(int t, int nt, const int32_t *tile_rows, const int32_t *goff)
{
    int lev = 0;
    for (int l = 1; l <= 6; ++l) {
        const int a = (t >> l) << l, b = min(nt, a + (1 << l));
        if (tile_rows[b] - tile_rows[a] > TILE_NZ || goff[b] - goff[a] > TILE_NZ) break;
        lev = l;
    }
    return lev;
}

__global__ __launch_bounds__(BLOCK) void vc_runs_k(int nt, const int32_t *tile_rows, const int32_t *goff,
                                                   int32_t *head)
{
    for (int t = blockIdx.x * BLOCK + threadIdx.x; t < nt; t += gridDim.x * BLOCK) {
        const int l = run_level(t, nt, tile_rows, goff);
        head[t] = ((t >> l) << l) == t ? 1 : 0;
    }
}

// One workgroup: positions of the run heads and the number of items.
__global__ __launch_bounds__(BLOCK) void vc_hscan_k(const int32_t *head, int nt, int32_t *hpos, Ctl *ctl)
{
    block_exclusive_scan<ITEM_SCAN_PER>(head, nt, hpos);
    if (threadIdx.x == 0) ctl->act_nitems = hpos[nt];   // written by this thread
}

// The items in order, one thread per run head.
__global__ __launch_bounds__(BLOCK) void vc_items_k(const Tile *tiles, int nt, const int32_t *tile_rows,
                                                    const int32_t *goff, const int32_t *head,
                                                    const int32_t *hpos, Tile *items)
{
    for (int t = blockIdx.x * BLOCK + threadIdx.x; t < nt; t += gridDim.x * BLOCK) {
        if (!head[t]) continue;
        const int l = run_level(t, nt, tile_rows, goff);
        const int last = min(nt, t + (1 << l)) - 1;
        Tile it = tiles[t];
        it.s1 = tiles[last].s1;
        it.k0 = goff[t];
        it.k1 = goff[last + 1];
        items[hpos[t]] = it;   // a chunk tile keeps its lid and cidx (runs of length 1)
    }
}

// Concatenate the packed neighbours of every tile at its offset goff, and
// the concatenated start of every row of a multi-row tile.
template <class T>
__global__ __launch_bounds__(BLOCK) void vc_concat_k(VcDev<T> vd)
{
    for (int t = blockIdx.x; t < vd.nftiles; t += gridDim.x) {
        const Tile tl = vd.ftiles[t];
        const int na = vd.tile_na[t], g = vd.goff[t];
        for (int i = threadIdx.x; i < na; i += BLOCK) vd.ccol[g + i] = vd.fcol_pk[tl.k0 + i];
        if (tl.lid < 0)
            for (int r = tl.s0 + threadIdx.x; r < tl.s1; r += BLOCK) vd.cst[r] = g + (vd.fptr_pk[r] - tl.k0);
    }
}

// Edge range of block b in the active-list build: contiguous, whole waves.
MWU_DEV void act_range(int ne, int &e0, int &e1)
{
    const int G = gridDim.x;
    const int ch = ((ne + G - 1) / G + BLOCK - 1) / BLOCK * BLOCK;
    e0 = min(ne, blockIdx.x * ch);
    e1 = min(ne, e0 + ch);
}

// Per block: active edges of its range, and min z over the left-out ones.
template <class T>
__global__ __launch_bounds__(BLOCK) void vc_act_count_k(VcDev<T> vd, const Ctl *ctl, double mu, double *part)
{
    __shared__ double s_wave[4 * 2];
    __shared__ double s_rec[QMAX];
    const double eta = ctl->eta, L = ctl->LC;
    int e0, e1;
    act_range(vd.ne, e0, e1);
    double v[2] = {0.0, INFINITY};   // active count | min z left out
    for (int e = e0 + threadIdx.x; e < e1; e += BLOCK) {
        const double z = (double)vd.xs[vd.eu[e]] + (double)vd.xs[vd.ew[e]];
        if (left_out<T>(z, eta, L, mu, ctl->drop != 0)) v[1] = fmin(v[1], z);
        else v[0] += 1.0;
    }
    const Red red{1, 1, 0};
    block_combine<2>(v, red, 0, s_wave, s_rec);
    if (threadIdx.x == 0) vd.acnt[blockIdx.x] = (int32_t)s_rec[0];
    store_record(s_rec, 2, part);
}

// One workgroup: exclusive scan of the block counts (in place), the list
// length, the floor of the left-out minima, and the lists switched on.
__global__ __launch_bounds__(BLOCK) void vc_act_scan_k(int32_t *acnt, int G, Ctl *ctl, const double *part,
                                                       double mu)
{
    __shared__ int32_t s_sum[BLOCK];
    __shared__ double s_wave[4];
    __shared__ double s_rec[QMAX];
    const int per = (G + BLOCK - 1) / BLOCK;
    const int i0 = min(G, threadIdx.x * per), i1 = min(G, i0 + per);
    int tot = 0;
    for (int i = i0; i < i1; ++i) tot += acnt[i];
    s_sum[threadIdx.x] = tot;
    __syncthreads();
    if (threadIdx.x == 0) {
        int run = 0;
        for (int t = 0; t < BLOCK; ++t) {
            const int c = s_sum[t];
            s_sum[t] = run;
            run += c;
        }
        ctl->act_ne = run;
    }
    __syncthreads();
    int run = s_sum[threadIdx.x];
    for (int i = i0; i < i1; ++i) {
        const int c = acnt[i];
        acnt[i] = run;
        run += c;
    }
    const Red red{0, 1, 0};
    double v[1] = {INFINITY};
    for (int b = threadIdx.x; b < G; b += BLOCK) v[0] = fmin(v[0], part[(size_t)b * QMAX + 1]);
    block_combine<1>(v, red, 0, s_wave, s_rec);
    if (threadIdx.x == 0) {
        ctl->act_zfloor = s_rec[0];
        ctl->act_L = ctl->LC;
        ctl->act_mu = mu;
        ctl->act_on = 1;
    }
}

// Scatter the active edges of each block's range to its offset, in order.
template <class T>
__global__ __launch_bounds__(BLOCK) void vc_act_scatter_k(VcDev<T> vd, const Ctl *ctl, double mu)
{
    __shared__ int32_t s_cnt[BLOCK / 64];
    const double eta = ctl->eta, L = ctl->act_L;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    int e0, e1;
    act_range(vd.ne, e0, e1);
    int base = vd.acnt[blockIdx.x];
    for (int c0 = e0; c0 < e1; c0 += BLOCK) {
        const int e = c0 + threadIdx.x;
        int u = 0, w = 0;
        bool keep = false;
        if (e < e1) {
            u = vd.eu[e];
            w = vd.ew[e];
            keep = !left_out<T>((double)vd.xs[u] + (double)vd.xs[w], eta, L, mu, ctl->drop != 0);
        }
        const unsigned long long m = __ballot(keep);
        if (lane == 0) s_cnt[wv] = __popcll(m);
        __syncthreads();
        int off = 0, total = 0;
        for (int q = 0; q < BLOCK / 64; ++q) {
            if (q < wv) off += s_cnt[q];
            total += s_cnt[q];
        }
        if (keep) {
            const int pos = base + off + __popcll(m & ((1ull << lane) - 1ull));
            if (pos < vd.ne) {   // always: the count pass made the same decisions
                vd.aeu[pos] = u;
                vd.aew[pos] = w;
            }
        }
        base += total;
        __syncthreads();
    }
}

// ------------------------------------------------------------------ launchers

#define VLAUNCH(kernel, grid, ...) hipLaunchKernelGGL(kernel, dim3(grid), dim3(BLOCK), 0, st, __VA_ARGS__)

template <class T>
void vc_init(const VcDev<T> &v, Ctl *ctl, const VcLaunch &L, hipStream_t st, bool have_x0)
{
    VLAUNCH(vc_init_x<T>, L.grid_v, v, ctl, have_x0 ? 1 : 0, L.partials);
    VLAUNCH(vc_init_x_fin, 1, ctl, (const double *)L.partials, L.grid_v);
    VLAUNCH(vc_minz<T>, L.grid_e, v, ctl, L.partials);
    VLAUNCH(vc_minz_fin, 1, ctl, (const double *)L.partials, L.grid_e);
}

template <class T>
void vc_passA(const VcDev<T> &v, Ctl *ctl, const VcLaunch &L, hipStream_t st)
{
    VLAUNCH(vc_commit_k<T>, L.grid_v, v, ctl);
    VLAUNCH(vc_passA_k<T>, L.grid_ftile, v, ctl, L.partials);
    // up to 2 BLOCK long rows are completed by the finisher itself
    const int with_long = v.flong.nlong <= 2 * BLOCK;
    VLAUNCH(vc_passA_fin<T>, 1, v, ctl, (const double *)L.partials, L.grid_ftile, with_long);
}

template <class T>
void vc_passB(const VcDev<T> &v, Ctl *ctl, const VcLaunch &L, hipStream_t st)
{
    VLAUNCH(vc_passB_k<T>, L.grid_v, v, ctl, L.partials);
    VLAUNCH(vc_passB_fin<T>, 1, v, ctl, (const double *)L.partials, L.grid_v);
}

template <class T>
void vc_search(const VcDev<T> &v, Ctl *ctl, const VcLaunch &L, hipStream_t st)
{
    VLAUNCH(vc_search_k<T>, L.grid_e, v, ctl, L.partials);
    VLAUNCH(vc_search_fin, 1, ctl, (const double *)L.partials, L.grid_e);
}

// One iteration slot with a single search launch: most iterations finish
// their step search in the combined first pass; one that needs more passes
// takes them in the following slots, whose other passes see the search phase
// and return at once.
template <class T>
void vc_iteration(const VcDev<T> &v, Ctl *ctl, const VcLaunch &L, hipStream_t st)
{
    vc_passA(v, ctl, L, st);
    vc_passB(v, ctl, L, st);
    vc_search(v, ctl, L, st);
}

template <class T>
void vc_build_active(const VcDev<T> &v, Ctl *ctl, const VcLaunch &L, hipStream_t st, double mu)
{
    VLAUNCH(vc_pack_k<T>, L.grid_ftile, v, ctl, mu);
    VLAUNCH(vc_goff_k, 1, (const int32_t *)v.tile_na, v.nftiles, v.goff);
    const int gt = std::max(1, std::min(GRID_MAX, (v.nftiles + BLOCK - 1) / BLOCK));
    VLAUNCH(vc_runs_k, gt, v.nftiles, (const int32_t *)v.tile_rows, (const int32_t *)v.goff, v.thead);
    VLAUNCH(vc_hscan_k, 1, (const int32_t *)v.thead, v.nftiles, v.thpos, ctl);
    VLAUNCH(vc_items_k, gt, v.ftiles, v.nftiles, (const int32_t *)v.tile_rows, (const int32_t *)v.goff,
            (const int32_t *)v.thead, (const int32_t *)v.thpos, v.items);
    VLAUNCH(vc_concat_k<T>, L.grid_ftile, v);
    VLAUNCH(vc_act_count_k<T>, L.grid_act, v, ctl, mu, L.partials);
    VLAUNCH(vc_act_scan_k, 1, v.acnt, L.grid_act, ctl, (const double *)L.partials, mu);
    VLAUNCH(vc_act_scatter_k<T>, L.grid_act, v, ctl, mu);
}

template <class T>
void vc_export(const VcDev<T> &v, int which, double *out, hipStream_t st)
{
    const int g = which < 2 ? std::max(1, std::min(GRID_MAX, (v.nv + BLOCK - 1) / BLOCK))
                            : std::max(1, std::min(GRID_MAX, (v.ne + BLOCK - 1) / BLOCK));
    VLAUNCH(vc_export_k<T>, g, v, which, out);
}

template <class T>
void vc_import_x(const VcDev<T> &v, const double *src, hipStream_t st)
{
    const int g = std::max(1, std::min(GRID_MAX, (v.nv + BLOCK - 1) / BLOCK));
    VLAUNCH(vc_import_k<T>, g, v, src);
}

// The main kernel of one pass alone (no finisher): timing of held passes.
template <class T>
void vc_main(const VcDev<T> &v, Ctl *ctl, const VcLaunch &L, hipStream_t st, int which)
{
    switch (which) {
    case 0: VLAUNCH(vc_passA_k<T>, L.grid_ftile, v, ctl, L.partials); break;
    case 1: VLAUNCH(vc_passB_k<T>, L.grid_v, v, ctl, L.partials); break;
    case 2: break;
    default: VLAUNCH(vc_search_k<T>, L.grid_e, v, ctl, L.partials); break;
    }
}

// Workgroups of the tile and edge kernels that fit on one CU at once: the
// persistent grids are sized to exactly fill the chip in one round.
template <class T>
void vc_occupancy(int *per_cu_ftile, int *per_cu_edge)
{
    int a = 0, b = 0;
    HIP_CHECK_OCC(hipOccupancyMaxActiveBlocksPerMultiprocessor(&a, vc_passA_k<T>, BLOCK, 0));
    HIP_CHECK_OCC(hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, vc_search_k<T>, BLOCK, 0));
    *per_cu_ftile = a > 0 ? a : 1;
    *per_cu_edge = b > 0 ? b : 1;
}

#define MWU_VC_INSTANTIATE(T)                                                                    \
    template void vc_init<T>(const VcDev<T> &, Ctl *, const VcLaunch &, hipStream_t, bool);      \
    template void vc_iteration<T>(const VcDev<T> &, Ctl *, const VcLaunch &, hipStream_t);       \
    template void vc_passA<T>(const VcDev<T> &, Ctl *, const VcLaunch &, hipStream_t);           \
    template void vc_passB<T>(const VcDev<T> &, Ctl *, const VcLaunch &, hipStream_t);           \
    template void vc_search<T>(const VcDev<T> &, Ctl *, const VcLaunch &, hipStream_t);          \
    template void vc_build_active<T>(const VcDev<T> &, Ctl *, const VcLaunch &, hipStream_t, double); \
    template void vc_export<T>(const VcDev<T> &, int, double *, hipStream_t);                    \
    template void vc_import_x<T>(const VcDev<T> &, const double *, hipStream_t);                 \
    template void vc_occupancy<T>(int *, int *);                                                  \
    template void vc_main<T>(const VcDev<T> &, Ctl *, const VcLaunch &, hipStream_t, int);

MWU_VC_INSTANTIATE(float)
MWU_VC_INSTANTIATE(double)

}  // namespace mwu
