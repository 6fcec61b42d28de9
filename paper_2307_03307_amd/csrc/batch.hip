// Batched program (gfx950): many independent bipartite-matching packing LPs,
// max 1^T x s.t. M_k x <= 1 (Section 3), each run as the mixed problem with
// the objective row (1/M_k) 1^T x >= 1 (end of Section 2.2) through Algorithm
// 2 with the step search of Algorithm 3 (Section 4), all in the same kernels.
//
// Every instance keeps its own control block, so instances sit in different
// phases of their own probes at the same time; each kernel visits the tiles
// of the instances that are in its phase and skips the others.  The iteration
// slot launched (and captured in a hipGraph) is
//   init-x, init-y (probe start), row, column, forward, search (one or more
//   passes), statistics (probe end)
// with one finisher per pass that runs one workgroup per instance.  The host
// drives only the outer search over M_k from a compact status array.
#include <algorithm>

#include "device_common.h"

namespace mwu {

template <class T>
MWU_DEV void write_stat(const BatchDev<T> &b, int k, const Ctl *c)
{
    b.stat[4 * k + 0] = c->phase;
    b.stat[4 * k + 1] = c->status;
    b.stat[4 * k + 2] = c->iter;
}

// Visit this workgroup's tiles (t = blockIdx.x + j gridDim.x, ascending)
// whose instance is in one of two phases.  The phases of up to BLOCK tiles are
// read in parallel from the compact status array and the matching tiles are
// compacted through LDS in ascending order (wave ballots, no atomics), so a
// pass that most instances sit out costs one parallel read per BLOCK tiles
// instead of one dependent read per tile.  body(t) runs with the whole
// workgroup.
template <class T, class Body>
MWU_DEV void for_phase_tiles(const BatchDev<T> &b, const BTile *tiles, int ntiles, int ph1, int ph2,
                             Body &body)
{
    __shared__ int32_t s_list[BLOCK];
    __shared__ int32_t s_cnt[BLOCK / 64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int G = gridDim.x;
    for (int base = blockIdx.x; base < ntiles; base += G * BLOCK) {
        const int t = base + threadIdx.x * G;
        bool hit = false;
        if (t < ntiles) {
            const int ph = b.stat[4 * tiles[t].inst];
            hit = ph == ph1 || ph == ph2;
        }
        const unsigned long long m = __ballot(hit);
        if (lane == 0) s_cnt[wv] = __popcll(m);
        __syncthreads();
        int off = 0, total = 0;
        for (int w = 0; w < BLOCK / 64; ++w) {
            if (w < wv) off += s_cnt[w];
            total += s_cnt[w];
        }
        if (hit) s_list[off + __popcll(m & ((1ull << lane) - 1ull))] = t;
        __syncthreads();
        for (int i = 0; i < total; ++i) body(s_list[i]);
        __syncthreads();
    }
}

// ------------------------------------------------------------------ probe start

template <class T>
__global__ __launch_bounds__(BLOCK) void kb_initx(BatchDev<T> b)
{
    __shared__ double s_wave[4];
    __shared__ double s_rec[QMAX];
    auto body = [&](int t) {
        const BTile tl = b.et[t];
        const Ctl *c = b.ctl + tl.inst;
        // Algorithm 1: x_i = eps / (n max_j P_ji) with P_ji = 1 on incident rows
        const T x0 = (T)(c->eps / (double)b.nedge[tl.inst]);
        double v[1] = {0.0};
        for (int e = tl.i0 + threadIdx.x; e < tl.i1; e += BLOCK) {
            b.x[e] = x0;
            b.d[e] = T(0);
            v[0] += (double)x0;
        }
        const Red red{1, 0, 0};
        block_combine<1>(v, red, 0, s_wave, s_rec);
        if (threadIdx.x == 0) b.epart[(size_t)t * QMAX] = s_rec[0];
    };
    for_phase_tiles(b, b.et, b.net, PH_INIT, PH_INIT, body);
}

template <class T>
__global__ __launch_bounds__(BLOCK) void kb_initx_fin(BatchDev<T> b)
{
    __shared__ double s_wave[4];
    __shared__ double s_rec[QMAX];
    const int k = blockIdx.x;
    Ctl *c = b.ctl + k;
    if (c->phase != PH_INIT) return;
    const Red red{1, 0, 0};
    fold_records<1>(b.epart + (size_t)b.erec0[k] * QMAX, b.erecn[k], red, 0, s_wave, s_rec);
    if (threadIdx.x == 0) {
        finish_sumx(c, s_rec[0]);
        c->phase = PH_INIT_Y;
        write_stat(b, k, c);
    }
}

// Tile of vertex tiles as a plain segment tile.
MWU_DEV Tile as_tile(const BTile &b)
{
    Tile t;
    t.s0 = b.i0; t.s1 = b.i1; t.k0 = b.k0; t.k1 = b.k1; t.lid = b.lid; t.cidx = b.cidx;
    return t;
}

// Vertex sums over incident edges, nnz-balanced: INIT_Y gives y = P x0 (and
// clears dy), FWD gives dy = P d.  Incidence indices are staged through LDS
// with coalesced loads; vertices longer than a tile are summed in chunks and
// completed by the finisher.  Record [min over covering rows (none) | max].
template <class T>
__global__ __launch_bounds__(BLOCK) void kb_vfwd(BatchDev<T> b)
{
    __shared__ T s_acc[TILE_LDS];
    __shared__ int32_t s_ptr[TILE_NZ + 1];
    __shared__ T s_tacc[BLOCK / 64];
    __shared__ double s_wave[4 * 2];
    __shared__ double s_rec[QMAX];
    auto body = [&](int t) {
        const BTile bt = b.vt[t];
        const Ctl *c = b.ctl + bt.inst;
        const int ph = c->phase;
        const bool init = ph == PH_INIT_Y;
        const T *src = init ? b.x : b.d;
        const T sP = (T)c->sP;
        double v[2] = {INFINITY, -INFINITY};
        auto elem = [&](int k) -> T { return src[b.vedge[k]]; };
        auto epi = [&](int i, T acc) {
            acc = sP * acc;
            if (init) { b.y[i] = acc; b.dy[i] = T(0); }
            else b.dy[i] = acc;
            v[1] = fmax(v[1], (double)acc);
        };
        const Tile tl = as_tile(bt);
        if (tl.lid < 0) seg_tile<T>(tl, b.vptr, elem, epi, s_acc, s_ptr, nullptr, nullptr);
        else chunk_tile<T>(tl, elem, s_tacc, b.lpart, b.vlong.lfirst);
        const Red red{0, 1, 1};
        block_combine<2>(v, red, 0, s_wave, s_rec);
        if (threadIdx.x < 2) b.vpart[(size_t)t * QMAX + threadIdx.x] = s_rec[threadIdx.x];
    };
    for_phase_tiles(b, b.vt, b.nvt, PH_INIT_Y, PH_FWD, body);
}

template <class T>
__global__ __launch_bounds__(BLOCK) void kb_vfwd_fin(BatchDev<T> b)
{
    __shared__ double s_wave[4 * 2];
    __shared__ double s_rec[QMAX];
    __shared__ double s_lng[QMAX];
    const int k = blockIdx.x;
    Ctl *c = b.ctl + k;
    const int ph = c->phase;
    if (ph != PH_INIT_Y && ph != PH_FWD) return;
    const bool init = ph == PH_INIT_Y;
    const T sP = (T)c->sP;
    const Red red{0, 1, 1};
    double v[2] = {INFINITY, -INFINITY};
    for (int l = b.lrec0[k] + threadIdx.x; l < b.lrec0[k] + b.lrecn[k]; l += BLOCK) {
        const T acc = sP * long_sum<T>(l, b.lpart, b.vlong.lfirst, b.vlong.lcount);
        const int i = b.vlong.lseg[l];
        if (init) { b.y[i] = acc; b.dy[i] = T(0); }
        else b.dy[i] = acc;
        v[1] = fmax(v[1], (double)acc);
    }
    block_combine<2>(v, red, 0, s_wave, s_lng);
    fold_records<2>(b.vpart + (size_t)b.vrec0[k] * QMAX, b.vrecn[k], red, 0, s_wave, s_rec);
    on_ctl(c, [&](Ctl *cl) {
        for (int q = 0; q < 2; ++q) s_rec[q] = red_op(s_rec[q], s_lng[q], q, red);
        if (init) {
            finish_init_fwd(cl, s_rec);
        } else {
            cl->dymax = s_rec[1];
            begin_search(cl, nullptr);
        }
        write_stat(b, k, cl);
    });
}

// ------------------------------------------------------------------ iteration

// Row pass: y += a dy, w = exp(eta (y - L_P)).  Record [sum w | - | - | max y].
template <class T>
__global__ __launch_bounds__(BLOCK) void kb_row(BatchDev<T> b)
{
    __shared__ double s_wave[4 * 4];
    __shared__ double s_rec[QMAX];
    auto body = [&](int t) {
        const BTile tl = b.wt[t];
        const Ctl *c = b.ctl + tl.inst;
        const T a = (T)c->alpha;
        const double eta = c->eta, LP = c->LP;
        double v[4] = {0.0, 0.0, INFINITY, -INFINITY};
        for (int i = tl.i0 + threadIdx.x; i < tl.i1; i += BLOCK) {
            const T y = b.y[i] + a * b.dy[i];
            b.y[i] = y;
            const T w = exp_arg(eta * ((double)y - LP), T(0));
            b.w[i] = w;
            v[0] += (double)w;
            v[3] = fmax(v[3], (double)y);
        }
        const Red red{2, 1, 1};
        block_combine<4>(v, red, 0, s_wave, s_rec);
        if (threadIdx.x < 4) b.wpart[(size_t)t * QMAX + threadIdx.x] = s_rec[threadIdx.x];
    };
    for_phase_tiles(b, b.wt, b.nwt, PH_ROW, PH_ROW, body);
}

template <class T>
__global__ __launch_bounds__(BLOCK) void kb_row_fin(BatchDev<T> b)
{
    __shared__ double s_wave[4 * 4];
    __shared__ double s_rec[QMAX];
    const int k = blockIdx.x;
    Ctl *c = b.ctl + k;
    if (c->phase != PH_ROW) return;
    const Red red{2, 1, 1};
    fold_records<4>(b.wpart + (size_t)b.wrec0[k] * QMAX, b.wrecn[k], red, 0, s_wave, s_rec);
    on_ctl(c, [&](Ctl *cl) {
        finish_row(cl, s_rec);
        write_stat(b, k, cl);
    });
}

// Column pass over edges: commit x += a d, then g = (w_u + w_v) / sum w,
// h = 1/M (the objective row) and the direction.  Record [sum d | min g |
// max d | max h].  In PH_COMMIT only the commit.
template <class T>
__global__ __launch_bounds__(BLOCK) void kb_col(BatchDev<T> b)
{
    __shared__ double s_wave[4 * 4];
    __shared__ double s_rec[QMAX];
    auto body = [&](int t) {
        const BTile tl = b.et[t];
        const Ctl *c = b.ctl + tl.inst;
        const int ph = c->phase;
        const T a = (T)c->alpha;
        if (ph == PH_COMMIT) {
            for (int e = tl.i0 + threadIdx.x; e < tl.i1; e += BLOCK) b.x[e] = b.x[e] + a * b.d[e];
            return;
        }
        const double sP = c->sP, sC = c->sC, invSw = c->invSw, step = c->step, qmin = c->qmin;
        double v[4] = {0.0, INFINITY, -INFINITY, -INFINITY};
        for (int e = tl.i0 + threadIdx.x; e < tl.i1; e += BLOCK) {
            const T x = b.x[e] + a * b.d[e];
            b.x[e] = x;
            const double g = sP * (double)(b.w[b.eu[e]] + b.w[b.ev[e]]) * invSw;
            const double h = sC;
            double di = 0.0;
            const double q = 1.0 - g / h;
            if (q > qmin) di = step * q * (double)x;
            const T dt = (T)di;
            b.d[e] = dt;
            v[0] += (double)dt;
            v[1] = fmin(v[1], g);
            v[2] = fmax(v[2], (double)dt);
            v[3] = fmax(v[3], h);
        }
        const Red red{1, 1, 2};
        block_combine<4>(v, red, 0, s_wave, s_rec);
        if (threadIdx.x < 4) b.epart[(size_t)t * QMAX + threadIdx.x] = s_rec[threadIdx.x];
    };
    for_phase_tiles(b, b.et, b.net, PH_COL, PH_COMMIT, body);
}

template <class T>
__global__ __launch_bounds__(BLOCK) void kb_col_fin(BatchDev<T> b)
{
    __shared__ double s_wave[4 * 4];
    __shared__ double s_rec[QMAX];
    const int k = blockIdx.x;
    Ctl *c = b.ctl + k;
    const int ph = c->phase;
    if (ph != PH_COL && ph != PH_COMMIT) return;
    if (ph == PH_COMMIT) {
        if (threadIdx.x == 0) {
            c->alpha = 0.0;
            c->phase = PH_STATS;
            write_stat(b, k, c);
        }
        return;
    }
    const Red red{1, 1, 2};
    fold_records<4>(b.epart + (size_t)b.erec0[k] * QMAX, b.erecn[k], red, 0, s_wave, s_rec);
    on_ctl(c, [&](Ctl *cl) {
        finish_col(cl, s_rec);
        if (cl->phase == PH_DONE) cl->phase = PH_STATS;
        write_stat(b, k, cl);
    });
}

// ------------------------------------------------------------------ step search

// Packing sums of one search pass over the vertex rows of a tile (KIND fixed
// per pass): s1P[k] = sum_v w_v expm1(eta a_k dy_v).
template <class T, int KIND>
MWU_DEV void kb_search_rows(const BatchDev<T> &b, const BTile &tl, const Ctl *c, double *s_wave,
                            double *s_rec)
{
    const double eta = c->eta, a0 = c->cand[0], ga0 = c->ga0, gdel = c->gdelta, dymax = c->dymax;
    const uint32_t shm = shifted_mask(c);
    const int nc = c->ncand;
    const bool deriv = c->skind == SK_NEWTON;
    double s1[KC];
#pragma unroll
    for (int k = 0; k < KC; ++k) s1[k] = 0.0;
    for (int i = tl.i0 + threadIdx.x; i < tl.i1; i += BLOCK)
        pack_terms<T, KIND>(nc, c->cand, a0, ga0, gdel, eta, b.w[i], b.dy[i], dymax, shm, s1, deriv);
    const Red redp{KC, 0, 0};
    block_combine<KC>(s1, redp, 0, s_wave, s_rec);
}

template <class T>
__global__ __launch_bounds__(BLOCK) void kb_search(BatchDev<T> b)
{
    __shared__ double s_wave[4 * KC];
    __shared__ double s_rec[QMAX];
    auto body = [&](int t) {
        const BTile tl = b.wt[t];
        const Ctl *c = b.ctl + tl.inst;
        double *rec = b.wpart + (size_t)t * QMAX;
        if (c->skind == SK_REFINE) {
            const double a = c->ref_alpha, eta = c->eta;
            double v[2];
            const int i1 = tl.i1;
            int nq = 2;
            if (c->ref_valid == 0) {          // pass 1: [min z' (no covering rows) | max eta y']
                v[0] = INFINITY;
                v[1] = -INFINITY;
                for (int i = tl.i0 + threadIdx.x; i < i1; i += BLOCK)
                    v[1] = fmax(v[1], eta * ((double)b.y[i] + a * (double)b.dy[i]));
                const Red red{0, 1, 1};
                block_combine<2>(v, red, 0, s_wave, s_rec);
            } else {                          // pass 2: [sum exp(eta y' - pm) | - | its derivative sum | -]
                const double pm = c->rfPm;
                double v4[4] = {0.0, 0.0, 0.0, 0.0};
                for (int i = tl.i0 + threadIdx.x; i < i1; i += BLOCK) {
                    const double dv = (double)b.dy[i];
                    const double t = exp(eta * ((double)b.y[i] + a * dv) - pm);
                    v4[0] += t;
                    v4[2] += dv * t;
                }
                const Red red{4, 0, 0};
                block_combine<4>(v4, red, 0, s_wave, s_rec);
                nq = 4;
            }
            if (threadIdx.x < nq) rec[threadIdx.x] = s_rec[threadIdx.x];
            return;
        }
        switch (c->skind) {
        case SK_EXP: kb_search_rows<T, SK_EXP>(b, tl, c, s_wave, s_rec); break;
        case SK_GRID: kb_search_rows<T, SK_GRID>(b, tl, c, s_wave, s_rec); break;
        case SK_COMBO: kb_search_rows<T, SK_COMBO>(b, tl, c, s_wave, s_rec); break;
        default: kb_search_rows<T, SK_LIST>(b, tl, c, s_wave, s_rec); break;
        }
        if (threadIdx.x < KC) rec[threadIdx.x] = s_rec[threadIdx.x];
    };
    for_phase_tiles(b, b.wt, b.nwt, PH_SEARCH, PH_SEARCH, body);
}

template <class T>
__global__ __launch_bounds__(BLOCK) void kb_search_fin(BatchDev<T> b)
{
    __shared__ double s_wave[4 * KC];
    __shared__ double s_rec[QMAX];
    const int k = blockIdx.x;
    Ctl *c = b.ctl + k;
    if (c->phase != PH_SEARCH) return;
    const double *part = b.wpart + (size_t)b.wrec0[k] * QMAX;
    const int G = b.wrecn[k];
    if (c->skind == SK_REFINE) {
        if (c->ref_valid == 0) fold_records<2>(part, G, Red{0, 1, 1}, 0, s_wave, s_rec);
        else fold_records<4>(part, G, Red{4, 0, 0}, 0, s_wave, s_rec);
    } else {
        const Red red{KC, 0, 0};
        fold_records<KC>(part, G, red, 0, s_wave, s_rec);
        // no explicit covering rows: their sums are unused (the objective row
        // is evaluated in closed form)
        for (int q = KC + threadIdx.x; q < 4 * KC; q += BLOCK) s_rec[q] = 0.0;
        __syncthreads();
    }
    auto pre = [&](Ctl *cl) {   // all candidates at once, one per lane
        if (cl->skind != SK_REFINE && !cl->hold) pre_eval_search(cl, s_rec);
    };
    on_ctl_all(c, pre, [&](Ctl *cl) {
        finish_search(cl, s_rec, cl->skind != SK_REFINE);
        if (cl->phase == PH_DONE) cl->phase = PH_STATS;
        write_stat(b, k, cl);
    });
}

// ------------------------------------------------------------------ probe end

// FP64 statistics of the final x: max over vertices of sum_{e ~ v} x_e, and
// sum x (the objective row before scaling).
template <class T>
__global__ __launch_bounds__(BLOCK) void kb_stats_v(BatchDev<T> b)
{
    __shared__ double s_acc[TILE_LDS];
    __shared__ int32_t s_ptr[TILE_NZ + 1];
    __shared__ double s_tacc[BLOCK / 64];
    __shared__ double s_wave[4];
    __shared__ double s_rec[QMAX];
    auto body = [&](int t) {
        const BTile bt = b.vt[t];
        double v[1] = {-INFINITY};
        auto elem = [&](int k) -> double { return (double)b.x[b.vedge[k]]; };
        auto epi = [&](int, double acc) { v[0] = fmax(v[0], acc); };
        const Tile tl = as_tile(bt);
        if (tl.lid < 0) seg_tile<double>(tl, b.vptr, elem, epi, s_acc, s_ptr, nullptr, nullptr);
        else chunk_tile<double>(tl, elem, s_tacc, b.lpart64, b.vlong.lfirst);
        const Red red{0, 0, 1};
        block_combine<1>(v, red, 0, s_wave, s_rec);
        if (threadIdx.x == 0) b.vpart[(size_t)t * QMAX] = s_rec[0];
    };
    for_phase_tiles(b, b.vt, b.nvt, PH_STATS, PH_STATS, body);
}

template <class T>
__global__ __launch_bounds__(BLOCK) void kb_stats_e(BatchDev<T> b)
{
    __shared__ double s_wave[4];
    __shared__ double s_rec[QMAX];
    auto body = [&](int t) {
        const BTile tl = b.et[t];
        double v[1] = {0.0};
        for (int e = tl.i0 + threadIdx.x; e < tl.i1; e += BLOCK) v[0] += (double)b.x[e];
        const Red red{1, 0, 0};
        block_combine<1>(v, red, 0, s_wave, s_rec);
        if (threadIdx.x == 0) b.epart[(size_t)t * QMAX] = s_rec[0];
    };
    for_phase_tiles(b, b.et, b.net, PH_STATS, PH_STATS, body);
}

template <class T>
__global__ __launch_bounds__(BLOCK) void kb_stats_fin(BatchDev<T> b)
{
    __shared__ double s_wave[4];
    __shared__ double s_rec[QMAX];
    __shared__ double s_rec2[QMAX];
    const int k = blockIdx.x;
    Ctl *c = b.ctl + k;
    if (c->phase != PH_STATS) return;
    const Red rmax{0, 0, 1}, rsum{1, 0, 0};
    double lv[1] = {-INFINITY};
    for (int l = b.lrec0[k] + threadIdx.x; l < b.lrec0[k] + b.lrecn[k]; l += BLOCK)
        lv[0] = fmax(lv[0], long_sum<double>(l, b.lpart64, b.vlong.lfirst, b.vlong.lcount));
    block_combine<1>(lv, rmax, 0, s_wave, s_rec2);
    const double lmax = s_rec2[0];
    __syncthreads();
    fold_records<1>(b.vpart + (size_t)b.vrec0[k] * QMAX, b.vrecn[k], rmax, 0, s_wave, s_rec);
    fold_records<1>(b.epart + (size_t)b.erec0[k] * QMAX, b.erecn[k], rsum, 0, s_wave, s_rec2);
    if (threadIdx.x == 0) {
        c->sumx = s_rec2[0];
        c->ymax = c->sP * fmax(s_rec[0], lmax);
        c->zmin = c->sC * s_rec2[0];
        c->phase = PH_IDLE;
        write_stat(b, k, c);
    }
}

// ------------------------------------------------------------------ launchers

#define BLAUNCH(kernel, grid) hipLaunchKernelGGL(kernel, dim3(grid), dim3(BLOCK), 0, st, b)

template <class T>
void batch_slots(const BatchDev<T> &b, const BLaunch &L, int slots, hipStream_t st)
{
    for (int s = 0; s < slots; ++s) {
        BLAUNCH(kb_initx<T>, L.grid_e);
        BLAUNCH(kb_initx_fin<T>, b.nb);
        BLAUNCH(kb_vfwd<T>, L.grid_v);       // INIT_Y instances
        BLAUNCH(kb_vfwd_fin<T>, b.nb);
        BLAUNCH(kb_row<T>, L.grid_w);
        BLAUNCH(kb_row_fin<T>, b.nb);
        BLAUNCH(kb_col<T>, L.grid_e);
        BLAUNCH(kb_col_fin<T>, b.nb);
        BLAUNCH(kb_vfwd<T>, L.grid_v);       // FWD instances
        BLAUNCH(kb_vfwd_fin<T>, b.nb);
        for (int j = 0; j < L.nsearch; ++j) {
            BLAUNCH(kb_search<T>, L.grid_w);
            BLAUNCH(kb_search_fin<T>, b.nb);
        }
        BLAUNCH(kb_stats_v<T>, L.grid_v);
        BLAUNCH(kb_stats_e<T>, L.grid_e);
        BLAUNCH(kb_stats_fin<T>, b.nb);
    }
}

template <class T>
void batch_occupancy(int *per_cu_v, int *per_cu_e)
{
    int a = 0, c = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&a, kb_vfwd<T>, BLOCK, 0) != hipSuccess) a = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&c, kb_col<T>, BLOCK, 0) != hipSuccess) c = 0;
    *per_cu_v = a > 0 ? a : 1;
    *per_cu_e = c > 0 ? c : 1;
}

template void batch_slots<float>(const BatchDev<float> &, const BLaunch &, int, hipStream_t);
template void batch_slots<double>(const BatchDev<double> &, const BLaunch &, int, hipStream_t);
template void batch_occupancy<float>(int *, int *);
template void batch_occupancy<double>(int *, int *);

}  // namespace mwu
