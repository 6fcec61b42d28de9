// Host side of the batched matching program: layout of many instances in
// concatenated arrays, the captured iteration slots, and the outer search
// over M_k of every instance (the same rules as the single-instance driver,
// run per instance while all probes advance together on the device).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>

#include "host.h"

namespace mwu {

namespace {

constexpr double kTuneSeconds = 0.4;   // timed window per candidate layout
constexpr double kMixedQminB = 1.0 / 65536.0;
constexpr int kMaxHalvingsB = 2;

struct Inst {
    int64_t v0 = 0, nv = 0, e0 = 0, ne = 0;   // ranges in the concatenated arrays
    int64_t user_v = 0;                       // vertices as given (before dropping isolated ones)
    double lo0 = 0, hi0 = 0;                  // starting bracket
    double lo = 0, hi = 0, slo = 0, shi = 0, eps_probe = 0, param = 0;
    int halvings = 0, probes = 0, serial = 0;
    int64_t iters = 0, passes = 0, final_iters = 0, evals = 0;
    bool done = false, have_best = false, failed = false;
    double best_scale = 1.0, x_start_scale = 1.0, max_violation = 0.0;
};

}  // namespace

template <class T>
class BatchMatching : public BatchProgram {
  public:
    BatchMatching(Solver &s, const mwu_problem *probs, int32_t count) : s_(s)
    {
        nb_ = count;
        inst_.resize(count);
        std::vector<int32_t> eu, ev, vptr(1, 0), vedge;
        std::vector<BTile> vt, et;
        std::vector<int32_t> vrec0(count), vrecn(count), nedge(count);
        std::vector<int32_t> lrec0(count), lrecn(count), lseg, lfirst, lcount;
        int32_t nslots = 0;
        int64_t V = 0, E = 0;
        for (int32_t k = 0; k < count; ++k) {
            const mwu_problem &p = probs[k];
            if (p.form != MWU_PACKING || p.P.kind != MWU_MAT_INCIDENCE || p.b_P || p.c)
                throw ApiError{MWU_ERR_INVALID_ARG,
                               "batched solve supports matching LPs (PACKING, INCIDENCE, b = c = 1)"};
            const mwu_matrix &m = p.P;
            if (!(m.num_vertices > 0 && m.num_edges > 0 && m.edge_u && m.edge_v))
                throw ApiError{MWU_ERR_INVALID_ARG, "empty or NULL edge list"};
            const int64_t nv = m.num_vertices, ne = m.num_edges;
            // validate: range, self-loops, duplicates
            std::vector<uint64_t> key(ne);
            for (int64_t e = 0; e < ne; ++e) {
                const int64_t a = m.edge_u[e], b = m.edge_v[e];
                if (a < 0 || a >= nv || b < 0 || b >= nv) throw ApiError{MWU_ERR_GRAPH, "vertex id out of range"};
                if (a == b) throw ApiError{MWU_ERR_GRAPH, "self-loop"};
                key[e] = (uint64_t)std::min(a, b) * (uint64_t)nv + (uint64_t)std::max(a, b);
            }
            std::sort(key.begin(), key.end());
            for (int64_t e = 1; e < ne; ++e)
                if (key[e] == key[e - 1]) throw ApiError{MWU_ERR_GRAPH, "duplicate edge"};
            // compact the non-isolated vertices (empty rows never bind)
            std::vector<int64_t> deg(nv, 0), id(nv, -1);
            for (int64_t e = 0; e < ne; ++e) { deg[m.edge_u[e]]++; deg[m.edge_v[e]]++; }
            int64_t kept = 0, maxdeg = 0;
            for (int64_t v = 0; v < nv; ++v)
                if (deg[v] > 0) { id[v] = kept++; maxdeg = std::max(maxdeg, deg[v]); }
            if (V + kept >= INT32_MAX || 2 * (E + ne) >= INT32_MAX)
                throw ApiError{MWU_ERR_TOO_LARGE, "batch exceeds 32-bit device indices"};
            Inst &I = inst_[k];
            I.v0 = V; I.nv = kept; I.e0 = E; I.ne = ne; I.user_v = nv;
            nedge[k] = (int32_t)ne;
            for (int64_t e = 0; e < ne; ++e) {
                eu.push_back((int32_t)(V + id[m.edge_u[e]]));
                ev.push_back((int32_t)(V + id[m.edge_v[e]]));
            }
            // incidence rows: for every vertex its edges (in edge order)
            std::vector<int32_t> cnt(kept + 1, 0);
            for (int64_t e = 0; e < ne; ++e) { cnt[id[m.edge_u[e]] + 1]++; cnt[id[m.edge_v[e]] + 1]++; }
            for (int64_t v = 0; v < kept; ++v) cnt[v + 1] += cnt[v];
            std::vector<int32_t> inc(2 * ne);
            std::vector<int64_t> fill(cnt.begin(), cnt.end() - 1);
            for (int64_t e = 0; e < ne; ++e) {
                inc[fill[id[m.edge_u[e]]]++] = (int32_t)(E + e);
                inc[fill[id[m.edge_v[e]]]++] = (int32_t)(E + e);
            }
            const int64_t base = vedge.size();
            for (int64_t v = 0; v < kept; ++v) vptr.push_back((int32_t)(base + cnt[v + 1]));
            vedge.insert(vedge.end(), inc.begin(), inc.end());
            // nnz-balanced vertex tiles of this instance (never across instances)
            vrec0[k] = (int32_t)vt.size();
            lrec0[k] = (int32_t)lseg.size();
            {
                const TilePlan tp = build_tiles(cnt, kept);
                const int32_t lbase = (int32_t)lseg.size();
                for (const Tile &t : tp.tiles)
                    vt.push_back(BTile{k, (int32_t)(V + t.s0), (int32_t)(V + t.s1), (int32_t)(base + t.k0),
                                       (int32_t)(base + t.k1), t.lid < 0 ? -1 : lbase + t.lid, t.cidx, 0});
                for (size_t l = 0; l < tp.lseg.size(); ++l) {
                    lseg.push_back((int32_t)(V + tp.lseg[l]));
                    lfirst.push_back(nslots + tp.lfirst[l]);
                    lcount.push_back(tp.lcount[l]);
                }
                nslots += tp.nslots;
            }
            vrecn[k] = (int32_t)vt.size() - vrec0[k];
            lrecn[k] = (int32_t)lseg.size() - lrec0[k];
            max_ne_ = std::max(max_ne_, ne);
            // outer-search bracket (as for any packing LP with unit entries):
            // hi = sum_i 1 / min_j P_ji = |E|; lo from the rescaled Algorithm 1 point
            I.hi0 = (double)ne;
            I.lo0 = (double)ne / (double)maxdeg;
            I.x_start_scale = 1.0 / (double)maxdeg;   // x_start = 1/maxdeg on every edge
            V += kept;
            E += ne;
        }
        nv_ = V;
        ne_ = E;
        auto up = [&](DevBuf &b, const void *src, size_t bytes) {
            b.alloc(std::max<size_t>(bytes, 8));
            if (bytes) HIP_OK(hipMemcpy(b.p, src, bytes, hipMemcpyHostToDevice));
        };
        up(eu_, eu.data(), eu.size() * 4);
        up(ev_, ev.data(), ev.size() * 4);
        up(vptr_, vptr.data(), vptr.size() * 4);
        up(vedge_, vedge.data(), vedge.size() * 4);
        up(vt_, vt.data(), vt.size() * sizeof(BTile));
        up(vrec0_, vrec0.data(), count * 4);
        up(vrecn_, vrecn.data(), count * 4);
        up(nedge_, nedge.data(), count * 4);
        up(lrec0_, lrec0.data(), count * 4);
        up(lrecn_, lrecn.data(), count * 4);
        up(lseg_, lseg.data(), lseg.size() * 4);
        up(lfirst_, lfirst.data(), lfirst.size() * 4);
        up(lcount_, lcount.data(), lcount.size() * 4);
        lpart_.alloc(std::max<size_t>((size_t)nslots, 1) * sizeof(T));
        lpart64_.alloc(std::max<size_t>((size_t)nslots, 1) * 8);
        x_.alloc(E * sizeof(T));
        d_.alloc(E * sizeof(T));
        xbest_.alloc(E * sizeof(T));
        y_.alloc(V * sizeof(T));
        dy_.alloc(V * sizeof(T));
        w_.alloc(V * sizeof(T));
        vpart_.alloc(vt.size() * QMAX * 8);
        ctl_.alloc((size_t)count * sizeof(Ctl));
        stat_.alloc((size_t)count * 16);
        HIP_OK(hipMemset(ctl_.p, 0, ctl_.bytes));
        HIP_OK(hipMemset(stat_.p, 0, stat_.bytes));
        HIP_OK(hipHostMalloc((void **)&ctl_host_, (size_t)count * sizeof(Ctl), hipHostMallocDefault));
        HIP_OK(hipHostMalloc((void **)&stat_host_, (size_t)count * 16, hipHostMallocDefault));
        std::memset(ctl_host_, 0, (size_t)count * sizeof(Ctl));
        std::memset(stat_host_, 0, (size_t)count * 16);

        bd_ = BatchDev<T>{};
        bd_.nb = count; bd_.nv = (int32_t)V; bd_.ne = (int32_t)E;
        bd_.vptr = vptr_.as<int32_t>(); bd_.vedge = vedge_.as<int32_t>();
        bd_.eu = eu_.as<int32_t>(); bd_.ev = ev_.as<int32_t>();
        bd_.x = x_.as<T>(); bd_.d = d_.as<T>();
        bd_.y = y_.as<T>(); bd_.dy = dy_.as<T>(); bd_.w = w_.as<T>();
        bd_.vt = vt_.as<BTile>();
        bd_.nvt = (int32_t)vt.size();
        bd_.vrec0 = vrec0_.as<int32_t>(); bd_.vrecn = vrecn_.as<int32_t>();
        bd_.nedge = nedge_.as<int32_t>();
        bd_.vlong = LongSegs{lseg_.as<int32_t>(), lfirst_.as<int32_t>(), lcount_.as<int32_t>(),
                             (int32_t)lseg.size()};
        bd_.lrec0 = lrec0_.as<int32_t>(); bd_.lrecn = lrecn_.as<int32_t>();
        bd_.lpart = lpart_.as<T>(); bd_.lpart64 = lpart64_.as<double>();
        bd_.ctl = ctl_.as<Ctl>();
        bd_.stat = stat_.as<int32_t>();
        bd_.vpart = vpart_.as<double>();
        batch_occupancy<T>(&occ_v_, &occ_e_);
        slots_ = s.opt.iters_per_launch > 0 ? s.opt.iters_per_launch : 8;
        choose_layout();
    }

    ~BatchMatching() override
    {
        if (graph_) (void)hipGraphExecDestroy(graph_);
        if (ctl_host_) (void)hipHostFree(ctl_host_);
        if (stat_host_) (void)hipHostFree(stat_host_);
    }

    int32_t count() const override { return nb_; }
    int64_t total_variables() const override { return ne_; }
    mwu_batch_layout layout() const override { return layout_; }

    void set_layout(const mwu_batch_layout &L) override
    {
        relayout(L);
        layout_.source = MWU_LAYOUT_SET;
        layout_.candidates_timed = 0;
        layout_.edge_iters_per_sec = 0.0;
    }

    void solve(double *x_out, double *obj_out, int64_t *iters_out, mwu_result_info *info) override
    {
        const auto t0 = std::chrono::steady_clock::now();
        const double eps = s_.opt.eps;
        start_all();
        ensure_graph();
        drive(INFINITY);
        HIP_OK(hipStreamSynchronize(s_.stream));
        const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        // outputs
        std::vector<T> xb;
        if (x_out) {
            xb.resize(ne_);
            HIP_OK(hipMemcpy(xb.data(), xbest_.p, ne_ * sizeof(T), hipMemcpyDeviceToHost));
        }
        int64_t total = 0;
        for (int32_t k = 0; k < nb_; ++k) {
            const Inst &I = inst_[k];
            total += I.iters;
            const bool cert = !I.failed && I.hi <= (1.0 + eps) * I.lo;
            if (x_out)
                for (int64_t e = 0; e < I.ne; ++e)
                    x_out[I.e0 + e] = I.have_best ? (double)xb[I.e0 + e] * I.best_scale : I.x_start_scale;
            if (obj_out) obj_out[k] = I.lo;
            if (info) {
                mwu_result_info &r = info[k];
                r.status = cert ? MWU_CERTIFIED : MWU_FEASIBLE_UNCERTIFIED;
                r.objective = I.lo;
                r.lower_bound = I.lo;
                r.upper_bound = I.hi;
                r.total_iterations = I.iters;
                r.final_probe_iterations = I.final_iters;
                r.search_passes = I.passes;
                r.probes = I.probes;
                r.max_violation = I.max_violation;
                r.seconds_solve = secs;
                r.evaluations = I.evals;
            }
        }
        if (iters_out) *iters_out = total;
    }

    void probe_run(const double *params, int32_t max_iters, mwu_probe_info *info) override
    {
        for (int32_t k = 0; k < nb_; ++k)
            if (!(params[k] > 0.0) || !std::isfinite(params[k]))
                throw ApiError{MWU_ERR_INVALID_ARG, "probe parameters must be positive"};
        if (tiled_active_ != nb_) relayout(layout_);
        const int32_t cap_iter = s_.opt.max_iter;
        if (!trace_.p) trace_.alloc((size_t)nb_ * cap_iter * 8);
        for (int32_t k = 0; k < nb_; ++k) {
            Inst &I = inst_[k];
            I.eps_probe = s_.opt.eps;
            I.param = params[k];
            I.done = false;
            configure_probe(k);
            Ctl &c = ctl_host_[k];
            c.trace = trace_.as<double>() + (size_t)k * cap_iter;
            c.trace_cap = cap_iter;
            c.iter_stop = max_iters > 0 ? max_iters : 0;
        }
        push_state();
        ensure_graph();
        // every instance ends its probe (PH_IDLE after the statistics pass)
        // or pauses at the iteration stop (PH_IDLE, still running)
        const int64_t cap = ((int64_t)cap_iter + 8) * 8 / std::max(1, slots_) + 64;
        for (int64_t l = 0;; ++l) {
            if (l > cap) throw ApiError{MWU_ERR_DEVICE, "batched probe did not finish"};
            HIP_OK(hipGraphLaunch(graph_, s_.stream));
            HIP_OK(hipMemcpyAsync(stat_host_, stat_.p, (size_t)nb_ * 16, hipMemcpyDeviceToHost, s_.stream));
            HIP_OK(hipStreamSynchronize(s_.stream));
            bool all = true;
            for (int32_t k = 0; k < nb_ && all; ++k) all = stat_host_[4 * k] == PH_IDLE;
            if (all) break;
        }
        HIP_OK(hipMemcpyAsync(ctl_host_, ctl_.p, (size_t)nb_ * sizeof(Ctl), hipMemcpyDeviceToHost, s_.stream));
        HIP_OK(hipStreamSynchronize(s_.stream));
        for (int32_t k = 0; k < nb_; ++k) {
            inst_[k].done = true;   // a later solve starts every search afresh
            if (!info) continue;
            const Ctl &c = ctl_host_[k];
            mwu_probe_info &r = info[k];
            r.status = c.status;
            r.iterations = c.iter;
            r.search_passes = c.search_passes;
            r.alpha = c.last_alpha;
            r.L_P = c.LP;
            r.L_C = c.LC;
            r.pack_bound = c.pack_bound;
            r.cover_bound = c.cover_bound;
            r.evaluations = c.evaluations;
        }
        probed_ = true;
    }

    void probe_read(int32_t k, int32_t which, double *out, int64_t len) override
    {
        if (!probed_) throw ApiError{MWU_ERR_STATE, "no batched probe has run"};
        if (k < 0 || k >= nb_) throw ApiError{MWU_ERR_INVALID_ARG, "instance out of range"};
        const Inst &I = inst_[k];
        auto get = [&](const T *base, int64_t off, int64_t n) {
            if (len != n) throw ApiError{MWU_ERR_INVALID_ARG, "length mismatch"};
            std::vector<T> t((size_t)std::max<int64_t>(n, 1));
            HIP_OK(hipMemcpy(t.data(), base + off, n * sizeof(T), hipMemcpyDeviceToHost));
            for (int64_t i = 0; i < n; ++i) out[i] = (double)t[i];
        };
        switch (which) {
        case 0: get(x_.as<T>(), I.e0, I.ne); return;
        case 1: get(d_.as<T>(), I.e0, I.ne); return;
        case 4: get(y_.as<T>(), I.v0, I.nv); return;
        case 6: get(dy_.as<T>(), I.v0, I.nv); return;
        case 8: {
            const int64_t it = ctl_host_[k].iter;
            if (len != it) throw ApiError{MWU_ERR_INVALID_ARG, "length mismatch"};
            if (it > 0)
                HIP_OK(hipMemcpy(out, trace_.as<double>() + (size_t)k * s_.opt.max_iter, it * 8,
                                 hipMemcpyDeviceToHost));
            return;
        }
        }
        throw ApiError{MWU_ERR_INVALID_ARG, "unknown vector"};
    }

  private:
    // The outer search of every instance: launch the captured slots, poll the
    // status array, hand finished probes to the host rules and start the next
    // ones, until every search is over or the wall-clock limit has passed
    // (false then).
    bool drive(double seconds)
    {
        const auto t0 = std::chrono::steady_clock::now();
        int64_t launches = 0;
        const int64_t cap = ((int64_t)s_.opt.max_probes * (s_.opt.max_iter + 8) * 4) / std::max(1, slots_) + 64;
        std::vector<int32_t> finished;
        std::vector<int32_t> last((size_t)nb_ * 4, -1);
        int stalled = 0;
        while (true) {
            int active = 0;
            for (const Inst &I : inst_) active += !I.done;
            if (!active) return true;
            if (2 * active <= tiled_active_) {
                retile_active(active);
                ensure_graph();
            }
            if (std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count() > seconds)
                return false;
            if (launches++ > cap) throw ApiError{MWU_ERR_DEVICE, "batched solve did not finish"};
            HIP_OK(hipGraphLaunch(graph_, s_.stream));
            HIP_OK(hipMemcpyAsync(stat_host_, stat_.p, (size_t)nb_ * 16, hipMemcpyDeviceToHost, s_.stream));
            HIP_OK(hipStreamSynchronize(s_.stream));
            // every running instance advances its phase or iteration in a launch
            if (std::equal(last.begin(), last.end(), stat_host_)) {
                if (++stalled > 64) throw ApiError{MWU_ERR_DEVICE, "batched solve makes no progress"};
            } else {
                stalled = 0;
                std::copy(stat_host_, stat_host_ + (size_t)nb_ * 4, last.begin());
            }
            finished.clear();
            for (int32_t k = 0; k < nb_; ++k) {
                const Inst &I = inst_[k];
                if (I.done) continue;
                if (stat_host_[4 * k] == PH_IDLE && stat_host_[4 * k + 3] == I.serial) finished.push_back(k);
            }
            if (finished.empty()) continue;
            HIP_OK(hipMemcpyAsync(ctl_host_, ctl_.p, (size_t)nb_ * sizeof(Ctl), hipMemcpyDeviceToHost, s_.stream));
            HIP_OK(hipStreamSynchronize(s_.stream));
            for (int32_t k : finished) {
                probe_outcome(k);
                if (!inst_[k].done && !next_probe(k)) inst_[k].done = true;
            }
            // nothing runs between the pull above and this push (one stream), so
            // the blocks of running instances go back unchanged
            push_state();
        }
    }

    // Every instance back to the start of its outer search, first probe
    // configured and pushed.
    void start_all()
    {
        if (tiled_active_ != nb_) relayout(layout_);
        for (int32_t k = 0; k < nb_; ++k) {
            Inst &I = inst_[k];
            I.lo = I.lo0; I.hi = I.hi0;
            I.slo = I.lo; I.shi = I.hi; I.eps_probe = s_.opt.eps; I.halvings = 0; I.probes = 0;
            I.iters = I.passes = I.final_iters = I.evals = 0;
            I.done = false; I.have_best = false; I.failed = false; I.best_scale = 1.0;
            I.max_violation = 0.0;
            if (!next_probe(k)) I.done = true;
        }
        push_state();
    }

    // The layout L for the whole batch: tiles, grids and the reported layout.
    void relayout(const mwu_batch_layout &L)
    {
        tile(L, L.tile_edges, L.tile_vertices, false);
        layout_ = L;
        tiled_active_ = nb_;
    }

    // As instances finish their searches, the tiles of the others are
    // rebuilt (finished instances get none) with the tile sizes of the layout
    // halved while the tiles of one kind would not fill one round of resident
    // workgroups: the few instances left at the end of a solve then still
    // spread over the whole chip.  Called between graph launches.
    void retile_active(int active)
    {
        const mwu_batch_layout &L = layout_;
        int64_t ev = 0, vv = 0;
        for (const Inst &I : inst_)
            if (!I.done) { ev += I.ne; vv += I.nv; }
        const int64_t round_e = (int64_t)std::min(occ_e_, L.workgroups_per_cu) * s_.num_cus;
        int32_t te = L.tile_edges, tv = L.tile_vertices;
        while (te > BLOCK && (ev + te - 1) / te < round_e) te /= 2;
        while (tv > BLOCK && (vv + tv - 1) / tv < round_e) tv /= 2;
        tile(L, te % BLOCK ? BLOCK : te, tv % BLOCK ? BLOCK : tv, true);
        tiled_active_ = active;
    }

    // Edge tiles and element tiles of every instance (never across
    // instances; of the instances still searching when active_only), their
    // record buffers and the persistent grids of layout L.
    void tile(const mwu_batch_layout &L, int32_t tile_edges, int32_t tile_vertices, bool active_only)
    {
        std::vector<BTile> et, wt;
        std::vector<int32_t> erec0(nb_), erecn(nb_), wrec0(nb_), wrecn(nb_);
        for (int32_t k = 0; k < nb_; ++k) {
            const Inst &I = inst_[k];
            const bool skip = active_only && I.done;
            wrec0[k] = (int32_t)wt.size();
            for (int64_t i = 0; !skip && i < I.nv; i += tile_vertices)
                wt.push_back(BTile{k, (int32_t)(I.v0 + i), (int32_t)(I.v0 + std::min<int64_t>(i + tile_vertices, I.nv)),
                                   0, 0, -1, 0, 0});
            wrecn[k] = (int32_t)wt.size() - wrec0[k];
            erec0[k] = (int32_t)et.size();
            for (int64_t i = 0; !skip && i < I.ne; i += tile_edges)
                et.push_back(BTile{k, (int32_t)(I.e0 + i), (int32_t)(I.e0 + std::min<int64_t>(i + tile_edges, I.ne)),
                                   0, 0, -1, 0, 0});
            erecn[k] = (int32_t)et.size() - erec0[k];
        }
        if (graph_) {
            HIP_OK(hipStreamSynchronize(s_.stream));
            (void)hipGraphExecDestroy(graph_);
            graph_ = nullptr;
        }
        auto up = [&](DevBuf &b, const void *src, size_t bytes) {
            b.alloc(std::max<size_t>(bytes, 8));
            if (bytes) HIP_OK(hipMemcpy(b.p, src, bytes, hipMemcpyHostToDevice));
        };
        up(et_, et.data(), et.size() * sizeof(BTile));
        up(wt_, wt.data(), wt.size() * sizeof(BTile));
        up(erec0_, erec0.data(), nb_ * 4);
        up(erecn_, erecn.data(), nb_ * 4);
        up(wrec0_, wrec0.data(), nb_ * 4);
        up(wrecn_, wrecn.data(), nb_ * 4);
        epart_.alloc(et.size() * QMAX * 8);
        wpart_.alloc(wt.size() * QMAX * 8);
        bd_.et = et_.as<BTile>(); bd_.net = (int32_t)et.size();
        bd_.erec0 = erec0_.as<int32_t>(); bd_.erecn = erecn_.as<int32_t>();
        bd_.wt = wt_.as<BTile>(); bd_.nwt = (int32_t)wt.size();
        bd_.wrec0 = wrec0_.as<int32_t>(); bd_.wrecn = wrecn_.as<int32_t>();
        bd_.epart = epart_.as<double>(); bd_.wpart = wpart_.as<double>();
        auto grid = [&](int64_t tiles, int occ) {
            const int64_t per_cu = std::min<int64_t>(occ, L.workgroups_per_cu);
            return (int)std::max<int64_t>(1, std::min<int64_t>({tiles, per_cu * s_.num_cus, (int64_t)65535}));
        };
        L_.grid_v = grid(bd_.nvt, occ_v_);
        L_.grid_w = grid(bd_.nwt, occ_e_);
        L_.grid_e = grid(bd_.net, occ_e_);
        L_.nsearch = L.search_launches;
    }

    // Edge-iterations per second of the current layout over the opening of a
    // solve: the whole outer-search loop (probe turnovers included) from the
    // start for a fixed wall-clock window, or to the end if it comes first.
    double rate_current()
    {
        start_all();
        ensure_graph();
        const auto t0 = std::chrono::steady_clock::now();
        const bool all_done = drive(kTuneSeconds);
        const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        double work = 0.0;
        for (int32_t k = 0; k < nb_; ++k) {
            const Inst &I = inst_[k];
            int64_t it = I.iters;
            if (!all_done && !I.done) it += std::max(0, stat_host_[4 * k + 2]);
            work += (double)I.ne * (double)it;
        }
        return secs > 0.0 ? work / secs : 0.0;
    }

    // Layout at create: the built-in one, or with MWU_FLAG_TUNE the process's
    // or the cache file's record for this device and batch shape, else a sweep.
    void choose_layout()
    {
        mwu_batch_layout L = default_layout();
        if (!(s_.opt.flags & MWU_FLAG_TUNE) || (s_.opt.flags & MWU_FLAG_NO_TUNE)) {
            relayout(L);
            return;
        }
        const std::string key = tune_key("batch-matching", s_.fp32, s_.opt.device, s_.num_cus, nb_, nv_, ne_,
                                         max_ne_);
        double r = 0.0;
        if (tune_lookup(key, s_.opt.tune_cache, &L, &r)) {
            relayout(L);
            layout_.source = MWU_LAYOUT_CACHED;
            layout_.candidates_timed = 0;
            layout_.edge_iters_per_sec = r;
            return;
        }
        const std::vector<std::vector<int32_t>> cands = {
            {BLOCK * 8, BLOCK * 16, BLOCK * 32},
            {BLOCK * 4, BLOCK * 8, BLOCK * 16, BLOCK * 32},
            {4, 8},
            {1, 2},
        };
        int timed = 0;
        const mwu_batch_layout best = tune_descent(
            L, cands,
            [&](const mwu_batch_layout &c) {
                relayout(c);
                return rate_current();
            },
            &timed, &r);
        relayout(best);
        HIP_OK(hipStreamSynchronize(s_.stream));
        layout_.source = MWU_LAYOUT_TUNED;
        layout_.candidates_timed = timed;
        layout_.edge_iters_per_sec = r;
        tune_store(key, s_.opt.tune_cache, layout_, r);
    }

    // Configure instance k's next probe in the host copy of its control block
    // (phase PH_INIT); false when its search is over.
    bool next_probe(int32_t k)
    {
        Inst &I = inst_[k];
        const double eps = s_.opt.eps;
        while (true) {
            if (I.probes >= s_.opt.max_probes || I.hi <= (1.0 + eps) * I.lo) return false;
            if (I.shi > (1.0 + eps / 16.0) * I.slo) break;
            if (I.halvings == kMaxHalvingsB) return false;
            ++I.halvings;
            I.eps_probe *= 0.5;
            I.slo = I.lo;
            I.shi = I.hi;
        }
        I.param = std::sqrt(I.slo * I.shi);
        configure_probe(k);
        return true;
    }

    // Instance k's probe at I.param and I.eps_probe in the host copy of its
    // control block (phase PH_INIT), with a new serial number.
    void configure_probe(int32_t k)
    {
        Inst &I = inst_[k];
        Ctl &c = ctl_host_[k];
        std::memset(&c, 0, sizeof(Ctl));
        const int64_t m = I.nv + 1;                              // vertex rows + objective row
        c.eta = 10.0 * std::log((double)m) / I.eps_probe;        // Algorithm 1, natural log
        c.eps = I.eps_probe;
        const double sfac = (s_.opt.flags & MWU_FLAG_NO_FACTOR2) ? 0.5 : 1.0;   // one covering row
        c.step = sfac / c.eta;
        c.sP = 1.0;
        c.sC = 1.0 / I.param;
        c.psi_lim = s_.fp32 ? 80.0 : 700.0;
        c.s2_min = s_.fp32 ? 1e-25 : 1e-280;
        c.qmin = s_.fp32 ? kMixedQminB : 0.0;
        c.psi_shift = s_.fp32 ? 1 : 0;
        c.onesP = 0;
        c.onesC = 1;
        c.step_rule = s_.opt.step_rule;
        c.max_iter = s_.opt.max_iter;
        c.pack_bound = INFINITY;
        c.cover_bound = 0.0;
        c.trace = nullptr;
        c.status = ST_RUNNING;
        c.phase = PH_INIT;
        ++I.serial;
        stat_host_[4 * k + 0] = PH_INIT;      // pushed with the control blocks
        stat_host_[4 * k + 2] = 0;
        stat_host_[4 * k + 3] = I.serial;
    }

    // Apply the finished probe of instance k to its brackets (the packing
    // rules of the single-instance driver).
    void probe_outcome(int32_t k)
    {
        Inst &I = inst_[k];
        const Ctl &c = ctl_host_[k];
        const double cf = s_.fp32 ? 1.0 - kMixedQminB : 1.0;
        I.probes++;
        I.iters += c.iter;
        I.final_iters = c.iter;
        I.passes += c.search_passes;
        I.evals += c.evaluations;
        I.max_violation = std::max({0.0, c.ymax - 1.0, 1.0 - c.zmin});
        if (c.status == ST_NUMERIC) { I.failed = true; I.done = true; return; }
        if (c.pack_bound < I.hi) I.hi = c.pack_bound;
        if (c.status == ST_FEASIBLE) {
            const double val = c.sumx / c.ymax;
            if (val > I.lo) {
                I.lo = val;
                HIP_OK(hipMemcpyAsync(xbest_.as<T>() + I.e0, x_.as<T>() + I.e0, I.ne * sizeof(T),
                                      hipMemcpyDeviceToDevice, s_.stream));
                I.have_best = true;
                I.best_scale = 1.0 / c.ymax;
            }
            I.slo = I.param;
        } else {
            if (c.status == ST_INFEASIBLE) I.hi = std::min(I.hi, I.param / cf);
            I.shi = I.param;
        }
        I.slo = std::max(I.slo, I.lo);
        I.shi = std::min(I.shi, I.hi);
    }

    void push_state()
    {
        HIP_OK(hipMemcpyAsync(ctl_.p, ctl_host_, (size_t)nb_ * sizeof(Ctl), hipMemcpyHostToDevice, s_.stream));
        HIP_OK(hipMemcpyAsync(stat_.p, stat_host_, (size_t)nb_ * 16, hipMemcpyHostToDevice, s_.stream));
    }

    void ensure_graph()
    {
        if (graph_) return;
        hipGraph_t g;
        HIP_OK(hipStreamBeginCapture(s_.stream, hipStreamCaptureModeThreadLocal));
        batch_slots<T>(bd_, L_, slots_, s_.stream);
        HIP_OK(hipStreamEndCapture(s_.stream, &g));
        HIP_OK(hipGraphInstantiate(&graph_, g, nullptr, nullptr, 0));
        (void)hipGraphDestroy(g);
    }

    Solver &s_;
    int32_t nb_ = 0;
    int64_t nv_ = 0, ne_ = 0;
    int64_t max_ne_ = 0;
    int slots_ = 8;
    int occ_v_ = 1, occ_e_ = 1;
    mwu_batch_layout layout_{};
    int32_t tiled_active_ = 0;   // instances the current tiles were built for (nb_: the whole batch)
    std::vector<Inst> inst_;
    BatchDev<T> bd_{};
    BLaunch L_{};
    Ctl *ctl_host_ = nullptr;
    int32_t *stat_host_ = nullptr;
    hipGraphExec_t graph_ = nullptr;
    DevBuf eu_, ev_, vptr_, vedge_, vt_, et_, vrec0_, vrecn_, erec0_, erecn_, nedge_;
    DevBuf lrec0_, lrecn_, lseg_, lfirst_, lcount_, lpart_, lpart64_, wt_, wrec0_, wrecn_, wpart_;
    DevBuf x_, d_, xbest_, y_, dy_, w_, vpart_, epart_, ctl_, stat_;
    DevBuf trace_;          // accepted steps of the probe API's probes (max_iter per instance)
    bool probed_ = false;
};

std::unique_ptr<BatchProgram> make_batch_matching(Solver &s, const mwu_problem *probs, int32_t count)
{
    if (s.fp32) return std::unique_ptr<BatchProgram>(new BatchMatching<float>(s, probs, count));
    return std::unique_ptr<BatchProgram>(new BatchMatching<double>(s, probs, count));
}

}  // namespace mwu
