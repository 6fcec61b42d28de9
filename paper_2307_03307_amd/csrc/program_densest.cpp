// Host side of the fused densest-subgraph program: vertex rows of the
// non-isolated vertices (in vertex order, as the level-set rounding expects),
// edge rows in the caller's edge order, variables 2e / 2e+1 on the two ends.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "host.h"

namespace mwu {

template <class T>
class DensestProgram : public Program {
  public:
    // el: validated edge list; vid: compact id of every vertex (-1 isolated)
    DensestProgram(Solver &s, const EdgeList &el, const std::vector<int64_t> &vid, int64_t nv) : s_(s)
    {
        nv_ = nv;
        ne_ = el.ne;
        n_ = 2 * ne_;
        if (n_ >= INT32_MAX) throw ApiError{MWU_ERR_TOO_LARGE, "too many edges"};
        // Internal vertex ids by descending degree (ties: compact id), so the
        // vertices most edges touch share cache lines.
        std::vector<int64_t> deg(nv, 0);
        for (int64_t e = 0; e < ne_; ++e) { deg[vid[el.u[e]]]++; deg[vid[el.v[e]]]++; }
        int64_t maxdeg = 0;
        for (int64_t v = 0; v < nv; ++v) maxdeg = std::max(maxdeg, deg[v]);
        vorder_.assign(nv, 0);
        std::vector<int32_t> vint(nv);
        {
            std::vector<int64_t> cnt(maxdeg + 2, 0);
            for (int64_t v = 0; v < nv; ++v) cnt[maxdeg - deg[v] + 1]++;
            for (int64_t b = 0; b <= maxdeg; ++b) cnt[b + 1] += cnt[b];
            for (int64_t v = 0; v < nv; ++v) vorder_[cnt[maxdeg - deg[v]]++] = (int32_t)v;
            for (int64_t r = 0; r < nv; ++r) vint[vorder_[r]] = (int32_t)r;
        }
        // Internal edges sorted by (first end, second end), first < second in
        // the internal ids: a stable counting sort by the second end, then by
        // the first.
        std::vector<int32_t> fa(ne_), sb(ne_);
        std::vector<uint8_t> flip(ne_);
        for (int64_t e = 0; e < ne_; ++e) {
            const int32_t a = vint[vid[el.u[e]]], b = vint[vid[el.v[e]]];
            fa[e] = std::min(a, b);
            sb[e] = std::max(a, b);
            flip[e] = a > b;   // the caller's first end is the internal second end
        }
        std::vector<int32_t> tmp(ne_), order(ne_);
        {
            std::vector<int64_t> cnt(nv + 1, 0);
            for (int64_t e = 0; e < ne_; ++e) cnt[sb[e] + 1]++;
            for (int64_t v = 0; v < nv; ++v) cnt[v + 1] += cnt[v];
            for (int64_t e = 0; e < ne_; ++e) tmp[cnt[sb[e]]++] = (int32_t)e;
            std::fill(cnt.begin(), cnt.end(), 0);
            for (int64_t e = 0; e < ne_; ++e) cnt[fa[e] + 1]++;
            for (int64_t v = 0; v < nv; ++v) cnt[v + 1] += cnt[v];
            for (int64_t i = 0; i < ne_; ++i) order[cnt[fa[tmp[i]]]++] = tmp[i];
        }
        edge_of_.assign(order.begin(), order.end());   // internal edge -> caller edge
        std::vector<int32_t> eu(ne_), ev(ne_), vptr(nv + 1, 0), vvar(n_);
        cpos_.resize(n_);
        for (int64_t ie = 0; ie < ne_; ++ie) {
            const int32_t e = order[ie];
            eu[ie] = fa[e];
            ev[ie] = sb[e];
            // caller variable 2e + j (j = 0: the caller's first end)
            cpos_[ie] = (int32_t)(2 * (int64_t)e + (flip[e] ? 1 : 0));
            cpos_[ne_ + ie] = (int32_t)(2 * (int64_t)e + (flip[e] ? 0 : 1));
            vptr[eu[ie] + 1]++;
            vptr[ev[ie] + 1]++;
        }
        for (int64_t v = 0; v < nv; ++v) vptr[v + 1] += vptr[v];
        {
            // the variables of a vertex in increasing position: its first ends
            // (one run of internal edges), then its second ends
            std::vector<int32_t> fill(vptr.begin(), vptr.end() - 1);
            for (int64_t ie = 0; ie < ne_; ++ie) vvar[fill[eu[ie]]++] = (int32_t)ie;
            for (int64_t ie = 0; ie < ne_; ++ie) vvar[fill[ev[ie]]++] = (int32_t)(ne_ + ie);
        }
        TilePlan vt = build_tiles(vptr, nv);
        auto up = [&](DevBuf &b, const void *src, size_t bytes) {
            b.alloc(std::max<size_t>(bytes, 8));
            if (bytes) HIP_OK(hipMemcpy(b.p, src, bytes, hipMemcpyHostToDevice));
        };
        up(eu_, eu.data(), ne_ * 4);
        up(ev_, ev.data(), ne_ * 4);
        up(cpos_d_, cpos_.data(), n_ * 4);
        up(vptr_, vptr.data(), vptr.size() * 4);
        up(vvar_, vvar.data(), vvar.size() * 4);
        up(vtiles_, vt.tiles.data(), vt.tiles.size() * sizeof(Tile));
        up(lseg_, vt.lseg.data(), vt.lseg.size() * 4);
        up(lfirst_, vt.lfirst.data(), vt.lfirst.size() * 4);
        up(lcount_, vt.lcount.data(), vt.lcount.size() * 4);
        lpart_.alloc(std::max<int32_t>(vt.nslots, 1) * 8);
        lpart64_.alloc(std::max<int32_t>(vt.nslots, 1) * 8);
        // x, d, y, z, Pd, Cd in FP64 in both forms; the weights in T
        x_.alloc(n_ * 8); d_.alloc(n_ * 8); xbest_.alloc(n_ * 8);
        y_.alloc(nv * 8); dy_.alloc(nv * 8); w_.alloc(nv * sizeof(T));
        z_.alloc(ne_ * 8); dz_.alloc(ne_ * 8); u_.alloc(ne_ * sizeof(T));
        HIP_OK(hipMemset(x_.p, 0, x_.bytes));
        HIP_OK(hipMemset(d_.p, 0, d_.bytes));
        partials_.alloc((size_t)GRID_MAX * QMAX * 8);
        partials2_.alloc((size_t)GRID_MAX * QMAX * 8);

        dd_ = DnDev<T>{};
        dd_.nv = (int32_t)nv; dd_.ne = (int32_t)ne_; dd_.n = (int32_t)n_;
        dd_.vptr = vptr_.as<int32_t>(); dd_.vvar = vvar_.as<int32_t>();
        dd_.vtiles = vtiles_.as<Tile>(); dd_.nvtiles = (int32_t)vt.tiles.size();
        dd_.vlong = LongSegs{lseg_.as<int32_t>(), lfirst_.as<int32_t>(), lcount_.as<int32_t>(),
                             (int32_t)vt.lseg.size()};
        dd_.lpart = lpart_.as<double>(); dd_.lpart64 = lpart64_.as<double>();
        dd_.eu = eu_.as<int32_t>(); dd_.ev = ev_.as<int32_t>(); dd_.cpos = cpos_d_.as<int32_t>();
        dd_.x = x_.as<double>(); dd_.d = d_.as<double>();
        dd_.y = y_.as<double>(); dd_.dy = dy_.as<double>(); dd_.w = w_.as<T>();
        dd_.z = z_.as<double>(); dd_.dz = dz_.as<double>(); dd_.u = u_.as<T>();
        dd_.g_dbg = nullptr; dd_.h_dbg = nullptr; dd_.forced = nullptr;
        dd_.grad = nullptr; dd_.grad_scale = 0.0;
        vslots_ = vt.nslots;
        int occ_v = 1, occ_s = 1;
        dn_occupancy<T>(&occ_v, &occ_s);
        auto clampg = [](int64_t items, int64_t per, int64_t cap) {
            return (int)std::max<int64_t>(1, std::min<int64_t>((items + per - 1) / per, cap));
        };
        L_.grid_vt = clampg((int64_t)vt.tiles.size(), 1, std::min<int64_t>(GRID_MAX, (int64_t)occ_v * s.num_cus));
        L_.grid_e = clampg(ne_, BLOCK * 4, GRID_MAX);
        L_.grid_n = clampg(n_, BLOCK * 4, GRID_MAX);
        L_.grid_r = clampg(std::max<int64_t>(nv, ne_), BLOCK * 4, GRID_MAX);
        L_.grid_s = clampg(std::max<int64_t>(nv, ne_), BLOCK * 4,
                           std::min<int64_t>(GRID_MAX, (int64_t)occ_s * s.num_cus));
        L_.partials = partials_.as<double>();
        L_.partials2 = partials2_.as<double>();
    }

    int64_t n() const override { return n_; }
    int64_t mP() const override { return nv_; }
    int64_t mC() const override { return ne_; }
    Ctl *ctl() const { return s_.ctl_buf.as<Ctl>(); }

    void probe_init(bool have_x0) override { dn_init<T>(dd_, ctl(), L_, s_.stream, have_x0, nullptr); }

    void upload_x(const double *host_x) override
    {
        std::vector<double> t(n_);
        for (int64_t p = 0; p < n_; ++p) t[p] = host_x[cpos_[p]];
        HIP_OK(hipMemcpyAsync(dd_.x, t.data(), n_ * 8, hipMemcpyHostToDevice, s_.stream));
        HIP_OK(hipStreamSynchronize(s_.stream));
    }

    void scale_x(double th) override { scale_vec<double>(dd_.x, n_, 1, th, s_.stream); }

    void iterations(int slots) override
    {
        for (int i = 0; i < slots; ++i) dn_iteration<T>(dd_, ctl(), L_, s_.stream);
    }

    void final_stats() override { dn_stats<T>(dd_, ctl(), L_, s_.stream); }

    void save_best() override
    {
        HIP_OK(hipMemcpyAsync(xbest_.p, x_.p, n_ * 8, hipMemcpyDeviceToDevice, s_.stream));
    }

    void best_to_host(double *out) override { vars_to_host(xbest_.as<double>(), out); }

    void read(int which, double *out, int64_t len) override
    {
        switch (which) {
        case 0: need(len, n_); vars_to_host(dd_.x, out); return;
        case 1: need(len, n_); vars_to_host(dd_.d, out); return;
        case 2:
        case 3:
            need(len, n_);
            if (!dbg_g_.p) throw ApiError{MWU_ERR_STATE, "g/h are recorded by mwu_probe_direction"};
            vars_to_host(which == 2 ? dbg_g_.as<double>() : dbg_h_.as<double>(), out);
            return;
        case 4: need(len, nv_); rows_to_host(dd_.y, nv_, vorder_, out); return;
        case 6: need(len, nv_); rows_to_host(dd_.dy, nv_, vorder_, out); return;
        case 5: need(len, ne_); rows_to_host(dd_.z, ne_, edge_of_, out); return;
        case 7: need(len, ne_); rows_to_host(dd_.dz, ne_, edge_of_, out); return;
        }
        throw ApiError{MWU_ERR_INVALID_ARG, "unknown vector"};
    }

    void row_pass() override { dn_row_pass<T>(dbg(), ctl(), L_, s_.stream); }
    void col_pass() override { dn_col_pass<T>(dbg(), ctl(), L_, s_.stream); }
    void fwd_pass() override { dn_fwd_pass<T>(dbg(), ctl(), L_, s_.stream); }
    void search_pass() override { dn_search_pass<T>(dbg(), ctl(), L_, s_.stream); }
    void main_kernel(int which) override { dn_main<T>(dd_, ctl(), L_, s_.stream, which); }

    void set_debug(bool on) override
    {
        if (on && !dbg_g_.p) { dbg_g_.alloc(n_ * 8); dbg_h_.alloc(n_ * 8); }
        debug_ = on;
    }

    void resume_search() override { mwu::resume_search(ctl(), dd_.forced, s_.stream); }

    void set_forced(const double *host, int count) override
    {
        if (count > 0) {
            forced_.alloc((size_t)count * 8);
            HIP_OK(hipMemcpy(forced_.p, host, (size_t)count * 8, hipMemcpyHostToDevice));
            dd_.forced = forced_.as<double>();
        } else {
            dd_.forced = nullptr;
        }
        s_.graph_slots = -1;
    }

    void potential(const double *x_dev, double *val_dev, double scale, double *grad_dev,
                   hipStream_t st) override
    {
        // x_dev and grad_dev are in the caller's variable order: the column
        // pass writes grad_dev through the position map
        DnDev<T> g = dd_;
        g.grad = grad_dev;
        g.grad_scale = scale;
        dn_init<T>(g, ctl(), L_, st, true, x_dev);
        dn_row_pass<T>(g, ctl(), L_, st);
        dn_col_pass<T>(g, ctl(), L_, st);
        if (val_dev) potential_finish(nullptr, nullptr, 0, scale, nullptr, nullptr, ctl(), val_dev, st);
    }

    bool potential_static(const double *x_dev, double grad_scale, double *grad_dev, void *scr, size_t bytes,
                          hipStream_t st) override
    {
        // [records of the vertex passes | records of the edge passes | chunk partials]
        auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
        const size_t rec = al((size_t)GRID_MAX * QMAX * 8);
        const size_t lp = al((size_t)std::max<int32_t>(vslots_, 1) * 8);
        if (2 * rec + lp > bytes) return false;
        char *b = static_cast<char *>(scr);
        DnDev<T> g = dd_;
        g.lpart = reinterpret_cast<double *>(b + 2 * rec);
        g.g_dbg = nullptr;
        g.h_dbg = nullptr;
        g.grad = grad_dev;
        g.grad_scale = grad_scale;
        DnLaunch L = L_;
        L.partials = reinterpret_cast<double *>(b);
        L.partials2 = reinterpret_cast<double *>(b + rec);
        dn_init<T>(g, ctl(), L, st, true, x_dev);
        dn_row_pass<T>(g, ctl(), L, st);
        dn_col_pass<T>(g, ctl(), L, st);
        return true;
    }

    // t: bytes of a stored weight; x, d, y, z, dy, dz are 8-byte values
    double algo_bytes(int which) const override
    {
        const double t = sizeof(T), V = (double)nv_, E = (double)ne_;
        switch (which) {
        case 0: return (24.0 + t) * (V + E);                            // y rw, dy, w; z rw, dz, u
        // eu, ev; x, d read and written (2E variables); y (V) and z (E) for
        // the log-domain ratio, or the weights w (V) and u (E) in FP64; Cd
        // written (E)
        case 1: return 8.0 * E + 32.0 * 2.0 * E + 8.0 * (V + E) + 8.0 * E;
        // the vertex rows (the kernel timed for this pass): vptr, vvar, d
        // gathered, Pd written; the edge rows (d read, Cd written) are a
        // separate kernel of 24E bytes
        case 2: return 4.0 * (V + 1) + 4.0 * 2.0 * E + 8.0 * 2.0 * E + 8.0 * V;
        case 3: return (t + 8.0) * V + (t + 16.0) * E;                  // w, dy; u, z, dz
        }
        return 0.0;
    }
    double pass_nnz(int which) const override { return which == 2 ? 2.0 * (double)ne_ : 0.0; }

    // Largest density |E(S_k)| / k over the prefixes S_k of the vertices in
    // descending load (ties to the smaller id): the level-set rounding that
    // gives the outer search its lower bound.  Ranks come from a stable LSD
    // radix sort of the loads on the host; the number of edges of every prefix
    // is the prefix sum, in rank order, of each vertex's neighbours ranked
    // before it, counted on the device.
    bool level_set_density(double *out) override
    {
        const int64_t nv = nv_;
        std::vector<double> load(nv);
        copy_host(dd_.y, nv, load.data());
        std::vector<uint64_t> key(nv), k2(nv);
        std::vector<int32_t> id(nv), id2(nv);
        for (int64_t v = 0; v < nv; ++v) {
            uint64_t b;
            const double l = load[v] > 0.0 ? load[v] : 0.0;
            std::memcpy(&b, &l, 8);
            key[v] = ~b;              // non-negative doubles order as their bits; ~ for descending
            id[v] = (int32_t)v;
        }
        for (int shift = 0; shift < 64; shift += 16) {   // stable: ties keep id order
            std::vector<int64_t> cnt(65537, 0);
            for (int64_t v = 0; v < nv; ++v) cnt[((key[v] >> shift) & 0xffff) + 1]++;
            for (int b = 0; b < 65536; ++b) cnt[b + 1] += cnt[b];
            for (int64_t v = 0; v < nv; ++v) {
                const int64_t p = cnt[(key[v] >> shift) & 0xffff]++;
                k2[p] = key[v];
                id2[p] = id[v];
            }
            key.swap(k2);
            id.swap(id2);
        }
        std::vector<int32_t> rank(nv);
        for (int64_t r = 0; r < nv; ++r) rank[id[r]] = (int32_t)r;
        if (!rank_.p) { rank_.alloc(nv * 4); back_.alloc(nv * 4); }
        HIP_OK(hipMemcpyAsync(rank_.p, rank.data(), nv * 4, hipMemcpyHostToDevice, s_.stream));
        dn_backcounts<T>(dd_, rank_.as<int32_t>(), back_.as<int32_t>(), s_.stream);
        std::vector<int32_t> back(nv);
        HIP_OK(hipMemcpyAsync(back.data(), back_.p, nv * 4, hipMemcpyDeviceToHost, s_.stream));
        HIP_OK(hipStreamSynchronize(s_.stream));
        double best = 0.0;
        int64_t edges = 0;
        for (int64_t r = 0; r < nv; ++r) {
            edges += back[id[r]];
            best = std::max(best, (double)edges / (double)(r + 1));
        }
        *out = best;
        return true;
    }

  private:
    DnDev<T> dbg() const
    {
        DnDev<T> g = dd_;
        if (debug_) { g.g_dbg = dbg_g_.as<double>(); g.h_dbg = dbg_h_.as<double>(); }
        return g;
    }
    static void need(int64_t len, int64_t want)
    {
        if (len != want) throw ApiError{MWU_ERR_INVALID_ARG, "length mismatch"};
    }
    // internal variables (first ends, second ends) -> the caller's order,
    // permuted on the device before the copy
    void vars_to_host(const double *src, double *out)
    {
        if (!export_.p) export_.alloc(n_ * 8);
        dn_to_caller(src, dd_.cpos, export_.as<double>(), n_, s_.stream);
        copy_host(export_.as<double>(), n_, out);
    }
    // internal rows -> the caller's order (map: internal index -> caller index)
    void rows_to_host(const double *src, int64_t len, const std::vector<int32_t> &map, double *out)
    {
        std::vector<double> t(len);
        copy_host(src, len, t.data());
        for (int64_t i = 0; i < len; ++i) out[map[i]] = t[i];
    }

    void copy_host(const double *src, int64_t len, double *out)
    {
        HIP_OK(hipMemcpyAsync(out, src, len * 8, hipMemcpyDeviceToHost, s_.stream));
        HIP_OK(hipStreamSynchronize(s_.stream));
    }

    Solver &s_;
    int64_t nv_ = 0, ne_ = 0, n_ = 0;
    bool debug_ = false;
    DnDev<T> dd_{};
    DnLaunch L_{};
    DevBuf eu_, ev_, vptr_, vvar_, vtiles_, lseg_, lfirst_, lcount_, lpart_, lpart64_;
    DevBuf x_, d_, xbest_, y_, dy_, w_, z_, dz_, u_, partials_, partials2_, forced_, dbg_g_, dbg_h_;
    DevBuf rank_, back_, cpos_d_, export_;
    std::vector<int32_t> cpos_;     // internal variable -> caller variable (2e + j)
    std::vector<int32_t> vorder_;   // internal vertex -> compact vertex id (vertex order)
    std::vector<int32_t> edge_of_;  // internal edge -> caller edge
    int32_t vslots_ = 0;   // chunk partial slots of the long vertex rows
};

std::unique_ptr<Program> make_densest_program(Solver &s, const EdgeList &el, const std::vector<int64_t> &vid,
                                              int64_t nv)
{
    if (s.fp32) return std::unique_ptr<Program>(new DensestProgram<float>(s, el, vid, nv));
    return std::unique_ptr<Program>(new DensestProgram<double>(s, el, vid, nv));
}

}  // namespace mwu
