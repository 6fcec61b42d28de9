// Host side of the fused vertex-cover program: canonical upper and full
// adjacency of the non-isolated vertices, their tiles, and the Program
// interface.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "host.h"

namespace mwu {

// Interleave the bits of a (even positions) and b (odd positions).
static uint64_t morton2(uint32_t a, uint32_t b)
{
    auto spread = [](uint64_t x) {
        x &= 0xffffffffull;
        x = (x | (x << 16)) & 0x0000ffff0000ffffull;
        x = (x | (x << 8)) & 0x00ff00ff00ff00ffull;
        x = (x | (x << 4)) & 0x0f0f0f0f0f0f0f0full;
        x = (x | (x << 2)) & 0x3333333333333333ull;
        x = (x | (x << 1)) & 0x5555555555555555ull;
        return x;
    };
    return spread(a) | (spread(b) << 1);
}

template <class T>
class VcoverProgram : public Program {
  public:
    VcoverProgram(Solver &s, const EdgeList &el, const std::vector<int64_t> &newid, int64_t nv) : s_(s)
    {
        nv_ = nv;
        ne_ = el.ne;
        if (2 * ne_ >= INT32_MAX) throw ApiError{MWU_ERR_TOO_LARGE, "too many edges"};
        // device vertex order: degree descending, ties by compact id, so the
        // neighbours gathered most often share cache lines
        std::vector<int64_t> deg(nv, 0);
        for (int64_t e = 0; e < el.ne; ++e) { deg[newid[el.u[e]]]++; deg[newid[el.v[e]]]++; }
        std::vector<int32_t> order(nv);
        for (int64_t i = 0; i < nv; ++i) order[i] = (int32_t)i;
        std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return deg[a] > deg[b]; });
        dev_.assign(nv, 0);
        for (int64_t r = 0; r < nv; ++r) dev_[order[r]] = (int32_t)r;
        // edges (u, w), u < w in device ids, sorted: rows of the full adjacency
        std::vector<uint64_t> key(el.ne);
        for (int64_t e = 0; e < el.ne; ++e) {
            const int64_t a = dev_[newid[el.u[e]]], b = dev_[newid[el.v[e]]];
            key[e] = (uint64_t)std::min(a, b) * (uint64_t)nv + (uint64_t)std::max(a, b);
        }
        std::sort(key.begin(), key.end());
        std::vector<int32_t> eu(ne_), ew(ne_), fptr(nv + 1, 0), fcol(2 * ne_);
        for (int64_t e = 0; e < ne_; ++e) {
            const int64_t a = key[e] / nv, b = key[e] % nv;
            eu[e] = (int32_t)a;
            ew[e] = (int32_t)b;
            fptr[a + 1]++;
            fptr[b + 1]++;
        }
        for (int64_t v = 0; v < nv; ++v) fptr[v + 1] += fptr[v];
        {
            std::vector<int32_t> fill(fptr.begin(), fptr.end() - 1);
            for (int64_t e = 0; e < ne_; ++e) fcol[fill[ew[e]]++] = eu[e];   // sorted rows
            for (int64_t e = 0; e < ne_; ++e) fcol[fill[eu[e]]++] = ew[e];
        }
        // The edge passes are plain sums over edges, so the edge list is kept
        // in Z-order of (u, w): neighbouring lanes then gather from nearby
        // vertices on both endpoints (about half the cache lines per wave of
        // a row-sorted list on power-law graphs).
        for (int64_t e = 0; e < ne_; ++e) key[e] = morton2((uint32_t)eu[e], (uint32_t)ew[e]);
        std::vector<int64_t> zp(ne_);
        for (int64_t e = 0; e < ne_; ++e) zp[e] = e;
        std::sort(zp.begin(), zp.end(), [&](int64_t a, int64_t b) { return key[a] < key[b]; });
        {
            std::vector<int32_t> t(ne_);
            for (int64_t e = 0; e < ne_; ++e) t[e] = eu[zp[e]];
            eu.swap(t);
            for (int64_t e = 0; e < ne_; ++e) t[e] = ew[zp[e]];
            ew.swap(t);
        }
        key.clear();
        key.shrink_to_fit();
        TilePlan ft = build_tiles(fptr, nv);
        auto up = [&](DevBuf &b, const void *src, size_t bytes) {
            b.alloc(bytes);
            if (bytes) HIP_OK(hipMemcpy(b.p, src, bytes, hipMemcpyHostToDevice));
        };
        up(eu_, eu.data(), eu.size() * 4);
        up(ew_, ew.data(), ew.size() * 4);
        up(fptr_, fptr.data(), fptr.size() * 4);
        up(fcol_, fcol.data(), fcol.size() * 4);
        up(ftiles_, ft.tiles.data(), ft.tiles.size() * sizeof(Tile));
        up(flseg_, ft.lseg.data(), ft.lseg.size() * 4);
        up(flfirst_, ft.lfirst.data(), ft.lfirst.size() * 4);
        up(flcount_, ft.lcount.data(), ft.lcount.size() * 4);
        flpart_.alloc(std::max<int32_t>(ft.nslots, 1) * sizeof(T));
        fcol_pk_.alloc(fcol.size() * 4);
        fptr_pk_.alloc((size_t)(nv + 1) * 4);
        tile_na_.alloc(std::max<size_t>(ft.tiles.size(), 1) * 4);
        nftiles_ = (int64_t)ft.tiles.size();
        ccol_.alloc(fcol.size() * 4);
        cst_.alloc((size_t)(nv + 1) * 4);
        goff_.alloc((size_t)(nftiles_ + 1) * 4);
        items_.alloc(std::max<size_t>(ft.tiles.size(), 1) * sizeof(Tile));
        thead_.alloc((size_t)(nftiles_ + 1) * 4);
        thpos_.alloc((size_t)(nftiles_ + 1) * 4);
        {   // rows per tile, prefix (a chunk tile counts as more rows than a run may hold)
            std::vector<int32_t> rp(nftiles_ + 1, 0);
            for (int64_t t = 0; t < nftiles_; ++t) {
                const Tile &tl = ft.tiles[t];
                rp[t + 1] = rp[t] + (tl.lid >= 0 ? TILE_NZ + 1 : tl.s1 - tl.s0);
            }
            up(tile_rows_, rp.data(), rp.size() * 4);
        }
        aeu_.alloc(std::max<int64_t>(ne_, 1) * 4);
        aew_.alloc(std::max<int64_t>(ne_, 1) * 4);
        xd_.alloc(nv * sizeof(XD<T>));
        xbest_.alloc(nv * sizeof(XD<T>));
        h_.alloc(nv * sizeof(T));
        xs_.alloc(nv * sizeof(T));
        HIP_OK(hipMemset(xd_.p, 0, xd_.bytes));
        partials_.alloc((size_t)GRID_MAX * QMAX * 8);

        vd_ = VcDev<T>{};
        vd_.nv = (int32_t)nv; vd_.ne = (int32_t)ne_;
        vd_.eu = eu_.as<int32_t>(); vd_.ew = ew_.as<int32_t>();
        vd_.fptr = fptr_.as<int32_t>(); vd_.fcol = fcol_.as<int32_t>();
        vd_.ftiles = ftiles_.as<Tile>(); vd_.nftiles = (int32_t)ft.tiles.size();
        vd_.flong = LongSegs{flseg_.as<int32_t>(), flfirst_.as<int32_t>(), flcount_.as<int32_t>(),
                             (int32_t)ft.lseg.size()};
        vd_.flpart = flpart_.as<T>();
        vd_.xd = xd_.as<XD<T>>(); vd_.h = h_.as<T>(); vd_.xs = xs_.as<T>();
        vd_.h_dbg = nullptr; vd_.forced = nullptr;
        vd_.fcol_pk = fcol_pk_.as<int32_t>();
        vd_.fptr_pk = fptr_pk_.as<int32_t>();
        vd_.tile_na = tile_na_.as<int32_t>();
        vd_.ccol = ccol_.as<int32_t>(); vd_.cst = cst_.as<int32_t>(); vd_.goff = goff_.as<int32_t>();
        vd_.tile_rows = tile_rows_.as<int32_t>(); vd_.items = items_.as<Tile>();
        vd_.thead = thead_.as<int32_t>(); vd_.thpos = thpos_.as<int32_t>();
        vd_.aeu = aeu_.as<int32_t>(); vd_.aew = aew_.as<int32_t>();
        // Rows longer than a tile are chunked and the vertices are in degree
        // order, so the long rows are the vertices [0, nlong).  Up to 2 BLOCK
        // of them the pass A finisher completes; more, pass B does (vertex i
        // is long row i).
        for (size_t l = 0; l < ft.lseg.size(); ++l)
            if (ft.lseg[l] != (int32_t)l) throw ApiError{MWU_ERR_DEVICE, "long rows are not the leading vertices"};
        vd_.nlong_b = (int64_t)ft.lseg.size() > 2 * BLOCK ? (int32_t)ft.lseg.size() : 0;
        auto clampg = [](int64_t items, int64_t per, int64_t cap) {
            int64_t g = (items + per - 1) / per;
            return (int)std::max<int64_t>(1, std::min<int64_t>(g, cap));
        };
        int occ_f = 1, occ_e = 1;
        vc_occupancy<T>(&occ_f, &occ_e);
        L_.grid_v = clampg(nv, BLOCK * 2, GRID_MAX);
        // persistent tile and edge grids: one full round of resident workgroups
        L_.grid_ftile = clampg((int64_t)ft.tiles.size(), 1, std::min<int64_t>(GRID_MAX, (int64_t)occ_f * s.num_cus));
        // (at most 4 per CU: measured faster than 5 for the FP32 search, whose
        // per-workgroup combine is then amortized over more edges)
        L_.grid_e = clampg(ne_, BLOCK * 8, std::min<int64_t>(GRID_MAX, (int64_t)std::min(occ_e, 4) * s.num_cus));
        L_.grid_act = clampg(ne_, BLOCK * 16, GRID_MAX);
        acnt_.alloc((size_t)L_.grid_act * 4);
        vd_.acnt = acnt_.as<int32_t>();
        L_.partials = partials_.as<double>();
    }

    int64_t n() const override { return nv_; }
    int64_t mP() const override { return 1; }
    int64_t mC() const override { return ne_; }
    Ctl *ctl() const { return s_.ctl_buf.as<Ctl>(); }

    void probe_init(bool have_x0) override { vc_init<T>(vd_, ctl(), L_, s_.stream, have_x0); }

    void upload_x(const double *host_x) override
    {
        std::vector<double> xv(nv_);
        for (int64_t c = 0; c < nv_; ++c) xv[dev_[c]] = host_x[c];
        DevBuf tmp;
        tmp.alloc(nv_ * 8);
        HIP_OK(hipMemcpyAsync(tmp.p, xv.data(), nv_ * 8, hipMemcpyHostToDevice, s_.stream));
        vc_import_x<T>(vd_, tmp.as<double>(), s_.stream);
        HIP_OK(hipStreamSynchronize(s_.stream));
    }

    // x of the interleaved (x, d) pairs; the probe start copies it to xs
    void scale_x(double th) override { scale_vec<T>(reinterpret_cast<T *>(vd_.xd), nv_, 2, th, s_.stream); }

    void iterations(int slots) override
    {
        for (int i = 0; i < slots; ++i) vc_iteration<T>(vd_, ctl(), L_, s_.stream);
    }

    void final_stats() override { vc_init<T>(vd_, ctl(), L_, s_.stream, true); }

    // Active lists of the sparse passes: built once a probe has run a few
    // iterations, rebuilt when the weight shift has used half the margin (the
    // passes fall back to the full lists once it is used up).  A build costs
    // about one full pass A plus two reads of the edge list.
    void between_launches(const Ctl &c) override
    {
        if (c.eval_mode || c.hold || c.status != ST_RUNNING || c.phase == PH_DONE) return;
        if (c.iter < kActFirstIter) return;
        if (c.act_on) {
            const double drift = c.eta * (c.LC - c.act_L);
            if (drift <= 0.5 * kActMu) return;
        }
        vc_build_active<T>(vd_, ctl(), L_, s_.stream, kActMu);
    }

    void save_best() override
    {
        HIP_OK(hipMemcpyAsync(xbest_.p, xd_.p, xd_.bytes, hipMemcpyDeviceToDevice, s_.stream));
    }

    void best_to_host(double *out) override
    {
        VcDev<T> b = vd_;
        b.xd = xbest_.as<XD<T>>();
        export_to_host(b, 0, nv_, out);
    }

    void read(int which, double *out, int64_t len) override
    {
        switch (which) {
        case 0: need(len, nv_); export_to_host(vd_, 0, nv_, out); return;
        case 1: need(len, nv_); export_to_host(vd_, 1, nv_, out); return;
        case 2: {
            need(len, nv_);
            Ctl c = pull();
            std::fill(out, out + nv_, c.sP);
            return;
        }
        case 3: {
            need(len, nv_);
            if (!hdbg_.p) throw ApiError{MWU_ERR_STATE, "h is recorded by mwu_probe_direction"};
            std::vector<double> t(nv_);
            HIP_OK(hipMemcpyAsync(t.data(), hdbg_.p, nv_ * 8, hipMemcpyDeviceToHost, s_.stream));
            HIP_OK(hipStreamSynchronize(s_.stream));
            for (int64_t c = 0; c < nv_; ++c) out[c] = t[dev_[c]];
            return;
        }
        case 4: need(len, 1); out[0] = pull().y1; return;
        case 6: need(len, 1); out[0] = pull().dy1; return;
        case 5: need(len, ne_); export_to_host(vd_, 2, ne_, out); return;
        case 7: need(len, ne_); export_to_host(vd_, 3, ne_, out); return;
        }
        throw ApiError{MWU_ERR_INVALID_ARG, "unknown vector"};
    }

    void row_pass() override { vc_passA<T>(dbg(), ctl(), L_, s_.stream); }
    void col_pass() override { vc_passB<T>(dbg(), ctl(), L_, s_.stream); }
    void fwd_pass() override {}
    void search_pass() override { vc_search<T>(dbg(), ctl(), L_, s_.stream); }
    void main_kernel(int which) override { vc_main<T>(vd_, ctl(), L_, s_.stream, which); }

    void set_debug(bool on) override
    {
        if (on && !hdbg_.p) hdbg_.alloc(nv_ * 8);
        debug_ = on;
    }

    void resume_search() override { mwu::resume_search(ctl(), vd_.forced, s_.stream); }

    void set_forced(const double *host, int count) override
    {
        if (count > 0) {
            forced_.alloc((size_t)count * 8);
            HIP_OK(hipMemcpy(forced_.p, host, (size_t)count * 8, hipMemcpyHostToDevice));
            vd_.forced = forced_.as<double>();
        } else {
            vd_.forced = nullptr;
        }
        s_.graph_slots = -1;
    }

    void potential(const double *, double *, double, double *, hipStream_t) override
    {
        throw ApiError{MWU_ERR_STATE, "potential is provided by the generic engine (MWU_FLAG_GENERIC)"};
    }

    // Algorithmic bytes of one launch at the current (held) state: over the
    // active lists when the pass runs on them.
    double algo_bytes(int which) const override
    {
        const double t = sizeof(T), V = (double)nv_;
        const PassSize p = pass_size(which);
        switch (which) {
        case 0:   // row starts, columns (+ the work items when packed), x, h
            return p.sparse ? 4.0 * (V + 1) + 4.0 * p.nnz + (double)sizeof(Tile) * p.items + 2.0 * t * V
                            : 4.0 * (V + 1) + 4.0 * p.nnz + 2.0 * t * V;
        case 1: return 4.0 * t * V + t * V;                           // xd read+write, h
        case 3: return 8.0 * p.edges + 2.0 * t * V;                   // eu, ew (active), xd
        }
        return 0.0;
    }
    double pass_nnz(int which) const override
    {
        const PassSize p = pass_size(which);
        return which == 0 ? p.nnz : which == 3 ? p.edges : 0.0;
    }

  private:
    // Nonzeros of pass A and edges of the search at the current state (the
    // same test the kernels make on the control block).
    struct PassSize { bool sparse; double nnz, edges, items; };
    PassSize pass_size(int which) const
    {
        Ctl c;
        HIP_OK(hipMemcpyAsync(&c, ctl(), sizeof(Ctl), hipMemcpyDeviceToHost, s_.stream));
        HIP_OK(hipStreamSynchronize(s_.stream));
        const double Lw = which == 0 ? c.LC : c.LCw;
        PassSize p{c.act_on && (which == 0 || !c.eval_mode) && c.eta * (Lw - c.act_L) <= c.act_mu, 2.0 * (double)ne_,
                   (double)ne_, (double)nftiles_};
        if (!p.sparse) return p;
        p.edges = (double)c.act_ne;
        p.items = (double)c.act_nitems;
        std::vector<int32_t> na(std::max<int64_t>(nftiles_, 1));
        HIP_OK(hipMemcpyAsync(na.data(), tile_na_.p, na.size() * 4, hipMemcpyDeviceToHost, s_.stream));
        HIP_OK(hipStreamSynchronize(s_.stream));
        p.nnz = 0.0;
        for (int64_t i = 0; i < nftiles_; ++i) p.nnz += na[i];
        return p;
    }
    VcDev<T> dbg() const
    {
        VcDev<T> v = vd_;
        if (debug_) v.h_dbg = hdbg_.as<double>();
        return v;
    }
    static void need(int64_t len, int64_t want)
    {
        if (len != want) throw ApiError{MWU_ERR_INVALID_ARG, "length mismatch"};
    }
    Ctl pull()
    {
        Ctl c;
        HIP_OK(hipMemcpyAsync(&c, ctl(), sizeof(Ctl), hipMemcpyDeviceToHost, s_.stream));
        HIP_OK(hipStreamSynchronize(s_.stream));
        return c;
    }
    // Export a vector in the caller's order: vertices by compact id, edges in
    // the canonical order (sorted (min, max) of compact ids).
    void export_to_host(const VcDev<T> &v, int which, int64_t len, double *out)
    {
        DevBuf tmp;
        tmp.alloc(len * 8);
        vc_export<T>(v, which, tmp.as<double>(), s_.stream);
        std::vector<double> t(len);
        HIP_OK(hipMemcpyAsync(t.data(), tmp.p, len * 8, hipMemcpyDeviceToHost, s_.stream));
        HIP_OK(hipStreamSynchronize(s_.stream));
        if (which < 2) {
            for (int64_t c = 0; c < nv_; ++c) out[c] = t[dev_[c]];
            return;
        }
        const std::vector<int64_t> &pos = canonical_edges();
        for (int64_t e = 0; e < ne_; ++e) out[e] = t[pos[e]];
    }

    // canonical edge e -> position in the device edge list (built on first use)
    const std::vector<int64_t> &canonical_edges()
    {
        if ((int64_t)canon_.size() == ne_) return canon_;
        std::vector<int32_t> eu(ne_), ew(ne_), cid(nv_);
        HIP_OK(hipMemcpy(eu.data(), eu_.p, ne_ * 4, hipMemcpyDeviceToHost));
        HIP_OK(hipMemcpy(ew.data(), ew_.p, ne_ * 4, hipMemcpyDeviceToHost));
        for (int64_t c = 0; c < nv_; ++c) cid[dev_[c]] = (int32_t)c;
        std::vector<std::pair<uint64_t, int64_t>> k(ne_);
        for (int64_t e = 0; e < ne_; ++e) {
            const uint64_t a = cid[eu[e]], b = cid[ew[e]];
            k[e] = {std::min(a, b) * (uint64_t)nv_ + std::max(a, b), e};
        }
        std::sort(k.begin(), k.end());
        canon_.resize(ne_);
        for (int64_t e = 0; e < ne_; ++e) canon_[e] = k[e].second;
        return canon_;
    }

    static constexpr double kActMu = 64.0;       // margin, in units of 1 / eta
    static constexpr int kActFirstIter = 8;
    Solver &s_;
    int64_t nv_ = 0, ne_ = 0, nftiles_ = 0;
    bool debug_ = false;
    VcDev<T> vd_{};
    VcLaunch L_{};
    std::vector<int32_t> dev_;     // compact vertex id -> device vertex id
    std::vector<int64_t> canon_;
    DevBuf eu_, ew_, fptr_, fcol_, ftiles_, flseg_, flfirst_, flcount_, flpart_;
    DevBuf xd_, xs_, xbest_, h_, partials_, forced_, hdbg_, fcol_pk_, fptr_pk_, tile_na_, aeu_, aew_, acnt_;
    DevBuf ccol_, cst_, goff_, items_, tile_rows_, thead_, thpos_;
};

std::unique_ptr<Program> make_vcover_program(Solver &s, const EdgeList &el,
                                             const std::vector<int64_t> &newid, int64_t nv)
{
    if (s.fp32) return std::unique_ptr<Program>(new VcoverProgram<float>(s, el, newid, nv));
    return std::unique_ptr<Program>(new VcoverProgram<double>(s, el, newid, nv));
}

}  // namespace mwu
