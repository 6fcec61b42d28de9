// Host side of the generic CSR engine: device layout of the concatenated row
// structure and its transpose, nnz-balanced tiles, and the Program interface.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "host.h"

namespace mwu {

// Split segments [0, nseg) of a CSR-like pointer array into tiles of at most
// TILE_NZ nonzeros and TILE_NZ segments; longer segments become chunk tiles.
TilePlan build_tiles(const std::vector<int32_t> &ptr, int64_t nseg)
{
    TilePlan tp;
    int64_t s = 0;
    while (s < nseg) {
        const int64_t len = (int64_t)ptr[s + 1] - ptr[s];
        if (len > TILE_NZ) {
            const int32_t lid = (int32_t)tp.lfirst.size();
            const int32_t nch = (int32_t)((len + TILE_NZ - 1) / TILE_NZ);
            tp.lseg.push_back((int32_t)s);
            tp.lfirst.push_back(tp.nslots);
            tp.lcount.push_back(nch);
            tp.nslots += nch;
            for (int32_t c = 0; c < nch; ++c) {
                Tile t;
                t.s0 = (int32_t)s; t.s1 = (int32_t)(s + 1);
                t.k0 = ptr[s] + c * TILE_NZ;
                t.k1 = std::min<int64_t>((int64_t)ptr[s] + (int64_t)(c + 1) * TILE_NZ, ptr[s + 1]);
                t.lid = lid; t.cidx = c;
                tp.tiles.push_back(t);
            }
            ++s;
            continue;
        }
        const int64_t s0 = s;
        const int64_t k0 = ptr[s];
        while (s < nseg && (int64_t)ptr[s + 1] - k0 <= TILE_NZ && s - s0 < TILE_NZ) ++s;
        Tile t;
        t.s0 = (int32_t)s0; t.s1 = (int32_t)s; t.k0 = (int32_t)k0; t.k1 = ptr[s];
        t.lid = -1; t.cidx = 0;
        tp.tiles.push_back(t);
    }
    return tp;
}

// Whether the generic engine lays out its columns and rows by length: the
// flags decide when set; otherwise heavy-tailed column lengths (at least
// 4096 columns, the longest at least 32 times the mean) do.
static bool locality_order(uint64_t flags, const std::vector<int64_t> &clen, int64_t nnz)
{
    if (flags & MWU_FLAG_KEEP_ORDER) return false;
    if (flags & MWU_FLAG_LOCALITY_ORDER) return true;
    const int64_t n = (int64_t)clen.size();
    if (n < 4096 || nnz == 0) return false;
    const int64_t longest = *std::max_element(clen.begin(), clen.end());
    return (double)longest >= 32.0 * (double)nnz / (double)n;
}

template <class T>
class GenericProgram : public Program {
  public:
    GenericProgram(Solver &s, const HostCSR *P, const HostCSR *C, int64_t obj_row) : s_(s)
    {
        const int64_t mPc = s.onesP ? 0 : P->rows;
        const int64_t mCc = s.onesC ? 0 : C->rows;
        n_ = s.onesP ? C->cols : P->cols;
        mPc_ = mPc;
        mR_ = mPc + mCc;
        if (mR_ < 1) throw ApiError{MWU_ERR_INVALID_ARG, "no explicit constraint rows"};
        const bool vals = (!s.onesP && !P->val.empty()) || (!s.onesC && !C->val.empty()) || obj_row >= 0;
        const int64_t nnz = (s.onesP ? 0 : P->nnz()) + (s.onesC ? 0 : C->nnz());
        if (nnz >= INT32_MAX || mR_ >= INT32_MAX || n_ >= INT32_MAX)
            throw ApiError{MWU_ERR_TOO_LARGE, "structure exceeds 32-bit device indices"};
        // concatenated row r < mPc is row r of P, else row r - mPc of C
        auto side = [&](int64_t r) -> const HostCSR & { return r < mPc ? *P : *C; };
        auto local = [&](int64_t r) { return r < mPc ? r : r - mPc; };
        // ---- internal order: columns by length, rows of each side by length
        // (descending, stable) when the column lengths are heavy-tailed
        std::vector<int64_t> clen(n_, 0);
        if (!s.onesP) for (auto c : P->idx) clen[c]++;
        if (!s.onesC) for (auto c : C->idx) clen[c]++;
        reorder_ = locality_order(s.opt.flags, clen, nnz);
        cperm_.resize(n_);
        rperm_.resize(mR_);
        for (int64_t i = 0; i < n_; ++i) cperm_[i] = (int32_t)i;
        for (int64_t r = 0; r < mR_; ++r) rperm_[r] = (int32_t)r;
        if (reorder_) {
            std::stable_sort(cperm_.begin(), cperm_.end(), [&](int32_t a, int32_t b) { return clen[a] > clen[b]; });
            auto rlen = [&](int32_t r) { const HostCSR &A = side(r); return A.ptr[local(r) + 1] - A.ptr[local(r)]; };
            auto longer = [&](int32_t a, int32_t b) { return rlen(a) > rlen(b); };
            std::stable_sort(rperm_.begin(), rperm_.begin() + mPc, longer);
            std::stable_sort(rperm_.begin() + mPc, rperm_.end(), longer);
        }
        std::vector<int32_t> cinv(n_), rinv(mR_);
        for (int64_t i = 0; i < n_; ++i) cinv[cperm_[i]] = (int32_t)i;
        for (int64_t r = 0; r < mR_; ++r) rinv[rperm_[r]] = (int32_t)r;
        const int64_t obj_int = obj_row >= 0 ? rinv[obj_row] : -1;
        // concatenated row structure in the internal order, its exact FP64
        // coefficients (certificate statistics) and max_j P_ji per column
        // (Algorithm 1 initial point; an objective row in P enters at each
        // probe, since its level changes)
        std::vector<int32_t> rptr(mR_ + 1), rcol(nnz);
        std::vector<T> rval(vals ? nnz : 0);
        std::vector<double> r64(vals ? nnz : 0);
        std::vector<double> colmax(s.onesP ? 0 : n_, 0.0);
        std::vector<std::pair<int32_t, double>> row;
        int64_t k = 0;
        for (int64_t r = 0; r < mR_; ++r) {
            rptr[r] = (int32_t)k;
            const int64_t kr = rperm_[r];
            const HostCSR &A = side(kr);
            const int64_t li = local(kr);
            row.clear();
            for (int64_t q = A.ptr[li]; q < A.ptr[li + 1]; ++q) row.emplace_back(cinv[A.idx[q]], A.v(q));
            if (reorder_) std::sort(row.begin(), row.end());
            for (const auto &e : row) {
                rcol[k] = e.first;
                if (vals) { rval[k] = (T)e.second; r64[k] = e.second; }
                if (r < mPc && r != obj_int) colmax[e.first] = std::max(colmax[e.first], e.second);
                ++k;
            }
        }
        rptr[mR_] = (int32_t)k;
        // column structure (transpose); rows visited in order keep each column sorted
        std::vector<int32_t> cptr(n_ + 1, 0), crow(nnz);
        std::vector<T> cval(vals ? nnz : 0);
        for (int64_t q = 0; q < nnz; ++q) cptr[rcol[q] + 1]++;
        for (int64_t i = 0; i < n_; ++i) cptr[i + 1] += cptr[i];
        std::vector<int32_t> opos;   // positions of the objective row's entries in the column structure
        {
            std::vector<int32_t> fill(cptr.begin(), cptr.end() - 1);
            for (int64_t rr = 0; rr < mR_; ++rr)
                for (int32_t q = rptr[rr]; q < rptr[rr + 1]; ++q) {
                    const int32_t pos = fill[rcol[q]]++;
                    crow[pos] = (int32_t)rr;
                    if (vals) cval[pos] = rval[q];
                    if (rr == obj_int) opos.push_back(pos);
                }
        }
        if (obj_row >= 0) {
            // the row covers every column, its entries in internal column order
            obj_k0_ = rptr[obj_int];
            obj_n_ = rptr[obj_int + 1] - rptr[obj_int];
            obj_in_P_ = obj_int < mPc;
        }
        nnz_ = nnz;
        vals_ = vals;
        TilePlan rt = build_tiles(rptr, mR_);
        TilePlan ct = build_tiles(cptr, n_);

        auto up = [&](DevBuf &b, const void *src, size_t bytes) {
            b.alloc(bytes);
            if (bytes) HIP_OK(hipMemcpy(b.p, src, bytes, hipMemcpyHostToDevice));
        };
        up(rptr_, rptr.data(), rptr.size() * 4);
        up(rcol_, rcol.data(), rcol.size() * 4);
        up(rval_, rval.data(), rval.size() * sizeof(T));
        up(cptr_, cptr.data(), cptr.size() * 4);
        up(crow_, crow.data(), crow.size() * 4);
        up(cval_, cval.data(), cval.size() * sizeof(T));
        up(colmax_, colmax.data(), colmax.size() * 8);
        if (obj_row >= 0) {
            up(opos_, opos.data(), opos.size() * 4);
            up(colmax_base_, colmax.data(), colmax.size() * 8);
        }
        up(rtiles_, rt.tiles.data(), rt.tiles.size() * sizeof(Tile));
        up(ctiles_, ct.tiles.data(), ct.tiles.size() * sizeof(Tile));
        up(rlseg_, rt.lseg.data(), rt.lseg.size() * 4);
        up(rlfirst_, rt.lfirst.data(), rt.lfirst.size() * 4);
        up(rlcount_, rt.lcount.data(), rt.lcount.size() * 4);
        up(clseg_, ct.lseg.data(), ct.lseg.size() * 4);
        up(clfirst_, ct.lfirst.data(), ct.lfirst.size() * 4);
        up(clcount_, ct.lcount.data(), ct.lcount.size() * 4);
        rlpart_.alloc(std::max<int32_t>(rt.nslots, 1) * sizeof(T));
        rlpart64_.alloc(std::max<int32_t>(rt.nslots, 1) * sizeof(double));
        if (vals) up(rval64_, r64.data(), r64.size() * 8);   // exact coefficients, FP64 statistics
        if (reorder_) up(cmap_, cperm_.data(), cperm_.size() * 4);
        clpart_.alloc(std::max<int32_t>(ct.nslots, 1) * 2 * sizeof(T));
        x_.alloc(n_ * sizeof(T));
        d_.alloc(n_ * sizeof(T));
        xbest_.alloc(n_ * sizeof(T));
        yz_.alloc(mR_ * sizeof(T));
        dyz_.alloc(mR_ * sizeof(T));
        wu_.alloc(mR_ * sizeof(T));
        HIP_OK(hipMemset(d_.p, 0, d_.bytes));
        HIP_OK(hipMemset(dyz_.p, 0, dyz_.bytes));
        partials_.alloc((size_t)GRID_MAX * QMAX * 8);

        gd_ = GenericDev<T>{};
        gd_.n = (int32_t)n_; gd_.mPc = (int32_t)mPc_; gd_.mR = (int32_t)mR_;
        gd_.rptr = rptr_.as<int32_t>(); gd_.rcol = rcol_.as<int32_t>(); gd_.rval = vals ? rval_.as<T>() : nullptr;
        gd_.rtiles = rtiles_.as<Tile>(); gd_.nrtiles = (int32_t)rt.tiles.size();
        gd_.cptr = cptr_.as<int32_t>(); gd_.crow = crow_.as<int32_t>(); gd_.cval = vals ? cval_.as<T>() : nullptr;
        gd_.ctiles = ctiles_.as<Tile>(); gd_.nctiles = (int32_t)ct.tiles.size();
        gd_.colmaxP = s.onesP ? nullptr : colmax_.as<double>();
        gd_.rlong = LongSegs{rlseg_.as<int32_t>(), rlfirst_.as<int32_t>(), rlcount_.as<int32_t>(),
                             (int32_t)rt.lseg.size()};
        gd_.clong = LongSegs{clseg_.as<int32_t>(), clfirst_.as<int32_t>(), clcount_.as<int32_t>(),
                             (int32_t)ct.lseg.size()};
        gd_.rlpart = rlpart_.as<T>(); gd_.clpart = clpart_.p; gd_.rlpart64 = rlpart64_.as<double>();
        gd_.x = x_.as<T>(); gd_.d = d_.as<T>(); gd_.yz = yz_.as<T>(); gd_.dyz = dyz_.as<T>();
        gd_.wu = wu_.as<T>();
        gd_.g_dbg = nullptr; gd_.h_dbg = nullptr; gd_.forced = nullptr;
        gd_.grad = nullptr; gd_.grad_scale = 0.0;
        gd_.cmap = reorder_ ? cmap_.as<int32_t>() : nullptr;
        rslots_ = rt.nslots;
        cslots_ = ct.nslots;

        auto clampg = [](int64_t items, int64_t per) {
            int64_t g = (items + per - 1) / per;
            return (int)std::max<int64_t>(1, std::min<int64_t>(g, GRID_MAX));
        };
        L_.grid_elem_rows = clampg(mR_, BLOCK * 2);
        L_.grid_elem_cols = clampg(n_, BLOCK * 2);
        int occ_f = 1, occ_c = 1, occ_s = 1;
        generic_occupancy<T>(&occ_f, &occ_c, &occ_s);
        auto round1 = [&](int64_t items, int64_t per, int occ) {   // one full round of workgroups
            return (int)std::max<int64_t>(1, std::min<int64_t>({(items + per - 1) / per, (int64_t)GRID_MAX,
                                                               (int64_t)occ * s.num_cus}));
        };
        L_.grid_rtile = round1((int64_t)rt.tiles.size(), 1, occ_f);
        L_.grid_ctile = round1((int64_t)ct.tiles.size(), 1, occ_c);
        L_.grid_search = round1(mR_, BLOCK * 4, occ_s);
        L_.partials = partials_.as<double>();
    }

    int64_t n() const override { return n_; }
    int64_t mP() const override { return s_.onesP ? 1 : mPc_; }
    int64_t mC() const override { return s_.onesC ? 1 : mR_ - mPc_; }

    Ctl *ctl() const { return s_.ctl_buf.as<Ctl>(); }

    void probe_init(bool have_x0) override { generic_init<T>(gd_, ctl(), L_, s_.stream, have_x0); }

    void upload_x(const double *host_x) override
    {
        std::vector<double> hx;
        if (reorder_) {
            hx.resize(n_);
            for (int64_t i = 0; i < n_; ++i) hx[i] = host_x[cperm_[i]];
            host_x = hx.data();
        }
        DevBuf tmp;
        tmp.alloc(n_ * 8);
        HIP_OK(hipMemcpyAsync(tmp.p, host_x, n_ * 8, hipMemcpyHostToDevice, s_.stream));
        narrow<T>(tmp.as<double>(), gd_.x, n_, s_.stream);
        HIP_OK(hipStreamSynchronize(s_.stream));
    }

    void scale_x(double th) override { scale_vec<T>(gd_.x, n_, 1, th, s_.stream); }

    void set_objective_level(double v) override
    {
        if (obj_n_ <= 0) throw ApiError{MWU_ERR_STATE, "no objective row"};
        generic_set_row<T>(rval_.as<T>(), rval64_.as<double>(), obj_k0_, obj_n_, cval_.as<T>(), opos_.as<int32_t>(), v,
                           obj_in_P_ ? colmax_.as<double>() : nullptr, colmax_base_.as<double>(), s_.stream);
    }

    void iterations(int slots) override
    {
        for (int i = 0; i < slots; ++i) generic_iteration<T>(gd_, ctl(), L_, s_.stream);
    }

    void final_stats() override
    {
        generic_stats<T>(gd_, ctl(), L_, s_.stream, rval64_.p ? rval64_.as<double>() : nullptr);
    }

    void save_best() override
    {
        HIP_OK(hipMemcpyAsync(xbest_.p, x_.p, n_ * sizeof(T), hipMemcpyDeviceToDevice, s_.stream));
    }

    void best_to_host(double *out) override { to_host(xbest_.as<T>(), n_, out, cols_out()); }

    // Every vector leaves in the caller's order: column i of the internal
    // order is the caller's cperm_[i], row r is the caller's rperm_[r].
    void read(int which, double *out, int64_t len) override
    {
        const int64_t mCc = mR_ - mPc_;
        switch (which) {
        case 0: need(len, n_); to_host(gd_.x, n_, out, cols_out()); return;
        case 1: need(len, n_); to_host(gd_.d, n_, out, cols_out()); return;
        case 2:
        case 3: {
            need(len, n_);
            if (!dbg_g_.p) throw ApiError{MWU_ERR_STATE, "g/h are recorded by mwu_probe_direction"};
            std::vector<double> tmp(n_);
            HIP_OK(hipMemcpyAsync(tmp.data(), which == 2 ? dbg_g_.p : dbg_h_.p, n_ * 8, hipMemcpyDeviceToHost,
                                  s_.stream));
            HIP_OK(hipStreamSynchronize(s_.stream));
            for (int64_t i = 0; i < n_; ++i) out[reorder_ ? cperm_[i] : i] = tmp[i];
            return;
        }
        case 4:
        case 6:
            if (s_.onesP) { need(len, 1); out[0] = scalar(which == 4 ? 0 : 2); return; }
            need(len, mPc_);
            to_host((which == 4 ? gd_.yz : gd_.dyz), mPc_, out, rows_out(0));
            return;
        case 5:
        case 7:
            if (s_.onesC) { need(len, 1); out[0] = scalar(which == 5 ? 1 : 3); return; }
            need(len, mCc);
            to_host((which == 5 ? gd_.yz : gd_.dyz) + mPc_, mCc, out, rows_out(mPc_));
            return;
        }
        throw ApiError{MWU_ERR_INVALID_ARG, "unknown vector"};
    }

    void row_pass() override { generic_row<T>(dbg_gd(), ctl(), L_, s_.stream); }
    void col_pass() override { generic_col<T>(dbg_gd(), ctl(), L_, s_.stream); }
    void fwd_pass() override { generic_fwd<T>(dbg_gd(), ctl(), L_, s_.stream); }
    void search_pass() override { generic_search<T>(dbg_gd(), ctl(), L_, s_.stream); }
    void main_kernel(int which) override { generic_main<T>(gd_, ctl(), L_, s_.stream, which); }

    void set_debug(bool on) override
    {
        if (on && !dbg_g_.p) { dbg_g_.alloc(n_ * 8); dbg_h_.alloc(n_ * 8); }
        debug_ = on;
    }

    void resume_search() override { mwu::resume_search(ctl(), gd_.forced, s_.stream); }

    void set_forced(const double *host, int count) override
    {
        if (count > 0) {
            forced_.alloc((size_t)count * 8);
            HIP_OK(hipMemcpy(forced_.p, host, (size_t)count * 8, hipMemcpyHostToDevice));
            gd_.forced = forced_.as<double>();
        } else {
            gd_.forced = nullptr;
        }
        s_.graph_slots = -1;   // graph holds the old parameters: recapture
    }

    void potential(const double *x_dev, double *val_dev, double scale, double *grad_dev,
                   hipStream_t st) override
    {
        set_debug(true);
        GenericDev<T> g = dbg_gd();
        generic_load_x<T>(g, ctl(), L_, st, x_dev);
        generic_row<T>(g, ctl(), L_, st);
        generic_col<T>(g, ctl(), L_, st);
        if (grad_dev || val_dev)
            potential_finish(dbg_g_.as<double>(), dbg_h_.as<double>(), grad_dev ? (int)n_ : 0, scale,
                             grad_dev, gd_.cmap, ctl(), val_dev, st);
    }

    bool potential_static(const double *x_dev, double grad_scale, double *grad_dev, void *scr, size_t bytes,
                          hipStream_t st) override
    {
        // [reduction records | row chunk partials | column chunk partials]
        auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
        const size_t rec = al((size_t)GRID_MAX * QMAX * 8);
        const size_t rl = al((size_t)std::max<int32_t>(rslots_, 1) * sizeof(T));
        const size_t cl = al((size_t)std::max<int32_t>(cslots_, 1) * 2 * sizeof(T));
        if (rec + rl + cl > bytes) return false;
        char *b = static_cast<char *>(scr);
        GenericDev<T> g = gd_;
        g.rlpart = reinterpret_cast<T *>(b + rec);
        g.clpart = b + rec + rl;
        g.g_dbg = nullptr;
        g.h_dbg = nullptr;
        g.grad = grad_dev;
        g.grad_scale = grad_scale;
        Launch L = L_;
        L.partials = reinterpret_cast<double *>(b);
        generic_load_x<T>(g, ctl(), L, st, x_dev);
        generic_row<T>(g, ctl(), L, st);
        generic_col<T>(g, ctl(), L, st);
        return true;
    }

    double algo_bytes(int which) const override
    {
        const double t = sizeof(T), nnz = (double)nnz_, vb = vals_ ? t : 0.0;
        switch (which) {
        case 0: return 4.0 * t * mR_;
        case 1: return 4.0 * (n_ + 1) + (4.0 + vb) * nnz + t * mR_ + 4.0 * t * n_;
        case 2: return 4.0 * (mR_ + 1) + (4.0 + vb) * nnz + t * n_ + t * mR_;
        case 3: return 3.0 * t * mR_;
        }
        return 0.0;
    }
    double pass_nnz(int which) const override { return (which == 1 || which == 2) ? (double)nnz_ : 0.0; }

  private:
    GenericDev<T> dbg_gd() const
    {
        GenericDev<T> g = gd_;
        if (debug_) { g.g_dbg = dbg_g_.as<double>(); g.h_dbg = dbg_h_.as<double>(); }
        return g;
    }
    static void need(int64_t len, int64_t want)
    {
        if (len != want) throw ApiError{MWU_ERR_INVALID_ARG, "length mismatch"};
    }
    double scalar(int which)
    {
        Ctl c;
        HIP_OK(hipMemcpyAsync(&c, ctl(), sizeof(Ctl), hipMemcpyDeviceToHost, s_.stream));
        HIP_OK(hipStreamSynchronize(s_.stream));
        return which == 0 ? c.y1 : which == 1 ? c.z1 : which == 2 ? c.dy1 : c.dz1;
    }
    // map (nullable): internal index i goes to out[map[i] - base]
    struct OutMap { const int32_t *map; int64_t base; };
    OutMap cols_out() const { return {reorder_ ? cperm_.data() : nullptr, 0}; }
    OutMap rows_out(int64_t base) const { return {reorder_ ? rperm_.data() + base : nullptr, base}; }
    void to_host(const T *src, int64_t len, double *out, OutMap m = {nullptr, 0})
    {
        if (len == 0) return;
        DevBuf tmp;
        tmp.alloc(len * 8);
        widen<T>(src, tmp.as<double>(), len, s_.stream);
        std::vector<double> h;
        double *dst = out;
        if (m.map) { h.resize(len); dst = h.data(); }
        HIP_OK(hipMemcpyAsync(dst, tmp.p, len * 8, hipMemcpyDeviceToHost, s_.stream));
        HIP_OK(hipStreamSynchronize(s_.stream));
        if (m.map) for (int64_t i = 0; i < len; ++i) out[m.map[i] - m.base] = h[i];
    }

    Solver &s_;
    int64_t n_ = 0, mPc_ = 0, mR_ = 0, nnz_ = 0;
    bool vals_ = false;
    bool debug_ = false;
    GenericDev<T> gd_{};
    Launch L_{};
    DevBuf rptr_, rcol_, rval_, cptr_, crow_, cval_, colmax_, rtiles_, ctiles_;
    DevBuf rlseg_, rlfirst_, rlcount_, clseg_, clfirst_, clcount_, rlpart_, clpart_, rlpart64_, rval64_;
    DevBuf x_, d_, xbest_, yz_, dyz_, wu_, partials_, forced_, dbg_g_, dbg_h_;
    int32_t rslots_ = 0, cslots_ = 0;   // chunk partial slots of the long rows and columns
    DevBuf opos_, colmax_base_;         // embedded objective row: its column positions, colmax without it
    bool reorder_ = false;              // internal order by length (locality_order)
    std::vector<int32_t> cperm_, rperm_;   // internal column / row -> the caller's
    DevBuf cmap_;                       // cperm_ on the device (potential x and gradient)
    int64_t obj_k0_ = 0, obj_n_ = 0;
    bool obj_in_P_ = false;
};

std::unique_ptr<Program> make_generic_program(Solver &s, const HostCSR *P, const HostCSR *C, int64_t obj_row)
{
    if (s.fp32) return std::unique_ptr<Program>(new GenericProgram<float>(s, P, C, obj_row));
    return std::unique_ptr<Program>(new GenericProgram<double>(s, P, C, obj_row));
}

}  // namespace mwu
