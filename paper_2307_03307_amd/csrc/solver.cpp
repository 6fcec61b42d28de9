// C ABI of the solver: validation and normalization of the LP, program
// selection, the probe driver and the outer search over M (pure problems) or
// lambda = D (mixed problems).
//
// Normalization follows Section 2.1 of the paper: P_ij = A_ij / (b_i c_j)
// with x' = c * x.  The objective of a pure packing (covering) problem is
// embedded as the single covering (packing) row (1/M) 1^T x and M is searched
// (end of Section 2.2); the densest-subgraph dual fixes D and searches it
// (Section 3).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <new>

#include "host.h"

namespace mwu {

Solver::~Solver()
{
    if (graph) (void)hipGraphExecDestroy(graph);
    prog.reset();
    batch.reset();
    if (ctl_host) (void)hipHostFree(ctl_host);
    if (own_stream && stream) (void)hipStreamDestroy(stream);
}

// ------------------------------------------------------------ validation

static void check(bool ok, mwu_status code, const char *msg)
{
    if (!ok) throw ApiError{code, msg};
}

static void validate_edges(const mwu_matrix &m, EdgeList &el)
{
    check(m.num_vertices > 0 && m.num_edges > 0, MWU_ERR_INVALID_ARG, "empty graph");
    check(m.edge_u && m.edge_v, MWU_ERR_INVALID_ARG, "edge list is NULL");
    check(m.num_vertices < INT32_MAX && 2 * m.num_edges < INT32_MAX, MWU_ERR_TOO_LARGE,
          "graph exceeds 32-bit device indices");
    el.nv = m.num_vertices;
    el.ne = m.num_edges;
    el.u.assign(m.edge_u, m.edge_u + m.num_edges);
    el.v.assign(m.edge_v, m.edge_v + m.num_edges);
    std::vector<uint64_t> key(el.ne);
    for (int64_t e = 0; e < el.ne; ++e) {
        const int64_t a = el.u[e], b = el.v[e];
        check(a >= 0 && a < el.nv && b >= 0 && b < el.nv, MWU_ERR_GRAPH, "vertex id out of range");
        check(a != b, MWU_ERR_GRAPH, "self-loop");
        key[e] = (uint64_t)std::min(a, b) * (uint64_t)el.nv + (uint64_t)std::max(a, b);
    }
    std::sort(key.begin(), key.end());
    for (int64_t e = 1; e < el.ne; ++e) check(key[e] != key[e - 1], MWU_ERR_GRAPH, "duplicate edge");
}

// Explicit CSR of any matrix kind (pattern-only kinds have empty val).
static HostCSR to_csr(const mwu_matrix &m, EdgeList *el_out)
{
    HostCSR A;
    if (m.kind == MWU_MAT_CSR) {
        check(m.rows >= 1 && m.cols >= 1 && m.row_ptr && m.col_idx, MWU_ERR_INVALID_ARG, "bad CSR");
        check(m.rows < INT32_MAX && m.cols < INT32_MAX, MWU_ERR_TOO_LARGE, "CSR too large");
        check(m.row_ptr[0] == 0, MWU_ERR_INVALID_ARG, "row_ptr[0] != 0");
        for (int64_t r = 0; r < m.rows; ++r)
            check(m.row_ptr[r + 1] >= m.row_ptr[r], MWU_ERR_INVALID_ARG, "row_ptr not monotone");
        const int64_t nnz = m.row_ptr[m.rows];
        check(nnz < INT32_MAX, MWU_ERR_TOO_LARGE, "too many nonzeros");
        A.rows = m.rows; A.cols = m.cols;
        A.ptr.assign(m.row_ptr, m.row_ptr + m.rows + 1);
        A.idx.assign(m.col_idx, m.col_idx + nnz);
        for (int64_t k = 0; k < nnz; ++k)
            check(A.idx[k] >= 0 && A.idx[k] < m.cols, MWU_ERR_INVALID_ARG, "column index out of range");
        if (m.values) {
            A.val.assign(m.values, m.values + nnz);
            for (double v : A.val) {
                check(std::isfinite(v), MWU_ERR_NONFINITE, "non-finite matrix value");
                check(v >= 0.0, MWU_ERR_NEGATIVE_ENTRY, "negative matrix value");
            }
        }
        return A;
    }
    EdgeList el;
    validate_edges(m, el);
    const int64_t nv = el.nv, ne = el.ne;
    switch (m.kind) {
    case MWU_MAT_INCIDENCE:     // rows = vertices, columns = edges
    case MWU_MAT_EDGE_PAIR: {   // rows = vertices, columns = 2e (first end), 2e+1 (second end)
        const bool pair = m.kind == MWU_MAT_EDGE_PAIR;
        A.rows = nv; A.cols = pair ? 2 * ne : ne;
        A.ptr.assign(nv + 1, 0);
        for (int64_t e = 0; e < ne; ++e) { A.ptr[el.u[e] + 1]++; A.ptr[el.v[e] + 1]++; }
        for (int64_t v = 0; v < nv; ++v) A.ptr[v + 1] += A.ptr[v];
        A.idx.resize(2 * ne);
        std::vector<int64_t> fill(A.ptr.begin(), A.ptr.end() - 1);
        for (int64_t e = 0; e < ne; ++e) {   // edge order keeps every row sorted
            A.idx[fill[el.u[e]]++] = (int32_t)(pair ? 2 * e : e);
            A.idx[fill[el.v[e]]++] = (int32_t)(pair ? 2 * e + 1 : e);
        }
        if (pair)
            for (int64_t v = 0; v < nv; ++v) std::sort(A.idx.begin() + A.ptr[v], A.idx.begin() + A.ptr[v + 1]);
        break;
    }
    case MWU_MAT_INCIDENCE_T: {   // rows = edges, row e = {u_e, v_e}
        A.rows = ne; A.cols = nv;
        A.ptr.resize(ne + 1);
        A.idx.resize(2 * ne);
        for (int64_t e = 0; e < ne; ++e) {
            A.ptr[e] = 2 * e;
            A.idx[2 * e] = std::min(el.u[e], el.v[e]);
            A.idx[2 * e + 1] = std::max(el.u[e], el.v[e]);
        }
        A.ptr[ne] = 2 * ne;
        break;
    }
    case MWU_MAT_INTERWEAVE: {    // rows = edges, row e = {2e, 2e+1}
        A.rows = ne; A.cols = 2 * ne;
        A.ptr.resize(ne + 1);
        A.idx.resize(2 * ne);
        for (int64_t e = 0; e < ne; ++e) {
            A.ptr[e] = 2 * e;
            A.idx[2 * e] = (int32_t)(2 * e);
            A.idx[2 * e + 1] = (int32_t)(2 * e + 1);
        }
        A.ptr[ne] = 2 * ne;
        break;
    }
    default:
        throw ApiError{MWU_ERR_INVALID_ARG, "unknown matrix kind"};
    }
    if (el_out) *el_out = std::move(el);
    return A;
}

static void scale_rows_cols(HostCSR &A, const double *b, const std::vector<double> &c)
{
    if (!b && c.empty()) return;
    if (A.val.empty()) A.val.assign(A.nnz(), 1.0);
    for (int64_t r = 0; r < A.rows; ++r)
        for (int64_t k = A.ptr[r]; k < A.ptr[r + 1]; ++k) {
            double den = (b ? b[r] : 1.0) * (c.empty() ? 1.0 : c[A.idx[k]]);
            A.val[k] /= den;
        }
}

static void check_rhs(const double *b, int64_t len, const char *what)
{
    if (!b) return;
    for (int64_t i = 0; i < len; ++i) {
        check(std::isfinite(b[i]), MWU_ERR_NONFINITE, what);
        check(b[i] > 0.0, MWU_ERR_BAD_RHS, what);
    }
}

static HostCSR drop_rows(const HostCSR &A, const std::vector<char> &keep)
{
    HostCSR B;
    B.cols = A.cols;
    B.ptr.push_back(0);
    for (int64_t r = 0; r < A.rows; ++r) {
        if (!keep[r]) continue;
        for (int64_t k = A.ptr[r]; k < A.ptr[r + 1]; ++k) {
            B.idx.push_back(A.idx[k]);
            if (!A.val.empty()) B.val.push_back(A.val[k]);
        }
        B.ptr.push_back((int64_t)B.idx.size());
        B.rows++;
    }
    return B;
}

// Renumbers the columns of A by newid; entries of removed columns (newid < 0)
// leave the structure with them.
static void remap_cols(HostCSR &A, const std::vector<int64_t> &newid, int64_t ncols)
{
    int64_t k = 0;
    const bool vals = !A.val.empty();
    for (int64_t r = 0; r < A.rows; ++r) {
        const int64_t q0 = A.ptr[r], q1 = A.ptr[r + 1];
        A.ptr[r] = k;
        for (int64_t q = q0; q < q1; ++q) {
            const int64_t c = newid[A.idx[q]];
            if (c < 0) continue;
            A.idx[k] = (int32_t)c;
            if (vals) A.val[k] = A.val[q];
            ++k;
        }
    }
    A.ptr[A.rows] = k;
    A.idx.resize(k);
    if (vals) A.val.resize(k);
    A.cols = ncols;
}

static bool all_ones(const HostCSR &A)
{
    for (double v : A.val) if (v != 1.0) return false;
    return true;
}

// ------------------------------------------------------------ construction

static void fill_defaults(mwu_options *o)
{
    std::memset(o, 0, sizeof(*o));
    o->eps = 0.1;
    o->max_iter = 5000;
    o->max_probes = 64;
    o->step_rule = MWU_STEP_BIN;
    o->precision = MWU_MIXED_FP32_FP64;
    o->iters_per_launch = 0;   // the program's default
    o->device = 0;
}

static void setup_device(Solver &s)
{
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count == 0)
        throw ApiError{MWU_ERR_DEVICE, "no HIP device"};
    check(s.opt.device >= 0 && s.opt.device < count, MWU_ERR_INVALID_ARG, "bad device ordinal");
    HIP_OK(hipSetDevice(s.opt.device));
    hipDeviceProp_t prop;
    HIP_OK(hipGetDeviceProperties(&prop, s.opt.device));
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        throw ApiError{MWU_ERR_DEVICE, "device is not gfx950"};
    s.num_cus = std::max(1, prop.multiProcessorCount);
    if (s.opt.hip_stream) {
        s.stream = (hipStream_t)s.opt.hip_stream;
    } else {
        HIP_OK(hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking));
        s.own_stream = true;
    }
    s.ctl_buf.alloc(sizeof(Ctl));
    HIP_OK(hipMemset(s.ctl_buf.p, 0, sizeof(Ctl)));
    HIP_OK(hipHostMalloc((void **)&s.ctl_host, sizeof(Ctl), hipHostMallocDefault));
    std::memset(s.ctl_host, 0, sizeof(Ctl));
}

static_assert(MWU_STEP_STD == SR_STD && MWU_STEP_BIN == SR_BIN && MWU_STEP_BIN_WARM == SR_BIN_WARM &&
                  MWU_STEP_NEWTON == SR_NEWTON,
              "device step rules follow the C interface");

static void build(Solver &s, const mwu_problem &p)
{
    s.form = p.form;
    check(p.form == MWU_PACKING || p.form == MWU_COVERING || p.form == MWU_MIXED || p.form == MWU_MIXED_MAX ||
              p.form == MWU_MIXED_MIN,
          MWU_ERR_INVALID_ARG, "bad form");
    const bool mixed_opt = p.form == MWU_MIXED_MAX || p.form == MWU_MIXED_MIN;
    check(s.opt.eps > 0.0 && s.opt.eps < 1.0, MWU_ERR_INVALID_ARG, "eps must be in (0,1)");
    check(s.opt.max_iter >= 1 && s.opt.max_probes >= 1, MWU_ERR_INVALID_ARG, "bad iteration caps");
    check(s.opt.step_rule == MWU_STEP_STD || s.opt.step_rule == MWU_STEP_BIN ||
              s.opt.step_rule == MWU_STEP_BIN_WARM || s.opt.step_rule == MWU_STEP_NEWTON,
          MWU_ERR_INVALID_ARG, "bad step rule");
    check(s.opt.precision == MWU_FP64 || s.opt.precision == MWU_MIXED_FP32_FP64,
          MWU_ERR_INVALID_ARG, "bad precision");
    // 16 iterations per graph launch: one host synchronisation per 16
    // iterations (measured best for the vertex-cover LP at scale 20; 8 and 32
    // are about 3% slower)
    if (s.opt.iters_per_launch <= 0) s.opt.iters_per_launch = 16;
    s.fp32 = s.opt.precision == MWU_MIXED_FP32_FP64;

    HostCSR P, C;
    EdgeList elP, elC;
    std::vector<double> cvec;
    if (p.form == MWU_PACKING) {
        P = to_csr(p.P, &elP);
        s.onesC = 1;
        s.n_user = P.cols;
        if (p.c) { cvec.assign(p.c, p.c + P.cols); check_rhs(p.c, P.cols, "bad c"); }
        check_rhs(p.b_P, P.rows, "bad b");
        scale_rows_cols(P, p.b_P, cvec);
    } else if (p.form == MWU_COVERING) {
        C = to_csr(p.C, &elC);
        s.onesP = 1;
        s.n_user = C.cols;
        if (p.c) { cvec.assign(p.c, p.c + C.cols); check_rhs(p.c, C.cols, "bad c"); }
        check_rhs(p.b_C, C.rows, "bad b");
        scale_rows_cols(C, p.b_C, cvec);
    } else if (mixed_opt) {
        check(p.c != nullptr, MWU_ERR_INVALID_ARG, "the mixed optimization forms need c");
        P = to_csr(p.P, &elP);
        C = to_csr(p.C, &elC);
        check(P.cols == C.cols, MWU_ERR_INVALID_ARG, "P and C column counts differ");
        s.n_user = P.cols;
        check_rhs(p.b_P, P.rows, "bad b_P");
        check_rhs(p.b_C, C.rows, "bad b_C");
        check_rhs(p.c, P.cols, "bad c");
        cvec.assign(p.c, p.c + P.cols);
        // x' = c x: the objective row becomes (1/M) 1^T x'
        scale_rows_cols(P, p.b_P, cvec);
        scale_rows_cols(C, p.b_C, cvec);
    } else {
        check(!p.c, MWU_ERR_INVALID_ARG, "c is not used by MWU_MIXED");
        P = to_csr(p.P, &elP);
        C = to_csr(p.C, &elC);
        check(P.cols == C.cols, MWU_ERR_INVALID_ARG, "P and C column counts differ");
        s.n_user = P.cols;
        check_rhs(p.b_P, P.rows, "bad b_P");
        check_rhs(p.b_C, C.rows, "bad b_C");
        scale_rows_cols(P, p.b_P, cvec);
        scale_rows_cols(C, p.b_C, cvec);
        s.level_sets = p.P.kind == MWU_MAT_EDGE_PAIR && p.C.kind == MWU_MAT_INTERWEAVE &&
                       elP.ne == elC.ne && elP.u == elC.u && elP.v == elC.v;
    }
    const int64_t n = s.n_user;
    // ---- drop empty rows and columns (never-binding rows; variables fixed at 0)
    std::vector<int64_t> pcnt(n, 0), ccnt(n, 0);
    if (!s.onesP) {
        std::vector<char> keep(P.rows);
        for (int64_t r = 0; r < P.rows; ++r) keep[r] = P.ptr[r + 1] > P.ptr[r];
        P = drop_rows(P, keep);
        check(P.rows >= 1, MWU_ERR_INVALID_ARG, "packing matrix has no nonzero");
        for (auto c : P.idx) pcnt[c]++;
    }
    if (!s.onesC) {
        for (int64_t r = 0; r < C.rows; ++r)
            check(C.ptr[r + 1] > C.ptr[r], MWU_ERR_INVALID_ARG, "covering row without nonzero");
        for (auto c : C.idx) ccnt[c]++;
    }
    std::vector<int64_t> newid(n, -1);
    int64_t kept = 0;
    for (int64_t i = 0; i < n; ++i) {
        bool keep;
        if (p.form == MWU_PACKING) {
            check(pcnt[i] > 0, MWU_ERR_UNBOUNDED, "packing column without nonzero: LP unbounded");
            keep = true;
        } else if (p.form == MWU_COVERING) {
            keep = ccnt[i] > 0;
        } else if (p.form == MWU_MIXED_MAX) {
            // every column is in the objective row; the packing rows bound it
            check(pcnt[i] > 0, MWU_ERR_UNBOUNDED, "column without packing entry: LP unbounded");
            keep = true;
        } else if (p.form == MWU_MIXED_MIN) {
            // every column is in the objective row (a packing row); one without
            // a covering entry never moves from its start (h = 0)
            keep = true;
        } else {
            keep = ccnt[i] > 0;
            if (keep) check(pcnt[i] > 0, MWU_ERR_UNBOUNDED, "column with covering but no packing entry");
        }
        if (keep) { newid[i] = kept++; s.col_user.push_back(i); s.col_c.push_back(cvec.empty() ? 1.0 : cvec[i]); }
    }
    if (!s.onesP) {
        remap_cols(P, newid, kept);
        // packing rows whose entries all sat in removed columns never bind
        std::vector<char> keep(P.rows);
        for (int64_t r = 0; r < P.rows; ++r) keep[r] = P.ptr[r + 1] > P.ptr[r];
        P = drop_rows(P, keep);
        check(P.rows >= 1, MWU_ERR_INVALID_ARG, "packing matrix has no nonzero in a kept column");
    }
    if (!s.onesC) remap_cols(C, newid, kept);
    if (!P.val.empty() && all_ones(P)) P.val.clear();
    if (!C.val.empty() && all_ones(C)) C.val.clear();
    int64_t obj_row = -1;
    if (mixed_opt) {
        check(C.rows >= 1, MWU_ERR_INVALID_ARG, "the mixed optimization forms need covering rows");
        const double eps = s.opt.eps;
        std::vector<double> cmax(kept, 0.0), colsum(kept, 0.0), xt(kept, 0.0);
        for (int64_t k = 0; k < P.nnz(); ++k) cmax[P.idx[k]] = std::max(cmax[P.idx[k]], P.v(k));
        for (int64_t r = 0; r < C.rows; ++r) {
            const double nz = (double)(C.ptr[r + 1] - C.ptr[r]);
            for (int64_t k = C.ptr[r]; k < C.ptr[r + 1]; ++k) {
                colsum[C.idx[k]] += C.v(k);
                xt[C.idx[k]] = std::max(xt[C.idx[k]], 1.0 / (C.v(k) * nz));
            }
        }
        if (p.form == MWU_MIXED_MAX) {
            double hi = 0.0;   // x'_i <= 1 / max_j P'_ji
            for (int64_t i = 0; i < kept; ++i) hi += 1.0 / cmax[i];
            s.hi0 = hi;
            s.lo0 = 0.0;
        } else {
            // uniform dual weights on the covering rows; the covering-feasible
            // point's value starts the search
            s.lo0 = (double)C.rows / *std::max_element(colsum.begin(), colsum.end());
            double v = 0.0;
            for (double t : xt) v += t;
            s.hi0 = std::max(v, 2.0 * s.lo0);
        }
        (void)eps;
        // the objective row: every kept column, its values set before each probe
        HostCSR &A = p.form == MWU_MIXED_MAX ? C : P;
        if (A.val.empty()) A.val.assign(A.nnz(), 1.0);
        for (int64_t i = 0; i < kept; ++i) { A.idx.push_back((int32_t)i); A.val.push_back(1.0); }
        A.ptr.push_back(A.ptr.back() + kept);
        A.rows += 1;
        obj_row = p.form == MWU_MIXED_MAX ? P.rows + C.rows - 1 : P.rows - 1;
    }
    // ---- outer-search starting bracket (same rules as the CPU reference)
    const double eps = s.opt.eps;
    if (mixed_opt) {
        // set above
    } else if (p.form == MWU_PACKING) {
        std::vector<double> cmin(kept, INFINITY), cmax(kept, 0.0);
        for (int64_t k = 0; k < P.nnz(); ++k) {
            const double v = P.v(k);
            if (v > 0.0) cmin[P.idx[k]] = std::min(cmin[P.idx[k]], v);
            cmax[P.idx[k]] = std::max(cmax[P.idx[k]], v);
        }
        double hi = 0.0;
        for (int64_t i = 0; i < kept; ++i) {
            check(std::isfinite(cmin[i]) && cmax[i] > 0.0, MWU_ERR_UNBOUNDED, "packing column of zeros");
            hi += 1.0 / cmin[i];
        }
        std::vector<double> x0(kept), y(P.rows, 0.0);
        double sx = 0.0;
        for (int64_t i = 0; i < kept; ++i) { x0[i] = eps / ((double)kept * cmax[i]); sx += x0[i]; }
        for (int64_t r = 0; r < P.rows; ++r)
            for (int64_t k = P.ptr[r]; k < P.ptr[r + 1]; ++k) y[r] += P.v(k) * x0[P.idx[k]];
        const double ymax = *std::max_element(y.begin(), y.end());
        s.lo0 = sx / ymax;
        s.hi0 = hi;
        s.x_start.resize(kept);
        for (int64_t i = 0; i < kept; ++i) s.x_start[i] = x0[i] / ymax;
    } else {
        // covering-feasible point x_i = max_{j: C_ji>0} 1/(C_ji nnz_j)
        std::vector<double> xt(kept, 0.0), colsum(kept, 0.0);
        for (int64_t r = 0; r < C.rows; ++r) {
            const double nz = (double)(C.ptr[r + 1] - C.ptr[r]);
            for (int64_t k = C.ptr[r]; k < C.ptr[r + 1]; ++k) {
                const double v = C.v(k);
                colsum[C.idx[k]] += v;
                if (v > 0.0) xt[C.idx[k]] = std::max(xt[C.idx[k]], 1.0 / (v * nz));
            }
        }
        if (p.form == MWU_COVERING) {
            const double csmax = *std::max_element(colsum.begin(), colsum.end());
            s.lo0 = (double)C.rows / csmax;
            double hi = 0.0;
            for (double v : xt) hi += v;
            s.hi0 = hi;
            s.x_start = xt;
        } else {
            std::vector<double> px(P.rows, 0.0), pcs(kept, 0.0);
            for (int64_t r = 0; r < P.rows; ++r)
                for (int64_t k = P.ptr[r]; k < P.ptr[r + 1]; ++k) {
                    px[r] += P.v(k) * xt[P.idx[k]];
                    pcs[P.idx[k]] += P.v(k);
                }
            s.hi0 = *std::max_element(px.begin(), px.end());
            double lo = INFINITY;   // weak duality with uniform weights
            for (int64_t i = 0; i < kept; ++i)
                if (colsum[i] > 0.0)
                    lo = std::min(lo, (pcs[i] / (double)P.rows) / (colsum[i] / (double)C.rows));
            s.lo0 = lo;
            s.x_start = xt;
        }
    }
    std::vector<int64_t> vid;
    int64_t nv = 0;
    if (s.level_sets) {
        // non-isolated vertex ids of the densest-subgraph graph
        vid.assign(elP.nv, -1);
        for (int64_t e = 0; e < elP.ne; ++e) {
            if (vid[elP.u[e]] < 0) vid[elP.u[e]] = 0;
            if (vid[elP.v[e]] < 0) vid[elP.v[e]] = 0;
        }
        for (auto &v : vid) if (v == 0) v = nv++; else v = -1;
        // rows of P (O) were compacted in vertex order
        s.dens_graph.nv = nv;
        s.dens_graph.ne = elP.ne;
        s.dens_graph.u.resize(elP.ne);
        s.dens_graph.v.resize(elP.ne);
        for (int64_t e = 0; e < elP.ne; ++e) {
            s.dens_graph.u[e] = (int32_t)vid[elP.u[e]];
            s.dens_graph.v[e] = (int32_t)vid[elP.v[e]];
        }
    }
    setup_device(s);
    const bool fused_vc = p.form == MWU_COVERING && p.C.kind == MWU_MAT_INCIDENCE_T && !p.b_C && !p.c &&
                          !(s.opt.flags & MWU_FLAG_GENERIC);
    const bool fused_dn = s.level_sets && !p.b_P && !p.b_C && !(s.opt.flags & MWU_FLAG_GENERIC);
    if (fused_vc) {
        C = HostCSR();
        s.prog = make_vcover_program(s, elC, newid, kept);
    } else if (fused_dn) {
        P = HostCSR();
        C = HostCSR();
        s.prog = make_densest_program(s, elP, vid, nv);
    } else {
        s.prog = make_generic_program(s, s.onesP ? nullptr : &P, s.onesC ? nullptr : &C, obj_row);
    }
}

// ------------------------------------------------------------ probes

static bool mixed_opt_form(const Solver &s) { return s.form == MWU_MIXED_MAX || s.form == MWU_MIXED_MIN; }

// Uniform scales of the two sides in a probe at param (the mixed optimization
// forms scale their embedded objective row instead)
static double probe_scale_P(const Solver &s, double param)
{
    return s.form == MWU_PACKING || mixed_opt_form(s) ? 1.0 : 1.0 / param;
}
static double probe_scale_C(const Solver &s, double param)
{
    return s.form == MWU_PACKING ? 1.0 / param : 1.0;
}

static void pull_ctl(Solver &s)
{
    HIP_OK(hipMemcpyAsync(s.ctl_host, s.ctl_buf.p, sizeof(Ctl), hipMemcpyDeviceToHost, s.stream));
    HIP_OK(hipStreamSynchronize(s.stream));
}

static void push_ctl(Solver &s)
{
    HIP_OK(hipMemcpyAsync(s.ctl_buf.p, s.ctl_host, sizeof(Ctl), hipMemcpyHostToDevice, s.stream));
}

// Direction threshold of the mixed form: the relative rounding of g_i and h_i
// (FP32 weights and per-thread partials) stays well below this, so a
// coordinate is moved only when g_i < h_i holds beyond that rounding.
static constexpr double kMixedQmin = 1.0 / 65536.0;
// Times the probe tolerance may be halved when the search bracket closes
// without a certified (1 + eps) bracket.
static constexpr int kMaxHalvings = 2;

// Start a probe at param: from the Algorithm 1 point, from the host point x0,
// or (device_x0) from the point the device holds, with the warm-started
// search beginning at start_alpha in its first iteration.
static void begin_probe(Solver &s, double param, const double *x0, double eps_probe = 0.0,
                        bool device_x0 = false, double start_alpha = 0.0)
{
    Ctl &c = *s.ctl_host;
    std::memset(&c, 0, sizeof(Ctl));
    const int64_t m = s.prog->mP() + s.prog->mC();
    const double eps = eps_probe > 0.0 ? eps_probe : s.opt.eps;
    c.eta = 10.0 * std::log((double)m) / eps;                // Algorithm 1, natural log
    c.eps = eps;
    const bool single = s.prog->mP() == 1 || s.prog->mC() == 1;
    const double sfac = (single && !(s.opt.flags & MWU_FLAG_NO_FACTOR2)) ? 1.0 : 0.5;
    c.step = sfac / c.eta;
    c.sP = probe_scale_P(s, param);
    c.sC = probe_scale_C(s, param);
    c.psi_lim = s.fp32 ? 80.0 : 700.0;
    c.s2_min = s.fp32 ? 1e-25 : 1e-280;
    c.qmin = s.fp32 ? kMixedQmin : 0.0;
    c.psi_shift = s.fp32 ? 1 : 0;
    c.onesP = s.onesP;
    c.onesC = s.onesC;
    c.step_rule = s.opt.step_rule;
    c.max_iter = s.opt.max_iter;
    c.pack_bound = INFINITY;
    c.cover_bound = 0.0;
    if (!s.trace_buf.p) s.trace_buf.alloc((size_t)s.opt.max_iter * 8);
    c.trace = s.trace_buf.as<double>();
    c.trace_cap = s.opt.max_iter;
    c.status = ST_RUNNING;
    c.phase = PH_IDLE;
    c.last_alpha = start_alpha;
    c.drop = (s.opt.flags & MWU_FLAG_DROP_SATISFIED) ? 1 : 0;
    push_ctl(s);
    if (mixed_opt_form(s)) s.prog->set_objective_level(1.0 / param);   // the row (1/M) 1^T x'
    if (x0) s.prog->upload_x(x0);
    s.prog->probe_init(x0 != nullptr || device_x0);
    s.in_probe = true;
    s.dir_pending = false;
    s.probe_param = param;
}

static void ensure_graph(Solver &s)
{
    if (s.graph && s.graph_slots == s.opt.iters_per_launch) return;
    if (s.graph) { (void)hipGraphExecDestroy(s.graph); s.graph = nullptr; }
    hipGraph_t g;
    HIP_OK(hipStreamBeginCapture(s.stream, hipStreamCaptureModeThreadLocal));
    s.prog->iterations(s.opt.iters_per_launch);
    HIP_OK(hipStreamEndCapture(s.stream, &g));
    HIP_OK(hipGraphInstantiate(&s.graph, g, nullptr, nullptr, 0));
    (void)hipGraphDestroy(g);
    s.graph_slots = s.opt.iters_per_launch;
}

// Run until the probe stops or max_iters more iterations were taken.
static void run_probe(Solver &s, int64_t max_iters)
{
    ensure_graph(s);
    pull_ctl(s);
    const int64_t start = s.ctl_host->iter;
    const int64_t cap_launches = (max_iters + 4) * 8 / std::max(1, s.opt.iters_per_launch) + 16;
    for (int64_t l = 0; l < cap_launches; ++l) {
        if (s.ctl_host->phase == PH_DONE || s.ctl_host->status != ST_RUNNING) break;
        if (s.ctl_host->phase == PH_IDLE) break;   // paused at the probe API's iteration stop
        if (s.ctl_host->iter - start >= max_iters) break;
        HIP_OK(hipGraphLaunch(s.graph, s.stream));
        pull_ctl(s);
        s.prog->between_launches(*s.ctl_host);
    }
}

// A probe paused by mwu_probe_run's iteration stop (a pending step, PH_IDLE)
// continues at its next row pass.
static void unpause(Solver &s)
{
    Ctl &c = *s.ctl_host;
    if (!s.dir_pending && c.phase == PH_IDLE && c.status == ST_RUNNING) c.phase = PH_ROW;
}

static void finish_probe_stats(Solver &s)
{
    s.prog->final_stats();
    pull_ctl(s);
}

// ------------------------------------------------------------ level sets

static double level_set_density(const EdgeList &g, const std::vector<double> &score)
{
    const int64_t nv = g.nv;
    std::vector<int32_t> order(nv);
    for (int64_t i = 0; i < nv; ++i) order[i] = (int32_t)i;
    std::stable_sort(order.begin(), order.end(),
                     [&](int32_t a, int32_t b) { return score[a] > score[b]; });
    std::vector<int64_t> rank(nv), cnt(nv + 1, 0);
    for (int64_t i = 0; i < nv; ++i) rank[order[i]] = i;
    for (int64_t e = 0; e < g.ne; ++e) cnt[std::max(rank[g.u[e]], rank[g.v[e]]) + 1]++;
    double best = 0.0;
    int64_t acc = 0;
    for (int64_t k = 1; k <= nv; ++k) {
        acc += cnt[k];
        best = std::max(best, (double)acc / (double)k);
    }
    return best;
}

// ------------------------------------------------------------ outer search

struct SolveOut {
    int32_t status;
    double objective, lower, upper, best_scale;
    int64_t probes, total_iters, final_iters, passes, evals;
    double max_violation;
    bool have_best_dev;
};

static SolveOut solve_impl(Solver &s)
{
    SolveOut o{};
    const double eps = s.opt.eps;
    double lo = s.lo0, hi = s.hi0;
    o.have_best_dev = false;
    o.best_scale = 1.0;
    double eps_probe = eps;
    // probes after the first may start from their predecessor's point (R21):
    // its iterate scaled so that the largest packing row of the next probe is
    // eps (the level of the Algorithm 1 point), and its last step
    const bool reuse = (s.opt.flags & MWU_FLAG_REUSE) != 0 && !mixed_opt_form(s);
    double prev_pmax = 0.0, prev_sP = 0.0, prev_alpha = 0.0;   // max(P x) in the previous probe's scale
    auto probe_done = [&](double param) {
        const double sPn = probe_scale_P(s, param);
        const double pmax = prev_sP > 0.0 ? prev_pmax * sPn / prev_sP : 0.0;
        if (reuse && o.probes > 0 && pmax > 0.0 && std::isfinite(pmax)) {
            s.prog->scale_x(eps_probe / pmax);
            begin_probe(s, param, nullptr, eps_probe, true, prev_alpha);
        } else {
            begin_probe(s, param, nullptr, eps_probe);
        }
        run_probe(s, s.opt.max_iter);
        pull_ctl(s);
        Ctl c = *s.ctl_host;
        // the iteration cap was reached before the device could flag it
        if (c.status == ST_RUNNING) c.status = ST_MAX_ITER;
        o.probes++;
        o.total_iters += c.iter;
        o.final_iters = c.iter;
        o.passes += c.search_passes;
        o.evals += c.evaluations;
        prev_alpha = c.last_alpha;
        return c;
    };
    // the statistics of the probe just ended (for the next probe's start)
    auto note_stats = [&](const Ctl &f) {
        prev_pmax = f.ymax;
        prev_sP = f.sP;
    };
    if (s.form == MWU_MIXED && s.opt.mixed_fixed_lambda > 0.0) {
        const double lam = s.opt.mixed_fixed_lambda;
        Ctl c = probe_done(lam);
        finish_probe_stats(s);
        const Ctl f = *s.ctl_host;
        // x_out, objective_out and max_violation all describe the probe's
        // final point x (not rescaled): objective = lambda(x) = max_i (P x)_i
        // in the caller's scale, and with C x >= 1 at a feasible stop it
        // bounds the least lambda from above
        s.prog->save_best();
        o.have_best_dev = true;
        o.best_scale = 1.0;
        o.status = c.status == ST_FEASIBLE ? MWU_FEASIBLE_POINT
                   : c.status == ST_INFEASIBLE ? MWU_INFEASIBLE : MWU_MAX_ITER;
        o.objective = f.ymax / f.sP;
        const double cf = s.fp32 ? 1.0 - kMixedQmin : 1.0;
        o.lower = c.status == ST_INFEASIBLE ? lam * cf : 0.0;
        o.upper = c.status == ST_FEASIBLE ? o.objective : INFINITY;
        o.max_violation = std::max({0.0, f.ymax - 1.0, 1.0 - f.zmin});
        return o;
    }
    const bool trace = std::getenv("MWU_TRACE") != nullptr;
    // An infeasible verdict proves OPT < param (packing) or OPT > param
    // (covering, densest) up to the direction threshold qmin.
    const double cf = s.fp32 ? 1.0 - kMixedQmin : 1.0;
    if (mixed_opt_form(s)) {
        // the objective embedded as a row at level M (reading of the last
        // sentence of Section 2.2): the same search as the CPU reference
        const bool maxi = s.form == MWU_MIXED_MAX;
        double mlo = maxi ? 0.0 : s.lo0, mhi = maxi ? s.hi0 : INFINITY;
        double slo = maxi ? s.hi0 / 1048576.0 : s.lo0, shi = s.hi0;
        bool have = false;
        o.status = MWU_INFEASIBLE;
        while (o.probes < s.opt.max_probes && !(mhi <= (1.0 + eps) * mlo)) {
            const bool grow = !maxi && !have;   // minimizing: probe the top until one is feasible
            if (!grow && !(shi > (1.0 + eps / 16.0) * slo)) break;
            const double M = grow ? shi : std::sqrt(slo * shi);
            const Ctl c = probe_done(M);
            finish_probe_stats(s);
            const Ctl f = *s.ctl_host;
            if (c.status == ST_NUMERIC) throw ApiError{MWU_ERR_DEVICE, "numerical failure in a probe"};
            if (trace)
                std::fprintf(stderr, "[mwu] probe %lld M %.10g status %d iters %d sumx %.10g ymax %.10g\n",
                             (long long)o.probes, M, c.status, c.iter, f.sumx, f.ymax);
            if (c.status == ST_FEASIBLE) {
                if (!have || (maxi ? M > mlo : M < mhi)) {
                    s.prog->save_best();
                    o.have_best_dev = true;
                    o.best_scale = 1.0;
                    o.objective = f.sumx;   // 1^T x' = c^T x
                    o.max_violation = std::max(0.0, f.ymax - 1.0);
                    have = true;
                }
                if (maxi) { mlo = std::max(mlo, M); slo = M; }
                else { mhi = std::min(mhi, M); shi = M; }
            } else if (maxi) {
                if (c.status == ST_INFEASIBLE) mhi = std::min(mhi, M / cf);
                shi = M;
            } else {
                if (c.status == ST_INFEASIBLE) mlo = std::max(mlo, M * cf);
                slo = M;
                if (grow) shi = 4.0 * M;
            }
            slo = std::max(slo, mlo);
            shi = std::min(shi, mhi);
        }
        o.lower = mlo;
        o.upper = mhi;
        if (have) o.status = mhi <= (1.0 + eps) * mlo ? MWU_CERTIFIED : MWU_FEASIBLE_UNCERTIFIED;
        return o;
    }
    // search bracket for the parameter: moves to every probed value, while
    // lo/hi (the certified bracket on OPT) move only with certificates
    double slo = lo, shi = hi;
    int halvings = 0;
    while (o.probes < s.opt.max_probes && hi > (1.0 + eps) * lo) {
        if (!(shi > (1.0 + eps / 16.0) * slo)) {
            // the search bracket closed without a certified bracket: continue
            // at half the probe tolerance from the certified bracket
            if (halvings == kMaxHalvings) break;
            ++halvings;
            eps_probe *= 0.5;
            slo = lo;
            shi = hi;
            continue;
        }
        const double param = std::sqrt(slo * shi);
        const Ctl c = probe_done(param);
        finish_probe_stats(s);
        const Ctl f = *s.ctl_host;
        note_stats(f);
        if (trace)
            std::fprintf(stderr, "[mwu] probe %lld eps %.4g param %.10g status %d iters %d passes %lld alpha %.6g "
                         "sumx %.10g ymax %.10g zmin %.10g bounds %.10g %.10g bracket %.10g %.10g\n",
                         (long long)o.probes, eps_probe, param, c.status, c.iter, (long long)c.search_passes,
                         c.last_alpha, f.sumx, f.ymax, f.zmin, c.pack_bound, c.cover_bound, lo, hi);
        o.max_violation = std::max({0.0, f.ymax - 1.0, 1.0 - f.zmin});
        if (c.status == ST_NUMERIC) throw ApiError{MWU_ERR_DEVICE, "numerical failure in a probe"};
        const bool feasible = c.status == ST_FEASIBLE;
        if (s.form == MWU_PACKING) {
            if (c.pack_bound < hi) hi = c.pack_bound;
            if (feasible) {
                const double val = f.sumx / f.ymax;
                if (val > lo) { lo = val; s.prog->save_best(); o.have_best_dev = true; o.best_scale = 1.0 / f.ymax; }
                slo = param;
            } else {
                if (c.status == ST_INFEASIBLE) hi = std::min(hi, param / cf);
                shi = param;
            }
        } else {
            if (s.form == MWU_COVERING && c.cover_bound > lo) lo = c.cover_bound;
            if (s.level_sets) {
                double lsd = 0.0;
                if (!s.prog->level_set_density(&lsd)) {
                    std::vector<double> load(s.prog->mP());
                    s.prog->read(4, load.data(), (int64_t)load.size());
                    lsd = level_set_density(s.dens_graph, load);
                }
                lo = std::max(lo, lsd);
            }
            if (feasible) {
                const double val = s.form == MWU_COVERING ? f.sumx / f.zmin : (f.ymax / f.sP) / f.zmin;
                if (val < hi) { hi = val; s.prog->save_best(); o.have_best_dev = true; o.best_scale = 1.0 / f.zmin; }
                shi = param;
            } else {
                if (c.status == ST_INFEASIBLE) lo = std::max(lo, param * cf);
                slo = param;
            }
        }
        slo = std::max(slo, lo);
        shi = std::min(shi, hi);
    }
    o.lower = lo;
    o.upper = hi;
    o.objective = s.form == MWU_PACKING ? lo : hi;
    o.status = hi <= (1.0 + eps) * lo ? MWU_CERTIFIED : MWU_FEASIBLE_UNCERTIFIED;
    return o;
}

}  // namespace mwu

// ================================================================== C ABI

using namespace mwu;

static mwu_status run_guarded(const std::function<void()> &f)
{
    try {
        f();
        return MWU_OK;
    } catch (const ApiError &e) {
        return e.code;
    } catch (const DeviceError &) {
        return MWU_ERR_DEVICE;
    } catch (const std::bad_alloc &) {
        return MWU_ERR_OOM;
    }
}

extern "C" {

void mwu_default_options(mwu_options *opt)
{
    if (opt) fill_defaults(opt);
}

const char *mwu_status_string(mwu_status st)
{
    switch (st) {
    case MWU_OK: return "MWU_OK";
    case MWU_ERR_INVALID_ARG: return "MWU_ERR_INVALID_ARG";
    case MWU_ERR_NEGATIVE_ENTRY: return "MWU_ERR_NEGATIVE_ENTRY";
    case MWU_ERR_NONFINITE: return "MWU_ERR_NONFINITE";
    case MWU_ERR_BAD_RHS: return "MWU_ERR_BAD_RHS";
    case MWU_ERR_GRAPH: return "MWU_ERR_GRAPH";
    case MWU_ERR_TOO_LARGE: return "MWU_ERR_TOO_LARGE";
    case MWU_ERR_OOM: return "MWU_ERR_OOM";
    case MWU_ERR_DEVICE: return "MWU_ERR_DEVICE";
    case MWU_ERR_UNBOUNDED: return "MWU_ERR_UNBOUNDED";
    case MWU_ERR_STATE: return "MWU_ERR_STATE";
    default: return "MWU_UNKNOWN";
    }
}

mwu_status mwu_create(const mwu_problem *prob, const mwu_options *opt, void **out)
{
    if (!out) return MWU_ERR_INVALID_ARG;
    *out = nullptr;
    if (!prob) return MWU_ERR_INVALID_ARG;
    Solver *s = new (std::nothrow) Solver();
    if (!s) return MWU_ERR_OOM;
    if (opt) s->opt = *opt; else fill_defaults(&s->opt);
    mwu_status st = run_guarded([&] { build(*s, *prob); });
    if (st != MWU_OK) { delete s; return st; }
    *out = s;
    return MWU_OK;
}

mwu_status mwu_create_batch(const mwu_problem *probs, int32_t count, const mwu_options *opt, void **out)
{
    if (!out) return MWU_ERR_INVALID_ARG;
    *out = nullptr;
    if (!probs || count < 1) return MWU_ERR_INVALID_ARG;
    for (int32_t k = 0; k < count; ++k)   // the batched program solves matching LPs
        if (probs[k].form != MWU_PACKING || probs[k].P.kind != MWU_MAT_INCIDENCE || probs[k].b_P || probs[k].c)
            return MWU_ERR_INVALID_ARG;
    Solver *s = new (std::nothrow) Solver();
    if (!s) return MWU_ERR_OOM;
    if (opt) s->opt = *opt; else fill_defaults(&s->opt);
    mwu_status st = run_guarded([&] {
        check(s->opt.eps > 0.0 && s->opt.eps < 1.0, MWU_ERR_INVALID_ARG, "eps must be in (0,1)");
        check(s->opt.max_iter >= 1 && s->opt.max_probes >= 1, MWU_ERR_INVALID_ARG, "bad iteration caps");
        check(s->opt.step_rule == MWU_STEP_STD || s->opt.step_rule == MWU_STEP_BIN ||
                  s->opt.step_rule == MWU_STEP_BIN_WARM || s->opt.step_rule == MWU_STEP_NEWTON,
              MWU_ERR_INVALID_ARG, "bad step rule");
        check(s->opt.precision == MWU_FP64 || s->opt.precision == MWU_MIXED_FP32_FP64, MWU_ERR_INVALID_ARG,
              "bad precision");
        s->fp32 = s->opt.precision == MWU_MIXED_FP32_FP64;
        s->form = MWU_PACKING;
        setup_device(*s);
        s->batch = make_batch_matching(*s, probs, count);
        s->n_user = s->batch->total_variables();
    });
    if (st != MWU_OK) { delete s; return st; }
    *out = s;
    return MWU_OK;
}

void mwu_destroy(void *h)
{
    delete static_cast<Solver *>(h);
}

int64_t mwu_num_variables(void *h)
{
    return h ? static_cast<Solver *>(h)->n_user : -1;
}

mwu_status mwu_batch_get_layout(void *h, mwu_batch_layout *out)
{
    if (!h || !out) return MWU_ERR_INVALID_ARG;
    Solver &s = *static_cast<Solver *>(h);
    if (!s.batch) return MWU_ERR_STATE;
    *out = s.batch->layout();
    return MWU_OK;
}

mwu_status mwu_batch_set_layout(void *h, const mwu_batch_layout *layout)
{
    if (!h || !layout) return MWU_ERR_INVALID_ARG;
    Solver &s = *static_cast<Solver *>(h);
    if (!s.batch) return MWU_ERR_STATE;
    if (!layout_valid(*layout)) return MWU_ERR_INVALID_ARG;
    return run_guarded([&] {
        HIP_OK(hipSetDevice(s.opt.device));
        s.batch->set_layout(*layout);
    });
}

mwu_status mwu_batch_probe_run(void *h, const double *params, int32_t max_iters, mwu_probe_info *info)
{
    if (!h || !params || max_iters < 0) return MWU_ERR_INVALID_ARG;
    Solver &s = *static_cast<Solver *>(h);
    if (!s.batch) return MWU_ERR_STATE;
    return run_guarded([&] {
        HIP_OK(hipSetDevice(s.opt.device));
        s.batch->probe_run(params, max_iters, info);
    });
}

mwu_status mwu_batch_probe_read(void *h, int32_t instance, int32_t which, double *out, int64_t len)
{
    if (!h || !out || len < 0) return MWU_ERR_INVALID_ARG;
    Solver &s = *static_cast<Solver *>(h);
    if (!s.batch) return MWU_ERR_STATE;
    return run_guarded([&] {
        HIP_OK(hipSetDevice(s.opt.device));
        s.batch->probe_read(instance, which, out, len);
    });
}

mwu_status mwu_solve(void *h, double *x_out, double *objective_out, int64_t *iterations_out,
                     mwu_result_info *info)
{
    if (!h) return MWU_ERR_INVALID_ARG;
    Solver &s = *static_cast<Solver *>(h);
    if (s.batch) {
        return run_guarded([&] {
            HIP_OK(hipSetDevice(s.opt.device));
            s.batch->solve(x_out, objective_out, iterations_out, info);
        });
    }
    return run_guarded([&] {
        HIP_OK(hipSetDevice(s.opt.device));
        const auto t0 = std::chrono::steady_clock::now();
        SolveOut o = solve_impl(s);
        if (x_out) {
            std::vector<double> xi(s.prog->n());
            if (o.have_best_dev) s.prog->best_to_host(xi.data());
            else xi = s.x_start;
            std::fill(x_out, x_out + s.n_user, 0.0);
            for (size_t i = 0; i < xi.size(); ++i) {
                const double sc = o.have_best_dev ? o.best_scale : 1.0;
                x_out[s.col_user[i]] = xi[i] * sc / s.col_c[i];
            }
        }
        const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        if (objective_out) *objective_out = o.objective;
        if (iterations_out) *iterations_out = o.total_iters;
        if (info) {
            info->status = o.status;
            info->objective = o.objective;
            info->lower_bound = o.lower;
            info->upper_bound = o.upper;
            info->total_iterations = o.total_iters;
            info->final_probe_iterations = o.final_iters;
            info->search_passes = o.passes;
            info->probes = o.probes;
            info->max_violation = o.max_violation;
            info->seconds_solve = secs;
            info->evaluations = o.evals;
        }
        s.in_probe = false;
    });
}

mwu_status mwu_probe_sizes(void *h, mwu_sizes *out)
{
    if (!h || !out) return MWU_ERR_INVALID_ARG;
    Solver &s = *static_cast<Solver *>(h);
    if (s.batch) return MWU_ERR_STATE;   // probe-level calls need a single problem
    out->n = s.prog->n();
    out->m_P = s.prog->mP();
    out->m_C = s.prog->mC();
    out->eta = 10.0 * std::log((double)(out->m_P + out->m_C)) / s.opt.eps;
    return MWU_OK;
}

mwu_status mwu_probe_begin(void *h, double param, const double *x0)
{
    if (!h || !(param > 0.0)) return MWU_ERR_INVALID_ARG;
    Solver &s = *static_cast<Solver *>(h);
    if (s.batch) return MWU_ERR_STATE;   // probe-level calls need a single problem
    return run_guarded([&] {
        HIP_OK(hipSetDevice(s.opt.device));
        s.prog->set_forced(nullptr, 0);
        begin_probe(s, param, x0);
        HIP_OK(hipStreamSynchronize(s.stream));
    });
}

static void fill_probe_info(const Ctl &c, mwu_probe_info *info)
{
    if (!info) return;
    info->status = c.status;
    info->iterations = c.iter;
    info->search_passes = c.search_passes;
    info->alpha = c.last_alpha;
    info->L_P = c.LP;
    info->L_C = c.LC;
    info->pack_bound = c.pack_bound;
    info->cover_bound = c.cover_bound;
    info->evaluations = c.evaluations;
}

mwu_status mwu_probe_run(void *h, int32_t max_iters, const double *forced_alpha, int32_t n_forced,
                         mwu_probe_info *info)
{
    if (!h || max_iters < 0 || n_forced < 0) return MWU_ERR_INVALID_ARG;
    Solver &s = *static_cast<Solver *>(h);
    if (s.batch) return MWU_ERR_STATE;   // probe-level calls need a single problem
    if (!s.in_probe) return MWU_ERR_STATE;
    return run_guarded([&] {
        HIP_OK(hipSetDevice(s.opt.device));
        pull_ctl(s);
        if (forced_alpha && n_forced > 0) {
            s.prog->set_forced(forced_alpha, n_forced);
            s.ctl_host->n_forced = n_forced;
            s.ctl_host->forced_pos = 0;
        } else {
            s.prog->set_forced(nullptr, 0);
            s.ctl_host->n_forced = 0;
        }
        s.ctl_host->eval_mode = 0;
        // pause after exactly max_iters more accepted steps
        s.ctl_host->iter_stop = (int32_t)std::min<int64_t>((int64_t)s.ctl_host->iter + std::max(1, max_iters),
                                                           INT32_MAX - 1);
        unpause(s);
        push_ctl(s);
        if (s.dir_pending) {
            // the direction of this iteration was formed by mwu_probe_direction:
            // continue at its step search, as an uninterrupted iteration would
            s.prog->resume_search();
            s.dir_pending = false;
        }
        run_probe(s, max_iters);
        pull_ctl(s);
        fill_probe_info(*s.ctl_host, info);
    });
}

mwu_status mwu_probe_direction(void *h)
{
    if (!h) return MWU_ERR_INVALID_ARG;
    Solver &s = *static_cast<Solver *>(h);
    if (s.batch) return MWU_ERR_STATE;   // probe-level calls need a single problem
    if (!s.in_probe) return MWU_ERR_STATE;
    return run_guarded([&] {
        pull_ctl(s);
        unpause(s);
        if (s.ctl_host->phase != PH_ROW) throw ApiError{MWU_ERR_STATE, "probe is not at an iteration start"};
        s.ctl_host->eval_mode = 1;
        push_ctl(s);
        s.prog->set_debug(true);
        s.prog->row_pass();
        s.prog->col_pass();
        s.prog->fwd_pass();
        s.prog->set_debug(false);
        HIP_OK(hipStreamSynchronize(s.stream));
        // the pending step is committed and the direction formed; the device
        // waits in PH_IDLE until mwu_probe_run resumes at the step search
        s.dir_pending = true;
    });
}

mwu_status mwu_probe_read(void *h, int32_t which, double *out, int64_t len)
{
    if (!h || !out) return MWU_ERR_INVALID_ARG;
    Solver &s = *static_cast<Solver *>(h);
    if (s.batch) return MWU_ERR_STATE;   // probe-level calls need a single problem
    return run_guarded([&] {
        if (which == 8) {   // accepted steps of the current probe
            pull_ctl(s);
            if (len != s.ctl_host->iter) throw ApiError{MWU_ERR_INVALID_ARG, "length mismatch"};
            if (len > 0) {
                HIP_OK(hipMemcpyAsync(out, s.trace_buf.p, (size_t)len * 8, hipMemcpyDeviceToHost, s.stream));
                HIP_OK(hipStreamSynchronize(s.stream));
            }
            return;
        }
        s.prog->read(which, out, len);
    });
}

// One evaluation pass of the candidates alphas[0..count) in evaluation mode
// (kind SK_NEWTON also forms Psi', Phi' at alphas[0]), with the
// refinements it needs; leaves the results in the host copy of the control
// block and the probe waiting at this iteration's step search (the
// evaluations change no vector, so mwu_probe_run resumes there).
static void eval_pass(Solver &s, int kind, const double *alphas, int count)
{
    if (!s.dir_pending) throw ApiError{MWU_ERR_STATE, "no direction formed (mwu_probe_direction)"};
    pull_ctl(s);
    Ctl &c = *s.ctl_host;
    c.skind = kind;
    c.ncand = count;
    for (int k = 0; k < KC; ++k) c.cand[k] = k < count ? alphas[k] : 0.0;
    c.ga0 = alphas[0];
    c.gdelta = 0.0;
    c.eval_mode = 1;
    c.ref_valid = 0;
    for (int k = 0; k < KC; ++k) c.ev_ok[k] = 1;
    c.phase = PH_SEARCH;
    push_ctl(s);
    for (int pass = 0; pass < 3 * KC + 2; ++pass) {
        s.prog->search_pass();
        pull_ctl(s);
        if (s.ctl_host->phase != PH_SEARCH) break;
    }
    if (s.ctl_host->phase != PH_IDLE) throw ApiError{MWU_ERR_STATE, "evaluation did not finish"};
}

static void eval_resume(Solver &s)
{
    s.ctl_host->eval_mode = 1;
    s.ctl_host->phase = PH_IDLE;
    push_ctl(s);
    HIP_OK(hipStreamSynchronize(s.stream));
}

mwu_status mwu_probe_eval_steps(void *h, const double *alphas, int32_t count, double *psi,
                                double *phi, double *zmin_new)
{
    if (!h || !alphas || count < 1 || count > KL || !psi || !phi) return MWU_ERR_INVALID_ARG;
    Solver &s = *static_cast<Solver *>(h);
    if (s.batch) return MWU_ERR_STATE;   // probe-level calls need a single problem
    if (!s.in_probe) return MWU_ERR_STATE;
    return run_guarded([&] {
        // a doubling ladder of KE values runs as the exponential-grid pass
        bool dbl = count == KE;
        for (int k = 1; k < count; ++k) {
            if (alphas[k] != 2.0 * alphas[k - 1]) dbl = false;
        }
        eval_pass(s, dbl ? SK_EXP : SK_LIST, alphas, count);
        const Ctl &r = *s.ctl_host;
        for (int k = 0; k < count; ++k) {
            psi[k] = r.ev_psi[k];
            phi[k] = r.ev_phi[k];
            if (zmin_new) zmin_new[k] = r.ev_zmin[k];
        }
        eval_resume(s);
    });
}

mwu_status mwu_probe_eval_newton(void *h, double alpha, double *psi, double *phi, double *dpsi,
                                 double *dphi)
{
    if (!h || !(alpha > 0.0) || !std::isfinite(alpha) || !psi || !phi || !dpsi || !dphi)
        return MWU_ERR_INVALID_ARG;
    Solver &s = *static_cast<Solver *>(h);
    if (s.batch) return MWU_ERR_STATE;   // probe-level calls need a single problem
    if (!s.in_probe) return MWU_ERR_STATE;
    return run_guarded([&] {
        eval_pass(s, SK_NEWTON, &alpha, 1);
        const Ctl &r = *s.ctl_host;
        *psi = r.ev_psi[0];
        *phi = r.ev_phi[0];
        *dpsi = r.ev_dpsi;
        *dphi = r.ev_dphi;
        eval_resume(s);
    });
}

mwu_status mwu_time_pass(void *h, int32_t which, int32_t reps, double *avg_us, double *bytes,
                         double *nnz)
{
    if (!h || which < 0 || which > 5 || reps < 1 || !avg_us) return MWU_ERR_INVALID_ARG;
    Solver &s = *static_cast<Solver *>(h);
    if (s.batch) return MWU_ERR_STATE;   // probe-level calls need a single problem
    if (!s.in_probe) return MWU_ERR_STATE;
    return run_guarded([&] {
        HIP_OK(hipSetDevice(s.opt.device));
        pull_ctl(s);
        unpause(s);
        if (s.ctl_host->phase != PH_ROW) throw ApiError{MWU_ERR_STATE, "probe is not at an iteration start"};
        // one direction so that d, Pd, Cd are those of a real iteration
        s.ctl_host->eval_mode = 1;
        push_ctl(s);
        s.prog->row_pass();
        s.prog->col_pass();
        s.prog->fwd_pass();
        pull_ctl(s);
        // the pending step is committed now: the probe resumes from this point
        Ctl resume = *s.ctl_host;
        Ctl &c = *s.ctl_host;
        c.eval_mode = 0;
        static const int phase_of[6] = {PH_ROW, PH_COL, PH_FWD, PH_SEARCH, PH_SEARCH, PH_SEARCH};
        c.hold = phase_of[which];
        c.phase = phase_of[which];
        c.alpha = 0.0;
        if (which == 4) {   // bisection grid of [1, 2] to depth 4
            c.skind = SK_GRID;
            c.ncand = KG;
            for (int k = 0; k < KC; ++k) c.cand[k] = 1.0 + (k + 1) / 16.0;
            c.ga0 = 1.0 + 1.0 / 16.0;
            c.gdelta = 1.0 / 16.0;
        } else if (which == 5) {   // exponential grid from 1 and the bisection tree of [2, 4]
            c.skind = SK_COMBO;
            c.ncand = KC;
            for (int k = 0; k < KE; ++k) c.cand[k] = std::ldexp(1.0, k);
            for (int k = 0; k < KG; ++k) c.cand[KE + k] = 2.0 + 2.0 * (k + 1) / 16.0;
            c.ga0 = 2.0 + 2.0 / 16.0;
            c.gdelta = 2.0 / 16.0;
        } else {            // exponential grid from 1
            c.skind = SK_EXP;
            c.ncand = KE;
            for (int k = 0; k < KC; ++k) c.cand[k] = std::ldexp(1.0, k);
            c.ga0 = 1.0;
            c.gdelta = 0.0;
        }
        push_ctl(s);
        // the pass's main kernel only (its finisher leaves a held state alone)
        auto launch = [&] { s.prog->main_kernel(which >= 4 ? 3 : which); };
        launch();   // warm caches
        hipEvent_t e0, e1;
        HIP_OK(hipEventCreate(&e0));
        HIP_OK(hipEventCreate(&e1));
        HIP_OK(hipEventRecord(e0, s.stream));
        for (int r = 0; r < reps; ++r) launch();
        HIP_OK(hipEventRecord(e1, s.stream));
        HIP_OK(hipEventSynchronize(e1));
        float ms = 0.0f;
        HIP_OK(hipEventElapsedTime(&ms, e0, e1));
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        *avg_us = 1000.0 * ms / reps;
        if (bytes) *bytes = s.prog->algo_bytes(which >= 4 ? 3 : which);
        if (nnz) *nnz = s.prog->pass_nnz(which >= 4 ? 3 : which);
        // The held launches rewrote the weights and the direction at the
        // committed point; the probe continues there with a full iteration
        // (a row pass with no step renormalizes the LSE totals and weights).
        resume.phase = PH_ROW;
        resume.alpha = 0.0;
        resume.hold = 0;
        resume.eval_mode = 0;
        *s.ctl_host = resume;
        push_ctl(s);
        s.dir_pending = false;
        HIP_OK(hipStreamSynchronize(s.stream));
    });
}

mwu_status mwu_potential_forward(void *h, const double *x_dev, double *value_out, void *stream)
{
    if (!h || !x_dev || !value_out) return MWU_ERR_INVALID_ARG;
    Solver &s = *static_cast<Solver *>(h);
    if (s.batch) return MWU_ERR_STATE;   // probe-level calls need a single problem
    if (!s.in_probe) return MWU_ERR_STATE;
    return run_guarded([&] {
        hipStream_t st = stream ? (hipStream_t)stream : s.stream;
        pull_ctl(s);
        s.ctl_host->eval_mode = 2;
        s.ctl_host->drop = 0;   // the potential is over every row
        HIP_OK(hipMemcpyAsync(s.ctl_buf.p, s.ctl_host, sizeof(Ctl), hipMemcpyHostToDevice, st));
        DevBuf val;
        val.alloc(8);
        s.dir_pending = false;
        s.prog->potential(x_dev, val.as<double>(), 1.0, nullptr, st);
        HIP_OK(hipMemcpyAsync(value_out, val.p, 8, hipMemcpyDeviceToHost, st));
        HIP_OK(hipStreamSynchronize(st));
        HIP_OK(hipMemcpy(s.ctl_host, s.ctl_buf.p, sizeof(Ctl), hipMemcpyDeviceToHost));
    });
}

mwu_status mwu_potential_backward(void *h, const double *x_dev, double grad_scale, double *grad_dev,
                                  void *stream)
{
    if (!h || !x_dev || !grad_dev) return MWU_ERR_INVALID_ARG;
    Solver &s = *static_cast<Solver *>(h);
    if (s.batch) return MWU_ERR_STATE;   // probe-level calls need a single problem
    if (!s.in_probe) return MWU_ERR_STATE;
    return run_guarded([&] {
        hipStream_t st = stream ? (hipStream_t)stream : s.stream;
        pull_ctl(s);
        s.ctl_host->eval_mode = 2;
        s.ctl_host->drop = 0;   // the potential is over every row
        HIP_OK(hipMemcpyAsync(s.ctl_buf.p, s.ctl_host, sizeof(Ctl), hipMemcpyHostToDevice, st));
        s.dir_pending = false;
        s.prog->potential(x_dev, nullptr, grad_scale, grad_dev, st);
        HIP_OK(hipStreamSynchronize(st));
        HIP_OK(hipMemcpy(s.ctl_host, s.ctl_buf.p, sizeof(Ctl), hipMemcpyDeviceToHost));
    });
}

mwu_status mwu_potential_backward_noalloc(void *h, const double *x_dev, double grad_scale, double *grad_dev,
                                          double *value_out, void *stream)
{
    if (!h || !x_dev || !grad_dev) return MWU_ERR_INVALID_ARG;
    Solver &s = *static_cast<Solver *>(h);
    if (s.batch) return MWU_ERR_STATE;   // probe-level calls need a single problem
    if (!s.in_probe) return MWU_ERR_STATE;
    return run_guarded([&] {
        HIP_OK(hipSetDevice(s.opt.device));
        void *scr = noalloc_scratch(s.opt.device);
        hipStream_t st = stream ? (hipStream_t)stream : s.stream;
        pull_ctl(s);
        s.ctl_host->eval_mode = 2;
        s.ctl_host->drop = 0;   // the potential is over every row
        HIP_OK(hipMemcpyAsync(s.ctl_buf.p, s.ctl_host, sizeof(Ctl), hipMemcpyHostToDevice, st));
        s.dir_pending = false;
        if (!s.prog->potential_static(x_dev, grad_scale, grad_dev, scr, kNoAllocScratchBytes, st))
            throw ApiError{MWU_ERR_TOO_LARGE, "reduction records and chunk partials exceed the static scratch"};
        HIP_OK(hipStreamSynchronize(st));
        HIP_OK(hipMemcpy(s.ctl_host, s.ctl_buf.p, sizeof(Ctl), hipMemcpyDeviceToHost));
        // after the row pass L_P and L_C are smax(Px) and smin(Cx) at x
        if (value_out) *value_out = s.ctl_host->LP - s.ctl_host->LC;
    });
}

}  // extern "C"
