// Host-side internal structures of the solver library.
#pragma once

#include <cstdint>
#include <functional>
#include <memory>
#include <string>
#include <vector>

#include "../../include/mwu.h"
#include "engine.h"

namespace mwu {

#define HIP_OK(expr)                                                    \
    do {                                                                \
        hipError_t e_ = (expr);                                         \
        if (e_ != hipSuccess) throw DeviceError(e_, #expr);             \
    } while (0)

struct DeviceError {
    hipError_t code;
    const char *what;
    DeviceError(hipError_t c, const char *w) : code(c), what(w) {}
};

struct ApiError {
    mwu_status code;
    std::string msg;
};

// Explicit CSR on the host (normalized values).
struct HostCSR {
    int64_t rows = 0, cols = 0;
    std::vector<int64_t> ptr;
    std::vector<int32_t> idx;
    std::vector<double> val;   // empty = every entry is 1
    int64_t nnz() const { return ptr.empty() ? 0 : ptr.back(); }
    double v(int64_t k) const { return val.empty() ? 1.0 : val[k]; }
};

// Edge list after validation (caller order) for the graph programs.
struct EdgeList {
    int64_t nv = 0, ne = 0;
    std::vector<int32_t> u, v;
};

// Owning device buffer.
struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    ~DevBuf() { if (p) (void)hipFree(p); }
    void alloc(size_t b) {
        if (p) { (void)hipFree(p); p = nullptr; }
        bytes = b;
        if (b == 0) return;
        hipError_t e = hipMalloc(&p, b);
        if (e != hipSuccess) { p = nullptr; throw ApiError{MWU_ERR_OOM, "device allocation failed"}; }
    }
    template <class T> T *as() const { return static_cast<T *>(p); }
};

// Size of the static device scratch of mwu_potential_backward_noalloc
// (noalloc.hip): the reduction records of two passes (2 x GRID_MAX x QMAX
// doubles, 3.1 MiB) and the chunk partials of the long rows and columns.
constexpr size_t kNoAllocScratchBytes = (size_t)8 << 20;
// Device address of this GPU's scratch array (the device must be current).
void *noalloc_scratch(int device);

// Interface of a device program (the generic CSR engine, the fused graph
// programs).  All launches go to the solver stream.
struct Program {
    virtual ~Program() {}
    virtual int64_t n() const = 0;
    virtual int64_t mP() const = 0;     // packing rows as the method sees them
    virtual int64_t mC() const = 0;
    virtual void probe_init(bool have_x0) = 0;
    virtual void upload_x(const double *host_x) = 0;   // host double -> device x
    virtual void scale_x(double th) = 0;               // device x *= th (the next probe's start)
    virtual void iterations(int slots) = 0;            // enqueue iteration slots
    virtual void final_stats() = 0;                    // fresh Px, Cx statistics into ctl
    virtual void save_best() = 0;
    virtual void best_to_host(double *out) = 0;        // internal variable space
    virtual void read(int which, double *out, int64_t len) = 0;
    virtual void row_pass() = 0;
    virtual void col_pass() = 0;
    virtual void fwd_pass() = 0;
    virtual void search_pass() = 0;
    virtual void main_kernel(int which) = 0;          // a pass's main kernel alone (timing)
    virtual void potential(const double *x_dev, double *val_dev, double scale, double *grad_dev,
                           hipStream_t st) = 0;
    // The same gradient with every record and chunk partial in the caller's
    // scratch (no allocation): grad = scale (g - h) written by the column
    // pass.  False when the scratch is too small for this problem.
    virtual bool potential_static(const double *, double, double *, void *, size_t, hipStream_t)
    {
        throw ApiError{MWU_ERR_STATE, "this program has no potential (use MWU_FLAG_GENERIC)"};
    }
    virtual void set_debug(bool on) = 0;
    virtual void set_forced(const double *host, int count) = 0;
    // Continue the probe after a direction formed in evaluation mode
    // (mwu_probe_direction): its stop tests, then the step search.
    virtual void resume_search() = 0;
    // Algorithmic HBM bytes of one launch of a pass (0 row/transpose, 1 column/direction,
    // 2 forward, 3 search): every index once, every dense vector once, every output once.
    virtual double algo_bytes(int which) const = 0;
    virtual double pass_nnz(int which) const = 0;
    // Called by the probe driver after every graph launch with the pulled
    // control block; may enqueue work on the solver stream before the next.
    virtual void between_launches(const Ctl &) {}
    // Level-set rounding of the current vertex loads (densest subgraph):
    // false when the program has no such structure (the host computes it).
    virtual bool level_set_density(double *) { return false; }
    // Mixed optimization (MWU_MIXED_MAX/MIN): the embedded objective row's
    // value v = 1/M on every entry, set before each probe.
    virtual void set_objective_level(double) { throw ApiError{MWU_ERR_STATE, "no objective row"}; }
};

// Many independent problems solved together (the batched programs).
struct BatchProgram {
    virtual ~BatchProgram() {}
    virtual int32_t count() const = 0;
    virtual int64_t total_variables() const = 0;
    // x_out: concatenated variables of all instances (nullable); obj_out and
    // info: one entry per instance (nullable); iters_out: total iterations.
    virtual void solve(double *x_out, double *obj_out, int64_t *iters_out, mwu_result_info *info) = 0;
    virtual mwu_batch_layout layout() const = 0;
    virtual void set_layout(const mwu_batch_layout &L) = 0;   // L already validated
    // One probe on every instance at once (instance k at params[k]), in the
    // batched kernels, pausing after max_iters accepted steps (0: no pause);
    // info: one entry per instance (nullable).
    virtual void probe_run(const double *params, int32_t max_iters, mwu_probe_info *info) = 0;
    // A vector of instance k after probe_run (the mwu_probe_read codes 0 x,
    // 1 d, 4 y, 6 dy, 8 accepted steps).
    virtual void probe_read(int32_t k, int32_t which, double *out, int64_t len) = 0;
};

// Autotuner of batched layouts (autotune.cpp).
bool layout_valid(const mwu_batch_layout &L);
mwu_batch_layout default_layout();
std::string tune_key(const char *program, bool fp32, int device, int num_cus, int32_t count, int64_t nv,
                     int64_t ne, int64_t max_ne);
bool tune_lookup(const std::string &key, const char *path, mwu_batch_layout *L, double *rate);
void tune_store(const std::string &key, const char *path, const mwu_batch_layout &L, double rate);
// One coordinate-descent pass over the fields in order (tile_edges,
// tile_vertices, workgroups_per_cu, search_launches); cands[f] lists the
// values tried for field f; rate() times a layout (higher is better).
mwu_batch_layout tune_descent(const mwu_batch_layout &start, const std::vector<std::vector<int32_t>> &cands,
                              const std::function<double(const mwu_batch_layout &)> &rate, int *timed,
                              double *best_rate);

struct Solver {
    mwu_options opt{};
    mwu_form form = MWU_PACKING;
    int onesP = 0, onesC = 0;
    bool fp32 = true;
    int64_t n_user = 0;
    std::vector<int64_t> col_user;   // internal column -> caller variable
    std::vector<double> col_c;       // c_j of the internal column (x_user = x'/c)
    // outer-search starting bracket and trivially feasible points
    double lo0 = 0, hi0 = 0;
    std::vector<double> x_start;     // rescaled feasible start (internal space)
    // densest subgraph level-set rounding (mixed problems built from an edge list)
    bool level_sets = false;
    EdgeList dens_graph;             // non-isolated vertex ids, canonical
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int num_cus = 256;
    int device = 0;
    DevBuf ctl_buf;
    DevBuf trace_buf;                // accepted steps of the current probe (max_iter doubles)
    Ctl *ctl_host = nullptr;         // pinned mirror
    std::unique_ptr<Program> prog;
    std::unique_ptr<BatchProgram> batch;
    hipGraphExec_t graph = nullptr;
    int graph_slots = 0;
    bool in_probe = false;
    bool dir_pending = false;        // a direction was formed in evaluation mode: resume at its search
    double probe_param = 0.0;
    ~Solver();
};

struct TilePlan {
    std::vector<Tile> tiles;
    std::vector<int32_t> lseg, lfirst, lcount;   // long segments and their chunk slots
    int32_t nslots = 0;
};
TilePlan build_tiles(const std::vector<int32_t> &ptr, int64_t nseg);

// Program builders.
// obj_row: index (in the concatenated packing-then-covering row space) of an
// embedded objective row whose values set_objective_level rewrites, or -1.
std::unique_ptr<Program> make_generic_program(Solver &s, const HostCSR *P, const HostCSR *C,
                                              int64_t obj_row = -1);
// Vertex cover from a validated edge list; newid maps vertices to compact ids (-1 = isolated).
// Densest subgraph from the edge list of an (O/D, W) problem; vid maps vertices
// to compact ids (-1 isolated), in vertex order.
std::unique_ptr<Program> make_densest_program(Solver &s, const EdgeList &el, const std::vector<int64_t> &vid,
                                              int64_t nv);
std::unique_ptr<BatchProgram> make_batch_matching(Solver &s, const mwu_problem *probs, int32_t count);
std::unique_ptr<Program> make_vcover_program(Solver &s, const EdgeList &el,
                                             const std::vector<int64_t> &newid, int64_t nv);

}  // namespace mwu
