// Internal definitions shared by the host driver (solver.cpp and the
// program_*.cpp files) and the gfx950 kernels (the .hip files).  Not part of the public C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace mwu {

constexpr int BLOCK = 256;               // threads per workgroup (4 wave64)
constexpr int ITEMS = 8;                 // nonzeros per thread in a segment tile
constexpr int TILE_NZ = BLOCK * ITEMS;   // nonzeros per tile
constexpr int KE = 8;                    // candidates of an exponential-grid pass (1 .. 128 from a0 = 1)
constexpr int KG = 15;                   // candidates of a bisection pass (complete tree of depth 4)
constexpr int KC = KE + KG;              // most step candidates in one search pass
constexpr int KL = 16;                   // most candidates of a list pass (direct evaluation)
constexpr int KN = KL - 1;               // values of a Newton pass; its slot KN holds the derivative sums
constexpr int QMAX = 4 * KC + 8;         // doubles per block in a reduction record

// Phase of the per-probe state machine.  Every kernel of the iteration graph
// runs only in its own phase and returns at once otherwise, so a graph that
// captures a fixed launch sequence can follow a data-dependent number of
// search passes.
enum Phase : int32_t {
    PH_IDLE = 0,
    PH_ROW = 1,      // apply pending step to the rows, weights and LSE totals
    PH_COL = 2,      // apply pending step to x, transpose product, direction
    PH_FWD = 3,      // forward product of the direction
    PH_SEARCH = 4,   // K-candidate step search passes
    PH_COMMIT = 5,   // apply pending step to x only, then stop
    PH_DONE = 6,
    // batched program only
    PH_INIT = 7,     // probe start: x = x0
    PH_INIT_Y = 8,   // probe start: y = P x0 and the first LSE shift
    PH_STATS = 9     // probe ended: FP64 statistics of x, then PH_IDLE
};

enum Status : int32_t { ST_RUNNING = 0, ST_FEASIBLE = 1, ST_INFEASIBLE = 2, ST_MAX_ITER = 3,
                        ST_NUMERIC = 4 };

// Kind of candidate set evaluated by one search pass.
enum SKind : int32_t {
    SK_EXP = 0,      // cand[k] = a0 * 2^k           (exponential phase of Algorithm 3)
    SK_GRID = 1,     // cand[j] ~ a0 + j * delta      (bisection tree of depth 4)
    SK_LIST = 2,     // arbitrary values, direct evaluation
    SK_REFINE = 3,   // one value, max-shifted evaluation of both LSE differences
    SK_COMBO = 4,    // the exponential grid from 1 (KE) followed by the bisection tree of the
                     // octave the previous step fell in (KG): cand[KE + j] ~ ga0 + j * delta
    SK_NEWTON = 5    // a list pass (at most KN values, the Newton iterate first) that also
                     // forms, in slot KN, the sums of Psi' and Phi' at cand[0]
};

enum AMode : int32_t { AM_EXP = 0, AM_BIS = 1, AM_FORCED = 2, AM_EVAL = 3, AM_DOWN = 4, AM_NEWTON = 5,
                       AM_BACKOFF = 6 };
// Ctl::step_rule values (the MWU_STEP_* of the C interface)
enum StepRule : int32_t { SR_STD = 0, SR_BIN = 1, SR_BIN_WARM = 2, SR_NEWTON = 3 };

// A contiguous piece of a CSR-like structure handled by one workgroup:
// segments [s0, s1) with nonzeros [k0, k1).  A segment longer than TILE_NZ is
// split into chunk tiles (lid >= 0): chunk cidx of long segment lid.
struct Tile {
    int32_t s0, s1, k0, k1, lid, cidx;
};

// Device-resident control block of one probe (one per handle).
struct Ctl {
    // ---- configuration (set by the host at probe start)
    double eta, eps, step;      // step = s / eta of the direction formula
    double sP, sC;              // uniform scale of P and C (1/M, 1/D or 1)
    double psi_lim;             // largest eta*alpha*max(dy) for the expm1 form
    double s2_min;              // smallest trusted direct sum of the C-side LSE
    double qmin;                // d_i = 0 unless 1 - g_i/h_i exceeds this (0 in FP64)
    int32_t onesP, onesC;       // side is the implicit objective row (1 row, all ones)
    int32_t step_rule, max_iter;
    int32_t n_forced, forced_pos;
    int32_t eval_mode, ev_cur;
    int32_t hold;               // nonzero: finishers keep this phase and change nothing (timing)
    int32_t iter_stop;          // > 0: a probe pauses (PH_IDLE, still running) once iter reaches it
    // ---- status
    int32_t status, phase, iter, pad1;
    int64_t search_passes, evaluations;
    // ---- point state
    double alpha;               // pending step (applied by the next row/column pass)
    double LP, LC;              // LSE totals; predicted before a row pass, exact after
    double LCw;                 // shift the stored/recomputed covering weights were formed with
    double invSw, invSu;        // 1 / sum of the stored (unnormalized) weights
    double y1, z1, dy1, dz1;    // value of an implicit objective row and of its product with d
    double dymax;               // max over packing rows of P d
    double dmax, dsum;
    double ymax, zmin;
    double gmin, hmax;          // of the last direction (certificates)
    double pack_bound, cover_bound;
    double last_alpha;
    double sumx;                // sum of x (init / final statistics)
    double *trace;              // nullable device array: accepted step of each iteration
    int32_t trace_cap;
    int32_t drop;               // nonzero: covering rows with z >= 1 are left out (weight 0)
    // ---- sparse passes (fused vertex cover): covering rows whose weight is
    // exactly zero in the storage type are left out of the passes
    int32_t act_on, act_ne;     // lists built; edges in the active search list
    int32_t act_nitems;         // work items of the packed transpose pass
    int32_t psi_shift;          // search passes form max-shifted packing sums past psi_lim
    int32_t pass_sparse;        // the last search pass ran over the active list
    int32_t ev_cached;          // ev_* hold the evaluations of the last grid or list pass
    double act_L;               // weight shift the lists were built against
    double act_mu;              // eta * (shift drift) the lists stay valid for
    double act_zfloor;          // min z over the left-out edges when the lists were built
    // ---- search state (replay of Algorithm 3)
    int32_t skind, ncand, amode, have_cur;
    double cand[KC];
    double ga0, gdelta;
    double exp_next, cur_alpha, cur_psi, cur_phi;
    double lb, ub, lb_psi, lb_phi;
    int32_t ref_valid, nw_evals;       // nw_evals: Newton evaluations of this search
    int32_t ref_short, ref_pad;        // ref_short: the pending refinement took its shifts from the grid pass
    double ref_alpha, ref_psi, ref_phi, ref_zmin;
    double ref_dpsi, ref_dphi;          // Psi', Phi' at ref_alpha (refine pass 2)
    double ev_dpsi, ev_dphi;            // evaluation mode: Psi', Phi' at cand[0] of a Newton pass
    // results of the last grid pass (raw sums, before normalization)
    double rS1P[KC], rS1C[KC], rS2C[KC], rZmin[KC];
    // results of the last refine pass (max-shifted pairs)
    double rfPm, rfPs, rfCm, rfCs, rfZmin;
    // evaluation outputs (probe API)
    double ev_psi[KC], ev_phi[KC], ev_zmin[KC];
    int32_t ev_ok[KC];
};

// Long segments (longer than one tile) are split into chunk tiles whose
// partial sums the finisher kernel of the pass folds: lseg[l] is the segment,
// its chunks are partial slots lfirst[l] .. lfirst[l] + lcount[l] - 1.
struct LongSegs {
    const int32_t *lseg, *lfirst, *lcount;
    int32_t nlong;
};

// Generic engine over explicit CSR sides.  Rows of P (if not the implicit
// objective row) come first in the concatenated row space, then rows of C.
template <class T>
struct GenericDev {
    int32_t n, mPc, mR;                 // variables, explicit P rows, all explicit rows
    // row structure (forward products)
    const int32_t *rptr, *rcol;
    const T *rval;                      // nullable: all ones
    const Tile *rtiles; int32_t nrtiles;
    LongSegs rlong;
    T *rlpart;                          // chunk partials of the forward products
    double *rlpart64;                   // chunk partials of the FP64 statistics
    // column structure (transpose products); crow indexes the row space
    const int32_t *cptr, *crow;
    const T *cval;                      // nullable
    const Tile *ctiles; int32_t nctiles;
    LongSegs clong;
    void *clpart;                       // chunk partials (g, h pairs) of the transpose products
    const double *colmaxP;              // max_j P_ji (unscaled) per column, nullable if onesP
    // vectors
    T *x, *d, *yz, *dyz, *wu;
    double *g_dbg, *h_dbg;              // nullable: debug copies of g, h
    double *grad;                       // nullable: grad_scale (g - h) per column
    double grad_scale;
    const double *forced;               // forced steps (host-provided), nullable
    const int32_t *cmap;                // nullable: internal column -> the caller's column, for
                                        // vectors in the caller's order (a given x, the gradient)
};

// Fused vertex-cover program: C = M^T read from the edge list, P = the
// objective row.  Edge-indexed vectors (z = x_u + x_v, dz, u) are never
// stored; every pass recomputes them from the vertex vectors.
template <class T>
struct XD { T x, d; };

template <class T>
struct VcDev {
    int32_t nv, ne;
    const int32_t *eu, *ew;             // edges (u, w), u < w, sorted: one visit per covering row
    const int32_t *fptr, *fcol;         // full adjacency (both directions)
    const Tile *ftiles; int32_t nftiles;
    LongSegs flong;
    T *flpart;
    XD<T> *xd;                          // x and d interleaved (one 2T gather per edge endpoint)
    T *xs;                              // copy of x for the transpose pass (half the footprint)
    T *h;                               // unnormalized C^T u per vertex
    double *h_dbg;                      // nullable
    const double *forced;
    // sparse passes: the active neighbours of each adjacency tile packed at
    // the start of its range, the packed row starts and the tiles' active
    // counts; the same neighbours concatenated over all tiles (ccol, row
    // starts cst, tile offsets goff) and the work items of the packed pass
    // (runs of consecutive tiles that fit one tile together); the static row
    // prefix over tiles; the active edges of the search in edge-list order;
    // per-block counts of the build
    int32_t *fcol_pk, *fptr_pk, *tile_na, *ccol, *cst, *goff, *tile_rows, *thead, *thpos;
    Tile *items;
    int32_t *aeu, *aew, *acnt;
    // long rows completed by pass B from the chunk partials of pass A (in
    // chunk order): the vertices [0, nlong_b) of the degree order when there
    // are more than the pass A finisher takes, else 0
    int32_t nlong_b;
};

// Fused densest-subgraph program: the variables of edge e are its two ends;
// vertex rows (packing, scaled by 1/D) are segmented sums over vptr/vvar,
// edge rows (covering) are pairs.  Internally vertices are numbered by
// descending degree and edges sorted by (first end, second end), and the
// variables are two arrays: the first end of internal edge e at e, its second
// end at ne + e.  A vertex's first-end variables are then one contiguous run
// and its second-end variables advance together with those of its
// neighbouring ids.  Every variable lies in one row
// of each side, so g_i and h_i are single weights and nothing averages the
// rounding of the direction out: the iterate x, the direction d, the rows y,
// z, the products Pd, Cd and the LSE totals are FP64 in both forms.  T is the
// type of the stored weights w, u and of the search terms built from them.
template <class T>
struct DnDev {
    int32_t nv, ne, n;                    // non-isolated vertices, edges, variables (2 ne)
    const int32_t *vptr, *vvar;           // variables of each vertex row
    const Tile *vtiles;
    int32_t nvtiles;
    LongSegs vlong;
    double *lpart;                        // chunk partials of the forward products
    double *lpart64;                      // chunk partials of the statistics
    const int32_t *eu, *ev;               // first and second end of internal edge e (eu[e] < ev[e])
    const int32_t *cpos;                  // caller's index (2e' + j) of internal variable p
    double *x, *d;                        // variables: [first ends (ne) | second ends (ne)]
    double *y;                            // vertex rows (scaled by sP)
    double *dy;
    T *w;
    double *z;                            // edge rows
    double *dz;
    T *u;
    double *g_dbg, *h_dbg;                // nullable
    double *grad;                         // nullable: grad_scale (g - h) per variable
    double grad_scale;
    const double *forced;
};

struct DnLaunch {
    int grid_vt, grid_e, grid_n, grid_r, grid_s;
    double *partials, *partials2;
};

template <class T> void dn_init(const DnDev<T> &dd, Ctl *ctl, const DnLaunch &L, hipStream_t st, bool have_x0,
                                const double *src);
template <class T> void dn_row_pass(const DnDev<T> &dd, Ctl *ctl, const DnLaunch &L, hipStream_t st);
template <class T> void dn_col_pass(const DnDev<T> &dd, Ctl *ctl, const DnLaunch &L, hipStream_t st);
template <class T> void dn_fwd_pass(const DnDev<T> &dd, Ctl *ctl, const DnLaunch &L, hipStream_t st);
template <class T> void dn_search_pass(const DnDev<T> &dd, Ctl *ctl, const DnLaunch &L, hipStream_t st);
template <class T> void dn_iteration(const DnDev<T> &dd, Ctl *ctl, const DnLaunch &L, hipStream_t st);
template <class T> void dn_stats(const DnDev<T> &dd, Ctl *ctl, const DnLaunch &L, hipStream_t st);
template <class T> void dn_main(const DnDev<T> &dd, Ctl *ctl, const DnLaunch &L, hipStream_t st, int which);
template <class T> void dn_occupancy(int *per_cu_vt, int *per_cu_search);
template <class T> void dn_backcounts(const DnDev<T> &dd, const int32_t *rank, int32_t *back, hipStream_t st);
// dst[cpos[p]] = src[p] for p < n (internal variables to the caller's order)
void dn_to_caller(const double *src, const int32_t *cpos, double *dst, int64_t n, hipStream_t st);

// Batched matching program: many independent packing LPs max 1^T x s.t.
// M_k x <= 1 (bipartite matching, Section 3) in concatenated arrays.  Tiles
// never cross instances; every tile of a pass writes one record, and the
// finisher of instance k folds its contiguous range of tile records.
struct BTile {
    int32_t inst, i0, i1;   // instance; item range (vertices or edges)
    int32_t k0, k1;         // vertex tiles: incidence nonzeros [k0, k1) (nnz-balanced)
    int32_t lid, cidx;      // vertex tiles: chunk cidx of long vertex lid (lid < 0: whole vertices)
    int32_t pad;
};

template <class T>
struct BatchDev {
    int32_t nb, nv, ne;
    const int32_t *vptr, *vedge;          // incident edges of each vertex (global edge ids)
    const int32_t *eu, *ev;               // endpoints of each edge (global vertex ids)
    T *x, *d;                             // per edge (variables)
    T *y, *dy, *w;                        // per vertex (packing rows)
    const BTile *vt, *et;                 // vertex tiles, edge tiles (grouped by instance)
    int32_t nvt, net;
    const int32_t *vrec0, *vrecn;         // per instance: first vertex tile, count
    const BTile *wt;                      // element tiles over vertices (row and search passes)
    int32_t nwt;
    const int32_t *wrec0, *wrecn;         // per instance: first element tile, count
    double *wpart;                        // one record per element tile
    const int32_t *erec0, *erecn;         // per instance: first edge tile, count
    const int32_t *nedge;                 // per instance: number of edges (variables)
    LongSegs vlong;                       // vertices longer than one tile (global long ids)
    const int32_t *lrec0, *lrecn;         // per instance: first long vertex, count
    T *lpart;                             // chunk partials (storage type)
    double *lpart64;                      // chunk partials of the FP64 statistics
    Ctl *ctl;                             // one control block per instance
    int32_t *stat;                        // per instance: phase, status, iter, serial
    double *vpart, *epart;                // one record (QMAX doubles) per tile
};

struct BLaunch {
    int grid_v, grid_e, grid_w;           // persistent grids over vertex / edge / element tiles
    int nsearch;                          // search passes launched per iteration slot
};

template <class T> void batch_slots(const BatchDev<T> &b, const BLaunch &L, int slots, hipStream_t st);
template <class T> void batch_occupancy(int *per_cu_v, int *per_cu_e);

// Launch helpers implemented in the .hip files.
struct Launch {
    int grid_elem_rows;  // persistent grid for element-wise passes over rows
    int grid_elem_cols;  // persistent grid for element-wise passes over columns
    int grid_rtile;      // persistent grid for row tiles
    int grid_ctile;      // persistent grid for column tiles
    int grid_search;     // persistent grid of the search pass
    double *partials;    // GRID_MAX * QMAX doubles: one reduction record per workgroup
};

constexpr int GRID_MAX = 2048;

// Probe start: x0 (Algorithm 1 point unless have_x0), y = Px, z = Cx and the
// max/min used as the first LSE shift.  Leaves the state machine in PH_ROW.
template <class T> void generic_init(const GenericDev<T> &g, Ctl *ctl, const Launch &L,
                                     hipStream_t st, bool have_x0);
// One iteration slot of the graph: row pass, column pass, forward pass and
// two search passes (each a no-op outside its phase).
template <class T> void generic_iteration(const GenericDev<T> &g, Ctl *ctl, const Launch &L,
                                          hipStream_t st);
// FP64 statistics of x: sum x, max over packing rows, min over covering rows.
template <class T> void generic_stats(const GenericDev<T> &g, Ctl *ctl, const Launch &L,
                                      hipStream_t st, const double *rval64);
// Individual passes (probe API).
template <class T> void generic_row(const GenericDev<T> &g, Ctl *ctl, const Launch &L, hipStream_t st);
template <class T> void generic_col(const GenericDev<T> &g, Ctl *ctl, const Launch &L, hipStream_t st);
template <class T> void generic_fwd(const GenericDev<T> &g, Ctl *ctl, const Launch &L, hipStream_t st);
template <class T> void generic_search(const GenericDev<T> &g, Ctl *ctl, const Launch &L,
                                       hipStream_t st);
// Copy a double device vector into x (T) and compute sum(x) into the control block.
template <class T> void generic_load_x(const GenericDev<T> &g, Ctl *ctl, const Launch &L,
                                       hipStream_t st, const double *x_dev);
// out[i] = scale * (g_dbg[i] - h_dbg[i]); val (nullable) = LP - LC.
// out[map[i]] = scale (g_i - h_i) (map nullable: the identity); val = LP - LC
void potential_finish(const double *g_dbg, const double *h_dbg, int n, double scale, double *out,
                      const int32_t *map, const Ctl *ctl, double *val, hipStream_t st);
// Copy a device vector of T to a double device vector.
template <class T> void widen(const T *src, double *dst, int64_t n, hipStream_t st);
template <class T> void narrow(const double *src, T *dst, int64_t n, hipStream_t st);
// Set ctl->phase (single thread).
void set_phase(Ctl *ctl, int phase, hipStream_t st);
// v[i * stride] *= th for i < n (a probe started from a scaled earlier point)
template <class T> void scale_vec(T *v, int64_t n, int64_t stride, double th, hipStream_t st);
// Every entry of one row set to v: its row-structure values rval[k0, k0+n)
// (and the FP64 copy), its column-structure values cval[pos[j]]; with colmax
// (an objective row among the packing rows) colmax[j] = max(base[j], v).
template <class T> void generic_set_row(T *rval, double *rval64, int64_t k0, int64_t n, T *cval,
                                        const int32_t *pos, double v, double *colmax, const double *base,
                                        hipStream_t st);
// Continue a probe whose direction was formed in evaluation mode: the stop
// tests of the iteration, then its step search (forced: the program's forced
// steps, nullable).
void resume_search(Ctl *ctl, const double *forced, hipStream_t st);

struct VcLaunch {
    int grid_v;        // element-wise over vertices
    int grid_ftile;    // full-adjacency tiles
    int grid_e;        // edge passes (search, min z, export)
    int grid_act;      // blocks of the active-list build (contiguous edge ranges)
    double *partials;
};
template <class T> void vc_init(const VcDev<T> &v, Ctl *ctl, const VcLaunch &L, hipStream_t st,
                                bool have_x0);
template <class T> void vc_iteration(const VcDev<T> &v, Ctl *ctl, const VcLaunch &L, hipStream_t st);
template <class T> void vc_passA(const VcDev<T> &v, Ctl *ctl, const VcLaunch &L, hipStream_t st);
template <class T> void vc_passB(const VcDev<T> &v, Ctl *ctl, const VcLaunch &L, hipStream_t st);
template <class T> void vc_search(const VcDev<T> &v, Ctl *ctl, const VcLaunch &L, hipStream_t st);
// Build the active lists against the current weight shift (margin mu).
template <class T> void vc_build_active(const VcDev<T> &v, Ctl *ctl, const VcLaunch &L, hipStream_t st,
                                        double mu);
// which: 0 = x, 1 = d (vertex vectors, double out); 2 = z, 3 = dz (edge vectors, canonical order)
template <class T> void vc_export(const VcDev<T> &v, int which, double *out, hipStream_t st);
template <class T> void vc_import_x(const VcDev<T> &v, const double *src, hipStream_t st);
template <class T> void vc_occupancy(int *per_cu_ftile, int *per_cu_edge);
template <class T> void generic_occupancy(int *per_cu_fwd, int *per_cu_col, int *per_cu_search);
// Main kernel of pass `which` (0 row, 1 column, 2 forward, 3 search) alone.
template <class T> void generic_main(const GenericDev<T> &g, Ctl *ctl, const Launch &L, hipStream_t st,
                                     int which);
template <class T> void vc_main(const VcDev<T> &v, Ctl *ctl, const VcLaunch &L, hipStream_t st, int which);

}  // namespace mwu
