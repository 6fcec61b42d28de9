// Device building blocks shared by the gfx950 programs: deterministic
// block/grid reductions, nnz-balanced segment tiles, and the step-search
// replay that runs on the device after each search pass.
#pragma once

#include "engine.h"

namespace mwu {

#define MWU_DEV __device__ __forceinline__

// ------------------------------------------------------------------ math

MWU_DEV float expm1_t(float v) { return expm1f(v); }
MWU_DEV double expm1_t(double v) { return expm1(v); }
MWU_DEV float exp_t(float v) { return expf(v); }
MWU_DEV double exp_t(double v) { return exp(v); }

// e^v for a double argument, returned in T.  Float: the argument is split
// in base 2 in double, v log2(e) = n + f with |f| <= 1/2, so the hardware
// 2^f (v_exp_f32, about 1 ulp) sees a small reduced argument and ldexp adds
// n exactly; the result carries no error from rounding a large argument to
// float.  The argument is first clamped to |v| <= 1e4 (far outside the
// float range either way): beyond 2^52 the contracted v log2(e) - n keeps the
// product's rounding error, which can exceed the range of 2^f.  Double: the
// library exp.
MWU_DEV float exp_arg(double v, float)
{
    const double a = fmin(fmax(v, -1.0e4), 1.0e4) * 1.4426950408889634;
    const double n = rint(a);
    return ldexpf(__builtin_amdgcn_exp2f((float)(a - n)), (int)fmax(n, -300.0));
}
MWU_DEV double exp_arg(double v, double) { return exp(v); }

// ------------------------------------------------------------ reductions
// A reduction record holds ns sums, then nmn minima, then nmx maxima.

struct Red {
    int ns, nmn, nmx;
    MWU_DEV int q() const { return ns + nmn + nmx; }
};

MWU_DEV double red_op(double a, double b, int q, Red r)
{
    if (q < r.ns) return a + b;
    if (q < r.ns + r.nmn) return fmin(a, b);
    return fmax(a, b);
}

MWU_DEV double red_id(int q, Red r)
{
    if (q < r.ns) return 0.0;
    if (q < r.ns + r.nmn) return INFINITY;
    return -INFINITY;
}

// Reduce-scatter inside a wave64.  The Q values of every lane are halved at
// each exchange while Q stays even: a lane keeps one half (chosen by its bit
// of the exchange mask), sends the other half to its partner and folds the
// half it receives, so the cost is about Q exchanges instead of 6 Q.  When
// the count is odd the remaining exchanges are a full butterfly.  Afterwards
// lane l holds the wave totals of quantities qb .. qb + N - 1 (N = rs_count),
// and lanes that differ only in the butterfly bits hold identical values.
constexpr int rs_count(int n, int m) { return m == 0 ? n : (n % 2 == 0 ? rs_count(n / 2, m / 2) : n); }
constexpr int rs_full(int n, int m) { return m == 0 ? 0 : (n % 2 == 0 ? rs_full(n / 2, m / 2) : m); }

template <int N, int M>
struct WaveRS {
    static MWU_DEV void run(double *v, int lane, int &qb, Red r, int qoff)
    {
        if constexpr (M == 0) {
            return;
        } else if constexpr (N % 2 == 0) {
            constexpr int H = N / 2;
            const bool up = (lane & M) != 0;
#pragma unroll
            for (int i = 0; i < H; ++i) {
                const double keep = up ? v[i + H] : v[i];
                const double send = up ? v[i] : v[i + H];
                const double recv = __shfl_xor(send, M);
                v[i] = red_op(keep, recv, qb + i + (up ? H : 0) + qoff, r);
            }
            qb += up ? H : 0;
            WaveRS<H, M / 2>::run(v, lane, qb, r, qoff);
        } else {
#pragma unroll
            for (int i = 0; i < N; ++i) v[i] = red_op(v[i], __shfl_xor(v[i], M), qb + i + qoff, r);
            WaveRS<N, M / 2>::run(v, lane, qb, r, qoff);
        }
    }
};

// Combine per-thread values v[0..Q) over the block into out[0..Q) (LDS):
// reduce-scatter inside each wave, then the four wave results in a fixed
// order.  The result does not depend on timing.
template <int Q>
MWU_DEV void block_combine(const double (&v)[Q], Red r, int qoff, double *s_wave, double *out)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    constexpr int N = rs_count(Q, 32);
    constexpr int F = rs_full(Q, 32);
    double w[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) w[q] = v[q];
    int qb = 0;
    WaveRS<Q, 32>::run(w, lane, qb, r, qoff);
    if (F == 0 || (lane & (2 * F - 1)) == 0) {
#pragma unroll
        for (int i = 0; i < N; ++i) s_wave[wv * Q + qb + i] = w[i];
    }
    __syncthreads();
    if (threadIdx.x < Q) {
        const int q = threadIdx.x;
        double a = s_wave[q];
        for (int k = 1; k < BLOCK / 64; ++k) a = red_op(a, s_wave[k * Q + q], q + qoff, r);
        out[q] = a;
    }
    __syncthreads();
}

// Cross-workgroup reduction without fences or atomics.  Every workgroup of a
// pass stores its record (plain stores) in partials[blockIdx.x]; the one-
// workgroup finisher kernel launched right after the pass folds the records
// in block order.  The kernel boundary makes the stores visible, so the hot
// kernels never write back or invalidate the L2 (an agent-scope fence on
// gfx950 does both, and throws away the cached vertex vectors).
MWU_DEV void store_record(const double *s_rec, int Q, double *partials)
{
    if ((int)threadIdx.x < Q) partials[(size_t)blockIdx.x * QMAX + threadIdx.x] = s_rec[threadIdx.x];
}

// Records stored entry-major (entry q of workgroup b at q * G + b, G the
// grid): a finisher then reads each entry of all records with full-width
// coalesced loads, which matters for records of dozens of entries.
MWU_DEV void store_record_qmajor(const double *s_rec, int Q, double *partials)
{
    if ((int)threadIdx.x < Q) partials[(size_t)threadIdx.x * gridDim.x + blockIdx.x] = s_rec[threadIdx.x];
}

// Fold of entry-major records: wave w owns entries w, w + 4, ...; each lane
// folds records lane, lane + 64, ... of its entries (one coalesced row per
// entry, every entry's load in flight at once), and a butterfly over the wave
// finishes each entry.  A lane holds one value per owned entry, so records of
// dozens of entries fold without the register pressure and the block-wide
// exchanges of a fold that keeps every entry in every thread.  out (LDS) is
// complete on return; s_wave is not used.
template <int Q>
MWU_DEV void fold_records_qmajor(const double *partials, int G, Red r, double *s_wave, double *out)
{
    (void)s_wave;
    constexpr int NW = BLOCK / 64;
    constexpr int PER = (Q + NW - 1) / NW;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    double v[PER];
#pragma unroll
    for (int i = 0; i < PER; ++i) v[i] = red_id(wv + i * NW, r);
    for (int b = lane; b < G; b += 64) {
        double t[PER];
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int q = wv + i * NW;
            t[i] = q < Q ? partials[(size_t)q * G + b] : 0.0;
        }
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int q = wv + i * NW;
            if (q < Q) v[i] = red_op(v[i], t[i], q, r);
        }
    }
    // lanes at or above G hold identities: with fewer than 64 records the
    // butterfly stops once it spans them (same values, fewer exchanges)
    int span = 64;
    if (G < 64) { span = 1; while (span < G) span <<= 1; }
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        const int q = wv + i * NW;
        double x = v[i];
#pragma unroll
        for (int m = 32; m > 0; m >>= 1)
            if (m < span) x = red_op(x, __shfl_xor(x, m), q, r);
        if (lane == 0 && q < Q) out[q] = x;
    }
    __syncthreads();
}

// Fold the G records of a pass (finisher kernel, one workgroup): thread t
// folds whole records t, t + BLOCK, ... in order (all Q loads of a record in
// flight at once), then the block combines.  Record entry q is reduced with
// the operation of layout position q + qoff.
template <int Q>
MWU_DEV void fold_records(const double *partials, int G, Red r, int qoff, double *s_wave, double *out)
{
    double v[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) v[q] = red_id(q + qoff, r);
    for (int b = threadIdx.x; b < G; b += BLOCK) {
        const double *rec = partials + (size_t)b * QMAX;
        double t[Q];
#pragma unroll
        for (int q = 0; q < Q; ++q) t[q] = rec[q];
#pragma unroll
        for (int q = 0; q < Q; ++q) v[q] = red_op(v[q], t[q], q + qoff, r);
    }
    block_combine<Q>(v, r, qoff, s_wave, out);
}

// ------------------------------------------------------------ accumulators

template <class T>
struct Pair {
    T g, h;
    MWU_DEV Pair &operator+=(const Pair &o) { g += o.g; h += o.h; return *this; }
};

template <class T> MWU_DEV T acc_zero() { return T{}; }

// Lane exchanges of an accumulator (a scalar or a Pair).
template <class T> MWU_DEV T shfl_up_acc(T v, int d) { return __shfl_up(v, d); }
template <class T> MWU_DEV Pair<T> shfl_up_acc(Pair<T> v, int d)
{
    return Pair<T>{__shfl_up(v.g, d), __shfl_up(v.h, d)};
}
template <class T> MWU_DEV T shfl_xor_acc(T v, int m) { return __shfl_xor(v, m); }
template <class T> MWU_DEV Pair<T> shfl_xor_acc(Pair<T> v, int m)
{
    return Pair<T>{__shfl_xor(v.g, m), __shfl_xor(v.h, m)};
}

// Completion of segments that cross thread boundaries inside a tile.
// Thread t holds the partial tacc of its last segment tseg when that segment
// continues past its items (else tseg = -1), and pend >= 0 when its first
// segment began in an earlier thread and ends in its items.  Threads whose
// tail partials belong to one segment form a contiguous run, so a segmented
// inclusive scan (in-wave shuffles, then a fixed-order carry across the four
// waves) gives every owner the sum of the run right before it.  Returns that
// sum for owners and zero for every other thread.  All threads must call.
template <class Acc>
MWU_DEV Acc seg_carry(int tseg, Acc tacc, int pend)
{
    __shared__ int32_t s_kf[BLOCK / 64], s_kl[BLOCK / 64];
    __shared__ Acc s_vl[BLOCK / 64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    Acc v = tacc;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const Acc o = shfl_up_acc(v, d);
        const int ko = __shfl_up(tseg, d);
        if (lane >= d && tseg >= 0 && ko == tseg) v += o;
    }
    const Acc pv = shfl_up_acc(v, 1);
    const int pk = __shfl_up(tseg, 1);
    const int kf = __shfl(tseg, 0);
    if (lane == 0) s_kf[w] = tseg;
    if (lane == 63) { s_kl[w] = tseg; s_vl[w] = v; }
    __syncthreads();
    // inclusive run value at the last thread of each wave, waves in order
    Acc incl[BLOCK / 64];
    incl[0] = s_vl[0];
#pragma unroll
    for (int i = 1; i < BLOCK / 64; ++i) {
        incl[i] = s_vl[i];
        if (s_kl[i] >= 0 && s_kf[i] == s_kl[i] && s_kl[i - 1] == s_kl[i]) incl[i] += incl[i - 1];
    }
    Acc carry = acc_zero<Acc>();
    if (pend >= 0) {
        if (lane > 0) {
            if (pk == pend) {
                carry = pv;
                if (w > 0 && kf == pend && s_kl[w - 1] == pend) {
                    Acc c = incl[0];
#pragma unroll
                    for (int i = 1; i < BLOCK / 64; ++i)
                        if (i == w - 1) c = incl[i];
                    Acc t = c;
                    t += carry;
                    carry = t;
                }
            }
        } else if (w > 0 && s_kl[w - 1] == pend) {
#pragma unroll
            for (int i = 0; i < BLOCK / 64; ++i)
                if (i == w - 1) carry = incl[i];
        }
    }
    return carry;
}

// ------------------------------------------------------------ segment tiles

MWU_DEV int pad_idx(int k) { return k + (k >> 3); }   // one spare slot per 8: no LDS bank conflicts
constexpr int TILE_LDS = TILE_NZ + TILE_NZ / 8 + 8;

// Sum the nonzeros of every segment of a multi-segment tile and call
// epi(segment, sum) once per segment (empty segments get a zero sum).
// elem(k) returns the term of global nonzero k.  Nonzeros are staged through
// LDS with coalesced loads; each thread then walks ITEMS consecutive terms and
// segments crossing thread boundaries are completed by their owner (the
// thread holding their last term) in a fixed order.
template <class Acc, class ElemF, class EpiF>
MWU_DEV void seg_tile(const Tile &tl, const int32_t *__restrict__ ptr, ElemF &elem, EpiF &epi,
                      Acc *s_acc, int32_t *s_ptr, int32_t *s_tseg, Acc *s_tacc)
{
    const int tid = threadIdx.x;
    const int S = tl.s1 - tl.s0;
    const int base = tl.k0;
    const int N = tl.k1 - tl.k0;
    for (int i = tid; i <= S; i += BLOCK) s_ptr[i] = ptr[tl.s0 + i] - base;
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
        const int k = j * BLOCK + tid;
        if (k < N) s_acc[pad_idx(k)] = elem(base + k);
    }
    __syncthreads();
    const int a = tid * ITEMS;
    const int b = min(a + ITEMS, N);
    int pend = -1, tseg = -1;
    Acc pacc = acc_zero<Acc>(), tacc = acc_zero<Acc>();
    if (a < N) {
        int lo = 0, hi = S;   // s_ptr[lo] <= a < s_ptr[hi]
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (s_ptr[mid] <= a) lo = mid; else hi = mid;
        }
        int s = lo;
        bool started = (s_ptr[s] == a);
        int end = s_ptr[s + 1];
        Acc acc = acc_zero<Acc>();
        for (int k = a; k < b; ++k) {
            while (k >= end) {
                if (s_ptr[s] < end) {
                    if (started) epi(tl.s0 + s, acc);
                    else { pend = s; pacc = acc; }
                }
                ++s;
                started = true;
                acc = acc_zero<Acc>();
                end = s_ptr[s + 1];
            }
            acc += s_acc[pad_idx(k)];
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
    for (int s = tid; s < S; s += BLOCK)
        if (s_ptr[s] == s_ptr[s + 1]) epi(tl.s0 + s, acc_zero<Acc>());
    __syncthreads();
}

// Chunk tile of a long segment: reduce the chunk and store its partial sum;
// a later kernel completes the segment.  Returns the chunk's sum in thread 0
// (zero in the other threads).
template <class Acc, class ElemF>
MWU_DEV Acc chunk_tile(const Tile &tl, ElemF &elem, Acc *s_tacc, Acc *lpart, const int32_t *lfirst)
{
    const int tid = threadIdx.x;
    Acc acc = acc_zero<Acc>();
    for (int k = tl.k0 + tid; k < tl.k1; k += BLOCK) acc += elem(k);
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) acc += shfl_xor_acc(acc, m);
    if ((tid & 63) == 0) s_tacc[tid >> 6] = acc;
    __syncthreads();
    Acc tot = acc_zero<Acc>();
    if (tid == 0) {
        tot = s_tacc[0];
        for (int w = 1; w < BLOCK / 64; ++w) tot += s_tacc[w];
        lpart[lfirst[tl.lid] + tl.cidx] = tot;
    }
    __syncthreads();
    return tot;
}

// Sum of the chunk partials of long segment lid, in chunk order.
template <class Acc>
MWU_DEV Acc long_sum(int lid, const Acc *lpart, const int32_t *lfirst, const int32_t *lcount)
{
    Acc tot = acc_zero<Acc>();
    const int f = lfirst[lid], c = lcount[lid];
    for (int i = 0; i < c; ++i) tot += lpart[f + i];
    return tot;
}

// Candidates carried by a pass of each kind (the list kind checks k < nc).
template <int KIND>
constexpr int pass_cands()
{
    return KIND == SK_EXP ? KE : KIND == SK_GRID ? KG : KIND == SK_LIST ? KL : KC;
}
// Leading candidates whose minima min(z + a dz) the replay can read: those of
// the exponential phase (the bisection never reads them).
template <int KIND>
constexpr int pass_minima()
{
    return KIND == SK_EXP || KIND == SK_COMBO ? KE : KIND == SK_LIST ? KL : 0;
}

// Covering terms s1[k] += u expm1(-b_k), s2[k] += u e^{-b_k} for b_k = b0
// 2^k, k < N: expm1(2x) = expm1(x)(expm1(x) + 2) and e^{-2x} by squaring
// (float re-seeds the squared term from exp every 4 candidates).
template <class T, int N>
MWU_DEV void cov_doubling(double b0d, T u, T *s1, T *s2)
{
    const T b0 = (T)b0d;
    T m = expm1_t(-b0);
    T t = exp_arg(-b0d, T(0));
#pragma unroll
    for (int k = 0; k < N; ++k) {
        s1[k] += u * m;
        s2[k] += u * t;
        m = m * (m + T(2));
        if (sizeof(T) == 4 && (k & 3) == 3 && k + 1 < N)
            t = exp_arg(-b0d * (double)(1 << (k + 1)), T(0));
        else
            t = t * t;
    }
}

// The same for b_k = b0 + k bd: expm1(x + y) = expm1(x) + expm1(y) +
// expm1(x) expm1(y) and e^{-(x+y)} = e^{-x} e^{-y}.
template <class T, int N>
MWU_DEV void cov_adding(double b0d, double bdd, T u, T *s1, T *s2)
{
    T m = expm1_t(-(T)b0d);
    T t = exp_arg(-b0d, T(0));
    const T mr = expm1_t(-(T)bdd);
    const T tr = exp_arg(-bdd, T(0));
#pragma unroll
    for (int k = 0; k < N; ++k) {
        s1[k] += u * m;
        s2[k] += u * t;
        m = m + mr + m * mr;
        t = t * tr;
    }
}

// Covering-row terms of one search pass (KIND fixed per launch, no
// data-dependent branches): acc[k] += u expm1(-b_k), acc[KC+k] += u
// e^{-b_k}, zmn[k] = min(zmn[k], z + a_k dz) for the leading pass_minima
// candidates, with b_k = eta a_k dz.  On the exponential grid a_k = a0 2^k,
// on the bisection grid a_k = a0 + k gdel, on the combined pass both (the
// bisection part from ga0).  A zero weight or a zero dz needs no special
// case: the terms come out as 0 and u.
template <class T, int KIND, class Z = T>
MWU_DEV void cov_terms(int nc, const double *cand, double a0, double ga0, double gdel, double eta, T u, Z z,
                       T dz, T *acc, Z *zmn, bool deriv = false)
{
    if constexpr (KIND == SK_LIST) {   // arbitrary candidates, direct evaluation
#pragma unroll
        for (int k = 0; k < KL; ++k)
            if (k < nc) {
                const double a = cand[k];
                zmn[k] = fmin(zmn[k], z + (Z)a * (Z)dz);
                const T b = (T)(eta * a * (double)dz);
                acc[k] += u * expm1_t(-b);
                acc[KC + k] += u * exp_t(-b);
            }
        // Newton pass: the sum of Phi' at cand[0], u dz e^{-b_0} (slot KN, past its values)
        if (deriv) acc[KN] += u * dz * exp_t(-(T)(eta * cand[0] * (double)dz));
    } else {
        if constexpr (pass_minima<KIND>() > 0) {
            Z ak = (Z)a0;
#pragma unroll
            for (int k = 0; k < pass_minima<KIND>(); ++k) {
                zmn[k] = fmin(zmn[k], z + ak * (Z)dz);
                ak = ak + ak;
            }
        }
        const double dzd = (double)dz;
        if constexpr (KIND == SK_EXP || KIND == SK_COMBO) cov_doubling<T, KE>(eta * a0 * dzd, u, acc, acc + KC);
        if constexpr (KIND == SK_GRID) cov_adding<T, KG>(eta * a0 * dzd, eta * gdel * dzd, u, acc, acc + KC);
        if constexpr (KIND == SK_COMBO)
            cov_adding<T, KG>(eta * ga0 * dzd, eta * gdel * dzd, u, acc + KE, acc + KC + KE);
    }
}

// Candidates of a pass whose packing exponent eta a dymax passes psi_lim
// (bit k for candidate k): their packing sums are formed max-shifted (see
// pack_terms) when psi_shift is on (the chosen form; FP64 refines such steps
// in two exact passes instead).  The replay makes the same test on the same
// doubles.
MWU_DEV uint32_t shifted_mask(const Ctl *c)
{
    uint32_t m = 0;
    if (!c->psi_shift) return m;
    for (int k = 0; k < c->ncand && k < 32; ++k)
        if (c->eta * c->cand[k] * c->dymax > c->psi_lim) m |= 1u << k;
    return m;
}

// Packing-row terms of one search pass: s1[k] += w expm1(eta a_k dy) with
// the candidates of cov_terms, or, for the candidates in shmask, the
// max-shifted s1[k] += w e^{eta a_k (dy - dymax)}, which cannot overflow
// (dy <= dymax); Psi of such a candidate is (eta a_k dymax + log(s1 / sum w))
// / eta.  The shifted terms follow the same recurrences (squaring on the
// exponential grid, float re-seeded every 4 steps; products on the bisection
// grid).
//
// With SH64 the shifted terms are formed in double from the row's FP64 state
// instead: lw = eta (y - L) for the L the stored weight w = e^{lw} was formed
// with, and dy64 the FP64 direction.  A float w underflows once lw < -103,
// and the rows that set dymax can be such rows; a shifted sum of float terms
// is then 0 at large steps even though its exact value is far inside the
// double range.  The unshifted terms still use w and dy.
template <class T, int KIND, bool SH64 = false>
MWU_DEV void pack_terms(int nc, const double *cand, double a0, double ga0, double gdel, double eta, T w, T dy,
                        double dymax, uint32_t shmask, double *s1, bool deriv = false, double lw = 0.0,
                        double dy64 = 0.0)
{
    const double dyd = (double)dy;
    const double dsh = (SH64 ? dy64 : dyd) - dymax;   // <= 0
    const double w64 = SH64 && shmask ? exp(lw) : 0.0;
    auto doubling = [&](double b0, double c0, double *o) {
        T m = expm1_t((T)b0);
        if (!shmask) {
#pragma unroll
            for (int k = 0; k < KE; ++k) {
                o[k] += (double)(w * m);
                m = m * (m + T(2));                  // expm1(2x) = expm1(x)(expm1(x)+2)
            }
            return;
        }
        if constexpr (SH64) {
            double t = exp(c0);
#pragma unroll
            for (int k = 0; k < KE; ++k) {
                o[k] += ((shmask >> k) & 1u) ? w64 * t : (double)(w * m);
                m = m * (m + T(2));
                t = t * t;
            }
            return;
        }
        T t = exp_arg(c0, T(0));
#pragma unroll
        for (int k = 0; k < KE; ++k) {
            o[k] += (double)(w * (((shmask >> k) & 1u) ? t : m));
            m = m * (m + T(2));
            if (sizeof(T) == 4 && (k & 3) == 3 && k + 1 < KE) t = exp_arg(c0 * (double)(1 << (k + 1)), T(0));
            else t = t * t;
        }
    };
    auto adding = [&](double b0, double bd, double c0, double cd, int k0, double *o) {
        T m = expm1_t((T)b0);
        const T mr = expm1_t((T)bd);
        if (!shmask) {
#pragma unroll
            for (int k = 0; k < KG; ++k) {
                o[k] += (double)(w * m);
                m = m + mr + m * mr;                 // expm1(x+y) from expm1(x), expm1(y)
            }
            return;
        }
        if constexpr (SH64) {
            double t = exp(c0);
            const double tr = exp(cd);
#pragma unroll
            for (int k = 0; k < KG; ++k) {
                o[k] += ((shmask >> (k0 + k)) & 1u) ? w64 * t : (double)(w * m);
                m = m + mr + m * mr;
                t = t * tr;
            }
            return;
        }
        T t = exp_arg(c0, T(0));
        const T tr = exp_arg(cd, T(0));
#pragma unroll
        for (int k = 0; k < KG; ++k) {
            o[k] += (double)(w * (((shmask >> (k0 + k)) & 1u) ? t : m));
            m = m + mr + m * mr;
            t = t * tr;
        }
    };
    if constexpr (KIND == SK_LIST) {
#pragma unroll
        for (int k = 0; k < KL; ++k)
            if (k < nc) {
                if (SH64 && ((shmask >> k) & 1u)) {
                    s1[k] += w64 * exp(eta * cand[k] * dsh);
                    continue;
                }
                const T v = ((shmask >> k) & 1u) ? exp_arg(eta * cand[k] * dsh, T(0))
                                                 : expm1_t((T)(eta * cand[k] * dyd));
                s1[k] += (double)(w * v);
            }
        // Newton pass: the sum of Psi' at cand[0], w dy e^{eta a_0 dy}, max-shifted as
        // cand[0]'s own sum is (slot KN, past its values)
        if (deriv) {
            if (SH64 && (shmask & 1u)) {
                s1[KN] += w64 * dy64 * exp(eta * cand[0] * dsh);
            } else {
                const T v0 = (shmask & 1u) ? exp_arg(eta * cand[0] * dsh, T(0)) : exp_arg(eta * cand[0] * dyd, T(0));
                s1[KN] += (double)(w * dy * v0);
            }
        }
    } else {
        if constexpr (KIND == SK_EXP || KIND == SK_COMBO) doubling(eta * a0 * dyd, eta * a0 * dsh, s1);
        if constexpr (KIND == SK_GRID) adding(eta * a0 * dyd, eta * gdel * dyd, eta * a0 * dsh, eta * gdel * dsh, 0, s1);
        if constexpr (KIND == SK_COMBO)
            adding(eta * ga0 * dyd, eta * gdel * dyd, eta * ga0 * dsh, eta * gdel * dsh, KE, s1 + KE);
    }
}

// Per-thread accumulators of the covering side of a search pass.  The
// per-thread partial sums (same-sign terms, a few dozen per thread) are kept
// in the storage type; block and grid totals are double.
template <class T, class Z = T>
struct CovAcc {
    T acc[2 * KC];
    Z zmn[KC];
    // Minima past the first nmin stay at -inf: the replay never reads them,
    // and -inf can never pass for an early return.
    MWU_DEV void init(int nmin)
    {
#pragma unroll
        for (int k = 0; k < 2 * KC; ++k) acc[k] = T(0);
#pragma unroll
        for (int k = 0; k < KC; ++k) zmn[k] = k < nmin ? Z(INFINITY) : Z(-INFINITY);
    }
    // Compact block record of a pass of kind KIND, [s1C(N) | s2C(N) |
    // zmin(M)] with N = pass_cands and M = pass_minima: the finisher folds
    // only what the pass produced.
    template <int KIND>
    MWU_DEV void combine_compact(double *s_wave, double *out)
    {
        constexpr int N = pass_cands<KIND>(), M = pass_minima<KIND>();
        double ad[2 * N];
#pragma unroll
        for (int k = 0; k < N; ++k) {
            ad[k] = (double)acc[k];
            ad[N + k] = (double)acc[KC + k];
        }
        const Red rs{2 * N, 0, 0};
        block_combine<2 * N>(ad, rs, 0, s_wave, out);
        if constexpr (M > 0) {
            double zd[M];
#pragma unroll
            for (int k = 0; k < M; ++k) zd[k] = (double)zmn[k];
            const Red rm{0, M, 0};
            block_combine<M>(zd, rm, 0, s_wave, out + 2 * N);
        }
    }
    // block-combine into out[0..3KC): [s1C | s2C | zmin]
    MWU_DEV void combine(double *s_wave, double *out)
    {
        double ad[2 * KC];
#pragma unroll
        for (int k = 0; k < 2 * KC; ++k) ad[k] = (double)acc[k];
        const Red rs{2 * KC, 0, 0};
        block_combine<2 * KC>(ad, rs, 0, s_wave, out);
        double zd[KC];
#pragma unroll
        for (int k = 0; k < KC; ++k) zd[k] = (double)zmn[k];
        const Red rm{0, KC, 0};
        block_combine<KC>(zd, rm, 0, s_wave, out + 2 * KC);
    }
};

// Doubles in a compact covering record of a pass of kind KIND.
template <int KIND>
constexpr int cov_record_q()
{
    return 2 * pass_cands<KIND>() + pass_minima<KIND>();
}

// Finisher side of the compact records (stored entry-major): fold them and
// spread the totals to
// out = [s1C(KC) | s2C(KC) | zmin(KC)] (sums the pass did not form are 0,
// minima it did not form -inf, which no early return can take).  All threads
// call; out is complete on return.
template <int KIND>
MWU_DEV void fold_cov_compact(const double *part, int G, double *s_wave, double *s_tmp, double *out)
{
    constexpr int N = pass_cands<KIND>(), M = pass_minima<KIND>();
    const Red r{2 * N, M, 0};
    fold_records_qmajor<cov_record_q<KIND>()>(part, G, r, s_wave, s_tmp);
    for (int k = threadIdx.x; k < KC; k += blockDim.x) {
        out[k] = k < N ? s_tmp[k] : 0.0;
        out[KC + k] = k < N ? s_tmp[N + k] : 0.0;
        out[2 * KC + k] = k < M ? s_tmp[2 * N + k] : -INFINITY;
    }
    __syncthreads();
}

// ------------------------------------------------------ step-search replay
//
// The search kernels evaluate up to KC candidate steps per pass.  After a
// pass the last block replays Algorithm 3 sequentially over the evaluated
// values; when the sequential algorithm needs a value that the pass did not
// produce, the next pass is set up and the replay resumes from its state.

struct Eval { double psi, phi, zmin; int ok, pok; };   // pok: the packing side is resolved

// eta (z - L) beyond which a covering row is left out of the sparse passes.
// Double: exp(-746) is exactly zero (below half the smallest subnormal), so
// the sums are those of the full pass.  Float: the weights left out are below
// e^-40 of the weights at the shift, whose sum is about 1, so they move the
// sums by less than m e^-40 (7e-11 for m = 1.6e7), far below the rounding of
// the float terms themselves.  Either way the row holding min z stays in,
// since eta (min z - L) <= ln m.
template <class T>
constexpr double skip_exponent()
{
    return sizeof(T) == 4 ? 40.0 : 746.0;
}

// A covering row the iteration leaves out when satisfied rows are dropped
// (Algorithms 1 and 2 keep only the rows with c_i^T x < 1): its weight is 0,
// so it adds nothing to the smoothed minimum, h, Phi or their refinements.
// z only grows, so a row once met stays out.  The minimum of z is still
// taken over every row: a met row is at least 1, so it changes neither the
// stop test nor the early return.
MWU_DEV bool row_met(const Ctl *c, double z) { return c->drop && z >= 1.0; }

// The active lists of the sparse passes hold every covering row that is not
// negligible while the weight shift Lw has moved by at most act_mu / eta
// since they were built: z only grows (x and d are nonnegative), so a row
// left out then still has eta (z - Lw) above the skip exponent.
// The transpose pass may use them in evaluation mode too (its sums and
// minimum are exact either way); the search never does there, since its
// minima over the active rows alone are only bounds (act_valid).
MWU_DEV bool act_rows_valid(const Ctl *c, double Lw)
{
    return c->act_on && c->eta * (Lw - c->act_L) <= c->act_mu;
}
MWU_DEV bool act_valid(const Ctl *c, double Lw)
{
    return !c->eval_mode && act_rows_valid(c, Lw);
}

// A finisher's state update is one thread walking long dependent chains of
// control-block fields (the replay above all); from device memory every link
// costs an L2 round trip.  The workgroup stages the block in LDS with one
// load per thread, thread 0 runs f on the copy, and the workgroup writes the
// whole block back.  All threads of the workgroup must call.
// A finisher may stage the block before anything else: its phase test then
// reads the staged copy, so the block is fetched in the same round trip as
// the test and not again after the fold.  All threads call ctl_stage (which
// returns the staged block) and, when the finisher changed it,
// ctl_write_back.
constexpr int CTL_WORDS = sizeof(Ctl) / 8;
MWU_DEV Ctl *ctl_stage(const Ctl *g, uint64_t *s_ctl)
{
    static_assert(sizeof(Ctl) % 8 == 0, "control block is copied in 8-byte words");
    const uint64_t *src = reinterpret_cast<const uint64_t *>(g);
    for (int i = threadIdx.x; i < CTL_WORDS; i += blockDim.x) s_ctl[i] = src[i];
    __syncthreads();
    return reinterpret_cast<Ctl *>(s_ctl);
}
MWU_DEV void ctl_write_back(Ctl *g, const uint64_t *s_ctl)
{
    __syncthreads();
    uint64_t *dst = reinterpret_cast<uint64_t *>(g);
    for (int i = threadIdx.x; i < CTL_WORDS; i += blockDim.x) dst[i] = s_ctl[i];
}

template <class F>
MWU_DEV void on_ctl(Ctl *g, F &&f);

// The same with a step all threads run on the staged copy first (it
// synchronizes on its own where it needs to).
template <class P, class F>
MWU_DEV void on_ctl_all(Ctl *g, P &&pre, F &&f)
{
    static_assert(sizeof(Ctl) % 8 == 0, "control block is copied in 8-byte words");
    constexpr int W = sizeof(Ctl) / 8;
    __shared__ uint64_t s_ctl[W];
    const uint64_t *src = reinterpret_cast<const uint64_t *>(g);
    for (int i = threadIdx.x; i < W; i += blockDim.x) s_ctl[i] = src[i];
    __syncthreads();
    Ctl *c = reinterpret_cast<Ctl *>(s_ctl);
    pre(c);
    __syncthreads();
    if (threadIdx.x == 0) f(c);
    __syncthreads();
    uint64_t *dst = reinterpret_cast<uint64_t *>(g);
    for (int i = threadIdx.x; i < W; i += blockDim.x) dst[i] = s_ctl[i];
}

template <class F>
MWU_DEV void on_ctl(Ctl *g, F &&f)
{
    static_assert(sizeof(Ctl) % 8 == 0, "control block is copied in 8-byte words");
    constexpr int W = sizeof(Ctl) / 8;
    __shared__ uint64_t s_ctl[W];
    const uint64_t *src = reinterpret_cast<const uint64_t *>(g);
    for (int i = threadIdx.x; i < W; i += blockDim.x) s_ctl[i] = src[i];
    __syncthreads();
    if (threadIdx.x == 0) f(reinterpret_cast<Ctl *>(s_ctl));
    __syncthreads();
    uint64_t *dst = reinterpret_cast<uint64_t *>(g);
    for (int i = threadIdx.x; i < W; i += blockDim.x) dst[i] = s_ctl[i];
}

MWU_DEV Eval eval_cand(const Ctl *c, int k, double alpha)
{
    Eval e;
    e.ok = 1;
    e.pok = 1;
    if (c->onesP) {
        e.psi = alpha * c->dy1;
    } else {
        const double s1 = c->rS1P[k] * c->invSw;
        const double B = c->eta * alpha * c->dymax;
        if (B > c->psi_lim && !c->psi_shift) { e.ok = 0; e.psi = 0; }   // full-list refinement
        else if (B > c->psi_lim) {   // the pass formed the max-shifted sum (shifted_mask)
            if (s1 > 0.0 && isfinite(s1)) e.psi = (B + log(s1)) / c->eta;
            else { e.ok = 0; e.psi = 0; }
        } else if (!isfinite(s1)) { e.ok = 0; e.psi = 0; }
        else e.psi = log1p(s1) / c->eta;
        e.pok = e.ok;
    }
    if (c->onesC) {
        e.phi = alpha * c->dz1;
        e.zmin = c->z1 + alpha * c->dz1;
    } else {
        const double s1 = c->rS1C[k] * c->invSu;
        e.zmin = c->rZmin[k];
        // a pass over the active list gives the minima of the active rows; a
        // left-out row can only decide min z' >= 1 when it started below 1,
        // and then the full-list refinement settles it
        if (c->pass_sparse && e.zmin >= 1.0 && c->act_zfloor < 1.0) e.ok = 0;
        if (1.0 + s1 >= 0.5) {
            e.phi = -log1p(s1) / c->eta;
        } else {
            const double s2 = c->rS2C[k] * c->invSu;
            if (s2 >= c->s2_min && isfinite(s2)) e.phi = -log(s2) / c->eta;
            else { e.ok = 0; e.phi = 0; }
        }
    }
    return e;
}

// Timing mode: a pass can be replayed with the state frozen.
MWU_DEV bool held(Ctl *c)
{
    if (!c->hold) return false;
    c->phase = c->hold;
    return true;
}

MWU_DEV void setup_exp(Ctl *c, double a0)
{
    c->skind = SK_EXP;
    c->ncand = KE;
    double a = a0;
    for (int k = 0; k < KE; ++k) { c->cand[k] = a; a *= 2.0; }
    c->ga0 = a0;
    c->gdelta = 0.0;
}

// Candidates of the bisection of [lb, ub] to depth 4, computed with exactly
// the midpoint arithmetic of the sequential search, in ascending order.
MWU_DEV void grid_values(double lb, double ub, double *v)
{
    // in-order positions of a complete binary tree of depth 4
    double lo1 = lb, hi1 = ub;
    double m1 = (lo1 + hi1) / 2.0;
    double m2a = (lo1 + m1) / 2.0, m2b = (m1 + hi1) / 2.0;
    double m3a = (lo1 + m2a) / 2.0, m3b = (m2a + m1) / 2.0, m3c = (m1 + m2b) / 2.0,
           m3d = (m2b + hi1) / 2.0;
    v[0] = (lo1 + m3a) / 2.0;  v[1] = m3a; v[2] = (m3a + m2a) / 2.0; v[3] = m2a;
    v[4] = (m2a + m3b) / 2.0;  v[5] = m3b; v[6] = (m3b + m1) / 2.0;  v[7] = m1;
    v[8] = (m1 + m3c) / 2.0;   v[9] = m3c; v[10] = (m3c + m2b) / 2.0; v[11] = m2b;
    v[12] = (m2b + m3d) / 2.0; v[13] = m3d; v[14] = (m3d + hi1) / 2.0;
}

MWU_DEV void setup_grid(Ctl *c, double lb, double ub)
{
    double v[KG];
    grid_values(lb, ub, v);
    c->skind = SK_GRID;
    c->ncand = KG;
    for (int k = 0; k < KG; ++k) c->cand[k] = v[k];
    c->ga0 = v[0];
    c->gdelta = (ub - lb) / 16.0;
}

// First pass of an iteration: the exponential grid from 1 and, when the
// previous step lay in an octave [2^j, 2^(j+1)) whose upper end the grid
// reaches, the bisection tree of that octave in the same pass.  Steps change
// slowly from one iteration to the next, so the sequential search usually
// finds every value it asks for in this one pass; otherwise the replay sets
// up the pass it needs, as after a plain exponential pass.
MWU_DEV void setup_first(Ctl *c)
{
    setup_exp(c, 1.0);
    const double la = c->last_alpha;
    if (!(la >= 1.0 && la < (double)(1 << (KE - 1)))) return;
    int e = 0;
    (void)frexp(la, &e);                       // la = f 2^e, f in [0.5, 1)
    const double lb = ldexp(1.0, e - 1), ub = 2.0 * lb;
    double v[KG];
    grid_values(lb, ub, v);
    for (int k = 0; k < KG; ++k) c->cand[KE + k] = v[k];
    c->skind = SK_COMBO;
    c->ncand = KC;
    c->ga0 = v[0];
    c->gdelta = (ub - lb) / 16.0;
}

// First pass of a warm-started search (step rule MWU_STEP_BIN_WARM, from
// the previous step la > 1): the ladder la/8 .. 16 la, which holds the
// first halvings and doublings, and the bisection tree of [la, 2 la), the
// bracket when the step stays in its octave.
MWU_DEV void setup_first_warm(Ctl *c, double la)
{
    setup_exp(c, la / 8.0);
    double v[KG];
    grid_values(la, 2.0 * la, v);
    for (int k = 0; k < KG; ++k) c->cand[KE + k] = v[k];
    c->skind = SK_COMBO;
    c->ncand = KC;
    c->ga0 = v[0];
    c->gdelta = la / 16.0;
}

// Values per Newton pass: the iterate and the first back-off values below it.
constexpr int NB = 4;
// Most Newton evaluations of one step search before the back-off.
constexpr int NEWTON_STEPS = 8;

// A list pass over a and the back-off values after it, a (1-eps), a
// (1-eps)^2, ..., each the previous one times (1 - eps) with exactly the
// arithmetic of the sequential back-off, the first one at most 1 clamped to
// 1 and last; at most nmax values.  A Newton pass (kind SK_NEWTON) also forms
// the derivative sums at a.
MWU_DEV void setup_ladder(Ctl *c, double a, int kind, int nmax)
{
    int n = 0;
    double b = a;
    c->cand[n++] = b;
    while (n < nmax && b > 1.0) {
        b *= 1.0 - c->eps;
        if (b < 1.0) b = 1.0;
        c->cand[n++] = b;
    }
    c->skind = kind;
    c->ncand = n;
    c->ga0 = a;
    c->gdelta = 0.0;
}

// The two-pass refinement of step a: pass 1 forms the shifts (max eta y',
// min z'), pass 2 the shifted sums.  When a is a candidate of the pass just
// made, that pass resolved its packing side and formed its min z' (the
// exponential-grid and list passes do, over the full list), only the
// covering sum fell out of range: pass 2 then starts at once, shifted by
// eta (L_P + Psi(a)) (the exact log of the packing sum at a, so that sum is
// about 1) and by that minimum.
MWU_DEV void setup_refine(Ctl *c, double a)
{
    c->skind = SK_REFINE;
    c->ref_alpha = a;
    c->ref_valid = 0;
    c->ref_short = 0;
    if (c->pass_sparse || c->onesC) return;
    int k = -1;
    for (int j = 0; j < c->ncand && j < KC; ++j)
        if (c->cand[j] == a) { k = j; break; }
    if (k < 0 || !isfinite(c->rZmin[k])) return;
    const Eval e = eval_cand(c, k, a);
    if (!e.pok) return;
    c->rfZmin = c->rZmin[k];
    c->rfPm = c->onesP ? 0.0 : c->eta * (c->LP + e.psi);
    c->ref_valid = -1;
    c->ref_short = 1;
}

MWU_DEV void accept_step(Ctl *c, double a, double psi, double phi)
{
    if (c->trace && c->iter < c->trace_cap) c->trace[c->iter] = a;
    c->alpha = a;
    c->LP += psi;
    c->LC += phi;
    c->iter += 1;
    c->last_alpha = a;
    c->amode = AM_EXP;
    c->have_cur = 0;
    c->ref_valid = 0;
    // the step is pending: the next row pass applies it (the probe API may
    // stop here after a given number of iterations and resume later)
    c->phase = (c->iter_stop > 0 && c->iter >= c->iter_stop) ? PH_IDLE : PH_ROW;
}

MWU_DEV void stop_infeasible(Ctl *c)
{
    c->status = ST_INFEASIBLE;
    c->phase = PH_DONE;
}

// The candidates of the pass being replayed, copied once into registers of
// the replaying thread: the control block sits in shared memory, and a search
// over it would be a chain of dependent loads, one per candidate, at every
// lookup.  The candidates do not change during a replay (a new pass ends it).
struct CandRegs {
    double v[KC];
    int n;
    MWU_DEV explicit CandRegs(const Ctl *c) : n(c->ncand)
    {
#pragma unroll
        for (int k = 0; k < KC; ++k) v[k] = c->cand[k];
    }
    // index of the first candidate equal to a, or -1
    MWU_DEV int find(double a) const
    {
        int hit = -1;
#pragma unroll
        for (int k = KC - 1; k >= 0; --k)
            if (k < n && v[k] == a) hit = k;
        return hit;
    }
};

// Find the evaluation of step a: a refined value, or a grid candidate.
// Returns 0 = found (e filled), 1 = not in the grid, 2 = needs refinement.
MWU_DEV int lookup(const Ctl *c, const CandRegs &cr, double a, Eval *e)
{
    if (c->ref_valid == 1 && c->ref_alpha == a) {
        e->psi = c->ref_psi; e->phi = c->ref_phi; e->zmin = c->ref_zmin; e->ok = 1;
        return 0;
    }
    const int k = cr.find(a);
    if (k < 0) return 1;
    if (c->ev_cached) {
        e->psi = c->ev_psi[k]; e->phi = c->ev_phi[k]; e->zmin = c->ev_zmin[k]; e->ok = c->ev_ok[k];
    } else {
        *e = eval_cand(c, k, a);
    }
    return e->ok ? 0 : 2;
}

// Psi'(a) and Phi'(a) at the first value a of a Newton pass (Section 4.2):
// the averages of P d and C d under the weights of the moved point, each the
// pass's slot-KN sum over a's own sum (sum w e^{eta a dy} = sum w + the
// expm1 sum, or the max-shifted sum when a's packing sum took that form;
// sum u e^{-eta a dz} on the covering side).  False when a denominator is
// not usable: the refinement then forms both with exact shifts.
MWU_DEV bool newton_derivs(const Ctl *c, double *dpsi, double *dphi)
{
    if (c->onesP) {
        *dpsi = c->dy1;
    } else {
        const bool sh = c->psi_shift && c->eta * c->cand[0] * c->dymax > c->psi_lim;
        const double den = sh ? c->rS1P[0] : 1.0 / c->invSw + c->rS1P[0];
        if (!(den > 0.0)) return false;
        *dpsi = c->rS1P[KN] / den;
    }
    if (c->onesC) {
        *dphi = c->dz1;
    } else {
        const double den = c->rS2C[0];
        if (!(den > 0.0)) return false;
        *dphi = c->rS1C[KN] / den;
    }
    return isfinite(*dpsi) && isfinite(*dphi);
}

// The evaluation of a Newton iterate a with its derivatives: from a
// refinement at a, or as the first value of a Newton pass.  Returns 0 =
// found, 1 = no pass has it, 2 = needs refinement.
MWU_DEV int newton_lookup(const Ctl *c, double a, Eval *e, double *dpsi, double *dphi)
{
    if (c->ref_valid == 1 && c->ref_alpha == a) {
        e->psi = c->ref_psi; e->phi = c->ref_phi; e->zmin = c->ref_zmin; e->ok = 1;
        *dpsi = c->ref_dpsi; *dphi = c->ref_dphi;
        return 0;
    }
    if (c->skind != SK_NEWTON || c->cand[0] != a) return 1;
    if (c->ev_cached) {
        e->psi = c->ev_psi[0]; e->phi = c->ev_phi[0]; e->zmin = c->ev_zmin[0]; e->ok = c->ev_ok[0];
    } else {
        *e = eval_cand(c, 0, a);
    }
    if (!e->ok) return 2;
    return newton_derivs(c, dpsi, dphi) ? 0 : 2;
}

// Store the reduced record of a grid or list pass and evaluate all its
// candidates at once, candidate k on lane k, into the ev_ arrays: the
// sequential replay then reads them instead of forming each logarithm on one
// lane.  All threads of the finisher call, with c staged in LDS; follow with
// finish_search(c, rec, true) on one thread.
MWU_DEV void pre_eval_search(Ctl *c, const double *rec)
{
    const int k = threadIdx.x;
    if (k < KC) {
        c->rS1P[k] = rec[k];
        c->rS1C[k] = rec[KC + k];
        c->rS2C[k] = rec[2 * KC + k];
        c->rZmin[k] = rec[3 * KC + k];
    }
    __syncthreads();
    if (k < c->ncand) {
        const Eval e = eval_cand(c, k, c->cand[k]);
        c->ev_psi[k] = e.psi; c->ev_phi[k] = e.phi; c->ev_zmin[k] = e.zmin; c->ev_ok[k] = e.ok;
    }
    if (k == 0) c->ev_cached = 1;
    __syncthreads();
}

constexpr double ALPHA_CAP = 1125899906842624.0;   // 2^50

MWU_DEV void replay(Ctl *c)
{
    const CandRegs cr(c);
    for (int guard = 0; guard < 256; ++guard) {
        if (c->amode == AM_FORCED) {
            const double a = c->cur_alpha;
            Eval e;
            int r = lookup(c, cr, a, &e);
            if (r == 1) { c->skind = SK_LIST; c->ncand = 1; c->cand[0] = a; return; }
            if (r == 2) { setup_refine(c, a); return; }
            c->evaluations += 1;
            if (a < 1.0) { stop_infeasible(c); return; }
            accept_step(c, a, e.psi, e.phi);
            return;
        }
        if (c->amode == AM_EXP) {
            const double a = c->exp_next;
            Eval e;
            int r = lookup(c, cr, a, &e);
            if (r == 1) { setup_exp(c, a); return; }
            if (r == 2) { setup_refine(c, a); return; }
            c->evaluations += 1;
            if (!(e.phi >= e.psi)) {
                if (!c->have_cur) {
                    // T fails at the start: at 1 the probe ends (alpha < 1);
                    // at a warm start above 1 the search halves downward
                    if (!(a > 1.0)) { stop_infeasible(c); return; }
                    c->ub = a;
                    c->amode = AM_DOWN;
                    continue;
                }
                c->lb = c->cur_alpha; c->ub = a;
                c->lb_psi = c->cur_psi; c->lb_phi = c->cur_phi;
                c->amode = AM_BIS;
                continue;
            }
            c->have_cur = 1;
            c->cur_alpha = a; c->cur_psi = e.psi; c->cur_phi = e.phi;
            if (e.zmin >= 1.0 || a >= ALPHA_CAP) { accept_step(c, a, e.psi, e.phi); return; }
            c->exp_next = 2.0 * a;
            continue;
        }
        if (c->amode == AM_DOWN) {   // halving from a failing warm start (never below 1)
            const double b = fmax(c->ub / 2.0, 1.0);
            Eval e;
            int r = lookup(c, cr, b, &e);
            if (r == 1) { setup_exp(c, b / (double)(1 << (KE - 1))); return; }   // the next KE halvings
            if (r == 2) { setup_refine(c, b); return; }
            c->evaluations += 1;
            if (e.phi >= e.psi) {
                if (e.zmin >= 1.0) { accept_step(c, b, e.psi, e.phi); return; }
                c->lb = b; c->lb_psi = e.psi; c->lb_phi = e.phi;   // ub: the last failing value
                c->amode = AM_BIS;
                continue;
            }
            if (!(b > 1.0)) { stop_infeasible(c); return; }
            c->ub = b;
            continue;
        }
        if (c->amode == AM_NEWTON) {
            // Newton's method on g = Phi/Psi - 1 inside the bracket (lb, ub) of
            // the values tested (Section 4.2, reading R20): one evaluation
            // per iterate, which leads its own pass
            const double a = c->cur_alpha;
            Eval e;
            double dps = 0.0, dph = 0.0;
            const int r = newton_lookup(c, a, &e, &dps, &dph);
            if (r == 1) { setup_ladder(c, a, SK_NEWTON, NB); return; }
            if (r == 2) { setup_refine(c, a); return; }
            c->evaluations += 1;
            c->nw_evals += 1;
            const bool pass = e.phi >= e.psi;
            if (pass) {
                if (e.zmin >= 1.0 || a >= ALPHA_CAP) { accept_step(c, a, e.psi, e.phi); return; }
                c->lb = a; c->lb_psi = e.psi; c->lb_phi = e.phi;
            } else {
                if (!(a > 1.0)) { stop_infeasible(c); return; }
                c->ub = a;
            }
            if (c->ub <= (1.0 + c->eps) * c->lb) { accept_step(c, c->lb, c->lb_psi, c->lb_phi); return; }
            bool stop = c->nw_evals >= NEWTON_STEPS;
            double next = NAN;
            if (!stop && e.psi > 0.0) {
                const double g = e.phi / e.psi - 1.0;
                const double gp = (e.psi * dph - e.phi * dps) / (e.psi * e.psi);
                if (gp < 0.0 && isfinite(g)) {
                    const double corr = g / gp;
                    if (fabs(corr) <= c->eps * a) stop = true;   // converged at a
                    else next = a - corr;
                }
            }
            if (stop) {
                if (pass) { accept_step(c, a, e.psi, e.phi); return; }
                c->amode = AM_BACKOFF;   // from a (cur_alpha)
                continue;
            }
            if (!(next > c->lb && next < c->ub)) {   // safeguard step
                if (c->ub == INFINITY) next = 2.0 * a;
                else if (c->lb == 0.0) next = c->ub / 2.0;
                else next = sqrt(c->lb * c->ub);
            }
            if (next < 1.0) next = 1.0;
            if (next > ALPHA_CAP) next = ALPHA_CAP;
            c->cur_alpha = next;
            continue;
        }
        if (c->amode == AM_BACKOFF) {   // b = a (1-eps)^p below the value Newton stopped at
            double b = c->cur_alpha * (1.0 - c->eps);
            if (b <= c->lb) { accept_step(c, c->lb, c->lb_psi, c->lb_phi); return; }
            if (b < 1.0) b = 1.0;
            Eval e;
            const int r = lookup(c, cr, b, &e);
            if (r == 1) { setup_ladder(c, b, SK_LIST, KN); return; }
            if (r == 2) { setup_refine(c, b); return; }
            c->evaluations += 1;
            if (e.phi >= e.psi) { accept_step(c, b, e.psi, e.phi); return; }
            if (!(b > 1.0)) { stop_infeasible(c); return; }
            c->cur_alpha = b;
            continue;
        }
        // AM_BIS
        if (!(c->ub - c->lb > c->eps * c->lb)) { accept_step(c, c->lb, c->lb_psi, c->lb_phi); return; }
        const double beta = (c->lb + c->ub) / 2.0;
        Eval e;
        int r = lookup(c, cr, beta, &e);
        if (r == 1) { setup_grid(c, c->lb, c->ub); return; }
        if (r == 2) { setup_refine(c, beta); return; }
        c->evaluations += 1;
        if (e.phi >= e.psi) { c->lb = beta; c->lb_psi = e.psi; c->lb_phi = e.phi; }
        else c->ub = beta;
    }
    c->status = ST_NUMERIC;
    c->phase = PH_DONE;
}

// Called after the forward product: start the step decision of this iteration.
MWU_DEV void begin_search(Ctl *c, const double *forced)
{
    c->ref_valid = 0;
    if (c->eval_mode) { c->phase = PH_IDLE; return; }
    if (forced && c->forced_pos < c->n_forced) {
        c->amode = AM_FORCED;
        c->cur_alpha = forced[c->forced_pos++];
        c->skind = SK_LIST;
        c->ncand = 1;
        c->cand[0] = c->cur_alpha;
        c->phase = PH_SEARCH;
        return;
    }
    if (c->step_rule == SR_STD) {   // standard step alpha = 1; predicted LSE moves are safe bounds
        accept_step(c, 1.0, c->onesP ? 0.0 : c->dymax, 0.0);
        return;
    }
    c->amode = AM_EXP;
    c->have_cur = 0;
    if (c->step_rule == SR_NEWTON && c->last_alpha >= 1.0) {   // Newton from the previous step
        c->amode = AM_NEWTON;
        c->cur_alpha = c->last_alpha;
        c->lb = 0.0;
        c->ub = INFINITY;
        c->nw_evals = 0;
        setup_ladder(c, c->cur_alpha, SK_NEWTON, NB);
    } else if (c->step_rule == SR_BIN_WARM && c->last_alpha > 1.0) {   // warm start at the previous step
        c->exp_next = c->last_alpha;
        setup_first_warm(c, c->last_alpha);
    } else {
        c->exp_next = 1.0;
        setup_first(c);
    }
    c->phase = PH_SEARCH;
}

// Store the reduced record of a search pass and advance the state machine.
// rec layout: grid passes [s1P(KC) | s1C(KC) | s2C(KC) | zmin'(KC)];
// refine pass 1 [min z' | max eta*y']; refine pass 2 [sumP | sumC | sumP' |
// sumC'], the last two the derivative sums sum dy e^{eta y' - pm} and
// sum dz e^{-eta (z' - zm)} with the shifts of the first two.
MWU_DEV void finish_search(Ctl *c, const double *rec, bool pre_evaluated = false)
{
    if (held(c)) return;
    c->search_passes += 1;
    if (c->skind == SK_REFINE) {
        if (c->ref_valid == 0) {        // pass 1 produced the shifts
            c->rfZmin = rec[0];
            c->rfPm = rec[1];
            c->ref_valid = -1;          // pass 2 pending
            return;
        }
        // shifts taken from the grid pass that leave a sum out of range:
        // form them exactly, in the two-pass way
        if (c->ref_short && !((c->onesP || (rec[0] > 0.0 && isfinite(rec[0]))) && rec[1] > 0.0 && isfinite(rec[1]))) {
            c->ref_short = 0;
            c->ref_valid = 0;
            return;
        }
        const double a = c->ref_alpha;
        double psi, phi, zmn, dps, dph;
        if (c->onesP) { psi = a * c->dy1; dps = c->dy1; }
        else { psi = (c->rfPm + log(rec[0])) / c->eta - c->LP; dps = rec[2] / rec[0]; }
        if (c->onesC) { phi = a * c->dz1; zmn = c->z1 + a * c->dz1; dph = c->dz1; }
        else { zmn = c->rfZmin; phi = zmn - c->LC - log(rec[1]) / c->eta; dph = rec[3] / rec[1]; }
        c->ref_psi = psi; c->ref_phi = phi; c->ref_zmin = zmn;
        c->ref_dpsi = dps; c->ref_dphi = dph;
        c->ref_valid = 1;
        if (c->eval_mode) {
            const int k = c->ev_cur;
            c->ev_psi[k] = psi; c->ev_phi[k] = phi; c->ev_zmin[k] = zmn; c->ev_ok[k] = 1;
            if (k == 0) { c->ev_dpsi = dps; c->ev_dphi = dph; }
        }
    } else if (!pre_evaluated) {
        for (int k = 0; k < KC; ++k) {
            c->rS1P[k] = rec[k];
            c->rS1C[k] = rec[KC + k];
            c->rS2C[k] = rec[2 * KC + k];
            c->rZmin[k] = rec[3 * KC + k];
        }
        c->ev_cached = 0;
        if (c->eval_mode) {
            for (int k = 0; k < c->ncand; ++k) {
                Eval e = eval_cand(c, k, c->cand[k]);
                c->ev_psi[k] = e.psi; c->ev_phi[k] = e.phi; c->ev_zmin[k] = e.zmin; c->ev_ok[k] = e.ok;
            }
        }
    }
    if (c->eval_mode && c->skind == SK_NEWTON) {
        // derivatives at cand[0]; when the pass cannot give them, cand[0] is refined
        double dps, dph;
        if (c->ev_ok[0] && newton_derivs(c, &dps, &dph)) { c->ev_dpsi = dps; c->ev_dphi = dph; }
        else c->ev_ok[0] = 0;
    }
    if (c->eval_mode) {
        // refine, one at a time, every candidate the grid pass could not resolve
        for (int k = 0; k < c->ncand; ++k)
            if (!c->ev_ok[k]) {
                c->ev_cur = k;
                setup_refine(c, c->cand[k]);
                c->phase = PH_SEARCH;
                return;
            }
        c->phase = PH_IDLE;
        return;
    }
    replay(c);
}

// ------------------------------------------------- finishers of the CSR passes
// Shared by the generic engine and the batched program: they turn the reduced
// record of a pass into the next state of the probe (Algorithm 2).

MWU_DEV void finish_row(Ctl *c, const double *rec)
{
    // rec: [sum w | sum u | min z | max y]
    if (held(c)) return;
    const double a = c->alpha;
    bool bad = false;
    if (c->onesP) {
        c->y1 += a * c->dy1;
        c->LP = c->y1;
        c->invSw = 1.0;
        c->ymax = c->y1;
    } else {
        const double sw = rec[0];
        bad |= !(sw > 0.0) || !isfinite(sw);
        c->LP += log(sw) / c->eta;
        c->invSw = 1.0 / sw;
        c->ymax = rec[3];
    }
    if (c->onesC) {
        c->z1 += a * c->dz1;
        c->LC = c->z1;
        c->invSu = 1.0;
        c->zmin = c->z1;
    } else {
        const double su = rec[1];
        c->zmin = rec[2];
        if (c->drop && c->zmin >= 1.0) {
            // every row met and left out: no weights, the probe ends below
        } else {
            bad |= !(su > 0.0) || !isfinite(su);
            c->LC -= log(su) / c->eta;
            c->invSu = 1.0 / su;
        }
    }
    if (c->eval_mode) { c->phase = PH_COL; return; }
    if (bad) { c->status = ST_NUMERIC; c->phase = PH_COMMIT; return; }
    if (c->zmin >= 1.0) { c->status = ST_FEASIBLE; c->phase = PH_COMMIT; }
    else if (c->iter >= c->max_iter) { c->status = ST_MAX_ITER; c->phase = PH_COMMIT; }
    else c->phase = PH_COL;
}

MWU_DEV void finish_col(Ctl *c, const double *rec)
{
    // rec: [sum d | min g | max d | max h]
    if (held(c)) return;
    c->alpha = 0.0;
    c->dsum = rec[0];
    c->gmin = rec[1];
    c->dmax = rec[2];
    c->hmax = rec[3];
    const double cf = 1.0 - c->qmin;   // margin for the rounding of g and h
    if (c->gmin > 0.0 && 1.0 / (cf * c->gmin) < c->pack_bound) c->pack_bound = 1.0 / (cf * c->gmin);
    if (c->hmax > 0.0 && cf / c->hmax > c->cover_bound) c->cover_bound = cf / c->hmax;
    c->dy1 = c->onesP ? c->sP * c->dsum : 0.0;
    c->dz1 = c->onesC ? c->sC * c->dsum : 0.0;
    if (c->eval_mode) { c->phase = PH_FWD; return; }
    if (!(c->dmax > 0.0)) { c->status = ST_INFEASIBLE; c->phase = PH_DONE; return; }
    c->phase = PH_FWD;
}

MWU_DEV void finish_init_fwd(Ctl *c, const double *rec)
{
    // rec: [min z | max y]
    c->zmin = c->onesC ? c->z1 : rec[0];
    c->ymax = c->onesP ? c->y1 : rec[1];
    c->LP = c->ymax;        // first shifts; the row pass turns them into exact LSE totals
    c->LC = c->zmin;
    c->alpha = 0.0;
    c->status = ST_RUNNING;
    c->phase = PH_ROW;
}

MWU_DEV void finish_sumx(Ctl *c, double sumx)
{
    c->sumx = sumx;
    c->y1 = c->sP * sumx;
    c->z1 = c->sC * sumx;
    c->dy1 = 0.0;
    c->dz1 = 0.0;
}

}  // namespace mwu
