// Classical algebraic multigrid (Section 4.2: Algorithms 3 and 4, eq. (4);
// the defaults of Figure 34) on a scalar matrix: a preconditioner of its own
// and the pressure stage of CPR.
//
// Setup (Algorithm 3) runs on the host, level by level:
//   strength      j is a strong dependency of i when
//                 -s a_ij >= theta max_{k != i} (-s a_ik), s = sign(a_ii);
//                 a row with |sum_j a_ij| > max_row_sum |a_ii| has none
//   coarse points Ruge-Stueben: first pass takes the undecided point with
//                 the largest measure, ties to the smallest index, as C and
//                 the undecided points depending on it as F.  A measure
//                 starts at the number of points depending on the point,
//                 rises by one when one of those becomes F beside a new C
//                 point and falls by one when one becomes C; a point taken
//                 with measure 0 becomes F.  The second pass makes sure a
//                 strong F-F pair shares a C point.
//   interpolation classical: strong F neighbours distributed over the C
//                 points through their entries of sign opposite to their
//                 diagonal, weak neighbours lumped into the diagonal;
//                 weights under trunc times the row's largest dropped and
//                 the row rescaled to its former sum
//   coarse matrix A_{l+1} = P^T (A_l P) (eq. (4)), R = P^T
// Row sums and products are accumulated in ascending column order (these
// values decide the splitting of the next level).  The coarsest level's
// inverse is formed on the GPU by Gauss-Jordan elimination.
//
// Apply (Algorithm 4), one V-cycle from x = 0 on every level:
//   hybrid Gauss-Seidel smoothing: Gauss-Seidel inside chunks of CH
//   consecutive rows, Jacobi between chunks.  Each row splits into its
//   diagonal, its entries on earlier rows of its chunk (a dense CH x CH
//   lower block per chunk) and the rest, which read only the old iterate.
//   A team of T lanes per chunk (T from the level's mean row length) sums
//   the rest for all CH rows at once, combining with shuffles; then the
//   chunk's rows are solved in order against the lower block.  The rest is
//   stored chunk-interleaved: a wavefront holds 64 / T chunks; entry e of
//   row t of chunk c sits at off_g + (t K_g + e / T) 64 + c T + e % T,
//   K_g = the group's longest such row / T rounded up, so every load is
//   coalesced.  Then r = b - A x, b_c = R r, the coarse cycle, x += P x_c,
//   and the smoothing again.
#include <algorithm>
#include <cmath>
#include <numeric>
#include <queue>
#include <thread>
#include <vector>

#include "device.hpp"
#include "internal.hpp"

namespace kry {

namespace {

// ---------------------------------------------------------------------------
// host setup
// ---------------------------------------------------------------------------
// [0, n) cut into contiguous ranges, one per worker thread (at most 16, and
// at least grain items each):
// f(lo, hi, w) for worker w; rows are independent, so the result does not
// depend on the cut
template <typename F>
void for_ranges(int n, int &nw, F f, int grain = 1024) {
    const unsigned hw = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    nw = std::max(1, std::min((int)hw, n / grain));
    if (nw == 1) {
        f(0, n, 0);
        return;
    }
    std::vector<std::thread> th;
    for (int w = 0; w < nw; w++)
        th.emplace_back(f, (int)((int64_t)n * w / nw), (int)((int64_t)n * (w + 1) / nw), w);
    for (auto &x : th) x.join();
}

// rows computed in pieces: per piece its row lengths and entries, then
// concatenated in order (each piece copied by its own thread once the
// offsets are known)
struct Piece {
    std::vector<int> len, ci;
    std::vector<double> v;
    int err = 0, err_row = -1;
};
void join_pieces(int n, std::vector<Piece> &pc, HVec<int> &rp, HVec<int> &ci, HVec<double> *v) {
    const int np = (int)pc.size();
    std::vector<size_t> at(np + 1, 0);
    std::vector<int> r0(np + 1, 0);
    for (int w = 0; w < np; w++) {
        at[w + 1] = at[w] + pc[w].ci.size();
        r0[w + 1] = r0[w] + (int)pc[w].len.size();
    }
    rp.resize(n + 1);
    rp[0] = 0;
    ci.resize(at[np]);
    if (v) v->resize(at[np]);
    auto copy = [&](int w) {
        const Piece &p = pc[w];
        size_t off = at[w];
        int r = r0[w];
        for (int L : p.len) {
            off += L;
            rp[++r] = (int)off;
        }
        std::copy(p.ci.begin(), p.ci.end(), ci.begin() + at[w]);
        if (v) std::copy(p.v.begin(), p.v.end(), v->begin() + at[w]);
    };
    if (np == 1 || at[np] < 65536) {
        for (int w = 0; w < np; w++) copy(w);
        return;
    }
    std::vector<std::thread> th;
    for (int w = 0; w < np; w++) th.emplace_back(copy, w);
    for (auto &x : th) x.join();
}

// strong dependencies of each row (ascending)
void find_strong(const AmgCsr &A, double theta, double mrs, HVec<int> &srp, HVec<int> &sci) {
    std::vector<Piece> pc(16);
    int nw = 1;
    for_ranges(A.n, nw, [&](int lo, int hi, int w) {
        Piece &P = pc[w];
        for (int i = lo; i < hi; i++) {
            const size_t before = P.ci.size();
            double d = 0.0, sum = 0.0;
            for (int q = A.rp[i]; q < A.rp[i + 1]; q++) {
                if (A.ci[q] == i) d = A.v[q];
                sum += A.v[q];
            }
            const double sg = d < 0.0 ? -1.0 : 1.0;
            double big = 0.0;
            for (int q = A.rp[i]; q < A.rp[i + 1]; q++)
                if (A.ci[q] != i && -sg * A.v[q] > big) big = -sg * A.v[q];
            const bool weak_row = mrs < 1.0 && std::fabs(sum) > mrs * std::fabs(d);
            if (!weak_row && big > 0.0)
                for (int q = A.rp[i]; q < A.rp[i + 1]; q++)
                    if (A.ci[q] != i && -sg * A.v[q] >= theta * big) P.ci.push_back(A.ci[q]);
            P.len.push_back((int)(P.ci.size() - before));
        }
    }, 128);
    pc.resize(nw);
    join_pieces(A.n, pc, srp, sci, nullptr);
}

// set of indices in [0, n) as a 64-ary tree of bit words: leaves hold one
// bit per index, each upper word one bit per non-empty word below; insert,
// erase and the smallest element cost one word per level
struct IndexSet {
    std::vector<std::vector<uint64_t>> lv;   // lv[0]: leaves ... lv.back(): one word
    void init(int n) {
        lv.clear();
        size_t bits = (size_t)std::max(n, 1);
        do {
            const size_t words = (bits + 63) / 64;
            lv.emplace_back(words, 0);
            bits = words;
        } while (lv.back().size() > 1);
    }
    void insert(int i) {
        size_t x = (size_t)i;
        for (auto &w : lv) {
            const bool had = w[x >> 6] != 0;
            w[x >> 6] |= 1ull << (x & 63);
            if (had) break;
            x >>= 6;
        }
    }
    void erase(int i) {
        size_t x = (size_t)i;
        for (auto &w : lv) {
            w[x >> 6] &= ~(1ull << (x & 63));
            if (w[x >> 6] != 0) break;
            x >>= 6;
        }
    }
    bool empty() const { return lv.back()[0] == 0; }
    int first() const {
        size_t x = 0;
        for (int l = (int)lv.size() - 1; l >= 0; l--) x = (x << 6) | (size_t)__builtin_ctzll(lv[l][x]);
        return (int)x;
    }
};

// C/F splitting: cf[i] = 1 for C, 0 for F
void split_cf(int n, const HVec<int> &srp, const HVec<int> &sci,
              std::vector<int> &cf) {
    // who depends on i: the transpose of the strong pattern
    std::vector<int> drp(n + 1, 0), dci(sci.size());
    for (int j : sci) drp[j + 1]++;
    std::partial_sum(drp.begin(), drp.end(), drp.begin());
    {
        std::vector<int> at(drp.begin(), drp.end() - 1);
        for (int i = 0; i < n; i++)
            for (int q = srp[i]; q < srp[i + 1]; q++) dci[at[sci[q]]++] = i;
    }
    constexpr int UND = -1;
    std::vector<int> meas(n);
    cf.assign(n, UND);
    // one ordered index set per measure value; the next point is the
    // smallest index in the largest non-empty set.  Every undecided point
    // sits in the set of its current measure.
    int mmax = 0;
    for (int i = 0; i < n; i++) {
        meas[i] = drp[i + 1] - drp[i];
        mmax = std::max(mmax, meas[i]);
    }
    // a measure grows by at most the points depending on it: bounded by
    // twice the longest column of the strong pattern
    std::vector<IndexSet> bucket(2 * (mmax + 1) + 1);
    for (auto &b : bucket) b.init(n);
    for (int i = 0; i < n; i++) {
        if (srp[i + 1] == srp[i] && meas[i] == 0) cf[i] = 0;
        else bucket[meas[i]].insert(i);
    }
    auto shift = [&](int k, int d) {
        bucket[meas[k]].erase(k);
        meas[k] += d;
        bucket[meas[k]].insert(k);
    };
    int top = (int)bucket.size() - 1;
    for (;;) {
        while (top >= 0 && bucket[top].empty()) top--;
        if (top < 0) break;
        const int i = bucket[top].first();
        bucket[top].erase(i);
        if (meas[i] == 0) {
            cf[i] = 0;
            continue;
        }
        cf[i] = 1;
        for (int q = drp[i]; q < drp[i + 1]; q++) {
            const int j = dci[q];
            if (cf[j] != UND) continue;
            bucket[meas[j]].erase(j);
            cf[j] = 0;
            for (int p = srp[j]; p < srp[j + 1]; p++)
                if (cf[sci[p]] == UND) {
                    shift(sci[p], +1);
                    top = std::max(top, meas[sci[p]]);
                }
        }
        for (int q = srp[i]; q < srp[i + 1]; q++)
            if (cf[sci[q]] == UND) shift(sci[q], -1);
    }
    // second pass
    std::vector<int> tag(n, -1);
    for (int i = 0; i < n; i++) {
        if (cf[i] != 0) continue;
        for (int q = srp[i]; q < srp[i + 1]; q++)
            if (cf[sci[q]] == 1) tag[sci[q]] = i;
        int cand = -1;
        bool promote_i = false;
        for (int q = srp[i]; q < srp[i + 1]; q++) {
            const int j = sci[q];
            if (cf[j] != 0 || j == cand) continue;
            bool shared = false;
            for (int p = srp[j]; p < srp[j + 1] && !shared; p++) shared = tag[sci[p]] == i;
            if (shared) continue;
            if (cand >= 0) {
                promote_i = true;
                break;
            }
            cand = j;
            tag[j] = i;
        }
        if (promote_i) cf[i] = 1;
        else if (cand >= 0) cf[cand] = 1;
    }
}

inline bool signs_differ(double d, double x) { return (d > 0.0 && x < 0.0) || (d < 0.0 && x > 0.0); }

int build_prolongation(const AmgCsr &A, const HVec<int> &srp, const HVec<int> &sci,
                       const std::vector<int> &cf, double trunc, AmgCsr &P) {
    const int n = A.n;
    std::vector<int> cnum(n, -1);
    int nc = 0;
    for (int i = 0; i < n; i++)
        if (cf[i]) cnum[i] = nc++;
    auto diag_of = [&](int r) {
        for (int q = A.rp[r]; q < A.rp[r + 1]; q++)
            if (A.ci[q] == r) return A.v[q];
        return 0.0;
    };
    std::vector<Piece> pc(16);
    int nw = 1;
    for_ranges(n, nw, [&](int lo, int hi, int wk) {
        Piece &out = pc[wk];
        std::vector<int> strong_of(n, -1), slot(n, -1), cpts;
        std::vector<double> w;
        for (int i = lo; i < hi && !out.err; i++) {
            const size_t before = out.ci.size();
            if (cf[i]) {
                out.ci.push_back(cnum[i]);
                out.v.push_back(1.0);
                out.len.push_back(1);
                continue;
            }
            cpts.clear();
            w.clear();
            for (int q = srp[i]; q < srp[i + 1]; q++) {
                const int j = sci[q];
                strong_of[j] = i;
                if (cf[j]) {
                    slot[j] = (int)cpts.size();
                    cpts.push_back(j);
                    w.push_back(0.0);
                }
            }
            if (!cpts.empty()) {
                double dd = diag_of(i);
                for (int q = A.rp[i]; q < A.rp[i + 1]; q++) {
                    const int j = A.ci[q];
                    if (j == i) continue;
                    if (strong_of[j] != i) {
                        dd += A.v[q];   // weak neighbour
                    } else if (cf[j]) {
                        w[slot[j]] += A.v[q];
                    } else {
                        const double akk = diag_of(j);
                        double den = 0.0;
                        for (int p = A.rp[j]; p < A.rp[j + 1]; p++) {
                            const int m = A.ci[p];
                            if (strong_of[m] == i && cf[m] && signs_differ(akk, A.v[p])) den += A.v[p];
                        }
                        if (den == 0.0) {
                            dd += A.v[q];
                        } else {
                            for (int p = A.rp[j]; p < A.rp[j + 1]; p++) {
                                const int m = A.ci[p];
                                if (strong_of[m] == i && cf[m] && signs_differ(akk, A.v[p]))
                                    w[slot[m]] += A.v[q] * A.v[p] / den;
                            }
                        }
                    }
                }
                if (dd == 0.0) {
                    out.err = KRY_ERR_ZERO_PIVOT;
                    out.err_row = i;
                    break;
                }
                double wmax = 0.0, total = 0.0, kept = 0.0;
                for (double &x : w) {
                    x = -x / dd;
                    wmax = std::max(wmax, std::fabs(x));
                    total += x;
                }
                for (double x : w)
                    if (std::fabs(x) >= trunc * wmax) kept += x;
                const double sc = kept != 0.0 ? total / kept : 1.0;
                for (size_t t = 0; t < cpts.size(); t++)
                    if (std::fabs(w[t]) >= trunc * wmax) {
                        out.ci.push_back(cnum[cpts[t]]);
                        out.v.push_back(w[t] * sc);
                    }
                for (int j : cpts) slot[j] = -1;
            }
            out.len.push_back((int)(out.ci.size() - before));
        }
    }, 128);
    pc.resize(nw);
    for (auto &p : pc)
        if (p.err) return set_error(p.err, "AMG: zero interpolation diagonal in row %d", p.err_row);
    P.n = n;
    P.m = nc;
    join_pieces(n, pc, P.rp, P.ci, &P.v);
    return KRY_OK;
}

AmgCsr transpose_csr(const AmgCsr &P) {
    AmgCsr T;
    T.n = P.m;
    T.m = P.n;
    T.rp.assign(T.n + 1, 0);
    for (int c : P.ci) T.rp[c + 1]++;
    std::partial_sum(T.rp.begin(), T.rp.end(), T.rp.begin());
    T.ci.resize(P.ci.size());
    T.v.resize(P.v.size());
    std::vector<int> at(T.rp.begin(), T.rp.end() - 1);
    for (int i = 0; i < P.n; i++)
        for (int q = P.rp[i]; q < P.rp[i + 1]; q++) {
            const int p = at[P.ci[q]]++;
            T.ci[p] = i;
            T.v[p] = P.v[q];
        }
    return T;
}

// X Y, each row accumulated over X's entries in ascending order
AmgCsr multiply(const AmgCsr &X, const AmgCsr &Y) {
    AmgCsr Z;
    Z.n = X.n;
    Z.m = Y.m;
    std::vector<Piece> pc(16);
    int nw = 1;
    for_ranges(X.n, nw, [&](int lo, int hi, int wk) {
        Piece &out = pc[wk];
        std::vector<double> acc(Y.m, 0.0);
        std::vector<int> seen(Y.m, -1), cols;
        // room for the products of this range's entries (an upper bound on
        // its output when every product lands in a new column)
        size_t est = 0;
        for (int q = X.rp[lo]; q < X.rp[hi]; q++) est += Y.rp[X.ci[q] + 1] - Y.rp[X.ci[q]];
        out.ci.reserve(est);
        out.v.reserve(est);
        out.len.reserve(hi - lo);
        for (int i = lo; i < hi; i++) {
            cols.clear();
            for (int q = X.rp[i]; q < X.rp[i + 1]; q++) {
                const int k = X.ci[q];
                for (int p = Y.rp[k]; p < Y.rp[k + 1]; p++) {
                    const int j = Y.ci[p];
                    if (seen[j] != i) {
                        seen[j] = i;
                        acc[j] = 0.0;
                        cols.push_back(j);
                    }
                    acc[j] += X.v[q] * Y.v[p];
                }
            }
            // insertion sort for short rows, std::sort for the long rows of
            // coarse levels
            if (cols.size() > 32) {
                std::sort(cols.begin(), cols.end());
            } else {
                for (size_t a = 1; a < cols.size(); a++) {
                    const int c = cols[a];
                    size_t b = a;
                    while (b > 0 && cols[b - 1] > c) {
                        cols[b] = cols[b - 1];
                        b--;
                    }
                    cols[b] = c;
                }
            }
            for (int j : cols) {
                out.ci.push_back(j);
                out.v.push_back(acc[j]);
            }
            out.len.push_back((int)cols.size());
        }
    }, 128);
    pc.resize(nw);
    join_pieces(X.n, pc, Z.rp, Z.ci, &Z.v);
    return Z;
}

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------
// sum over the T lanes of a team (aligned groups of T lanes)
template <int T>
__device__ __forceinline__ double team_sum(double v) {
#pragma unroll
    for (int o = T / 2; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// the chunk's diagonal and lower block: slot m of chunk c of group g at
// (g NL + m) CPW + c, NL = CH (CH + 1) / 2; slot t (t + 1) / 2 + u holds
// row t's entry on row u < t, slot t (t + 1) / 2 + t its diagonal
template <int CH>
constexpr int lower_slots() { return CH * (CH + 1) / 2; }

// sums over the entries that read the old iterate: s[t] for the CH rows.
// Every slot k < K of the group exists (padding holds column -1, value 0),
// so the loads are unconditional and overlap; a padded slot gathers x[0]
// and its product is dropped.
template <int CH, int T>
__device__ __forceinline__ void rest_sums(int K, int64_t base, int lt, const int *len,
                                          const int *__restrict__ ecol,
                                          const double *__restrict__ eval,
                                          const double *__restrict__ x, double (&s)[CH]) {
#pragma unroll
    for (int t = 0; t < CH; t++) s[t] = 0.0;
#pragma unroll 4
    for (int k = 0; k < K; k++) {
#pragma unroll
        for (int t = 0; t < CH; t++) {
            const int64_t p = base + ((int64_t)(t * K + k) << 6);
            const int j = ecol[p];
            const double a = eval[p];
            const double xv = x[j < 0 ? 0 : j];
            s[t] += k * T + lt < len[t] ? a * xv : 0.0;
        }
    }
#pragma unroll
    for (int t = 0; t < CH; t++) s[t] = team_sum<T>(s[t]);
}

// one hybrid Gauss-Seidel sweep: xn from xo (xo == nullptr: from zero)
template <int CH, int T>
__global__ __launch_bounds__(256) void k_amg_smooth(int n, int nch, const int64_t *__restrict__ goff,
                                                    const int *__restrict__ gk,
                                                    const int *__restrict__ rlen,
                                                    const int *__restrict__ ecol,
                                                    const double *__restrict__ eval,
                                                    const double *__restrict__ low,
                                                    const double *__restrict__ b,
                                                    const double *__restrict__ xo,
                                                    double *__restrict__ xn) {
    constexpr int CPW = 64 / T, NL = lower_slots<CH>();
    const int gl = blockIdx.x * blockDim.x + threadIdx.x;
    const int grp = gl >> 6, lane = gl & 63;
    const int c = lane / T, lt = lane % T;
    const int q = grp * CPW + c;                      // this team's chunk
    if (grp * CPW >= nch) return;                     // whole wavefront idle
    const bool live = q < nch;
    const int r0 = q * CH;
    int len[CH];
#pragma unroll
    for (int t = 0; t < CH; t++)
        len[t] = live && r0 + t < n ? rlen[((int64_t)grp * CH + t) * CPW + c] : 0;
    double s[CH];
    if (xo) {
        rest_sums<CH, T>(gk[grp], goff[grp] + lane, lt, len, ecol, eval, xo, s);
    } else {
#pragma unroll
        for (int t = 0; t < CH; t++) s[t] = 0.0;
    }
    if (!live || lt != 0) return;
    const double *lw = low + (int64_t)grp * NL * CPW + c;
    double xl[CH];
#pragma unroll
    for (int t = 0; t < CH; t++) {
        const int r = r0 + t;
        xl[t] = 0.0;
        if (r >= n) continue;
        double v = b[r] - s[t];
#pragma unroll
        for (int u = 0; u < t; u++) v -= lw[(t * (t + 1) / 2 + u) * CPW] * xl[u];
        xl[t] = v / lw[(t * (t + 1) / 2 + t) * CPW];
        xn[r] = xl[t];
    }
}

// r = b - A x in the same layout
template <int CH, int T>
__global__ __launch_bounds__(256) void k_amg_resid(int n, int nch, const int64_t *__restrict__ goff,
                                                   const int *__restrict__ gk,
                                                   const int *__restrict__ rlen,
                                                   const int *__restrict__ ecol,
                                                   const double *__restrict__ eval,
                                                   const double *__restrict__ low,
                                                   const double *__restrict__ b,
                                                   const double *__restrict__ x,
                                                   double *__restrict__ r) {
    constexpr int CPW = 64 / T, NL = lower_slots<CH>();
    const int gl = blockIdx.x * blockDim.x + threadIdx.x;
    const int grp = gl >> 6, lane = gl & 63;
    const int c = lane / T, lt = lane % T;
    const int q = grp * CPW + c;
    if (grp * CPW >= nch) return;
    const bool live = q < nch;
    const int r0 = q * CH;
    int len[CH];
#pragma unroll
    for (int t = 0; t < CH; t++)
        len[t] = live && r0 + t < n ? rlen[((int64_t)grp * CH + t) * CPW + c] : 0;
    double s[CH];
    rest_sums<CH, T>(gk[grp], goff[grp] + lane, lt, len, ecol, eval, x, s);
    if (!live || lt != 0) return;
    const double *lw = low + (int64_t)grp * NL * CPW + c;
#pragma unroll
    for (int t = 0; t < CH; t++) {
        const int row = r0 + t;
        if (row >= n) continue;
        double v = s[t];
#pragma unroll
        for (int u = 0; u <= t; u++) v += lw[(t * (t + 1) / 2 + u) * CPW] * x[r0 + u];
        r[row] = b[row] - v;
    }
}

// y = M x (add = 0) or y += M x (add = 1), one row per thread
__global__ __launch_bounds__(256) void k_amg_csr(int rows, const int *__restrict__ rp,
                                                 const int *__restrict__ ci,
                                                 const double *__restrict__ v,
                                                 const double *__restrict__ x,
                                                 double *__restrict__ y, int add) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= rows) return;
    double s = 0.0;
    for (int q = rp[i]; q < rp[i + 1]; q++) s += v[q] * x[ci[q]];
    y[i] = add ? y[i] + s : s;
}

// x = Minv b, one wavefront per row of the dense inverse
__global__ __launch_bounds__(256) void k_amg_dense(int n, const double *__restrict__ Minv,
                                                   const double *__restrict__ b,
                                                   double *__restrict__ x) {
    const int row = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (row >= n) return;
    const double *m = Minv + (int64_t)row * n;
    double s = 0.0;
    for (int j = lane; j < n; j += 64) s += m[j] * b[j];
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    if (lane == 0) x[row] = s;
}

// step k of in-place Gauss-Jordan inversion without pivoting, M -> Mn:
// Gauss-Jordan inversion of the coarsest matrix in panels of GJ_RB pivots.
// One pivot k: the pivot row is divided by the pivot, the pivot column
// negated and divided, the rest reduced, and the pivot becomes its
// reciprocal.  A panel K of rb pivots does rb such steps at once: with
// P = M_KK^-1 (the steps applied to the diagonal block alone) and
// W = P M_KR, the new matrix is M_KK = P, M_KR = W, M_RK = -M_RK P and
// M_RR = M_RR - M_RK W.
constexpr int GJ_RB = 32;

// P = inverse of the rb x rb diagonal block at (k0, k0), one thread per
// entry; err is set if a pivot is zero or not finite
__global__ __launch_bounds__(1024) void k_amg_gj_panel(int n, int k0, int rb,
                                                       const double *__restrict__ M,
                                                       double *__restrict__ P, int *err) {
    __shared__ double a[2][GJ_RB][GJ_RB];
    __shared__ int bad;
    const int t = threadIdx.x, i = t / GJ_RB, j = t % GJ_RB;
    const bool in = i < rb && j < rb;
    if (t == 0) bad = 0;
    a[0][i][j] = in ? M[(int64_t)(k0 + i) * n + k0 + j] : 0.0;
    __syncthreads();
    int c = 0;
    for (int k = 0; k < rb; k++) {
        const double piv = a[c][k][k];
        const bool ok = std::fabs(piv) > 0.0 && std::isfinite(piv);
        if (!ok && t == 0) bad = 1;
        double val = 0.0;
        if (in && ok) {
            if (i == k) val = j == k ? 1.0 / piv : a[c][k][j] / piv;
            else if (j == k) val = -a[c][i][k] / piv;
            else val = a[c][i][j] - a[c][i][k] * a[c][k][j] / piv;
        }
        a[c ^ 1][i][j] = val;
        __syncthreads();
        c ^= 1;
    }
    if (in) P[i * GJ_RB + j] = a[c][i][j];
    if (t == 0 && bad) *err = 1;
}

// W = P M_K., rb rows of n (row b at W + b n)
__global__ __launch_bounds__(256) void k_amg_gj_w(int n, int k0, int rb, const double *__restrict__ M,
                                                  const double *__restrict__ P,
                                                  double *__restrict__ W) {
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= (int64_t)rb * n) return;
    const int b = (int)(e / n), j = (int)(e - (int64_t)b * n);
    double s = 0.0;
    for (int c = 0; c < rb; c++) s += P[b * GJ_RB + c] * M[(int64_t)(k0 + c) * n + j];
    W[e] = s;
}

// the matrix after the panel's rb steps, out of place (Mn from M)
__global__ __launch_bounds__(256) void k_amg_gj_update(int n, int k0, int rb,
                                                       const double *__restrict__ M,
                                                       const double *__restrict__ P,
                                                       const double *__restrict__ W,
                                                       double *__restrict__ Mn) {
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= (int64_t)n * n) return;
    const int i = (int)(e / n), j = (int)(e - (int64_t)i * n);
    const bool ik = i >= k0 && i < k0 + rb, jk = j >= k0 && j < k0 + rb;
    const double *mi = M + (int64_t)i * n + k0;   // row i of the panel's columns
    double val;
    if (ik && jk) {
        val = P[(i - k0) * GJ_RB + (j - k0)];
    } else if (ik) {
        val = W[(int64_t)(i - k0) * n + j];
    } else if (jk) {
        double s = 0.0;
        for (int b = 0; b < rb; b++) s += mi[b] * P[b * GJ_RB + (j - k0)];
        val = -s;
    } else {
        double s = M[e];
        for (int b = 0; b < rb; b++) s -= mi[b] * W[(int64_t)b * n + j];
        val = s;
    }
    Mn[e] = val;
}

constexpr int AMG_DENSE_MAX = 8192;

}  // namespace

// team size for a level: about 4 entries of a row per lane
static int team_size(const AmgCsr &A) {
    const double mean = A.n ? (double)A.ci.size() / A.n : 0.0;
    int T = 1;
    while (T < 32 && mean > 4.0 * T) T *= 2;
    return T;
}

// chunk-interleaved rows of A (see the head of the file), built on the
// host: every wavefront group owns its own ranges of the arrays, so the
// groups are filled in parallel
struct EllHost {
    int n = 0, nch = 0, team = 1, ngrp = 0;
    std::vector<int64_t> goff;
    std::vector<int> gk;
    HVec<int> rlen, ecol;
    HVec<double> eval, low;
};
static void build_ell(const AmgCsr &A, int ch, EllHost &E) {
    const int n = A.n, T = team_size(A), cpw = 64 / T, nl = ch * (ch + 1) / 2;
    const int nch = (n + ch - 1) / ch, ngrp = (nch + cpw - 1) / cpw;
    const int gr = cpw * ch;   // rows per group
    // an entry (r, j) is "lower" when j lies in r's chunk at or before r
    auto lower = [&](int r, int j) { return j <= r && j >= r / ch * ch; };
    E.n = n;
    E.nch = nch;
    E.team = T;
    E.ngrp = ngrp;
    E.goff.assign(ngrp + 1, 0);
    E.gk.assign(ngrp, 0);
    int nw = 1;
    for_ranges(ngrp, nw, [&](int glo, int ghi, int) {
        for (int g = glo; g < ghi; g++) {
            int K = 0;
            for (int r = g * gr; r < std::min(n, (g + 1) * gr); r++) {
                int rest = 0;
                for (int q = A.rp[r]; q < A.rp[r + 1]; q++) rest += !lower(r, A.ci[q]);
                K = std::max(K, rest);
            }
            E.gk[g] = (K + T - 1) / T;
        }
    }, 64);
    for (int g = 0; g < ngrp; g++) E.goff[g + 1] = E.goff[g] + (int64_t)ch * E.gk[g] * 64;
    const size_t ne = std::max<int64_t>(E.goff[ngrp], 1);
    E.rlen.resize((size_t)ngrp * ch * cpw);
    E.ecol.resize(ne);
    E.eval.resize(ne);
    E.low.resize((size_t)ngrp * nl * cpw);
    if (E.goff[ngrp] == 0) {
        E.ecol[0] = -1;
        E.eval[0] = 0.0;
    }
    for_ranges(ngrp, nw, [&](int glo, int ghi, int) {
        std::fill(E.ecol.begin() + E.goff[glo], E.ecol.begin() + E.goff[ghi], -1);
        std::fill(E.eval.begin() + E.goff[glo], E.eval.begin() + E.goff[ghi], 0.0);
        std::fill(E.rlen.begin() + (size_t)glo * ch * cpw, E.rlen.begin() + (size_t)ghi * ch * cpw, 0);
        std::fill(E.low.begin() + (size_t)glo * nl * cpw, E.low.begin() + (size_t)ghi * nl * cpw, 0.0);
        for (int r = glo * gr; r < std::min(n, ghi * gr); r++) {
            const int q = r / ch, t = r % ch, g = q / cpw, c = q % cpw;
            int e = 0;
            for (int k = A.rp[r]; k < A.rp[r + 1]; k++) {
                const int j = A.ci[k];
                if (lower(r, j)) {
                    E.low[((size_t)g * nl + t * (t + 1) / 2 + (j - q * ch)) * cpw + c] += A.v[k];
                    continue;
                }
                const int64_t p = E.goff[g] + (int64_t)(t * E.gk[g] + e / T) * 64 + c * T + e % T;
                E.ecol[p] = j;
                E.eval[p] = A.v[k];
                e++;
            }
            E.rlen[((size_t)g * ch + t) * cpw + c] = e;
        }
    }, 64);
}

static int upload_level(hipStream_t s, const AmgCsr &A, int ch, AmgLevel &L) {
    EllHost E;
    build_ell(A, ch, E);
    const int ngrp = E.ngrp;
    L.n = E.n;
    L.nch = E.nch;
    L.team = E.team;
    KRY_TRY(L.goff.alloc(ngrp));
    KRY_TRY(L.gk.alloc(ngrp));
    KRY_TRY(L.rlen.alloc(E.rlen.size()));
    KRY_TRY(L.ecol.alloc(E.ecol.size()));
    KRY_TRY(L.eval.alloc(E.eval.size()));
    KRY_TRY(L.low.alloc(E.low.size()));
    KRY_HIP(hipMemcpyAsync(L.low.p, E.low.data(), sizeof(double) * E.low.size(), hipMemcpyHostToDevice, s));
    KRY_HIP(hipMemcpyAsync(L.goff.p, E.goff.data(), sizeof(int64_t) * ngrp, hipMemcpyHostToDevice, s));
    KRY_HIP(hipMemcpyAsync(L.gk.p, E.gk.data(), sizeof(int) * ngrp, hipMemcpyHostToDevice, s));
    KRY_HIP(hipMemcpyAsync(L.rlen.p, E.rlen.data(), sizeof(int) * E.rlen.size(), hipMemcpyHostToDevice, s));
    KRY_HIP(hipMemcpyAsync(L.ecol.p, E.ecol.data(), sizeof(int) * E.ecol.size(), hipMemcpyHostToDevice, s));
    KRY_HIP(hipMemcpyAsync(L.eval.p, E.eval.data(), sizeof(double) * E.eval.size(), hipMemcpyHostToDevice, s));
    L.ell_bytes = (int64_t)E.ecol.size() * (sizeof(int) + sizeof(double));
    KRY_HIP(hipStreamSynchronize(s));   // the host vectors go out of scope
    return KRY_OK;
}

static int upload_csr(hipStream_t s, const AmgCsr &M, DBuf<int> &rp, DBuf<int> &ci, DBuf<double> &v) {
    KRY_TRY(rp.alloc(M.n + 1));
    KRY_TRY(ci.alloc(std::max<size_t>(M.ci.size(), 1)));
    KRY_TRY(v.alloc(std::max<size_t>(M.v.size(), 1)));
    KRY_HIP(hipMemcpyAsync(rp.p, M.rp.data(), sizeof(int) * (M.n + 1), hipMemcpyHostToDevice, s));
    if (!M.ci.empty()) {
        KRY_HIP(hipMemcpyAsync(ci.p, M.ci.data(), sizeof(int) * M.ci.size(), hipMemcpyHostToDevice, s));
        KRY_HIP(hipMemcpyAsync(v.p, M.v.data(), sizeof(double) * M.v.size(), hipMemcpyHostToDevice, s));
    }
    KRY_HIP(hipStreamSynchronize(s));
    return KRY_OK;
}

int amg_setup(hipStream_t s, int n, const int *h_rowptr, const int *h_col, const double *d_val,
              const AmgOpts &o, AmgPC &M, int *d_err) {
    if (n < 1) return set_error(KRY_ERR_ARG, "AMG: empty matrix");
    if (o.max_levels < 1 || o.num_sweeps < 1 || !(o.strength > 0.0) || o.trunc < 0.0)
        return set_error(KRY_ERR_ARG, "AMG: bad options");
    const int ch = o.gs_chunk;
    if (ch != 1 && ch != 2 && ch != 4 && ch != 8 && ch != 16)
        return set_error(KRY_ERR_UNSUPPORTED, "AMG: Gauss-Seidel chunk %d (1, 2, 4, 8 or 16)", ch);
    M.o = o;
    M.host.clear();
    M.lev.clear();
    // level 0 on the host
    AmgLevelHost H0;
    H0.A.n = H0.A.m = n;
    H0.A.rp.assign(h_rowptr, h_rowptr + n + 1);
    const int nnz = h_rowptr[n];
    H0.A.ci.assign(h_col, h_col + nnz);
    H0.A.v.resize(nnz);
    KRY_HIP(hipMemcpyAsync(H0.A.v.data(), d_val, sizeof(double) * nnz, hipMemcpyDeviceToHost, s));
    KRY_HIP(hipStreamSynchronize(s));
    M.host.push_back(std::move(H0));
    for (int l = 0;; l++) {
        AmgLevelHost &H = M.host[l];
        bool last = l == o.max_levels - 1 || H.A.n <= o.coarse_size;
        if (!last) {
            HVec<int> srp, sci;
            find_strong(H.A, o.strength, o.max_row_sum, srp, sci);
            split_cf(H.A.n, srp, sci, H.cf);
            KRY_TRY(build_prolongation(H.A, srp, sci, H.cf, o.trunc, H.P));
            if (H.P.m == 0 || H.P.m == H.A.n) {   // no coarsening: solve here
                H.cf.clear();
                H.P = AmgCsr();
                last = true;
            }
        }
        if (last) break;
        AmgLevelHost next;
        next.A = multiply(transpose_csr(H.P), multiply(H.A, H.P));
        M.host.push_back(std::move(next));
    }
    const int nlev = (int)M.host.size();
    const int nl = M.host.back().A.n;
    if (nl > AMG_DENSE_MAX)
        return set_error(KRY_ERR_UNSUPPORTED, "AMG: coarsest level of %d rows is too large for its dense "
                         "solve (raise max_levels)", nl);
    // device levels
    for (int l = 0; l < nlev; l++) M.lev.emplace_back(new AmgLevel());
    for (int l = 0; l < nlev; l++) {
        AmgLevelHost &H = M.host[l];
        AmgLevel &L = *M.lev[l];
        L.n = H.A.n;
        KRY_TRY(L.x.alloc(L.n));
        KRY_TRY(L.t.alloc(L.n));
        KRY_TRY(L.r.alloc(L.n));
        KRY_TRY(L.b.alloc(L.n));
        if (l == nlev - 1) break;
        KRY_TRY(upload_level(s, H.A, ch, L));
        L.nc = H.P.m;
        KRY_TRY(upload_csr(s, H.P, L.prp, L.pci, L.pv));
        KRY_TRY(upload_csr(s, transpose_csr(H.P), L.rrp, L.rci, L.rv));
    }
    // dense inverse of the coarsest matrix
    {
        const AmgCsr &C = M.host.back().A;
        std::vector<double> dense((size_t)nl * nl, 0.0);
        for (int i = 0; i < nl; i++)
            for (int q = C.rp[i]; q < C.rp[i + 1]; q++) dense[(size_t)i * nl + C.ci[q]] += C.v[q];
        DBuf<double> tmp, pb, wb;
        KRY_TRY(M.cinv.alloc((size_t)nl * nl));
        KRY_TRY(tmp.alloc((size_t)nl * nl));
        KRY_TRY(pb.alloc((size_t)GJ_RB * GJ_RB));
        KRY_TRY(wb.alloc((size_t)GJ_RB * nl));
        KRY_HIP(hipMemcpyAsync(M.cinv.p, dense.data(), sizeof(double) * dense.size(),
                               hipMemcpyHostToDevice, s));
        const int64_t ne = (int64_t)nl * nl;
        const dim3 g((unsigned)((ne + 255) / 256)), blk(256);
        double *cur = M.cinv.p, *nxt = tmp.p;
        for (int k0 = 0; k0 < nl; k0 += GJ_RB) {
            const int rb = std::min(GJ_RB, nl - k0);
            hipLaunchKernelGGL(k_amg_gj_panel, dim3(1), dim3(GJ_RB * GJ_RB), 0, s, nl, k0, rb, cur,
                               pb.p, d_err);
            hipLaunchKernelGGL(k_amg_gj_w, dim3((unsigned)(((int64_t)rb * nl + 255) / 256)), blk, 0,
                               s, nl, k0, rb, cur, pb.p, wb.p);
            hipLaunchKernelGGL(k_amg_gj_update, g, blk, 0, s, nl, k0, rb, cur, pb.p, wb.p, nxt);
            std::swap(cur, nxt);
        }
        KRY_HIP(hipGetLastError());
        if (cur != M.cinv.p)
            KRY_HIP(hipMemcpyAsync(M.cinv.p, cur, sizeof(double) * ne, hipMemcpyDeviceToDevice, s));
        KRY_HIP(hipStreamSynchronize(s));
    }
    return KRY_OK;
}

// lanes of a level's smoother and residual launches
static dim3 amg_grid(const AmgLevel &L) {
    const int cpw = 64 / L.team;
    const int64_t waves = (L.nch + cpw - 1) / cpw;
    return dim3((unsigned)((waves + 3) / 4));
}

template <int CH, int T>
static void launch_pair(hipStream_t s, bool sm, const AmgLevel &L, const double *b,
                        const double *xin, double *out) {
    if (sm)
        hipLaunchKernelGGL((k_amg_smooth<CH, T>), amg_grid(L), dim3(256), 0, s, L.n, L.nch, L.goff.p,
                           L.gk.p, L.rlen.p, L.ecol.p, L.eval.p, L.low.p, b, xin, out);
    else
        hipLaunchKernelGGL((k_amg_resid<CH, T>), amg_grid(L), dim3(256), 0, s, L.n, L.nch, L.goff.p,
                           L.gk.p, L.rlen.p, L.ecol.p, L.eval.p, L.low.p, b, xin, out);
}

template <int CH>
static void launch_team(hipStream_t s, bool sm, const AmgLevel &L, const double *b,
                        const double *xin, double *out) {
    switch (L.team) {
    case 1: launch_pair<CH, 1>(s, sm, L, b, xin, out); break;
    case 2: launch_pair<CH, 2>(s, sm, L, b, xin, out); break;
    case 4: launch_pair<CH, 4>(s, sm, L, b, xin, out); break;
    case 8: launch_pair<CH, 8>(s, sm, L, b, xin, out); break;
    case 16: launch_pair<CH, 16>(s, sm, L, b, xin, out); break;
    default: launch_pair<CH, 32>(s, sm, L, b, xin, out); break;
    }
}

// smoothing sweep (sm) or residual on level L
static void level_op(hipStream_t s, int ch, bool sm, const AmgLevel &L, const double *b,
                     const double *xin, double *out) {
    switch (ch) {
    case 1: launch_team<1>(s, sm, L, b, xin, out); break;
    case 2: launch_team<2>(s, sm, L, b, xin, out); break;
    case 4: launch_team<4>(s, sm, L, b, xin, out); break;
    case 8: launch_team<8>(s, sm, L, b, xin, out); break;
    default: launch_team<16>(s, sm, L, b, xin, out); break;
    }
}

int amg_apply(hipStream_t s, AmgPC &M, const double *b, double *x, int *d_err) {
    (void)d_err;
    TimedScope ts("amg_vcycle", s);
    const int nlev = (int)M.lev.size(), ch = M.o.gs_chunk, ns = M.o.num_sweeps;
    const dim3 blk(256);
    // level l's right-hand side and result; cur[l] holds the running iterate
    std::vector<const double *> bl(nlev);
    std::vector<double *> cur(nlev), alt(nlev);
    for (int l = 0; l < nlev; l++) {
        bl[l] = l == 0 ? b : M.lev[l]->b.p;
        cur[l] = M.lev[l]->x.p;
        alt[l] = M.lev[l]->t.p;
    }
    // level 0 works in x itself: 2 ns sweeps (an even number of swaps) end there
    cur[0] = x;
    auto sweeps = [&](int l, bool from_zero) {
        for (int k = 0; k < ns; k++) {
            level_op(s, ch, true, *M.lev[l], bl[l], from_zero && k == 0 ? nullptr : cur[l], alt[l]);
            std::swap(cur[l], alt[l]);
        }
    };
    for (int l = 0; l < nlev - 1; l++) {
        AmgLevel &L = *M.lev[l];
        sweeps(l, true);
        level_op(s, ch, false, L, bl[l], cur[l], L.r.p);
        hipLaunchKernelGGL(k_amg_csr, dim3((L.nc + 255) / 256), blk, 0, s, L.nc, L.rrp.p, L.rci.p,
                           L.rv.p, L.r.p, M.lev[l + 1]->b.p, 0);
    }
    {
        AmgLevel &C = *M.lev[nlev - 1];
        hipLaunchKernelGGL(k_amg_dense, dim3((C.n + 3) / 4), blk, 0, s, C.n, M.cinv.p, bl[nlev - 1],
                           cur[nlev - 1]);
    }
    for (int l = nlev - 2; l >= 0; l--) {
        AmgLevel &L = *M.lev[l];
        hipLaunchKernelGGL(k_amg_csr, dim3((L.n + 255) / 256), blk, 0, s, L.n, L.prp.p, L.pci.p,
                           L.pv.p, cur[l + 1], cur[l], 1);
        sweeps(l, false);
    }
    if (cur[0] != x)
        KRY_HIP(hipMemcpyAsync(x, cur[0], sizeof(double) * M.lev[0]->n, hipMemcpyDeviceToDevice, s));
    KRY_HIP(hipGetLastError());
    return KRY_OK;
}

}  // namespace kry
