// Portability tuning on an execution-time table (host code of libfewfit).
//
// Sec. IV-B: PortabilityTune returns a set kappa of variants that is best by a
// summary metric over a set of inputs.  Sec. IV-D-1, Eq. 1: the metric for a
// library is the geometric mean, over inputs, of the runtime the set achieves
// relative to the best known variant for that input.  The set performs like
// its best member on each input (Fig. 1), so the numerator is the minimum
// runtime over kappa.
//
// Work is done in log space: L[v][s] = log(t[v][s] / best[s]) >= 0, so the
// cost of a set is exp(mean_s min_{v in kappa} L[v][s]); log is monotone, so
// the minimising member per shape is the same as for runtimes.
//
// Search (Sec. IV-C-1): the paper notes exhaustive search over |K|^|kappa|
// combinations becomes intractable beyond |kappa| = 2 for 1,343 variants.
// Two things keep it exact here for k <= 4 on a few hundred variants:
//   * dominance pruning: a variant that is no faster than some other variant
//     on every selected shape can be replaced by it in any set without raising
//     the cost, so it is dropped (keeping the lower id among equals);
//   * a depth-first walk over unordered subsets with running per-shape minima.
// For larger k a greedy construction is refined by single swaps until no
// swap lowers the cost (a local optimum).

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <limits>
#include <vector>

#include "../../include/fewfit.h"
#include "ptune_internal.h"

#define FF_EXPORT extern "C" __attribute__((visibility("default")))

double ptune_log2_size(int64_t x) { return std::log2((double)std::max<int64_t>(1, x)); }

namespace {

const double kInf = std::numeric_limits<double>::infinity();

bool finite_pos(double x) { return std::isfinite(x) && x > 0.0; }

// Per-shape best over all variants (the paper's per-input "Oracle").
void column_best(int nv, int ns, const double* t, std::vector<double>& best, std::vector<int>& best_id)
{
    best.assign(ns, kInf);
    best_id.assign(ns, -1);
    for (int s = 0; s < ns; ++s)
        for (int v = 0; v < nv; ++v) {
            const double x = t[(int64_t)v * ns + s];
            if (finite_pos(x) && x < best[s]) {
                best[s] = x;
                best_id[s] = v;
            }
        }
}

struct LogTable {
    int nv = 0, nsel = 0;
    std::vector<double> L;  // nv x nsel, +inf for failed entries
    bool ok = true;         // every selected shape has some finite entry
    double at(int v, int j) const { return L[(size_t)v * nsel + j]; }
};

LogTable make_log_table(int nv, int ns, const double* t, const std::vector<int>& sel)
{
    std::vector<double> best;
    std::vector<int> bid;
    column_best(nv, ns, t, best, bid);
    LogTable lt;
    lt.nv = nv;
    lt.nsel = (int)sel.size();
    lt.L.assign((size_t)nv * lt.nsel, kInf);
    for (int j = 0; j < lt.nsel; ++j) {
        const int s = sel[j];
        if (bid[s] < 0) lt.ok = false;
        for (int v = 0; v < nv; ++v) {
            const double x = t[(int64_t)v * ns + s];
            if (finite_pos(x) && bid[s] >= 0) lt.L[(size_t)v * lt.nsel + j] = std::log(x / best[s]);
        }
    }
    return lt;
}

// Weighted-time table for the fleet objective: L[v][j] = w_j * t[v][s_j]
// (+inf where failed); a set's cost is the plain sum of per-shape minima.
LogTable make_time_table(int nv, int ns, const double* t, const std::vector<int>& sel, const double* w)
{
    LogTable lt;
    lt.nv = nv;
    lt.nsel = (int)sel.size();
    lt.L.assign((size_t)nv * lt.nsel, kInf);
    for (int j = 0; j < lt.nsel; ++j) {
        bool any = false;
        for (int v = 0; v < nv; ++v) {
            const double x = t[(int64_t)v * ns + sel[j]];
            if (finite_pos(x)) {
                lt.L[(size_t)v * lt.nsel + j] = w[j] * x;
                any = true;
            }
        }
        if (!any) lt.ok = false;
    }
    return lt;
}

double set_logsum(const LogTable& lt, const int* kappa, int k)
{
    double sum = 0.0;
    for (int j = 0; j < lt.nsel; ++j) {
        double m = kInf;
        for (int i = 0; i < k; ++i) m = std::min(m, lt.at(kappa[i], j));
        if (m == kInf) return kInf;
        sum += m;
    }
    return sum;
}

double cost_of(const LogTable& lt, double logsum)
{
    return logsum == kInf ? kInf : std::exp(logsum / lt.nsel);
}

bool selection(int ns, int nsel, const int* shapes, std::vector<int>& sel)
{
    sel.clear();
    if (shapes == nullptr) {
        for (int s = 0; s < ns; ++s) sel.push_back(s);
    } else {
        for (int j = 0; j < nsel; ++j) {
            if (shapes[j] < 0 || shapes[j] >= ns) return false;
            sel.push_back(shapes[j]);
        }
    }
    return !sel.empty();
}

// Variants not dominated on the selected shapes, in ascending id order.
std::vector<int> undominated(const LogTable& lt)
{
    std::vector<int> keep;
    for (int v = 0; v < lt.nv; ++v) {
        bool any_finite = false;
        for (int j = 0; j < lt.nsel; ++j) any_finite |= (lt.at(v, j) != kInf);
        if (!any_finite) continue;
        bool dominated = false;
        for (int u = 0; u < lt.nv && !dominated; ++u) {
            if (u == v) continue;
            bool le = true, lt_strict = false;
            for (int j = 0; j < lt.nsel && le; ++j) {
                const double a = lt.at(u, j), b = lt.at(v, j);
                if (a > b) le = false;
                else if (a < b) lt_strict = true;
            }
            // u dominates v if no worse anywhere and better somewhere, or
            // identical everywhere with a lower id.
            if (le && (lt_strict || u < v)) dominated = true;
        }
        if (!dominated) keep.push_back(v);
    }
    return keep;
}

struct Exhaustive {
    const LogTable& lt;
    const std::vector<int>& cand;
    int k;
    std::vector<int> cur, best_set;
    double best_sum = kInf;
    int64_t evals = 0;
    std::vector<std::vector<double>> mins;  // running per-shape minima by depth

    Exhaustive(const LogTable& l, const std::vector<int>& c, int kk) : lt(l), cand(c), k(kk)
    {
        mins.assign(k + 1, std::vector<double>(lt.nsel, kInf));
        cur.resize(k);
    }
    void run(int depth, int start)
    {
        if (depth == k) {
            ++evals;
            double sum = 0.0;
            for (int j = 0; j < lt.nsel; ++j) sum += mins[depth][j];
            if (sum < best_sum) {
                best_sum = sum;
                best_set = cur;
            }
            return;
        }
        const int n = (int)cand.size();
        for (int i = start; i <= n - (k - depth); ++i) {
            const int v = cand[i];
            cur[depth] = v;
            const std::vector<double>& prev = mins[depth];
            std::vector<double>& next = mins[depth + 1];
            for (int j = 0; j < lt.nsel; ++j) next[j] = std::min(prev[j], lt.at(v, j));
            run(depth + 1, i + 1);
        }
    }
};

int64_t n_choose_k_capped(int64_t n, int64_t k, int64_t cap)
{
    if (k < 0 || k > n) return 0;
    k = std::min(k, n - k);
    double r = 1.0;
    for (int64_t i = 1; i <= k; ++i) {
        r = r * (double)(n - k + i) / (double)i;
        if (r > (double)cap) return cap + 1;
    }
    return (int64_t)std::llround(r);
}

// Greedy: add the member that lowers the cost most; then single swaps.
std::vector<int> greedy_swap(const LogTable& lt, const std::vector<int>& cand, int k, int64_t& evals)
{
    std::vector<int> set;
    std::vector<double> mins(lt.nsel, kInf);
    auto sum_with = [&](const std::vector<double>& m, int v) {
        double sum = 0.0;
        for (int j = 0; j < lt.nsel; ++j) sum += std::min(m[j], lt.at(v, j));
        return sum;
    };
    for (int step = 0; step < k; ++step) {
        int bv = -1;
        double bs = kInf;
        bool have = false;
        for (int v : cand) {
            if (std::find(set.begin(), set.end(), v) != set.end()) continue;
            const double s = sum_with(mins, v);
            ++evals;
            if (!have || s < bs) {
                have = true;
                bs = s;
                bv = v;
            }
        }
        if (bv < 0) break;
        set.push_back(bv);
        for (int j = 0; j < lt.nsel; ++j) mins[j] = std::min(mins[j], lt.at(bv, j));
    }
    double cur = set_logsum(lt, set.data(), (int)set.size());
    bool improved = true;
    while (improved) {
        improved = false;
        for (size_t p = 0; p < set.size() && !improved; ++p) {
            for (int v : cand) {
                if (std::find(set.begin(), set.end(), v) != set.end()) continue;
                std::vector<int> trial = set;
                trial[p] = v;
                const double s = set_logsum(lt, trial.data(), (int)trial.size());
                ++evals;
                if (s < cur - 1e-12 * std::max(1.0, std::fabs(cur))) {
                    set = trial;
                    cur = s;
                    improved = true;
                    break;
                }
            }
        }
    }
    return set;
}

}  // namespace

FF_EXPORT int ptune_postprocess(int nv, int ns, const double* t, double* best, double* worst, int* best_id,
                                double* slowdown, double* speedup)
{
    if (nv < 0 || ns < 0 || (nv * ns > 0 && t == nullptr) || (ns > 0 && (!best || !worst || !best_id)))
        return FF_ERR_ARG;
    std::vector<double> b;
    std::vector<int> bid;
    column_best(nv, ns, t, b, bid);
    for (int s = 0; s < ns; ++s) {
        double w = -kInf;
        for (int v = 0; v < nv; ++v) {
            const double x = t[(int64_t)v * ns + s];
            if (finite_pos(x)) w = std::max(w, x);
        }
        best[s] = b[s];
        best_id[s] = bid[s];
        worst[s] = bid[s] >= 0 ? w : kInf;
    }
    for (int v = 0; v < nv; ++v)
        for (int s = 0; s < ns; ++s) {
            const int64_t i = (int64_t)v * ns + s;
            const double x = t[i];
            const bool ok = finite_pos(x) && bid[s] >= 0;
            if (slowdown) slowdown[i] = ok ? x / b[s] : kInf;
            if (speedup) speedup[i] = ok ? worst[s] / x : 0.0;
        }
    return FF_OK;
}

FF_EXPORT int ptune_cost(int nv, int ns, const double* t, int k, const int* kappa, int nsel, const int* shapes,
                         double* cost)
{
    std::vector<int> sel;
    if (nv <= 0 || ns <= 0 || t == nullptr || k < 1 || kappa == nullptr || cost == nullptr ||
        !selection(ns, nsel, shapes, sel))
        return FF_ERR_ARG;
    for (int i = 0; i < k; ++i)
        if (kappa[i] < 0 || kappa[i] >= nv) return FF_ERR_ARG;
    const LogTable lt = make_log_table(nv, ns, t, sel);
    *cost = lt.ok ? cost_of(lt, set_logsum(lt, kappa, k)) : kInf;
    return FF_OK;
}

namespace {

// Minimise the summed per-shape minimum of lt over sets of kk variants.
std::vector<int> search(const LogTable& lt, int nv, int kk, int method, int64_t& evals)
{
    std::vector<int> cand = undominated(lt);
    std::vector<int> result;
    evals = 0;
    if ((int)cand.size() <= kk) {
        // Every undominated variant fits; fill up with the lowest other ids.
        result = cand;
        for (int v = 0; v < nv && (int)result.size() < kk; ++v)
            if (std::find(result.begin(), result.end(), v) == result.end()) result.push_back(v);
        evals = 1;
    } else {
        const int64_t cap = 200000000;
        const bool exhaustive =
            method == 0 || (method == -1 && n_choose_k_capped((int64_t)cand.size(), kk, cap) <= cap);
        if (exhaustive) {
            Exhaustive ex(lt, cand, kk);
            ex.run(0, 0);
            result = ex.best_set.empty() ? std::vector<int>(cand.begin(), cand.begin() + kk) : ex.best_set;
            evals = ex.evals;
        } else {
            result = greedy_swap(lt, cand, kk, evals);
            for (int v = 0; v < nv && (int)result.size() < kk; ++v)
                if (std::find(result.begin(), result.end(), v) == result.end()) result.push_back(v);
        }
    }
    std::sort(result.begin(), result.end());
    return result;
}

}  // namespace

FF_EXPORT int ptune_select(int nv, int ns, const double* t, int nsel, const int* shapes, int k, int method,
                           int* kappa_out, double* cost_out, int64_t* evals_out)
{
    std::vector<int> sel;
    if (nv <= 0 || ns <= 0 || t == nullptr || k < 1 || kappa_out == nullptr || method < -1 || method > 1 ||
        !selection(ns, nsel, shapes, sel))
        return FF_ERR_ARG;
    const int kk = std::min(k, nv);
    const LogTable lt = make_log_table(nv, ns, t, sel);
    int64_t evals = 0;
    const std::vector<int> result = search(lt, nv, kk, method, evals);
    for (int i = 0; i < kk; ++i) kappa_out[i] = result[i];
    if (cost_out) *cost_out = lt.ok ? cost_of(lt, set_logsum(lt, result.data(), kk)) : kInf;
    if (evals_out) *evals_out = evals;
    return kk;
}

FF_EXPORT int ptune_select_total(int nv, int ns, const double* t, int nsel, const int* shapes,
                                 const double* weights, int k, int method, int* kappa_out, double* total_out,
                                 int64_t* evals_out)
{
    std::vector<int> sel;
    if (nv <= 0 || ns <= 0 || t == nullptr || weights == nullptr || k < 1 || kappa_out == nullptr ||
        method < -1 || method > 1 || !selection(ns, nsel, shapes, sel))
        return FF_ERR_ARG;
    for (size_t j = 0; j < sel.size(); ++j)
        if (!(weights[j] > 0.0) || !std::isfinite(weights[j])) return FF_ERR_ARG;
    const int kk = std::min(k, nv);
    const LogTable lt = make_time_table(nv, ns, t, sel, weights);
    int64_t evals = 0;
    const std::vector<int> result = search(lt, nv, kk, method, evals);
    for (int i = 0; i < kk; ++i) kappa_out[i] = result[i];
    if (total_out) *total_out = lt.ok ? set_logsum(lt, result.data(), kk) : kInf;
    if (evals_out) *evals_out = evals;
    return kk;
}

namespace {

// Relative performance vectors best_s / t[v][s] (0 where failed), one per
// selected shape, best over all nv variants.
std::vector<std::vector<double>> perf_vectors(int nv, int ns, const double* t, const std::vector<int>& sel)
{
    std::vector<double> best;
    std::vector<int> bid;
    column_best(nv, ns, t, best, bid);
    std::vector<std::vector<double>> p(sel.size(), std::vector<double>(nv, 0.0));
    for (size_t j = 0; j < sel.size(); ++j)
        for (int v = 0; v < nv; ++v) {
            const double x = t[(int64_t)v * ns + sel[j]];
            if (finite_pos(x) && bid[sel[j]] >= 0) p[j][v] = best[sel[j]] / x;
        }
    return p;
}

// The best variant of each representative vector; a variant already taken
// is replaced by that vector's next best.  Sorted, at most k.
// Each representative's variant (largest component, lowest id on ties; a
// variant already taken goes to the representative's next best), in
// representative order, until k are chosen.
std::vector<int> pick_each(const std::vector<std::vector<double>>& reps, int k, int nv)
{
    std::vector<int> chosen;
    for (const auto& vec : reps) {
        std::vector<int> order(nv);
        for (int v = 0; v < nv; ++v) order[v] = v;
        std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return vec[a] > vec[b]; });
        for (int v : order)
            if (std::find(chosen.begin(), chosen.end(), v) == chosen.end()) {
                chosen.push_back(v);
                break;
            }
        if ((int)chosen.size() == k) break;
    }
    return chosen;
}

std::vector<int> pick_distinct(const std::vector<std::vector<double>>& reps, int k, int nv)
{
    std::vector<int> chosen = pick_each(reps, k, nv);
    std::sort(chosen.begin(), chosen.end());
    return chosen;
}

double sq_dist(const std::vector<double>& a, const std::vector<double>& b)
{
    double d = 0.0;
    for (size_t i = 0; i < a.size(); ++i) d += (a[i] - b[i]) * (a[i] - b[i]);
    return d;
}

}  // namespace

FF_EXPORT int ptune_kmeans(int nv, int ns, const double* t, int nsel, const int* shapes, int k, const int* init,
                           int max_iter, int* kappa_out, int* assign_out, int* iters_out)
{
    std::vector<int> sel;
    if (nv <= 0 || ns <= 0 || t == nullptr || k < 1 || init == nullptr || kappa_out == nullptr || max_iter < 1 ||
        !selection(ns, nsel, shapes, sel))
        return FF_ERR_ARG;
    const int np = (int)sel.size();
    for (int j = 0; j < k; ++j)
        if (init[j] < 0 || init[j] >= np) return FF_ERR_ARG;
    const auto pts = perf_vectors(nv, ns, t, sel);
    std::vector<std::vector<double>> cents;
    for (int j = 0; j < k; ++j) cents.push_back(pts[init[j]]);
    std::vector<int> assign(np, -1);
    int it = 0;
    for (it = 1; it <= max_iter; ++it) {
        bool changed = false;
        for (int i = 0; i < np; ++i) {
            int bj = 0;
            double bd = sq_dist(pts[i], cents[0]);
            for (int j = 1; j < k; ++j) {
                const double d = sq_dist(pts[i], cents[j]);
                if (d < bd) {
                    bd = d;
                    bj = j;
                }
            }
            if (bj != assign[i]) changed = true;
            assign[i] = bj;
        }
        for (int j = 0; j < k; ++j) {
            std::vector<double> mean(nv, 0.0);
            int cnt = 0;
            for (int i = 0; i < np; ++i)
                if (assign[i] == j) {
                    ++cnt;
                    for (int v = 0; v < nv; ++v) mean[v] += pts[i][v];
                }
            if (cnt > 0) {
                for (int v = 0; v < nv; ++v) mean[v] /= cnt;
                cents[j] = mean;
            }
        }
        if (!changed) break;
    }
    if (it > max_iter) it = max_iter;
    const std::vector<int> kap = pick_distinct(cents, k, nv);
    for (size_t i = 0; i < kap.size(); ++i) kappa_out[i] = kap[i];
    if (assign_out)
        for (int i = 0; i < np; ++i) assign_out[i] = assign[i];
    if (iters_out) *iters_out = it;
    return (int)kap.size();
}

namespace {

double leaf_sse(const std::vector<std::vector<double>>& pts, const std::vector<int>& idx, int nv)
{
    if (idx.empty()) return 0.0;
    std::vector<double> mean(nv, 0.0);
    for (int i : idx)
        for (int v = 0; v < nv; ++v) mean[v] += pts[i][v];
    for (int v = 0; v < nv; ++v) mean[v] /= (double)idx.size();
    double s = 0.0;
    for (int i : idx)
        for (int v = 0; v < nv; ++v) s += (pts[i][v] - mean[v]) * (pts[i][v] - mean[v]);
    return s;
}

struct Split {
    bool ok = false;
    double gain = 0.0;
    int f = -1;          // feature and threshold: x[f] <= thr goes left
    double thr = 0.0;
    std::vector<int> left, right;
};

Split best_split(const std::vector<std::vector<double>>& pts, const std::vector<int>& idx, int nv, int nf,
                 const double* feat)
{
    Split b;
    const double base = leaf_sse(pts, idx, nv);
    for (int f = 0; f < nf; ++f) {
        std::vector<double> vals;
        for (int i : idx) vals.push_back(feat[(size_t)i * nf + f]);
        std::sort(vals.begin(), vals.end());
        vals.erase(std::unique(vals.begin(), vals.end()), vals.end());
        for (size_t a = 0; a + 1 < vals.size(); ++a) {
            const double thr = 0.5 * (vals[a] + vals[a + 1]);
            std::vector<int> l, r;
            for (int i : idx) (feat[(size_t)i * nf + f] <= thr ? l : r).push_back(i);
            const double gain = base - leaf_sse(pts, l, nv) - leaf_sse(pts, r, nv);
            if (!b.ok || gain > b.gain + 1e-12) {
                b.ok = true;
                b.gain = gain;
                b.f = f;
                b.thr = thr;
                b.left = l;
                b.right = r;
            }
        }
    }
    return b;
}

}  // namespace

FF_EXPORT int ptune_tree(int nv, int ns, const double* t, int nsel, const int* shapes, int nfeat,
                         const double* features, int k, int* kappa_out, int* leaf_out, int* node_feat,
                         double* node_thr, int* node_child, int* leaf_variant)
{
    std::vector<int> sel;
    if (nv <= 0 || ns <= 0 || t == nullptr || k < 1 || nfeat < 1 || features == nullptr || kappa_out == nullptr ||
        !selection(ns, nsel, shapes, sel))
        return FF_ERR_ARG;
    const auto pts = perf_vectors(nv, ns, t, sel);
    const int np = (int)pts.size();
    std::vector<std::vector<int>> leaves(1);
    for (int i = 0; i < np; ++i) leaves[0].push_back(i);
    // The tree: node 0 is the root; a split turns its leaf node into an
    // internal node with two new leaf nodes (left first).
    struct Node { int feat = -1; double thr = 0.0; int left = -1, right = -1; };
    std::vector<Node> nodes(1);
    std::vector<int> leaf_node(1, 0);
    while ((int)leaves.size() < k) {
        int bl = -1;
        Split bs;
        for (size_t li = 0; li < leaves.size(); ++li) {
            Split s = best_split(pts, leaves[li], nv, nfeat, features);
            if (s.ok && (bl < 0 || s.gain > bs.gain)) {
                bl = (int)li;
                bs = s;
            }
        }
        if (bl < 0) break;
        const int n = leaf_node[bl], a = (int)nodes.size(), b = a + 1;
        nodes.resize(nodes.size() + 2);
        nodes[n].feat = bs.f;
        nodes[n].thr = bs.thr;
        nodes[n].left = a;
        nodes[n].right = b;
        leaves[bl] = bs.left;
        leaves.insert(leaves.begin() + bl + 1, bs.right);
        leaf_node[bl] = a;
        leaf_node.insert(leaf_node.begin() + bl + 1, b);
    }
    std::vector<std::vector<double>> reps;
    for (const auto& idx : leaves) {
        std::vector<double> mean(nv, 0.0);
        for (int i : idx)
            for (int v = 0; v < nv; ++v) mean[v] += pts[i][v];
        for (int v = 0; v < nv; ++v) mean[v] /= (double)idx.size();
        reps.push_back(mean);
    }
    const std::vector<int> each = pick_each(reps, k, nv);
    std::vector<int> kap = each;
    std::sort(kap.begin(), kap.end());
    for (size_t i = 0; i < kap.size(); ++i) kappa_out[i] = kap[i];
    if (leaf_out)
        for (size_t li = 0; li < leaves.size(); ++li)
            for (int i : leaves[li]) leaf_out[i] = (int)li;
    if (node_feat && node_thr && node_child) {
        std::vector<int> leaf_of_node(nodes.size(), -1);
        for (size_t li = 0; li < leaf_node.size(); ++li) leaf_of_node[leaf_node[li]] = (int)li;
        for (size_t n = 0; n < nodes.size(); ++n) {
            node_feat[n] = nodes[n].feat;
            node_thr[n] = nodes[n].thr;
            node_child[2 * n] = nodes[n].feat >= 0 ? nodes[n].left : leaf_of_node[n];
            node_child[2 * n + 1] = nodes[n].feat >= 0 ? nodes[n].right : -1;
        }
    }
    if (leaf_variant)
        for (size_t li = 0; li < leaves.size(); ++li) leaf_variant[li] = li < each.size() ? each[li] : -1;
    return (int)kap.size();
}

FF_EXPORT int ptune_tree_route(int nnodes, const int* node_feat, const double* node_thr, const int* node_child,
                               int nfeat, const double* x)
{
    if (nnodes < 1 || node_feat == nullptr || node_thr == nullptr || node_child == nullptr || nfeat < 1 ||
        x == nullptr)
        return FF_ERR_ARG;
    int n = 0;
    for (int step = 0; step < nnodes; ++step) {
        const int f = node_feat[n];
        if (f < 0) return node_child[2 * n];
        if (f >= nfeat) return FF_ERR_ARG;
        const int next = x[f] <= node_thr[n] ? node_child[2 * n] : node_child[2 * n + 1];
        if (next <= n || next >= nnodes) return FF_ERR_ARG;   // children always follow their parent
        n = next;
    }
    return FF_ERR_ARG;
}

FF_EXPORT int ptune_assign(int nv, int ns, const double* t, int k, const int* kappa, int nsel, const int* shapes,
                           int* winners)
{
    std::vector<int> sel;
    if (nv <= 0 || ns <= 0 || t == nullptr || k < 1 || kappa == nullptr || winners == nullptr ||
        !selection(ns, nsel, shapes, sel))
        return FF_ERR_ARG;
    std::vector<int> members(kappa, kappa + k);
    for (int v : members)
        if (v < 0 || v >= nv) return FF_ERR_ARG;
    std::sort(members.begin(), members.end());
    for (size_t j = 0; j < sel.size(); ++j) {
        int bv = -1;
        double bt = kInf;
        for (int v : members) {
            const double x = t[(int64_t)v * ns + sel[j]];
            if (finite_pos(x) && x < bt) {
                bt = x;
                bv = v;
            }
        }
        winners[j] = bv;
    }
    return FF_OK;
}

namespace {

// L1 distances over log2 sizes (sizes below 1 count as 1) into d[0..ntrain).
// train_lg, when given, holds the training shapes' log2 sizes already computed.
void shape_distances(int ntrain, const int64_t* train_mnk, const double* train_lg, int64_t M, int64_t N, int64_t K,
                     double* d)
{
    const double q[3] = {ptune_log2_size(M), ptune_log2_size(N), ptune_log2_size(K)};
    for (int i = 0; i < ntrain; ++i) {
        double t[3];
        for (int c = 0; c < 3; ++c) t[c] = train_lg ? train_lg[3 * i + c] : ptune_log2_size(train_mnk[3 * i + c]);
        d[i] = std::fabs(q[0] - t[0]) + std::fabs(q[1] - t[1]) + std::fabs(q[2] - t[2]);
    }
}

}  // namespace

FF_EXPORT int ptune_nearest(int ntrain, const int64_t* train_mnk, int64_t M, int64_t N, int64_t K)
{
    if (ntrain < 1 || train_mnk == nullptr) return FF_ERR_ARG;
    std::vector<double> d(ntrain);
    shape_distances(ntrain, train_mnk, nullptr, M, N, K, d.data());
    int best = 0;
    for (int i = 1; i < ntrain; ++i)
        if (d[i] < d[best]) best = i;
    return best;
}

double ptune_log_wave_efficiency(int64_t groups, int cus)
{
    if (groups <= 0) return 0.0;
    const int64_t waves = (groups + cus - 1) / cus;
    return std::log((double)groups / (double)(waves * cus));
}

int ptune_dispatch_lw(int ntrain, const int64_t* train_mnk, const double* train_lg, int k, const int* members,
                      const double* cost, const double* lw_train, const double* lw_query, int64_t M, int64_t N,
                      int64_t K)
{
    // Distances on the stack for the usual small training sets (this runs on
    // every dispatched sgemm call).
    double dsmall[64];
    std::vector<double> dbig;
    double* d = dsmall;
    if (ntrain > 64) {
        dbig.resize(ntrain);
        d = dbig.data();
    }
    shape_distances(ntrain, train_mnk, train_lg, M, N, K, d);
    const double dmin = *std::min_element(d, d + ntrain);
    int bj = -1;
    double bs = kInf;
    for (int j = 0; j < k; ++j) {
        double sum = 0.0;
        for (int i = 0; i < ntrain; ++i) {
            if (d[i] > dmin + 1e-9) continue;
            const double corr = lw_train ? lw_train[(size_t)i * k + j] - lw_query[j] : 0.0;
            sum += cost[(size_t)i * k + j] + corr;
        }
        if (bj < 0 || sum < bs) {
            bj = j;
            bs = sum;
        }
    }
    if (bs == kInf) {
        // No member is finite on every nearest shape: the member that is
        // finite on the first nearest shape with the lowest cost there.
        int i0 = 0;
        while (d[i0] > dmin + 1e-9) ++i0;
        bj = 0;
        for (int j = 1; j < k; ++j)
            if (cost[(size_t)i0 * k + j] < cost[(size_t)i0 * k + bj]) bj = j;
    }
    return members[bj];
}

FF_EXPORT int ptune_dispatch(int ntrain, const int64_t* train_mnk, int k, const int* members, const double* cost,
                             const int64_t* groups_train, const int64_t* groups_query, int cus, int64_t M,
                             int64_t N, int64_t K)
{
    if (ntrain < 1 || train_mnk == nullptr || k < 1 || members == nullptr || cost == nullptr) return FF_ERR_ARG;
    const bool waves = groups_train != nullptr && groups_query != nullptr && cus >= 1;
    if (!waves) return ptune_dispatch_lw(ntrain, train_mnk, nullptr, k, members, cost, nullptr, nullptr, M, N, K);
    std::vector<double> lt((size_t)ntrain * k), lq(k);
    for (size_t x = 0; x < lt.size(); ++x) lt[x] = ptune_log_wave_efficiency(groups_train[x], cus);
    for (int j = 0; j < k; ++j) lq[j] = ptune_log_wave_efficiency(groups_query[j], cus);
    return ptune_dispatch_lw(ntrain, train_mnk, nullptr, k, members, cost, lt.data(), lq.data(), M, N, K);
}
