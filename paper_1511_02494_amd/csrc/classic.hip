// The paper's feature classifiers (Section 3.2.2, Tables 4 and 5): a CART
// decision tree with the Gini criterion and Gaussian naive Bayes over the
// twelve structural features.  Fitting is host code (a few thousand samples);
// inference for selection runs on the device.
//
// CART: a node splits on (feature j, threshold t), left x_j <= t.  Candidate
// thresholds lie between consecutive distinct values a < b of the node's
// samples, t = a/2 + b/2 (a if that rounding leaves [a, b)); children keep at
// least min_leaf samples.  Minimising the weighted Gini impurity equals
// maximising sum_k cL_k^2 / n_L + sum_k cR_k^2 / n_R, which is compared
// exactly in integers; the first maximum in (feature, threshold) order wins
// and a split must lower the impurity strictly.  Leaves: depth max_depth,
// pure nodes, nodes with fewer than 2 min_leaf samples, no qualifying split.
// Nodes are numbered in pre-order and keep their class counts; a prediction
// takes the feasible class with the largest leaf count (lowest on ties).
//
// Gaussian NB on g = (plog2(1 + f_k) for k < 8, f_k otherwise): per class,
// means and population variances (sums in sample order) plus 1e-9 times the
// largest feature variance over all samples; stored as mu, w = 0.5 / var and
// c = log(n_k / n) - 0.5 sum_j log(2 pi var_j).  Score
// s_k = c_k - sum_j w_kj (g_j - mu_kj)^2, every operation rounded separately;
// the feasible class with samples and the largest score wins.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <vector>

#include "dev.h"
#include "feat_acc.h"
#include "internal.h"

namespace spmvsel {
namespace {

constexpr int kNF = 12;
constexpr int kMaxClasses = 8;
constexpr int kMaxTreeDepth = 64;

struct F12 {
    double f[kNF];
};

double plog2_host(double v) {
    int e;
    const double m = frexp(v, &e);
    return (double)(e - 1) + (2.0 * m - 1.0);
}

void nb_inputs(const double *f, double *g) {
    for (int k = 0; k < kNF; ++k) g[k] = k < 8 ? plog2_host(1.0 + f[k]) : f[k];
}

// ---------------------------------------------------------------- CART fit
typedef __int128 i128;

// aL/nL + bL... : (a1/n1 + b1/m1) > (a2/n2 + b2/m2) for positive counts
bool q_greater(int64_t a1, int64_t n1, int64_t b1, int64_t m1, int64_t a2, int64_t n2, int64_t b2,
               int64_t m2) {
    const i128 lhs = ((i128)a1 * m1 + (i128)b1 * n1) * ((i128)n2 * m2);
    const i128 rhs = ((i128)a2 * m2 + (i128)b2 * n2) * ((i128)n1 * m1);
    return lhs > rhs;
}

struct TreeFit {
    const double *X;
    const int32_t *y;
    int C, max_depth, min_leaf, max_nodes;
    std::vector<int32_t> feature, left, right, counts;
    std::vector<double> thr;
    bool full = false;

    int grow(const std::vector<int32_t> &idx, int depth) {
        const int id = (int)feature.size();
        if (id >= max_nodes) {
            full = true;
            return -1;
        }
        const int64_t n = (int64_t)idx.size();
        std::vector<int64_t> c(C, 0);
        for (int32_t i : idx) ++c[y[i]];
        feature.push_back(-1);
        thr.push_back(0.0);
        left.push_back(-1);
        right.push_back(-1);
        for (int k = 0; k < C; ++k) counts.push_back((int32_t)c[k]);
        int present = 0;
        int64_t sq = 0;
        for (int k = 0; k < C; ++k) {
            present += c[k] > 0;
            sq += c[k] * c[k];
        }
        if (depth >= max_depth || n < 2 * (int64_t)min_leaf || present <= 1) return id;

        bool have = false;
        int64_t bA = 0, bL = 0, bB = 0, bR = 0;
        int bj = -1;
        double bt = 0.0;
        std::vector<int32_t> ord(idx);
        std::vector<int64_t> cl(C), cr(C);
        for (int j = 0; j < kNF; ++j) {
            std::sort(ord.begin(), ord.end(), [&](int32_t a, int32_t b) {
                const double va = X[(int64_t)a * kNF + j], vb = X[(int64_t)b * kNF + j];
                return va < vb || (va == vb && a < b);
            });
            std::fill(cl.begin(), cl.end(), 0);
            cr = c;
            int64_t A = 0, B = sq;
            for (int64_t p = 0; p + 1 < n; ++p) {
                const int k = y[ord[p]];
                A += 2 * cl[k] + 1;  // (c+1)^2 - c^2
                ++cl[k];
                B -= 2 * cr[k] - 1;  // c^2 - (c-1)^2
                --cr[k];
                const double a = X[(int64_t)ord[p] * kNF + j], b = X[(int64_t)ord[p + 1] * kNF + j];
                if (a == b) continue;
                const int64_t nl = p + 1, nr = n - p - 1;
                if (nl < min_leaf || nr < min_leaf) continue;
                if (!have || q_greater(A, nl, B, nr, bA, bL, bB, bR)) {
                    have = true;
                    bA = A, bL = nl, bB = B, bR = nr;
                    bj = j;
                    double t = a / 2.0 + b / 2.0;
                    if (!(a <= t && t < b)) t = a;
                    bt = t;
                }
            }
        }
        if (!have) return id;
        // the split must lower the impurity: Q > sum_k c_k^2 / n
        if (!(((i128)bA * bR + (i128)bB * bL) * n > (i128)sq * bL * bR)) return id;
        std::vector<int32_t> li, ri;
        li.reserve(bL);
        ri.reserve(bR);
        for (int32_t i : idx) (X[(int64_t)i * kNF + bj] <= bt ? li : ri).push_back(i);
        feature[id] = bj;
        thr[id] = bt;
        const int l = grow(li, depth + 1);
        if (l < 0) return -1;
        left[id] = l;
        const int r = grow(ri, depth + 1);
        if (r < 0) return -1;
        right[id] = r;
        return id;
    }
};

// ---------------------------------------------------------------- models
struct Classic {
    bool loaded = false;
    int n_classes = 0, label_kind = 0;
    // tree
    int n_nodes = 0;
    std::vector<int32_t> ints;   // feature | left | right | counts
    std::vector<double> dbls;    // threshold (tree) or mu | w | c (NB)
    std::vector<int32_t> count;  // NB class sample counts
    std::map<int, DevBuf *> dev;
};
std::mutex g_cmu;
Classic g_clf[2];

void drop_device(Classic &m) {
    for (auto &kv : m.dev) delete kv.second;
    m.dev.clear();
}

// device copy: ints (padded to 8 bytes) then doubles
spmv_status_t device_model(int which, const int32_t **di, const double **dd, Classic *snap) {
    int d = 0;
    SPMV_HIP(hipGetDevice(&d));
    std::lock_guard<std::mutex> lk(g_cmu);
    Classic &m = g_clf[which];
    if (!m.loaded)
        return fail(SPMV_ERR_NO_MODEL, "no %s model loaded", which == 0 ? "decision tree" : "naive Bayes");
    auto it = m.dev.find(d);
    const size_t ib = (m.ints.size() * 4 + 7) & ~(size_t)7;
    if (it == m.dev.end()) {
        DevBuf *b = new DevBuf();
        spmv_status_t st = b->alloc(ib + m.dbls.size() * 8 + 8);
        if (st != SPMV_OK) {
            delete b;
            return st;
        }
        hipError_t e = hipMemcpy(b->p, m.ints.data(), m.ints.size() * 4, hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = hipMemcpy(static_cast<char *>(b->p) + ib, m.dbls.data(), m.dbls.size() * 8,
                          hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            delete b;
            return fail_hip(e, "hipMemcpy(classifier)", __FILE__, __LINE__);
        }
        it = m.dev.emplace(d, b).first;
    }
    *di = it->second->as<int32_t>();
    *dd = reinterpret_cast<const double *>(static_cast<const char *>(it->second->p) + ib);
    snap->n_classes = m.n_classes;
    snap->label_kind = m.label_kind;
    snap->n_nodes = m.n_nodes;
    snap->count = m.count;
    return SPMV_OK;
}

}  // namespace

// ---------------------------------------------------------------- kernels
// out: int32 [label, leaf, fallback, pad], then double scores[kMaxClasses]

// The tree walk and decision for features x (one thread).
__device__ void tree_decide(const int32_t *__restrict__ ints, int n_nodes, int C,
                            const double *__restrict__ thr, const double *x, uint32_t feasible,
                            int32_t *__restrict__ out) {
    const int32_t *feat = ints, *lft = ints + n_nodes, *rgt = ints + 2 * n_nodes,
                  *cnt = ints + 3 * n_nodes;
    int node = 0;
    for (int steps = 0; steps < n_nodes && feat[node] >= 0; ++steps) {
        double v = 0.0;
        const int j = feat[node];
#pragma unroll
        for (int q = 0; q < kNF; ++q)
            if (q == j) v = x[q];
        node = v <= thr[node] ? lft[node] : rgt[node];
    }
    int best = -1, bc = 0;
    for (int k = 0; k < C; ++k) {
        const int v = cnt[node * C + k];
        if (((feasible >> k) & 1) && v > bc) {
            best = k;
            bc = v;
        }
    }
    out[0] = best < 0 ? 0 : best;
    out[1] = node;
    out[2] = best < 0;
}

// The class scores and decision for inputs g (all threads of the
// workgroup, C <= its size; ends with the decision written by thread 0).
__device__ void gnb_decide(const int32_t *__restrict__ count, const double *__restrict__ mu,
                           const double *__restrict__ w, const double *__restrict__ c, int C,
                           const double *g, uint32_t feasible, int32_t *__restrict__ out) {
    __shared__ double s[kMaxClasses];
    const int k = threadIdx.x;
    if (k < C) {
        double acc = 0.0;
        for (int j = 0; j < kNF; ++j) {
            const double d = g[j] - mu[k * kNF + j];
            acc = acc + w[k * kNF + j] * (d * d);
        }
        s[k] = count[k] > 0 ? c[k] - acc : -INFINITY;
    }
    __syncthreads();
    if (k == 0) {
        double *sc = reinterpret_cast<double *>(out + 4);
        int best = -1;
        for (int q = 0; q < C; ++q) {
            sc[q] = s[q];
            if (((feasible >> q) & 1) && count[q] > 0 && (best < 0 || s[q] > s[best])) best = q;
        }
        out[0] = best < 0 ? 0 : best;
        out[1] = -1;
        out[2] = best < 0;
    }
}

__global__ __launch_bounds__(64) void k_tree_infer(const int32_t *__restrict__ ints, int n_nodes,
                                                   int C, const double *__restrict__ thr, F12 x,
                                                   uint32_t feasible, int32_t *__restrict__ out) {
    if (threadIdx.x != 0) return;
    tree_decide(ints, n_nodes, C, thr, x.f, feasible, out);
}

__global__ __launch_bounds__(64) void k_gnb_infer(const int32_t *__restrict__ count,
                                                  const double *__restrict__ mu,
                                                  const double *__restrict__ w,
                                                  const double *__restrict__ c, int C, F12 g,
                                                  uint32_t feasible, int32_t *__restrict__ out) {
    gnb_decide(count, mu, w, c, C, g.f, feasible, out);
}

// One-pass selection with classifier `which` (0 tree, 1 NB): the features,
// feasibility and record from the selection kernel's partials (as for the
// MLP), then the classifier on the device.  Class labels (label_variants 0)
// take every class as feasible; the host maps the class to a variant.
// out: the classifier record above in bytes 0..79, then the common part.
__global__ __launch_bounds__(64) void k_classic_select(int which, const int32_t *__restrict__ ints,
                                                       int n_nodes, const double *__restrict__ dd,
                                                       int C, int label_variants,
                                                       const uint64_t *__restrict__ partials,
                                                       int nparts, int64_t n, int64_t m,
                                                       int64_t nnz, int vb, int xb, int two_heights,
                                                       uint32_t feas_base, char *__restrict__ out) {
    __shared__ uint64_t w[16];
    __shared__ double f[kNF], g[kNF];
    __shared__ uint32_t feas;
    feat::select_prologue(nparts, partials, n, m, nnz, vb, xb, two_heights, feas_base, w, f, &feas);
    if (threadIdx.x == 0) feat::select_store_common(out, f, feas, w);
    const uint32_t lab_feas = label_variants ? feas : 0xFu;
    int32_t *o = reinterpret_cast<int32_t *>(out);
    if (which == 0) {
        if (threadIdx.x == 0) tree_decide(ints, n_nodes, C, dd, f, lab_feas, o);
    } else {
        if (threadIdx.x < kNF) g[threadIdx.x] = threadIdx.x < 8 ? feat::plog2(1.0 + f[threadIdx.x]) : f[threadIdx.x];
        __syncthreads();
        gnb_decide(ints, dd, dd + C * kNF, dd + 2 * C * kNF, C, g, lab_feas, o);
    }
}

namespace {

// Device inference of classifier `which` (0 tree, 1 NB).  `feas` is the
// feasible-variant mask; class labels map to variants through Table 2.
spmv_status_t classic_run(int which, const double f[12], uint32_t feas, const double th[4],
                          hipStream_t s, int32_t *d_out, int32_t *variant, int32_t *label,
                          int32_t *fallback, int32_t *leaf, double *scores) {
    const int32_t *di;
    const double *dd;
    Classic m;
    SPMV_TRY(device_model(which, &di, &dd, &m));
    const uint32_t lab_feas = m.label_kind == 0 ? feas : 0xFu;
    F12 x;
    if (which == 0) {
        memcpy(x.f, f, sizeof x.f);
        hipLaunchKernelGGL(k_tree_infer, dim3(1), dim3(64), 0, s, di, m.n_nodes, m.n_classes, dd, x,
                           lab_feas, d_out);
    } else {
        nb_inputs(f, x.f);
        const int C = m.n_classes;
        hipLaunchKernelGGL(k_gnb_infer, dim3(1), dim3(64), 0, s, di, dd, dd + C * kNF,
                           dd + 2 * C * kNF, C, x, lab_feas, d_out);
    }
    SPMV_HIP(hipGetLastError());
    int32_t h[4 + 2 * kMaxClasses];
    SPMV_HIP(hipMemcpyAsync(h, d_out, sizeof h, hipMemcpyDeviceToHost, s));
    SPMV_HIP(hipStreamSynchronize(s));
    const int lab = h[0];
    if (label) *label = lab;
    if (fallback) *fallback = h[2];
    if (leaf) *leaf = h[1];
    if (scores) {
        for (int k = 0; k < kMaxClasses; ++k) scores[k] = 0.0;
        if (which == 1) memcpy(scores, h + 4, (size_t)m.n_classes * 8);
    }
    if (variant) *variant = m.label_kind == 0 ? lab : class_variant(lab, f, th, feas);
    return SPMV_OK;
}

}  // namespace

bool classic_loaded(int which) {
    std::lock_guard<std::mutex> lk(g_cmu);
    return g_clf[which].loaded;
}

spmv_status_t classic_select_launch(int which, const uint64_t *d_partials, int nparts, int64_t n,
                                    int64_t m, int64_t nnz, int vb, int xb, int two_heights,
                                    uint32_t feas_base, void *out, hipStream_t s,
                                    int *label_kind) {
    const int32_t *di;
    const double *dd;
    Classic snap;
    SPMV_TRY(device_model(which, &di, &dd, &snap));
    *label_kind = snap.label_kind;
    hipLaunchKernelGGL(k_classic_select, dim3(1), dim3(64), 0, s, which, di, snap.n_nodes,
                       dd, snap.n_classes, snap.label_kind == 0 ? 1 : 0, d_partials, nparts, n, m,
                       nnz, vb, xb, two_heights, feas_base, static_cast<char *>(out));
    SPMV_HIP(hipGetLastError());
    return SPMV_OK;
}

spmv_status_t classic_predict(int which, const double f[12], uint32_t feas, const double th[4],
                              hipStream_t s, void *d_out, int32_t *variant, int32_t *label,
                              int32_t *fallback) {
    return classic_run(which, f, feas, th, s, static_cast<int32_t *>(d_out), variant, label,
                       fallback, nullptr, nullptr);
}

}  // namespace spmvsel

using namespace spmvsel;

extern "C" {

spmv_status_t spmv_dtree_fit(const double *X, const int32_t *y, int64_t n, int32_t n_classes,
                             int32_t max_depth, int32_t min_leaf, int32_t max_nodes,
                             int32_t *feature, double *threshold, int32_t *left, int32_t *right,
                             int32_t *counts, int32_t *n_nodes) {
    clear_error();
    if (!X || !y || !feature || !threshold || !left || !right || !counts || !n_nodes)
        return fail(SPMV_ERR_ARG, "NULL argument");
    if (n < 1 || n > (1 << 24) || n_classes < 1 || n_classes > kMaxClasses || max_depth < 0 ||
        max_depth > kMaxTreeDepth || min_leaf < 1 || max_nodes < 1)
        return fail(SPMV_ERR_ARG, "bad tree parameters");
    for (int64_t i = 0; i < n; ++i)
        if (y[i] < 0 || y[i] >= n_classes) return fail(SPMV_ERR_ARG, "label %d out of range", y[i]);
    for (int64_t i = 0; i < n * kNF; ++i)
        if (!(X[i] == X[i])) return fail(SPMV_ERR_ARG, "NaN feature");
    TreeFit T{X, y, n_classes, max_depth, min_leaf, max_nodes, {}, {}, {}, {}, {}, false};
    std::vector<int32_t> idx(n);
    for (int64_t i = 0; i < n; ++i) idx[i] = (int32_t)i;
    T.grow(idx, 0);
    if (T.full) return fail(SPMV_ERR_ARG, "the tree needs more than %d nodes", max_nodes);
    const int nn = (int)T.feature.size();
    memcpy(feature, T.feature.data(), (size_t)nn * 4);
    memcpy(threshold, T.thr.data(), (size_t)nn * 8);
    memcpy(left, T.left.data(), (size_t)nn * 4);
    memcpy(right, T.right.data(), (size_t)nn * 4);
    memcpy(counts, T.counts.data(), (size_t)nn * n_classes * 4);
    *n_nodes = nn;
    return SPMV_OK;
}

spmv_status_t spmv_gnb_fit(const double *F, const int32_t *y, int64_t n, int32_t n_classes,
                           double *mu, double *w, double *c, int32_t *count) {
    clear_error();
    if (!F || !y || !mu || !w || !c || !count) return fail(SPMV_ERR_ARG, "NULL argument");
    if (n < 1 || n_classes < 1 || n_classes > kMaxClasses) return fail(SPMV_ERR_ARG, "bad sizes");
    for (int64_t i = 0; i < n; ++i)
        if (y[i] < 0 || y[i] >= n_classes) return fail(SPMV_ERR_ARG, "label %d out of range", y[i]);
    std::vector<double> G((size_t)n * kNF);
    for (int64_t i = 0; i < n; ++i) nb_inputs(F + i * kNF, &G[(size_t)i * kNF]);
    double vmax = 0.0;
    for (int j = 0; j < kNF; ++j) {
        double sum = 0.0;
        for (int64_t i = 0; i < n; ++i) sum = sum + G[(size_t)i * kNF + j];
        const double m = sum / (double)n;
        double q = 0.0;
        for (int64_t i = 0; i < n; ++i) {
            const double t = G[(size_t)i * kNF + j] - m;
            q = q + t * t;
        }
        vmax = std::max(vmax, q / (double)n);
    }
    const double eps = 1e-9 * vmax;
    for (int k = 0; k < n_classes; ++k) {
        int64_t nk = 0;
        for (int64_t i = 0; i < n; ++i) nk += y[i] == k;
        count[k] = (int32_t)nk;
        c[k] = 0.0;
        for (int j = 0; j < kNF; ++j) mu[k * kNF + j] = w[k * kNF + j] = 0.0;
        if (nk == 0) continue;
        double logvar = 0.0;
        for (int j = 0; j < kNF; ++j) {
            double sum = 0.0;
            for (int64_t i = 0; i < n; ++i)
                if (y[i] == k) sum = sum + G[(size_t)i * kNF + j];
            const double m = sum / (double)nk;
            double q = 0.0;
            for (int64_t i = 0; i < n; ++i)
                if (y[i] == k) {
                    const double t = G[(size_t)i * kNF + j] - m;
                    q = q + t * t;
                }
            const double var = q / (double)nk + eps;
            mu[k * kNF + j] = m;
            w[k * kNF + j] = 0.5 / var;
            logvar = logvar + log(2.0 * M_PI * var);
        }
        c[k] = log((double)nk / (double)n) - 0.5 * logvar;
    }
    return SPMV_OK;
}

spmv_status_t spmv_dtree_load(int32_t n_nodes, int32_t n_classes, int32_t label_kind,
                              const int32_t *feature, const double *threshold, const int32_t *left,
                              const int32_t *right, const int32_t *counts) {
    clear_error();
    if (!feature || !threshold || !left || !right || !counts) return fail(SPMV_ERR_ARG, "NULL argument");
    if (n_nodes < 1 || n_classes < 1 || n_classes > kMaxClasses || (label_kind != 0 && label_kind != 1) ||
        (label_kind == 1 && n_classes != 4) || (label_kind == 0 && n_classes != SPMV_N_VARIANTS))
        return fail(SPMV_ERR_ARG, "bad tree header");
    // structure: pre-order children (i < child < n), features in range, so a
    // walk from the root ends within n steps
    for (int i = 0; i < n_nodes; ++i) {
        if (feature[i] < -1 || feature[i] >= kNF) return fail(SPMV_ERR_ARG, "node %d: bad feature", i);
        if (feature[i] >= 0 && (left[i] <= i || left[i] >= n_nodes || right[i] <= i ||
                                right[i] >= n_nodes || !(threshold[i] == threshold[i])))
            return fail(SPMV_ERR_ARG, "node %d: bad children or threshold", i);
        for (int k = 0; k < n_classes; ++k)
            if (counts[(int64_t)i * n_classes + k] < 0) return fail(SPMV_ERR_ARG, "negative count");
    }
    std::lock_guard<std::mutex> lk(g_cmu);
    Classic &m = g_clf[0];
    drop_device(m);
    m.n_nodes = n_nodes;
    m.n_classes = n_classes;
    m.label_kind = label_kind;
    m.ints.assign(feature, feature + n_nodes);
    m.ints.insert(m.ints.end(), left, left + n_nodes);
    m.ints.insert(m.ints.end(), right, right + n_nodes);
    m.ints.insert(m.ints.end(), counts, counts + (int64_t)n_nodes * n_classes);
    m.dbls.assign(threshold, threshold + n_nodes);
    m.loaded = true;
    return SPMV_OK;
}

spmv_status_t spmv_gnb_load(int32_t n_classes, int32_t label_kind, const double *mu,
                            const double *w, const double *c, const int32_t *count) {
    clear_error();
    if (!mu || !w || !c || !count) return fail(SPMV_ERR_ARG, "NULL argument");
    if (n_classes < 1 || n_classes > kMaxClasses || (label_kind != 0 && label_kind != 1) ||
        (label_kind == 1 && n_classes != 4) || (label_kind == 0 && n_classes != SPMV_N_VARIANTS))
        return fail(SPMV_ERR_ARG, "bad naive Bayes header");
    for (int k = 0; k < n_classes; ++k)
        if (count[k] < 0) return fail(SPMV_ERR_ARG, "negative count");
    std::lock_guard<std::mutex> lk(g_cmu);
    Classic &m = g_clf[1];
    drop_device(m);
    m.n_classes = n_classes;
    m.label_kind = label_kind;
    m.ints.assign(count, count + n_classes);
    m.count = m.ints;
    m.dbls.assign(mu, mu + n_classes * kNF);
    m.dbls.insert(m.dbls.end(), w, w + n_classes * kNF);
    m.dbls.insert(m.dbls.end(), c, c + n_classes);
    m.loaded = true;
    return SPMV_OK;
}

spmv_status_t spmv_classifier_unload(int32_t which) {
    clear_error();
    if (which != SPMV_CLF_DTREE && which != SPMV_CLF_GNB) return fail(SPMV_ERR_ARG, "unknown classifier");
    std::lock_guard<std::mutex> lk(g_cmu);
    drop_device(g_clf[which]);
    g_clf[which] = Classic();
    return SPMV_OK;
}

spmv_status_t spmv_classifier_predict(int32_t which, const double features[12], uint32_t feasible,
                                      int32_t *variant, int32_t *label, int32_t *fallback,
                                      int32_t *leaf, double scores[8]) {
    clear_error();
    if (which != SPMV_CLF_DTREE && which != SPMV_CLF_GNB) return fail(SPMV_ERR_ARG, "unknown classifier");
    if (!features) return fail(SPMV_ERR_ARG, "NULL features");
    double th[4];
    spmv_get_thresholds(th);
    DevBuf out;
    SPMV_TRY(out.alloc(256));
    return classic_run(which, features, feasible, th, nullptr, out.as<int32_t>(), variant, label,
                       fallback, leaf, scores);
}

}  // extern "C"
