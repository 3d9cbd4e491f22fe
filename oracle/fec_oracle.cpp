// CPU oracle for fixed-radius Euclidean clustering (FEC, arXiv 2208.07678).
//
// TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, single-threaded
// reference that the GPU path is checked against.  Only the tests, the
// package smoke check and the benchmark's CPU-baseline leg load it; the
// product path never does.  It shares no code, header or constant table with
// the GPU library.
//
// What it computes (the paper's clustering, Sec. 2.2 Eq. (1) and Alg. 1):
//   * edge predicate E(i,j): the strict "closer than d" test of Eq. (1),
//     evaluated in IEEE binary32 with the fixed order
//        s = fl(fl(fl(dx*dx) + fl(dy*dy)) + fl(dz*dz)),  E <=> s < fl(d*d)
//     with dx = fl(x_i - x_j) etc. (no contraction; built -ffp-contract=off);
//   * the point-wise main loop of Alg. 1: visit points in index order, query
//     the neighbours within d (a kd-tree replaces the paper's kd-tree radius
//     search one for one), take the smallest non-zero label among them (or a
//     fresh segment label), give it to unlabelled neighbours and relabel
//     every point that carries a larger neighbour label (the segment-merge
//     loop);
//   * the output convention of the GPU boundary: labels canonicalised to the
//     smallest point index of each cluster, clusters outside
//     [min_size, max_size] set to -1.
//
// Readings of the paper taken where it is silent or ambiguous:
//   - every point is visited, including already-labelled ones (the printed
//     "only if unlabelled" test splits some clusters, see the 4-point chain
//     test);
//   - the neighbour cap Th_max is unlimited (a capped variant, which keeps
//     the Th_max nearest neighbours of p_i besides p_i itself, ties by index,
//     exists for measuring its effect only);
//   - unlabelled neighbours receive the minimum label (the printed merge
//     loop only handles larger labels, which would leave every label 0);
//   - the neighbour set of p_i contains p_i itself;
//   - non-finite points have no neighbours (every comparison is false).
//
// The segment-merge loop of Alg. 1 rescans all points to relabel one label.
// Here each label value owns a member list and the smaller list is moved
// into the larger one; the label value every point carries after every step
// is the same as with the full rescan (the literal rescan is kept behind a
// flag and a test compares the two after every step).

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <limits>
#include <new>
#include <vector>

namespace {

// ---------------------------------------------------------------- predicate
// Eq. (1): two points are in one cluster when their distance is below d.
inline bool linked(const float *a, const float *b, float d2) {
    float dx = a[0] - b[0];
    float dy = a[1] - b[1];
    float dz = a[2] - b[2];
    float sx = dx * dx;
    float sy = dy * dy;
    float sz = dz * dz;
    float s = sx + sy;
    s = s + sz;
    return s < d2;
}

inline bool finite3(const float *p) {
    return std::isfinite(p[0]) && std::isfinite(p[1]) && std::isfinite(p[2]);
}

// ---------------------------------------------------------------- kd-tree
// Median-split kd-tree over the finite points (Alg. 1, "Constructing
// kd-tree").  A subtree is pruned when the squared distance from the query
// to its bounding box (double) is at least (d * (1 + 2^-10))^2, which cannot
// drop a pair the binary32 predicate accepts: that predicate only accepts
// pairs whose true distance is below d * (1 + 2^-22).
struct KdTree {
    struct Node {
        float lo[3], hi[3];
        int64_t begin, end;
        int64_t left, right;  // -1 for leaves
    };
    static constexpr int64_t kLeaf = 12;

    const float *xyz = nullptr;
    int64_t n = 0;
    float d2 = 0.f;
    double rc2 = 0.0;
    std::vector<int64_t> idx;   // point indices in leaf order
    std::vector<float> pts;     // their coordinates, same order
    std::vector<Node> nodes;

    KdTree(const float *xyz_, int64_t n_, float d) : xyz(xyz_), n(n_) {
        d2 = d * d;
        double rc = (double)d * (1.0 + std::ldexp(1.0, -10));
        rc2 = rc * rc;
        idx.reserve(n);
        for (int64_t i = 0; i < n; ++i)
            if (finite3(xyz + 3 * i)) idx.push_back(i);
        if (!idx.empty()) {
            nodes.reserve(2 * (idx.size() / kLeaf + 1) + 1);
            build(0, (int64_t)idx.size());
        }
        pts.resize(3 * idx.size());
        for (size_t k = 0; k < idx.size(); ++k)
            std::memcpy(&pts[3 * k], xyz + 3 * idx[k], 3 * sizeof(float));
    }

    int64_t build(int64_t b, int64_t e) {
        Node nd;
        for (int a = 0; a < 3; ++a) {
            nd.lo[a] = std::numeric_limits<float>::infinity();
            nd.hi[a] = -std::numeric_limits<float>::infinity();
        }
        for (int64_t k = b; k < e; ++k) {
            const float *p = xyz + 3 * idx[k];
            for (int a = 0; a < 3; ++a) {
                nd.lo[a] = std::min(nd.lo[a], p[a]);
                nd.hi[a] = std::max(nd.hi[a], p[a]);
            }
        }
        nd.begin = b;
        nd.end = e;
        nd.left = nd.right = -1;
        int64_t id = (int64_t)nodes.size();
        nodes.push_back(nd);
        if (e - b > kLeaf) {
            int ax = 0;
            float ext = -1.f;
            for (int a = 0; a < 3; ++a) {
                float w = nd.hi[a] - nd.lo[a];
                if (w > ext) { ext = w; ax = a; }
            }
            int64_t m = b + (e - b) / 2;
            const float *base = xyz;
            std::nth_element(idx.begin() + b, idx.begin() + m, idx.begin() + e,
                             [base, ax](int64_t u, int64_t v) {
                                 return base[3 * u + ax] < base[3 * v + ax];
                             });
            int64_t l = build(b, m);
            int64_t r = build(m, e);
            nodes[id].left = l;
            nodes[id].right = r;
        }
        return id;
    }

    // Calls f(j) for every indexed (finite) point j with E(q, p_j).  When q
    // is itself an indexed point it is reported too (distance 0 < d).
    template <class F>
    void radius(const float *q, F &&f) const {
        if (nodes.empty() || !finite3(q)) return;
        int64_t stack[128];
        int sp = 0;
        stack[sp++] = 0;
        while (sp > 0) {
            const Node &nd = nodes[stack[--sp]];
            double s = 0.0;
            for (int a = 0; a < 3; ++a) {
                double v = 0.0;
                if (q[a] < nd.lo[a]) v = (double)nd.lo[a] - (double)q[a];
                else if (q[a] > nd.hi[a]) v = (double)q[a] - (double)nd.hi[a];
                s += v * v;
            }
            if (s >= rc2) continue;
            if (nd.left < 0) {
                for (int64_t k = nd.begin; k < nd.end; ++k)
                    if (linked(q, &pts[3 * k], d2)) f(idx[k]);
            } else {
                stack[sp++] = nd.right;
                stack[sp++] = nd.left;
            }
        }
    }
};

// ---------------------------------------------------------------- Alg. 1
enum : int32_t { kLiteralScan = 1, kSkipLabelled = 2 };

// Binary32 squared distance in the predicate's order (for the capped
// variant's nearest-first choice).
inline float sq_dist(const float *p, const float *q) {
    const float ex = p[0] - q[0], ey = p[1] - q[1], ez = p[2] - q[2];
    const float t = ex * ex + ey * ey;
    return t + ez * ez;
}

// Runs the point-wise loop over points 0..steps-1 and writes the label
// value (0 = unlabelled, segment labels from 1) of every point.  th_max > 0
// caps FindNeighbor at the th_max nearest neighbours besides p_i.
void fec_loop(const float *xyz, int64_t n, float d, int64_t steps, int32_t flags,
              int64_t *lab_out, int64_t th_max = 0) {
    KdTree tree(xyz, n, d);
    const bool literal = (flags & kLiteralScan) != 0;
    const bool skip = (flags & kSkipLabelled) != 0;

    // label bookkeeping: point -> set, set -> label value, value -> set
    std::vector<int64_t> set_of(n, -1);
    std::vector<int64_t> val;                       // per set
    std::vector<std::vector<int64_t>> members;      // per set
    std::vector<int64_t> set_of_value(n + 2, -1);   // per label value
    std::vector<int64_t> lab(literal ? n : 0, 0);   // literal mode only

    auto label = [&](int64_t p) -> int64_t {
        if (literal) return lab[p];
        int64_t s = set_of[p];
        return s < 0 ? 0 : val[s];
    };
    auto assign = [&](int64_t p, int64_t m) {  // p unlabelled -> label m
        if (literal) { lab[p] = m; return; }
        int64_t s = set_of_value[m];
        if (s < 0) {
            s = (int64_t)val.size();
            val.push_back(m);
            members.emplace_back();
            set_of_value[m] = s;
        }
        set_of[p] = s;
        members[s].push_back(p);
    };
    auto relabel = [&](int64_t from, int64_t to) {  // every label `from` -> `to`
        if (literal) {
            for (int64_t k = 0; k < n; ++k)
                if (lab[k] == from) lab[k] = to;
            return;
        }
        int64_t a = set_of_value[from];
        int64_t b = set_of_value[to];
        if (b < 0) {  // `to` has no member yet: the set simply takes the value
            val[a] = to;
            set_of_value[to] = a;
            set_of_value[from] = -1;
            return;
        }
        if (members[a].size() > members[b].size()) std::swap(a, b);
        for (int64_t p : members[a]) set_of[p] = b;
        members[b].insert(members[b].end(), members[a].begin(), members[a].end());
        std::vector<int64_t>().swap(members[a]);
        val[b] = to;
        set_of_value[to] = b;
        set_of_value[from] = -1;
    };

    int64_t seg = 1;
    std::vector<int64_t> nn;
    for (int64_t i = 0; i < steps; ++i) {
        if (skip && label(i) != 0) continue;
        nn.clear();
        nn.push_back(i);
        tree.radius(xyz + 3 * i, [&](int64_t j) { if (j != i) nn.push_back(j); });
        if (th_max > 0 && (int64_t)nn.size() - 1 > th_max) {
            const float *q = xyz + 3 * i;
            std::sort(nn.begin() + 1, nn.end(), [&](int64_t u, int64_t v) {
                const float su = sq_dist(q, xyz + 3 * u), sv = sq_dist(q, xyz + 3 * v);
                return su < sv || (su == sv && u < v);
            });
            nn.resize((size_t)th_max + 1);
        }
        int64_t m = seg;
        for (int64_t j : nn) {
            int64_t l = label(j);
            if (l != 0 && l < m) m = l;
        }
        for (int64_t j : nn) {
            int64_t l = label(j);
            if (l == 0) assign(j, m);
            else if (l > m) relabel(l, m);
        }
        ++seg;
    }
    for (int64_t p = 0; p < n; ++p) lab_out[p] = label(p);
}

bool d_ok(float d) {
    if (!std::isfinite(d) || !(d > 0.f)) return false;
    float d2 = d * d;
    return std::isnormal(d2);
}

}  // namespace

extern "C" {

// Raw Alg. 1 label values after `steps` iterations (0 <= steps <= n).
// flags: 1 = relabel by rescanning all points (as printed), 2 = skip
// points that already carry a label (as printed).  Returns 0, or -1 on bad
// arguments.
int32_t oracle_fec_raw(const float *xyz, int64_t n, float d, int64_t steps, int32_t flags,
                       int64_t *lab_out) {
    if (n < 0 || steps < 0 || steps > n || !d_ok(d)) return -1;
    if (n == 0) return 0;
    fec_loop(xyz, n, d, steps, flags, lab_out);
    return 0;
}

// Full clustering: canonical labels (smallest member index, -1 when the
// cluster size is outside [min_size, max_size]).  Returns the number of
// kept clusters, or -1 on bad arguments.  th_max > 0: the capped variant
// (measurement only).  When canon_out is not null it also receives the
// canonical labels before the size filter, and *ncomp the number of
// clusters (one loop serves both outputs).
int64_t oracle_fec_full(const float *xyz, int64_t n, float d, int32_t min_size,
                        int32_t max_size, int32_t flags, int64_t th_max, int32_t *labels_out,
                        int32_t *canon_out, int64_t *ncomp) {
    if (n < 0 || !d_ok(d) || min_size > max_size || th_max < 0) return -1;
    if (ncomp) *ncomp = 0;
    if (n == 0) return 0;
    std::vector<int64_t> lab(n);
    fec_loop(xyz, n, d, n, flags, lab.data(), th_max);
    // canonicalise: smallest index per label value, and cluster sizes
    std::vector<int64_t> first(n + 2, -1), size(n + 2, 0);
    for (int64_t i = 0; i < n; ++i) {
        int64_t l = lab[i];
        if (first[l] < 0) first[l] = i;
        ++size[l];
    }
    int64_t lo = min_size < 1 ? 1 : min_size;
    int64_t k = 0, all = 0;
    for (int64_t l = 0; l < n + 2; ++l) {
        if (size[l] > 0 && size[l] >= lo && size[l] <= max_size) ++k;
        if (size[l] > 0) ++all;
    }
    for (int64_t i = 0; i < n; ++i) {
        int64_t l = lab[i];
        labels_out[i] = (size[l] >= lo && size[l] <= max_size) ? (int32_t)first[l] : -1;
        if (canon_out) canon_out[i] = (int32_t)first[l];
    }
    if (ncomp) *ncomp = all;
    return k;
}

int64_t oracle_fec_ex(const float *xyz, int64_t n, float d, int32_t min_size, int32_t max_size,
                      int32_t flags, int64_t th_max, int32_t *labels_out) {
    return oracle_fec_full(xyz, n, d, min_size, max_size, flags, th_max, labels_out, nullptr,
                           nullptr);
}

// Full clustering as Alg. 1 with the readings above (no cap).
int64_t oracle_fec(const float *xyz, int64_t n, float d, int32_t min_size, int32_t max_size,
                   int32_t flags, int32_t *labels_out) {
    return oracle_fec_ex(xyz, n, d, min_size, max_size, flags, 0, labels_out);
}

// ------------------------------------------------------------ index queries
// A kd-tree over a cloud, kept alive for sampled checks on clouds too large
// to cluster in full.  The cloud must outlive the handle.
void *oracle_index_new(const float *xyz, int64_t n, float d) {
    if (n < 0 || !d_ok(d)) return nullptr;
    return new (std::nothrow) KdTree(xyz, n, d);
}

void oracle_index_free(void *h) { delete static_cast<KdTree *>(h); }

// Neighbours j != i of point i (E(i, j) true).  Writes at most `cap` indices
// and returns the total count.
int64_t oracle_index_neighbors(void *h, int64_t i, int64_t *out, int64_t cap) {
    const KdTree *t = static_cast<const KdTree *>(h);
    int64_t c = 0;
    t->radius(t->xyz + 3 * i, [&](int64_t j) {
        if (j == i) return;
        if (c < cap) out[c] = j;
        ++c;
    });
    return c;
}

// Breadth-first search of the component of `seed` in the graph of E.
// Stops once more than `cap` points were reached.  Returns the number of
// points reached (cap + 1 when stopped early); *min_index receives the
// smallest index reached.  If `members` is non-null the first
// min(count, cap) reached indices are written there.
int64_t oracle_component(void *h, int64_t seed, int64_t cap, int64_t *min_index,
                         int64_t *members) {
    const KdTree *t = static_cast<const KdTree *>(h);
    std::vector<uint8_t> seen((size_t)t->n, 0);
    std::vector<int64_t> q;
    q.push_back(seed);
    seen[seed] = 1;
    int64_t mn = seed;
    size_t head = 0;
    while (head < q.size() && (int64_t)q.size() <= cap) {
        int64_t u = q[head++];
        t->radius(t->xyz + 3 * u, [&](int64_t j) {
            if (!seen[j]) {
                seen[j] = 1;
                q.push_back(j);
                if (j < mn) mn = j;
            }
        });
    }
    int64_t c = (int64_t)q.size();
    if (c > cap) c = cap + 1;
    if (min_index) *min_index = mn;
    if (members) {
        int64_t w = std::min<int64_t>(c, cap);
        for (int64_t k = 0; k < w; ++k) members[k] = q[k];
    }
    return c;
}

// Closure check on sampled points: counts the pairs (i in sample, j) with
// E(i, j) and labels[i] != labels[j].
int64_t oracle_closure_violations(void *h, const int32_t *labels, const int64_t *sample,
                                  int64_t ns) {
    const KdTree *t = static_cast<const KdTree *>(h);
    int64_t bad = 0;
    for (int64_t s = 0; s < ns; ++s) {
        int64_t i = sample[s];
        t->radius(t->xyz + 3 * i, [&](int64_t j) {
            if (labels[j] != labels[i]) ++bad;
        });
    }
    return bad;
}

// Number of (ordered, i != j) neighbour pairs over the sampled points;
// used to report neighbours per point.
int64_t oracle_count_neighbors(void *h, const int64_t *sample, int64_t ns) {
    const KdTree *t = static_cast<const KdTree *>(h);
    int64_t c = 0;
    for (int64_t s = 0; s < ns; ++s) {
        int64_t i = sample[s];
        t->radius(t->xyz + 3 * i, [&](int64_t j) { c += (j != i); });
    }
    return c;
}

}  // extern "C"
