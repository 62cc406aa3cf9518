// tree.cpp -- thread pool and the adaptive cluster tree (Sec. 2.3).
//
// Tree rules (the paper fixes the ideas, these are the exact readings):
//  * the root is the minimal bounding box of the set; every cluster is shrunk
//    to the minimal box of its particles;
//  * a cluster is a leaf when it holds at most `leaf` particles, when its box
//    has zero extent, or when the split leaves a single non-empty child;
//  * otherwise it is bisected at the box midpoint in 1, 2 or 3 dimensions:
//    a dimension qualifies when its length L_d satisfies 2 L_d^2 >= L_max^2
//    (aspect ratio at most sqrt 2); at most one dimension is split when the
//    cluster holds at most 2*leaf particles, two when at most 4*leaf, else
//    three; the longest qualifying dimensions are taken first, equal lengths
//    in axis order x, y, z;
//  * a particle goes to the lower half of dimension d iff its coordinate is
//    below the midpoint; the child code is sum_d bit_d 2^d; empty children are
//    dropped; the partition is stable;
//  * clusters are numbered in depth-first preorder, children by increasing code.
//
// Large clusters are partitioned by all threads at once; subtrees below
// kSerialCutoff particles are then built independently in parallel and
// spliced into the preorder numbering.
#include <algorithm>
#include <array>
#include <atomic>
#include <cmath>
#include <condition_variable>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <thread>

#include "engine.hpp"

namespace bldtt {

// ---------------------------------------------------------------------------
// Thread pool
// ---------------------------------------------------------------------------
namespace {

class Pool {
public:
    Pool() {
        int n = (int)std::thread::hardware_concurrency();
        if (const char* e = std::getenv("BLDTT_THREADS")) n = std::atoi(e);
        if (n < 1) n = 1;
        if (n > 64) n = 64;
        nthreads_ = n;
        for (int i = 1; i < n; ++i) workers_.emplace_back([this] { loop(); });
    }
    ~Pool() {
        {
            std::lock_guard<std::mutex> g(m_);
            stop_ = true;
            ++gen_;
        }
        cv_.notify_all();
        for (auto& t : workers_) t.join();
    }
    int size() const { return nthreads_; }

    void run(int64_t n, const std::function<void(int64_t)>& fn) {
        if (n <= 0) return;
        if (nthreads_ == 1 || n == 1) {
            for (int64_t i = 0; i < n; ++i) fn(i);
            return;
        }
        std::unique_lock<std::mutex> outer(run_m_);   // one parallel region at a time
        {
            std::lock_guard<std::mutex> g(m_);
            fn_ = &fn;
            n_ = n;
            next_.store(0);
            active_ = (int)workers_.size();
            ++gen_;
        }
        cv_.notify_all();
        work();
        std::unique_lock<std::mutex> g(m_);
        done_cv_.wait(g, [this] { return active_ == 0; });
        fn_ = nullptr;
    }

private:
    void work() {
        for (;;) {
            int64_t i = next_.fetch_add(1);
            if (i >= n_) break;
            (*fn_)(i);
        }
    }
    void loop() {
        uint64_t seen = 0;
        for (;;) {
            {
                std::unique_lock<std::mutex> g(m_);
                cv_.wait(g, [&] { return gen_ != seen; });
                seen = gen_;
                if (stop_) return;
            }
            work();
            std::lock_guard<std::mutex> g(m_);
            if (--active_ == 0) done_cv_.notify_one();
        }
    }
    int nthreads_ = 1;
    std::vector<std::thread> workers_;
    std::mutex m_, run_m_;
    std::condition_variable cv_, done_cv_;
    const std::function<void(int64_t)>* fn_ = nullptr;
    int64_t n_ = 0;
    std::atomic<int64_t> next_{0};
    int active_ = 0;
    uint64_t gen_ = 0;
    bool stop_ = false;
};

Pool& pool() {
    static Pool p;
    return p;
}

}  // namespace

int num_threads() { return pool().size(); }
void parallel_run(int64_t ntasks, const std::function<void(int64_t)>& fn) { pool().run(ntasks, fn); }

// ---------------------------------------------------------------------------
// Tree build
// ---------------------------------------------------------------------------
namespace {

constexpr int64_t kSerialCutoff = 1 << 16;

struct Node {
    double lo[3], hi[3];
    int64_t b, e;
    int32_t level;
    int32_t nchild;
    int64_t child[8];     // index into the same node array, or -(job + 1) for a deferred subtree
};

struct BuildBufs {
    double* X[3];         // coordinates in tree order (permuted in place)
    int64_t* I;           // caller index in tree order
    double* tX[3];        // scratch of the same size
    int64_t* tI;
    int64_t leaf;
};

}  // namespace

// Which dimensions to split; 0 means the cluster is a leaf.
int split_mask(const double lo[3], const double hi[3], int64_t cnt, int64_t leaf) {
    double L[3] = {hi[0] - lo[0], hi[1] - lo[1], hi[2] - lo[2]};
    double Lmax = L[0];
    if (L[1] > Lmax) Lmax = L[1];
    if (L[2] > Lmax) Lmax = L[2];
    if (cnt <= leaf || Lmax == 0.0) return 0;
    int cap = cnt <= 2 * leaf ? 1 : (cnt <= 4 * leaf ? 2 : 3);
    int order[3] = {0, 1, 2};
    std::stable_sort(order, order + 3, [&](int a, int b) { return L[a] > L[b]; });
    int mask = 0, used = 0;
    for (int a = 0; a < 3 && used < cap; ++a) {
        int d = order[a];
        if (2.0 * (L[d] * L[d]) >= Lmax * Lmax) {
            mask |= 1 << d;
            ++used;
        }
    }
    return mask;
}

namespace {

inline int code_of(const BuildBufs& w, int64_t p, int mask, const double mid[3]) {
    int c = 0;
    for (int d = 0; d < 3; ++d)
        if ((mask >> d & 1) && !(w.X[d][p] < mid[d])) c |= 1 << d;
    return c;
}

struct Part {
    int64_t start[8], cnt[8];
    double lo[8][3], hi[8][3];
};

void box_init(double lo[3], double hi[3]) {
    for (int d = 0; d < 3; ++d) {
        lo[d] = HUGE_VAL;
        hi[d] = -HUGE_VAL;
    }
}

inline void box_add(double lo[3], double hi[3], double x, double y, double z) {
    double v[3] = {x, y, z};
    for (int d = 0; d < 3; ++d) {
        if (v[d] < lo[d]) lo[d] = v[d];
        if (v[d] > hi[d]) hi[d] = v[d];
    }
}

// Stable partition of [b, e) by child code, child boxes computed on the way.
void partition_serial(BuildBufs& w, int64_t b, int64_t e, int mask, const double mid[3], Part& out) {
    int64_t hist[8] = {0};
    for (int64_t p = b; p < e; ++p) hist[code_of(w, p, mask, mid)]++;
    int64_t fill[8], off = b;
    for (int k = 0; k < 8; ++k) {
        out.start[k] = off;
        out.cnt[k] = hist[k];
        fill[k] = off;
        off += hist[k];
        box_init(out.lo[k], out.hi[k]);
    }
    for (int64_t p = b; p < e; ++p) {
        int c = code_of(w, p, mask, mid);
        int64_t dst = fill[c]++;
        for (int d = 0; d < 3; ++d) w.tX[d][dst] = w.X[d][p];
        w.tI[dst] = w.I[p];
        box_add(out.lo[c], out.hi[c], w.X[0][p], w.X[1][p], w.X[2][p]);
    }
    for (int d = 0; d < 3; ++d) std::memcpy(w.X[d] + b, w.tX[d] + b, sizeof(double) * (e - b));
    std::memcpy(w.I + b, w.tI + b, sizeof(int64_t) * (e - b));
}

// Same result as partition_serial, all threads cooperating.
void partition_parallel(BuildBufs& w, int64_t b, int64_t e, int mask, const double mid[3], Part& out) {
    int64_t n = e - b;
    int nt = num_threads();
    int64_t chunks = std::min<int64_t>(4 * nt, std::max<int64_t>(1, n / 4096));
    std::vector<std::array<int64_t, 8>> hist(chunks);
    std::vector<std::array<double, 48>> boxes(chunks);
    auto range = [&](int64_t c, int64_t& cb, int64_t& ce) {
        cb = b + n * c / chunks;
        ce = b + n * (c + 1) / chunks;
    };
    parallel_run(chunks, [&](int64_t c) {
        int64_t cb, ce;
        range(c, cb, ce);
        hist[c].fill(0);
        for (int64_t p = cb; p < ce; ++p) hist[c][code_of(w, p, mask, mid)]++;
    });
    std::vector<std::array<int64_t, 8>> fill(chunks);
    int64_t off = b;
    for (int k = 0; k < 8; ++k) {
        out.start[k] = off;
        for (int64_t c = 0; c < chunks; ++c) {
            fill[c][k] = off;
            off += hist[c][k];
        }
        out.cnt[k] = off - out.start[k];
    }
    parallel_run(chunks, [&](int64_t c) {
        int64_t cb, ce;
        range(c, cb, ce);
        double* bx = boxes[c].data();
        for (int k = 0; k < 8; ++k) box_init(bx + 6 * k, bx + 6 * k + 3);
        auto& f = fill[c];
        for (int64_t p = cb; p < ce; ++p) {
            int k = code_of(w, p, mask, mid);
            int64_t dst = f[k]++;
            for (int d = 0; d < 3; ++d) w.tX[d][dst] = w.X[d][p];
            w.tI[dst] = w.I[p];
            box_add(bx + 6 * k, bx + 6 * k + 3, w.X[0][p], w.X[1][p], w.X[2][p]);
        }
    });
    parallel_run(chunks, [&](int64_t c) {
        int64_t cb, ce;
        range(c, cb, ce);
        for (int d = 0; d < 3; ++d) std::memcpy(w.X[d] + cb, w.tX[d] + cb, sizeof(double) * (ce - cb));
        std::memcpy(w.I + cb, w.tI + cb, sizeof(int64_t) * (ce - cb));
    });
    for (int k = 0; k < 8; ++k) {
        box_init(out.lo[k], out.hi[k]);
        for (int64_t c = 0; c < chunks; ++c) {
            const double* bx = boxes[c].data() + 6 * k;
            for (int d = 0; d < 3; ++d) {
                if (bx[d] < out.lo[k][d]) out.lo[k][d] = bx[d];
                if (bx[3 + d] > out.hi[k][d]) out.hi[k][d] = bx[3 + d];
            }
        }
    }
}

// Builds nodes in preorder into `nodes`; children at or below the cutoff are
// deferred into `jobs` when defer is set.
struct Builder {
    BuildBufs& w;
    std::vector<Node>& nodes;
    std::vector<Node>* jobs;   // deferred subtree roots (null: build everything here)

    int64_t build(const double lo[3], const double hi[3], int64_t b, int64_t e, int32_t level, bool parallel) {
        int64_t id = (int64_t)nodes.size();
        nodes.emplace_back();
        Node nd;
        std::memcpy(nd.lo, lo, sizeof nd.lo);
        std::memcpy(nd.hi, hi, sizeof nd.hi);
        nd.b = b;
        nd.e = e;
        nd.level = level;
        nd.nchild = 0;
        int mask = split_mask(lo, hi, e - b, w.leaf);
        if (mask) {
            double mid[3];
            for (int d = 0; d < 3; ++d) mid[d] = 0.5 * (lo[d] + hi[d]);
            Part part;
            if (parallel) partition_parallel(w, b, e, mask, mid, part);
            else partition_serial(w, b, e, mask, mid, part);
            int nonempty = 0;
            for (int k = 0; k < 8; ++k) nonempty += part.cnt[k] > 0;
            if (nonempty > 1) {
                for (int k = 0; k < 8; ++k) {
                    if (!part.cnt[k]) continue;
                    int64_t cb = part.start[k], ce = cb + part.cnt[k];
                    int64_t cid;
                    if (jobs && ce - cb <= kSerialCutoff) {
                        Node j;
                        std::memcpy(j.lo, part.lo[k], sizeof j.lo);
                        std::memcpy(j.hi, part.hi[k], sizeof j.hi);
                        j.b = cb;
                        j.e = ce;
                        j.level = level + 1;
                        j.nchild = 0;
                        jobs->push_back(j);
                        cid = -(int64_t)jobs->size();
                    } else {
                        cid = build(part.lo[k], part.hi[k], cb, ce, level + 1, parallel && ce - cb > kSerialCutoff);
                    }
                    nd.child[nd.nchild++] = cid;
                }
            }
        }
        nodes[id] = nd;
        return id;
    }
};

}  // namespace

void tree_from_nodes(const std::vector<BuildNode>& nodes, int64_t n, std::vector<int64_t> perm, Tree& t) {
    const int64_t total = (int64_t)nodes.size();
    t = Tree();
    t.n_particles = n;
    t.lo.resize(3 * total); t.hi.resize(3 * total); t.center.resize(3 * total);
    t.radius.resize(total);
    t.begin.resize(total); t.count.resize(total); t.parent.resize(total);
    t.child.assign(8 * total, -1);
    t.level.resize(total); t.nchild.resize(total);
    int64_t next = 0;
    int32_t depth = 0;
    std::function<int64_t(int64_t, int64_t)> emit = [&](int64_t li, int64_t par) -> int64_t {
        const BuildNode& nd = nodes[li];
        int64_t g = next++;
        double L[3];
        for (int d = 0; d < 3; ++d) {
            t.lo[3 * g + d] = nd.lo[d];
            t.hi[3 * g + d] = nd.hi[d];
            t.center[3 * g + d] = 0.5 * (nd.lo[d] + nd.hi[d]);
            L[d] = nd.hi[d] - nd.lo[d];
        }
        t.radius[g] = 0.5 * std::sqrt((L[0] * L[0] + L[1] * L[1]) + L[2] * L[2]);
        t.begin[g] = nd.b;
        t.count[g] = nd.e - nd.b;
        t.parent[g] = par;
        t.level[g] = nd.level;
        t.nchild[g] = nd.nchild;
        if (nd.level > depth) depth = nd.level;
        for (int k = 0; k < nd.nchild; ++k) t.child[8 * g + k] = emit(nd.child[k], g);
        return g;
    };
    emit(0, -1);
    t.depth = depth;
    t.perm = std::move(perm);
}

void build_tree(int64_t n, const double* x, const double* y, const double* z, int64_t leaf, Tree& t,
                std::vector<double>& xs, std::vector<double>& ys, std::vector<double>& zs) {
    xs.assign(x, x + n);
    ys.assign(y, y + n);
    zs.assign(z, z + n);
    std::vector<int64_t> idx(n);
    std::vector<double> s0(n), s1(n), s2(n);
    std::vector<int64_t> sI(n);
    BuildBufs w;
    w.X[0] = xs.data(); w.X[1] = ys.data(); w.X[2] = zs.data();
    w.tX[0] = s0.data(); w.tX[1] = s1.data(); w.tX[2] = s2.data();
    w.I = idx.data();
    w.tI = sI.data();
    w.leaf = leaf;
    const bool big = n > kSerialCutoff;
    int64_t chunks = big ? 4 * num_threads() : 1;

    // Root box (exact min/max, order independent).
    std::vector<std::array<double, 6>> rb(chunks);
    parallel_run(chunks, [&](int64_t c) {
        int64_t cb = n * c / chunks, ce = n * (c + 1) / chunks;
        double* bx = rb[c].data();
        box_init(bx, bx + 3);
        for (int64_t p = cb; p < ce; ++p) {
            idx[p] = p;
            box_add(bx, bx + 3, x[p], y[p], z[p]);
        }
    });
    double lo[3], hi[3];
    box_init(lo, hi);
    for (auto& bx : rb)
        for (int d = 0; d < 3; ++d) {
            if (bx[d] < lo[d]) lo[d] = bx[d];
            if (bx[3 + d] > hi[d]) hi[d] = bx[3 + d];
        }

    // Top of the tree with all threads, then the deferred subtrees in parallel.
    std::vector<Node> top, jobs;
    Builder tb{w, top, big ? &jobs : nullptr};
    tb.build(lo, hi, 0, n, 0, big);
    std::vector<std::vector<Node>> sub(jobs.size());
    parallel_run((int64_t)jobs.size(), [&](int64_t j) {
        Builder sb{w, sub[j], nullptr};
        sb.build(jobs[j].lo, jobs[j].hi, jobs[j].b, jobs[j].e, jobs[j].level, false);
    });

    // Splice into one preorder numbering.
    int64_t total = (int64_t)top.size();
    for (auto& s : sub) total += (int64_t)s.size();
    t = Tree();
    t.n_particles = n;
    t.lo.resize(3 * total); t.hi.resize(3 * total); t.center.resize(3 * total);
    t.radius.resize(total);
    t.begin.resize(total); t.count.resize(total); t.parent.resize(total);
    t.child.assign(8 * total, -1);
    t.level.resize(total); t.nchild.resize(total);
    int64_t next = 0;
    int32_t depth = 0;
    // emit(node array, local index, parent global id) -> global id, preorder
    std::function<int64_t(const std::vector<Node>&, int64_t, int64_t)> emit =
        [&](const std::vector<Node>& arr, int64_t li, int64_t par) -> int64_t {
        const Node& nd = arr[li];
        int64_t g = next++;
        double L[3];
        for (int d = 0; d < 3; ++d) {
            t.lo[3 * g + d] = nd.lo[d];
            t.hi[3 * g + d] = nd.hi[d];
            t.center[3 * g + d] = 0.5 * (nd.lo[d] + nd.hi[d]);
            L[d] = nd.hi[d] - nd.lo[d];
        }
        t.radius[g] = 0.5 * std::sqrt((L[0] * L[0] + L[1] * L[1]) + L[2] * L[2]);
        t.begin[g] = nd.b;
        t.count[g] = nd.e - nd.b;
        t.parent[g] = par;
        t.level[g] = nd.level;
        t.nchild[g] = nd.nchild;
        if (nd.level > depth) depth = nd.level;
        for (int k = 0; k < nd.nchild; ++k) {
            int64_t c = nd.child[k];
            int64_t cg = c >= 0 ? emit(arr, c, g) : emit(sub[-c - 1], 0, g);
            t.child[8 * g + k] = cg;
        }
        return g;
    };
    emit(top, 0, -1);
    t.depth = depth;
    t.perm = std::move(idx);
}

}  // namespace bldtt
