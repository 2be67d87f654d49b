// Host driver and C ABI of the batch hierarchical Tucker library.
//
// A handle keeps the dimension tree, the host mirror of the HT ranks and the
// device pointers into the caller's workspace.  BHT-l2r (Alg. 1) and HT-RISE
// (Alg. 2) are driven layer by layer from the leaves; every arithmetic step runs
// in the device kernels of ht_kernels.hip / ht_eig.hip.  The host reads back the
// norms (skip test) and the rank decisions of each layer, because they size the
// launches of the next step.
//
// Two precision forms.  HT_FP64: every contraction and Gram product on FP64 matrix
// cores.  HT_FP32 (mixed): in HT-RISE updates, contractions with modes of at most
// 128 rows and their residual Grams run on FP32 matrix cores with FP64 partial
// sums, level tensors are stored in FP32, and the skip test sums the explicit
// residual energy each contraction discards (||Y||^2 - ||C1||^2 telescopes into
// these, and the difference of two FP32-accurate norms would not resolve
// eps^2 ||Y||^2).  The first batch (BHT-l2r: Grams of the data itself), the
// eigen-decompositions, truncation decisions, basis expansion and the cores stay
// FP64.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "ht_internal.h"
#include "ht_rise.h"
#include "ht_rise_testing.h"

using ht::Elem;
using ht::ModeView;

namespace {

thread_local std::string g_last_error;

ht_status fail(ht_status st, const std::string& msg) {
  g_last_error = msg;
  return st;
}

#define HT_HIP(call)                                                                       \
  do {                                                                                     \
    hipError_t e_ = (call);                                                                \
    if (e_ != hipSuccess)                                                                  \
      return fail(HT_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_));          \
  } while (0)

// --------------------------------------------------------------------------
// Dimension tree (Sec. 2.3): balanced, the first half of a node's modes to its first
// successor, or any binary tree over runs of consecutive modes given by a parent
// array; nodes numbered layer by layer, left to right.
// --------------------------------------------------------------------------
struct TNode {
  int layer = 0, lo = 0, hi = 0, parent = -1, child[2] = {-1, -1}, child_pos = -1;
  bool leaf() const { return child[0] < 0; }
};

struct Tree {
  int d = 0, depth = 0;
  std::vector<TNode> nodes;

  void build(int d_) {
    d = d_;
    struct Raw {
      int layer, lo, hi, parent, pos;
    };
    std::vector<Raw> raw;
    struct Rec {
      static void go(std::vector<Raw>& raw, int lo, int hi, int layer, int parent, int pos) {
        const int me = (int)raw.size();
        raw.push_back({layer, lo, hi, parent, pos});
        if (hi - lo > 1) {
          const int mid = lo + (hi - lo + 1) / 2;
          go(raw, lo, mid, layer + 1, me, 0);
          go(raw, mid, hi, layer + 1, me, 1);
        }
      }
    };
    Rec::go(raw, 0, d, 0, -1, -1);
    std::vector<int> order(raw.size());
    for (size_t i = 0; i < raw.size(); ++i) order[i] = (int)i;
    std::sort(order.begin(), order.end(), [&](int a, int b) {
      return raw[a].layer != raw[b].layer ? raw[a].layer < raw[b].layer : raw[a].lo < raw[b].lo;
    });
    std::vector<int> newid(raw.size());
    for (size_t i = 0; i < order.size(); ++i) newid[order[i]] = (int)i;
    nodes.assign(raw.size(), TNode());
    depth = 0;
    for (size_t i = 0; i < order.size(); ++i) {
      const Raw& r = raw[order[i]];
      TNode& t = nodes[i];
      t.layer = r.layer;
      t.lo = r.lo;
      t.hi = r.hi;
      t.parent = r.parent >= 0 ? newid[r.parent] : -1;
      t.child_pos = r.pos;
      depth = std::max(depth, r.layer);
    }
    for (size_t i = 0; i < nodes.size(); ++i) {
      const int p = nodes[i].parent;
      if (p >= 0) nodes[p].child[nodes[i].child_pos] = (int)i;
    }
  }

  // The tree of a parent array (2d - 1 entries, parent[0] = -1, numbered layer by layer
  // from the root, left to right): a node's successors are the nodes naming it, the
  // lower index first; the leaves, read left to right, are modes 0 .. d-1.
  bool from_parent(int d_, const int32_t* parent, std::string& why) {
    d = d_;
    const int nn = 2 * d - 1;
    if (parent[0] != -1) return why = "tree_parent[0] must be -1 (the root)", false;
    nodes.assign(nn, TNode());
    for (int i = 1; i < nn; ++i) {
      const int p = parent[i];
      if (p < 0 || p >= i) return why = "tree_parent: every node's parent must precede it", false;
      TNode& q = nodes[p];
      if (q.child[1] >= 0) return why = "tree_parent: a node has more than two successors", false;
      q.child[q.child[0] < 0 ? 0 : 1] = i;
      nodes[i].parent = p;
      nodes[i].child_pos = q.child[1] == i ? 1 : 0;
    }
    for (int i = 0; i < nn; ++i)
      if (nodes[i].child[0] >= 0 && nodes[i].child[1] < 0)
        return why = "tree_parent: an inner node has a single successor", false;
    // layers and mode runs by a walk from the root, leaves numbered left to right
    int next = 0;
    std::vector<int> stack{0};
    std::vector<int> order;
    while (!stack.empty()) {
      const int i = stack.back();
      stack.pop_back();
      order.push_back(i);
      if (!nodes[i].leaf()) {
        for (int c : {nodes[i].child[1], nodes[i].child[0]}) {
          nodes[c].layer = nodes[i].layer + 1;
          stack.push_back(c);
        }
      }
    }
    for (int i : order)
      if (nodes[i].leaf()) {
        nodes[i].lo = next;
        nodes[i].hi = ++next;
      }
    if (next != d) return why = "tree_parent must describe a tree with d leaves", false;
    for (auto it = order.rbegin(); it != order.rend(); ++it) {
      TNode& t = nodes[*it];
      if (!t.leaf()) {
        t.lo = nodes[t.child[0]].lo;
        t.hi = nodes[t.child[1]].hi;
      }
    }
    depth = 0;
    for (int i = 0; i < nn; ++i) {
      depth = std::max(depth, nodes[i].layer);
      if (i > 0 && (nodes[i].layer < nodes[i - 1].layer ||
                    (nodes[i].layer == nodes[i - 1].layer && nodes[i].lo < nodes[i - 1].lo)))
        return why = "tree_parent must number the nodes layer by layer, left to right", false;
    }
    return true;
  }

  // modes of the level tensor entering layer ell, in mode order
  std::vector<int> frontier(int ell) const {
    std::vector<int> f;
    for (size_t i = 0; i < nodes.size(); ++i)
      if (nodes[i].layer == ell || (nodes[i].leaf() && nodes[i].layer < ell)) f.push_back((int)i);
    std::sort(f.begin(), f.end(), [&](int a, int b) { return nodes[a].lo < nodes[b].lo; });
    return f;
  }
};

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// ---- page-locked staging for the small device -> host read-backs (the skip
//      test's scalars, a layer's ranks and discarded energies).  A read-back into
//      pageable memory goes through a runtime staging copy and costs tens of
//      microseconds per synchronisation; each handle instead takes one block of
//      kPinnedBytes from a process-wide pool when it is created and returns it
//      when destroyed.  Blocks are kept until the process ends.
constexpr size_t kPinnedBytes = 16384;
std::mutex g_pin_mu;
std::vector<void*> g_pin_free;

void* pinned_take() {
  {
    std::lock_guard<std::mutex> lk(g_pin_mu);
    if (!g_pin_free.empty()) {
      void* p = g_pin_free.back();
      g_pin_free.pop_back();
      return p;
    }
  }
  void* p = nullptr;
  if (hipHostMalloc(&p, kPinnedBytes, hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  return p;
}

void pinned_give(void* p) {
  if (p == nullptr) return;
  std::lock_guard<std::mutex> lk(g_pin_mu);
  g_pin_free.push_back(p);
}

// Waits for everything enqueued on s: the waits of an update are short (a few
// kernels), so the stream is polled for up to 2 ms before the blocking call.
hipError_t wait_stream(hipStream_t s) {
  const auto t0 = std::chrono::steady_clock::now();
  for (;;) {
    const hipError_t e = hipStreamQuery(s);
    if (e != hipErrorNotReady) return e;
    if (std::chrono::steady_clock::now() - t0 > std::chrono::milliseconds(2)) return hipStreamSynchronize(s);
  }
}

hipError_t wait_event(hipEvent_t ev) {
  const auto t0 = std::chrono::steady_clock::now();
  for (;;) {
    const hipError_t e = hipEventQuery(ev);
    if (e != hipErrorNotReady) return e;
    if (std::chrono::steady_clock::now() - t0 > std::chrono::milliseconds(2)) return hipEventSynchronize(ev);
  }
}

}  // namespace

// ============================================================================
// handle
// ============================================================================
struct ht_state {
  // configuration
  int d = 0;
  std::vector<int64_t> n;
  double eps = 0.0;
  int rank_cap = 0;
  int64_t max_batch = 0, n_cap = 0;
  Elem in_t = Elem::F32;
  bool mixed = false;     // HT_FP32 requested
  bool mixed_ok = false;  // and the FP32 error floor lies well inside eps_nw (precision gate)
  bool adaptive = false;  // HT_ADAPTIVE_BUDGET: nodewise tolerance recomputed after every layer
  int shares = 0;         // truncations the budget is split over: 2d - 2, or 2d - 3 (HT_PLAIN_HT_BUDGET)
  bool st_hosvd = false;  // HT_ST_HOSVD: the nodes of a layer truncated one after the other
  Tree tree;
  // per-node capacities: rows of the basis matrix (alpha) and rank bound
  std::vector<int64_t> alpha_cap;
  std::vector<int> rc;
  // live state
  std::vector<int> rank;
  int64_t n_acc = 0;
  // workspace carve (device pointers)
  char* ws = nullptr;
  size_t ws_bytes = 0;
  std::vector<double*> core, gram, vecs, evals, eigsc;
  double* core_backup = nullptr;
  size_t core_backup_elems = 0;
  double* root = nullptr;
  double* bufA = nullptr;
  double* bufB = nullptr;
  double* resid = nullptr;
  size_t resid_elems = 0;
  double* bufZ = nullptr;
  double* gpart = nullptr;
  double* scal = nullptr;
  double* sspart = nullptr;
  double* nrmpart = nullptr;
  double* respart = nullptr;  // one partial array per node (the skip test's sums are deferred)
  double* ssnode = nullptr;   // two sum-of-squares partial arrays per node
  double* orthsc = nullptr;
  double* padtmp = nullptr;
  double* tails = nullptr;
  double* aux = nullptr;  // two per node: trace(G), lambda_r (the mixed form's certificates)
  int* ranks_dev = nullptr;
  // host staging for small read-backs: h_scal (kScalars doubles), h_tails and
  // h_ranks (one per node), h_aux (two per node), in a page-locked block when one
  // was available
  void* pin = nullptr;
  std::vector<double> pin_fallback;
  double* h_scal = nullptr;
  double* h_tails = nullptr;
  int* h_ranks = nullptr;
  double* h_aux = nullptr;
  hipStream_t last_stream = nullptr;
  ht_state() = default;
  ht_state(const ht_state&) = delete;
  ht_state& operator=(const ht_state&) = delete;
  ~ht_state() { pinned_give(pin); }
};

namespace {

struct Layout {
  size_t total = 0;
  // offsets (bytes)
  std::vector<size_t> core, gram, vecs, evals, eigsc;
  size_t core_backup = 0, core_backup_elems = 0, root = 0, bufA = 0, bufB = 0, buf_elems = 0, resid = 0, bufZ = 0,
         resid_elems = 0, gpart = 0, scal = 0, sspart = 0, nrmpart = 0, respart = 0, ssnode = 0, orthsc = 0, padtmp = 0,
         tails = 0, aux = 0,
         ranks_dev = 0;
};

// device scalars: ||Y||^2, ||C1||^2, then two per node (mixed-form energies)
size_t kScalars(int nn) { return 8 + 2 * (size_t)nn; }
size_t res_stride() { return std::max<size_t>(ht::ttm_norm_partials(), ht::kSumsqBlocks); }

// Queues this thread's final reduction sums for one batched launch while alive.
struct DeferSums {
  explicit DeferSums(std::vector<ht::SumJob>* list) { ht::sums_defer_begin(list); }
  ~DeferSums() { ht::sums_defer_end(); }
  DeferSums(const DeferSums&) = delete;
  DeferSums& operator=(const DeferSums&) = delete;
};

size_t take(Layout& L, size_t bytes) {
  const size_t off = L.total;
  L.total += align256(bytes);
  return off;
}

// Capacities and the level-tensor chain sizes for a configuration.
void capacities(const Tree& tree, const std::vector<int64_t>& n, int rank_cap, std::vector<int64_t>& alpha_cap,
                std::vector<int>& rc) {
  const int nn = (int)tree.nodes.size();
  alpha_cap.assign(nn, 0);
  rc.assign(nn, 0);
  for (int ell = tree.depth; ell >= 0; --ell) {
    for (int i = 0; i < nn; ++i) {
      const TNode& t = tree.nodes[i];
      if (t.layer != ell) continue;
      if (t.leaf())
        alpha_cap[i] = n[t.lo];
      else
        alpha_cap[i] = (int64_t)rc[t.child[0]] * rc[t.child[1]];
      rc[i] = (int)std::min<int64_t>(rank_cap, alpha_cap[i]);
    }
  }
}

// Largest intermediate of the projection chains at capacity (elements, FP64),
// and the largest level tensor entering any layer (for the residual buffer).
void chain_sizes(const Tree& tree, const std::vector<int64_t>& n, const std::vector<int64_t>& alpha_cap,
                 const std::vector<int>& rc, int64_t N, size_t& max_inter, size_t& max_level) {
  max_inter = 1;
  max_level = 1;
  for (int ell = tree.depth; ell >= 1; --ell) {
    const std::vector<int> f = tree.frontier(ell);
    std::vector<int64_t> sz(f.size());
    for (size_t k = 0; k < f.size(); ++k) {
      const TNode& t = tree.nodes[f[k]];
      sz[k] = t.leaf() ? n[t.lo] : alpha_cap[f[k]];
    }
    auto total = [&]() {
      size_t p = (size_t)N;
      for (int64_t s : sz) p *= (size_t)s;
      return p;
    };
    max_level = std::max(max_level, total());
    for (size_t k = 0; k < f.size(); ++k) {
      if (tree.nodes[f[k]].layer != ell) continue;
      sz[k] = rc[f[k]];
      max_inter = std::max(max_inter, total());
    }
  }
}

bool valid_config(const ht_config* c, std::string& why) {
  if (c == nullptr) return why = "cfg is NULL", false;
  if (c->d < 2 || c->d > 64) return why = "d must lie in [2, 64]", false;
  if (c->n == nullptr) return why = "cfg->n is NULL", false;
  for (int i = 0; i < c->d; ++i)
    if (c->n[i] < 1 || c->n[i] > (int64_t)1 << 31) return why = "mode sizes must lie in [1, 2^31]", false;
  if (!(c->eps_rel > 0.0 && c->eps_rel < 1.0)) return why = "eps_rel must lie in (0, 1)", false;
  if (c->rank_cap < 1 || c->rank_cap > 64) return why = "rank_cap must lie in [1, 64]", false;
  if (c->max_batch < 1) return why = "max_batch must be >= 1", false;
  if (c->n_cap < 1) return why = "n_cap must be >= 1", false;
  if (c->prec != HT_FP64 && c->prec != HT_FP32) return why = "prec must be HT_FP64 or HT_FP32", false;
  if (c->in_dtype != HT_F32 && c->in_dtype != HT_F64) return why = "in_dtype must be HT_F32 or HT_F64", false;
  if ((c->flags & ~(uint64_t)(HT_ADAPTIVE_BUDGET | HT_PLAIN_HT_BUDGET | HT_ST_HOSVD)) != 0)
    return why = "unknown bits in flags", false;
  if (c->tree_parent != nullptr) {
    Tree t;
    if (!t.from_parent(c->d, c->tree_parent, why)) return false;
  }
  return true;
}

// the configuration's dimension tree (balanced without tree_parent)
bool make_tree(const ht_config* c, Tree& t, std::string& why) {
  if (c->tree_parent == nullptr) {
    t.build(c->d);
    return true;
  }
  return t.from_parent(c->d, c->tree_parent, why);
}

Layout make_layout(const ht_config* c, const Tree& tree, std::vector<int64_t>& alpha_cap, std::vector<int>& rc) {
  std::vector<int64_t> n(c->n, c->n + c->d);
  capacities(tree, n, c->rank_cap, alpha_cap, rc);
  const int nn = (int)tree.nodes.size();
  Layout L;
  L.core.assign(nn, 0);
  L.gram.assign(nn, 0);
  L.vecs.assign(nn, 0);
  L.evals.assign(nn, 0);
  L.eigsc.assign(nn, 0);
  size_t max_core = 1, gpart = 1;
  for (int i = 1; i < nn; ++i) {
    const size_t a = (size_t)alpha_cap[i], r = (size_t)rc[i];
    L.core[i] = take(L, a * r * sizeof(double));
    L.core_backup_elems += a * r;
    max_core = std::max(max_core, a * r);
    L.gram[i] = take(L, a * a * sizeof(double));
    L.vecs[i] = take(L, a * r * sizeof(double));
    L.evals[i] = take(L, a * sizeof(double));
    L.eigsc[i] = take(L, ht::eig_scratch_doubles((int)a, (int)r) * sizeof(double));
    gpart = std::max(gpart, ht::gram_partial_bound((int64_t)a));
  }
  L.core_backup = take(L, L.core_backup_elems * sizeof(double));
  L.root = take(L, (size_t)c->n_cap * c->rank_cap * c->rank_cap * sizeof(double));
  size_t max_inter = 1, max_level = 1;
  chain_sizes(tree, n, alpha_cap, rc, c->max_batch, max_inter, max_level);
  L.buf_elems = max_inter;
  L.bufA = take(L, max_inter * sizeof(double));
  L.bufB = take(L, max_inter * sizeof(double));
  L.resid_elems = max_level;
  L.resid = take(L, max_level * sizeof(double));
  L.bufZ = take(L, max_level * sizeof(double));
  L.gpart = take(L, gpart * sizeof(double));
  L.scal = take(L, kScalars(nn) * sizeof(double));
  L.sspart = take(L, ht::kSumsqBlocks * sizeof(double));
  L.nrmpart = take(L, std::max<size_t>(ht::ttm_norm_partials(), ht::kSumsqBlocks) * sizeof(double));
  L.respart = take(L, (size_t)nn * res_stride() * sizeof(double));
  L.ssnode = take(L, (size_t)nn * 2 * ht::kSumsqBlocks * sizeof(double));
  L.orthsc = take(L, ht::orth_scratch_doubles(64) * sizeof(double));
  L.padtmp = take(L, max_core * sizeof(double));
  // the layer read-back block, laid out as its host staging: the nodes' discarded
  // energies, their ranks (in nn doubles of room), two certificate values per node
  L.tails = take(L, 4 * (size_t)nn * sizeof(double));
  L.ranks_dev = L.tails + (size_t)nn * sizeof(double);
  L.aux = L.tails + 2 * (size_t)nn * sizeof(double);
  return L;
}

// ---- the mixed form's error model ----------------------------------------------
// u = 2^-24.  Forming a residual X - U (U^T X) on FP32 matrix cores (r columns in U)
// errs by at most kResidK u sqrt(r + 1) ||X|| in the Frobenius norm (measured on the
// part against FP64 residuals of the test streams: at most 0.5 u sqrt(r + 1) ||X||);
// an FP32 contraction U^T X stored as an FP32 level tensor errs by at most
// kChainK u sqrt(r + 1) ||X|| (measured over whole contraction chains: at most
// 0.23 u sqrt(sum (r + 1)) ||Y||); independent steps add in quadrature.  The rounding
// of the Gram product R R^T moves its tail sums by at most kGramK u trace(G)
// (measured: at most 1.0 u trace(G)).  ||X|| <= ||Y|| for every level tensor of a
// batch.
constexpr double kU32 = 5.9604644775390625e-08;  // 2^-24
constexpr double kU64 = 1.1102230246251565e-16;  // 2^-53
constexpr double kResidK = 2.0;
constexpr double kChainK = 0.75;
constexpr double kGramK = 4.0;

// A residual Gram taken as (I - U U^T) M M^T (I - U U^T) from the FP64 Gram of M
// carries the rounding of M M^T, relative to ||M||^2 <= ||Y||^2 rather than to the
// residual's trace: its tail sums move by at most kGramProjK u64 ||Y||^2 (measured on
// the register-direct shapes of the test streams: at most 16 u64 ||M||^2).  It is used
// where that stays below a thousandth of the threshold.
constexpr double kGramProjK = 1024.0;
bool gram_proj_ok(double ny, double thr) { return kGramProjK * kU64 * ny * ny <= 1e-3 * thr; }

// Frobenius error bound of a residual formed (own = rank + 1 when formed in FP32, else
// 0) from a level tensor with the FP32 history chain = sum (rank + 1).
double resid_err(double ny, double own, double chain) {
  return kU32 * ny * std::sqrt(kResidK * kResidK * own + kChainK * kChainK * chain);
}

// Precision gate: the mixed form runs only when the largest residual error the model
// allows (every node at its rank capacity, all in one chain) stays below half of
// eps_nw / ||Y|| = eps / sqrt(2d - 2); otherwise no FP32 decision could be certified
// and the updates run in FP64 from the start.
bool fp32_gate(double eps, int d, const std::vector<int>& rc) {
  double c = 0.0;
  for (size_t i = 1; i < rc.size(); ++i) c += rc[i] + 1.0;
  return kResidK * kU32 * std::sqrt(c) <= 0.5 * eps / std::sqrt(2.0 * d - 2.0);
}

// Certificate of one rank decision taken on a Gram whose tail sums t(j) may differ
// from the exact ones by at most Delta(t) = 2 sqrt(t) dR + dR^2 + gerr: sqrt(t(j)) is
// the distance of the residual to the matrices of rank j, which moves by at most the
// residual's error dR, and gerr bounds the Gram product's rounding.  The rule chose
// rank r in [rmin, room] with tail t_r and smallest kept eigenvalue lam_r (so the tail
// one rank lower is t_r + lam_r).  Certified when every Gram within that error leads
// to the same decision: the kept side stays within thr, the side one rank lower stays
// above it, and a rank that the capacity cut short (r == room, t_r > thr) needs more
// under every such Gram.
bool decision_certified(int r, int rmin, int room, double t_r, double lam_r, double thr, double dR, double gerr) {
  auto delta = [&](double t) { return 2.0 * std::sqrt(std::max(t, 0.0)) * dR + dR * dR + gerr; };
  if (r == room && t_r > thr) return t_r - delta(t_r) > thr;
  if (t_r + delta(t_r) > thr) return false;
  if (r > rmin) {
    const double t_prev = t_r + lam_r;
    if (t_prev - delta(t_prev) <= thr) return false;
  }
  return true;
}

int64_t prod(const std::vector<int64_t>& v, size_t lo, size_t hi) {
  int64_t p = 1;
  for (size_t i = lo; i < hi; ++i) p *= v[i];
  return p;
}

// A level tensor: data pointer, element type, batch size and mode sizes (C order).
struct Level {
  const void* ptr;
  Elem t;
  int64_t N;
  std::vector<int64_t> modes;
  size_t elems() const { return (size_t)N * (size_t)prod(modes, 0, modes.size()); }
};

ModeView view_of(const Level& L, size_t k) {
  ModeView v;
  v.P = L.N * prod(L.modes, 0, k);
  v.m = L.modes[k];
  v.S = prod(L.modes, k + 1, L.modes.size());
  return v;
}

int alpha_now(const ht_state* h, int node) {
  const TNode& t = h->tree.nodes[node];
  if (t.leaf()) return (int)h->n[t.lo];
  return h->rank[t.child[0]] * h->rank[t.child[1]];
}

// Sizes of frontier(ell) before layer ell is processed.
std::vector<int64_t> frontier_sizes(const ht_state* h, int ell) {
  const std::vector<int> f = h->tree.frontier(ell);
  std::vector<int64_t> s(f.size());
  for (size_t k = 0; k < f.size(); ++k) s[k] = alpha_now(h, f[k]);
  return s;
}

double* other(const ht_state* h, const void* p) { return p == h->bufA ? h->bufB : h->bufA; }

// Order in which the nodes of layer ell contract the level tensor (frontier positions).
// The contractions of one layer act on different modes and commute (every node of a
// layer projects the same tensor), so the order only changes the cost: contracting
// mode k (m rows onto r) costs ~2 r T flops on a tensor of T elements and leaves
// T r / m, and the order that minimises the sum takes the modes by ascending
// r / (1 - r / m) (an exchange argument on two adjacent steps); modes that do not
// shrink come last, ties keep the frontier order.
std::vector<int> contraction_order(const ht_state* h, int ell, const std::vector<int64_t>& modes) {
  const std::vector<int> f = h->tree.frontier(ell);
  std::vector<int> ks;
  std::vector<double> key(f.size(), 0.0);
  for (size_t k = 0; k < f.size(); ++k) {
    if (h->tree.nodes[f[k]].layer != ell) continue;
    const double r = h->rank[f[k]], m = (double)modes[k];
    key[k] = r < m ? r / (1.0 - r / m) : HUGE_VAL;
    ks.push_back((int)k);
  }
  std::stable_sort(ks.begin(), ks.end(), [&](int a, int b) { return key[a] < key[b]; });
  return ks;
}

// Contract every node of layer ell with U^T (in contraction_order), then merge siblings.
// With norm_out the first contraction also writes the squared norm of the input.
// mixed: contractions of modes with at most 128 rows on FP32 matrix cores (FP32
// level tensor out); with energy, every contraction also writes the residual
// energy it discards: FP32 ones the explicit sum into energy[2 node] (explicit[node]
// set), FP64 ones ||in||^2 and ||out||^2 into energy[2 node] and [2 node + 1].
// With only (frontier positions) just those nodes are contracted, in that order, and
// the tensor is not merged (the ST-HOSVD steps of a layer); merge_level finishes it.
Level merge_level(const ht_state* h, int ell, const Level& cur);

// One contraction of a projection chain: frontier position k (node) of the level
// tensor cur, into dst.  Mixed form (modes of at most 128 rows): FP32 products and an
// FP32 result, with energy the explicit residual energy of the contraction; else FP64,
// with energy the energies before and after it.  norm_out also takes ||X||^2.  With
// group, a contraction that qualifies is added to it instead of being launched.
void contract_one(const ht_state* h, Level& cur, int k, int node, double* dst, hipStream_t s, double* norm_out,
                  bool mixed, double* energy, std::vector<char>* expl, std::vector<ht::TtmJob>* group = nullptr) {
  const ModeView v = view_of(cur, k);
  // the residual buffer is free during contractions: row chunks of few-column ones
  const ht::SplitScratch split(h->resid, h->resid_elems);
  const bool grouped = group != nullptr && ht::ttm_groupable(v, h->rank[node]) &&
                       (mixed ? v.m <= ht::kResidGramMaxM : energy == nullptr);
  if (mixed && v.m <= ht::kResidGramMaxM) {
    double* np = norm_out ? h->nrmpart : nullptr;
    double* rp = energy ? h->respart + (size_t)node * res_stride() : nullptr;
    double* ro = energy ? energy + 2 * node : nullptr;
    if (grouped)
      group->push_back(ht::TtmJob{cur.ptr, cur.t, v, h->core[node], h->rank[node], dst, Elem::F32, np, norm_out, rp,
                                  ro});
    else
      ht::ttm_contract_f32(cur.ptr, cur.t, v, h->core[node], h->rank[node], reinterpret_cast<float*>(dst), np,
                           norm_out, rp, ro, s);
    if (expl) (*expl)[node] = 1;
    cur.ptr = dst;
    cur.t = Elem::F32;
  } else if (grouped) {
    group->push_back(ht::TtmJob{cur.ptr, cur.t, v, h->core[node], h->rank[node], dst, Elem::F64,
                                norm_out ? h->nrmpart : nullptr, norm_out, nullptr, nullptr});
    if (expl) (*expl)[node] = 0;
    cur.ptr = dst;
    cur.t = Elem::F64;
  } else {
    double* ssp = h->ssnode + (size_t)node * 2 * ht::kSumsqBlocks;
    if (expl) (*expl)[node] = 0;
    // the energies before and after the contraction, from the contraction itself
    // where it can, else by two sums of squares
    const bool fused = energy != nullptr && norm_out == nullptr &&
                       ht::ttm_contract_sq(cur.ptr, cur.t, v, h->core[node], h->rank[node], dst, ssp,
                                           energy + 2 * node, ssp + ht::kSumsqBlocks, energy + 2 * node + 1,
                                           ht::kSumsqBlocks, s);
    if (!fused) {
      if (energy) ht::sumsq(cur.ptr, cur.t, (int64_t)cur.elems(), ssp, energy + 2 * node, s);
      if (norm_out != nullptr)
        ht::ttm_contract_norm(cur.ptr, cur.t, v, h->core[node], h->rank[node], dst, h->nrmpart, norm_out, s);
      else
        ht::ttm_contract(cur.ptr, cur.t, v, h->core[node], h->rank[node], dst, s);
    }
    cur.ptr = dst;
    cur.t = Elem::F64;
    if (energy && !fused) {
      cur.modes[k] = h->rank[node];
      ht::sumsq(cur.ptr, cur.t, (int64_t)cur.elems(), ssp + ht::kSumsqBlocks, energy + 2 * node + 1, s);
    }
  }
  cur.modes[k] = h->rank[node];
}

Level project_layer(const ht_state* h, int ell, const Level& in, hipStream_t s, double* norm_out = nullptr,
                    bool mixed = false, double* energy = nullptr, std::vector<char>* expl = nullptr,
                    double* const* pp = nullptr, const std::vector<int>* only = nullptr) {
  const std::vector<int> f = h->tree.frontier(ell);
  Level cur = in;
  for (const int k : only ? *only : contraction_order(h, ell, in.modes)) {
    // intermediates alternate between the handle's two level buffers, or the pair pp
    double* dst = pp ? (cur.ptr == pp[0] ? pp[1] : pp[0]) : other(h, cur.ptr);
    contract_one(h, cur, k, f[k], dst, s, norm_out, mixed, energy, expl);
    norm_out = nullptr;
  }
  return only ? cur : merge_level(h, ell, cur);
}

// Merge to the frontier of layer ell - 1 (a reshape: adjacent siblings fuse).
Level merge_level(const ht_state* h, int ell, const Level& cur) {
  Level out = cur;
  if (ell >= 1) out.modes = frontier_sizes(h, ell - 1 >= 1 ? ell - 1 : 1);
  if (ell == 1) {
    const TNode& root = h->tree.nodes[0];
    out.modes = {h->rank[root.child[0]], h->rank[root.child[1]]};
  }
  return out;
}

Level project_all(const ht_state* h, const void* Y, int64_t N, hipStream_t s, double* norm_out = nullptr,
                  bool mixed = false, double* energy = nullptr, std::vector<char>* expl = nullptr) {
  Level cur{Y, h->in_t, N, h->n};
  for (int ell = h->tree.depth; ell >= 1; --ell) {
    cur = project_layer(h, ell, cur, s, norm_out, mixed, energy, expl);
    norm_out = nullptr;
  }
  return cur;
}

// Root-to-leaves expansion (Eq. htucker_reconstruction) of N latent slices
// [N][r11][r12] (FP64, at lat, which may be a caller's buffer) into out (C-order
// [N][n_1]...[n_d] of type ot).  Each layer expands its nodes in the reverse of
// contraction_order (the transposed chain, so it costs what the projection costs);
// intermediates alternate between the handle's two level buffers.
void expand_all(const ht_state* h, const double* lat, int64_t N, void* out, Elem ot, hipStream_t s) {
  const int r11 = h->rank[h->tree.nodes[0].child[0]], r12 = h->rank[h->tree.nodes[0].child[1]];
  Level cur{lat, Elem::F64, N, {r11, r12}};
  for (int ell = 1; ell <= h->tree.depth; ++ell) {
    const std::vector<int> f = h->tree.frontier(ell);
    // split merged modes: sizes of frontier(ell) after its layer is processed
    std::vector<int64_t> sz(f.size());
    for (size_t k = 0; k < f.size(); ++k) {
      const TNode& t = h->tree.nodes[f[k]];
      sz[k] = (t.layer == ell) ? h->rank[f[k]] : h->n[t.lo];
    }
    cur.modes = sz;
    std::vector<int> order = contraction_order(h, ell, frontier_sizes(h, ell));
    std::reverse(order.begin(), order.end());
    for (size_t q = 0; q < order.size(); ++q) {
      const int k = order[q];
      const int node = f[k];
      const int64_t alpha = alpha_now(h, node);
      const ModeView v = view_of(cur, (size_t)k);
      const bool final_step = (ell == h->tree.depth) && (q + 1 == order.size());
      void* dst = final_step ? out : static_cast<void*>(other(h, cur.ptr));
      ht::ttm_expand(static_cast<const double*>(cur.ptr), v.P, h->rank[node], v.S, h->core[node], alpha, nullptr,
                     Elem::F64, dst, final_step ? ot : Elem::F64, s);
      cur.ptr = dst;
      cur.modes[k] = alpha;
    }
  }
}

ht_status sync_read(ht_state* h, hipStream_t s, const double* dev, size_t count, double* host) {
  HT_HIP(hipMemcpyAsync(host, dev, count * sizeof(double), hipMemcpyDeviceToHost, s));
  HT_HIP(wait_stream(s));
  (void)h;
  return HT_OK;
}

ht_status check_device() {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail(HT_EDEVICE, std::string("no HIP device: ") + hipGetErrorString(e));
  hipDeviceProp_t prop;
  e = hipGetDeviceProperties(&prop, dev);
  if (e != hipSuccess) return fail(HT_EDEVICE, std::string("hipGetDeviceProperties: ") + hipGetErrorString(e));
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(HT_EDEVICE, std::string("device is ") + prop.gcnArchName + ", this library is built for gfx950");
  return HT_OK;
}

// Device time of a call.  The two events are created once per host thread (and
// again when the thread's current device changes) instead of per call.
struct Timer {
  hipEvent_t a = nullptr, b = nullptr;
  hipStream_t s;
  explicit Timer(hipStream_t s_) : s(s_) {
    thread_local hipEvent_t ea = nullptr, eb = nullptr;
    thread_local int dev = -1;
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess) return;
    if (cur != dev || ea == nullptr || eb == nullptr) {
      if (ea) (void)hipEventDestroy(ea);
      if (eb) (void)hipEventDestroy(eb);
      ea = eb = nullptr;
      if (hipEventCreate(&ea) != hipSuccess || hipEventCreate(&eb) != hipSuccess) {
        (void)hipGetLastError();
        return;
      }
      dev = cur;
    }
    a = ea;
    b = eb;
    (void)hipEventRecord(a, s);
  }
  float stop() {
    float ms = 0.f;
    if (a && b) {
      (void)hipEventRecord(b, s);
      (void)wait_event(b);
      (void)hipEventElapsedTime(&ms, a, b);
    }
    return ms;
  }
};

void backup_cores(ht_state* h, hipStream_t s) {
  size_t off = 0;
  for (size_t i = 1; i < h->tree.nodes.size(); ++i) {
    const size_t n = (size_t)h->alpha_cap[i] * h->rc[i];
    ht::copy_f64(h->core[i], h->core_backup + off, (int64_t)n, s);
    off += n;
  }
}

void restore_cores(ht_state* h, hipStream_t s) {
  size_t off = 0;
  for (size_t i = 1; i < h->tree.nodes.size(); ++i) {
    const size_t n = (size_t)h->alpha_cap[i] * h->rc[i];
    ht::copy_f64(h->core_backup + off, h->core[i], (int64_t)n, s);
    off += n;
  }
}

// One layer of rank decisions: Gram (of the data, or of the explicit residual
// R = M - U_old U_old^T M), eigen-decomposition, truncation, expansion.
// rmin = 1 / r_old = 0 for BHT-l2r; rmin = 0 for HT-RISE.  Split in two so that
// the layers of many handles can share one eigen launch and one read-back.
struct LayerJobs {
  std::vector<ht::EigJob> jobs;
  std::vector<int> node, rold;
  std::vector<char> f32;  // the job's Gram has FP32 products (mixed form)
  std::vector<char> gm;   // the job's residual Gram is the projected FP64 Gram of M (mixed form)
  std::vector<ModeView> view;
};

// Gram launches of layer ell and the eigen jobs they feed.
// The Gram of node's unfolding (view v of cur): of the data (r_old = 0) or of the
// residual R = M - U_old U_old^T M (Eq. compute_residual): formed explicitly, with FP32
// products when f32 (modes of at most 128 rows), or with gm as
// (I - U_old U_old^T) M M^T (I - U_old U_old^T) from the FP64 Gram of M.
// pj: queue for the projections of gm Grams of at most 128 rows (launched by the caller).
void node_gram(ht_state* h, int node, const Level& cur, const ModeView& v, int r_old, bool f32, hipStream_t s,
               bool gm = false, std::vector<ht::ProjJob>* pj = nullptr) {
  if (r_old == 0) {
    ht::gram(cur.ptr, cur.t, v, h->gpart, h->gram[node], s);
  } else if (gm) {
    ht::resid_gram_proj(cur.ptr, cur.t, v, h->core[node], r_old, h->gpart, h->gram[node], h->bufZ, s, pj);
  } else if (v.m <= ht::kResidGramMaxM) {
    // formed in registers or tile by tile in LDS, never written out
    if (f32)
      ht::resid_gram_f32(cur.ptr, cur.t, v, h->core[node], r_old, h->gpart, h->gram[node], s);
    else
      ht::resid_gram(cur.ptr, cur.t, v, h->core[node], r_old, h->gpart, h->gram[node], s);
  } else {
    double* z = h->bufZ;  // U_old^T M: as large as the level tensor when alpha == r_old
    {
      // (row chunks through the residual buffer, which the expansion overwrites after)
      const ht::SplitScratch split(h->resid, h->resid_elems);
      ht::ttm_contract(cur.ptr, cur.t, v, h->core[node], r_old, z, s);
    }
    ht::ttm_expand(z, v.P, r_old, v.S, h->core[node], v.m, cur.ptr, cur.t, h->resid, Elem::F64, s);
    ht::gram(h->resid, Elem::F64, v, h->gpart, h->gram[node], s);
  }
}

// proj: the handle's error budget admits residual Grams from the Gram of M (gram_proj_ok).
void layer_grams(ht_state* h, int ell, const Level& cur, double thr, bool initial, bool mixed, hipStream_t s,
                 LayerJobs& L, int only_k = -1, const std::vector<char>* fp64 = nullptr, bool proj = false,
                 std::vector<ht::ProjJob>* pj = nullptr) {
  const std::vector<int> f = h->tree.frontier(ell);
  for (size_t k = 0; k < f.size(); ++k) {
    const int node = f[k];
    if (h->tree.nodes[node].layer != ell) continue;
    if (only_k >= 0 && (int)k != only_k) continue;
    const ModeView v = view_of(cur, k);
    const int alpha = (int)v.m;
    const int r_old = initial ? 0 : h->rank[node];
    if (alpha - r_old <= 0) continue;  // the basis already spans the whole mode
    // at the rank cap the decision still runs (rmax = 0) to detect a needed growth
    const int room = std::max(0, std::min(alpha, h->rank_cap) - r_old);
    const bool gm = mixed && proj && r_old > 0 && ht::resid_gram_proj_applies(cur.t, v, r_old) &&
                    ht::resid_gram_proj_work_doubles(v.m, r_old) <= h->resid_elems;
    const bool f32 = !gm && mixed && r_old > 0 && v.m <= ht::kResidGramMaxM && !(fp64 && (*fp64)[node]);
    node_gram(h, node, cur, v, r_old, f32, s, gm, pj);
    L.f32.push_back(f32 ? 1 : 0);
    L.gm.push_back(gm ? 1 : 0);
    L.view.push_back(v);
    ht::EigJob j;
    j.G = h->gram[node];
    j.scratch = h->eigsc[node];
    j.evals = h->evals[node];
    j.vecs = h->vecs[node];
    j.rank = h->ranks_dev + node;
    j.tail = h->tails + node;
    j.thr = thr;
    j.k = alpha;
    j.rmin = initial ? 1 : 0;
    j.rmax = room;
    j.method = ht::kEigAuto;
    L.jobs.push_back(j);
    L.node.push_back(node);
    L.rold.push_back(r_old);
  }
}

void launch_eig(const std::vector<ht::EigJob>& jobs, hipStream_t s) {
  for (size_t b = 0; b < jobs.size(); b += ht::kMaxEigJobs)
    ht::eig_trunc(jobs.data() + b, (int)std::min<size_t>(ht::kMaxEigJobs, jobs.size() - b), s);
}

// Ranks and discarded energies of the layer (device -> host staging, not yet
// synchronised), and after the wait their copies.
// The device block (tails, ranks, aux) and its host staging share one layout, so
// one copy brings back all three.
ht_status layer_readback(ht_state* h, hipStream_t s, bool with_aux = false) {
  const int nn = (int)h->tree.nodes.size();
  HT_HIP(hipMemcpyAsync(h->h_tails, h->tails, (with_aux ? 4 : 2) * nn * sizeof(double), hipMemcpyDeviceToHost, s));
  return HT_OK;
}

void layer_collect(const ht_state* h, std::vector<int>& rk, std::vector<double>& tl) {
  const int nn = (int)h->tree.nodes.size();
  rk.assign(h->h_ranks, h->h_ranks + nn);
  tl.assign(h->h_tails, h->h_tails + nn);
}

// After the read-back: capacity and finiteness checks, then [U_old, U_R] with U_R
// re-orthogonalised, and the zero padding of the parents.
// The expansions are appended to *orth when given (the caller launches them, with
// those of other handles, before anything reads the new cores), else launched here.
ht_status layer_finish(ht_state* h, double thr, bool initial, hipStream_t s, const LayerJobs& L,
                       const std::vector<int>& rk, const std::vector<double>& tl, int* growth,
                       std::vector<ht::OrthJob>* orth = nullptr) {
  for (size_t q = 0; q < L.jobs.size(); ++q) {
    const int node = L.node[q];
    const int r = rk[node];
    const int alpha = L.jobs[q].k;
    const int room = L.jobs[q].rmax;
    if (r == room && tl[node] > thr && L.rold[q] + room < alpha)
      return fail(HT_ERANKCAP, "rank of node " + std::to_string(node) + " would exceed rank_cap " +
                                   std::to_string(h->rank_cap));
    if (!std::isfinite(tl[node])) return fail(HT_ENUMERIC, "non-finite eigenvalues at node " + std::to_string(node));
  }
  std::vector<int> old_rank = h->rank;
  std::vector<ht::OrthJob> local;
  std::vector<ht::OrthJob>& oj = orth ? *orth : local;
  for (size_t q = 0; q < L.jobs.size(); ++q) {
    const int node = L.node[q];
    const int r = rk[node];
    if (r == 0) continue;
    oj.push_back(ht::OrthJob{h->core[node], h->vecs[node], h->core[node], L.jobs[q].k, L.rold[q], r});
    h->rank[node] = L.rold[q] + r;
    *growth += initial ? 0 : r;
  }
  if (!orth && !local.empty()) ht::orth_expand_batch(local.data(), (int)local.size(), s);
  // padWithZeros on every parent whose successors grew (the root's capacity layout pads itself)
  for (size_t q = 0; q < L.jobs.size(); ++q) {
    const int node = L.node[q];
    const int par = h->tree.nodes[node].parent;
    if (par <= 0 || initial) continue;
    if (h->tree.nodes[node].child_pos != 0 &&
        std::find(L.node.begin(), L.node.end(), h->tree.nodes[par].child[0]) != L.node.end())
      continue;  // parent handled once, at its first successor
    const int a = h->tree.nodes[par].child[0], b = h->tree.nodes[par].child[1];
    const int ra = old_rank[a], rb = old_rank[b], ra2 = h->rank[a], rb2 = h->rank[b];
    if (ra == ra2 && rb == rb2) continue;
    const int rp = h->rank[par];
    ht::pad_core(h->core[par], ra, rb, rp, h->padtmp, ra2, rb2, s);
    ht::copy_f64(h->padtmp, h->core[par], (int64_t)ra2 * rb2 * rp, s);
  }
  HT_HIP(hipGetLastError());
  return HT_OK;
}

ht_status decide_layer(ht_state* h, int ell, const Level& cur, double thr, bool initial, hipStream_t s,
                       int* growth, int only_k = -1) {
  LayerJobs L;
  layer_grams(h, ell, cur, thr, initial, false, s, L, only_k);
  launch_eig(L.jobs, s);
  HT_HIP(hipGetLastError());
  ht_status st = layer_readback(h, s);
  if (st != HT_OK) return st;
  HT_HIP(wait_stream(s));
  std::vector<int> rk;
  std::vector<double> tl;
  layer_collect(h, rk, tl);
  return layer_finish(h, thr, initial, s, L, rk, tl, growth);
}

ht_status setup_handle(const ht_config* cfg, void* ws, size_t ws_bytes, ht_state** out) {
  std::string why;
  if (!valid_config(cfg, why)) return fail(HT_EINVAL, why);
  if (ws == nullptr) return fail(HT_EINVAL, "ws is NULL");
  if (reinterpret_cast<uintptr_t>(ws) % 256 != 0) return fail(HT_EINVAL, "ws must be 256-byte aligned");
  ht_state* h = new (std::nothrow) ht_state();
  if (h == nullptr) return fail(HT_ENOMEM, "host allocation failed");
  h->d = cfg->d;
  h->n.assign(cfg->n, cfg->n + cfg->d);
  h->eps = cfg->eps_rel;
  h->rank_cap = cfg->rank_cap;
  h->max_batch = cfg->max_batch;
  h->n_cap = cfg->n_cap;
  h->in_t = cfg->in_dtype == HT_F32 ? Elem::F32 : Elem::F64;
  h->mixed = cfg->prec == HT_FP32;
  make_tree(cfg, h->tree, why);
  Layout L = make_layout(cfg, h->tree, h->alpha_cap, h->rc);
  h->mixed_ok = h->mixed && fp32_gate(h->eps, h->d, h->rc);
  h->adaptive = (cfg->flags & HT_ADAPTIVE_BUDGET) != 0;
  h->shares = (cfg->flags & HT_PLAIN_HT_BUDGET) ? 2 * cfg->d - 3 : 2 * cfg->d - 2;
  h->st_hosvd = (cfg->flags & HT_ST_HOSVD) != 0;
  if (ws_bytes < L.total) {
    delete h;
    return fail(HT_ENOMEM, "workspace of " + std::to_string(ws_bytes) + " bytes, " + std::to_string(L.total) +
                               " needed");
  }
  char* base = static_cast<char*>(ws);
  h->ws = base;
  h->ws_bytes = ws_bytes;
  const int nn = (int)h->tree.nodes.size();
  h->core.assign(nn, nullptr);
  h->gram.assign(nn, nullptr);
  h->vecs.assign(nn, nullptr);
  h->evals.assign(nn, nullptr);
  h->eigsc.assign(nn, nullptr);
  for (int i = 1; i < nn; ++i) {
    h->core[i] = reinterpret_cast<double*>(base + L.core[i]);
    h->gram[i] = reinterpret_cast<double*>(base + L.gram[i]);
    h->vecs[i] = reinterpret_cast<double*>(base + L.vecs[i]);
    h->evals[i] = reinterpret_cast<double*>(base + L.evals[i]);
    h->eigsc[i] = reinterpret_cast<double*>(base + L.eigsc[i]);
  }
  h->core_backup = reinterpret_cast<double*>(base + L.core_backup);
  h->core_backup_elems = L.core_backup_elems;
  h->root = reinterpret_cast<double*>(base + L.root);
  h->bufA = reinterpret_cast<double*>(base + L.bufA);
  h->bufB = reinterpret_cast<double*>(base + L.bufB);
  h->resid = reinterpret_cast<double*>(base + L.resid);
  h->resid_elems = L.resid_elems;
  h->bufZ = reinterpret_cast<double*>(base + L.bufZ);
  h->gpart = reinterpret_cast<double*>(base + L.gpart);
  h->scal = reinterpret_cast<double*>(base + L.scal);
  h->sspart = reinterpret_cast<double*>(base + L.sspart);
  h->nrmpart = reinterpret_cast<double*>(base + L.nrmpart);
  h->respart = reinterpret_cast<double*>(base + L.respart);
  h->ssnode = reinterpret_cast<double*>(base + L.ssnode);
  h->orthsc = reinterpret_cast<double*>(base + L.orthsc);
  h->padtmp = reinterpret_cast<double*>(base + L.padtmp);
  h->tails = reinterpret_cast<double*>(base + L.tails);
  h->aux = reinterpret_cast<double*>(base + L.aux);
  h->ranks_dev = reinterpret_cast<int*>(base + L.ranks_dev);
  h->rank.assign(nn, 0);
  {
    const size_t nd = kScalars(nn) + 4 * (size_t)nn;  // the ranks take at most nn doubles
    if (nd * sizeof(double) <= kPinnedBytes) h->pin = pinned_take();
    if (h->pin == nullptr) h->pin_fallback.assign(nd, 0.0);
    double* b = h->pin ? static_cast<double*>(h->pin) : h->pin_fallback.data();
    h->h_scal = b;
    h->h_tails = b + kScalars(nn);
    h->h_ranks = reinterpret_cast<int*>(b + kScalars(nn) + nn);
    h->h_aux = b + kScalars(nn) + 2 * nn;
  }
  *out = h;
  return HT_OK;
}

// ---- the static scratch of ht_project_static: one copy per GPU, in the code object,
//      so that the call allocates nothing.  Host code must never pass the array's
//      name to a kernel (in host code it is a stand-in, not a device address): the
//      device address comes from hipGetSymbolAddress, taken once per device with that
//      device current, and only that pointer is used.
constexpr size_t kStaticScratchDoubles = (size_t)1 << 25;  // 256 MiB
static __device__ __align__(256) double scratch[kStaticScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

ht_status static_scratch(double** out) {
  int dev = -1;
  HT_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(HT_EDEVICE, "device index out of range");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[dev] == nullptr) {
    void* p = nullptr;
    HT_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (p == nullptr) return fail(HT_EDEVICE, "hipGetSymbolAddress returned NULL");
    g_scratch_ptr[dev] = static_cast<double*>(p);
  }
  *out = g_scratch_ptr[dev];
  return HT_OK;
}

}  // namespace

// ============================================================================
// HT-RISE over one or many handles (Alg. 2).  The handles advance in lock step:
// the projections of every handle are launched before the one read-back of the
// skip tests; then, layer by layer from the leaves, every updating handle's Gram
// launches precede one shared eigen launch and one read-back of the decisions.
// A handle whose update fails is rolled back alone.
// ============================================================================
namespace {

struct Upd {
  ht_state* h = nullptr;
  const void* Y = nullptr;
  int64_t N = 0;
  Level c1, cur;
  std::vector<char> expl;
  std::vector<int> saved;
  double ny = 0, eps_des = 0, eps_proj = 0, thr = 0;
  double lost2 = 0, lost_err = 0, thr_err = 0;  // adaptive budget: error so far and its FP32 bound
  double chain_extra = 0;  // ST-HOSVD: FP32 contractions of this layer before the current node
  bool skip = false, busy = false;
  bool began = false;  // started an update in this call (its cores were backed up)
  bool mixed = false;  // this pass runs the FP32 kernels
  bool redo = false;   // an FP32 decision could not be certified: the call runs again in FP64
  int growth = 0;
  int recomputed = 0;  // decisions taken from FP64 residual Grams (directly or again)
  std::vector<double> e1;  // mixed form: each node's residual energy in the skip test
  ht_status st = HT_OK;
  std::string err;
  LayerJobs L;
  std::vector<int> rk;
  std::vector<double> tl;
};

// Sum of rank + 1 over the FP32 contractions that produced the level tensor entering
// layer ell: every node of a deeper layer whose mode has at most 128 rows.
double fp32_chain(const ht_state* h, int ell) {
  double c = 0.0;
  for (size_t i = 1; i < h->tree.nodes.size(); ++i)
    if (h->tree.nodes[i].layer > ell && alpha_now(h, (int)i) <= ht::kResidGramMaxM) c += h->rank[i] + 1.0;
  return c;
}

// App. C: number of truncated SVDs still to come after layer ell (every non-root node
// of the layers above it).
int svd_remaining(const ht_state* h, int ell) {
  int c = 0;
  for (size_t i = 1; i < h->tree.nodes.size(); ++i)
    if (h->tree.nodes[i].layer < ell) ++c;
  // under the plain-HT budget the root's two successors share one SVD
  return h->shares == 2 * h->d - 3 ? c - 1 : c;
}

// App. C: the nodewise threshold eps_nw^2 = (eps_abs^2 - eps_l^2) / svd_rem for the
// layers above ell, where eps_l^2 = lost2 is the energy the approximation has lost so
// far (clamped at 0).
double adapted_thr(double eps_abs, double lost2, const ht_state* h, int ell) {
  return std::max(0.0, eps_abs * eps_abs - lost2) / svd_remaining(h, ell);
}

// Mixed-form skip test certificate: the telescoped residual energies carry, per
// contraction j, the error of the model on a residual of energy e_j (its own FP32
// step and those before it), and the FP32 block sums a relative kGramK u.  True
// when the decision eps_proj <= eps_des holds under every such error.
bool skip_certified(const Upd& u, double lost) {
  const ht_state* h = u.h;
  double chain = 0.0, delta = kGramK * kU32 * std::fabs(lost);
  for (int ell = h->tree.depth; ell >= 1; --ell) {
    const std::vector<int> f = h->tree.frontier(ell);
    for (const int k : contraction_order(h, ell, frontier_sizes(h, ell))) {
      const int node = f[k];
      const double* e = h->h_scal + 8 + 2 * node;
      const bool ex = u.expl[node] != 0;
      const double ej = ex ? e[0] : e[0] - e[1];
      const double own = ex ? h->rank[node] + 1.0 : 0.0;
      const double dj = resid_err(u.ny, own, chain);
      delta += 2.0 * std::sqrt(std::max(ej, 0.0)) * dj + dj * dj + (ex ? 0.0 : 4.0 * kU64 * e[0]);
      chain += own;
    }
  }
  return std::fabs(lost - u.eps_des * u.eps_des) > delta;
}

// Certificates of a mixed layer's decisions (after the read-back of ranks, tails and
// the aux pairs).  A decision from an FP32 Gram that fails is listed in *redo_jobs for
// an FP64 Gram; one that fails with an FP64 Gram (its level tensor's FP32 history
// alone is too coarse) marks the whole update for an FP64 run.
void certify_layer(Upd& u, int ell, bool fp64_pass, std::vector<int>* redo_jobs) {
  const ht_state* h = u.h;
  const double chain = fp32_chain(h, ell) + u.chain_extra;
  for (size_t q = 0; q < u.L.jobs.size(); ++q) {
    if (fp64_pass && std::find(redo_jobs->begin(), redo_jobs->end(), (int)q) == redo_jobs->end()) continue;
    const int node = u.L.node[q];
    const bool f32 = !fp64_pass && u.L.f32[q];
    const double own = f32 ? u.L.rold[q] + 1.0 : 0.0;
    const double dR = resid_err(u.ny, own, chain);
    const double tr = h->h_aux[2 * node];
    const bool gm = !fp64_pass && u.L.gm[q];
    const double gerr = (gm ? kGramProjK * kU64 * u.ny * u.ny : kGramK * (f32 ? kU32 : kU64) * tr) + u.thr_err;
    bool ok = decision_certified(u.rk[node], u.L.jobs[q].rmin, u.L.jobs[q].rmax, u.tl[node],
                                 h->h_aux[2 * node + 1], u.thr, dR, gerr);
    // The kept vectors must be accurate too, not only their number: a Gram error E
    // turns a kept direction by ~|E| / gap, and the part of its energy left behind
    // reappears in later batches' residuals (measured on the 48^4 x 4 stream: with
    // FP32 vectors the projection errors of later batches drift up to 3.5x the
    // oracle's and a rank differs after 80 batches).  E is the product rounding plus
    // the residual's own error against the residual, 2 sqrt(trace) dR; near the
    // threshold the gap may be as small as thr, so a growing node whose E exceeds 1 %
    // of thr takes its Gram again in FP64.
    if (ok && f32 && u.rk[node] > 0 && gerr + 2.0 * std::sqrt(std::max(tr, 0.0)) * dR > 0.01 * u.thr) ok = false;
    if (ok) continue;
    if (f32)
      redo_jobs->push_back((int)q);
    else
      u.redo = true;
  }
}

void aux_jobs(const Upd& u, const std::vector<int>* only, std::vector<ht::AuxJob>& out) {
  for (size_t q = 0; q < u.L.jobs.size(); ++q) {
    if (only && std::find(only->begin(), only->end(), (int)q) == only->end()) continue;
    const ht::EigJob& j = u.L.jobs[q];
    out.push_back(ht::AuxJob{j.G, j.rank, j.evals, u.h->aux + 2 * u.L.node[q], j.k});
  }
}

// Rolls a handle back to its state before the call (cores from the backup, the ranks).
void roll_back(Upd& u, hipStream_t s) {
  restore_cores(u.h, s);
  u.h->rank = u.saved;
  u.busy = false;
}

// One pass of HT-RISE over the handles in act (each with u.mixed set): Step 1 and
// the skip tests, then the layers in lock step, then the root appends.  Handles
// whose FP32 decisions cannot be certified come out with u.redo set and unchanged.
// Mixed form: the nodes of layer ell whose residual Gram goes straight to FP64.  The
// skip test's residual energy e of a node's contraction bounds the trace of its
// residual Gram from below (it was taken on a tensor with less energy: the other
// contractions of the layer before it and the old bases of the layers below, whose
// coordinates the updated level tensor contains).  With e above twice the threshold
// the node grows, and with 2 sqrt(e) dR above a hundredth of it the kept vectors of
// an FP32 Gram would fail the accuracy criterion of certify_layer: its FP32 Gram would
// only be taken again in FP64, which costs a second eigen launch and read-back.
void fp64_nodes(const Upd& u, int ell, std::vector<char>& out) {
  const ht_state* h = u.h;
  out.assign(h->tree.nodes.size(), 0);
  if (!u.mixed || u.e1.empty() || h->st_hosvd) return;  // (ST-HOSVD: no such bound)
  const double chain = fp32_chain(h, ell) + u.chain_extra;
  for (size_t node = 1; node < h->tree.nodes.size(); ++node) {
    if (h->tree.nodes[node].layer != ell || h->rank[node] == 0) continue;
    if (alpha_now(h, (int)node) > ht::kResidGramMaxM) continue;  // an FP64 Gram anyway
    const double e = u.e1[node];
    const double dR = resid_err(u.ny, h->rank[node] + 1.0, chain);
    if (e > 2.0 * u.thr && 2.0 * std::sqrt(e) * dR > 0.01 * u.thr) out[node] = 1;
  }
}

ht_status rise_pass(std::vector<Upd*>& act, hipStream_t s) {
  // ---- Step 1 for every handle: projection onto the existing cores; the first
  //      contraction also returns ||Y||^2 (mixed form: and the residual energies)
  //      The final sums of every handle's reductions run as one launch.
  //      The chains advance in lock step, one contraction of every handle per step,
  //      and the small contractions of a step go out as one grouped launch.
  {
    std::vector<ht::SumJob> sums;
    {
      const DeferSums defer(&sums);
      struct Chain {
        Upd* u;
        Level cur;
        int ell;
        std::vector<int> order;
        size_t pos;
        double* norm_out;
      };
      std::vector<Chain> ch;
      for (Upd* up : act) {
        Upd& u = *up;
        ht_state* h = u.h;
        h->last_stream = s;
        if (u.mixed) u.expl.assign(h->tree.nodes.size(), 0);
        Level cur{u.Y, h->in_t, u.N, h->n};
        ch.push_back(Chain{&u, cur, h->tree.depth, contraction_order(h, h->tree.depth, cur.modes), 0, h->scal});
      }
      std::vector<ht::TtmJob> group;
      for (bool more = true; more;) {
        more = false;
        group.clear();
        for (Chain& c : ch) {
          ht_state* h = c.u->h;
          while (c.ell >= 1 && c.pos == c.order.size()) {  // layer done: merge, next layer
            c.cur = merge_level(h, c.ell, c.cur);
            if (--c.ell >= 1) {
              c.order = contraction_order(h, c.ell, c.cur.modes);
              c.pos = 0;
            }
          }
          if (c.ell < 1) continue;
          const int k = c.order[c.pos++];
          const int node = h->tree.frontier(c.ell)[k];
          Upd& u = *c.u;
          contract_one(h, c.cur, k, node, other(h, c.cur.ptr), s, c.norm_out, u.mixed,
                       u.mixed ? h->scal + 8 : nullptr, u.mixed ? &u.expl : nullptr, &group);
          c.norm_out = nullptr;
          more = true;
        }
        if (!group.empty()) ht::ttm_group(group, s);
      }
      for (Chain& c : ch) {
        Upd& u = *c.u;
        u.c1 = c.cur;
        if (!u.mixed) ht::sumsq(u.c1.ptr, u.c1.t, (int64_t)u.c1.elems(), u.h->sspart, u.h->scal + 1, s);
      }
    }
    ht::reduce_batch(sums, s);
  }
  // The root slices of the batch as a skip leaves them are written before the skip
  // test is read back: a skipped batch then needs no launch after its decision, and an
  // updated one appends its own slices over the same slots (n_acc only advances when
  // the call succeeds).
  for (Upd* up : act) {
    ht_state* h = up->h;
    const int r11 = h->rank[h->tree.nodes[0].child[0]], r12 = h->rank[h->tree.nodes[0].child[1]];
    ht::root_append(up->c1.ptr, up->c1.t, up->N, r11, r12, h->root, h->n_acc, h->rank_cap, s);
    const size_t ns = up->mixed ? kScalars((int)h->tree.nodes.size()) : 2;
    HT_HIP(hipMemcpyAsync(h->h_scal, h->scal, ns * sizeof(double), hipMemcpyDeviceToHost, s));
  }
  HT_HIP(hipGetLastError());
  HT_HIP(wait_stream(s));
  // ---- skip tests (Eq. relative_error_threshold)
  for (Upd* up : act) {
    Upd& u = *up;
    ht_state* h = u.h;
    const double ny2 = h->h_scal[0];
    double lost = 0.0;
    if (u.mixed) {
      u.e1.assign(h->tree.nodes.size(), 0.0);
      for (int ell = h->tree.depth; ell >= 1; --ell)
        for (int node : h->tree.frontier(ell))
          if (h->tree.nodes[node].layer == ell) {
            u.e1[node] =
                u.expl[node] ? h->h_scal[8 + 2 * node] : h->h_scal[8 + 2 * node] - h->h_scal[8 + 2 * node + 1];
            lost += u.e1[node];
          }
    } else {
      lost = ny2 - h->h_scal[1];
    }
    if (!std::isfinite(ny2) || !std::isfinite(lost)) {
      u.st = HT_ENUMERIC;
      u.err = "non-finite norm";
      continue;
    }
    u.ny = std::sqrt(ny2);
    u.eps_des = h->eps * u.ny;
    u.eps_proj = std::sqrt(std::max(0.0, lost));
    if (u.mixed && !skip_certified(u, lost)) {
      u.redo = true;
      continue;
    }
    u.skip = u.eps_proj <= u.eps_des;
    if (!u.skip) {
      u.busy = true;
      u.began = true;
      u.saved = h->rank;
      backup_cores(h, s);
      const double eps_nw = u.eps_des / std::sqrt((double)h->shares);
      u.thr = eps_nw * eps_nw;
      u.lost2 = u.lost_err = u.thr_err = 0.0;
      u.cur = Level{u.Y, h->in_t, u.N, h->n};
    }
  }
  // ---- Step 2, layer by layer from the leaves (trees of different depths aligned
  //      at their leaves)
  int max_depth = 0;
  for (const Upd* up : act)
    if (up->busy) max_depth = std::max(max_depth, up->h->tree.depth);
  for (int t = 0; t < max_depth; ++t) {
    auto layer_of = [&](const Upd& u) { return u.busy ? u.h->tree.depth - t : 0; };
    // the nodes each handle truncates per step of this layer: all of them at once
    // (HOSVD: every node sees the same tensor), or one after the other in frontier
    // order (HT_ST_HOSVD: each on the tensor its predecessors have contracted)
    std::vector<std::vector<std::vector<int>>> steps(act.size());
    size_t nsteps = 0;
    for (size_t a = 0; a < act.size(); ++a) {
      Upd& u = *act[a];
      const int ell = layer_of(u);
      u.chain_extra = 0.0;
      if (ell < 1) continue;
      if (u.h->st_hosvd) {
        const std::vector<int> f = u.h->tree.frontier(ell);
        for (size_t k = 0; k < f.size(); ++k)
          if (u.h->tree.nodes[f[k]].layer == ell) steps[a].push_back({(int)k});
      } else {
        steps[a].push_back({});
      }
      nsteps = std::max(nsteps, steps[a].size());
      if (u.h->adaptive && u.mixed) u.expl.assign(u.h->tree.nodes.size(), 0);
    }
    for (size_t sub = 0; sub < nsteps; ++sub) {
      auto active = [&](size_t a) { return layer_of(*act[a]) >= 1 && sub < steps[a].size(); };
      auto only_of = [&](size_t a) -> const std::vector<int>* {
        return steps[a][sub].empty() ? nullptr : &steps[a][sub];
      };
      std::vector<ht::EigJob> all;
      std::vector<ht::AuxJob> aux;
      std::vector<ht::ProjJob> pj;  // projections of the layer's gm Grams, one launch
      for (size_t a = 0; a < act.size(); ++a) {
        Upd& u = *act[a];
        u.L = LayerJobs();
        if (!active(a)) continue;
        const std::vector<int>* only = only_of(a);
        std::vector<char> f64;
        fp64_nodes(u, layer_of(u), f64);
        layer_grams(u.h, layer_of(u), u.cur, u.thr, false, u.mixed, s, u.L, only ? (*only)[0] : -1, &f64,
                    u.mixed && gram_proj_ok(u.ny, u.thr), &pj);
        for (size_t q = 0; q < u.L.node.size(); ++q)
          if (u.mixed && !u.L.f32[q] && !u.L.gm[q] && f64[u.L.node[q]]) u.recomputed += 1;
        all.insert(all.end(), u.L.jobs.begin(), u.L.jobs.end());
        if (u.mixed) aux_jobs(u, nullptr, aux);
      }
      if (!pj.empty()) ht::gram_project_batch(pj.data(), (int)pj.size(), s);
      launch_eig(all, s);
      if (!aux.empty()) ht::decision_aux(aux.data(), (int)aux.size(), s);
      HT_HIP(hipGetLastError());
      for (size_t a = 0; a < act.size(); ++a) {
        if (!active(a)) continue;
        const ht_status st = layer_readback(act[a]->h, s, act[a]->mixed);
        if (st != HT_OK) return st;
      }
      HT_HIP(wait_stream(s));
      for (size_t a = 0; a < act.size(); ++a)
        if (active(a)) layer_collect(act[a]->h, act[a]->rk, act[a]->tl);
      // ---- certificates of the mixed decisions; FP64 Grams for the uncertified ones
      {
        std::vector<std::vector<int>> fix(act.size());
        std::vector<ht::EigJob> again;
        std::vector<ht::AuxJob> again_aux;
        for (size_t a = 0; a < act.size(); ++a) {
          Upd& u = *act[a];
          if (!active(a) || !u.mixed) continue;
          certify_layer(u, layer_of(u), false, &fix[a]);
          if (u.redo) continue;
          for (int q : fix[a]) {
            node_gram(u.h, u.L.node[q], u.cur, u.L.view[q], u.L.rold[q], false, s);
            again.push_back(u.L.jobs[q]);
            u.recomputed += 1;
          }
          if (!fix[a].empty()) aux_jobs(u, &fix[a], again_aux);
        }
        if (!again.empty()) {
          launch_eig(again, s);
          ht::decision_aux(again_aux.data(), (int)again_aux.size(), s);
          HT_HIP(hipGetLastError());
          for (size_t a = 0; a < act.size(); ++a) {
            if (fix[a].empty() || act[a]->redo) continue;
            const ht_status st = layer_readback(act[a]->h, s, true);
            if (st != HT_OK) return st;
          }
          HT_HIP(wait_stream(s));
          for (size_t a = 0; a < act.size(); ++a) {
            Upd& u = *act[a];
            if (fix[a].empty() || u.redo) continue;
            layer_collect(u.h, u.rk, u.tl);
            certify_layer(u, layer_of(u), true, &fix[a]);
          }
        }
        for (Upd* up : act)
          if (up->redo && up->busy) roll_back(*up, s);
      }
      std::vector<ht::OrthJob> orth;
      for (size_t a = 0; a < act.size(); ++a) {
        Upd& u = *act[a];
        if (!active(a)) continue;
        ht_status st = layer_finish(u.h, u.thr, false, s, u.L, u.rk, u.tl, &u.growth, &orth);
        if (st != HT_OK) {
          // roll this handle back (a failing handle has queued no expansion)
          u.st = st;
          u.err = g_last_error;
          roll_back(u, s);
          continue;
        }
      }
      if (!orth.empty()) ht::orth_expand_batch(orth.data(), (int)orth.size(), s);
      // ---- the projection of this step (merged into the next frontier after the last):
      //      the handles' contraction chains advance in lock step, the small
      //      contractions of a step in one grouped launch
      struct PChain {
        size_t a;
        std::vector<int> order, f;
        size_t pos;
      };
      std::vector<PChain> pc;
      for (size_t a = 0; a < act.size(); ++a) {
        Upd& u = *act[a];
        if (!active(a)) continue;
        ht_state* h = u.h;
        const int ell = layer_of(u);
        const std::vector<int>* only = only_of(a);
        if (only) {
          const int k = (*only)[0];
          if (u.mixed && u.cur.modes[k] <= ht::kResidGramMaxM) u.chain_extra += h->rank[h->tree.frontier(ell)[k]] + 1.0;
        }
        if (h->adaptive && ell > 1 && u.mixed) {
          // App. C in the mixed form: the energy each second-pass contraction discards,
          // summed (a difference of FP32-accurate norms would not resolve eps_des^2)
          u.cur = project_layer(h, ell, u.cur, s, nullptr, true, h->scal + 8, &u.expl, nullptr, only);
          if (only && sub + 1 == steps[a].size()) u.cur = merge_level(h, ell, u.cur);
          continue;
        }
        pc.push_back(PChain{a, only ? *only : contraction_order(h, ell, u.cur.modes), h->tree.frontier(ell), 0});
      }
      std::vector<ht::TtmJob> group;
      for (bool more = true; more;) {
        more = false;
        group.clear();
        for (PChain& c : pc) {
          if (c.pos == c.order.size()) continue;
          Upd& u = *act[c.a];
          const int k = c.order[c.pos++];
          contract_one(u.h, u.cur, k, c.f[k], other(u.h, u.cur.ptr), s, nullptr, u.mixed, nullptr, nullptr, &group);
          more = true;
        }
        if (!group.empty()) ht::ttm_group(group, s);
      }
      for (const PChain& c : pc) {
        Upd& u = *act[c.a];
        if (only_of(c.a) == nullptr || sub + 1 == steps[c.a].size()) u.cur = merge_level(u.h, layer_of(u), u.cur);
      }
    }
    // ---- App. C: the tolerance of the layers above from the energy lost so far
    bool adapt = false;
    for (Upd* up : act) {
      Upd& u = *up;
      const int ell = layer_of(u);
      if (ell <= 1 || !u.h->adaptive) continue;
      ht_state* h = u.h;
      if (!u.mixed) ht::sumsq(u.cur.ptr, u.cur.t, (int64_t)u.cur.elems(), h->sspart, h->scal + 1, s);
      HT_HIP(hipMemcpyAsync(h->h_scal, h->scal, kScalars((int)h->tree.nodes.size()) * sizeof(double),
                            hipMemcpyDeviceToHost, s));
      adapt = true;
    }
    if (adapt) {
      HT_HIP(wait_stream(s));
      for (Upd* up : act) {
        Upd& u = *up;
        const int ell = layer_of(u);
        if (ell <= 1 || !u.h->adaptive) continue;
        const ht_state* h = u.h;
        if (u.mixed) {
          // this layer's discarded energies and their error bound (as in the skip test)
          double chain = fp32_chain(h, ell);
          const std::vector<int> f = h->tree.frontier(ell);
          for (size_t k = 0; k < f.size(); ++k) {
            const int node = f[k];
            if (h->tree.nodes[node].layer != ell) continue;
            const double* e = h->h_scal + 8 + 2 * node;
            const bool ex = u.expl[node] != 0;
            const double ej = ex ? e[0] : e[0] - e[1];
            const double own = ex ? h->rank[node] + 1.0 : 0.0;
            const double dj = resid_err(u.ny, own, chain);
            u.lost2 += ej;
            u.lost_err += 2.0 * std::sqrt(std::max(ej, 0.0)) * dj + dj * dj + kGramK * kU32 * std::fabs(ej) +
                          (ex ? 0.0 : 4.0 * kU64 * e[0]);
            chain += own;
          }
        } else {
          u.lost2 = u.ny * u.ny - h->h_scal[1];
          u.lost_err = 4.0 * kU64 * u.ny * u.ny;
        }
        const int rem = svd_remaining(h, ell);
        u.thr = adapted_thr(u.eps_des, u.lost2, h, ell);
        u.thr_err = u.lost_err / rem;
      }
    }
  }
  for (Upd* up : act) {
    Upd& u = *up;
    if (!u.busy) continue;
    ht_state* h = u.h;
    const int q11 = h->rank[h->tree.nodes[0].child[0]], q12 = h->rank[h->tree.nodes[0].child[1]];
    ht::root_append(u.cur.ptr, u.cur.t, u.N, q11, q12, h->root, h->n_acc, h->rank_cap, s);
  }
  HT_HIP(hipGetLastError());
  return HT_OK;
}

// A failure inside a pass (a HIP error, a failed read-back): every handle that began an
// update in this call gets its cores and ranks back (the root slices past n_acc are not
// part of it yet), so the call leaves every handle as it was and returns the failure.
ht_status abandon_call(std::vector<Upd>& U, hipStream_t s, ht_status st) {
  const std::string err = g_last_error;
  for (Upd& u : U)
    if (u.began) {
      restore_cores(u.h, s);
      u.h->rank = u.saved;
      u.busy = false;
    }
  (void)hipStreamSynchronize(s);
  g_last_error = err;
  return st;
}

ht_status rise_many(ht_state* const* hs, const void* const* Ys, const int64_t* Ns, int count, hipStream_t s,
                    ht_update_info* infos) {
  std::vector<Upd> U(count);
  for (int i = 0; i < count; ++i) {
    Upd& u = U[i];
    u.h = hs[i];
    u.Y = Ys[i];
    u.N = Ns[i];
    if (u.h == nullptr) return fail(HT_EINVAL, "handle " + std::to_string(i) + " is NULL");
    if (u.Y == nullptr) return fail(HT_EINVAL, "Y of handle " + std::to_string(i) + " is NULL");
    if (u.N < 1) return fail(HT_EINVAL, "N of handle " + std::to_string(i) + " must be >= 1");
    if (u.N > u.h->max_batch) return fail(HT_ESHAPE, "N of handle " + std::to_string(i) + " exceeds max_batch");
    if (u.h->n_acc + u.N > u.h->n_cap)
      return fail(HT_ESHAPE, "accumulation of handle " + std::to_string(i) + " would exceed n_cap");
    u.mixed = u.h->mixed_ok;
  }
  Timer timer(s);
  std::vector<Upd*> act;
  for (Upd& u : U) act.push_back(&u);
  ht_status st = rise_pass(act, s);
  if (st != HT_OK) return abandon_call(U, s, st);
  // ---- handles whose FP32 decisions were not certified: the whole call in FP64
  act.clear();
  for (Upd& u : U)
    if (u.redo && u.st == HT_OK) {
      u.mixed = false;
      u.redo = false;
      u.skip = u.busy = false;
      u.growth = 0;
      u.recomputed += 1;
      act.push_back(&u);
    }
  if (!act.empty()) {
    st = rise_pass(act, s);
    if (st != HT_OK) return abandon_call(U, s, st);
  }
  const float ms = timer.stop();
  ht_status first = HT_OK;
  std::string first_err;
  for (int i = 0; i < count; ++i) {
    Upd& u = U[i];
    if (u.st == HT_OK) u.h->n_acc += u.N;
    if (u.st != HT_OK && first == HT_OK) {
      first = u.st;
      first_err = count > 1 ? "handle " + std::to_string(i) + ": " + u.err : u.err;
    }
    if (infos) {
      ht_update_info& in = infos[i];
      in.skipped = (u.st == HT_OK && u.skip) ? 1 : 0;
      in.rank_growth = u.st == HT_OK ? u.growth : 0;
      in.norm_y = u.ny;
      in.eps_des = u.eps_des;
      in.eps_proj = u.eps_proj;
      in.device_ms = ms;
      in.status = u.st;
      in.prec_used = u.mixed ? HT_FP32 : HT_FP64;
      in.recomputed = u.recomputed;
    }
  }
  if (first != HT_OK) return fail(first, first_err);
  return HT_OK;
}

}  // namespace

// ============================================================================
// C ABI
// ============================================================================
extern "C" {

const char* ht_status_str(ht_status s) {
  switch (s) {
    case HT_OK: return "ok";
    case HT_EINVAL: return "invalid argument";
    case HT_ESHAPE: return "batch or accumulation exceeds the configured capacity";
    case HT_ENOMEM: return "workspace too small";
    case HT_ERANKCAP: return "rank capacity exceeded";
    case HT_EDEVICE: return "device or HIP runtime error";
    case HT_ENUMERIC: return "non-finite value";
  }
  return "unknown status";
}

const char* ht_last_error(void) { return g_last_error.c_str(); }

ht_status ht_workspace_bytes(const ht_config* cfg, size_t* bytes) {
  std::string why;
  if (bytes == nullptr) return fail(HT_EINVAL, "bytes is NULL");
  if (!valid_config(cfg, why)) return fail(HT_EINVAL, why);
  Tree t;
  make_tree(cfg, t, why);
  std::vector<int64_t> ac;
  std::vector<int> rc;
  *bytes = make_layout(cfg, t, ac, rc).total;
  return HT_OK;
}

ht_status ht_update_precision(const ht_config* cfg, int32_t* prec) {
  std::string why;
  if (prec == nullptr) return fail(HT_EINVAL, "prec is NULL");
  if (!valid_config(cfg, why)) return fail(HT_EINVAL, why);
  Tree t;
  make_tree(cfg, t, why);
  std::vector<int64_t> ac;
  std::vector<int> rc;
  capacities(t, std::vector<int64_t>(cfg->n, cfg->n + cfg->d), cfg->rank_cap, ac, rc);
  *prec = (cfg->prec == HT_FP32 && fp32_gate(cfg->eps_rel, cfg->d, rc)) ? HT_FP32 : HT_FP64;
  return HT_OK;
}

int32_t ht_test_decision_certified(int32_t r, int32_t rmin, int32_t room, double t_r, double lam_r, double thr,
                                   double dR, double gerr) {
  return decision_certified(r, rmin, room, t_r, lam_r, thr, dR, gerr) ? 1 : 0;
}

ht_status ht_init_batch(const ht_config* cfg, void* ws, size_t ws_bytes, const void* Y, int64_t N, void* hip_stream,
                        ht_handle* out, ht_update_info* info) {
  g_last_error.clear();
  if (out == nullptr) return fail(HT_EINVAL, "out is NULL");
  *out = nullptr;
  if (Y == nullptr) return fail(HT_EINVAL, "Y is NULL");
  std::string why;
  if (!valid_config(cfg, why)) return fail(HT_EINVAL, why);
  if (N < 1) return fail(HT_EINVAL, "N must be >= 1");
  if (N > cfg->max_batch) return fail(HT_ESHAPE, "N exceeds max_batch");
  if (N > cfg->n_cap) return fail(HT_ESHAPE, "N exceeds n_cap");
  ht_status st = check_device();
  if (st != HT_OK) return st;
  ht_state* h = nullptr;
  st = setup_handle(cfg, ws, ws_bytes, &h);
  if (st != HT_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  h->last_stream = s;
  Timer timer(s);
  const int64_t E = N * prod(h->n, 0, h->n.size());
  ht::sumsq(Y, h->in_t, E, h->sspart, h->scal, s);
  st = sync_read(h, s, h->scal, 1, h->h_scal);
  if (st != HT_OK) {
    delete h;
    return st;
  }
  const double ny2 = h->h_scal[0];
  if (!std::isfinite(ny2)) {
    delete h;
    return fail(HT_ENUMERIC, "||Y|| is not finite");
  }
  if (ny2 == 0.0) {
    delete h;
    return fail(HT_EINVAL, "the initial batch is all zeros");
  }
  const double ny = std::sqrt(ny2);
  const double eps_nw = h->eps * ny / std::sqrt((double)h->shares);
  double thr = eps_nw * eps_nw;
  Level cur{Y, h->in_t, N, h->n};
  int growth = 0;
  for (int ell = h->tree.depth; ell >= 1; --ell) {
    if (h->st_hosvd) {
      // ST-HOSVD: the nodes of the layer one after the other, left to right, each on
      // the tensor its predecessors have contracted
      const std::vector<int> f = h->tree.frontier(ell);
      for (size_t k = 0; k < f.size(); ++k) {
        if (h->tree.nodes[f[k]].layer != ell) continue;
        st = decide_layer(h, ell, cur, thr, true, s, &growth, (int)k);
        if (st != HT_OK) {
          delete h;
          return st;
        }
        const std::vector<int> one{(int)k};
        cur = project_layer(h, ell, cur, s, nullptr, false, nullptr, nullptr, nullptr, &one);
      }
      cur = merge_level(h, ell, cur);
    } else {
      st = decide_layer(h, ell, cur, thr, true, s, &growth);
      if (st != HT_OK) {
        delete h;
        return st;
      }
      cur = project_layer(h, ell, cur, s);
    }
    if (h->adaptive && ell > 1) {
      // App. C: the energy lost so far sets the tolerance of the layers above
      ht::sumsq(cur.ptr, cur.t, (int64_t)cur.elems(), h->sspart, h->scal + 1, s);
      st = sync_read(h, s, h->scal + 1, 1, h->h_scal + 1);
      if (st != HT_OK) {
        delete h;
        return st;
      }
      thr = adapted_thr(h->eps * ny, ny2 - h->h_scal[1], h, ell);
    }
  }
  const int r11 = h->rank[h->tree.nodes[0].child[0]], r12 = h->rank[h->tree.nodes[0].child[1]];
  ht::sumsq(cur.ptr, cur.t, (int64_t)cur.elems(), h->sspart, h->scal + 1, s);
  ht::root_append(cur.ptr, cur.t, N, r11, r12, h->root, 0, h->rank_cap, s);
  if (hipGetLastError() != hipSuccess) {
    delete h;
    return fail(HT_EDEVICE, "kernel launch failed");
  }
  st = sync_read(h, s, h->scal + 1, 1, h->h_scal + 1);
  if (st != HT_OK) {
    delete h;
    return st;
  }
  h->n_acc = N;
  if (info) {
    info->skipped = 0;
    info->rank_growth = 0;
    for (size_t i = 1; i < h->rank.size(); ++i) info->rank_growth += h->rank[i];
    info->norm_y = ny;
    info->eps_des = h->eps * ny;
    info->eps_proj = std::sqrt(std::max(0.0, ny2 - h->h_scal[1]));
    info->device_ms = timer.stop();
    info->status = HT_OK;
    info->prec_used = HT_FP64;
    info->recomputed = 0;
  }
  *out = h;
  return HT_OK;
}

ht_status ht_rise_update(ht_handle h, const void* Y, int64_t N, void* hip_stream, ht_update_info* info) {
  g_last_error.clear();
  if (h == nullptr) return fail(HT_EINVAL, "handle is NULL");
  const void* ys[1] = {Y};
  const int64_t ns[1] = {N};
  ht_handle hs[1] = {h};
  return rise_many(hs, ys, ns, 1, static_cast<hipStream_t>(hip_stream), info);
}

ht_status ht_rise_update_many(ht_handle* hs, const void* const* Ys, const int64_t* Ns, int32_t count,
                              void* hip_stream, ht_update_info* infos) {
  g_last_error.clear();
  if (hs == nullptr || Ys == nullptr || Ns == nullptr) return fail(HT_EINVAL, "NULL argument");
  if (count < 1) return fail(HT_EINVAL, "count must be >= 1");
  for (int i = 0; i < count; ++i)
    for (int j = 0; j < i; ++j)
      if (hs[i] == hs[j]) return fail(HT_EINVAL, "a handle appears twice");
  return rise_many(hs, Ys, Ns, count, static_cast<hipStream_t>(hip_stream), infos);
}

ht_status ht_project(ht_handle h, const void* Y, int64_t N, void* latent, void* hip_stream) {
  g_last_error.clear();
  if (h == nullptr || Y == nullptr || latent == nullptr) return fail(HT_EINVAL, "NULL argument");
  if (N < 1) return fail(HT_EINVAL, "N must be >= 1");
  if (N > h->max_batch) return fail(HT_ESHAPE, "N exceeds max_batch");
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  h->last_stream = s;
  Level c1 = project_all(h, Y, N, s);
  ht::copy_f64(static_cast<const double*>(c1.ptr), static_cast<double*>(latent), (int64_t)c1.elems(), s);
  HT_HIP(hipGetLastError());
  HT_HIP(wait_stream(s));
  return HT_OK;
}

ht_status ht_project_static(ht_handle h, const void* Y, int64_t N, void* latent, void* hip_stream) {
  g_last_error.clear();
  if (h == nullptr || Y == nullptr || latent == nullptr) return fail(HT_EINVAL, "NULL argument");
  if (N < 1) return fail(HT_EINVAL, "N must be >= 1");
  double* base = nullptr;
  ht_status st = static_scratch(&base);
  if (st != HT_OK) return st;
  // per-sample sizes of the chain's intermediates, which alternate between two halves
  size_t half[2] = {0, 0};
  {
    int flip = 0;
    for (int ell = h->tree.depth; ell >= 1; --ell) {
      const std::vector<int> f = h->tree.frontier(ell);
      std::vector<int64_t> sz = frontier_sizes(h, ell);
      for (const int k : contraction_order(h, ell, frontier_sizes(h, ell))) {
        sz[k] = h->rank[f[k]];
        half[flip] = std::max(half[flip], (size_t)prod(sz, 0, sz.size()));
        flip ^= 1;
      }
    }
  }
  // the second half starts at a 256-byte boundary: 32 doubles of slack
  const size_t per = half[0] + half[1];
  const int64_t chunk = std::min<int64_t>(N, (int64_t)((kStaticScratchDoubles - 32) / per));
  if (chunk < 1)
    return fail(HT_ESHAPE, "one sample's projection needs " + std::to_string(per * sizeof(double)) +
                               " bytes of scratch, more than the static " +
                               std::to_string(kStaticScratchDoubles * sizeof(double)));
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  h->last_stream = s;
  double* pp[2] = {base, base + align256(half[0] * chunk * sizeof(double)) / sizeof(double)};
  const int r11 = h->rank[h->tree.nodes[0].child[0]], r12 = h->rank[h->tree.nodes[0].child[1]];
  const size_t esz = h->in_t == Elem::F32 ? 4 : 8;
  const int64_t sample = prod(h->n, 0, h->n.size());
  for (int64_t n0 = 0; n0 < N; n0 += chunk) {
    const int64_t cn = std::min<int64_t>(chunk, N - n0);
    Level cur{static_cast<const char*>(Y) + (size_t)n0 * sample * esz, h->in_t, cn, h->n};
    for (int ell = h->tree.depth; ell >= 1; --ell) cur = project_layer(h, ell, cur, s, nullptr, false, nullptr, nullptr, pp);
    ht::copy_f64(static_cast<const double*>(cur.ptr), static_cast<double*>(latent) + (size_t)n0 * r11 * r12,
                 cn * r11 * r12, s);
  }
  HT_HIP(hipGetLastError());
  HT_HIP(wait_stream(s));
  return HT_OK;
}

ht_status ht_reconstruct(ht_handle h, int64_t first, int64_t count, void* out, int32_t dtype, void* hip_stream) {
  g_last_error.clear();
  if (h == nullptr || out == nullptr) return fail(HT_EINVAL, "NULL argument");
  if (dtype != HT_F32 && dtype != HT_F64) return fail(HT_EINVAL, "dtype must be HT_F32 or HT_F64");
  if (first < 0 || count < 0 || first + count > h->n_acc) return fail(HT_EINVAL, "sample range out of bounds");
  if (count == 0) return HT_OK;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  h->last_stream = s;
  const Elem ot = dtype == HT_F32 ? Elem::F32 : Elem::F64;
  const size_t esz = dtype == HT_F32 ? 4 : 8;
  const int64_t per = prod(h->n, 0, h->n.size());
  const int r11 = h->rank[h->tree.nodes[0].child[0]], r12 = h->rank[h->tree.nodes[0].child[1]];
  for (int64_t c0 = 0; c0 < count; c0 += h->max_batch) {
    const int64_t cn = std::min<int64_t>(h->max_batch, count - c0);
    ht::root_extract(h->root, first + c0, cn, r11, r12, h->rank_cap, h->bufA, s);
    expand_all(h, h->bufA, cn, static_cast<char*>(out) + (size_t)c0 * per * esz, ot, s);
  }
  HT_HIP(hipGetLastError());
  HT_HIP(wait_stream(s));
  return HT_OK;
}

ht_status ht_decode(ht_handle h, const double* latent, int64_t N, void* out, int32_t dtype, void* hip_stream) {
  g_last_error.clear();
  if (h == nullptr || latent == nullptr || out == nullptr) return fail(HT_EINVAL, "NULL argument");
  if (dtype != HT_F32 && dtype != HT_F64) return fail(HT_EINVAL, "dtype must be HT_F32 or HT_F64");
  if (N < 0) return fail(HT_EINVAL, "N must be >= 0");
  if (N == 0) return HT_OK;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  h->last_stream = s;
  const Elem ot = dtype == HT_F32 ? Elem::F32 : Elem::F64;
  const size_t esz = dtype == HT_F32 ? 4 : 8;
  const int64_t per = prod(h->n, 0, h->n.size());
  const int r11 = h->rank[h->tree.nodes[0].child[0]], r12 = h->rank[h->tree.nodes[0].child[1]];
  for (int64_t c0 = 0; c0 < N; c0 += h->max_batch) {
    const int64_t cn = std::min<int64_t>(h->max_batch, N - c0);
    expand_all(h, latent + (size_t)c0 * r11 * r12, cn, static_cast<char*>(out) + (size_t)c0 * per * esz, ot, s);
  }
  HT_HIP(hipGetLastError());
  HT_HIP(wait_stream(s));
  return HT_OK;
}

ht_status ht_rte(ht_handle h, const void* Y, int64_t N, double* rel_err, void* hip_stream) {
  g_last_error.clear();
  if (h == nullptr || Y == nullptr || rel_err == nullptr) return fail(HT_EINVAL, "NULL argument");
  if (N < 1) return fail(HT_EINVAL, "N must be >= 1");
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  h->last_stream = s;
  const int r11 = h->rank[h->tree.nodes[0].child[0]], r12 = h->rank[h->tree.nodes[0].child[1]];
  const size_t esz = h->in_t == Elem::F32 ? 4 : 8;
  const int64_t per = prod(h->n, 0, h->n.size());
  // the residual buffer is idle outside updates: per-sample norms and their partials
  const int64_t cap = std::min<int64_t>(h->max_batch, (int64_t)(h->resid_elems / (2 + 2 * ht::kSegBlocks)));
  if (cap < 1) return fail(HT_ENOMEM, "workspace too small for the per-sample norms");
  double* y2 = h->resid;
  double* c2 = y2 + cap;
  double* part = c2 + cap;
  std::vector<double> hy(2 * cap);
  for (int64_t c0 = 0; c0 < N; c0 += cap) {
    const int64_t cn = std::min<int64_t>(cap, N - c0);
    const void* yc = static_cast<const char*>(Y) + (size_t)c0 * per * esz;
    Level c1 = project_all(h, yc, cn, s);
    ht::sumsq_segments(yc, h->in_t, cn, per, part, y2, s);
    ht::sumsq_segments(c1.ptr, c1.t, cn, (int64_t)r11 * r12, part + cap * ht::kSegBlocks, c2, s);
    HT_HIP(hipMemcpyAsync(hy.data(), y2, 2 * cap * sizeof(double), hipMemcpyDeviceToHost, s));
    HT_HIP(wait_stream(s));
    for (int64_t i = 0; i < cn; ++i) {
      const double a = hy[i], b = hy[cap + i];
      rel_err[c0 + i] = a > 0.0 ? std::sqrt(std::max(0.0, a - b) / a) : 0.0;
    }
  }
  return HT_OK;
}

ht_status ht_query_ranks(ht_handle h, int32_t* ranks, int32_t cap, int32_t* n_ranks, int64_t* n_accum) {
  g_last_error.clear();
  if (h == nullptr) return fail(HT_EINVAL, "handle is NULL");
  const int nr = (int)h->tree.nodes.size() - 1;
  if (ranks != nullptr && cap < nr) return fail(HT_EINVAL, "cap smaller than 2d-2");
  const hipError_t e = hipStreamSynchronize(h->last_stream);
  if (e != hipSuccess) return fail(HT_EDEVICE, hipGetErrorString(e));
  if (ranks != nullptr)
    for (int i = 0; i < nr; ++i) ranks[i] = h->rank[i + 1];
  if (n_ranks) *n_ranks = nr;
  if (n_accum) *n_accum = h->n_acc;
  return HT_OK;
}

ht_status ht_export_cores(ht_handle h, double* host_buf, size_t bytes, size_t* needed) {
  g_last_error.clear();
  if (h == nullptr) return fail(HT_EINVAL, "handle is NULL");
  const int nn = (int)h->tree.nodes.size();
  const int r11 = h->rank[h->tree.nodes[0].child[0]], r12 = h->rank[h->tree.nodes[0].child[1]];
  size_t total = 0;
  for (int i = 1; i < nn; ++i) total += (size_t)alpha_now(h, i) * h->rank[i];
  total += (size_t)h->n_acc * r11 * r12;
  if (needed) *needed = total * sizeof(double);
  if (host_buf == nullptr) return HT_OK;
  if (bytes < total * sizeof(double)) return fail(HT_ENOMEM, "export buffer too small");
  hipStream_t s = h->last_stream;
  HT_HIP(wait_stream(s));
  size_t off = 0;
  for (int i = 1; i < nn; ++i) {
    const size_t n = (size_t)alpha_now(h, i) * h->rank[i];
    HT_HIP(hipMemcpy(host_buf + off, h->core[i], n * sizeof(double), hipMemcpyDeviceToHost));
    off += n;
  }
  for (int64_t c0 = 0; c0 < h->n_acc; c0 += h->max_batch) {
    const int64_t cn = std::min<int64_t>(h->max_batch, h->n_acc - c0);
    ht::root_extract(h->root, c0, cn, r11, r12, h->rank_cap, h->bufA, s);
    HT_HIP(wait_stream(s));
    HT_HIP(hipMemcpy(host_buf + off, h->bufA, (size_t)cn * r11 * r12 * sizeof(double), hipMemcpyDeviceToHost));
    off += (size_t)cn * r11 * r12;
  }
  return HT_OK;
}

void ht_destroy(ht_handle h) { delete h; }

}  // extern "C"
