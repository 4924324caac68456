// plan.cpp -- from a signed Tait graph to a contraction plan for the PACI
// tensor network G_T (Sec. III of arXiv:1807.02119).
//
// 1. Simplification (Sec. III.A).  Loops (v, v) are removed; each leaves the
//    constant factor x_e = e^{J_e} because sigma_v == sigma_v always.  Parallel
//    edges are merged into one q x q matrix (elementwise product of the
//    interaction matrices, merged weight x_m = prod x_e).  With the Jones
//    couplings a merged class with as many + as - Tait signs has x_m = 1, an
//    all-ones matrix that couples nothing: that is the Reidemeister-II
//    "unpoke" and the edge is dropped.  A vertex of degree 1 (a spike) is
//    summed out: sum_b T(a, b) = x_m + q - 1 for every a, a constant factor.
//    A vertex of degree 0 contributes a factor q.
// 2. Tensor network (Sec. III, Eq. 5).  Every vertex carries a COPY tensor;
//    instead of materialising it, each merged edge matrix is absorbed into one
//    endpoint, so that a vertex tensor is indexed by spins:
//      F_v(s_v, s_w1, ..., s_wk) = prod_j T_{v wj}(s_v, s_wj).
//    Edges are oriented out of the endpoint that comes first in a
//    minimum-degree (degeneracy) order, which bounds k by the degeneracy of
//    the planar graph (<= 5).  A vertex spin that no other tensor mentions is
//    summed at build time.
// 3. Contraction order (Sec. III, "greedy").  Tensors that share a spin are
//    contracted pairwise; a spin is summed when the two operands are its last
//    holders, otherwise it stays as a batch index.  Each step is a batched
//    complex GEMM C[b,m,n] = sum_k A[b,m,k] B[b,k,n].  The greedy key is the
//    growth size(C) - size(A) - size(B) (strategy 0) or the rank of C
//    (strategy 1), ties broken by the flop count and then tensor ids.
// 4. Memory: first-fit arena over the tensors' live ranges.
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstring>
#include <map>
#include <new>
#include <memory>
#include <queue>
#include <set>
#include <unordered_map>

#include "decode.h"
#include "internal.h"

namespace kn {

int64_t elem_bytes(int32_t precision) { return precision == 1 ? 8 : 16; }

// Upper bound on the tiles of one step (a few per compute unit), and the
// multiply-adds one tile aims at.
constexpr double kMaxTiles = 1024;
constexpr double kMaxTileOutputs = 1 << 24;  // outputs of one tile (2^28 bytes in complex128)
constexpr int32_t kTileMacsLog2 = 15;    // multiply-adds a tile of outputs aims at
constexpr int32_t kTileOutsLog2 = 10;    // most outputs of one tile
constexpr int32_t kBigOutsLog2 = 12;     // steps with this many outputs are tiled

// Intermediate-size bucket of a step (its output C): at most 2^8, 2^12,
// 2^16, 2^20 entries, or more.
inline int32_t bucket_of(double outs) {
  int32_t b = 0;
  for (double lim = 256.0; b < KN_N_BUCKETS - 1 && outs > lim; lim *= 16.0) ++b;
  return b;
}
// Steps with fewer tiles than this split a long contracted index of nk
// entries, into at most nk / 2^kSplitMinLog2 segments: a task costs a few
// microseconds of claim, descriptor loads and release whatever its size, and
// the scalar products that end the workload's knots (3^9 to 3^12 contracted
// entries) ran fastest as segments of 2^12 to 2^13 (one 256-knot batch: 2.06
// ms with segments of 128 entries, 1.66 ms with 2^11, 1.64 ms with 2^12).
constexpr double kSplitBelow = 256;
constexpr int32_t kSplitMinLog2 = 12;
// Auto ordering also tries the greedy plan when the min-fill plan has at least
// this many flops (below it the greedy plan rarely wins and planning time
// matters more).
constexpr double kAutoGreedyFrom = 1e8;
// ... and separator orders when it has at least this many flops.
constexpr double kAutoSeparatorFrom = 1e11;
// Separator orders: hierarchies tried (default), their leaf sizes in turn,
// and search roots per split.
constexpr int32_t kSeparatorTrials = 12;
constexpr int32_t kSeparatorLeaf[3] = {8, 24, 64};
constexpr int32_t kSeparatorCandidates = 6;
// GEMM steps: tasks per step aimed at (log2) and most 32 x 32 blocks per task
constexpr int32_t kGemmTasksLog2 = 5;
constexpr int32_t kGemmMaxBlocks = 32;
// a GEMM step takes 64 x 64 blocks when their padded output count is at most
// this percentage of the 32 x 32 blocks' (both sides at least 64)
constexpr int32_t kGemm64Pct = 300;
// default threshold (log2 of the estimated time) above which a serial run is
// executed level by level over several workgroups
constexpr int32_t kSplitSerialLog2 = 40;
// ... and above which a run is forked into concurrent subtree tasks
// (measured on 256 knots of 200-600 crossings at q = 3: 2^10 shortens the
// launch by 4 % in complex128 and 7 % in complex64; 2^8-2^9 fork too many
// runs, 2^11 and above too few)
constexpr int32_t kForkSerialLog2 = 10;
// Slicing fixes at most this many spins, and makes at most kMaxSlices slices
// (the device runs the slices of a chain one after another from one copy of
// the knot's descriptors; the queue holds one slot per task and slice).
constexpr int32_t kMaxSliceSpins = 24;
// spins tried at each slicing step
constexpr int32_t kSliceCandidates = 4;
constexpr double kMaxSlices = 16777216;

namespace {

struct Simplified {
  int32_t n_spins = 0;                          // remaining spins (renumbered)
  std::vector<std::pair<int32_t, int32_t>> e;   // merged edges (spin ids)
  std::vector<int32_t> e_medge;                 // merged-edge id of each remaining edge
  // paper-model edge multiplicity of each remaining edge (for delta_h_paper)
  std::vector<int32_t> e_mult;
};

// Exact series-parallel reduction of the Potts network at the Jones couplings
// (their values are known at planning time), together with R-I on spikes.
// With T_e(a, b) = 1 + (x_e - 1) [a = b]:
//  - spike: a vertex on one edge m sums to the constant x_m + q - 1
//    (factor FAC_LEAF m);
//  - series: a vertex v on exactly two edges, x1 to u and x2 to w (u != w),
//    sums to c T'(s_u, s_w) with c = x1 + x2 + q - 2 and
//    x' = (x1 x2 + q - 1) / c, since for s_u = s_w the sum over s_v is
//    x1 x2 + (q - 1) and otherwise x1 + x2 + (q - 2);
//  - parallel: two edges between the same spins multiply their x.
// Series and parallel results are new merged edges whose x is a constant
// (k.consts, referenced by k.medge_const), c becomes a FAC_CONST factor.  A
// series step whose c is (nearly) zero is skipped.  Reductions repeat until
// every remaining spin has degree three or more.
void series_parallel(const kn_tait& g, PlanKnot& k, int32_t nv,
                     std::vector<std::pair<int32_t, int32_t>>& ends, std::vector<uint8_t>& alive_e,
                     std::vector<int32_t>& mult, const std::vector<int32_t>& ioff,
                     const std::vector<int32_t>& inc, std::vector<int32_t>& deg,
                     std::vector<uint8_t>& alive_v) {
  using C = std::complex<double>;
  const int32_t q = k.q;
  const C t(k.t_re, k.t_im);
  const int32_t nm = (int32_t)alive_e.size();
  // x of every merged edge: product of its members' Jones couplings -t^(-eps)
  std::vector<C> x(nm);
  for (int32_t m = 0; m < nm; ++m) {
    C v(1.0, 0.0);
    for (int32_t j = k.medge_off[m]; j < k.medge_off[m + 1]; ++j)
      v *= -(g.eps[k.medge_mem[j]] > 0 ? 1.0 / t : t);
    x[m] = v;
  }
  // live incident edges per spin (lists compacted lazily)
  std::vector<SpinList> adj(nv);
  for (int32_t v = 0; v < nv; ++v)
    for (int32_t j = ioff[v]; j < ioff[v + 1]; ++j) adj[v].push_back(inc[j]);
  auto live_edges = [&](int32_t v) -> const SpinList& {
    SpinList& l = adj[v];
    int32_t* h = l.mut();
    int32_t w = 0;
    for (int32_t i = 0; i < l.size(); ++i)
      if (alive_e[h[i]]) h[w++] = h[i];
    l.truncate(w);
    return l;
  };
  auto other = [&](int32_t m, int32_t v) { return ends[m].first == v ? ends[m].second : ends[m].first; };
  auto derived = [&](int32_t a, int32_t b, C val) {
    const int32_t m = (int32_t)alive_e.size();
    ends.emplace_back(std::min(a, b), std::max(a, b));
    alive_e.push_back(1);
    mult.push_back(1);
    x.push_back(val);
    k.medge_const.push_back((int32_t)k.consts.size());
    k.consts.push_back(val);
    k.medge_off.push_back(k.medge_off.back());  // no member edges
    adj[a].push_back(m);
    adj[b].push_back(m);
    return m;
  };
  std::vector<int32_t> stack;
  for (int32_t v = nv - 1; v >= 0; --v)
    if (deg[v] == 1 || deg[v] == 2) stack.push_back(v);
  while (!stack.empty()) {
    const int32_t v = stack.back();
    stack.pop_back();
    if (!alive_v[v] || deg[v] < 1 || deg[v] > 2) continue;
    const SpinList& l = live_edges(v);
    if (deg[v] == 1) {
      const int32_t m = l[0];
      alive_e[m] = 0;
      k.factors.push_back({FAC_LEAF, m});
      alive_v[v] = 0;
      deg[v] = 0;
      const int32_t w = other(m, v);
      if (--deg[w] == 1 || deg[w] == 2) stack.push_back(w);
      continue;
    }
    const int32_t m1 = l[0], m2 = l[1];
    const int32_t u = other(m1, v), w = other(m2, v);
    if (u == w) continue;  // cannot happen: parallel edges are merged
    const C c = x[m1] + x[m2] + (double)(q - 2);
    if (std::abs(c) <= 1e-9 * (std::abs(x[m1] * x[m2]) + (double)q)) continue;
    const C xs = (x[m1] * x[m2] + (double)(q - 1)) / c;
    alive_e[m1] = alive_e[m2] = 0;
    alive_v[v] = 0;
    deg[v] = 0;
    k.factors.push_back({FAC_CONST, (int32_t)k.consts.size()});
    k.consts.push_back(c);
    // an existing edge u - w absorbs the new one (parallel merge)
    int32_t m3 = -1;
    for (int32_t e : live_edges(u))
      if (other(e, u) == w) m3 = e;
    if (m3 >= 0) {
      alive_e[m3] = 0;
      derived(u, w, xs * x[m3]);
      --deg[u];
      --deg[w];
    } else {
      derived(u, w, xs);
    }
    for (int32_t z : {u, w})
      if (deg[z] == 1 || deg[z] == 2) stack.push_back(z);
  }
}

// Simplification of Sec. III.A; fills k.medges, k.factors, k.n_iso.
Simplified simplify(const kn_tait& g, int32_t flags, bool jones_only, PlanKnot& k) {
  const int32_t nv = g.n_vertices;
  const int32_t ne = (int32_t)g.eps.size();
  bool r1 = flags & 1, r2 = (flags & 2) && jones_only;
  // merge parallel classes; loops become factors (or stay as loops when R-I
  // is off: they are still constants, a loop never couples two spins)
  // (u * nv + v, edge) with u < v, sorted by key then edge: two stable
  // counting sorts, by v and then by u
  std::vector<std::pair<int64_t, int32_t>> keyed;
  {
    std::vector<int32_t> by_v, cnt(nv + 1, 0);
    by_v.reserve(ne);
    for (int32_t e = 0; e < ne; ++e) {
      const int32_t u = g.uv[2 * e], v = g.uv[2 * e + 1];
      if (u == v) {
        k.factors.push_back({FAC_LOOP, e});
        continue;
      }
      cnt[std::max(u, v) + 1]++;
      by_v.push_back(e);
    }
    for (int32_t v = 0; v < nv; ++v) cnt[v + 1] += cnt[v];
    std::vector<int32_t> tmp(by_v.size());
    for (int32_t e : by_v) tmp[cnt[std::max(g.uv[2 * e], g.uv[2 * e + 1])]++] = e;
    std::fill(cnt.begin(), cnt.end(), 0);
    for (int32_t e : tmp) cnt[std::min(g.uv[2 * e], g.uv[2 * e + 1]) + 1]++;
    for (int32_t v = 0; v < nv; ++v) cnt[v + 1] += cnt[v];
    keyed.resize(tmp.size());
    for (int32_t e : tmp) {
      const int32_t u = g.uv[2 * e], v = g.uv[2 * e + 1];
      keyed[cnt[std::min(u, v)]++] = {(int64_t)std::min(u, v) * nv + std::max(u, v), e};
    }
  }
  std::vector<std::pair<int32_t, int32_t>> ends;
  k.medge_off.assign(1, 0);
  k.medge_mem.clear();
  k.medge_mem.reserve(keyed.size());
  for (size_t i = 0; i < keyed.size(); ++i) {
    if (i > 0 && keyed[i].first != keyed[i - 1].first)
      k.medge_off.push_back((int32_t)k.medge_mem.size());
    if (i == 0 || keyed[i].first != keyed[i - 1].first)
      ends.emplace_back((int32_t)(keyed[i].first / nv), (int32_t)(keyed[i].first % nv));
    k.medge_mem.push_back(keyed[i].second);
  }
  if (!keyed.empty()) k.medge_off.push_back((int32_t)k.medge_mem.size());
  (void)r1;
  const int32_t nm = (int32_t)k.medge_off.size() - 1;
  std::vector<uint8_t> alive_e(nm, 1);
  std::vector<int32_t> mult(nm);
  for (int32_t m = 0; m < nm; ++m) {
    int32_t s = 0;
    for (int32_t j = k.medge_off[m]; j < k.medge_off[m + 1]; ++j) s += g.eps[k.medge_mem[j]];
    mult[m] = r2 ? std::abs(s) : k.medge_off[m + 1] - k.medge_off[m];
    if (r2 && s == 0) alive_e[m] = 0;  // Reidemeister II: x_m = 1
  }
  // incidence over live merged edges, in compressed rows
  std::vector<int32_t> ioff(nv + 1, 0), inc;
  for (int32_t m = 0; m < nm; ++m)
    if (alive_e[m]) {
      ioff[ends[m].first + 1]++;
      ioff[ends[m].second + 1]++;
    }
  for (int32_t v = 0; v < nv; ++v) ioff[v + 1] += ioff[v];
  inc.resize(ioff[nv]);
  {
    std::vector<int32_t> fp(ioff.begin(), ioff.end() - 1);
    for (int32_t m = 0; m < nm; ++m)
      if (alive_e[m]) {
        inc[fp[ends[m].first]++] = m;
        inc[fp[ends[m].second]++] = m;
      }
  }
  std::vector<int32_t> deg(nv);
  for (int32_t v = 0; v < nv; ++v) deg[v] = ioff[v + 1] - ioff[v];
  std::vector<uint8_t> alive_v(nv, 1);
  k.medge_const.assign(nm, -1);
  k.consts.clear();
  if ((flags & 4) && jones_only) {
    series_parallel(g, k, nv, ends, alive_e, mult, ioff, inc, deg, alive_v);
  } else if (flags & 1) {
    // Reidemeister I on spikes: peel degree-1 vertices repeatedly
    std::vector<int32_t> stack;
    for (int32_t v = 0; v < nv; ++v)
      if (deg[v] == 1) stack.push_back(v);
    while (!stack.empty()) {
      int32_t v = stack.back();
      stack.pop_back();
      if (!alive_v[v] || deg[v] != 1) continue;
      int32_t m = -1;
      for (int32_t j = ioff[v]; j < ioff[v + 1]; ++j)
        if (alive_e[inc[j]]) { m = inc[j]; break; }
      if (m < 0) continue;
      alive_e[m] = 0;
      k.factors.push_back({FAC_LEAF, m});
      alive_v[v] = 0;
      int32_t w = ends[m].first == v ? ends[m].second : ends[m].first;
      deg[v] = 0;
      if (--deg[w] == 1) stack.push_back(w);
    }
  }
  // isolated vertices and renumbering
  Simplified s;
  std::vector<int32_t> sid(nv, -1);
  for (int32_t v = 0; v < nv; ++v) {
    if (!alive_v[v]) continue;
    if (deg[v] == 0) {
      k.n_iso++;
      continue;
    }
    sid[v] = s.n_spins++;
  }
  for (int32_t m = 0; m < (int32_t)alive_e.size(); ++m)
    if (alive_e[m]) {
      s.e.emplace_back(sid[ends[m].first], sid[ends[m].second]);
      s.e_medge.push_back(m);
      s.e_mult.push_back(mult[m]);
    }
  return s;
}

// Max degree over the minors of the paper's greedy edge contraction on the
// multigraph (each merged edge counted with its multiplicity), Sec. III:
// repeatedly contract the edge whose merged vertex has the smallest degree
// deg(u) + deg(v) - 2 mult(u, v).  Merging u and v leaves every other
// vertex's degree unchanged, so only candidates at the merged vertex change;
// stale heap entries are skipped by a per-vertex version stamp.
int32_t paper_delta_h(const Simplified& s) {
  const int32_t n = s.n_spins;
  std::vector<std::unordered_map<int32_t, int32_t>> adj(n);
  std::vector<int32_t> deg(n, 0), ver(n, 0), rep(n);
  for (int32_t v = 0; v < n; ++v) rep[v] = v;
  for (size_t i = 0; i < s.e.size(); ++i) {
    auto [u, v] = s.e[i];
    int32_t w = std::max(1, s.e_mult[i]);
    adj[u][v] += w;
    adj[v][u] += w;
    deg[u] += w;
    deg[v] += w;
  }
  int32_t best = 0;
  for (int32_t v = 0; v < n; ++v) best = std::max(best, deg[v]);
  struct E {
    int32_t d, u, v, vu, vv;
    bool operator<(const E& o) const {
      if (d != o.d) return d > o.d;
      if (u != o.u) return u > o.u;
      return v > o.v;
    }
  };
  std::priority_queue<E> pq;
  auto push = [&](int32_t u, int32_t v, int32_t m) {
    if (u > v) std::swap(u, v);
    pq.push({deg[u] + deg[v] - 2 * m, u, v, ver[u], ver[v]});
  };
  for (int32_t u = 0; u < n; ++u)
    for (auto& [v, m] : adj[u])
      if (v > u) push(u, v, m);
  while (!pq.empty()) {
    E e = pq.top();
    pq.pop();
    if (e.vu != ver[e.u] || e.vv != ver[e.v]) continue;
    auto it = adj[e.u].find(e.v);
    if (it == adj[e.u].end()) continue;
    // merge the smaller adjacency into the larger
    int32_t a = e.u, b = e.v;
    if (adj[a].size() < adj[b].size()) std::swap(a, b);
    int32_t m_ab = adj[a][b];
    adj[a].erase(b);
    adj[b].erase(a);
    for (auto& [w, m] : adj[b]) {
      adj[w].erase(b);
      adj[w][a] += m;
      adj[a][w] += m;
    }
    adj[b].clear();
    deg[a] = deg[a] + deg[b] - 2 * m_ab;
    deg[b] = 0;
    ver[a]++;
    ver[b]++;
    best = std::max(best, deg[a]);
    for (auto& [w, m] : adj[a]) push(a, w, m);
  }
  return best;
}

struct Cand {
  double k1, k2;
  int32_t a, b;
  bool operator<(const Cand& o) const {  // max-heap: "less" = worse
    if (k1 != o.k1) return k1 > o.k1;
    if (k2 != o.k2) return k2 > o.k2;
    if (a != o.a) return a > o.a;
    return b > o.b;
  }
};

// Pairwise contraction of spin-indexed tensors.  A spin is summed when the two
// operands are its last holders (cnt == 2); otherwise it stays as a batch
// index of the result.
struct Orderer {
  int32_t n, q;
  std::vector<PTensor> T;
  std::vector<PStep> S;
  std::vector<int32_t> cnt;
  std::vector<SpinList> hold;  // live holders of each spin (lazily compacted)
  std::vector<uint8_t> alive;
  std::vector<uint32_t> mark;
  uint32_t stamp = 0;
  std::vector<double> qpow;

  Orderer(int32_t n_, int32_t q_, const std::vector<PTensor>& init)
      : n(n_), q(q_), T(init), cnt(n_, 0), hold(n_), alive(init.size(), 1), mark(n_, 0),
        qpow(64) {
    T.reserve(2 * init.size() + 1);
    S.reserve(init.size() + 1);
    alive.reserve(2 * init.size() + 1);
    for (int32_t t = 0; t < (int32_t)T.size(); ++t)
      for (int32_t sp : T[t].spins) {
        cnt[sp]++;
        hold[sp].push_back(t);
      }
    qpow[0] = 1;
    for (int i = 1; i < 64; ++i) qpow[i] = qpow[i - 1] * q;
  }

  // rank of the result and of the union
  void ranks(int32_t a, int32_t b, int32_t& rc, int32_t& uni) {
    const auto& A = T[a].spins;
    const auto& B = T[b].spins;
    ++stamp;
    for (int32_t x : A) mark[x] = stamp;
    int32_t kk = 0;
    uni = (int32_t)A.size();
    for (int32_t x : B) {
      if (mark[x] != stamp) uni++;
      else if (cnt[x] == 2) kk++;
    }
    rc = uni - kk;
  }

  int32_t contract(int32_t a, int32_t b) {
    // the larger operand first (its private spins are the GEMM rows)
    if (T[b].spins.size() > T[a].spins.size()) std::swap(a, b);
    PStep stp;
    stp.a = a;
    stp.b = b;
    {
      const auto& A = T[a].spins;
      const auto& B = T[b].spins;
      ++stamp;
      for (int32_t x : B) mark[x] = stamp;
      for (int32_t x : A) {
        if (mark[x] != stamp) stp.ms.push_back(x);
        else if (cnt[x] == 2) stp.ks.push_back(x);
        else stp.bs.push_back(x);
      }
      ++stamp;
      for (int32_t x : A) mark[x] = stamp;
      for (int32_t x : B)
        if (mark[x] != stamp) stp.ns.push_back(x);
    }
    PTensor ct;
    ct.spins.reserve(stp.bs.size() + stp.ms.size() + stp.ns.size());
    for (int32_t x : stp.bs) ct.spins.push_back(x);
    for (int32_t x : stp.ms) ct.spins.push_back(x);
    for (int32_t x : stp.ns) ct.spins.push_back(x);
    int32_t cid = (int32_t)T.size();
    stp.c = cid;
    for (int32_t x : stp.ks) cnt[x] = 0;
    for (int32_t x : stp.bs) cnt[x]--;
    alive[a] = alive[b] = 0;
    alive.push_back(1);
    for (int32_t x : ct.spins) hold[x].push_back(cid);
    T.push_back(std::move(ct));
    S.push_back(std::move(stp));
    return cid;
  }

  // live holders of spin x (compacts the list)
  const SpinList& holders(int32_t x) {
    SpinList& hl = hold[x];
    int32_t* h = hl.mut();
    int32_t w = 0;
    for (int32_t i = 0; i < hl.size(); ++i)
      if (alive[h[i]]) h[w++] = h[i];
    hl.truncate(w);
    return hl;
  }

  // Greedy: contract the pair (sharing a spin) with the smallest key.
  // strategy 0: size(C) - size(A) - size(B); 1: rank(C).  Ties: flops, ids.
  void greedy(int32_t strategy) {
    std::vector<uint32_t> seen(2 * T.size() + 2, 0);
    uint32_t tstamp = 0;
    auto cost = [&](int32_t a, int32_t b, Cand& c) {
      int32_t rc, uni;
      ranks(a, b, rc, uni);
      if (strategy == 1) c.k1 = rc;
      else c.k1 = qpow[std::min(rc, 63)] - qpow[T[a].spins.size()] - qpow[T[b].spins.size()];
      c.k2 = qpow[std::min(uni, 63)];
      c.a = std::min(a, b);
      c.b = std::max(a, b);
    };
    // a binary heap (std::less<Cand>: top = best) with lazy deletion; pairs
    // of contracted tensors are swept out in bulk every few contractions
    std::vector<Cand> heap;
    heap.reserve(16 * T.size() + 16);
    auto push = [&](const Cand& c) {
      heap.push_back(c);
      std::push_heap(heap.begin(), heap.end());
    };
    auto push_pairs = [&](int32_t a) {
      if ((size_t)a >= seen.size()) seen.resize(2 * a + 2, 0);
      ++tstamp;
      seen[a] = tstamp;
      for (int32_t sp : T[a].spins)
        for (int32_t b : holders(sp)) {
          if (seen[b] == tstamp) continue;
          seen[b] = tstamp;
          Cand c;
          cost(a, b, c);
          push(c);
        }
    };
    const int32_t n0 = (int32_t)T.size();
    for (int32_t t = 0; t < n0; ++t) push_pairs(t);
    int32_t since_sweep = 0;
    while (!heap.empty()) {
      std::pop_heap(heap.begin(), heap.end());
      const Cand c = heap.back();
      heap.pop_back();
      if (!alive[c.a] || !alive[c.b]) continue;
      Cand fresh;
      cost(c.a, c.b, fresh);
      if (fresh.k1 != c.k1 || fresh.k2 != c.k2) {  // counts changed since the push
        push(fresh);
        continue;
      }
      push_pairs(contract(c.a, c.b));
      if (++since_sweep == 16) {
        since_sweep = 0;
        heap.erase(std::remove_if(heap.begin(), heap.end(),
                                  [&](const Cand& x) { return !alive[x.a] || !alive[x.b]; }),
                   heap.end());
        std::make_heap(heap.begin(), heap.end());
      }
    }
  }

  // Variable elimination in min-fill order on the primal graph of the tensors
  // (spins adjacent when some tensor holds both); eliminating a spin contracts
  // its holders pairwise, smallest first, and the last pair sums it.
  //
  // With `rank` (one value per spin), spins are eliminated in increasing rank
  // and by least fill inside a rank: the order of a separator hierarchy.
  void minfill(const std::vector<int32_t>* rank = nullptr) {
    const int32_t W = (n + 63) / 64;
    std::vector<uint64_t> adj((size_t)n * W, 0);
    auto has = [&](int32_t a, int32_t b) { return (adj[(size_t)a * W + (b >> 6)] >> (b & 63)) & 1; };
    auto set = [&](int32_t a, int32_t b) {
      adj[(size_t)a * W + (b >> 6)] |= uint64_t(1) << (b & 63);
      adj[(size_t)b * W + (a >> 6)] |= uint64_t(1) << (a & 63);
    };
    for (const auto& t : T)
      for (size_t i = 0; i < t.spins.size(); ++i)
        for (size_t j = i + 1; j < t.spins.size(); ++j) set(t.spins[i], t.spins[j]);
    std::vector<int32_t> fill(n, 0), deg(n, 0);
    std::vector<int32_t> nb;
    auto neigh = [&](int32_t v, std::vector<int32_t>& out) {
      out.clear();
      for (int32_t w = 0; w < W; ++w) {
        uint64_t m = adj[(size_t)v * W + w];
        while (m) {
          int b = __builtin_ctzll(m);
          m &= m - 1;
          out.push_back(w * 64 + b);
        }
      }
    };
    auto eval = [&](int32_t v) {
      neigh(v, nb);
      deg[v] = (int32_t)nb.size();
      int64_t missing = 0;
      for (int32_t a : nb) {
        // neighbours of v not adjacent to a (a itself included once)
        int64_t c = 0;
        for (int32_t w = 0; w < W; ++w)
          c += __builtin_popcountll(adj[(size_t)v * W + w] & ~adj[(size_t)a * W + w]);
        missing += c - 1;
      }
      fill[v] = (int32_t)(missing / 2);
    };
    for (int32_t v = 0; v < n; ++v) eval(v);
    std::vector<int32_t> nv, touched;
    std::vector<uint32_t> tmark(n, 0);
    std::vector<uint64_t> xm(W, 0);  // N(x) + x as a bit set
    uint32_t ts = 0;
    // next spin: lowest rank, then least fill, then least degree, then
    // lowest id (a linear scan over packed keys, which for a few hundred
    // spins measured faster than a heap) over the spins still in the graph,
    // kept packed: key[slot[v]] is v's.  Fields: rank 10 bits, fill 22,
    // degree 11, id 21 (fill and degree saturate).
    std::vector<uint64_t> key(n);
    std::vector<int32_t> slot(n);
    int32_t live = n;
    auto pack = [&](int32_t v) {
      const uint64_t r = rank ? (uint64_t)std::min((*rank)[v], 1023) : 0;
      const uint64_t f = (uint64_t)std::min(fill[v], (1 << 22) - 1);
      const uint64_t d = (uint64_t)std::min(deg[v], (1 << 11) - 1);
      key[slot[v]] = r << 54 | f << 32 | d << 21 | (uint64_t)v;
    };
    for (int32_t v = 0; v < n; ++v) {
      slot[v] = v;
      pack(v);
    }
    constexpr uint64_t kIdMask = (uint64_t(1) << 21) - 1;
    for (int32_t it = 0; it < n; ++it) {
      uint64_t best = UINT64_MAX;
      for (int32_t i = 0; i < live; ++i) best = std::min(best, key[i]);
      const int32_t x = best == UINT64_MAX ? -1 : (int32_t)(best & kIdMask);
      if (x < 0) break;
      // contract the holders of x pairwise, smallest first
      if (cnt[x] > 0) {
        for (;;) {
          const SpinList& hl = holders(x);
          if (hl.size() < 2) break;
          int32_t a = -1, b = -1;
          for (int32_t t : hl) {
            if (a < 0 || T[t].spins.size() < T[a].spins.size()) {
              b = a;
              a = t;
            } else if (b < 0 || T[t].spins.size() < T[b].spins.size()) {
              b = t;
            }
          }
          contract(a, b);
        }
      }
      // eliminate x from the graph: its neighbours become a clique, then x
      // leaves.  Fill counts are kept exact incrementally.  Adding an edge
      // (u, w): each common neighbour z has that pair of N(z) joined
      // (fill - 1); u gains the pairs {w, y}, y in N(u) \ N(w) (and the same
      // for w).  Removing x: a neighbour a loses the pairs {x, y}, y in
      // N(a) not adjacent to x, i.e. outside N(x) + x once N(x) is a clique.
      neigh(x, nv);
      std::fill(xm.begin(), xm.end(), 0);
      for (int32_t a : nv) xm[a >> 6] |= uint64_t(1) << (a & 63);
      xm[x >> 6] |= uint64_t(1) << (x & 63);
      ++ts;
      for (size_t i = 0; i < nv.size(); ++i)
        for (size_t j = i + 1; j < nv.size(); ++j) {
          const int32_t u = nv[i], w = nv[j];
          if (has(u, w)) continue;
          const uint64_t* au = &adj[(size_t)u * W];
          const uint64_t* aw = &adj[(size_t)w * W];
          int32_t du = 0, dw = 0;
          for (int32_t ww = 0; ww < W; ++ww) {
            du += __builtin_popcountll(au[ww] & ~aw[ww]);
            dw += __builtin_popcountll(aw[ww] & ~au[ww]);
            uint64_t m = au[ww] & aw[ww];
            while (m) {
              const int32_t z = ww * 64 + __builtin_ctzll(m);
              m &= m - 1;
              --fill[z];
              if (tmark[z] != ts) {
                tmark[z] = ts;
                touched.push_back(z);
              }
            }
          }
          fill[u] += du;
          fill[w] += dw;
          ++deg[u];
          ++deg[w];
          set(u, w);
        }
      for (int32_t a : nv) {
        const uint64_t* aa = &adj[(size_t)a * W];
        int32_t c = 0;
        for (int32_t ww = 0; ww < W; ++ww) c += __builtin_popcountll(aa[ww] & ~xm[ww]);
        fill[a] -= c;
        --deg[a];
        adj[(size_t)a * W + (x >> 6)] &= ~(uint64_t(1) << (x & 63));
      }
      for (int32_t w = 0; w < W; ++w) adj[(size_t)x * W + w] = 0;
      {  // x leaves the packed keys: the last one takes its place
        const int32_t i = slot[x], last = (int32_t)(key[live - 1] & kIdMask);
        key[i] = key[live - 1];
        slot[last] = i;
        --live;
      }
      for (int32_t z : touched)
        if (z != x) pack(z);
      for (int32_t a : nv) pack(a);
      touched.clear();
    }
  }

  // Primal graph of the tensors (spins adjacent when some tensor holds
  // both) in compressed rows.
  void primal(std::vector<int32_t>& off, std::vector<int32_t>& nb) const {
    std::vector<std::pair<int32_t, int32_t>> e;
    for (const auto& t : T)
      for (int32_t i = 0; i < t.spins.size(); ++i)
        for (int32_t j = 0; j < t.spins.size(); ++j)
          if (i != j) e.emplace_back(t.spins[i], t.spins[j]);
    std::sort(e.begin(), e.end());
    e.erase(std::unique(e.begin(), e.end()), e.end());
    off.assign(n + 1, 0);
    nb.resize(e.size());
    for (size_t i = 0; i < e.size(); ++i) {
      off[e[i].first + 1]++;
      nb[i] = e[i].second;
    }
    for (int32_t v = 0; v < n; ++v) off[v + 1] += off[v];
  }

  // 8 flops per complex multiply-add over all steps.
  double flops() const {
    double f = 0;
    for (const auto& st : S)
      f += 8.0 * qpow[std::min<size_t>(st.bs.size() + st.ms.size() + st.ns.size() + st.ks.size(),
                                       63)];
    return f;
  }

  // Roofline-modelled time of the plan: per step max(flops/peak, bytes/bw),
  // plus a fixed per-step latency when `latency`.
  double model_cost(int32_t precision, bool latency) const {
    const double peak = precision == 1 ? 157.3e12 : 78.6e12, bw = 8.0e12, lat = 0.3e-6;
    const double es = precision == 1 ? 8 : 16;
    double t = 0;
    for (const auto& st : S) {
      double macs = qpow[std::min<size_t>(st.bs.size() + st.ms.size() + st.ns.size() +
                                              st.ks.size(), 63)];
      double by = es * (qpow[std::min<size_t>(T[st.a].spins.size(), 63)] +
                        qpow[std::min<size_t>(T[st.b].spins.size(), 63)] +
                        qpow[std::min<size_t>(T[st.c].spins.size(), 63)]);
      t += std::max(8.0 * macs / peak, by / bw) + (latency ? lat : 0.0);
    }
    return t;
  }
};

}  // namespace

// Reverse pass of the contraction for d log Z / d J.  For every component a
// seed tensor (the scalar 1) becomes dS/dS of its final scalar S; the forward
// steps are then walked backwards and each C = A . B (batch b, rows m, cols
// n, contracted k) adds two steps of the same kind:
//   dS/dA[b,m,k] = sum_n dS/dC[b,m,n] B[b,k,n]   (rows m, cols k, contracted n)
//   dS/dB[b,k,n] = sum_m A[b,m,k] dS/dC[b,m,n]   (rows k, cols n, contracted m)
// Seeds are numbered after the vertex tensors (n_vt grows by the number of
// components) so that step i still produces tensor n_vt + i.  Each vertex
// learns the id of its adjoint and its component.
void add_reverse(PlanKnot& k, int32_t& n_vt, int32_t drop_rank, int32_t max_depth,
                 int32_t& n_recompute) {
  const int32_t nc = (int32_t)k.comps.size();
  const int32_t ns = (int32_t)k.steps.size();
  n_recompute = 0;
  auto shifted = [&](int32_t t) { return t < n_vt ? t : t + nc; };
  std::vector<PTensor> tensors;
  tensors.reserve(k.tensors.size() + nc + 2 * ns);
  for (int32_t t = 0; t < n_vt; ++t) tensors.push_back(std::move(k.tensors[t]));
  for (int32_t c = 0; c < nc; ++c) tensors.emplace_back();  // seed: no spins, one entry
  for (size_t t = n_vt; t < k.tensors.size(); ++t) tensors.push_back(std::move(k.tensors[t]));
  for (auto& st : k.steps) {
    st.a = shifted(st.a);
    st.b = shifted(st.b);
    st.c = shifted(st.c);
  }
  for (auto& c : k.comps) c = shifted(c);
  for (int32_t c = 0; c < nc; ++c) {
    PVertex pv;
    pv.tensor = n_vt + c;
    pv.center = -1;
    pv.keep_center = false;
    pv.seed = true;
    pv.comp = c;
    k.vtx.push_back(std::move(pv));
  }
  n_vt += nc;
  const size_t total = tensors.size();
  std::vector<int32_t> adj(total, -1), comp(total, 0);
  for (int32_t c = 0; c < nc; ++c) {
    adj[k.comps[c]] = n_vt - nc + c;
    comp[k.comps[c]] = c;
  }
  // Checkpoints: the output of a forward step whose rank is at least
  // drop_rank is dropped after its forward use (its arena is reused) and
  // computed again from its operands just before the reverse step that reads
  // it, unless that would chain more than max_depth dropped steps (then it is
  // kept).  Component scalars are always kept.
  std::vector<int32_t> producer(total, -1);
  std::vector<uint8_t> depth(total, 0), dropped(total, 0), keep(total, 0);
  for (int32_t c : k.comps) keep[c] = 1;
  for (int32_t s = 0; s < ns; ++s) {
    const PStep& fw = k.steps[s];
    producer[fw.c] = s;
    if (keep[fw.c] || tensors[fw.c].spins.size() < drop_rank) continue;
    const int32_t d = 1 + std::max(depth[fw.a], depth[fw.b]);
    if (d > max_depth) continue;
    dropped[fw.c] = 1;
    depth[fw.c] = (uint8_t)d;
  }
  // a dropped tensor's fresh copy: its step again, on fresh copies of its
  // dropped operands (new tensor ids, the same spins in the same order)
  std::function<int32_t(int32_t)> remat = [&](int32_t x) -> int32_t {
    if (!dropped[x]) return x;
    PStep r = k.steps[producer[x]];
    r.a = remat(r.a);
    r.b = remat(r.b);
    r.c = (int32_t)tensors.size();
    PTensor t;
    t.spins = tensors[x].spins;
    tensors.push_back(std::move(t));
    adj.push_back(-1);
    comp.push_back(0);
    k.steps.push_back(std::move(r));
    ++n_recompute;
    return (int32_t)tensors.size() - 1;
  };
  k.steps.reserve(3 * (size_t)ns);
  for (int32_t s = ns - 1; s >= 0; --s) {
    const PStep fw = k.steps[s];
    const int32_t cbar = adj[fw.c];
    const int32_t fa = remat(fw.a), fb = remat(fw.b);
    PStep ra;  // dS/dA
    ra.a = cbar;
    ra.b = fb;
    ra.bs = fw.bs;
    ra.ms = fw.ms;
    ra.ns = fw.ks;
    ra.ks = fw.ns;
    PStep rb;  // dS/dB
    rb.a = fa;
    rb.b = cbar;
    rb.bs = fw.bs;
    rb.ms = fw.ks;
    rb.ns = fw.ns;
    rb.ks = fw.ms;
    for (PStep* r : {&ra, &rb}) {
      r->c = (int32_t)tensors.size();
      PTensor t;
      for (int32_t x : r->bs) t.spins.push_back(x);
      for (int32_t x : r->ms) t.spins.push_back(x);
      for (int32_t x : r->ns) t.spins.push_back(x);
      tensors.push_back(std::move(t));
      adj.push_back(-1);
      comp.push_back(0);
    }
    adj[fw.a] = ra.c;
    adj[fw.b] = rb.c;
    comp[fw.a] = comp[fw.b] = comp[fw.c];
    k.steps.push_back(std::move(ra));
    k.steps.push_back(std::move(rb));
  }
  for (auto& v : k.vtx)
    if (!v.seed) {
      v.adjoint = adj[v.tensor];
      v.comp = comp[v.tensor];
    }
  k.tensors = std::move(tensors);
}

// Serial steps that depend on each other only through earlier levels run
// concurrently on the waves of one workgroup.  Every maximal run of serial
// steps is reordered by dependency level (1 + the highest level among the
// producers of its operands inside the run; stable within a level), and the
// tensors are renumbered so that step i still produces tensor n_vt + i.
// Estimated time of a serial step: one unit per step plus one per 512
// multiply-adds (the unit the image builder uses for its runs).
double serial_est(const PStep& s, int32_t q) {
  double macs = 1;
  for (size_t r = 0; r < s.bs.size() + s.ms.size() + s.ns.size() + s.ks.size(); ++r) macs *= q;
  return 1.0 + macs / 512.0;
}

// Fork of a serial run: in a plain plan every intermediate is read by one
// step only, so the run's steps form a forest (a step's children are the
// steps of the run that produce its operands).  The heaviest subtrees are
// split at their root until every remaining subtree weighs at most 1/8 of
// the run; the split roots form the top, and the remaining subtrees are
// packed into at most kForkTasks tasks by weight (largest first, each to the
// lightest task).  part[u - i] receives the task of step u, or kForkTop.
// Returns false (no fork) when fewer than two tasks would result.
constexpr int32_t kForkTasks = 8;

bool fork_run(const PlanKnot& k, int32_t n_vt, int32_t i, int32_t j, std::vector<int32_t>& part) {
  const int32_t n = j - i;
  std::vector<int32_t> ch0(n, -1), ch1(n, -1);
  std::vector<uint8_t> used(n, 0);
  std::vector<double> w(n, 0.0);
  for (int32_t u = i; u < j; ++u) {
    int32_t nc = 0;
    for (int32_t op : {k.steps[u].a, k.steps[u].b}) {
      const int32_t ps = op - n_vt;
      if (ps < i || ps >= u) continue;
      if (used[ps - i]) return false;  // read twice: not a forest
      used[ps - i] = 1;
      (nc++ == 0 ? ch0 : ch1)[u - i] = ps - i;
    }
    w[u - i] = serial_est(k.steps[u], k.q) + (ch0[u - i] >= 0 ? w[ch0[u - i]] : 0.0) +
               (ch1[u - i] >= 0 ? w[ch1[u - i]] : 0.0);
  }
  double total = 0;
  std::vector<std::pair<double, int32_t>> heap;  // max-heap of subtree roots by weight
  for (int32_t u = 0; u < n; ++u)
    if (!used[u]) {
      heap.emplace_back(w[u], u);
      total += w[u];
    }
  std::make_heap(heap.begin(), heap.end());
  part.assign(n, -1);
  const double cap = total / kForkTasks;
  for (int32_t splits = 0; !heap.empty() && heap.front().first > cap && splits < 4 * kForkTasks;
       ++splits) {
    std::pop_heap(heap.begin(), heap.end());
    const int32_t u = heap.back().second;
    heap.pop_back();
    part[u] = kForkTop;
    for (int32_t c : {ch0[u], ch1[u]})
      if (c >= 0) {
        heap.emplace_back(w[c], c);
        std::push_heap(heap.begin(), heap.end());
      }
  }
  std::sort(heap.begin(), heap.end(), [](const std::pair<double, int32_t>& x,
                                         const std::pair<double, int32_t>& y) {
    return x.first != y.first ? x.first > y.first : x.second < y.second;
  });
  const int32_t n_tasks = std::min<int32_t>(kForkTasks, (int32_t)heap.size());
  if (n_tasks < 2) return false;
  std::vector<double> load(n_tasks, 0.0);
  std::vector<int32_t> stack;
  for (const auto& [wr, r] : heap) {
    const int32_t t = (int32_t)(std::min_element(load.begin(), load.end()) - load.begin());
    load[t] += wr;
    stack.push_back(r);
    while (!stack.empty()) {  // the subtree of r, all to task t
      const int32_t u = stack.back();
      stack.pop_back();
      part[u] = t;
      for (int32_t c : {ch0[u], ch1[u]})
        if (c >= 0) stack.push_back(c);
    }
  }
  return true;
}

void level_schedule(PlanKnot& k, int32_t n_vt) {
  const int32_t ns = (int32_t)k.steps.size();
  std::vector<int32_t> order;
  order.reserve(ns);
  std::vector<int32_t> lvl(ns, 0);    // by old step index
  std::vector<int32_t> prt(ns, -1);   // fork task by old step index
  std::vector<int32_t> fpart;
  for (int32_t i = 0; i < ns;) {
    if (k.tiling[i].mode != STEP_SERIAL) {
      order.push_back(i++);
      continue;
    }
    int32_t j = i;
    while (j < ns && k.tiling[j].mode == STEP_SERIAL) ++j;
    double est = 0;
    for (int32_t u = i; u < j; ++u) est += serial_est(k.steps[u], k.q);
    const bool forked = !k.gradient && est >= k.fork_est && fork_run(k, n_vt, i, j, fpart);
    if (forked)
      for (int32_t u = i; u < j; ++u) prt[u] = fpart[u - i];
    // levels inside each task of the run (operands made by another task or
    // before the run count as ready)
    int32_t top = 0;
    for (int32_t u = i; u < j; ++u) {
      int32_t l = 0;
      for (int32_t op : {k.steps[u].a, k.steps[u].b}) {
        const int32_t ps = op - n_vt;  // producing step
        if (ps >= i && ps < u && prt[ps] == prt[u]) l = std::max(l, lvl[ps]);
      }
      lvl[u] = l + 1;
      top = std::max(top, l + 1);
    }
    // counting sort by (task, level) keeps the original order within a level;
    // the tasks in turn, the top last
    const int32_t n_keys = forked ? kForkTasks + 1 : 1;
    auto key = [&](int32_t u) {
      const int32_t t = prt[u] < 0 ? 0 : (prt[u] == kForkTop ? kForkTasks : prt[u]);
      return t * (top + 1) + lvl[u];
    };
    std::vector<int32_t> cnt((size_t)n_keys * (top + 1) + 1, 0);
    for (int32_t u = i; u < j; ++u) cnt[key(u) + 1]++;
    for (size_t l = 1; l < cnt.size(); ++l) cnt[l] += cnt[l - 1];
    const size_t base = order.size();
    order.resize(base + (j - i));
    for (int32_t u = i; u < j; ++u) order[base + cnt[key(u)]++] = u;
    i = j;
  }
  std::vector<int32_t> pos(ns);
  for (int32_t r = 0; r < ns; ++r) pos[order[r]] = r;
  auto remap = [&](int32_t t) { return t < n_vt ? t : n_vt + pos[t - n_vt]; };
  std::vector<PStep> steps(ns);
  std::vector<PTiling> tiling(ns);
  std::vector<PTensor> tensors(k.tensors.size());
  for (int32_t t = 0; t < n_vt; ++t) tensors[t] = std::move(k.tensors[t]);
  for (int32_t r = 0; r < ns; ++r) {
    const int32_t u = order[r];
    PStep st = std::move(k.steps[u]);
    st.a = remap(st.a);
    st.b = remap(st.b);
    st.c = n_vt + r;
    tensors[n_vt + r] = std::move(k.tensors[n_vt + u]);
    steps[r] = std::move(st);
    tiling[r] = k.tiling[u];
    tiling[r].level = tiling[r].mode == STEP_SERIAL ? lvl[u] : 0;
    tiling[r].part = tiling[r].mode == STEP_SERIAL ? prt[u] : -1;
  }
  for (auto& c : k.comps) c = remap(c);
  for (auto& v : k.vtx)
    if (v.adjoint >= 0) v.adjoint = remap(v.adjoint);
  k.steps = std::move(steps);
  k.tiling = std::move(tiling);
  k.tensors = std::move(tensors);
}

// The graph whose tensor network is contracted: spins 0..n-1, edges (u, v)
// carrying merged edges, and per spin its pins (merged edge to a sliced spin,
// index of that sliced spin), in compressed rows.
struct NetGraph {
  int32_t n = 0;
  std::vector<std::pair<int32_t, int32_t>> e;
  std::vector<int32_t> e_medge;
  std::vector<int32_t> pin_off{0};
  std::vector<std::pair<int32_t, int32_t>> pins;
};

// Absorption of the edge matrices into vertex tensors and the pairwise order
// (Sec. III): fills k.vtx, k.tensors, k.steps, k.comps; n_vt = vertex tensors.
kn_status build_network(const NetGraph& G, int32_t q, const kn_plan_opts& o, PlanKnot& k,
                        int32_t& n_vt, double* model_time = nullptr) {
  const int32_t n = G.n;
  k.vtx.clear();
  k.tensors.clear();
  k.steps.clear();
  k.comps.clear();
  // ---- absorption: orient edges by a minimum-degree elimination order
  // adjacency (neighbour, merged edge) in compressed rows
  const int32_t ne2 = 2 * (int32_t)G.e.size();
  std::vector<int32_t> aoff(n + 1, 0), anb(ne2), amd(ne2);
  for (auto [u, v] : G.e) {
    aoff[u + 1]++;
    aoff[v + 1]++;
  }
  for (int32_t v = 0; v < n; ++v) aoff[v + 1] += aoff[v];
  {
    std::vector<int32_t> fp(aoff.begin(), aoff.end() - 1);
    for (size_t i = 0; i < G.e.size(); ++i) {
      auto [u, v] = G.e[i];
      anb[fp[u]] = v;
      amd[fp[u]++] = G.e_medge[i];
      anb[fp[v]] = u;
      amd[fp[v]++] = G.e_medge[i];
    }
  }
  std::vector<int32_t> deg(n), pos(n, -1);
  int32_t maxd = 0;
  for (int32_t v = 0; v < n; ++v) {
    deg[v] = aoff[v + 1] - aoff[v];
    maxd = std::max(maxd, deg[v]);
  }
  {
    // degree buckets as stacks threaded through one pool (entry: vertex, next)
    // with lazy deletion: a vertex whose degree dropped is pushed again and
    // its old entry skipped
    std::vector<int32_t> head(maxd + 1, -1), pool_v, pool_next;
    pool_v.reserve(n + ne2);
    pool_next.reserve(n + ne2);
    auto push = [&](int32_t d, int32_t v) {
      pool_v.push_back(v);
      pool_next.push_back(head[d]);
      head[d] = (int32_t)pool_v.size() - 1;
    };
    for (int32_t v = 0; v < n; ++v) push(deg[v], v);
    int32_t placed = 0, d = 0;
    while (placed < n) {
      d = std::max(0, d - 1);
      while (d <= maxd && head[d] < 0) ++d;
      const int32_t e = head[d];
      head[d] = pool_next[e];
      const int32_t v = pool_v[e];
      if (pos[v] >= 0 || deg[v] != d) continue;
      pos[v] = placed++;
      for (int32_t j = aoff[v]; j < aoff[v + 1]; ++j) {
        const int32_t w = anb[j];
        if (pos[w] < 0) {
          --deg[w];
          push(deg[w], w);
        }
      }
    }
  }
  // out-edges of v: to neighbours placed later, sorted by (neighbour, edge)
  std::vector<int32_t> holders(n, 0), ooff(n + 1, 0);
  std::vector<std::pair<int32_t, int32_t>> outs;
  outs.reserve(ne2 / 2);
  for (int32_t v = 0; v < n; ++v) {
    for (int32_t j = aoff[v]; j < aoff[v + 1]; ++j)
      if (pos[anb[j]] > pos[v]) outs.emplace_back(anb[j], amd[j]);
    ooff[v + 1] = (int32_t)outs.size();
    std::sort(outs.begin() + ooff[v], outs.end());
    if (ooff[v + 1] > ooff[v]) holders[v]++;
    for (int32_t j = ooff[v]; j < ooff[v + 1]; ++j) holders[outs[j].first]++;
  }
  // vertex tensors
  k.vtx.reserve(n);
  k.tensors.reserve(2 * n + 1);
  for (int32_t v = 0; v < n; ++v) {
    const bool none = ooff[v + 1] == ooff[v];
    const bool pinned = G.pin_off[v + 1] > G.pin_off[v];
    bool has = !none || pinned;  // pins multiply the vertex's own tensor
    if (!has && holders[v] == 1) has = true;  // lone holder elsewhere: add [v] of ones
    if (!has) continue;
    if (ooff[v + 1] - ooff[v] > 7) return KN_E_UNSUPPORTED;  // planar graphs give <= 5
    PVertex pv;
    pv.tensor = (int32_t)k.tensors.size();
    pv.center = v;
    int32_t cnt = holders[v] + (none ? 1 : 0);
    pv.keep_center = cnt >= 2;
    PTensor t;
    if (pv.keep_center) t.spins.push_back(v);
    for (int32_t j = ooff[v]; j < ooff[v + 1]; ++j) {
      pv.nbr.push_back(outs[j].first);
      pv.medge.push_back(outs[j].second);
      t.spins.push_back(outs[j].first);
    }
    for (int32_t j = G.pin_off[v]; j < G.pin_off[v + 1]; ++j) {
      pv.pin_medge.push_back(G.pins[j].first);
      pv.pin_slice.push_back(G.pins[j].second);
    }
    k.vtx.push_back(std::move(pv));
    k.tensors.push_back(std::move(t));
  }
  n_vt = (int32_t)k.tensors.size();

  // ---- pairwise contraction order
  {
    std::vector<int32_t> cnt0(n, 0);
    for (int32_t t = 0; t < n_vt; ++t)
      for (int32_t sp : k.tensors[t].spins) cnt0[sp]++;
    for (int32_t sp = 0; sp < n; ++sp)
      if (cnt0[sp] == 1) return KN_E_INVALID;  // private spin left: planner bug guard
  }
  {
    // auto (3): min-fill first; the greedy plan is also built, and the cheaper
    // kept, only when the min-fill plan's modelled compute is material, and
    // separator orders too when it is large
    const int32_t strat = o.strategy;
    std::unique_ptr<Orderer> best;
    double best_cost = 0;
    auto consider = [&](std::unique_ptr<Orderer> cand) {
      const double c = cand->model_cost(o.precision, true);
      if (!best || c < best_cost) {
        best = std::move(cand);
        best_cost = c;
      }
    };
    for (int32_t sgy : {2, 0, 1}) {
      if (strat != 3 && sgy != strat) continue;
      if (strat == 3 && sgy == 1) continue;
      if (strat == 3 && sgy == 0 && best && best->flops() < kAutoGreedyFrom) continue;
      auto cand = std::make_unique<Orderer>(n, q, k.tensors);
      if (sgy == 2) cand->minfill();
      else cand->greedy(sgy);
      consider(std::move(cand));
    }
    if (strat == 4 || (strat == 3 && best->flops() >= kAutoSeparatorFrom)) {
      // separator hierarchies from several seeds and leaf sizes, each
      // eliminated in rank order (least fill inside a rank)
      const int32_t trials = o.order_trials > 0 ? o.order_trials : kSeparatorTrials;
      std::vector<int32_t> off, nb, rank;
      Orderer(n, q, k.tensors).primal(off, nb);
      for (int32_t t = 0; t < trials; ++t) {
        separator_ranks(n, off, nb, kSeparatorLeaf[t % 3], kSeparatorCandidates,
                        (uint64_t)t + 1, rank);
        auto cand = std::make_unique<Orderer>(n, q, k.tensors);
        cand->minfill(&rank);
        consider(std::move(cand));
      }
    }
    if (model_time) *model_time = best_cost;
    k.tensors = std::move(best->T);
    k.steps = std::move(best->S);
    for (int32_t t = 0; t < (int32_t)k.tensors.size(); ++t)
      if (best->alive[t]) {
        if (!k.tensors[t].spins.empty()) return KN_E_INVALID;  // guard
        k.comps.push_back(t);
      }
  }
  return KN_OK;
}

// The simplified graph with the spins of `sliced` (simplified ids) fixed:
// they leave the network, each edge to one of them becomes a pin of its other
// end, and edges between two of them become pair factors (in `pairs`).
// new_id maps simplified ids to the sliced graph's spins (-1 for sliced).
NetGraph sliced_graph(const Simplified& s, const std::vector<int32_t>& sliced,
                      std::vector<int32_t>& new_id, std::vector<Factor>& pairs) {
  NetGraph G;
  std::vector<int32_t> slice_of(s.n_spins, -1);
  for (size_t j = 0; j < sliced.size(); ++j) slice_of[sliced[j]] = (int32_t)j;
  new_id.assign(s.n_spins, -1);
  for (int32_t v = 0; v < s.n_spins; ++v)
    if (slice_of[v] < 0) new_id[v] = G.n++;
  std::vector<std::vector<std::pair<int32_t, int32_t>>> pin(G.n);
  pairs.clear();
  for (size_t i = 0; i < s.e.size(); ++i) {
    const auto [u, v] = s.e[i];
    const int32_t m = s.e_medge[i];
    const int32_t su = slice_of[u], sv = slice_of[v];
    if (su < 0 && sv < 0) {
      G.e.emplace_back(new_id[u], new_id[v]);
      G.e_medge.push_back(m);
    } else if (su >= 0 && sv >= 0) {
      pairs.push_back(Factor{FAC_PAIR, m, su, sv});
    } else if (su >= 0) {
      pin[new_id[v]].emplace_back(m, su);
    } else {
      pin[new_id[u]].emplace_back(m, sv);
    }
  }
  for (int32_t v = 0; v < G.n; ++v) {
    for (auto& pp : pin[v]) G.pins.push_back(pp);
    G.pin_off.push_back((int32_t)G.pins.size());
  }
  return G;
}

// Build tensors, order and arena for one knot.  Returns KN_OK or an error.
// Statistics, how each step runs (tiles or inside a serial task),
// dependency levels and the arena of a plan whose steps are final.
kn_status lay_out(PlanKnot& k, const kn_plan_opts& o, kn_plan_stats& st, int32_t n_vt) {
  const int32_t q = k.q;
  st.n_vertex_tensors = n_vt;
  st.n_steps = (int32_t)k.steps.size();

  // ---- sizes, statistics, tile decisions
  std::vector<double> qpow(64);
  qpow[0] = 1;
  for (int i = 1; i < 64; ++i) qpow[i] = qpow[i - 1] * q;
  const int64_t es = elem_bytes(o.precision);
  double flops = 0, bytes = 0, maxlog = 0;
  int32_t maxrank = 0;
  for (auto& t : k.tensors) {
    int32_t r = (int32_t)t.spins.size();
    maxrank = std::max(maxrank, r);
    double sz = qpow[std::min(r, 63)];
    if (sz > 2147483647.0) {
      st.max_rank = r;
      st.log2_max_entries = r * std::log2((double)q);
      return KN_E_BUDGET;
    }
    t.size = (int64_t)sz;
    maxlog = std::max(maxlog, std::log2(sz));
  }
  k.tiling.assign(k.steps.size(), PTiling());
  for (size_t i = 0; i < k.steps.size(); ++i) {
    auto& sp = k.steps[i];
    double nb = qpow[sp.bs.size()], nm = qpow[sp.ms.size()], nn = qpow[sp.ns.size()],
           nk = qpow[sp.ks.size()];
    flops += 8.0 * nb * nm * nn * nk;
    bytes += es * double(k.tensors[sp.a].size + k.tensors[sp.b].size + k.tensors[sp.c].size);
    // every group index and operand offset the engine decodes must lie in
    // the range of its exact division by q (QDiv, decode.h)
    if (std::max({nb, nm, nn, nk, nb * nm * nn}) > (double)kDecodeMax) {
      st.max_rank = maxrank;
      st.log2_max_entries = maxlog;
      return KN_E_BUDGET;
    }
    double macs = nb * nm * nn * nk;
    const double outs = nb * nm * nn;
    // the tile shape knobs of this step's intermediate-size bucket
    const int32_t bk = bucket_of(outs);
    auto knob = [&](int32_t per_bucket, int32_t plan_wide, int32_t dflt) {
      return per_bucket > 0 ? per_bucket : plan_wide > 0 ? plan_wide : dflt;
    };
    const kn_bucket_opts& bo = o.bucket[bk];
    bool big = macs >= std::ldexp(1.0, k.big_log2) || outs >= std::ldexp(1.0, k.big_outs_log2);
    // a serial step generates its gather tables in LDS; larger ones are tiled
    if (2 * nb + nm + 2 * nk + nn > kTabBuf) big = true;
    if (!big) continue;
    PTiling& t = k.tiling[i];
    double base;
    // the engine writes each output block (BM rows of C) from one base, with
    // byte offsets below 2^31 (kOutRangeBytes in the engine)
    const bool block_range_ok = 64.0 * nn * es < 2147483647.0;
    if (o.tile_outputs == 0 && nm >= 16 && nn >= 16 && block_range_ok) {
      // 64 x 64 blocks do four times the work per staged chunk of 32 x 32
      // ones (better hiding of the operand loads) but pad ragged sides more
      const double pad32 = std::ceil(nm / 32) * std::ceil(nn / 32) * 1024.0;
      const double pad64 = std::ceil(nm / 64) * std::ceil(nn / 64) * 4096.0;
      const int32_t pct = knob(bo.gemm64_pct, o.gemm64_pct, kGemm64Pct);
      const bool wide = nm >= 64 && nn >= 64 && pad64 * 100 <= pad32 * pct;
      const double bm = wide ? 64 : kGemmBlock;
      t.mode = wide ? STEP_GEMM64 : STEP_GEMM;
      t.n_mb = (int32_t)std::ceil(nm / bm);
      t.n_nb = (int32_t)std::ceil(nn / bm);
      // blocks per task: a step with many blocks gives each task several,
      // so that it still has about 2^gemm_tasks_log2 tasks
      const double blocks = nb * t.n_mb * t.n_nb;
      const double target = std::ldexp(1.0, knob(bo.gemm_tasks_log2, o.gemm_tasks_log2, kGemmTasksLog2));
      const double most = wide ? kGemmMaxBlocks / 4 : kGemmMaxBlocks;
      t.tile = (int32_t)std::max(1.0, std::min(most, std::floor(blocks / target)));
      base = std::ceil(blocks / t.tile);
    } else {
      // tiles carry about kTileMacs multiply-adds (at most kMaxTiles per step)
      t.mode = STEP_TILES;
      const double tile_macs = std::ldexp(1.0, knob(bo.tile_macs_log2, o.tile_macs_log2, kTileMacsLog2));
      const double tile_outs = std::ldexp(1.0, knob(bo.tile_outs_log2, o.tile_outs_log2, kTileOutsLog2));
      double tile = o.tile_outputs > 0
                        ? (double)o.tile_outputs
                        : std::max(1.0, std::min(tile_outs, std::floor(tile_macs / std::min(nk, 1024.0))));
      if (outs > tile * kMaxTiles) tile = std::ceil(outs / kMaxTiles);
      // a tile's outputs are written from one base, byte offsets below 2^31
      tile = std::min({tile, outs, kMaxTileOutputs});
      t.tile = (int32_t)tile;
      base = std::ceil(outs / tile);
    }
    // few tiles over a long contracted index: split it (partial sums, then a
    // reduce task) so that the step spreads over the device
    t.n_ks = 1;
    t.kseg = (int32_t)nk;
    if (nk >= 256 && base < kSplitBelow) {
      const double seg = std::ldexp(1.0, o.split_min_log2 > 0 ? o.split_min_log2 : kSplitMinLog2);
      double want = std::ceil(kSplitBelow / base), most = std::ceil(nk / seg);
      double ks = std::min(std::min(want, most), 256.0);
      if (ks > 1) {
        int64_t kseg = (int64_t)std::ceil(nk / ks);
        kseg = (kseg + 15) / 16 * 16;
        t.kseg = (int32_t)kseg;
        t.n_ks = (int32_t)((int64_t(nk) + kseg - 1) / kseg);
      }
    }
    t.n_tiles = (int32_t)(base * t.n_ks);
  }
  st.flops = flops;
  st.bytes = bytes;
  st.log2_max_entries = maxlog;
  st.max_rank = maxrank;
  level_schedule(k, n_vt);

  // ---- arena: first fit over live ranges, in execution order.  A tensor
  // lives from its step to its last use; component scalars and the adjoints
  // of the vertex tensors (read after the last step) to the end.
  {
    std::vector<int32_t> last(k.tensors.size(), -1);
    for (size_t u = 0; u < k.steps.size(); ++u) {
      last[k.steps[u].a] = (int32_t)u;
      last[k.steps[u].b] = (int32_t)u;
    }
    for (int32_t c : k.comps) last[c] = INT32_MAX;
    for (const auto& v : k.vtx)
      if (v.adjoint >= 0) last[v.adjoint] = INT32_MAX;
    FitAlloc fa(INT64_MAX, 16);
    auto alloc = [&](int64_t len) { return fa.alloc(len); };
    auto release = [&](int64_t off, int64_t len) { fa.release(off, len); };
    for (int32_t t = 0; t < n_vt; ++t) k.tensors[t].off = alloc(k.tensors[t].size);
    // steps of one level run concurrently: their outputs are placed before
    // any of their operands is released
    const size_t ns = k.steps.size();
    for (size_t i = 0; i < ns;) {
      size_t j = i + 1;
      while (j < ns && same_level(k, j - 1)) ++j;
      for (size_t u = i; u < j; ++u) {
        const auto& sp = k.steps[u];
        k.tensors[sp.c].off = alloc(k.tensors[sp.c].size);
        PTiling& t = k.tiling[u];
        if (t.n_ks > 1) {
          const int64_t len = (int64_t)t.n_ks * k.tensors[sp.c].size;
          t.partial = alloc(len);
          release(t.partial, len);
        }
      }
      // operands leave at their last use (the consumer of a plain plan; in a
      // gradient plan the forward tensors are read again by the reverse steps)
      for (size_t u = i; u < j; ++u) {
        const auto& sp = k.steps[u];
        if (last[sp.a] == (int32_t)u) release(k.tensors[sp.a].off, k.tensors[sp.a].size);
        if (sp.b != sp.a && last[sp.b] == (int32_t)u)
          release(k.tensors[sp.b].off, k.tensors[sp.b].size);
      }
      i = j;
    }
    k.arena_elems = std::max<int64_t>(fa.top, 16);
  }
  return KN_OK;
}

// A gradient plan: the reverse pass appended to the forward steps, with
// forward tensors of rank >= r dropped and recomputed in chains of at most d
// steps (add_reverse).  The search takes d = 1, 2, 4, 8 in turn and for each
// the largest r (none dropped first) whose arena fits mem_budget_bytes next
// to an allowance for the device program.  Without a budget nothing is
// dropped.
kn_status plan_gradient(PlanKnot& k, const kn_plan_opts& o, kn_plan_stats& st, int32_t& n_vt) {
  const std::vector<PTensor> T0 = k.tensors;
  const std::vector<PStep> S0 = k.steps;
  const std::vector<PVertex> V0 = k.vtx;
  const std::vector<int32_t> C0 = k.comps;
  const int32_t nvt0 = n_vt;
  std::vector<int32_t> ranks{INT32_MAX};
  for (const auto& stp : S0) ranks.push_back(T0[stp.c].spins.size());
  std::sort(ranks.begin(), ranks.end(), std::greater<int32_t>());
  ranks.erase(std::unique(ranks.begin(), ranks.end()), ranks.end());
  const double es = (double)elem_bytes(o.precision);
  auto build = [&](int32_t rank, int32_t depth, double& need) {
    k.tensors = T0;
    k.steps = S0;
    k.vtx = V0;
    k.comps = C0;
    n_vt = nvt0;
    int32_t n_re = 0;
    add_reverse(k, n_vt, rank, depth, n_re);
    const kn_status rc = lay_out(k, o, st, n_vt);
    st.n_recompute_steps = n_re;
    // the arena plus an allowance for the device program and runtime state
    need = (double)k.arena_elems * es + 512.0 * (double)(k.steps.size() + k.tensors.size()) +
           65536.0;
    return rc;
  };
  // shallow recompute chains first, for each the largest rank that fits; if
  // nothing fits, the setting with the least memory
  int32_t best_rank = ranks[0], best_depth = 1;
  double best_need = -1, need = 0;
  for (int32_t depth : {1, 2, 4, 8}) {
    for (size_t i = depth == 1 ? 0 : 1; i < ranks.size(); ++i) {
      const kn_status rc = build(ranks[i], depth, need);
      if (rc != KN_OK) return rc;
      if (!o.mem_budget_bytes || need <= (double)o.mem_budget_bytes) return KN_OK;
      if (best_need < 0 || need < best_need) {
        best_rank = ranks[i];
        best_depth = depth;
        best_need = need;
      }
    }
  }
  return build(best_rank, best_depth, need);  // over budget: kn_plan_create says so
}

kn_status make_plan(const kn_tait& g, int32_t q, const kn_plan_opts& o, PlanKnot& k,
                    kn_plan_stats& st) {
  k.q = q;
  k.precision = o.precision;
  k.jones_only = o.jones_only != 0;
  k.gradient = o.gradient != 0;
  k.n_edges = (int32_t)g.eps.size();
  k.eps = g.eps;
  k.tile = o.tile_outputs > 0 ? o.tile_outputs : 256;
  // steps below 2^big_log2 multiply-adds run inside serial tasks, which write
  // a step's outputs from one base (at most 2^24 of them)
  k.big_log2 = std::min(o.big_step_macs_log2 > 0 ? o.big_step_macs_log2 : 16, 24);
  k.big_outs_log2 = std::min(o.big_step_outs_log2 > 0 ? o.big_step_outs_log2 : kBigOutsLog2, 24);
  k.lds_bytes = o.lds_bytes > 0 ? o.lds_bytes : 24576;
  k.split_est = std::ldexp(1.0, o.split_serial_log2 > 0 ? o.split_serial_log2 : kSplitSerialLog2);
  k.fork_est = std::ldexp(1.0, o.fork_serial_log2 > 0 ? o.fork_serial_log2 : kForkSerialLog2);
  {
    double qq = q;
    if (q < 4) {
      k.t_re = (qq - 2.0) / 2.0;
      k.t_im = std::sqrt(qq * (4.0 - qq)) / 2.0;
    } else {
      k.t_re = (qq - 2.0 + std::sqrt(qq * (qq - 4.0))) / 2.0;
      k.t_im = 0.0;
    }
  }
  Simplified s = simplify(g, o.simplify, k.jones_only, k);
  const int32_t n = s.n_spins;
  st.n_edges_simplified = (int32_t)s.e.size();
  st.n_vertices_simplified = n;
  st.delta_h_paper = o.paper_stats ? paper_delta_h(s) : -1;

  // ---- slicing (optional), then absorption and order of the network
  int32_t n_vt = 0;
  {
    std::vector<int32_t> sliced, new_id;
    std::vector<Factor> pairs;
    const double lq = std::log2((double)q);
    for (;;) {
      NetGraph G = sliced_graph(s, sliced, new_id, pairs);
      kn_status rc = build_network(G, q, o, k, n_vt);
      if (rc != KN_OK) return rc;
      if (o.slice_log2_budget <= 0) break;
      int32_t maxr = 0;
      for (const auto& t : k.tensors) maxr = std::max(maxr, (int32_t)t.spins.size());
      double slices = 1;
      for (size_t j = 0; j <= sliced.size(); ++j) slices *= q;  // after one more spin
      if (maxr * lq <= o.slice_log2_budget || (int32_t)sliced.size() >= kMaxSliceSpins ||
          slices > kMaxSlices || G.n == 0)
        break;
      // candidates: the spins held by most of the largest tensors (ties:
      // lowest id); each is tried, and the one whose plan has the smallest
      // largest tensor, then the smallest modelled time over all slices, is
      // fixed
      std::vector<int32_t> hits(G.n, 0);
      for (const auto& t : k.tensors)
        if ((int32_t)t.spins.size() >= maxr - 1)
          for (int32_t x : t.spins) hits[x]++;
      std::vector<int32_t> cand(G.n);
      for (int32_t v = 0; v < G.n; ++v) cand[v] = v;
      const int32_t n_cand = std::min<int32_t>(G.n, kSliceCandidates);
      std::partial_sort(cand.begin(), cand.begin() + n_cand, cand.end(),
                        [&](int32_t a, int32_t b) {
                          return hits[a] != hits[b] ? hits[a] > hits[b] : a < b;
                        });
      int32_t pick = -1, pick_rank = 0;
      double pick_cost = 0;
      for (int32_t c = 0; c < n_cand && n_cand > 1; ++c) {
        std::vector<int32_t> trial = sliced, tid;
        std::vector<Factor> tpairs;
        for (int32_t v = 0; v < s.n_spins; ++v)
          if (new_id[v] == cand[c]) trial.push_back(v);
        NetGraph TG = sliced_graph(s, trial, tid, tpairs);
        PlanKnot tk;
        int32_t t_vt = 0;
        double cost = 0;
        if (build_network(TG, q, o, tk, t_vt, &cost) != KN_OK) continue;
        int32_t r = 0;
        for (const auto& t : tk.tensors) r = std::max(r, (int32_t)t.spins.size());
        cost *= slices;
        if (pick < 0 || r < pick_rank || (r == pick_rank && cost < pick_cost)) {
          pick = cand[c];
          pick_rank = r;
          pick_cost = cost;
        }
      }
      if (pick < 0) pick = cand[0];
      for (int32_t v = 0; v < s.n_spins; ++v)
        if (new_id[v] == pick) sliced.push_back(v);
    }
    k.n_slice_spins = (int32_t)sliced.size();
    k.n_slices = 1;
    for (size_t j = 0; j < sliced.size(); ++j) k.n_slices *= q;
    for (const Factor& f : pairs) k.factors.push_back(f);
  }
  st.n_components = (int32_t)k.comps.size();
  kn_status rc = k.gradient ? plan_gradient(k, o, st, n_vt) : lay_out(k, o, st, n_vt);
  if (rc != KN_OK) return rc;
  // slices: work and traffic of all slices; chains share arenas within the
  // memory budget (16 GiB of arena by default)
  st.n_slices = k.n_slices;
  st.flops *= k.n_slices;
  st.bytes *= k.n_slices;
  {
    const double budget = o.mem_budget_bytes ? (double)o.mem_budget_bytes : 16.0 * (1 << 30);
    const double per = (double)k.arena_elems * (double)elem_bytes(o.precision);
    const double fit = std::floor(budget / std::max(per, 1.0));
    k.slice_chains = (int32_t)std::max(1.0, std::min({(double)k.n_slices, fit, 64.0}));
    st.slice_chains = k.slice_chains;
  }
  return KN_OK;
}

}  // namespace kn

namespace kn {

const Bytes& plan_image(const kn_plan* p) {
  std::lock_guard<std::mutex> lock(p->image_mu);
  if (p->image.empty() && p->laid_out) {
    std::vector<const PlanKnot*> one{&p->k};
    p->image = build_image(one);
  }
  return p->image;
}

}  // namespace kn

static kn_plan_opts default_opts() {
  kn_plan_opts o;
  std::memset(&o, 0, sizeof(o));
  o.strategy = 3;
  o.precision = 0;
  o.simplify = 3;
  o.jones_only = 1;
  o.mem_budget_bytes = 0;
  o.tile_outputs = 0;
  o.big_step_macs_log2 = 0;
  o.paper_stats = 0;
  o.lds_bytes = 0;
  o.gradient = 0;
  o.tile_macs_log2 = 0;
  o.slice_log2_budget = 0;
  o.split_serial_log2 = 0;
  o.gemm_tasks_log2 = 0;
  o.gemm64_pct = 0;
  return o;
}

extern "C" kn_status kn_plan_create(const kn_tait* g, int32_t q, const kn_plan_opts* opts,
                                    kn_plan** out) {
  if (!out) return KN_E_INVALID;
  *out = nullptr;
  if (!g) return KN_E_INVALID;
  if (q < 2 || q > 8) return KN_E_UNSUPPORTED;
  kn_plan_opts o = opts ? *opts : default_opts();
  if (o.strategy < 0 || o.strategy > 4 || o.order_trials < 0 || o.order_trials > 4096 || o.precision < 0 || o.precision > 1 ||
      o.simplify < 0 || o.simplify > 7 || o.tile_outputs < 0 || o.big_step_macs_log2 < 0 ||
      o.big_step_macs_log2 > 40 || o.lds_bytes < 0 || o.lds_bytes > 131072 ||
      o.tile_macs_log2 < 0 || o.tile_macs_log2 > 30)
    return KN_E_INVALID;
  if ((o.simplify & 6) && !o.jones_only) return KN_E_INVALID;  // need the Jones couplings
  if (o.gradient != 0 && o.gradient != 1) return KN_E_INVALID;
  if (o.gradient && (o.simplify & 6)) return KN_E_INVALID;
  if (o.slice_log2_budget < 0 || o.slice_log2_budget > 40) return KN_E_INVALID;
  if (o.split_serial_log2 < 0 || o.split_serial_log2 > 40) return KN_E_INVALID;
  if (o.fork_serial_log2 < 0 || o.fork_serial_log2 > 40) return KN_E_INVALID;
  if (o.split_min_log2 < 0 || o.split_min_log2 > 30) return KN_E_INVALID;
  if (o.gemm_tasks_log2 < 0 || o.gemm_tasks_log2 > 30) return KN_E_INVALID;
  if (o.gemm64_pct < 0 || o.gemm64_pct > 100000) return KN_E_INVALID;
  if (o.big_step_outs_log2 < 0 || o.big_step_outs_log2 > 31) return KN_E_INVALID;
  if (o.tile_outs_log2 < 0 || o.tile_outs_log2 > 24) return KN_E_INVALID;
  for (const kn_bucket_opts& b : o.bucket)
    if (b.tile_macs_log2 < 0 || b.tile_macs_log2 > 30 || b.tile_outs_log2 < 0 ||
        b.tile_outs_log2 > 24 || b.gemm64_pct < 0 || b.gemm64_pct > 100000 ||
        b.gemm_tasks_log2 < 0 || b.gemm_tasks_log2 > 30)
      return KN_E_INVALID;
  if (o.gradient && o.slice_log2_budget) return KN_E_UNSUPPORTED;
  kn_plan* p = new (std::nothrow) kn_plan();
  if (!p) return KN_E_NOMEM;
  kn_status rc;
  try {
    rc = kn::make_plan(*g, q, o, p->k, p->stats);
    if (rc == KN_OK) {
      kn::make_section(p->k);
      p->k.release_planning();
      std::vector<const kn::PlanKnot*> one{&p->k};
      const kn::Bytes hb = kn::build_image(one, true);
      if (hb.empty()) {
        rc = KN_E_BUDGET;
      } else {
        kn::ImgHeader h;
        std::memcpy(&h, hb.data(), sizeof(h));
        p->laid_out = true;
        p->stats.workspace_bytes = (uint64_t)h.workspace_bytes;
        p->stats.image_bytes = (uint64_t)h.image_bytes;
        p->stats.n_tasks = h.n_tasks;
        if (o.mem_budget_bytes && p->stats.workspace_bytes > o.mem_budget_bytes) rc = KN_E_BUDGET;
      }
    }
  } catch (const std::bad_alloc&) {
    delete p;
    return KN_E_NOMEM;
  }
  if (rc == KN_OK || rc == KN_E_BUDGET) {
    *out = p;
    return rc;
  }
  delete p;
  return rc;
}

extern "C" kn_status kn_plan_info(const kn_plan* p, kn_plan_stats* out) {
  if (!p || !out) return KN_E_INVALID;
  *out = p->stats;
  return KN_OK;
}

extern "C" kn_status kn_plan_image(const kn_plan* p, const void** data, size_t* bytes) {
  if (!p || !data || !bytes) return KN_E_INVALID;
  const kn::Bytes& img = kn::plan_image(p);
  *data = img.empty() ? nullptr : img.data();
  *bytes = img.size();
  return KN_OK;
}

extern "C" kn_status kn_plan_steps(const kn_plan* p, int32_t* ab) {
  if (!p || !ab) return KN_E_INVALID;
  const auto& sd = p->k.sec.sd;
  for (size_t i = 0; i < sd.size(); ++i) {
    ab[2 * i] = sd[i].a;
    ab[2 * i + 1] = sd[i].b;
  }
  return KN_OK;
}

extern "C" void kn_plan_free(kn_plan* p) { delete p; }
