// separator.cpp -- nested-dissection elimination ranks: the separator-
// hierarchy contraction order that Sec. III offers beside the greedy one
// (there built with METIS; here an own bisection code for the small planar
// graphs of knot diagrams).
//
// The graph is split recursively: a small set of spins (a vertex separator)
// whose removal leaves two parts of comparable size, then each part the same
// way, down to parts of at most `leaf` spins.  A spin's rank is the height of
// its node in that hierarchy (the separator of the whole graph has the
// largest rank, leaves the smallest): eliminating every spin of lower rank
// first means each part is contracted on its own, and the parts meet only in
// the tensors that carry their separator -- the coarse-graining order of the
// separator hierarchy.  The planner eliminates spins in rank order, least
// fill first inside a rank.
//
// A separator comes from the best of several candidates: levels of a
// breadth-first search (a single level separates the levels before it from
// those after it), and the vertex cover (Konig: from a maximum matching) of
// an edge cut refined by Fiduccia-Mattheyses passes.  Each candidate is then
// improved by moving separator spins into a side when that pulls fewer spins
// of the other side into the separator.  Roots of the searches are a
// pseudo-peripheral spin and spins drawn from a seeded generator, so the
// hierarchy is a deterministic function of (graph, seed).
#include "internal.h"

namespace kn {

namespace {

// splitmix64 (Steele, Lea, Flood 2014)
struct Rng {
  uint64_t s;
  uint64_t next() {
    uint64_t z = (s += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
  }
  int32_t below(int32_t n) { return (int32_t)(next() % (uint64_t)n); }
};

// Induced subgraph on a vertex list, local ids 0..m-1.
struct Sub {
  std::vector<int32_t> ids;  // local -> global
  std::vector<int32_t> off, nb;
  int32_t m() const { return (int32_t)ids.size(); }
};

void induce(const std::vector<int32_t>& goff, const std::vector<int32_t>& gnb,
            const std::vector<int32_t>& verts, std::vector<int32_t>& loc, Sub& s) {
  s.ids = verts;
  const int32_t m = (int32_t)verts.size();
  for (int32_t i = 0; i < m; ++i) loc[verts[i]] = i;
  s.off.assign(m + 1, 0);
  s.nb.clear();
  for (int32_t i = 0; i < m; ++i) {
    const int32_t v = verts[i];
    for (int32_t j = goff[v]; j < goff[v + 1]; ++j)
      if (loc[gnb[j]] >= 0) s.nb.push_back(loc[gnb[j]]);
    s.off[i + 1] = (int32_t)s.nb.size();
  }
  for (int32_t v : verts) loc[v] = -1;
}

// Breadth-first distances from root (-1: not reached) and the visit order.
int32_t bfs(const Sub& s, int32_t root, std::vector<int32_t>& dist, std::vector<int32_t>& order) {
  const int32_t m = s.m();
  dist.assign(m, -1);
  order.clear();
  dist[root] = 0;
  order.push_back(root);
  for (size_t h = 0; h < order.size(); ++h) {
    const int32_t v = order[h];
    for (int32_t j = s.off[v]; j < s.off[v + 1]; ++j)
      if (dist[s.nb[j]] < 0) {
        dist[s.nb[j]] = dist[v] + 1;
        order.push_back(s.nb[j]);
      }
  }
  return dist[order.back()];
}

// side: 0 = A, 1 = B, 2 = separator
struct Split {
  std::vector<int8_t> side;
  int32_t n[3] = {0, 0, 0};
  void count() {
    n[0] = n[1] = n[2] = 0;
    for (int8_t x : side) n[(int)x]++;
  }
};

constexpr double kMaxSide = 0.65;  // larger part at most this share of the non-separator spins

bool balanced(int32_t a, int32_t b) {
  const int32_t rest = a + b;
  return std::max(a, b) <= std::max<double>(1.0, kMaxSide * rest) && std::min(a, b) > 0;
}

// Better of two splits: balanced first, then fewer separator spins, then the
// more even parts.
bool better(const Split& x, const Split& y) {
  const bool bx = balanced(x.n[0], x.n[1]), by = balanced(y.n[0], y.n[1]);
  if (bx != by) return bx;
  if (x.n[2] != y.n[2]) return x.n[2] < y.n[2];
  return std::abs(x.n[0] - x.n[1]) < std::abs(y.n[0] - y.n[1]);
}

// Move separator spins into a side while that shrinks the separator (or
// keeps its size and evens out the parts): spin s joins side t, and its
// neighbours on the other side join the separator.
void refine_separator(const Sub& s, Split& sp) {
  const int32_t m = s.m();
  for (int pass = 0; pass < 16; ++pass) {
    bool moved = false;
    for (int32_t v = 0; v < m; ++v) {
      if (sp.side[v] != 2) continue;
      int32_t k[2] = {0, 0};
      for (int32_t j = s.off[v]; j < s.off[v + 1]; ++j) {
        const int8_t w = sp.side[s.nb[j]];
        if (w < 2) k[(int)w]++;
      }
      // try the smaller side first
      const int32_t first = sp.n[0] <= sp.n[1] ? 0 : 1;
      for (int32_t tt = 0; tt < 2; ++tt) {
        const int32_t t = tt == 0 ? first : 1 - first;
        const int32_t o = 1 - t;
        const int32_t gain = 1 - k[o];
        const int32_t na = sp.n[t] + 1, no = sp.n[o] - k[o];
        if (no <= 0) continue;
        const bool was_bal = balanced(sp.n[0], sp.n[1]);
        const bool now_bal = balanced(na, no);
        if (was_bal && !now_bal) continue;
        const bool evener = std::abs(na - no) < std::abs(sp.n[t] - sp.n[o]);
        if (!(gain > 0 || (gain == 0 && evener) || (!was_bal && now_bal))) continue;
        sp.side[v] = (int8_t)t;
        for (int32_t j = s.off[v]; j < s.off[v + 1]; ++j)
          if (sp.side[s.nb[j]] == o) sp.side[s.nb[j]] = 2;
        sp.count();
        moved = true;
        break;
      }
    }
    if (!moved) break;
  }
}

// Separator from the levels of a breadth-first search: the level whose spins
// split the earlier levels from the later ones best.
bool level_split(const Sub& s, const std::vector<int32_t>& dist, int32_t depth, Split& out) {
  const int32_t m = s.m();
  std::vector<int32_t> cnt(depth + 2, 0);
  for (int32_t v = 0; v < m; ++v)
    if (dist[v] >= 0) cnt[dist[v]]++;
  int32_t lev = -1;
  Split cand;
  int32_t before = cnt[0];
  for (int32_t l = 1; l < depth; ++l) {
    Split sp;
    sp.n[0] = before;
    sp.n[1] = m - before - cnt[l];
    sp.n[2] = cnt[l];
    before += cnt[l];
    if (lev < 0 || better(sp, cand)) {
      cand = sp;
      lev = l;
    }
  }
  if (lev < 0) return false;
  out.side.assign(m, 0);
  for (int32_t v = 0; v < m; ++v)
    out.side[v] = (int8_t)(dist[v] < lev ? 0 : dist[v] == lev ? 2 : 1);
  out.count();
  return true;
}

// Edge bisection: the first half of a breadth-first order against the rest,
// then Fiduccia-Mattheyses passes (moves with the best gain, the best prefix
// of each pass kept) with each side between 45 % and 55 % of the spins.
void fm_bisect(const Sub& s, const std::vector<int32_t>& order, std::vector<int8_t>& part) {
  const int32_t m = s.m();
  part.assign(m, 1);
  for (int32_t i = 0; i < m / 2; ++i) part[order[i]] = 0;
  const int32_t lo = (int32_t)std::floor(0.45 * m), hi = m - lo;
  std::vector<int32_t> gain(m), moves;
  std::vector<uint8_t> locked(m);
  int32_t size0 = m / 2;
  for (int pass = 0; pass < 6; ++pass) {
    for (int32_t v = 0; v < m; ++v) {
      int32_t g = 0;
      for (int32_t j = s.off[v]; j < s.off[v + 1]; ++j) g += part[s.nb[j]] != part[v] ? 1 : -1;
      gain[v] = g;
    }
    std::fill(locked.begin(), locked.end(), 0);
    moves.clear();
    int32_t cum = 0, best = 0, best_len = 0, sz = size0, best_sz = size0;
    for (int32_t step = 0; step < m; ++step) {
      int32_t pick = -1;
      for (int32_t v = 0; v < m; ++v) {
        if (locked[v]) continue;
        const int32_t ns = part[v] == 0 ? sz - 1 : sz + 1;
        if (ns < lo || ns > hi) continue;
        if (pick < 0 || gain[v] > gain[pick]) pick = v;
      }
      if (pick < 0) break;
      cum += gain[pick];
      sz += part[pick] == 0 ? -1 : 1;
      part[pick] ^= 1;
      locked[pick] = 1;
      moves.push_back(pick);
      gain[pick] = -gain[pick];
      for (int32_t j = s.off[pick]; j < s.off[pick + 1]; ++j) {
        const int32_t w = s.nb[j];
        gain[w] += part[w] == part[pick] ? -2 : 2;
      }
      if (cum > best || (cum == best && std::abs(2 * sz - m) < std::abs(2 * best_sz - m))) {
        best = cum;
        best_len = (int32_t)moves.size();
        best_sz = sz;
      }
    }
    for (int32_t i = (int32_t)moves.size() - 1; i >= best_len; --i) part[moves[i]] ^= 1;
    size0 = best_sz;
    if (best <= 0) break;
  }
}

// Smallest vertex cover of the cut edges of a bisection (Konig's theorem:
// from a maximum matching of the bipartite cut graph); the cover is the
// separator.
void cover_split(const Sub& s, const std::vector<int8_t>& part, Split& out) {
  const int32_t m = s.m();
  std::vector<int32_t> mate(m, -1);
  std::vector<uint32_t> seen(m, 0);
  uint32_t stamp = 0;
  // augmenting paths from side-0 spins (depth-first, iterative)
  std::vector<std::pair<int32_t, int32_t>> st;  // (left spin, next adjacency index)
  std::vector<int32_t> path;
  for (int32_t u = 0; u < m; ++u) {
    if (part[u] != 0 || mate[u] >= 0) continue;
    bool cut = false;
    for (int32_t j = s.off[u]; j < s.off[u + 1] && !cut; ++j) cut = part[s.nb[j]] == 1;
    if (!cut) continue;
    ++stamp;
    st.clear();
    path.clear();
    st.emplace_back(u, s.off[u]);
    bool done = false;
    while (!st.empty() && !done) {
      auto& [x, j] = st.back();
      if (j >= s.off[x + 1]) {
        st.pop_back();
        if (!path.empty()) path.pop_back();
        continue;
      }
      const int32_t y = s.nb[j++];
      if (part[y] != 1 || seen[y] == stamp) continue;
      seen[y] = stamp;
      if (mate[y] < 0) {
        // augment along the stack: left spins st[i].first, right spins path[i]
        path.push_back(y);
        for (size_t i = 0; i < st.size(); ++i) {
          mate[st[i].first] = path[i];
          mate[path[i]] = st[i].first;
        }
        done = true;
      } else {
        path.push_back(y);
        st.emplace_back(mate[y], s.off[mate[y]]);
      }
    }
  }
  // alternating reachability from unmatched side-0 spins with a cut edge
  std::vector<uint8_t> z(m, 0);
  std::vector<int32_t> q;
  for (int32_t u = 0; u < m; ++u) {
    if (part[u] != 0 || mate[u] >= 0) continue;
    bool cut = false;
    for (int32_t j = s.off[u]; j < s.off[u + 1] && !cut; ++j) cut = part[s.nb[j]] == 1;
    if (cut) {
      z[u] = 1;
      q.push_back(u);
    }
  }
  for (size_t h = 0; h < q.size(); ++h) {
    const int32_t x = q[h];  // a side-0 spin
    for (int32_t j = s.off[x]; j < s.off[x + 1]; ++j) {
      const int32_t y = s.nb[j];
      if (part[y] != 1 || z[y] || mate[x] == y) continue;
      z[y] = 1;
      if (mate[y] >= 0 && !z[mate[y]]) {
        z[mate[y]] = 1;
        q.push_back(mate[y]);
      }
    }
  }
  out.side.assign(m, 0);
  for (int32_t v = 0; v < m; ++v) {
    out.side[v] = part[v];
    bool cut = false;
    for (int32_t j = s.off[v]; j < s.off[v + 1] && !cut; ++j) cut = part[s.nb[j]] != part[v];
    if (!cut) continue;
    // cover: side-0 endpoints outside Z, side-1 endpoints inside Z
    if ((part[v] == 0 && !z[v]) || (part[v] == 1 && z[v])) out.side[v] = 2;
  }
  out.count();
}

// Connected components of a subgraph (as lists of local ids).
void components(const Sub& s, std::vector<std::vector<int32_t>>& comps) {
  const int32_t m = s.m();
  std::vector<int32_t> dist, order;
  std::vector<uint8_t> done(m, 0);
  comps.clear();
  for (int32_t r = 0; r < m; ++r) {
    if (done[r]) continue;
    bfs(s, r, dist, order);
    for (int32_t v : order) done[v] = 1;
    comps.push_back(order);
  }
}

}  // namespace

void separator_ranks(int32_t n, const std::vector<int32_t>& off, const std::vector<int32_t>& nb,
                     int32_t leaf, int32_t trials, uint64_t seed, std::vector<int32_t>& rank) {
  rank.assign(n, 0);
  if (n == 0) return;
  Rng rng{seed * 0x2545f4914f6cdd1dull + 1};
  std::vector<int32_t> depth(n, 0), loc(n, -1);
  struct Node {
    std::vector<int32_t> verts;
    int32_t depth;
  };
  std::vector<Node> stack;
  {
    Node root;
    root.verts.resize(n);
    for (int32_t v = 0; v < n; ++v) root.verts[v] = v;
    root.depth = 0;
    stack.push_back(std::move(root));
  }
  int32_t max_depth = 0;
  Sub s;
  std::vector<int32_t> dist, order;
  std::vector<std::vector<int32_t>> comps;
  std::vector<int8_t> part;
  while (!stack.empty()) {
    Node node = std::move(stack.back());
    stack.pop_back();
    max_depth = std::max(max_depth, node.depth);
    for (int32_t v : node.verts) depth[v] = node.depth;
    if ((int32_t)node.verts.size() <= std::max(leaf, 2)) continue;
    induce(off, nb, node.verts, loc, s);
    components(s, comps);
    if (comps.size() > 1) {  // disconnected: the components are the children
      for (const auto& c : comps) {
        Node ch;
        for (int32_t v : c) ch.verts.push_back(s.ids[v]);
        ch.depth = node.depth + 1;
        stack.push_back(std::move(ch));
      }
      continue;
    }
    const int32_t m = s.m();
    Split best;
    bool have = false;
    for (int32_t t = 0; t < std::max(trials, 1); ++t) {
      int32_t root = 0;
      if (t == 0) {  // pseudo-peripheral: the farthest spin from the farthest spin
        bfs(s, 0, dist, order);
        bfs(s, order.back(), dist, order);
        root = order.back();
      } else {
        root = rng.below(m);
      }
      const int32_t dep = bfs(s, root, dist, order);
      Split a;
      if (level_split(s, dist, dep, a)) {
        refine_separator(s, a);
        if (!have || better(a, best)) {
          best = a;
          have = true;
        }
      }
      fm_bisect(s, order, part);
      Split b;
      cover_split(s, part, b);
      refine_separator(s, b);
      if (!have || better(b, best)) {
        best = b;
        have = true;
      }
    }
    if (!have || best.n[0] == 0 || best.n[1] == 0) continue;  // no split: a leaf
    Node a, b;
    for (int32_t v = 0; v < m; ++v) {
      if (best.side[v] == 0) a.verts.push_back(s.ids[v]);
      else if (best.side[v] == 1) b.verts.push_back(s.ids[v]);
    }
    a.depth = b.depth = node.depth + 1;
    stack.push_back(std::move(a));
    stack.push_back(std::move(b));
  }
  for (int32_t v = 0; v < n; ++v) rank[v] = max_depth - depth[v];
}

}  // namespace kn
