// image.cpp -- lay one or more knot plans out as a device program (see
// program.h): descriptors, gather tables, task groups, ready-queue roots and
// LDS homes.
//
// The tasks of one knot form a chain of groups executed one after another (a
// serial run of small steps on one workgroup, or all tiles of one big step);
// the engine starts a group when every task of the previous group has
// finished, which also guarantees that arena memory freed by a group is not
// reused while that group still reads it.  Groups of different knots are
// independent.  The first groups of all knots seed the device ready queue,
// longest estimated chain first.
//
// A tensor produced and consumed inside the same serial task lives in that
// workgroup's LDS arena when it fits (first fit over its live range);
// everything else lives in the global arena.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <numeric>

#include "internal.h"

namespace kn {

namespace {
template <class T>
int64_t put(std::vector<uint8_t>& img, const std::vector<T>& v) {
  int64_t off = align256((int64_t)img.size());
  img.resize(off + v.size() * sizeof(T));
  if (!v.empty()) std::memcpy(img.data() + off, v.data(), v.size() * sizeof(T));
  return off;
}

// offset of each value of a spin group inside a tensor stored in `order`
void group_table(const std::vector<int32_t>& group, const std::vector<int32_t>& order, int32_t q,
                 std::vector<int32_t>& out) {
  // stride of each spin in the storage order (row-major, last fastest)
  std::vector<int64_t> gstride(group.size());
  for (size_t i = 0; i < group.size(); ++i) {
    int64_t s = 1;
    bool found = false;
    for (int64_t j = (int64_t)order.size() - 1; j >= 0; --j) {
      if (order[j] == group[i]) { found = true; break; }
      s *= q;
    }
    gstride[i] = found ? s : 0;
  }
  int64_t n = 1;
  for (size_t i = 0; i < group.size(); ++i) n *= q;
  size_t base = out.size();
  out.resize(base + n);
  // enumerate the group's values, first spin most significant (odometer)
  const int r = (int)group.size();
  int digit[64] = {0};
  int64_t off = 0;
  for (int64_t idx = 0; idx < n; ++idx) {
    out[base + idx] = (int32_t)off;
    for (int i = r - 1; i >= 0; --i) {
      if (++digit[i] < q) {
        off += gstride[i];
        break;
      }
      digit[i] = 0;
      off -= (int64_t)(q - 1) * gstride[i];
    }
  }
}

}  // namespace

void make_tables(PlanKnot& k) {
  k.tables.clear();
  k.tab_off.assign(k.steps.size(), 0);
  for (size_t si = 0; si < k.steps.size(); ++si) {
    const PStep& s = k.steps[si];
    k.tab_off[si] = (int32_t)k.tables.size();
    const auto& A = k.tensors[s.a].spins;
    const auto& B = k.tensors[s.b].spins;
    group_table(s.bs, A, k.q, k.tables);
    group_table(s.ms, A, k.q, k.tables);
    group_table(s.ks, A, k.q, k.tables);
    group_table(s.bs, B, k.q, k.tables);
    group_table(s.ks, B, k.q, k.tables);
    group_table(s.ns, B, k.q, k.tables);
  }
}

namespace {

// First-fit allocator over [0, cap) entries; alloc returns -1 when full.
struct FitAlloc {
  int64_t cap;
  int64_t top = 0;
  std::map<int64_t, int64_t> free_blk;  // off -> len
  explicit FitAlloc(int64_t c) : cap(c) {}
  static int64_t round(int64_t len) { return (len + 7) / 8 * 8; }
  int64_t alloc(int64_t len) {
    len = round(len);
    for (auto it = free_blk.begin(); it != free_blk.end(); ++it)
      if (it->second >= len) {
        int64_t off = it->first, rem = it->second - len;
        free_blk.erase(it);
        if (rem) free_blk.emplace(off + len, rem);
        return off;
      }
    if (!free_blk.empty()) {
      auto last = std::prev(free_blk.end());
      if (last->first + last->second == top && last->first + len <= cap) {
        int64_t off = last->first;
        free_blk.erase(last);
        top = off + len;
        return off;
      }
    }
    if (top + len > cap) return -1;
    int64_t off = top;
    top += len;
    return off;
  }
  void release(int64_t off, int64_t len) {
    len = round(len);
    auto it = free_blk.emplace(off, len).first;
    auto nx = std::next(it);
    if (nx != free_blk.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_blk.erase(nx);
    }
    if (it != free_blk.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_blk.erase(it);
      }
    }
  }
};

// A knot's groups before they are laid out.
struct PGroup {
  int32_t kind;         // TASK_SERIAL / TASK_TILE
  int32_t first, count; // knot-local steps
  int32_t flags;
  int32_t n_tiles;
};

}  // namespace

std::vector<uint8_t> build_image(const std::vector<const PlanKnot*>& knots) {
  ImgHeader h;
  std::memset(&h, 0, sizeof(h));
  h.magic = kMagic;
  h.precision = knots.empty() ? 0 : knots[0]->precision;

  std::vector<KnotDesc> kd;
  std::vector<TensorDesc> td;
  std::vector<StepDesc> sd;
  std::vector<VtxDesc> vd;
  std::vector<int32_t> vslot;
  std::vector<MEdge> md;
  std::vector<int32_t> members;
  std::vector<Factor> fac;
  std::vector<int32_t> tables;
  std::vector<int8_t> eps;
  std::vector<int32_t> comps;
  std::vector<TaskDesc> tasks;
  std::vector<GroupDesc> groups;
  std::vector<std::pair<double, int32_t>> roots;  // (-estimated chain time, group)
  int32_t lds_used = 0;

  int64_t arena = 0, n_edges = 0, n_medges = 0;
  for (size_t ki = 0; ki < knots.size(); ++ki) {
    const PlanKnot& k = *knots[ki];
    const int32_t q = k.q;
    const int32_t t0 = (int32_t)td.size();
    const int32_t s0 = (int32_t)sd.size();
    KnotDesc d;
    std::memset(&d, 0, sizeof(d));
    d.t_re = k.t_re;
    d.t_im = k.t_im;
    d.q = q;
    d.edge_off = (int32_t)n_edges;
    d.n_edges = k.n_edges;
    d.medge_off = (int32_t)n_medges;
    d.n_medges = (int32_t)k.medges.size();
    d.vtx_off = (int32_t)vd.size();
    d.n_vtx = (int32_t)k.vtx.size();
    d.factor_off = (int32_t)fac.size();
    d.n_factors = (int32_t)k.factors.size();
    d.comp_off = (int32_t)comps.size();
    d.n_comps = (int32_t)k.comps.size();
    d.n_iso = k.n_iso;
    d.out_slot = (int32_t)ki;
    d.step_off = s0;
    d.n_steps = (int32_t)k.steps.size();
    for (int8_t e : k.eps) eps.push_back(e);
    for (auto& m : k.medges) {
      md.push_back({(int32_t)members.size(), (int32_t)m.size()});
      for (int32_t e : m) members.push_back(e);
    }
    for (auto& f : k.factors) fac.push_back(f);
    for (int32_t c : k.comps) comps.push_back(t0 + c);
    const int64_t abase = arena;
    for (auto& t : k.tensors) td.push_back({abase + t.off, (int32_t)t.size, -1});
    arena += (k.arena_elems + 15) / 16 * 16;
    for (auto& v : k.vtx) {
      vd.push_back({t0 + v.tensor, (int32_t)v.nbr.size(), (int32_t)vslot.size(),
                    v.keep_center ? 1 : 0});
      for (int32_t m : v.medge) vslot.push_back(m);
    }
    // steps + tables (precomputed per knot)
    const int32_t tab0 = (int32_t)tables.size();
    tables.insert(tables.end(), k.tables.begin(), k.tables.end());
    for (size_t si = 0; si < k.steps.size(); ++si) {
      const PStep& s = k.steps[si];
      StepDesc x;
      x.a = t0 + s.a;
      x.b = t0 + s.b;
      x.c = t0 + s.c;
      auto pw = [&](size_t r) {
        int64_t v = 1;
        for (size_t i = 0; i < r; ++i) v *= q;
        return (int32_t)v;
      };
      x.nb = pw(s.bs.size());
      x.nm = pw(s.ms.size());
      x.nn = pw(s.ns.size());
      x.nk = pw(s.ks.size());
      x.tab = tab0 + k.tab_off[si];
      const int64_t outs = (int64_t)x.nb * x.nm * x.nn;
      const int32_t tile = k.step_tile[si];
      x.n_tiles = k.big[si] ? (int32_t)((outs + tile - 1) / tile) : 0;
      x.tile = tile;
      sd.push_back(x);
    }

    // ---- groups of this knot
    std::vector<PGroup> pg;
    {
      PGroup cur{TASK_SERIAL, 0, 0, TF_SETUP, 0};
      bool open = true;
      for (int32_t si = 0; si < (int32_t)k.steps.size(); ++si) {
        if (!k.big[si]) {
          if (!open) {
            cur = PGroup{TASK_SERIAL, si, 0, 0, 0};
            open = true;
          }
          cur.count++;
          continue;
        }
        if (open) {
          pg.push_back(cur);
          open = false;
        }
        pg.push_back(PGroup{TASK_TILE, si, 1, 0, sd[s0 + si].n_tiles});
      }
      if (!open) cur = PGroup{TASK_SERIAL, (int32_t)k.steps.size(), 0, 0, 0};
      cur.flags |= TF_FINAL;
      pg.push_back(cur);
    }

    // ---- LDS homes: tensors produced and consumed inside one serial group
    {
      const int32_t nt = (int32_t)k.tensors.size();
      std::vector<int32_t> consumer(nt, -1);  // step index, or n_steps for the final
      for (int32_t si = 0; si < (int32_t)k.steps.size(); ++si) {
        consumer[k.steps[si].a] = si;
        consumer[k.steps[si].b] = si;
      }
      for (int32_t c : k.comps) consumer[c] = (int32_t)k.steps.size();
      std::vector<int32_t> producer(nt, -1);  // -1: vertex tensor (setup)
      for (int32_t si = 0; si < (int32_t)k.steps.size(); ++si) producer[k.steps[si].c] = si;
      const int64_t es = elem_bytes(k.precision);
      const int64_t cap = k.lds_bytes / es;
      for (const PGroup& g : pg) {
        if (g.kind != TASK_SERIAL) continue;
        const int32_t lo = g.first, hi = g.first + g.count;  // steps [lo, hi)
        auto inside = [&](int32_t t) {
          int32_t c = consumer[t];
          if (c < 0) return false;
          if (c == (int32_t)k.steps.size()) return (g.flags & TF_FINAL) != 0;
          return c >= lo && c < hi;
        };
        FitAlloc la(cap);
        std::vector<int64_t> loff(nt, -1);
        int64_t peak = 0;
        if (g.flags & TF_SETUP)
          for (const auto& v : k.vtx)
            if (inside(v.tensor)) {
              int64_t o = la.alloc(k.tensors[v.tensor].size);
              if (o >= 0) loff[v.tensor] = o;
            }
        peak = std::max(peak, la.top);
        for (int32_t si = lo; si < hi; ++si) {
          const PStep& s = k.steps[si];
          if (inside(s.c)) {
            int64_t o = la.alloc(k.tensors[s.c].size);
            if (o >= 0) loff[s.c] = o;
          }
          peak = std::max(peak, la.top);
          for (int32_t op : {s.a, s.b})
            if (loff[op] >= 0) la.release(loff[op], k.tensors[op].size);
        }
        for (int32_t t = 0; t < nt; ++t)
          if (loff[t] >= 0) td[t0 + t].lds_off = (int32_t)loff[t];
        lds_used = std::max<int32_t>(lds_used, (int32_t)(peak * es));
      }
    }

    // ---- lay the groups out as tasks
    double est = 0;
    const int32_t g0 = (int32_t)groups.size();
    for (size_t gi = 0; gi < pg.size(); ++gi) {
      const PGroup& g = pg[gi];
      GroupDesc G;
      G.knot = (int32_t)ki;
      G.first_task = (int32_t)tasks.size();
      G.next = gi + 1 < pg.size() ? g0 + (int32_t)gi + 1 : -1;
      G.n_pred = gi == 0 ? 0 : groups.back().n_tasks;
      if (g.kind == TASK_SERIAL) {
        // tensors made here: vertex tensors (ids t0..) and step outputs, consecutive
        const int32_t n_vt = (int32_t)(k.tensors.size() - k.steps.size());
        int32_t lo = (g.flags & TF_SETUP) ? t0 : t0 + n_vt + g.first;
        int32_t len = ((g.flags & TF_SETUP) ? n_vt : 0) + g.count;
        tasks.push_back({TASK_SERIAL, (int32_t)ki, g0 + (int32_t)gi, s0 + g.first, g.count, g.flags,
                         lo, len});
        G.n_tasks = 1;
        for (int32_t si = g.first; si < g.first + g.count; ++si) {
          const StepDesc& x = sd[s0 + si];
          est += 1.0 + double(x.nb) * x.nm * x.nn * x.nk / 512.0;
        }
      } else {
        for (int32_t tl = 0; tl < g.n_tiles; ++tl)
          tasks.push_back({TASK_TILE, (int32_t)ki, g0 + (int32_t)gi, s0 + g.first, tl, 0, 0, 0});
        G.n_tasks = g.n_tiles;
        const StepDesc& x = sd[s0 + g.first];
        est += 3.0 + double(x.tile) * x.nk / 512.0;
      }
      groups.push_back(G);
    }
    roots.emplace_back(-est, g0);
    kd.push_back(d);
    n_edges += k.n_edges;
    n_medges += (int64_t)k.medges.size();
  }
  std::stable_sort(roots.begin(), roots.end(),
                   [](const std::pair<double, int32_t>& a, const std::pair<double, int32_t>& b) {
                     return a.first < b.first;
                   });
  std::vector<int32_t> root_tasks;
  for (auto& r : roots) root_tasks.push_back(groups[r.second].first_task);

  h.n_tasks = (int32_t)tasks.size();
  h.n_knots = (int32_t)knots.size();
  h.n_tensors = (int32_t)td.size();
  h.n_steps = (int32_t)sd.size();
  h.n_vtx = (int32_t)vd.size();
  h.n_medges = (int32_t)md.size();
  h.n_members = (int32_t)members.size();
  h.n_factors = (int32_t)fac.size();
  h.n_tables = (int32_t)tables.size();
  h.n_groups = (int32_t)groups.size();
  h.n_edges = (int32_t)n_edges;
  h.n_roots = (int32_t)root_tasks.size();
  h.lds_bytes = (lds_used + 255) / 256 * 256;

  std::vector<uint8_t> img(sizeof(ImgHeader));
  {
    size_t total = 4096 + 256 * 18;
    total += tasks.size() * sizeof(TaskDesc) + groups.size() * sizeof(GroupDesc) +
             root_tasks.size() * 4 + kd.size() * sizeof(KnotDesc) +
             td.size() * sizeof(TensorDesc) + sd.size() * sizeof(StepDesc) +
             vd.size() * sizeof(VtxDesc) + vslot.size() * 4 + md.size() * sizeof(MEdge) +
             members.size() * 4 + fac.size() * sizeof(Factor) + tables.size() * 4 + eps.size() +
             comps.size() * 4;
    img.reserve(total);
  }
  h.o_tasks = put(img, tasks);
  h.o_groups = put(img, groups);
  h.o_roots = put(img, root_tasks);
  h.o_knots = put(img, kd);
  h.o_tensors = put(img, td);
  h.o_steps = put(img, sd);
  h.o_vtx = put(img, vd);
  h.o_vslot = put(img, vslot);
  h.o_medges = put(img, md);
  h.o_members = put(img, members);
  h.o_factors = put(img, fac);
  h.o_tables = put(img, tables);
  h.o_eps = put(img, eps);
  h.o_comps = put(img, comps);
  h.image_bytes = align256((int64_t)img.size());
  img.resize(h.image_bytes);
  // runtime state: control words, ready queue, pending counters, tensor
  // states, weights
  h.state_off = h.image_bytes;
  int64_t st = CTRL_WORDS * 4;
  h.o_queue = st;
  st = align256(st + 4 * (int64_t)tasks.size());
  h.o_pending = st;
  st = align256(st + 4 * (int64_t)groups.size());
  h.o_tstate = st;
  st = align256(st + (int64_t)td.size() * (int64_t)sizeof(TensorState));
  h.o_weights = st;
  st = align256(st + 16 * (n_edges + n_medges));
  h.state_bytes = st;
  h.arena_off = align256(h.state_off + h.state_bytes);
  h.arena_elems = std::max<int64_t>(arena, 16);
  h.workspace_bytes = align256(h.arena_off + h.arena_elems * elem_bytes(h.precision));
  std::memcpy(img.data(), &h, sizeof(h));
  return img;
}

}  // namespace kn
