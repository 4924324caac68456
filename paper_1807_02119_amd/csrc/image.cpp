// image.cpp -- lay knot plans out as a device program (see program.h).
//
// Each plan is first turned into a relocatable section (make_section, run
// once per plan, on the planning thread): descriptors, gather tables, task
// groups and LDS homes with knot-local ids.  An image for one knot or a batch
// is then the concatenation of sections with ids and offsets shifted
// (build_image), which is a linear copy.
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
#include <atomic>
#include <climits>
#include <cmath>
#include <cstring>
#include <functional>
#include <numeric>
#include <thread>

#include "checks.h"
#include "internal.h"

namespace kn {

namespace {

// Element strides of spins in tensors stored row-major in a spin order (last
// spin fastest): load(order) records each spin's stride, 0 for spins the
// order does not hold; append(group) writes the strides of a group's spins.
struct StrideMap {
  std::vector<int32_t> stride, stamp;
  int32_t cur = 0;
  const int32_t* qpow;
  StrideMap(int32_t n_spins, const int32_t* qp) : stride(n_spins, 0), stamp(n_spins, 0), qpow(qp) {}
  void load(const SpinList& order) {
    ++cur;
    const int32_t r = order.size();
    for (int32_t j = 0; j < r; ++j) {
      stride[order[j]] = qpow[r - 1 - j];
      stamp[order[j]] = cur;
    }
  }
  void append(const SpinList& group, std::vector<int32_t>& out) const {
    for (int32_t sp : group) out.push_back(stamp[sp] == cur ? stride[sp] : 0);
  }
};

// A knot's groups before they are laid out.
struct PGroup {
  int32_t kind;          // TASK_SERIAL / TASK_TILE / TASK_REDUCE
  int32_t first, count;  // knot-local steps
  int32_t flags;
  int32_t n_tiles;       // tile and reduce groups: tasks
  // serial groups of one dependency level: its steps shared out to several
  // tasks as (first, count) chunks; empty = one task for all the steps
  std::vector<std::pair<int32_t, int32_t>> chunks;
  bool fork = false;  // the chunks are the concurrent subtree tasks of a forked run
};

// Estimated time of a serial step (arbitrary units: one per step plus one per
// 512 multiply-adds).  A task of a level-split run aims at 1/32 of the split
// threshold, and a level has at most kSplitMaxChunks tasks.
inline double step_est(const StepDesc& x) {
  return 1.0 + double(x.nb) * x.nm * x.nn * x.nk / 512.0;
}
constexpr int32_t kSplitMaxChunks = 16;

}  // namespace

void Section::assign(const SectionBuild& b) {
  size_t words = 0;
  auto count = [&](const auto& v) {
    words += (v.size() * sizeof(v[0]) + 7) / 8;
  };
  count(b.td), count(b.sd), count(b.vd), count(b.vslot), count(b.md), count(b.members);
  count(b.fac), count(b.strides), count(b.comps), count(b.pins), count(b.consts);
  count(b.tasks), count(b.groups);
  block.reset(new uint64_t[std::max<size_t>(1, words)]);
  uint64_t* at = block.get();
  auto take = [&](auto& dst, const auto& v) {
    using T = typename std::decay_t<decltype(v)>::value_type;
    static_assert(alignof(T) <= 8, "section arrays are 8-byte aligned");
    const size_t bytes = v.size() * sizeof(T);
    if (bytes) std::memcpy(at, v.data(), bytes);
    dst.p = reinterpret_cast<const T*>(at);
    dst.n = v.size();
    at += (bytes + 7) / 8;
  };
  take(td, b.td), take(sd, b.sd), take(vd, b.vd), take(vslot, b.vslot), take(md, b.md);
  take(members, b.members), take(fac, b.fac), take(strides, b.strides), take(comps, b.comps);
  take(pins, b.pins), take(consts, b.consts), take(tasks, b.tasks), take(groups, b.groups);
  kd = b.kd;
  est = b.est;
  lds_used = b.lds_used;
  arena_elems = b.arena_elems;
}

void make_section(PlanKnot& k) {
  SectionBuild S;
  const int32_t q = k.q;
  KnotDesc& d = S.kd;
  std::memset(&d, 0, sizeof(d));
  d.t_re = k.t_re;
  d.t_im = k.t_im;
  d.q = q;
  d.n_edges = k.n_edges;
  d.n_medges = (int32_t)k.medge_off.size() - 1;
  d.n_vtx = (int32_t)k.vtx.size();
  d.n_factors = (int32_t)k.factors.size();
  d.n_comps = (int32_t)k.comps.size();
  d.n_iso = k.n_iso;
  d.n_steps = (int32_t)k.steps.size();
  d.grad = k.gradient ? 1 : 0;
  d.n_slices = k.n_slices;
  d.n_slice_spins = k.n_slice_spins;
  // spin ids are below n_spins; powers of q up to the largest rank
  int32_t n_spins = 1, max_rank = 0;
  for (const auto& t : k.tensors) {
    max_rank = std::max(max_rank, t.spins.size());
    for (int32_t sp : t.spins) n_spins = std::max(n_spins, sp + 1);
  }
  std::vector<int32_t> qpow(max_rank + 1);
  qpow[0] = 1;
  for (int32_t i = 1; i <= max_rank; ++i) qpow[i] = qpow[i - 1] * q;
  StrideMap smap(n_spins, qpow.data());
  const size_t n_md = k.medge_off.size() - 1;
  S.md.reserve(n_md);
  S.members.reserve(k.medge_mem.size());
  for (size_t m = 0; m < n_md; ++m) {
    if (m < k.medge_const.size() && k.medge_const[m] >= 0) {
      S.md.push_back({k.medge_const[m], -1});  // derived: x is a constant
      continue;
    }
    S.md.push_back({(int32_t)S.members.size(), k.medge_off[m + 1] - k.medge_off[m]});
    for (int32_t j = k.medge_off[m]; j < k.medge_off[m + 1]; ++j) S.members.push_back(k.medge_mem[j]);
  }
  S.consts.reserve(2 * k.consts.size());
  for (const auto& c : k.consts) {
    S.consts.push_back(c.real());
    S.consts.push_back(c.imag());
  }
  S.fac = k.factors;
  S.comps = k.comps;
  S.td.reserve(k.tensors.size());
  for (auto& t : k.tensors) S.td.push_back({t.off, (int32_t)t.size, -1});
  S.arena_elems = (k.arena_elems + 15) / 16 * 16;
  {
    size_t n_tab = 0, n_slot = 0, n_pin = 0;
    for (const auto& v : k.vtx) {
      n_slot += v.medge.size();
      n_pin += 2 * v.pin_medge.size();
      if (v.adjoint >= 0) n_tab += 1 + v.nbr.size();
    }
    for (const auto& st : k.steps)
      n_tab += 2 * st.bs.size() + st.ms.size() + 2 * st.ks.size() + st.ns.size();
    S.strides.reserve(n_tab);
    S.vslot.reserve(n_slot);
    S.pins.reserve(n_pin);
    S.vd.reserve(k.vtx.size());
  }
  for (auto& v : k.vtx) {
    int32_t adj_str = -1;
    if (v.adjoint >= 0) {  // the adjoint's own spin order differs from F_v's
      adj_str = (int32_t)S.strides.size();
      SpinList vs;
      if (v.keep_center) vs.push_back(v.center);
      for (int32_t w : v.nbr) vs.push_back(w);
      smap.load(k.tensors[v.adjoint].spins);
      smap.append(vs, S.strides);
    }
    S.vd.push_back({v.tensor, (int32_t)v.nbr.size(), (int32_t)S.vslot.size(),
                    v.seed ? -1 : (v.keep_center ? 1 : 0), v.adjoint, v.comp, adj_str,
                    (int32_t)S.pins.size() / 2, v.pin_medge.size()});
    for (int32_t m : v.medge) S.vslot.push_back(m);
    for (int32_t j = 0; j < v.pin_medge.size(); ++j) {
      S.pins.push_back(v.pin_medge[j]);
      S.pins.push_back(v.pin_slice[j]);
    }
  }
  // steps + tables
  S.sd.reserve(k.steps.size());
  for (size_t si = 0; si < k.steps.size(); ++si) {
    const PStep& s = k.steps[si];
    StepDesc x{};
    x.a = s.a;
    x.b = s.b;
    x.c = s.c;
    x.nb = qpow[s.bs.size()];
    x.nm = qpow[s.ms.size()];
    x.nn = qpow[s.ns.size()];
    x.nk = qpow[s.ks.size()];
    x.str = (int32_t)S.strides.size();
    x.ranks = (int32_t)(s.bs.size() | (s.ms.size() << 8) | (s.ks.size() << 16) |
                        (s.ns.size() << 24));
    smap.load(k.tensors[s.a].spins);
    smap.append(s.bs, S.strides);
    smap.append(s.ms, S.strides);
    smap.append(s.ks, S.strides);
    smap.load(k.tensors[s.b].spins);
    smap.append(s.bs, S.strides);
    smap.append(s.ks, S.strides);
    smap.append(s.ns, S.strides);
    const PTiling& t = k.tiling[si];
    x.mode = t.mode;
    x.n_tiles = t.mode == STEP_SERIAL ? 0 : t.n_tiles;
    x.tile = t.tile;
    x.n_mb = t.n_mb;
    x.n_nb = t.n_nb;
    x.n_ks = t.n_ks;
    x.kseg = t.kseg;
    x.partial = t.partial >= 0 ? (int32_t)t.partial : -1;
    x.lvl = t.level;
    S.sd.push_back(x);
  }

  // ---- groups
  std::vector<PGroup> pg;
  {
    PGroup cur{TASK_SERIAL, 0, 0, TF_SETUP, 0};
    bool open = true;
    for (int32_t si = 0; si < (int32_t)k.steps.size(); ++si) {
      if (k.tiling[si].mode == STEP_SERIAL) {
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
      pg.push_back(PGroup{TASK_TILE, si, 1, 0, S.sd[si].n_tiles});
      if (S.sd[si].n_ks > 1) {
        const int64_t outs = (int64_t)S.sd[si].nb * S.sd[si].nm * S.sd[si].nn;
        pg.push_back(PGroup{TASK_REDUCE, si, 1, 0, (int32_t)((outs + kReduceChunk - 1) / kReduceChunk)});
      }
    }
    if (!open) cur = PGroup{TASK_SERIAL, (int32_t)k.steps.size(), 0, 0, 0};
    cur.flags |= TF_FINAL;
    pg.push_back(cur);
  }
  // ---- forked serial runs (the planner ordered their steps task by task,
  // the top last): the setup alone, the subtree tasks as one group, then the
  // top with the final product
  {
    std::vector<PGroup> out;
    out.reserve(pg.size() + 4);
    for (PGroup& g : pg) {
      if (g.kind != TASK_SERIAL || g.count == 0 || k.tiling[g.first].part < 0) {
        out.push_back(std::move(g));
        continue;
      }
      const int32_t end = g.first + g.count;
      if (g.flags & TF_SETUP) out.push_back(PGroup{TASK_SERIAL, g.first, 0, TF_SETUP, 0, {}});
      PGroup parts{TASK_SERIAL, g.first, 0, 0, 0, {}};
      parts.fork = true;
      int32_t a = g.first;
      while (a < end && k.tiling[a].part != kForkTop) {
        int32_t b = a + 1;
        while (b < end && k.tiling[b].part == k.tiling[a].part) ++b;
        parts.chunks.emplace_back(a, b - a);
        a = b;
      }
      parts.count = a - g.first;
      out.push_back(std::move(parts));
      if (a < end || (g.flags & TF_FINAL))
        out.push_back(PGroup{TASK_SERIAL, a, end - a, g.flags & TF_FINAL, 0, {}});
    }
    pg.swap(out);
  }
  // ---- long serial runs level by level: setup, one group per dependency
  // level (its independent steps in chunks over several tasks), final product
  {
    std::vector<PGroup> out;
    out.reserve(pg.size());
    for (PGroup& g : pg) {
      double est = 0;
      if (g.kind == TASK_SERIAL)
        for (int32_t si = g.first; si < g.first + g.count; ++si) est += step_est(S.sd[si]);
      if (g.kind != TASK_SERIAL || g.count < 2 || est < k.split_est || g.fork ||
          k.tiling[g.first].part >= 0) {
        out.push_back(std::move(g));
        continue;
      }
      if (g.flags & TF_SETUP) out.push_back(PGroup{TASK_SERIAL, g.first, 0, TF_SETUP, 0, {}});
      const int32_t end = g.first + g.count;
      for (int32_t a = g.first; a < end;) {
        int32_t b = a + 1;
        while (b < end && k.tiling[b].level == k.tiling[a].level) ++b;
        PGroup lg{TASK_SERIAL, a, b - a, 0, 0, {}};
        double lev = 0;
        for (int32_t si = a; si < b; ++si) lev += step_est(S.sd[si]);
        const double target = std::max(k.split_est / 32.0, lev / kSplitMaxChunks);
        double acc = 0;
        int32_t c0 = a;
        for (int32_t si = a; si < b; ++si) {
          acc += step_est(S.sd[si]);
          if (acc >= target || si + 1 == b) {
            lg.chunks.emplace_back(c0, si + 1 - c0);
            c0 = si + 1;
            acc = 0;
          }
        }
        out.push_back(std::move(lg));
        a = b;
      }
      if (g.flags & TF_FINAL) out.push_back(PGroup{TASK_SERIAL, end, 0, TF_FINAL, 0, {}});
    }
    pg.swap(out);
  }

  // ---- LDS homes: tensors produced and consumed inside one serial group
  // (gradient plans read every tensor again in the reverse pass: all global)
  if (!k.gradient) {
    const int32_t nt = (int32_t)k.tensors.size();
    const int32_t ns = (int32_t)k.steps.size();
    std::vector<int32_t> consumer(nt, -1);  // step index, or ns for the final product
    for (int32_t si = 0; si < ns; ++si) {
      consumer[k.steps[si].a] = si;
      consumer[k.steps[si].b] = si;
    }
    for (int32_t c : k.comps) consumer[c] = ns;
    const int64_t es = elem_bytes(k.precision);
    const int64_t cap = k.lds_bytes / es;
    // each task of a forked group runs on its own workgroup: one LDS arena
    // per task, and its levels only
    std::vector<std::pair<const PGroup*, std::pair<int32_t, int32_t>>> regions;
    for (const PGroup& g : pg) {
      if (g.kind != TASK_SERIAL) continue;
      if (g.fork)
        for (const auto& c : g.chunks) regions.push_back({&g, c});
      else
        regions.push_back({&g, {g.first, g.count}});
    }
    for (const auto& [gp, range] : regions) {
      const PGroup& g = *gp;
      const int32_t lo = range.first, hi = range.first + range.second;  // steps [lo, hi)
      auto inside = [&](int32_t t) {
        int32_t c = consumer[t];
        if (c < 0) return false;
        if (c == ns) return (g.flags & TF_FINAL) != 0;
        return c >= lo && c < hi;
      };
      auto concurrent = [&](int32_t i) {  // steps i and i + 1 of this task
        return g.fork ? k.tiling[i].level == k.tiling[i + 1].level : same_level(k, i);
      };
      FitAlloc la(cap, 8);
      int64_t peak = 0;
      if (g.flags & TF_SETUP)
        for (const auto& v : k.vtx)
          if (inside(v.tensor)) {
            int64_t o = la.alloc(k.tensors[v.tensor].size);
            if (o >= 0) S.td[v.tensor].lds_off = (int32_t)o;
          }
      peak = std::max(peak, la.top);
      // a level's outputs are placed before any of its operands is released
      for (int32_t si = lo; si < hi;) {
        int32_t sj = si + 1;
        while (sj < hi && concurrent(sj - 1)) ++sj;
        for (int32_t u = si; u < sj; ++u) {
          const PStep& s = k.steps[u];
          if (inside(s.c)) {
            int64_t o = la.alloc(k.tensors[s.c].size);
            if (o >= 0) S.td[s.c].lds_off = (int32_t)o;
          }
        }
        peak = std::max(peak, la.top);
        for (int32_t u = si; u < sj; ++u) {
          const PStep& s = k.steps[u];
          for (int32_t op : {s.a, s.b})
            if (S.td[op].lds_off >= 0) la.release(S.td[op].lds_off, k.tensors[op].size);
        }
        si = sj;
      }
      S.lds_used = std::max<int32_t>(S.lds_used, (int32_t)(peak * es));
    }
  }
  // a 64 x 64 GEMM step stages two 16 x 65 operand chunks in LDS from its
  // start, followed by the offset table of up to 1024 contracted entries; the
  // launch's LDS must hold them (gradient plans included)
  {
    const int64_t es = elem_bytes(k.precision);
    for (const StepDesc& x : S.sd)
      if (x.mode == STEP_GEMM64) {
        const int64_t need = 2 * kGemmChunk * 65 * es + 8 * std::min<int64_t>(x.kseg, 1024);
        S.lds_used = std::max<int32_t>(S.lds_used, (int32_t)std::max<int64_t>(0, need - kLdsArena));
      }
  }

  // ---- operand homes in the step descriptors (global offsets are knot-local)
  for (auto& x : S.sd) {
    auto home = [&](int32_t t) {
      const TensorDesc& d = S.td[t];
      return d.lds_off >= 0 ? -1 - d.lds_off : (int32_t)d.off;
    };
    x.home_a = home(x.a);
    x.home_b = home(x.b);
    x.home_c = home(x.c);
  }

  // ---- tasks
  const int32_t n_vt = (int32_t)(k.tensors.size() - k.steps.size());
  for (size_t gi = 0; gi < pg.size(); ++gi) {
    const PGroup& g = pg[gi];
    GroupDesc G;
    G.knot = 0;
    G.first_task = (int32_t)S.tasks.size();
    G.next = gi + 1 < pg.size() ? (int32_t)gi + 1 : -1;
    G.n_pred = gi == 0 ? 0 : S.groups.back().n_tasks;
    if (g.kind == TASK_SERIAL && !g.chunks.empty()) {
      // one dependency level over several tasks (no setup or final here)
      double longest = 0;
      for (const auto& [cf, cc] : g.chunks) {
        S.tasks.push_back({TASK_SERIAL, 0, (int32_t)gi, cf, cc, 0, n_vt + cf, cc});
        double e = 0;
        for (int32_t si = cf; si < cf + cc; ++si) e += step_est(S.sd[si]);
        longest = std::max(longest, e);
      }
      G.n_tasks = (int32_t)g.chunks.size();
      S.est += 3.0 + longest;
    } else if (g.kind == TASK_SERIAL) {
      // tensors made here: vertex tensors (ids 0..) and step outputs, consecutive
      int32_t lo = (g.flags & TF_SETUP) ? 0 : n_vt + g.first;
      int32_t len = ((g.flags & TF_SETUP) ? n_vt : 0) + g.count;
      S.tasks.push_back({TASK_SERIAL, 0, (int32_t)gi, g.first, g.count, g.flags, lo, len});
      G.n_tasks = 1;
      for (int32_t si = g.first; si < g.first + g.count; ++si) S.est += step_est(S.sd[si]);
    } else if (g.kind == TASK_TILE) {
      for (int32_t tl = 0; tl < g.n_tiles; ++tl)
        S.tasks.push_back({TASK_TILE, 0, (int32_t)gi, g.first, tl, 0, 0, 0});
      G.n_tasks = g.n_tiles;
      const StepDesc& x = S.sd[g.first];
      S.est += 3.0 + double(x.nb) * x.nm * x.nn * x.nk / (512.0 * x.n_tiles);
    } else {
      for (int32_t tl = 0; tl < g.n_tiles; ++tl)
        S.tasks.push_back({TASK_REDUCE, 0, (int32_t)gi, g.first, tl, 0, 0, 0});
      G.n_tasks = g.n_tiles;
      S.est += 2.0;
    }
    S.groups.push_back(G);
  }
  k.sec.assign(S);
}

int64_t build_image_into(const std::vector<const PlanKnot*>& knots,
                         const std::function<uint8_t*(size_t)>& buffer, ImgHeader* header) {
  ImgHeader h;
  std::memset(&h, 0, sizeof(h));
  h.magic = kMagic;
  h.precision = knots.empty() ? 0 : knots[0]->precision;

  // Every plan contributes one unit (knot descriptor) per chain of slices
  // (one for an unsliced plan): unit c of a plan with C chains runs slices
  // c, c + C, ... one after another in its own arena region, its final task
  // starting the next slice on the device.  Arrays that do not depend on the
  // slice (merged edges, members, factors, slot lists, pins, strides, Tait
  // signs) are stored once per plan; tensors, steps, vertices, components,
  // tasks, groups and weight slots once per unit.  Offsets are prefix sums;
  // the units are then written in parallel straight into the image.
  struct PlanOff {
    size_t VS, M, MEM, F, TAB, E, PIN, CONST, unit, zslice;
    int64_t arena;
  };
  struct UnitOff {
    size_t T, S, V, C, TK, G, W;
  };
  const size_t nP = knots.size();
  std::vector<PlanOff> poff(nP + 1);
  std::vector<UnitOff> uoff;
  std::vector<std::pair<int32_t, int32_t>> unit_of;  // (plan, chain)
  int32_t lds_used = 0;
  bool sliced = false;
  int64_t n_queue = 0;
  {
    PlanOff po{};
    UnitOff uo{};
    for (size_t ki = 0; ki < nP; ++ki) {
      poff[ki] = po;
      const PlanKnot& k = *knots[ki];
      const Section& S = k.sec;
      po.VS += S.vslot.size();
      po.M += S.md.size();
      po.MEM += S.members.size();
      po.F += S.fac.size();
      po.TAB += S.strides.size();
      po.E += k.eps.size();
      po.PIN += S.pins.size() / 2;
      po.CONST += S.consts.size() / 2;
      const int32_t chains = std::min(std::max(1, k.slice_chains), k.n_slices);
      po.unit += chains;
      if (k.n_slices > 1) po.zslice += k.n_slices;
      po.arena += S.arena_elems * chains;
      lds_used = std::max(lds_used, S.lds_used);
      sliced |= k.n_slices > 1;
      for (int32_t c = 0; c < chains; ++c) {
        n_queue += (int64_t)S.tasks.size() * ((k.n_slices - c + chains - 1) / chains);
        uoff.push_back(uo);
        unit_of.emplace_back((int32_t)ki, c);
        uo.T += S.td.size();
        uo.S += S.sd.size();
        uo.V += S.vd.size();
        uo.C += S.comps.size();
        uo.TK += S.tasks.size();
        uo.G += S.groups.size();
        uo.W += k.eps.size() + S.md.size();
      }
    }
    poff[nP] = po;
    uoff.push_back(uo);
  }
  const size_t nU = unit_of.size();
  const UnitOff& ut = uoff[nU];
  const PlanOff& pt = poff[nP];
  const size_t nT = ut.T, nS = ut.S, nV = ut.V, nC = ut.C, nTask = ut.TK, nG = ut.G;
  const size_t nVS = pt.VS, nM = pt.M, nMem = pt.MEM, nF = pt.F, nTab = pt.TAB, nE = pt.E,
               nPin = pt.PIN, nConst = pt.CONST;
  const int64_t arena = pt.arena;
  // image layout: header, then each array 256-byte aligned; the buffer is
  // not zero-filled (every array is written in full below, the padding is
  // cleared)
  h.n_tasks = (int32_t)nTask;
  h.n_knots = (int32_t)nU;
  h.n_tensors = (int32_t)nT;
  h.n_steps = (int32_t)nS;
  h.n_vtx = (int32_t)nV;
  h.n_medges = (int32_t)nM;
  h.n_members = (int32_t)nMem;
  h.n_factors = (int32_t)nF;
  h.n_strides = (int32_t)nTab;
  h.n_groups = (int32_t)nG;
  h.n_edges = (int32_t)nE;
  h.n_pins = (int32_t)nPin;
  h.n_wslots = (int32_t)ut.W;
  h.n_outputs = (int32_t)nP;
  h.sliced = sliced ? 1 : 0;
  h.n_consts = (int32_t)nConst;
  if (n_queue > INT32_MAX - 1 || pt.zslice > (size_t)INT32_MAX) return -1;
  h.n_queue = (int32_t)n_queue;
  h.n_zslice = (int32_t)pt.zslice;
  h.lds_bytes = (lds_used + 255) / 256 * 256;
  std::vector<std::pair<int64_t, int64_t>> used;  // (offset, bytes) of each array
  int64_t top = sizeof(ImgHeader);
  auto reserve = [&](size_t n, size_t elem) {
    const int64_t o = align256(top);
    used.emplace_back(o, (int64_t)(n * elem));
    top = o + (int64_t)(n * elem);
    return o;
  };
  h.o_tasks = reserve(nTask, sizeof(TaskDesc));
  h.o_groups = reserve(nG, sizeof(GroupDesc));
  h.o_knots = reserve(nU, sizeof(KnotDesc));
  h.o_tensors = reserve(nT, sizeof(TensorDesc));
  h.o_steps = reserve(nS, sizeof(StepDesc));
  h.o_vtx = reserve(nV, sizeof(VtxDesc));
  h.o_vslot = reserve(nVS, sizeof(int32_t));
  h.o_medges = reserve(nM, sizeof(MEdge));
  h.o_members = reserve(nMem, sizeof(int32_t));
  h.o_factors = reserve(nF, sizeof(Factor));
  h.o_strides = reserve(nTab, sizeof(int32_t));
  h.o_eps = reserve(nE, sizeof(int8_t));
  h.o_comps = reserve(nC, sizeof(int32_t));
  h.o_pins = reserve(2 * nPin, sizeof(int32_t));
  h.o_consts = reserve(2 * nConst, sizeof(double));
  // roots last: the first group of every unit
  const size_t n_roots = nU;
  h.n_roots = (int32_t)n_roots;
  h.o_roots = reserve(n_roots, sizeof(int32_t));
  h.image_bytes = align256(top);
  // runtime state: control words, ready queue, pending counters, tensor
  // states, weights, gradients, slice results
  h.state_off = h.image_bytes;
  int64_t st = CTRL_WORDS * 4;
  h.o_queue = st;
  st = align256(st + 4 * (int64_t)n_queue);
  h.o_pending = st;
  st = align256(st + 4 * (int64_t)nG);
  h.o_tstate = st;
  st = align256(st + (int64_t)nT * (int64_t)sizeof(TensorState));
  h.o_weights = st;
  st = align256(st + 16 * (int64_t)ut.W);
  h.o_mgrad = st;
  st = align256(st + 16 * (int64_t)nM);
  h.o_zslice = st;
  st = align256(st + (int64_t)sizeof(kn_scalar) * (int64_t)pt.zslice);
  h.o_uslice = st;
  st = align256(st + 4 * (int64_t)nU);
  h.state_bytes = st;
  h.arena_off = align256(h.state_off + h.state_bytes);
  h.arena_elems = std::max<int64_t>(arena, 16);
  if (h.arena_elems > INT32_MAX) return -1;  // step homes hold int32 offsets
  h.guard_off = align256(h.arena_off + h.arena_elems * elem_bytes(h.precision));
  h.workspace_bytes = h.guard_off + kGuardBytes;
  if (header) *header = h;
  uint8_t* base = buffer ? buffer((size_t)h.image_bytes) : nullptr;
  if (!base) return buffer ? -2 : h.image_bytes;  // -2: no memory; header only
  {
    int64_t end = sizeof(ImgHeader);
    for (auto [o, n] : used) {
      std::memset(base + end, 0, (size_t)(o - end));
      end = o + n;
    }
    std::memset(base + end, 0, (size_t)(h.image_bytes - end));
  }
  auto arr = [&](int64_t o, auto* type) { return reinterpret_cast<decltype(type)>(base + o); };
  KnotDesc* kd = arr(h.o_knots, (KnotDesc*)nullptr);
  TensorDesc* td = arr(h.o_tensors, (TensorDesc*)nullptr);
  StepDesc* sd = arr(h.o_steps, (StepDesc*)nullptr);
  VtxDesc* vd = arr(h.o_vtx, (VtxDesc*)nullptr);
  int32_t* vslot = arr(h.o_vslot, (int32_t*)nullptr);
  MEdge* md = arr(h.o_medges, (MEdge*)nullptr);
  int32_t* members = arr(h.o_members, (int32_t*)nullptr);
  Factor* fac = arr(h.o_factors, (Factor*)nullptr);
  int32_t* strides = arr(h.o_strides, (int32_t*)nullptr);
  int8_t* eps = arr(h.o_eps, (int8_t*)nullptr);
  int32_t* comps = arr(h.o_comps, (int32_t*)nullptr);
  int32_t* pins = arr(h.o_pins, (int32_t*)nullptr);
  double* consts = arr(h.o_consts, (double*)nullptr);
  TaskDesc* tasks = arr(h.o_tasks, (TaskDesc*)nullptr);
  GroupDesc* groups = arr(h.o_groups, (GroupDesc*)nullptr);
  // (-estimated chain time, root task) of the first unit of every chain
  std::vector<std::pair<double, int32_t>> roots(nU, {0.0, -1});

  auto place = [&](size_t ui) {
    const auto [pk, slice] = unit_of[ui];
    const PlanKnot& k = *knots[pk];
    const Section& S = k.sec;
    const PlanOff& o = poff[pk];
    const UnitOff& u = uoff[ui];
    const int32_t chains = std::min(std::max(1, k.slice_chains), k.n_slices);
    const int64_t arena0 = o.arena + S.arena_elems * slice;
    const size_t TAB0 = o.TAB, VS0 = o.VS, MEM0 = o.MEM, PIN0 = o.PIN;
    if (slice == 0) {  // per-plan arrays
      std::copy(S.vslot.begin(), S.vslot.end(), vslot + VS0);
      for (size_t i = 0; i < S.md.size(); ++i) {
        MEdge m = S.md[i];
        if (m.n_members >= 0) m.member_off += (int32_t)MEM0;  // constants stay plan-local
        md[o.M + i] = m;
      }
      std::copy(S.members.begin(), S.members.end(), members + MEM0);
      std::copy(S.fac.begin(), S.fac.end(), fac + o.F);
      std::copy(S.strides.begin(), S.strides.end(), strides + TAB0);
      std::copy(k.eps.begin(), k.eps.end(), eps + o.E);
      std::copy(S.pins.begin(), S.pins.end(), pins + 2 * PIN0);
      std::copy(S.consts.begin(), S.consts.end(), consts + 2 * o.CONST);
    }
    KnotDesc x = S.kd;
    x.edge_off = (int32_t)o.E;
    x.medge_off = (int32_t)o.M;
    x.vtx_off = (int32_t)u.V;
    x.factor_off = (int32_t)o.F;
    x.comp_off = (int32_t)u.C;
    x.step_off = (int32_t)u.S;
    x.slice = slice;
    x.slice_step = chains;
    x.plan_slot = (int32_t)pk;
    x.out_slot = k.n_slices > 1 ? (int32_t)o.zslice : (int32_t)pk;
    x.group_off = (int32_t)u.G;
    x.n_groups = (int32_t)S.groups.size();
    x.tensor_off = (int32_t)u.T;
    x.n_tensors = (int32_t)S.td.size();
    x.w_off = (int32_t)u.W;
    x.const_off = (int32_t)o.CONST;
    kd[ui] = x;
    const int32_t t0 = (int32_t)u.T, s0 = (int32_t)u.S, g0 = (int32_t)u.G, tk0 = (int32_t)u.TK;
    for (size_t i = 0; i < S.td.size(); ++i) {
      TensorDesc t = S.td[i];
      t.off += arena0;
      td[t0 + i] = t;
    }
    for (size_t i = 0; i < S.sd.size(); ++i) {
      StepDesc st = S.sd[i];
      st.a += t0;
      st.b += t0;
      st.c += t0;
      st.str += (int32_t)TAB0;
      if (st.home_a >= 0) st.home_a += (int32_t)arena0;
      if (st.home_b >= 0) st.home_b += (int32_t)arena0;
      if (st.home_c >= 0) st.home_c += (int32_t)arena0;
      if (st.partial >= 0) st.partial += (int32_t)arena0;
      sd[s0 + i] = st;
    }
    for (size_t i = 0; i < S.vd.size(); ++i) {
      VtxDesc v = S.vd[i];
      v.tensor += t0;
      if (v.adjoint >= 0) {
        v.adjoint += t0;
        v.adj_str += (int32_t)TAB0;
      }
      v.slot_off += (int32_t)VS0;
      v.pin_off += (int32_t)PIN0;
      vd[u.V + i] = v;
    }
    for (size_t i = 0; i < S.comps.size(); ++i) comps[u.C + i] = S.comps[i] + t0;
    for (size_t i = 0; i < S.tasks.size(); ++i) {
      TaskDesc t = S.tasks[i];
      t.knot = (int32_t)ui;
      t.group += g0;
      t.first += s0;
      t.state_lo += t0;
      tasks[tk0 + i] = t;
    }
    const size_t ng = S.groups.size();
    for (size_t i = 0; i < ng; ++i) {
      GroupDesc g = S.groups[i];
      g.knot = (int32_t)ui;
      g.first_task += tk0;
      if (g.next >= 0) g.next += g0;
      groups[g0 + i] = g;
    }
    const double per_chain = (double)((k.n_slices - slice + chains - 1) / chains);
    roots[ui] = {-S.est * per_chain, tk0 + S.groups[0].first_task};
  };
  // a few units per thread on the host pool when it is idle; small images,
  // and images built while the pool plans, are laid out on the calling thread
  const size_t nth = std::min<size_t>(std::max<size_t>(1, nU / 16), (size_t)usable_cpus());
  std::atomic<size_t> next{0};
  auto worker = [&] {
    for (size_t ui; (ui = next.fetch_add(1)) < nU;) place(ui);
  };
  if (!parallel_run_idle((int32_t)std::min<size_t>(nth, 16), worker)) worker();
  {
    std::vector<std::pair<double, int32_t>> rs;
    rs.reserve(n_roots);
    for (auto& r : roots)
      if (r.second >= 0) rs.push_back(r);
    std::stable_sort(rs.begin(), rs.end(),
                     [](const std::pair<double, int32_t>& a, const std::pair<double, int32_t>& b) {
                       return a.first < b.first;
                     });
    int32_t* root_tasks = arr(h.o_roots, (int32_t*)nullptr);
    for (size_t i = 0; i < rs.size(); ++i) root_tasks[i] = rs[i].second;
  }
  std::memcpy(base, &h, sizeof(h));
  return h.image_bytes;
}

Bytes build_image(const std::vector<const PlanKnot*>& knots, bool header_only) {
  Bytes img;
  ImgHeader h;
  if (header_only) {
    if (build_image_into(knots, nullptr, &h) < 0) return {};
    img.resize(sizeof(h));
    std::memcpy(img.data(), &h, sizeof(h));
    return img;
  }
  const int64_t n = build_image_into(
      knots,
      [&](size_t bytes) {
        img.resize(bytes);
        return img.data();
      },
      nullptr);
  if (n < 0) return {};
  return img;
}

}  // namespace kn

// ------------------------------------------------------------------ validation

extern "C" kn_status kn_image_check(const void* image, size_t bytes, int32_t* status) {
  using namespace kn;
  if (!image || !status || bytes < sizeof(ImgHeader) ||
      (reinterpret_cast<uintptr_t>(image) & 7) != 0)
    return KN_E_INVALID;
  const uint8_t* img = reinterpret_cast<const uint8_t*>(image);
  const ImgHeader& h = *reinterpret_cast<const ImgHeader*>(img);
  if (h.magic != kMagic || h.image_bytes < (int64_t)sizeof(ImgHeader) ||
      (uint64_t)h.image_bytes > bytes)
    return KN_E_INVALID;
  status[0] = CHK_OK;
  status[1] = status[2] = -1;
  status[3] = 0;
  // every section inside the image (info: the section's number)
  const struct {
    int64_t off, n, size;
  } sec[] = {{h.o_tasks, h.n_tasks, sizeof(TaskDesc)},     {h.o_groups, h.n_groups, sizeof(GroupDesc)},
             {h.o_knots, h.n_knots, sizeof(KnotDesc)},     {h.o_tensors, h.n_tensors, sizeof(TensorDesc)},
             {h.o_steps, h.n_steps, sizeof(StepDesc)},     {h.o_vtx, h.n_vtx, sizeof(VtxDesc)},
             {h.o_strides, h.n_strides, sizeof(int32_t)}, {h.o_roots, h.n_roots, sizeof(int32_t)}};
  for (int32_t i = 0; i < (int32_t)(sizeof(sec) / sizeof(sec[0])); ++i)
    if (sec[i].n < 0 || !range_in(sec[i].off, sec[i].n * sec[i].size, h.image_bytes) ||
        (sec[i].off & 3) != 0) {
      status[0] = CHK_TASK;
      status[3] = i;
      return KN_OK;
    }
  {  // the component list, whose length the knot records give
    const KnotDesc* kds = reinterpret_cast<const KnotDesc*>(img + h.o_knots);
    int64_t end = 0;
    for (int32_t i = 0; i < h.n_knots; ++i) {
      if (kds[i].comp_off < 0 || kds[i].n_comps < 0) {
        status[0] = CHK_TASK;
        return KN_OK;
      }
      end = std::max<int64_t>(end, (int64_t)kds[i].comp_off + kds[i].n_comps);
    }
    if (!range_in(h.o_comps, end * 4, h.image_bytes)) {
      status[0] = CHK_TASK;
      return KN_OK;
    }
  }
  if (h.arena_elems < 0 || h.guard_off < h.arena_off + h.arena_elems * elem_bytes(h.precision) ||
      h.workspace_bytes < h.guard_off + kGuardBytes) {
    status[0] = CHK_EXTENT;
    return KN_OK;
  }
  const ImageView v{&h,
                    reinterpret_cast<const TaskDesc*>(img + h.o_tasks),
                    reinterpret_cast<const GroupDesc*>(img + h.o_groups),
                    reinterpret_cast<const KnotDesc*>(img + h.o_knots),
                    reinterpret_cast<const TensorDesc*>(img + h.o_tensors),
                    reinterpret_cast<const StepDesc*>(img + h.o_steps),
                    reinterpret_cast<const VtxDesc*>(img + h.o_vtx),
                    reinterpret_cast<const int32_t*>(img + h.o_strides),
                    reinterpret_cast<const int32_t*>(img + h.o_comps)};
  const int64_t lds_elems = h.lds_bytes / elem_bytes(h.precision);
  for (int32_t t = 0; t < h.n_tasks; ++t) {
    int32_t bad = -1;
    const int32_t rc = task_check(v, t, lds_elems, &bad);
    if (rc != CHK_OK) {
      status[0] = rc;
      status[1] = t;
      status[2] = bad;
      return KN_OK;
    }
  }
  return KN_OK;
}
