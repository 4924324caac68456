// image.cpp -- lay one or more knot plans out as a device program (see
// program.h): descriptors, gather tables, task list with dependencies.
//
// Tasks of one knot form groups executed strictly one after another (a
// serial run of small steps, or all tiles of one big step); every group waits
// for the previous group's completion tensor, which also guarantees that
// arena memory freed by a group is not reused while that group still reads
// it.  Groups of different knots are independent; they are interleaved
// round-robin, largest knots first, so that many knots are in flight at once.
#include <algorithm>
#include <cmath>
#include <cstring>
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
  // enumerate the group's values, first spin most significant
  for (int64_t idx = 0; idx < n; ++idx) {
    int64_t rem = idx, off = 0;
    for (int64_t i = (int64_t)group.size() - 1; i >= 0; --i) {
      off += (rem % q) * gstride[i];
      rem /= q;
    }
    out[base + idx] = (int32_t)off;
  }
}

struct Group {
  int32_t knot;
  std::vector<TaskDesc> tasks;
};

}  // namespace

std::vector<uint8_t> build_image(const std::vector<const PlanKnot*>& knots) {
  ImgHeader h;
  std::memset(&h, 0, sizeof(h));
  h.magic = kMagic;
  h.precision = knots.empty() ? 0 : knots[0]->precision;
  h.tile = knots.empty() ? 256 : knots[0]->tile;

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
  std::vector<int32_t> deps;
  std::vector<std::vector<Group>> groups(knots.size());

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
    // tensors
    const int64_t abase = arena;
    for (auto& t : k.tensors) td.push_back({abase + t.off, (int32_t)t.size, 1});
    arena += (k.arena_elems + 15) / 16 * 16;
    for (auto& v : k.vtx) {
      vd.push_back({t0 + v.tensor, (int32_t)v.nbr.size(), (int32_t)vslot.size(),
                    v.keep_center ? 1 : 0});
      for (int32_t m : v.medge) vslot.push_back(m);
    }
    // steps + tables
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
      x.tab = (int32_t)tables.size();
      const auto& A = k.tensors[s.a].spins;
      const auto& B = k.tensors[s.b].spins;
      group_table(s.bs, A, q, tables);
      group_table(s.ms, A, q, tables);
      group_table(s.ks, A, q, tables);
      group_table(s.bs, B, q, tables);
      group_table(s.ks, B, q, tables);
      group_table(s.ns, B, q, tables);
      int64_t outs = (int64_t)x.nb * x.nm * x.nn;
      x.n_tiles = k.big[si] ? (int32_t)((outs + k.tile - 1) / k.tile) : 0;
      x.tile = k.tile;
      if (k.big[si]) td[x.c].target = x.n_tiles;
      sd.push_back(x);
    }
    // task groups
    auto& G = groups[ki];
    int32_t prev_done = -1;  // completion tensor of the previous group
    TaskDesc cur;
    bool open = true;
    std::memset(&cur, 0, sizeof(cur));
    cur.kind = TASK_SERIAL;
    cur.knot = (int32_t)ki;
    cur.first = s0;
    cur.count = 0;
    cur.flags = TF_SETUP;
    std::vector<int32_t> produced;  // tensors produced by the open serial group
    for (int32_t v = 0; v < (int32_t)k.vtx.size(); ++v) produced.push_back(t0 + k.vtx[v].tensor);
    std::vector<int32_t> cur_deps;
    auto add_dep = [&](std::vector<int32_t>& dl, int32_t t) {
      if (std::find(dl.begin(), dl.end(), t) == dl.end()) dl.push_back(t);
    };
    auto flush = [&]() {
      if (prev_done >= 0) add_dep(cur_deps, prev_done);
      cur.dep_off = (int32_t)deps.size();
      cur.n_deps = (int32_t)cur_deps.size();
      for (int32_t t : cur_deps) deps.push_back(t);
      // signal every produced tensor that someone outside may wait for
      cur.sig_off = (int32_t)deps.size();
      cur.n_sig = (int32_t)produced.size();
      for (int32_t t : produced) deps.push_back(t);
      Group g;
      g.knot = (int32_t)ki;
      g.tasks.push_back(cur);
      G.push_back(std::move(g));
      prev_done = produced.empty() ? prev_done : produced.back();
      cur_deps.clear();
      produced.clear();
    };
    for (int32_t si = 0; si < (int32_t)k.steps.size(); ++si) {
      const StepDesc& x = sd[s0 + si];
      if (!k.big[si]) {
        if (!open) {
          std::memset(&cur, 0, sizeof(cur));
          cur.kind = TASK_SERIAL;
          cur.knot = (int32_t)ki;
          cur.first = s0 + si;
          cur.count = 0;
          cur.flags = 0;
          open = true;
        }
        for (int32_t op : {x.a, x.b})
          if (std::find(produced.begin(), produced.end(), op) == produced.end())
            add_dep(cur_deps, op);
        cur.count++;
        produced.push_back(x.c);
        continue;
      }
      if (open) {
        flush();
        open = false;
      }
      Group g;
      g.knot = (int32_t)ki;
      std::vector<int32_t> dl{x.a, x.b};
      if (prev_done >= 0) add_dep(dl, prev_done);
      int32_t doff = (int32_t)deps.size();
      for (int32_t t : dl) deps.push_back(t);
      int32_t soff = (int32_t)deps.size();
      deps.push_back(x.c);
      for (int32_t tile = 0; tile < x.n_tiles; ++tile) {
        TaskDesc t;
        std::memset(&t, 0, sizeof(t));
        t.kind = TASK_TILE;
        t.knot = (int32_t)ki;
        t.first = s0 + si;
        t.count = tile;
        t.dep_off = doff;
        t.n_deps = (int32_t)dl.size();
        t.sig_off = soff;
        t.n_sig = 1;
        g.tasks.push_back(t);
      }
      G.push_back(std::move(g));
      prev_done = x.c;
    }
    if (!open) {
      std::memset(&cur, 0, sizeof(cur));
      cur.kind = TASK_SERIAL;
      cur.knot = (int32_t)ki;
      cur.first = s0 + (int32_t)k.steps.size();
      cur.count = 0;
      cur.flags = 0;
      open = true;
    }
    cur.flags |= TF_FINAL;
    for (int32_t c : k.comps)
      if (std::find(produced.begin(), produced.end(), t0 + c) == produced.end())
        add_dep(cur_deps, t0 + c);
    flush();
    kd.push_back(d);
    n_edges += k.n_edges;
    n_medges += (int64_t)k.medges.size();
  }

  // interleave groups round-robin, knots with more groups first
  std::vector<int32_t> order(knots.size());
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(),
                   [&](int32_t a, int32_t b) { return groups[a].size() > groups[b].size(); });
  std::vector<TaskDesc> tasks;
  size_t max_groups = 0;
  for (auto& g : groups) max_groups = std::max(max_groups, g.size());
  for (size_t r = 0; r < max_groups; ++r)
    for (int32_t ki : order)
      if (r < groups[ki].size())
        for (auto& t : groups[ki][r].tasks) tasks.push_back(t);

  h.n_tasks = (int32_t)tasks.size();
  h.n_knots = (int32_t)knots.size();
  h.n_tensors = (int32_t)td.size();
  h.n_steps = (int32_t)sd.size();
  h.n_vtx = (int32_t)vd.size();
  h.n_medges = (int32_t)md.size();
  h.n_members = (int32_t)members.size();
  h.n_factors = (int32_t)fac.size();
  h.n_tables = (int32_t)tables.size();
  h.n_deps = (int32_t)deps.size();
  h.n_edges = (int32_t)n_edges;

  std::vector<uint8_t> img(sizeof(ImgHeader));
  h.o_tasks = put(img, tasks);
  h.o_deps = put(img, deps);
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
  // runtime state: ticket/error words, tensor states, weights
  h.state_off = h.image_bytes;
  int64_t st = 256;  // control words
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
