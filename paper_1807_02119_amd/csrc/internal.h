// internal.h -- host-side objects behind the opaque handles of kn.h.
#pragma once
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/kn.h"
#include "program.h"

struct kn_tait {
  int32_t n_vertices = 0;
  std::vector<int32_t> uv;    // 2 per edge (edge k = crossing k)
  std::vector<int8_t> eps;    // Tait sign per edge
  std::vector<int8_t> twist;  // twist sign per crossing
  int32_t writhe = 0;
  int32_t tau = 0;
};

namespace kn {

// One knot's part of a device program with knot-local ids and offsets; an
// image is the concatenation of sections with the ids shifted (build_image).
struct Section {
  KnotDesc kd;                      // offsets relative to the section
  std::vector<TensorDesc> td;       // off relative to the knot's arena base
  std::vector<StepDesc> sd;         // a, b, c knot-local; str relative to `strides`
  std::vector<VtxDesc> vd;          // tensor knot-local; slot_off relative to `vslot`
  std::vector<int32_t> vslot;       // merged-edge ids (knot-local, stay local)
  std::vector<MEdge> md;            // member_off relative to `members`
  std::vector<int32_t> members;     // original edge ids (knot-local, stay local)
  std::vector<Factor> fac;          // ids knot-local (stay local)
  std::vector<int32_t> strides;     // spin-group strides of every step
  std::vector<int32_t> comps;       // knot-local tensor ids
  std::vector<TaskDesc> tasks;      // group, first, state_lo knot-local
  std::vector<GroupDesc> groups;    // first_task, next knot-local
  double est = 0;                   // estimated chain time (start priority)
  int32_t lds_used = 0;             // bytes of LDS arena the knot needs
  int64_t arena_elems = 0;
};

// How one step runs: inside a serial task, or as tiles over workgroups.
struct PTiling {
  int32_t mode = 0;     // STEP_SERIAL, STEP_TILES or STEP_GEMM (program.h)
  int32_t tile = 0;     // STEP_TILES: outputs per tile
  int32_t n_mb = 0;     // STEP_GEMM: row blocks and column blocks
  int32_t n_nb = 0;
  int32_t n_ks = 1;     // contracted-index splits (partial sums + reduce task)
  int32_t kseg = 0;     // contracted entries per split
  int32_t n_tiles = 0;  // tasks of the tile group
  int64_t partial = -1; // arena offset of the n_ks x outputs partial sums
};

// One pairwise contraction C = A . B over spin groups.
struct PStep {
  int32_t a, b, c;
  std::vector<int32_t> bs, ms, ns, ks;  // batch, rows (A only), cols (B only), contracted
};

struct PTensor {
  std::vector<int32_t> spins;  // storage order, first = most significant
  int64_t off = 0;             // arena offset (entries), knot-local
  int64_t size = 1;            // q^rank
};

struct PVertex {
  int32_t tensor;
  int32_t center;               // spin of the vertex itself
  bool keep_center;
  std::vector<int32_t> nbr;     // neighbour spins, slot order
  std::vector<int32_t> medge;   // merged edge per slot (knot-local)
};

// Everything about one knot's contraction, in knot-local ids.
struct PlanKnot {
  int32_t q = 3;
  double t_re = 0, t_im = 0;
  int32_t precision = 0;
  bool jones_only = true;
  int32_t n_edges = 0;                          // original Tait edges
  std::vector<int8_t> eps;                      // original Tait signs
  std::vector<std::vector<int32_t>> medges;     // members of each merged edge
  std::vector<Factor> factors;                  // simplification factors
  int32_t n_iso = 0;                            // isolated spins
  std::vector<PTensor> tensors;                 // vertex tensors, then step outputs
  std::vector<PVertex> vtx;
  std::vector<PStep> steps;
  std::vector<int32_t> comps;                   // final scalar tensor per component
  int64_t arena_elems = 0;
  int32_t tile = 256;
  int32_t big_log2 = 16;
  int32_t lds_bytes = 32768;
  std::vector<PTiling> tiling;                  // per step: how it is executed
  Section sec;  // device-program section (make_section)
};

// Lay the knot's plan out as a relocatable device-program section.
void make_section(PlanKnot& k);

// Build the device image for a list of knots (a batch of one or more) by
// concatenating their sections.  out_slot of knot i is i.
std::vector<uint8_t> build_image(const std::vector<const PlanKnot*>& knots);

int64_t elem_bytes(int32_t precision);

}  // namespace kn

struct kn_plan {
  kn::PlanKnot k;
  kn_plan_stats stats{};
  std::vector<uint8_t> image;  // single-knot device image
  uint64_t bwd_workspace = 0;
};

struct kn_batch {
  std::vector<uint8_t> image;
  kn_batch_stats stats{};
  std::vector<int64_t> edge_offset;
  int32_t precision = 0;
  bool jones_only = false;
  int32_t grid_override = 0;
  void* trace = nullptr;
  size_t trace_bytes = 0;
};
