// checks.h -- consistency predicates of a device program, shared by the
// engine's checking build (each task is checked just before it runs, and a
// task that fails is skipped, so that no access it would make leaves its
// tensor) and by the host's image validator (kn_image_check).
//
// A task passes when every tensor it reads or writes lies inside the memory
// it is addressed in (the global arena or the workgroup's LDS arena), the
// spin-group extents of each of its steps agree with their ranks, the largest
// offset its gathers can form from the stored strides stays inside each
// operand, and every index it holds (tensor ids, steps, tiles, reduction
// chunks, knot and vertex records) is in range.  Offsets inside a tensor are
// then in range by construction: the engine decodes indices below the group
// extents only (the decode itself is pinned by its own tests).
#pragma once
#include <stdint.h>

#include "decode.h"
#include "program.h"

namespace kn {

// Error codes in the runtime state's CTRL_ERROR word (the first error wins;
// CTRL_ERR_TASK / _STEP / _INFO say where).
enum CheckCode : int32_t {
  CHK_OK = 0,
  CHK_QUEUE_WAIT = 1,  // a queue slot stayed empty past the engine's time limit
  CHK_TASK = 2,        // task record out of range (kind, knot, group, steps, tile id)
  CHK_EXTENT = 3,      // a tensor outside its arena (global or LDS)
  CHK_SHAPE = 4,       // group extents disagree with ranks, or outputs with C's size
  CHK_GATHER = 5,      // the largest gathered offset leaves its operand
  CHK_TABLE = 6,       // a serial step's gather tables exceed the LDS table buffer
  CHK_GUARD = 7,       // the guard zone after the arena was overwritten
};

// Bytes of the guard zone that follows the arena in every workspace, and the
// word it is filled with by the checking build.
constexpr int64_t kGuardBytes = 4096;
constexpr uint32_t kGuardWord = 0x6b6e6775u;

KN_HD inline bool range_in(int64_t off, int64_t n, int64_t cap) {
  return off >= 0 && n >= 0 && off <= cap && n <= cap - off;
}

// A tensor's home: >= 0 global arena offset, < 0 LDS arena offset -1 - home.
KN_HD inline bool home_in(int32_t home, int64_t n, int64_t arena, int64_t lds) {
  return home >= 0 ? range_in(home, n, arena) : range_in(-1 - (int64_t)home, n, lds);
}

KN_HD inline bool tensor_in(const TensorDesc& t, int64_t arena, int64_t lds) {
  if (t.size < 0) return false;
  return t.lds_off >= 0 ? range_in(t.lds_off, t.size, lds) : range_in(t.off, t.size, arena);
}

KN_HD inline int64_t qpow(int32_t q, int32_t r) {
  int64_t v = 1;
  for (int32_t i = 0; i < r; ++i) v *= q;
  return v;
}

// Largest offset a group of `rank` spins with element strides `str` adds.
KN_HD inline int64_t group_max(const int32_t* str, int32_t rank, int32_t q) {
  int64_t m = 0;
  for (int32_t i = 0; i < rank; ++i) m += (int64_t)(q - 1) * str[i];
  return m;
}

// One pairwise step of a knot with q states: n_tensors tensor records,
// n_strides stride entries, global arena and LDS arena sizes in entries.
KN_HD inline int32_t step_check(const StepDesc& d, const TensorDesc* tens, int32_t n_tensors,
                                const int32_t* strides, int32_t n_strides, int32_t q,
                                int64_t arena, int64_t lds) {
  if (d.a < 0 || d.a >= n_tensors || d.b < 0 || d.b >= n_tensors || d.c < 0 || d.c >= n_tensors)
    return CHK_TASK;
  const int32_t rb = d.ranks & 255, rm = (d.ranks >> 8) & 255, rk = (d.ranks >> 16) & 255,
                rn = (d.ranks >> 24) & 255;
  if (rb + rm + rk > 31 || rb + rk + rn > 31 || rb + rm + rn > 31) return CHK_SHAPE;
  if (d.nb != qpow(q, rb) || d.nm != qpow(q, rm) || d.nk != qpow(q, rk) || d.nn != qpow(q, rn))
    return CHK_SHAPE;
  const int64_t outs = (int64_t)d.nb * d.nm * d.nn;
  const TensorDesc& A = tens[d.a];
  const TensorDesc& B = tens[d.b];
  const TensorDesc& C = tens[d.c];
  if (outs != C.size) return CHK_SHAPE;
  if (!home_in(d.home_a, A.size, arena, lds) || !home_in(d.home_b, B.size, arena, lds) ||
      !home_in(d.home_c, C.size, arena, lds))
    return CHK_EXTENT;
  if (d.n_ks > 1 && !range_in(d.partial, (int64_t)d.n_ks * outs, arena)) return CHK_EXTENT;
  const int32_t n_str = 2 * rb + rm + 2 * rk + rn;
  if (d.str < 0 || d.str > n_strides - n_str) return CHK_TASK;
  const int32_t* s = strides + d.str;
  for (int32_t i = 0; i < n_str; ++i)
    if (s[i] < 0) return CHK_GATHER;
  const int64_t amax = group_max(s, rb, q) + group_max(s + rb, rm, q) +
                       group_max(s + rb + rm, rk, q);
  const int64_t bmax = group_max(s + rb + rm + rk, rb, q) + group_max(s + 2 * rb + rm + rk, rk, q) +
                       group_max(s + 2 * rb + rm + 2 * rk, rn, q);
  if (amax >= (int64_t)A.size || bmax >= (int64_t)B.size) return CHK_GATHER;
  if (d.mode == STEP_SERIAL && (int64_t)2 * d.nb + d.nm + 2 * d.nk + d.nn > kTabBuf)
    return CHK_TABLE;
  return CHK_OK;
}

// Everything one task touches besides its steps: the task record itself, its
// knot's vertex tensors (setup) and component results (final reduction).
// n_* are the image header's counts.
struct ImageView {
  const ImgHeader* h;
  const TaskDesc* tasks;
  const GroupDesc* groups;
  const KnotDesc* knots;
  const TensorDesc* tens;
  const StepDesc* steps;
  const VtxDesc* vtx;
  const int32_t* strides;
  const int32_t* comps;
};

// The task's own record (not its steps): 0 or a CheckCode.
KN_HD inline int32_t task_record_check(const ImageView& v, int32_t ti, int64_t lds_elems) {
  const ImgHeader& h = *v.h;
  if (ti < 0 || ti >= h.n_tasks) return CHK_TASK;
  const TaskDesc& td = v.tasks[ti];
  if (td.knot < 0 || td.knot >= h.n_knots || td.group < 0 || td.group >= h.n_groups)
    return CHK_TASK;
  const KnotDesc& kd = v.knots[td.knot];
  if (kd.q < 2 || kd.q > 8) return CHK_TASK;
  if (td.kind == TASK_SERIAL) {
    if (td.count < 0 || td.first < 0 || td.first > h.n_steps - td.count) return CHK_TASK;
    if (td.state_len < 0 || td.state_lo < 0 || td.state_lo > h.n_tensors - td.state_len)
      return CHK_TASK;
    if (td.flags & TF_SETUP) {
      if (kd.vtx_off < 0 || kd.n_vtx < 0 || kd.vtx_off > h.n_vtx - kd.n_vtx) return CHK_TASK;
      for (int32_t i = 0; i < kd.n_vtx; ++i) {
        const VtxDesc& vd = v.vtx[kd.vtx_off + i];
        if (vd.tensor < 0 || vd.tensor >= h.n_tensors) return CHK_TASK;
        if (vd.keep_center >= 0 && vd.n_slots > 7) return CHK_SHAPE;
        if (!tensor_in(v.tens[vd.tensor], h.arena_elems, lds_elems)) return CHK_EXTENT;
      }
    }
    if (td.flags & TF_FINAL) {
      if (kd.comp_off < 0 || kd.n_comps < 0) return CHK_TASK;
      for (int32_t i = 0; i < kd.n_comps; ++i) {
        const int32_t t = v.comps[kd.comp_off + i];
        if (t < 0 || t >= h.n_tensors) return CHK_TASK;
        if (!tensor_in(v.tens[t], h.arena_elems, lds_elems) || v.tens[t].size < 1)
          return CHK_EXTENT;
      }
      if (kd.n_slices > 1 && (!range_in(kd.out_slot, kd.n_slices, h.n_zslice) ||
                              !range_in(kd.plan_slot, 1, h.n_outputs)))
        return CHK_TASK;
      if (kd.n_slices <= 1 && !range_in(kd.out_slot, 1, h.n_outputs)) return CHK_TASK;
    }
    return CHK_OK;
  }
  if (td.first < 0 || td.first >= h.n_steps) return CHK_TASK;
  const StepDesc& s = v.steps[td.first];
  if (td.kind == TASK_TILE) {
    if (s.mode == STEP_SERIAL || td.count < 0 || td.count >= s.n_tiles) return CHK_TASK;
    if (s.n_ks < 1 || s.kseg < 1 || (int64_t)(s.n_ks - 1) * s.kseg >= s.nk || s.tile < 1)
      return CHK_TASK;
    // tiles: n_ks contracted ranges times the output tiles (STEP_TILES) or
    // the task's runs of output blocks (STEP_GEMM, STEP_GEMM64)
    const int64_t outs = (int64_t)s.nb * s.nm * s.nn;
    int64_t per_ks;
    if (s.mode == STEP_TILES) {
      per_ks = (outs + s.tile - 1) / s.tile;
    } else {
      const int64_t bm = s.mode == STEP_GEMM64 ? 64 : kGemmBlock;
      if (s.n_mb < 1 || s.n_nb < 1 || s.n_mb * bm < s.nm || s.n_nb * bm < s.nn) return CHK_SHAPE;
      per_ks = ((int64_t)s.nb * s.n_mb * s.n_nb + s.tile - 1) / s.tile;
    }
    if ((int64_t)s.n_ks * per_ks != s.n_tiles) return CHK_TASK;
    return CHK_OK;
  }
  if (td.kind == TASK_REDUCE) {
    const int64_t outs = (int64_t)s.nb * s.nm * s.nn;
    if (s.n_ks < 2 || td.count < 0 || (int64_t)td.count * kReduceChunk >= outs) return CHK_TASK;
    return CHK_OK;
  }
  return CHK_TASK;
}

// Every check of task ti on the host: its record, then each of its steps.
// Returns 0 or a CheckCode; *bad_step receives the failing step, or -1.
inline int32_t task_check(const ImageView& v, int32_t ti, int64_t lds_elems, int32_t* bad_step) {
  *bad_step = -1;
  int32_t rc = task_record_check(v, ti, lds_elems);
  if (rc) return rc;
  const TaskDesc& td = v.tasks[ti];
  const int32_t q = v.knots[td.knot].q;
  const int32_t n = td.kind == TASK_SERIAL ? td.count : 1;
  for (int32_t i = 0; i < n; ++i) {
    if (td.kind == TASK_SERIAL && v.steps[td.first + i].mode != STEP_SERIAL) {
      *bad_step = td.first + i;
      return CHK_TASK;
    }
    rc = step_check(v.steps[td.first + i], v.tens, v.h->n_tensors, v.strides, v.h->n_strides, q,
                    v.h->arena_elems, lds_elems);
    if (rc) {
      *bad_step = td.first + i;
      return rc;
    }
  }
  return CHK_OK;
}

}  // namespace kn
