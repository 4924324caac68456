// engine.hip -- GPU contraction of PACI tensor networks (Sec. III of
// arXiv:1807.02119) for CDNA4 (gfx950).
//
// One persistent kernel executes the task groups of a device program (see
// program.h).  Ready tasks sit in a device queue: a workgroup claims the next
// queue slot, waits until a task id has been written there, runs the task,
// and when it finishes the last task of a group it appends every task of the
// knot's next group to the queue.  Completion is published with a release at
// device scope and taken with an acquire before a task reads its inputs, so
// data written on one XCD is visible on another.  Every task is enqueued
// exactly once and only after its predecessors finished, so every claimed
// slot is eventually filled and the kernel drains for any grid size.
//
// Work done by tasks:
//   setup   edge weights x_e = e^{J_e} (or the Jones couplings -t^{-eps_e},
//           Sec. II), merged weights x_m = prod x_e over parallel edges, and
//           every vertex tensor F_v(s_v, s_w...) = prod_j T_{v wj}(s_v, s_wj)
//           with T = 1 + (x - 1) delta (Eqs. 3, 5); a vertex spin private to
//           its tensor is summed here.
//   step    C[b,m,n] = sum_k A[b,m,k] B[b,k,n] (one pairwise contraction of
//           Eq. 6).  Operands are gathered through per-step offset tables
//           (staged in LDS), so the permutation that brings A and B into GEMM
//           order is fused into the loads and never materialised.  Tensors
//           that live inside one serial task are kept in that workgroup's LDS.
//           Each tensor is a raw mantissa array R with an int64 exponent e
//           (true = R 2^e) and a shift s = frexp exponent of max(|Re|,|Im|)
//           over R; the consumer scales by 2^-(sA+sB) while accumulating, so
//           every product stays bounded by the contracted extent and Z never
//           overflows.
//   final   Z = prod over components of (scalar R 2^e) times the
//           simplification factors (loops x_e, spikes x_m + q - 1) and q per
//           isolated spin, renormalised after every product.
#include <hip/hip_runtime.h>
#include <type_traits>

#include <climits>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <map>
#include <mutex>
#include <algorithm>
#include <new>

#include "checks.h"
#include "decode.h"
#include "internal.h"

namespace kn {

template <class T>
struct alignas(2 * sizeof(T)) Cx {
  T re, im;
};

struct DevProg {
  const ImgHeader* h;
  const TaskDesc* tasks;
  const GroupDesc* groups;
  const KnotDesc* knots;
  const TensorDesc* tens;
  const StepDesc* steps;
  const VtxDesc* vtx;
  const int32_t* vslot;
  const MEdge* medges;
  const int32_t* members;
  const Factor* factors;
  const int32_t* strides;
  const int8_t* eps;
  const int32_t* comps;
  const int32_t* pins;
  int32_t* ctrl;
  int32_t* queue;
  int32_t* pending;
  TensorState* ts;
  Cx<double>* weights;  // x_e (n_edges) then x_m (n_medges)
  Cx<double>* mgrad;    // d log Z / d J per merged edge (gradient plans)
  kn_scalar* zslice;    // result of every slice (sliced plans)
  int32_t* uslice;      // the slice each knot descriptor is running
};

__device__ inline DevProg make_prog(const uint8_t* img, uint8_t* state) {
  DevProg p;
  p.h = reinterpret_cast<const ImgHeader*>(img);
  const ImgHeader& h = *p.h;
  p.tasks = reinterpret_cast<const TaskDesc*>(img + h.o_tasks);
  p.groups = reinterpret_cast<const GroupDesc*>(img + h.o_groups);
  p.knots = reinterpret_cast<const KnotDesc*>(img + h.o_knots);
  p.tens = reinterpret_cast<const TensorDesc*>(img + h.o_tensors);
  p.steps = reinterpret_cast<const StepDesc*>(img + h.o_steps);
  p.vtx = reinterpret_cast<const VtxDesc*>(img + h.o_vtx);
  p.vslot = reinterpret_cast<const int32_t*>(img + h.o_vslot);
  p.medges = reinterpret_cast<const MEdge*>(img + h.o_medges);
  p.members = reinterpret_cast<const int32_t*>(img + h.o_members);
  p.factors = reinterpret_cast<const Factor*>(img + h.o_factors);
  p.strides = reinterpret_cast<const int32_t*>(img + h.o_strides);
  p.eps = reinterpret_cast<const int8_t*>(img + h.o_eps);
  p.comps = reinterpret_cast<const int32_t*>(img + h.o_comps);
  p.pins = reinterpret_cast<const int32_t*>(img + h.o_pins);
  p.ctrl = reinterpret_cast<int32_t*>(state);
  p.queue = reinterpret_cast<int32_t*>(state + h.o_queue);
  p.pending = reinterpret_cast<int32_t*>(state + h.o_pending);
  p.ts = reinterpret_cast<TensorState*>(state + h.o_tstate);
  p.weights = reinterpret_cast<Cx<double>*>(state + h.o_weights);
  p.mgrad = reinterpret_cast<Cx<double>*>(state + h.o_mgrad);
  p.zslice = reinterpret_cast<kn_scalar*>(state + h.o_zslice);
  p.uslice = reinterpret_cast<int32_t*>(state + h.o_uslice);
  return p;
}

// The plan constants of a knot (derived merged edges, FAC_CONST factors).
__device__ inline const Cx<double>* plan_consts(const DevProg& p, const KnotDesc& kd) {
  return reinterpret_cast<const Cx<double>*>(reinterpret_cast<const uint8_t*>(p.h) +
                                              p.h->o_consts) +
         kd.const_off;
}

__device__ inline Cx<double> cmul(Cx<double> a, Cx<double> b) {
  return {fma(a.re, b.re, -a.im * b.im), fma(a.re, b.im, a.im * b.re)};
}

// z <- z * f with z = (mantissa, exponent) renormalised to max(|re|,|im|) in [0.5, 1)
__device__ inline void acc_mul(Cx<double>& z, int64_t& e, Cx<double> f) {
  z = cmul(z, f);
  double m = fmax(fabs(z.re), fabs(z.im));
  if (m == 0.0 || !isfinite(m)) return;
  int s;
  frexp(m, &s);
  z.re = ldexp(z.re, -s);
  z.im = ldexp(z.im, -s);
  e += s;
}

__device__ inline int32_t shift_of(int32_t s) { return s == kShiftNone ? 0 : s; }

// Tensor data: the workgroup's LDS arena or the global arena (generic pointer).
template <class T>
__device__ inline Cx<T>* tptr(const TensorDesc& d, Cx<T>* arena, Cx<T>* lds) {
  return d.lds_off >= 0 ? lds + d.lds_off : arena + d.off;
}

// Operand pointers with their address space fixed at compile time: LDS
// operands are read with LDS instructions and global ones with global
// instructions.  A generic (flat) load shares the vector-memory counter with
// stores, so a flat operand load would wait for every earlier output store.
template <class T>
using LdsCx = __attribute__((address_space(3))) Cx<T>;
template <class T>
using GlbCx = __attribute__((address_space(1))) Cx<T>;

// Loads of complex entries through address-space-qualified pointers
// (member-wise, merged into one wide access by the compiler).
template <class P>
__device__ inline auto ldc(P p) {
  using T = decltype(+p->re);
  return Cx<T>{p->re, p->im};
}

// Output entries.  Tensor entries in global memory are written through the
// L2 to memory (system-scope cache policy, sc0 sc1) instead of leaving dirty
// lines there: a task that finishes then has little left to write back when
// it releases its results at device scope (the release itself is
// unchanged), which makes the per-task release noticeably cheaper.  One
// entry is one store instruction (16 bytes in complex128, 8 in complex64),
// so the lanes of a wavefront that write consecutive entries write whole
// lines.  The stores are buffer stores with the cache policy as an operand,
// through a buffer resource whose base is the start of the output range a
// workgroup or wavefront writes (uniform over the wavefront); offsets are
// byte offsets from it, below kOutRangeBytes (the planner keeps every
// range a step writes from one base below that size), and a store past the
// range is dropped by the hardware bounds check rather than written.
constexpr int32_t kOutRangeBytes = 0x7fffffff;
constexpr int32_t kRawBufferWord3 = 0x00020000;  // raw buffer, 32-bit elements
constexpr int32_t kWriteThrough = 1 | 16;        // sc0 | sc1: system scope

template <class T>
struct GlbOut {
  __amdgpu_buffer_rsrc_t r;
  __device__ explicit GlbOut(GlbCx<T>* base)
      : r(__builtin_amdgcn_make_buffer_rsrc((void*)base, 0, kOutRangeBytes, kRawBufferWord3)) {}
};

__device__ inline void put(const GlbOut<double>& o, int32_t i, Cx<double> v) {
  typedef double D2 __attribute__((ext_vector_type(2)));
  typedef uint32_t U4 __attribute__((ext_vector_type(4)));
  const D2 x = {v.re, v.im};
  __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(U4, x), o.r, i * 16, 0, kWriteThrough);
}
__device__ inline void put(const GlbOut<float>& o, int32_t i, Cx<float> v) {
  typedef float F2 __attribute__((ext_vector_type(2)));
  typedef uint32_t U2 __attribute__((ext_vector_type(2)));
  const F2 x = {v.re, v.im};
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(U2, x), o.r, i * 8, 0, kWriteThrough);
}
template <class T>
__device__ inline void put(LdsCx<T>* p, int32_t i, Cx<T> v) {
  p[i].re = v.re;
  p[i].im = v.im;
}

// Tensor states: those produced by the running serial task are cached in LDS,
// the rest live in global memory.
struct States {
  TensorState* g;
  int32_t* sh;  // LDS
  int64_t* ex;  // LDS
  int32_t lo, len;
  __device__ inline bool local(int32_t t) const { return (uint32_t)(t - lo) < (uint32_t)len; }
  __device__ inline void get(int32_t t, int32_t& shift, int64_t& e) const {
    if (local(t)) {
      shift = sh[t - lo];
      e = ex[t - lo];
    } else {
      shift = g[t].shift;
      e = g[t].exp2;
    }
  }
  __device__ inline void set(int32_t t, int32_t shift, int64_t e) const {
    if (local(t)) {
      sh[t - lo] = shift;
      ex[t - lo] = e;
    } else {
      g[t].shift = shift;
      g[t].exp2 = e;
    }
  }
};

// ------------------------------------------------------------------ reductions

template <class T>
__device__ inline T wave_max(T v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

template <class T>
__device__ inline T block_max(T v, T* red) {
  v = wave_max(v);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) red[wv] = v;
  __syncthreads();
  T r = red[0];
#pragma unroll
  for (int i = 1; i < kBlock / 64; ++i) r = fmax(r, red[i]);
  return r;
}

// ------------------------------------------------------------------ setup

// Lane u's value of a double held per lane (uniform result).
__device__ inline double rl_double(double x, int u) {
  const uint64_t b = __builtin_bit_cast(uint64_t, x);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int32_t)(uint32_t)b, u);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int32_t)(uint32_t)(b >> 32), u);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

template <class T>
__device__ __attribute__((always_inline)) void knot_setup(const DevProg& p, const KnotDesc& kd, Cx<T>* arena, Cx<T>* lds,
                           const double* J, const States& st, int32_t slice) {
  const int tid = threadIdx.x;
  const ImgHeader& h = *p.h;
  Cx<double>* xe = p.weights + kd.w_off;
  Cx<double>* xm = xe + kd.n_edges;
  // x_e = e^{J_e}, or the Jones coupling -t^{-eps_e} (Sec. II)
  const Cx<double> t{kd.t_re, kd.t_im};
  const double tn = t.re * t.re + t.im * t.im;
  const Cx<double> tinv{t.re / tn, -t.im / tn};
  for (int e = tid; e < kd.n_edges; e += kBlock) {
    Cx<double> x;
    if (J) {
      double jr = J[2 * (kd.edge_off + e)], ji = J[2 * (kd.edge_off + e) + 1];
      double er = exp(jr);
      double sn, cs;
      sincos(ji, &sn, &cs);
      x = {er * cs, er * sn};
    } else {
      Cx<double> b = p.eps[kd.edge_off + e] > 0 ? tinv : t;
      x = {-b.re, -b.im};
    }
    xe[e] = x;
  }
  __syncthreads();
  for (int m = tid; m < kd.n_medges; m += kBlock) {
    const MEdge me = p.medges[kd.medge_off + m];
    Cx<double> x{1.0, 0.0};
    if (me.n_members < 0) x = plan_consts(p, kd)[me.member_off];  // derived edge
    for (int i = 0; i < me.n_members; ++i) x = cmul(x, xe[p.members[me.member_off + i]]);
    xm[m] = x;
  }
  __syncthreads();
  // vertex tensors, one wavefront per tensor.  A wavefront takes its
  // vertices 64 at a time: lane l first loads the records of vertex l of the
  // block and its slot list (all lanes at once), and each vertex's values
  // are then read from its lane, so a vertex waits only for its weights
  const int lane = tid & 63, wv = tid >> 6;
  const int q = kd.q;
  const QDiv D(q);
  constexpr int kSlots = 7;  // the planner rejects vertex tensors with more slots
  for (int v0 = wv * 64; v0 < kd.n_vtx; v0 += kBlock) {
    const int mine = v0 + lane;
    const bool have = mine < kd.n_vtx;
    VtxDesc my{};
    int64_t my_off = 0;
    int32_t my_size = 0, my_lds = -1;
    if (have) {
      my = p.vtx[kd.vtx_off + mine];
      const TensorDesc t = p.tens[my.tensor];
      my_off = t.off;
      my_size = t.size;
      my_lds = t.lds_off;
    }
    // the slot lists of the block, one merged-edge id per slot, and the
    // weights x_m of those slots: loaded once per block, so that the entry
    // loop of a vertex reads no global memory (a load there would also wait
    // for the entries stored before it)
    int32_t sl[kSlots];
#pragma unroll
    for (int j = 0; j < kSlots; ++j) sl[j] = have && j < my.n_slots ? p.vslot[my.slot_off + j] : 0;
    Cx<double> wl[kSlots];
#pragma unroll
    for (int j = 0; j < kSlots; ++j)
      wl[j] = have && j < my.n_slots ? xm[sl[j]] : Cx<double>{1.0, 0.0};
    const int nv = min(64, kd.n_vtx - v0);
    for (int u = 0; u < nv; ++u) {
      // uniform values of vertex v0 + u, read from its lane
      auto from = [u](int32_t v) { return __builtin_amdgcn_readlane(v, u); };
      const int32_t tensor = from(my.tensor);
      const int32_t n_slots = from(my.n_slots);
      const int32_t keep = from(my.keep_center);
      const int32_t pin_off = from(my.pin_off);
      const int32_t n_pins = from(my.n_pins);
      const int32_t size = from(my_size);
      const int32_t lds_off = from(my_lds);
      const int64_t off = (int64_t)(((uint64_t)(uint32_t)from((int32_t)(my_off >> 32)) << 32) |
                                    (uint32_t)from((int32_t)my_off));
      Cx<double> w[kSlots];
#pragma unroll
      for (int j = 0; j < kSlots; ++j) w[j] = {rl_double(wl[j].re, u), rl_double(wl[j].im, u)};
      const bool in_lds = lds_off >= 0;
      Cx<T>* out = in_lds ? lds + lds_off : arena + off;
      const GlbOut<T> gout((GlbCx<T>*)(in_lds ? arena : out));
      for (int i = lane; i < size; i += 64) {
        // digits of i: last neighbour slot fastest (exact division by q
        // through a multiply-high, once per entry); a kept centre is the
        // leading index (what is left of i after the slot digits), a private
        // centre is summed over.  A reverse-pass seed (keep_center < 0, no
        // slots, one entry) takes the kept branch with an empty product: the
        // scalar 1.
        int dig[kSlots];
        int rem = i;
#pragma unroll
        for (int j = kSlots - 1; j >= 0; --j) {
          dig[j] = -1;
          if (j < n_slots) {
            const int32_t qt = D.div(rem);
            dig[j] = rem - qt * q;
            rem = qt;
          }
        }
        const int a_lo = keep ? rem : 0;
        const int a_hi = keep ? a_lo + 1 : q;
        Cx<double> acc{0.0, 0.0};
        for (int a = a_lo; a < a_hi; ++a) {
          Cx<double> prod{1.0, 0.0};
#pragma unroll
          for (int j = kSlots - 1; j >= 0; --j)
            if (dig[j] == a) prod = cmul(prod, w[j]);
          // slices: an edge to a fixed spin contributes x_m where this spin
          // takes the fixed value (digit j of the slice number, base q)
          for (int j = 0; j < n_pins; ++j) {
            const int32_t* pn = p.pins + 2 * (pin_off + j);
            int sv = slice;
            for (int r = 0; r < pn[1]; ++r) sv /= q;
            if (sv % q == a) prod = cmul(prod, xm[pn[0]]);
          }
          acc.re += prod.re;
          acc.im += prod.im;
        }
        if (in_lds) out[i] = Cx<T>{(T)acc.re, (T)acc.im};
        else put(gout, i, Cx<T>{(T)acc.re, (T)acc.im});
      }
      // entries are products of <= 8 weights: no scaling needed
      if (lane == 0) st.set(tensor, 0, 0);
    }
  }
}

// ------------------------------------------------------------------ step

// Lanes per output: enough to give each of the nthr threads work, at most 64
// (one wavefront, reduced with shuffles) and at most the contracted extent.
__device__ inline int32_t lanes_per_output(int64_t outs, int32_t nk, int32_t nthr = kBlock) {
  int32_t L = 1;
  while (L < 64 && 2 * L <= nk && outs * L < nthr) L *= 2;
  return L;
}

// Operand offsets from generated tables (serial steps: tables in LDS).
struct TabIx {
  const int32_t *ab, *am, *ak, *bb, *bk, *bn;
  __device__ inline int32_t a_row(int32_t b, int32_t m) const { return ab[b] + am[m]; }
  __device__ inline int32_t b_col(int32_t b, int32_t n) const { return bb[b] + bn[n]; }
  __device__ inline int32_t a_k(int32_t k) const { return ak[k]; }
  __device__ inline int32_t b_k(int32_t k) const { return bk[k]; }
};

// Operand offsets for tiles: each spin group's offsets come from a table
// generated in LDS when it fitted, else they are decoded from the strides.
struct GenIx {
  const int32_t *tab[6];  // A_b A_m A_k B_b B_k B_n (nullptr: decode)
  const int32_t *str[6];
  int32_t rank[6];
  int32_t klo;            // first contracted index the A_k and B_k tables hold
  QDiv D;
  __device__ inline int32_t off(int g, int32_t i) const {
    return tab[g] ? tab[g][i] : group_off(i, str[g], rank[g], D);
  }
  __device__ inline int32_t off_k(int g, int32_t k) const {
    return tab[g] ? tab[g][k - klo] : group_off(k, str[g], rank[g], D);
  }
  __device__ inline int32_t a_row(int32_t b, int32_t m) const { return off(0, b) + off(1, m); }
  __device__ inline int32_t b_col(int32_t b, int32_t n) const { return off(3, b) + off(5, n); }
  __device__ inline int32_t a_k(int32_t k) const { return off_k(2, k); }
  __device__ inline int32_t b_k(int32_t k) const { return off_k(4, k); }
};

// This lane's part of sum_k A[row, k] B[k, col] over k = k_first, k_first + L,
// ... < nk: four entries per round, the loads of a round issued before its
// products (entries past nk read as zero) so that a short contracted range
// does not serialise on memory latency.
template <class T, class Ix, class PA, class PB>
__device__ inline void lane_dot(PA ra, PB rb, const Ix& ix, int32_t k, int32_t nk, int32_t L,
                                T& cr, T& ci) {
  T cr0 = 0, ci0 = 0, cr1 = 0, ci1 = 0;
  const Cx<T> zero{0, 0};
  for (; k < nk; k += 4 * L) {
    const bool v1 = k + L < nk, v2 = k + 2 * L < nk, v3 = k + 3 * L < nk;
    const Cx<T> x0 = ldc(ra + ix.a_k(k));
    const Cx<T> y0 = ldc(rb + ix.b_k(k));
    Cx<T> x1 = zero, y1 = zero, x2 = zero, y2 = zero, x3 = zero, y3 = zero;
    if (v1) {
      x1 = ldc(ra + ix.a_k(k + L));
      y1 = ldc(rb + ix.b_k(k + L));
    }
    if (v2) {
      x2 = ldc(ra + ix.a_k(k + 2 * L));
      y2 = ldc(rb + ix.b_k(k + 2 * L));
    }
    if (v3) {
      x3 = ldc(ra + ix.a_k(k + 3 * L));
      y3 = ldc(rb + ix.b_k(k + 3 * L));
    }
    cr0 = fma(x0.re, y0.re, cr0); cr0 = fma(-x0.im, y0.im, cr0);
    ci0 = fma(x0.re, y0.im, ci0); ci0 = fma(x0.im, y0.re, ci0);
    cr1 = fma(x1.re, y1.re, cr1); cr1 = fma(-x1.im, y1.im, cr1);
    ci1 = fma(x1.re, y1.im, ci1); ci1 = fma(x1.im, y1.re, ci1);
    cr0 = fma(x2.re, y2.re, cr0); cr0 = fma(-x2.im, y2.im, cr0);
    ci0 = fma(x2.re, y2.im, ci0); ci0 = fma(x2.im, y2.re, ci0);
    cr1 = fma(x3.re, y3.re, cr1); cr1 = fma(-x3.im, y3.im, cr1);
    ci1 = fma(x3.re, y3.im, ci1); ci1 = fma(x3.im, y3.re, ci1);
  }
  cr = cr0 + cr1;
  ci = ci0 + ci1;
}

// lane_dot for two outputs at once (rows ra, ra2 and columns rb, rb2): a
// round issues the 16 loads of four contracted entries of both before any
// product, so a thread has twice the loads in flight of two lane_dot calls.
// Each output is summed in the same order as by lane_dot.
template <class T, class Ix, class PA, class PB>
__device__ inline void lane_dot2(PA ra, PB rb, PA ra2, PB rb2, const Ix& ix, int32_t k,
                                 int32_t nk, int32_t L, T& cr, T& ci, T& cr2, T& ci2) {
  T p0 = 0, q0 = 0, p1 = 0, q1 = 0, u0 = 0, w0 = 0, u1 = 0, w1 = 0;
  const Cx<T> zero{0, 0};
  for (; k < nk; k += 4 * L) {
    int32_t oa[4], ob[4];
    bool v[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      v[j] = j == 0 || k + j * L < nk;
      oa[j] = v[j] ? ix.a_k(k + j * L) : 0;
      ob[j] = v[j] ? ix.b_k(k + j * L) : 0;
    }
    Cx<T> x[4], y[4], x2[4], y2[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      x[j] = zero; y[j] = zero; x2[j] = zero; y2[j] = zero;
      if (v[j]) {
        x[j] = ldc(ra + oa[j]);
        y[j] = ldc(rb + ob[j]);
        x2[j] = ldc(ra2 + oa[j]);
        y2[j] = ldc(rb2 + ob[j]);
      }
    }
#pragma unroll
    for (int j = 0; j < 4; j += 2) {
      p0 = fma(x[j].re, y[j].re, p0); p0 = fma(-x[j].im, y[j].im, p0);
      q0 = fma(x[j].re, y[j].im, q0); q0 = fma(x[j].im, y[j].re, q0);
      p1 = fma(x[j + 1].re, y[j + 1].re, p1); p1 = fma(-x[j + 1].im, y[j + 1].im, p1);
      q1 = fma(x[j + 1].re, y[j + 1].im, q1); q1 = fma(x[j + 1].im, y[j + 1].re, q1);
      u0 = fma(x2[j].re, y2[j].re, u0); u0 = fma(-x2[j].im, y2[j].im, u0);
      w0 = fma(x2[j].re, y2[j].im, w0); w0 = fma(x2[j].im, y2[j].re, w0);
      u1 = fma(x2[j + 1].re, y2[j + 1].re, u1); u1 = fma(-x2[j + 1].im, y2[j + 1].im, u1);
      w1 = fma(x2[j + 1].re, y2[j + 1].im, w1); w1 = fma(x2[j + 1].im, y2[j + 1].re, w1);
    }
  }
  cr = p0 + p1;
  ci = q0 + q1;
  cr2 = u0 + u1;
  ci2 = w0 + w1;
}

// Outputs [o_begin, o_end) of C = A . B, each summed over k in [k0, nk) by L
// lanes of one wavefront; threads tid = 0..nthr-1 (a whole workgroup or one
// wavefront) share the outputs.  pc addresses the range itself: output o is
// entry o - o_begin of pc.  A thread computes two outputs together (their
// loads interleaved) before it stores either, so its stores overlap the next
// pair's loads.  Returns this thread's max |.|.
template <class T, class Ix, class PA, class PB, class PC>
__device__ __attribute__((always_inline)) T step_outputs(PA pa, PB pb, PC pc, const Ix& ix, int32_t nm, int32_t nn, int32_t k0,
                          int32_t nk, int64_t o_begin, int64_t o_end, T scale, int32_t L,
                          int32_t tid, int32_t nthr) {
  const int32_t mn = nm * nn;
  const int32_t ob = (int32_t)o_begin;
  const int32_t lsub = tid & (L - 1);
  const int32_t slot = tid / L;
  const int32_t nslot = nthr / L;
  T lmax = 0;
  for (int64_t o = o_begin + slot; o < o_end; o += 2 * nslot) {
    const int32_t oi = (int32_t)o;
    const int32_t oi2 = oi + nslot;
    const bool two = oi2 < o_end;  // the same for the L lanes of an output
    T cr, ci, cr2 = 0, ci2 = 0;
    const int32_t b = oi / mn;
    const int32_t r = oi - b * mn;
    const int32_t m = r / nn;
    const int32_t n = r - m * nn;
    if (two) {
      const int32_t b2 = oi2 / mn;
      const int32_t r2 = oi2 - b2 * mn;
      const int32_t m2 = r2 / nn;
      const int32_t n2 = r2 - m2 * nn;
      lane_dot2<T>(pa + ix.a_row(b, m), pb + ix.b_col(b, n), pa + ix.a_row(b2, m2),
                   pb + ix.b_col(b2, n2), ix, k0 + lsub, nk, L, cr, ci, cr2, ci2);
    } else {
      lane_dot<T>(pa + ix.a_row(b, m), pb + ix.b_col(b, n), ix, k0 + lsub, nk, L, cr, ci);
    }
    for (int32_t off = L >> 1; off >= 1; off >>= 1) {
      cr += __shfl_xor(cr, off, 64);
      ci += __shfl_xor(ci, off, 64);
      cr2 += __shfl_xor(cr2, off, 64);
      ci2 += __shfl_xor(ci2, off, 64);
    }
    if (lsub == 0) {
      cr *= scale;
      ci *= scale;
      put(pc, oi - ob, Cx<T>{cr, ci});
      lmax = fmax(lmax, fmax(fabs(cr), fabs(ci)));
      if (two) {
        cr2 *= scale;
        ci2 *= scale;
        put(pc, oi2 - ob, Cx<T>{cr2, ci2});
        lmax = fmax(lmax, fmax(fabs(cr2), fabs(ci2)));
      }
    }
  }
  return lmax;
}

// step_outputs with each operand's home (>= 0 global arena offset, < 0 LDS
// arena offset -1 - home) resolved to a pointer of its address space.
template <class T, class Ix>
__device__ __attribute__((always_inline)) T step_outputs_homes(int32_t ha, int32_t hb, int32_t hc, Cx<T>* arena, Cx<T>* lds,
                                const Ix& ix, int32_t nm, int32_t nn, int32_t k0, int32_t nk,
                                int64_t o_begin, int64_t o_end, T scale, int32_t L, int32_t tid,
                                int32_t nthr) {
  auto gl = [&](int32_t h) { return (GlbCx<T>*)(arena + h); };
  auto ld = [&](int32_t h) { return (LdsCx<T>*)(lds + (-1 - h)); };
  // the output range [o_begin, o_end) of C
  auto glo = [&](int32_t h) { return GlbOut<T>((GlbCx<T>*)(arena + h) + o_begin); };
  auto ldo = [&](int32_t h) { return (LdsCx<T>*)(lds + (-1 - h)) + o_begin; };
#define KN_RUN(A, B, C) \
  return step_outputs<T>(A(ha), B(hb), C(hc), ix, nm, nn, k0, nk, o_begin, o_end, scale, L, tid, nthr)
  if (ha < 0) {
    if (hb < 0) {
      if (hc < 0) KN_RUN(ld, ld, ldo);
      KN_RUN(ld, ld, glo);
    }
    if (hc < 0) KN_RUN(ld, gl, ldo);
    KN_RUN(ld, gl, glo);
  }
  if (hb < 0) {
    if (hc < 0) KN_RUN(gl, ld, ldo);
    KN_RUN(gl, ld, glo);
  }
  if (hc < 0) KN_RUN(gl, gl, ldo);
  KN_RUN(gl, gl, glo);
#undef KN_RUN
}

template <class T>
__device__ inline int32_t frexp_shift(T m) {
  if (!(m > 0)) return kShiftNone;
  int s;
  frexp((double)m, &s);
  return s;
}

// Scale 2^-(sA+sB) applied to the products, and the exponent of C.
template <class T>
__device__ inline T step_scale(const States& st, int32_t a, int32_t b, int64_t& e_out) {
  int32_t sa, sb;
  int64_t ea, eb;
  st.get(a, sa, ea);
  st.get(b, sb, eb);
  const int32_t sh = shift_of(sa) + shift_of(sb);
  e_out = ea + eb + sh;
  return (T)ldexp(1.0, -sh);
}

__device__ inline int32_t step_tab_entries(const StepDesc& d) {
  return 2 * d.nb + d.nm + 2 * d.nk + d.nn;
}

template <class T>
__device__ inline Cx<T>* home_ptr(int32_t home, Cx<T>* arena, Cx<T>* lds) {
  return home >= 0 ? arena + home : lds + (-1 - home);
}

// One serial step C = A . B on threads tid = 0..nthr-1, with the gather
// tables `tab` (A_b A_m A_k B_b B_k B_n, generated in LDS) and the states of
// operands made before the task in ext[0..1].  Returns this thread's max |.|
// and C's exponent.
//
// A step the whole workgroup computes (nthr = kBlock) first copies operands
// that live in the global arena into the staging area (entries stage_off ..
// stage_off + stage_elems - 1 of the LDS arena pointer), A first, each when it
// fits: one burst of independent coalesced loads, after which the step's
// gathers read LDS.  The products and their order are unchanged.
template <class T>
__device__ inline T serial_step(const StepDesc& d, const int32_t* tab, Cx<T>* arena, Cx<T>* lds,
                                const States& st, const TensorState* ext, int32_t tid,
                                int32_t nthr, int32_t stage_off, int32_t stage_elems,
                                int64_t& ec) {
  TabIx ix;
  ix.ab = tab;
  ix.am = ix.ab + d.nb;
  ix.ak = ix.am + d.nm;
  ix.bb = ix.ak + d.nk;
  ix.bk = ix.bb + d.nb;
  ix.bn = ix.bk + d.nk;
  int32_t sa, sb;
  int64_t ea, eb;
  if (st.local(d.a)) st.get(d.a, sa, ea);
  else { sa = ext[0].shift; ea = ext[0].exp2; }
  if (st.local(d.b)) st.get(d.b, sb, eb);
  else { sb = ext[1].shift; eb = ext[1].exp2; }
  const int32_t sh = shift_of(sa) + shift_of(sb);
  ec = ea + eb + sh;
  const T scale = (T)ldexp(1.0, -sh);
  const int64_t outs = (int64_t)d.nb * d.nm * d.nn;
  const int32_t L = lanes_per_output(outs, d.nk, nthr);
  int32_t ha = d.home_a, hb = d.home_b;
  if (nthr == kBlock && (ha >= 0 || hb >= 0)) {
    // sizes of A (spins b, m, k) and B (spins b, k, n)
    const int64_t na = (int64_t)d.nb * d.nm * d.nk, nbb = (int64_t)d.nb * d.nk * d.nn;
    const bool sa = ha >= 0 && na <= stage_elems;
    const int64_t used = sa ? na : 0;
    const bool sb = hb >= 0 && used + nbb <= stage_elems;
    if (sa || sb) {
      LdsCx<T>* stg = (LdsCx<T>*)(lds + stage_off);
      if (sa) {
        const GlbCx<T>* g = (const GlbCx<T>*)(arena + ha);
        for (int32_t i = tid; i < (int32_t)na; i += kBlock) put(stg, i, ldc(g + i));
        ha = -1 - stage_off;
      }
      if (sb) {
        const GlbCx<T>* g = (const GlbCx<T>*)(arena + hb);
        for (int32_t i = tid; i < (int32_t)nbb; i += kBlock) put(stg + used, i, ldc(g + i));
        hb = -1 - (stage_off + (int32_t)used);
      }
      __syncthreads();
    }
  }
  return step_outputs_homes<T>(ha, hb, d.home_c, arena, lds, ix, d.nm, d.nn, 0, d.nk, 0, outs,
                               scale, L, tid, nthr);
}

// Serial steps [first, first + count): descriptors are staged in LDS one
// chunk at a time and the chunk's gather tables are generated there from the
// strides; the chunk then runs with no global round trip except operands that
// live in the global arena.
// Serial steps of a level with fewer products than this run on one wavefront.
constexpr int64_t kWaveMacs = 2048;

template <class T>
__device__ __attribute__((always_inline)) void serial_steps(const DevProg& p, int32_t first, int32_t count, int32_t q,
                             Cx<T>* arena, Cx<T>* lds, int32_t* s_tab, StepDesc* s_desc,
                             int32_t* s_tb, TensorState* s_ext, const States& st, T* s_red,
                             int64_t* ph) {
  int64_t tk = ph ? wall_clock64() : 0;
  auto lap = [&](int i) {
    if (ph) {
      const int64_t t = wall_clock64();
      ph[i] += t - tk;
      tk = t;
    }
  };
  constexpr int32_t kDescWords = (int32_t)(sizeof(StepDesc) / 4);
  const QDiv D(q);
  // the staging area follows the tensor arena
  const int32_t stage_off = p.h->lds_bytes / (int32_t)sizeof(Cx<T>);
  const int32_t stage_elems = stage_bytes(p.h->lds_bytes) / (int32_t)sizeof(Cx<T>);
  int32_t s = first;
  const int32_t end = first + count;
  while (s < end) {
    const int32_t nd = min(end - s, kDescBuf);
    {
      const int32_t* src = reinterpret_cast<const int32_t*>(p.steps + s);
      int32_t* dst = reinterpret_cast<int32_t*>(s_desc);
      for (int32_t i = threadIdx.x; i < nd * kDescWords; i += kBlock) dst[i] = src[i];
    }
    __syncthreads();
    // steps of this chunk: as many as fit the table buffer (at least one)
    int32_t ce = 0, tab_end = 0;
    for (int32_t j = 0; j < nd; ++j) {
      const int32_t e = tab_end + step_tab_entries(s_desc[j]);
      if (e > kTabBuf) break;
      if (threadIdx.x == 0) s_tb[j] = tab_end;
      ce = j + 1;
      tab_end = e;
    }
    if (threadIdx.x == 0) s_tb[ce] = tab_end;
    // states of operands made before this task (already final) are fetched now
    if (threadIdx.x < 2 * ce) {
      const int32_t j = threadIdx.x >> 1;
      const int32_t t = (threadIdx.x & 1) ? s_desc[j].b : s_desc[j].a;
      if (!st.local(t)) s_ext[threadIdx.x] = p.ts[t];
    }
    __syncthreads();
    // generate the gather tables: entry i belongs to step j (binary search)
    for (int32_t i = threadIdx.x; i < tab_end; i += kBlock) {
      int32_t lo = 0, hi = ce - 1;
      while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (s_tb[mid] <= i) lo = mid;
        else hi = mid - 1;
      }
      const StepDesc& d = s_desc[lo];
      int32_t r = i - s_tb[lo];
      const int32_t rb = d.ranks & 255, rm = (d.ranks >> 8) & 255, rk = (d.ranks >> 16) & 255,
                    rn = (d.ranks >> 24) & 255;
      const int32_t* sp = p.strides + d.str;
      int32_t off;
      if (r < d.nb) {
        off = group_off(r, sp, rb, D);
      } else if ((r -= d.nb) < d.nm) {
        off = group_off(r, sp + rb, rm, D);
      } else if ((r -= d.nm) < d.nk) {
        off = group_off(r, sp + rb + rm, rk, D);
      } else if ((r -= d.nk) < d.nb) {
        off = group_off(r, sp + rb + rm + rk, rb, D);
      } else if ((r -= d.nb) < d.nk) {
        off = group_off(r, sp + 2 * rb + rm + rk, rk, D);
      } else {
        r -= d.nk;
        off = group_off(r, sp + 2 * rb + rm + 2 * rk, rn, D);
      }
      s_tab[i] = off;
    }
    __syncthreads();
    lap(1);
    // levels: a run of adjacent steps of equal level is independent; a lone
    // step uses the whole workgroup, otherwise each wavefront takes steps of
    // the level in turn, and one barrier ends the level
    for (int32_t j = 0; j < ce;) {
      int32_t je = j + 1;
      while (je < ce && s_desc[je].lvl == s_desc[j].lvl) ++je;
      // steps with many products use the whole workgroup, one after another;
      // the rest are shared out to the wavefronts
      for (int32_t u = j; u < je; ++u) {
        const StepDesc& d = s_desc[u];
        if (je - j > 1 && (int64_t)d.nb * d.nm * d.nn * d.nk < kWaveMacs) continue;
        int64_t ec;
        T lm = serial_step<T>(d, s_tab + s_tb[u], arena, lds, st, s_ext + 2 * u,
                              (int32_t)threadIdx.x, kBlock, stage_off, stage_elems, ec);
        lm = block_max<T>(lm, s_red);
        if (threadIdx.x == 0) st.set(d.c, frexp_shift<T>(lm), ec);
      }
      if (je - j > 1) {
        // the wavefront index is uniform within a wavefront: readfirstlane
        // lets the step's descriptor live in scalar registers
        const int32_t wv = __builtin_amdgcn_readfirstlane((int32_t)(threadIdx.x >> 6));
        const int32_t lane = threadIdx.x & 63;
        int32_t r = 0;  // rank among the level's small steps
        for (int32_t u = j; u < je; ++u) {
          const StepDesc& d = s_desc[u];
          if ((int64_t)d.nb * d.nm * d.nn * d.nk >= kWaveMacs) continue;
          if ((r++ & (kBlock / 64 - 1)) != wv) continue;
          int64_t ec;
          T lm = serial_step<T>(d, s_tab + s_tb[u], arena, lds, st, s_ext + 2 * u, lane, 64, 0, 0,
                                ec);
          lm = wave_max(lm);
          if (lane == 0) st.set(d.c, frexp_shift<T>(lm), ec);
        }
      }
      lap(2);
      __syncthreads();
      lap(3);
      j = je;
    }
    s += ce;
  }
}

// Output shift of a tiled step: every tile of an unsplit step folds its max
// into C's shift, and tile 0 writes C's exponent.
template <class T>
__device__ inline void tile_publish(const DevProg& p, int32_t c, int32_t tile_id, T lm, int64_t ec,
                                    T* s_red) {
  lm = block_max<T>(lm, s_red);
  if (threadIdx.x == 0) {
    const int32_t sh = frexp_shift<T>(lm);
    if (sh != kShiftNone)
      __hip_atomic_fetch_max(&p.ts[c].shift, sh, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (tile_id == 0) p.ts[c].exp2 = ec;
  }
}

// Offset tables of the six spin groups of step s (A_b A_m A_k B_b B_k B_n).
__device__ inline GenIx step_ix(const DevProg& p, const StepDesc& s, int32_t q) {
  const int32_t rb = s.ranks & 255, rm = (s.ranks >> 8) & 255, rk = (s.ranks >> 16) & 255,
                rn = (s.ranks >> 24) & 255;
  const int32_t* sp = p.strides + s.str;
  return GenIx{{nullptr, nullptr, nullptr, nullptr, nullptr, nullptr},
               {sp, sp + rb, sp + rb + rm, sp + rb + rm + rk, sp + 2 * rb + rm + rk,
                sp + 2 * rb + rm + 2 * rk},
               {rb, rm, rk, rb, rk, rn},
               0,
               QDiv(q)};
}

// STEP_TILES: `tile` consecutive outputs of C (row-major over b, m, n), over
// contracted range ks of the split.  Tile tasks use none of the serial-task
// LDS areas, so the whole dynamic LDS (tab_cap entries) holds generated offset
// tables: contracted group first (only this task's segment of it when the
// contracted index is split), then columns, rows, batch; the last 16 entries
// are kept for the partial sums of a one-output tile.
//
// A tile of one output over a long segment (the scalar product that ends a
// knot's contraction, split over many tasks) is summed by all four
// wavefronts, a quarter of the segment each; wavefront 0's thread 0 adds the
// four partial sums in wavefront order.
//
// ph (traced launches, thread 0; else null; ph[3] holds the task's start):
// from the start to the end of the tables and operand states, then the
// products, then the publish.
template <class T>
__device__ __attribute__((always_inline)) void tile_step(const DevProg& p, const StepDesc& s, int32_t tile_id, int32_t q,
                          Cx<T>* arena, int32_t* s_tab, int32_t tab_cap, const States& st,
                          T* s_red, int64_t* ph) {
  GenIx ix = step_ix(p, s, q);
  const int64_t outs = (int64_t)s.nb * s.nm * s.nn;
  const int32_t base = s.n_tiles / s.n_ks;
  const int32_t ks = tile_id / base, t = tile_id - ks * base;
  const int32_t k0 = ks * s.kseg, k1 = min(s.nk, k0 + s.kseg);
  const int64_t o0 = (int64_t)t * s.tile;
  const int64_t o1 = o0 + s.tile < outs ? o0 + s.tile : outs;
  constexpr int32_t kPartials = 16;  // 4 complex partial sums (64 bytes)
  const int32_t n_of[6] = {s.nb, s.nm, k1 - k0, s.nb, k1 - k0, s.nn};
  ix.klo = k0;
  int32_t used = 0;
  for (int g : {2, 4, 5, 1, 0, 3}) {
    if (used + n_of[g] > tab_cap - 2 * kPartials) continue;
    const int32_t lo = g == 2 || g == 4 ? k0 : 0;
    int32_t* tb = s_tab + used;
    for (int32_t i = threadIdx.x; i < n_of[g]; i += kBlock)
      tb[i] = group_off(lo + i, ix.str[g], ix.rank[g], ix.D);
    ix.tab[g] = tb;
    used += n_of[g];
  }
  int64_t ec;
  const T scale = step_scale<T>(st, s.a, s.b, ec);
  __syncthreads();
  int64_t tk = 0;
  if (ph) {
    tk = wall_clock64();
    ph[0] = tk - ph[3];
  }
  Cx<T>* pc = s.n_ks > 1 ? arena + s.partial + (int64_t)ks * outs : arena + s.home_c;
  const GlbCx<T>* pa = (const GlbCx<T>*)(arena + s.home_a);
  const GlbCx<T>* pb = (const GlbCx<T>*)(arena + s.home_b);
  T lm = 0;
  if (o1 - o0 == 1 && k1 - k0 >= 2 * kBlock) {
    LdsCx<T>* part = (LdsCx<T>*)(s_tab + ((used + 3) & ~3));  // 16-byte aligned
    const int32_t w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int32_t quarter = (k1 - k0 + 3) / 4;
    const int32_t kw0 = min(k1, k0 + w * quarter), kw1 = min(k1, kw0 + quarter);
    const int32_t mn = s.nm * s.nn, o = (int32_t)o0;
    const int32_t b = o / mn, m = (o - b * mn) / s.nn, n = o - b * mn - m * s.nn;
    T cr, ci;
    lane_dot<T>(pa + ix.a_row(b, m), pb + ix.b_col(b, n), ix, kw0 + lane, kw1, 64, cr, ci);
    for (int32_t off = 32; off >= 1; off >>= 1) {
      cr += __shfl_xor(cr, off, 64);
      ci += __shfl_xor(ci, off, 64);
    }
    if (lane == 0) put(part, w, Cx<T>{cr, ci});
    __syncthreads();
    if (threadIdx.x == 0) {
      T re = 0, im = 0;
      for (int i = 0; i < 4; ++i) {
        re += part[i].re;
        im += part[i].im;
      }
      re *= scale;
      im *= scale;
      put(GlbOut<T>((GlbCx<T>*)pc + o0), 0, Cx<T>{re, im});
      lm = fmax(fabs(re), fabs(im));
    }
  } else {
    const int32_t L = lanes_per_output(o1 - o0, k1 - k0);
    lm = step_outputs<T>(pa, pb, GlbOut<T>((GlbCx<T>*)pc + o0), ix, s.nm, s.nn, k0, k1, o0, o1,
                         scale, L, (int32_t)threadIdx.x, kBlock);
  }
  if (ph) {
    const int64_t t = wall_clock64();
    ph[1] = t - tk;
    tk = t;
  }
  if (s.n_ks == 1) tile_publish<T>(p, s.c, tile_id, lm, ec, s_red);
  if (ph) ph[2] = wall_clock64() - tk;
}

// Matrix-core products for the GEMM blocks: D = A B + C on one 16 x 16
// tile per wavefront, K = 4 (v_mfma_f64_16x16x4f64 / v_mfma_f32_16x16x4f32).
// Operands: lane l holds A[l % 16][l / 16] and B[l / 16][l % 16]; the four
// accumulator registers of lane l hold column l % 16 of D, at rows row(l, r)
// (measured lane layouts of the two instructions on gfx950).
template <class T>
struct Mfma;
template <>
struct Mfma<double> {
  typedef double V __attribute__((ext_vector_type(4)));
  static __device__ inline V mac(double a, double b, V c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ inline int32_t row(int32_t l, int32_t r) { return (l >> 4) + 4 * r; }
};
template <>
struct Mfma<float> {
  typedef float V __attribute__((ext_vector_type(4)));
  static __device__ inline V mac(float a, float b, V c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ inline int32_t row(int32_t l, int32_t r) { return 4 * (l >> 4) + r; }
};

// STEP_GEMM / STEP_GEMM64: BM x BM output blocks of C[b] (BM = 16 TM: 32
// or 64) over contracted range ks of the split, `tile` consecutive blocks per
// task.  Chunks of 16 contracted entries of A (BM rows) and B (BM columns)
// are gathered into LDS (row pitch BM + 1 entries), the next chunk's operands
// loaded into registers while the current one is multiplied.  The products
// run on the matrix cores: the four wavefronts split the block into 2 x 2
// quarters of WT x WT tiles of 16 x 16 (WT = TM / 2), and a complex tile
// takes four real MFMAs per 4 contracted entries,
//   Re += Re A Re B, Re += (-Im A) Im B, Im += Re A Im B, Im += Im A Re B.
// The contributions go to independent accumulators (with one tile per
// wavefront the real and imaginary parts are split once more) so that
// consecutive MFMAs do not wait on each other.  The contracted offsets come
// from a table generated in LDS when the range fits, else they are decoded
// from the strides.
template <class T, int TM>
__device__ __attribute__((always_inline)) void gemm_tile(const DevProg& p, const StepDesc& s, int32_t tile_id, int32_t q,
                          Cx<T>* __restrict__ arena, uint8_t* smem, int32_t smem_bytes,
                          const States& st, T* s_red, int64_t* ph) {
  constexpr int32_t BM = 16 * TM, BK = kGemmChunk, P = BM + 1;
  constexpr int32_t WT = TM / 2;             // 16 x 16 tiles per wavefront side
  constexpr int32_t NS = WT == 1 ? 2 : 1;    // accumulator chains per part
  static_assert(BK == 16 && kBlock == 256, "thread layout: 16 x 16 threads, 16 entries per chunk");
  using M = Mfma<T>;
  using V = typename M::V;
  const QDiv D(q);
  const int32_t rb = s.ranks & 255, rm = (s.ranks >> 8) & 255, rk = (s.ranks >> 16) & 255,
                rn = (s.ranks >> 24) & 255;
  const int32_t* sab = p.strides + s.str;
  const int32_t* sam = sab + rb;
  const int32_t* sak = sam + rm;
  const int32_t* sbb = sak + rk;
  const int32_t* sbk = sbb + rb;
  const int32_t* sbn = sbk + rk;
  const int32_t tid = threadIdx.x;
  // this task: contracted range ks of the split, blocks [blk0, blk1) of the
  // nb * n_mb * n_nb blocks (s.tile blocks per task)
  const int32_t mb_nb = s.n_mb * s.n_nb;
  const int32_t nblk = s.nb * mb_nb;
  const int32_t per = s.tile;
  const int32_t base = (nblk + per - 1) / per;
  const int32_t ks = tile_id / base;
  const int32_t blk0 = (tile_id - ks * base) * per, blk1 = min(nblk, blk0 + per);
  const int32_t k0 = ks * s.kseg, k1 = min(s.nk, k0 + s.kseg), kl = k1 - k0;

  Cx<T>* As = reinterpret_cast<Cx<T>*>(smem);
  Cx<T>* Bs = As + BK * P;
  int32_t* ktab = reinterpret_cast<int32_t*>(Bs + BK * P);
  const int32_t kcap = (smem_bytes - 2 * BK * P * (int32_t)sizeof(Cx<T>)) / 8;
  const bool use_tab = kl <= kcap;
  if (use_tab) {
    for (int32_t i = tid; i < kl; i += kBlock) {
      ktab[2 * i] = group_off(k0 + i, sak, rk, D);
      ktab[2 * i + 1] = group_off(k0 + i, sbk, rk, D);
    }
  }
  int64_t ec;
  const T scale = step_scale<T>(st, s.a, s.b, ec);
  // this thread's loads: contracted entry kk of rows / columns lr + 16 i
  const int32_t kk = tid & (BK - 1), lr = tid >> 4;
  // this wavefront's quarter of the block and its lane
  const int32_t lane = tid & 63, wv = tid >> 6;
  const int32_t qr = (wv >> 1) * 16 * WT, qc = (wv & 1) * 16 * WT;
  const int32_t l16 = lane & 15, lk = lane >> 4;
  const GlbCx<T>* A = (const GlbCx<T>*)(arena + s.home_a);
  const GlbCx<T>* B = (const GlbCx<T>*)(arena + s.home_b);
  const int64_t outs = (int64_t)s.nb * s.nm * s.nn;
  GlbCx<T>* C = (GlbCx<T>*)(s.n_ks > 1 ? arena + s.partial + (int64_t)ks * outs : arena + s.home_c);
  T lm = 0;
  __syncthreads();
  int64_t tk = 0;
  if (ph) {
    tk = wall_clock64();
    ph[0] = tk - ph[3];
  }

  struct Ops {
    Cx<T> a[TM], b[TM];
  };
  for (int32_t blk = blk0; blk < blk1; ++blk) {
    const int32_t b = blk / mb_nb;
    const int32_t r = blk - b * mb_nb;
    const int32_t mblk = r / s.n_nb, nbk = r - mblk * s.n_nb;
    const int32_t m0 = mblk * BM, n0 = nbk * BM;
    const int32_t oab = group_off(b, sab, rb, D), obb = group_off(b, sbb, rb, D);
    bool am[TM], bn[TM];
    int32_t ra[TM], cb[TM];
#pragma unroll
    for (int i = 0; i < TM; ++i) {
      am[i] = m0 + lr + 16 * i < s.nm;
      bn[i] = n0 + lr + 16 * i < s.nn;
      ra[i] = am[i] ? oab + group_off(m0 + lr + 16 * i, sam, rm, D) : 0;
      cb[i] = bn[i] ? obb + group_off(n0 + lr + 16 * i, sbn, rn, D) : 0;
    }
    auto load = [&](int32_t c0) -> Ops {
      const int32_t k = c0 + kk;
      Ops x;
#pragma unroll
      for (int i = 0; i < TM; ++i) {
        x.a[i] = Cx<T>{0, 0};
        x.b[i] = Cx<T>{0, 0};
      }
      if (k < kl) {
        int32_t oa, ob;
        if (use_tab) {
          oa = ktab[2 * k];
          ob = ktab[2 * k + 1];
        } else {
          oa = group_off(k0 + k, sak, rk, D);
          ob = group_off(k0 + k, sbk, rk, D);
        }
#pragma unroll
        for (int i = 0; i < TM; ++i) {
          if (am[i]) x.a[i] = ldc(A + ra[i] + oa);
          if (bn[i]) x.b[i] = ldc(B + cb[i] + ob);
        }
      }
      return x;
    };
    // accumulators: [row tile][column tile][chain], real and imaginary parts
    V cre[WT][WT][NS], cim[WT][WT][NS];
#pragma unroll
    for (int i = 0; i < WT; ++i)
#pragma unroll
      for (int j = 0; j < WT; ++j)
#pragma unroll
        for (int c = 0; c < NS; ++c) {
          cre[i][j][c] = V{0, 0, 0, 0};
          cim[i][j][c] = V{0, 0, 0, 0};
        }
    Ops x = load(0);
    for (int32_t c0 = 0; c0 < kl; c0 += BK) {
#pragma unroll
      for (int i = 0; i < TM; ++i) {
        As[kk * P + lr + 16 * i] = x.a[i];
        Bs[kk * P + lr + 16 * i] = x.b[i];
      }
      __syncthreads();
      if (c0 + BK < kl) x = load(c0 + BK);
      // only the groups of 4 contracted entries this chunk holds (a short
      // contracted index, K = 3 or 9, would otherwise multiply zero padding)
      const int32_t kv = min(BK, kl - c0);
#pragma unroll
      for (int32_t j4 = 0; j4 < kv; j4 += 4) {
        const int32_t kr = (j4 + lk) * P;
        Cx<T> a[WT], bb[WT];
#pragma unroll
        for (int i = 0; i < WT; ++i) {
          a[i] = As[kr + qr + 16 * i + l16];
          bb[i] = Bs[kr + qc + 16 * i + l16];
        }
        // the four contributions in turn over all tiles: each accumulator is
        // used again only after every other tile's MFMA of the same kind
        constexpr int c2 = NS - 1;
#pragma unroll
        for (int i = 0; i < WT; ++i)
#pragma unroll
          for (int j = 0; j < WT; ++j) cre[i][j][0] = M::mac(a[i].re, bb[j].re, cre[i][j][0]);
#pragma unroll
        for (int i = 0; i < WT; ++i)
#pragma unroll
          for (int j = 0; j < WT; ++j) cim[i][j][0] = M::mac(a[i].re, bb[j].im, cim[i][j][0]);
#pragma unroll
        for (int i = 0; i < WT; ++i)
#pragma unroll
          for (int j = 0; j < WT; ++j) cre[i][j][c2] = M::mac(-a[i].im, bb[j].im, cre[i][j][c2]);
#pragma unroll
        for (int i = 0; i < WT; ++i)
#pragma unroll
          for (int j = 0; j < WT; ++j) cim[i][j][c2] = M::mac(a[i].im, bb[j].re, cim[i][j][c2]);
      }
      __syncthreads();
    }
    // the block's outputs from its first entry C[b, m0, n0] (the planner
    // keeps BM rows of C within one output range)
    const GlbOut<T> out(C + ((int64_t)b * s.nm + m0) * s.nn + n0);
#pragma unroll
    for (int i = 0; i < WT; ++i)
#pragma unroll
      for (int j = 0; j < WT; ++j) {
        V vre = cre[i][j][0], vim = cim[i][j][0];
        if constexpr (NS == 2) {
          vre += cre[i][j][1];
          vim += cim[i][j][1];
        }
        const int32_t n = n0 + qc + 16 * j + l16;
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) {
          const int32_t mr = qr + 16 * i + M::row(lane, rr);
          if (m0 + mr < s.nm && n < s.nn) {
            const T vr = vre[rr] * scale, vi = vim[rr] * scale;
            put(out, mr * s.nn + (n - n0), Cx<T>{vr, vi});
            lm = fmax(lm, fmax(fabs(vr), fabs(vi)));
          }
        }
      }
  }
  if (ph) {
    const int64_t t = wall_clock64();
    ph[1] = t - tk;
    tk = t;
  }
  if (s.n_ks == 1) tile_publish<T>(p, s.c, tile_id, lm, ec, s_red);
  if (ph) ph[2] = wall_clock64() - tk;
}

// Outputs [part * kReduceChunk, ...) of a split step: C = sum over the n_ks
// partial results, in split order (the same bits on every run).
template <class T>
__device__ __attribute__((always_inline)) void reduce_step(const DevProg& p, const StepDesc& s, int32_t part, Cx<T>* arena,
                            const States& st, T* s_red) {
  const int64_t outs = (int64_t)s.nb * s.nm * s.nn;
  const int64_t o0 = (int64_t)part * kReduceChunk;
  const int64_t o1 = o0 + kReduceChunk < outs ? o0 + kReduceChunk : outs;
  const GlbCx<T>* P = (const GlbCx<T>*)(arena + s.partial);
  const GlbOut<T> C((GlbCx<T>*)(arena + s.home_c) + o0);
  T lm = 0;
  for (int64_t o = o0 + threadIdx.x; o < o1; o += kBlock) {
    T cr = 0, ci = 0;
    for (int32_t j = 0; j < s.n_ks; ++j) {
      const Cx<T> v = ldc(P + (int64_t)j * outs + o);
      cr += v.re;
      ci += v.im;
    }
    put(C, (int32_t)(o - o0), Cx<T>{cr, ci});
    lm = fmax(lm, fmax(fabs(cr), fabs(ci)));
  }
  int64_t ec;
  step_scale<T>(st, s.a, s.b, ec);
  tile_publish<T>(p, s.c, part, lm, ec, s_red);
}

// ------------------------------------------------------------------ final

template <class T>
__device__ __attribute__((always_inline)) void knot_final(const DevProg& p, const KnotDesc& kd, Cx<T>* arena, Cx<T>* lds,
                           kn_scalar* zout, const States& st, int32_t slice) {
  if (threadIdx.x != 0) return;
  const ImgHeader& h = *p.h;
  const Cx<double>* xe = p.weights + kd.w_off;
  const Cx<double>* xm = xe + kd.n_edges;
  Cx<double> z{1.0, 0.0};
  int64_t e = 0;
  for (int i = 0; i < kd.n_comps; ++i) {
    const int32_t t = p.comps[kd.comp_off + i];
    const Cx<T> r = *tptr<T>(p.tens[t], arena, lds);
    int32_t sh;
    int64_t et;
    st.get(t, sh, et);
    e += et;
    acc_mul(z, e, Cx<double>{(double)r.re, (double)r.im});
  }
  for (int i = 0; i < kd.n_factors; ++i) {
    const Factor f = p.factors[kd.factor_off + i];
    Cx<double> x = f.kind == FAC_LOOP ? xe[f.id]
                   : f.kind == FAC_CONST ? plan_consts(p, kd)[f.id]
                                         : xm[f.id];
    if (f.kind == FAC_LEAF) x.re += (double)(kd.q - 1);
    if (f.kind == FAC_PAIR) {  // equal fixed values: x_m, else 1
      int sa = slice, sb = slice;
      for (int r = 0; r < f.a; ++r) sa /= kd.q;
      for (int r = 0; r < f.b; ++r) sb /= kd.q;
      if (sa % kd.q != sb % kd.q) x = Cx<double>{1.0, 0.0};
    }
    acc_mul(z, e, x);
  }
  for (int i = 0; i < kd.n_iso; ++i) acc_mul(z, e, Cx<double>{(double)kd.q, 0.0});
  kn_scalar out;
  if (__hip_atomic_load(&p.ctrl[CTRL_ERROR], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
    out.re = out.im = __builtin_nan("");
    out.exp2 = 0;
  } else {
    out.re = z.re;
    out.im = z.im;
    out.exp2 = (z.re == 0.0 && z.im == 0.0) ? 0 : e;
  }
  // a slice's value goes to the slice array; sum_slices adds them up
  if (kd.n_slices > 1) p.zslice[kd.out_slot + slice] = out;
  else zout[kd.out_slot] = out;
}

__device__ inline Cx<double> cdiv(Cx<double> a, Cx<double> b) {
  const double s = fmax(fabs(b.re), fabs(b.im));
  const Cx<double> bs{b.re / s, b.im / s};
  const double d = bs.re * bs.re + bs.im * bs.im;
  return {(a.re * bs.re + a.im * bs.im) / (d * s), (a.im * bs.re - a.re * bs.im) / (d * s)};
}

// d log Z / d J_e for every original edge of a gradient plan (after the
// reverse steps).  For the merged edge m in slot j of vertex tensor
// F_v(s_v, s_w1..) = prod_l T_ml(s_v, s_wl) (Eq. 5; a private s_v summed),
//   dF_v/dx_m = delta(s_v, s_wj) prod_{l != j} T_ml(s_v, s_wl),
// so d log S / d J_m = x_m sum_i dS/dF_v[i] dF_v/dx_m[i] / S, S the scalar of
// the vertex's component.  A spike factor x_m + q - 1 gives
// x_m / (x_m + q - 1), a loop factor x_e gives 1, and each original edge takes
// the value of its merged edge (x_m is the product of its members' e^{J}).
// One wavefront per vertex tensor; the whole workgroup calls this, after the
// persistent kernel (tensor states and data are then all in global memory).
template <class T>
__device__ void knot_gradient(const DevProg& p, const KnotDesc& kd, const Cx<T>* arena,
                              double* grad) {
  const ImgHeader& h = *p.h;
  const Cx<double>* xm = p.weights + kd.w_off + kd.n_edges;
  Cx<double>* mg = p.mgrad + kd.medge_off;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int q = kd.q;
  constexpr int kMaxSlots = 7;
  for (int v = wv; v < kd.n_vtx; v += kBlock / 64) {
    const VtxDesc vd = p.vtx[kd.vtx_off + v];
    if (vd.keep_center < 0 || vd.adjoint < 0 || vd.n_slots == 0) continue;
    const int ns = vd.n_slots;
    const int32_t* slot_me = p.vslot + vd.slot_off;
    Cx<double> x[kMaxSlots];
#pragma unroll
    for (int j = 0; j < kMaxSlots; ++j) x[j] = j < ns ? xm[slot_me[j]] : Cx<double>{1.0, 0.0};
    int32_t qn = 1;
    for (int j = 0; j < ns; ++j) qn *= q;
    // gradient plans keep every tensor and state in global memory
    const TensorDesc td = p.tens[vd.adjoint];
    const Cx<T>* fb = arena + td.off;
    double ar[kMaxSlots], ai[kMaxSlots];
#pragma unroll
    for (int j = 0; j < kMaxSlots; ++j) ar[j] = ai[j] = 0.0;
    // entry i in F_v's order (kept centre leading, last slot fastest) sits at
    // sum of digit x stride in the adjoint's storage order
    const int32_t* astr = p.strides + vd.adj_str;
    const int32_t* sstr = astr + (vd.keep_center ? 1 : 0);
    for (int i = lane; i < td.size; i += 64) {
      int dig[kMaxSlots];
      int rem = i;
      int32_t off = 0;
#pragma unroll
      for (int j = kMaxSlots - 1; j >= 0; --j) {
        if (j < ns) {
          dig[j] = rem % q;
          rem /= q;
          off += dig[j] * sstr[j];
        } else {
          dig[j] = -1;
        }
      }
      const int centre = rem;  // kept centre (leading index); unused when private
      if (vd.keep_center) off += centre * astr[0];
      const Cx<T> f = fb[off];
#pragma unroll
      for (int j = 0; j < kMaxSlots; ++j) {
        if (j >= ns) continue;
        const int a = vd.keep_center ? centre : dig[j];
        if (dig[j] != a) continue;
        Cx<double> prod{(double)f.re, (double)f.im};
#pragma unroll
        for (int l = 0; l < kMaxSlots; ++l)
          if (l != j && l < ns && dig[l] == a) prod = cmul(prod, x[l]);
        ar[j] += prod.re;
        ai[j] += prod.im;
      }
    }
#pragma unroll
    for (int j = 0; j < kMaxSlots; ++j) {
      for (int o = 32; o >= 1; o >>= 1) {
        ar[j] += __shfl_xor(ar[j], o, 64);
        ai[j] += __shfl_xor(ai[j], o, 64);
      }
    }
    if (lane == 0) {
      const int64_t ef = p.ts[vd.adjoint].exp2;
      const int32_t root = p.comps[kd.comp_off + vd.comp];
      const Cx<T> r = arena[p.tens[root].off];
      const int64_t er = p.ts[root].exp2;
      const Cx<double> rs{(double)r.re, (double)r.im};
#pragma unroll
      for (int j = 0; j < kMaxSlots; ++j) {
        if (j >= ns) continue;
        Cx<double> g = cdiv(cmul(Cx<double>{ar[j], ai[j]}, x[j]), rs);
        g.re = ldexp(g.re, (int)(ef - er));
        g.im = ldexp(g.im, (int)(ef - er));
        mg[slot_me[j]] = g;
      }
    }
  }
  for (int i = tid; i < kd.n_factors; i += kBlock) {
    const Factor f = p.factors[kd.factor_off + i];
    if (f.kind == FAC_LEAF) {
      const Cx<double> x = xm[f.id];
      mg[f.id] = cdiv(x, Cx<double>{x.re + (double)(q - 1), x.im});
    }
  }
  __syncthreads();
  double* g = grad + 2 * (int64_t)kd.edge_off;
  for (int m = tid; m < kd.n_medges; m += kBlock) {
    const MEdge me = p.medges[kd.medge_off + m];
    const Cx<double> v = mg[m];
    for (int i = 0; i < me.n_members; ++i) {
      const int32_t e = p.members[me.member_off + i];
      g[2 * e] = v.re;
      g[2 * e + 1] = v.im;
    }
  }
  for (int i = tid; i < kd.n_factors; i += kBlock) {
    const Factor f = p.factors[kd.factor_off + i];
    if (f.kind == FAC_LOOP) {
      g[2 * f.id] = 1.0;
      g[2 * f.id + 1] = 0.0;
    }
  }
}

// ------------------------------------------------------------------ kernels

// Reset the runtime state of an image: control words, ready queue seeded
// with the knots' first groups, pending counters, tensor states; the results
// (every output scalar and slice value) start as NaN, so a knot whose final
// task never runs (the engine gave up on a queue slot) reads as NaN.
__global__ void clear_state(const uint8_t* __restrict__ img, uint8_t* __restrict__ state,
                            kn_scalar* __restrict__ zout) {
  const ImgHeader& h = *reinterpret_cast<const ImgHeader*>(img);
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const kn_scalar nan{__builtin_nan(""), __builtin_nan(""), 0};
  if (i < h.n_outputs) zout[i] = nan;
  if (i < h.n_zslice) reinterpret_cast<kn_scalar*>(state + h.o_zslice)[i] = nan;
  if (i < h.n_knots)
    reinterpret_cast<int32_t*>(state + h.o_uslice)[i] =
        reinterpret_cast<const KnotDesc*>(img + h.o_knots)[i].slice;
  int32_t* ctrl = reinterpret_cast<int32_t*>(state);
  if (i < CTRL_WORDS) ctrl[i] = (i == CTRL_TAIL) ? h.n_roots : 0;
  if (i < h.n_queue) {
    const int32_t* roots = reinterpret_cast<const int32_t*>(img + h.o_roots);
    reinterpret_cast<int32_t*>(state + h.o_queue)[i] = i < h.n_roots ? roots[i] : -1;
  }
  if (i < h.n_groups) {
    const GroupDesc* g = reinterpret_cast<const GroupDesc*>(img + h.o_groups);
    reinterpret_cast<int32_t*>(state + h.o_pending)[i] = g[i].n_pred;
  }
  if (i < h.n_tensors) {
    TensorState* ts = reinterpret_cast<TensorState*>(state + h.o_tstate);
    ts[i].shift = kShiftNone;
    ts[i].pad = 0;
    ts[i].exp2 = 0;
  }
}

// Z of a sliced plan = the sum of its slices' values: one thread per knot
// descriptor, the first slice of each plan adds up the plan's slices (they
// are consecutive), aligned to the largest exponent.
__global__ void sum_slices(const uint8_t* __restrict__ img, uint8_t* __restrict__ state,
                           kn_scalar* __restrict__ zout) {
  const ImgHeader& h = *reinterpret_cast<const ImgHeader*>(img);
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= h.n_knots) return;
  const KnotDesc* kds = reinterpret_cast<const KnotDesc*>(img + h.o_knots);
  const KnotDesc kd = kds[i];
  if (kd.n_slices <= 1 || kd.slice != 0) return;  // the plan's first chain adds its slices
  const kn_scalar* zs = reinterpret_cast<const kn_scalar*>(state + h.o_zslice) + kd.out_slot;
  int64_t emax = INT64_MIN;
  bool bad = false;
  for (int32_t j = 0; j < kd.n_slices; ++j) {
    const kn_scalar z = zs[j];
    if (!isfinite(z.re) || !isfinite(z.im)) bad = true;
    if (z.re != 0.0 || z.im != 0.0) emax = max(emax, z.exp2);
  }
  kn_scalar out{0.0, 0.0, 0};
  if (bad) {
    out.re = out.im = __builtin_nan("");
  } else if (emax != INT64_MIN) {
    double re = 0.0, im = 0.0;
    for (int32_t j = 0; j < kd.n_slices; ++j) {
      const kn_scalar z = zs[j];
      const int64_t d = z.exp2 - emax;  // <= 0
      if (d < -1100) continue;
      re += ldexp(z.re, (int)d);
      im += ldexp(z.im, (int)d);
    }
    const double m = fmax(fabs(re), fabs(im));
    if (m > 0.0) {
      int s;
      frexp(m, &s);
      out.re = ldexp(re, -s);
      out.im = ldexp(im, -s);
      out.exp2 = emax + s;
    }
  }
  zout[kd.plan_slot] = out;
}

// d log Z / d J of every knot of a gradient image: one workgroup per knot,
// launched after the persistent kernel on the same stream.
template <class T>
__global__ __launch_bounds__(kBlock) void gradient_kernel(const uint8_t* __restrict__ img,
                                                          uint8_t* __restrict__ state,
                                                          Cx<T>* __restrict__ arena,
                                                          double* __restrict__ grad) {
  const DevProg p = make_prog(img, state);
  const KnotDesc kd = p.knots[blockIdx.x];
  if (!kd.grad) return;
  knot_gradient<T>(p, kd, arena, grad);
}

// The checking build (KN_DEVICE_CHECKS) checks each task and its steps just
// before running it (checks.h) and skips a task that fails; it also fills the
// guard zone after the arena before a launch and checks it after.
#ifdef KN_DEVICE_CHECKS
constexpr bool kChecks = true;
#else
constexpr bool kChecks = false;
#endif

// Record an error: the first code wins, with the task, step and detail.
__device__ inline void report(const DevProg& p, int32_t code, int32_t task, int32_t step,
                              int32_t info) {
  int32_t expect = 0;
  if (__hip_atomic_compare_exchange_strong(&p.ctrl[CTRL_ERROR], &expect, code, __ATOMIC_RELAXED,
                                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
    __hip_atomic_store(&p.ctrl[CTRL_ERR_TASK], task, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(&p.ctrl[CTRL_ERR_STEP], step, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(&p.ctrl[CTRL_ERR_INFO], info, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// Checks of task ti before it runs (whole workgroup): thread 0 checks the
// record, then the threads share out its steps; the lowest failing step is
// reported.  True when the task may run.
template <class T>
__device__ bool task_ok(const DevProg& p, int32_t ti, int32_t* s_code, int32_t* s_step) {
  const ImageView v{p.h, p.tasks, p.groups, p.knots, p.tens, p.steps, p.vtx, p.strides, p.comps};
  const int64_t lds_elems = p.h->lds_bytes / (int64_t)sizeof(Cx<T>);
  if (threadIdx.x == 0) {
    *s_code = task_record_check(v, ti, lds_elems);
    *s_step = INT32_MAX;
  }
  __syncthreads();
  if (*s_code != CHK_OK) {
    if (threadIdx.x == 0) report(p, *s_code, ti, -1, 0);
    __syncthreads();
    return false;
  }
  const TaskDesc td = p.tasks[ti];
  const int32_t q = p.knots[td.knot].q;
  const int32_t n = td.kind == TASK_SERIAL ? td.count : 1;
  for (int32_t i = threadIdx.x; i < n; i += kBlock) {
    const StepDesc& d = p.steps[td.first + i];
    int32_t rc = step_check(d, p.tens, p.h->n_tensors, p.strides, p.h->n_strides, q,
                            p.h->arena_elems, lds_elems);
    if (td.kind == TASK_SERIAL && d.mode != STEP_SERIAL) rc = CHK_TASK;
    if (rc != CHK_OK) atomicMin(s_step, td.first + i);
  }
  __syncthreads();
  const int32_t bad = *s_step;
  if (bad != INT32_MAX && threadIdx.x == 0) {
    const StepDesc& d = p.steps[bad];
    int32_t rc = step_check(d, p.tens, p.h->n_tensors, p.strides, p.h->n_strides, q,
                            p.h->arena_elems, lds_elems);
    if (rc == CHK_OK) rc = CHK_TASK;
    report(p, rc, ti, bad, 0);
  }
  __syncthreads();
  return bad == INT32_MAX;
}

// Guard zone after the arena: filled before a launch, checked after it.
__global__ void fill_guard(uint8_t* __restrict__ ws) {
  const ImgHeader& h = *reinterpret_cast<const ImgHeader*>(ws);
  uint32_t* g = reinterpret_cast<uint32_t*>(ws + h.guard_off);
  for (int32_t i = threadIdx.x; i < (int32_t)(kGuardBytes / 4); i += blockDim.x) g[i] = kGuardWord;
}

__global__ void check_guard(const uint8_t* __restrict__ ws, uint8_t* __restrict__ state) {
  const ImgHeader& h = *reinterpret_cast<const ImgHeader*>(ws);
  const uint32_t* g = reinterpret_cast<const uint32_t*>(ws + h.guard_off);
  DevProg p;
  p.ctrl = reinterpret_cast<int32_t*>(state);
  for (int32_t i = threadIdx.x; i < (int32_t)(kGuardBytes / 4); i += blockDim.x)
    if (g[i] != kGuardWord) report(p, CHK_GUARD, -1, -1, i);
}

// Bound on the wait for a queue slot, in ticks of the 100 MHz device clock
// (20 s, far beyond any launch's critical path): a slot that is never filled
// (a planner bug) ends the kernel with the error flag set instead of hanging
// the device; the knots left unfinished keep the NaN that clear_state wrote.
constexpr int64_t kWaitTicks = 20LL * 100000000LL;

extern __shared__ __align__(16) uint8_t kn_dyn_smem[];

template <class T>
__global__ __launch_bounds__(kBlock, 2) void engine(const uint8_t* __restrict__ img,
                                                 uint8_t* __restrict__ state,
                                                 Cx<T>* __restrict__ arena,
                                                 const double* __restrict__ J,
                                                 kn_scalar* __restrict__ zout,
                                                 TraceRec* __restrict__ trace) {
  __shared__ int32_t s_task;
  __shared__ int32_t s_enq[3];
  __shared__ T s_red[kBlock / 64];
  __shared__ int32_t s_tb[kDescBuf + 1];
  __shared__ int64_t s_ph[4];
  __shared__ int32_t s_chk[2];
  int32_t* s_tab = reinterpret_cast<int32_t*>(kn_dyn_smem + kLdsTab);
  StepDesc* s_desc = reinterpret_cast<StepDesc*>(kn_dyn_smem + kLdsDesc);
  int32_t* s_shift = reinterpret_cast<int32_t*>(kn_dyn_smem + kLdsShift);
  int64_t* s_exp = reinterpret_cast<int64_t*>(kn_dyn_smem + kLdsExp);
  TensorState* s_ext = reinterpret_cast<TensorState*>(kn_dyn_smem + kLdsExt);
  Cx<T>* lds = reinterpret_cast<Cx<T>*>(kn_dyn_smem + kLdsArena);
  const DevProg p = make_prog(img, state);
  const int32_t n_queue = p.h->n_queue;
  const int tid = threadIdx.x;
  for (;;) {
    int64_t t_claim = 0;
    if (tid == 0) {
      if (trace) t_claim = wall_clock64();
      const int32_t slot = atomicAdd(&p.ctrl[CTRL_HEAD], 1);
      int32_t t = -1;
      if (slot < n_queue) {
        int32_t nap = 1;
        const int64_t t_wait = wall_clock64();
        while ((t = __hip_atomic_load(&p.queue[slot], __ATOMIC_RELAXED,
                                      __HIP_MEMORY_SCOPE_AGENT)) < 0) {
          if (nap < 16) {
            __builtin_amdgcn_s_sleep(1);
            ++nap;
          } else {
            __builtin_amdgcn_s_sleep(8);
            // after an error the slot may never be filled: give up at once
            if (__hip_atomic_load(&p.ctrl[CTRL_ERROR], __ATOMIC_RELAXED,
                                  __HIP_MEMORY_SCOPE_AGENT) != 0)
              break;
          }
          if (wall_clock64() - t_wait > kWaitTicks) {
            report(p, CHK_QUEUE_WAIT, -1, -1, slot);
            break;
          }
        }
      }
      s_task = t;
    }
    __syncthreads();
    const int32_t ti = s_task;
    __syncthreads();
    if (ti < 0) break;
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    const int64_t t_start = (trace && tid == 0) ? wall_clock64() : 0;
    const TaskDesc td = p.tasks[ti];
    // a sliced unit that starts its next slice after this task (its final task)
    int32_t next_slice = -1;
    // the checking build skips a task that fails its checks and only
    // publishes it, so the launch still drains
    const bool run = !kChecks || task_ok<T>(p, ti, &s_chk[0], &s_chk[1]);
    if (!run) {
      // skipped: it writes nothing, and its knot's result stays NaN
    } else if (td.kind == TASK_SERIAL) {
      const KnotDesc kd = p.knots[td.knot];
      const int32_t slice = p.uslice[td.knot];
      const States st{p.ts, s_shift, s_exp, td.state_lo, min(td.state_len, kStateCap)};
      int64_t ph_buf[4] = {0, 0, 0, 0};
      int64_t* ph = (trace && tid == 0) ? ph_buf : nullptr;
      if (td.flags & TF_SETUP) {
        knot_setup<T>(p, kd, arena, lds, J, st, slice);
        __syncthreads();
      }
      if (ph) ph[0] = wall_clock64() - t_start;
      serial_steps<T>(p, td.first, td.count, kd.q, arena, lds, s_tab, s_desc, s_tb, s_ext, st,
                      s_red, ph);
      if (td.flags & TF_FINAL) knot_final<T>(p, kd, arena, lds, zout, st, slice);
      if (ph)
        for (int i = 0; i < 4; ++i) s_ph[i] = ph[i];
      // states of this task's tensors go back to global memory for later groups
      for (int32_t i = tid; i < st.len; i += kBlock) {
        p.ts[st.lo + i].shift = s_shift[i];
        p.ts[st.lo + i].exp2 = s_exp[i];
      }
      // the last task of a slice whose chain has more: every group and tensor
      // of the unit is done with, so its counters and tensor states are reset
      // for the next slice here (published with this task's release below)
      if ((td.flags & TF_FINAL) && kd.n_slices > 1 && slice + kd.slice_step < kd.n_slices) {
        next_slice = slice + kd.slice_step;
        __syncthreads();
        for (int32_t g = tid; g < kd.n_groups; g += kBlock)
          p.pending[kd.group_off + g] = p.groups[kd.group_off + g].n_pred;
        for (int32_t t = tid; t < kd.n_tensors; t += kBlock) {
          p.ts[kd.tensor_off + t].shift = kShiftNone;
          p.ts[kd.tensor_off + t].exp2 = 0;
        }
        if (tid == 0) p.uslice[td.knot] = next_slice;
      }
    } else {
      const States st{p.ts, s_shift, s_exp, 0, 0};
      // traced launches: thread 0 writes the phases straight into s_ph
      int64_t* ph = (trace && tid == 0) ? s_ph : nullptr;
      if (ph) {
        for (int i = 0; i < 3; ++i) ph[i] = 0;
        ph[3] = t_start;
      }
      const StepDesc sd = p.steps[td.first];
      const int32_t q = p.knots[td.knot].q;
      const int32_t dyn = kLdsArena + p.h->lds_bytes;
      if (td.kind == TASK_REDUCE)
        reduce_step<T>(p, sd, td.count, arena, st, s_red);
      else if (sd.mode == STEP_GEMM)
        gemm_tile<T, 2>(p, sd, td.count, q, arena, kn_dyn_smem, dyn, st, s_red, ph);
      else if (sd.mode == STEP_GEMM64)
        gemm_tile<T, 4>(p, sd, td.count, q, arena, kn_dyn_smem, dyn, st, s_red, ph);
      else
        tile_step<T>(p, sd, td.count, q, arena, s_tab, dyn / 4, st, s_red, ph);
      if (ph) ph[3] = 0;
    }
    // ---- publish; the last task of a group releases the knot's next group
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    if (tid == 0) {
      s_enq[0] = 0;
      const int32_t next = p.groups[td.group].next;
      if (next_slice >= 0) {
        // the unit's first group again, for its next slice
        const GroupDesc g = p.groups[p.knots[td.knot].group_off];
        s_enq[0] = g.n_tasks;
        s_enq[1] = g.first_task;
        s_enq[2] = atomicAdd(&p.ctrl[CTRL_TAIL], g.n_tasks);
      } else if (next >= 0 && __hip_atomic_fetch_add(&p.pending[next], -1, __ATOMIC_ACQ_REL,
                                                     __HIP_MEMORY_SCOPE_AGENT) == 1) {
        const GroupDesc g = p.groups[next];
        s_enq[0] = g.n_tasks;
        s_enq[1] = g.first_task;
        s_enq[2] = atomicAdd(&p.ctrl[CTRL_TAIL], g.n_tasks);
      }
      if (trace) {
        TraceRec r{t_claim, t_start, wall_clock64(), ti, (int32_t)blockIdx.x, {0, 0, 0, 0}};
        for (int i = 0; i < 4; ++i) r.ph[i] = s_ph[i];
        trace[ti] = r;
      }
    }
    __syncthreads();
    const int32_t n_enq = s_enq[0];
    if (n_enq) {
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      const int32_t first = s_enq[1], base = s_enq[2];
      for (int32_t i = tid; i < n_enq; i += kBlock)
        __hip_atomic_store(&p.queue[base + i], first + i, __ATOMIC_RELEASE,
                           __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

// ------------------------------------------------------------------ host side

// Pool of host buffers for batch images.  Page-locked memory (hipHostMalloc)
// makes an image upload a DMA transfer with no staging copy on the CPU; it is
// slow to allocate, so buffers are kept and reused (best fit by capacity).
// Without a usable device the buffers are ordinary heap memory.
namespace {

std::mutex g_buf_mu;
std::multimap<size_t, std::pair<uint8_t*, bool>> g_buf_free;  // capacity -> (buffer, pinned)

}  // namespace

uint8_t* host_buf_get(size_t bytes, size_t* capacity, bool* pinned) {
  {
    std::lock_guard<std::mutex> lock(g_buf_mu);
    auto it = g_buf_free.lower_bound(bytes);
    if (it != g_buf_free.end() && it->first <= 2 * bytes + (1u << 20)) {
      *capacity = it->first;
      *pinned = it->second.second;
      uint8_t* p = it->second.first;
      g_buf_free.erase(it);
      return p;
    }
  }
  const size_t cap = (std::max<size_t>(bytes, 1) + (1u << 20) - 1) & ~size_t((1u << 20) - 1);
  void* p = nullptr;
  if (hipHostMalloc(&p, cap, hipHostMallocDefault) == hipSuccess && p) {
    *capacity = cap;
    *pinned = true;
    return static_cast<uint8_t*>(p);
  }
  (void)hipGetLastError();  // no device: fall back to the heap
  p = std::malloc(cap);
  if (!p) return nullptr;
  *capacity = cap;
  *pinned = false;
  return static_cast<uint8_t*>(p);
}

void host_buf_put(uint8_t* p, size_t capacity, bool pinned) {
  if (!p) return;
  std::lock_guard<std::mutex> lock(g_buf_mu);
  g_buf_free.emplace(capacity, std::make_pair(p, pinned));
  // keep the pool bounded: drop the largest buffers beyond 8
  while (g_buf_free.size() > 8) {
    auto last = std::prev(g_buf_free.end());
    if (last->second.second) (void)hipHostFree(last->second.first);
    else std::free(last->second.first);
    g_buf_free.erase(last);
  }
}

namespace {

int device_cus() {
  static int cus = 0;
  static std::once_flag once;
  std::call_once(once, [] {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) dev = 0;
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v <= 0)
      v = 256;
    cus = v;
  });
  return cus;
}

template <class T>
kn_status launch_engine(const ImgHeader& h, uint8_t* ws, hipStream_t st, const double* J,
                        kn_scalar* z, double* grad, int32_t grid_override, TraceRec* trace) {
  const size_t dyn = (size_t)kLdsArena + (size_t)h.lds_bytes + (size_t)stage_bytes(h.lds_bytes);
  static std::once_flag once;
  static bool attr_ok = true;
  std::call_once(once, [] {
    attr_ok = hipFuncSetAttribute(reinterpret_cast<const void*>(engine<T>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize,
                                  kLdsLimit) == hipSuccess;
  });
  if (!attr_ok) return KN_E_DEVICE;
  // default: one workgroup per compute unit (measured faster than filling
  // each CU with as many as fit: a workgroup running a knot's critical chain
  // then has its CU to itself)
  int32_t grid = grid_override;
  if (grid <= 0) grid = device_cus();
  if (grid > h.n_queue) grid = h.n_queue;
  if (grid < 1) grid = 1;
  hipLaunchKernelGGL(engine<T>, dim3(grid), dim3(kBlock), dyn, st, ws, ws + h.state_off,
                     reinterpret_cast<Cx<T>*>(ws + h.arena_off), J, z, trace);
  if (hipGetLastError() != hipSuccess) return KN_E_DEVICE;
  if (grad) {
    hipLaunchKernelGGL(gradient_kernel<T>, dim3(h.n_knots), dim3(kBlock), 0, st, ws,
                       ws + h.state_off, reinterpret_cast<Cx<T>*>(ws + h.arena_off), grad);
    if (hipGetLastError() != hipSuccess) return KN_E_DEVICE;
  }
  if (h.sliced) {
    hipLaunchKernelGGL(sum_slices, dim3((h.n_knots + 255) / 256), dim3(256), 0, st, ws,
                       ws + h.state_off, z);
    if (hipGetLastError() != hipSuccess) return KN_E_DEVICE;
  }
  return KN_OK;
}

kn_status launch(const ImgHeader& h, uint8_t* ws, hipStream_t st, const double* J,
                 kn_scalar* z, double* grad, int32_t grid_override, TraceRec* trace = nullptr) {
  int64_t n_clear = CTRL_WORDS;
  n_clear = std::max<int64_t>(n_clear, h.n_tasks);
  n_clear = std::max<int64_t>(n_clear, h.n_groups);
  n_clear = std::max<int64_t>(n_clear, h.n_tensors);
  n_clear = std::max<int64_t>(n_clear, h.n_knots);
  n_clear = std::max<int64_t>(n_clear, h.n_queue);
  n_clear = std::max<int64_t>(n_clear, h.n_zslice);
  hipLaunchKernelGGL(clear_state, dim3((unsigned)((n_clear + 255) / 256)), dim3(256), 0, st, ws,
                     ws + h.state_off, z);
  if (hipGetLastError() != hipSuccess) return KN_E_DEVICE;
  if (kChecks) {
    hipLaunchKernelGGL(fill_guard, dim3(1), dim3(256), 0, st, ws);
    if (hipGetLastError() != hipSuccess) return KN_E_DEVICE;
  }
  const kn_status rc = h.precision == 1
                           ? launch_engine<float>(h, ws, st, J, z, grad, grid_override, trace)
                           : launch_engine<double>(h, ws, st, J, z, grad, grid_override, trace);
  if (rc != KN_OK || !kChecks) return rc;
  hipLaunchKernelGGL(check_guard, dim3(1), dim3(256), 0, st, ws, ws + h.state_off);
  if (hipGetLastError() != hipSuccess) return KN_E_DEVICE;
  return KN_OK;
}

bool aligned256(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 255) == 0; }

}  // namespace
}  // namespace kn

using namespace kn;

namespace {

kn_status contract_plan(const kn_plan* p, const double* J, void* workspace,
                        size_t workspace_bytes, void* stream, kn_scalar* z_dev, double* grad) {
  if (!p || !workspace || !z_dev) return KN_E_INVALID;
  const Bytes& image = plan_image(p);
  if (image.empty()) return KN_E_BUDGET;
  if (J && p->k.jones_only) return KN_E_UNSUPPORTED;
  if (!aligned256(workspace)) return KN_E_INVALID;
  const ImgHeader& h = *reinterpret_cast<const ImgHeader*>(image.data());
  if ((int64_t)workspace_bytes < h.workspace_bytes) return KN_E_BUDGET;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  if (hipMemcpyAsync(workspace, image.data(), (size_t)h.image_bytes, hipMemcpyHostToDevice, st) !=
      hipSuccess)
    return KN_E_DEVICE;
  return launch(h, reinterpret_cast<uint8_t*>(workspace), st, J, z_dev, grad, 0);
}

}  // namespace

extern "C" kn_status kn_contract(const kn_plan* p, const double* J, void* workspace,
                                 size_t workspace_bytes, void* stream, kn_scalar* z_dev) {
  return contract_plan(p, J, workspace, workspace_bytes, stream, z_dev, nullptr);
}

// ------------------------------------------------------------------ fixed scratch
// Workspace of kn_contract_noalloc: one library-owned array per device, in
// place of the caller's workspace, so that the call allocates nothing.  In
// host code `scratch` names a host-side stand-in, never the device memory:
// its device address is looked up once per device (hipGetSymbolAddress) and
// only that address is handed to the kernels.
static __device__ __align__(256) uint8_t scratch[KN_NOALLOC_MAX_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices];  // device address of `scratch` per device (null: not looked up)

// Device address of the current device's copy of `scratch`.
kn_status scratch_address(void** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return KN_E_DEVICE;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
      (void)hipGetLastError();
      return KN_E_DEVICE;
    }
    g_scratch_dev[dev] = ptr;
  }
  *out = g_scratch_dev[dev];
  return KN_OK;
}

}  // namespace

extern "C" kn_status kn_contract_noalloc(const kn_plan* p, const double* J, void* stream,
                                         kn_scalar* z_dev) {
  if (!p || !z_dev) return KN_E_INVALID;
  const Bytes& image = plan_image(p);
  if (image.empty()) return KN_E_BUDGET;
  const ImgHeader& h = *reinterpret_cast<const ImgHeader*>(image.data());
  if (h.workspace_bytes > (int64_t)KN_NOALLOC_MAX_BYTES) return KN_E_BUDGET;
  void* ws = nullptr;
  const kn_status rc = scratch_address(&ws);
  if (rc != KN_OK) return rc;
  return contract_plan(p, J, ws, KN_NOALLOC_MAX_BYTES, stream, z_dev, nullptr);
}

extern "C" kn_status kn_batch_create(const kn_plan* const* plans, int32_t n, kn_batch** out) {
  if (!out) return KN_E_INVALID;
  *out = nullptr;
  if (!plans || n <= 0) return KN_E_INVALID;
  std::vector<const PlanKnot*> ks;
  bool jones_only = false, gradient = true;
  for (int32_t i = 0; i < n; ++i) {
    if (!plans[i] || !plans[i]->laid_out) return KN_E_INVALID;
    if (plans[i]->k.precision != plans[0]->k.precision) return KN_E_INVALID;
    jones_only |= plans[i]->k.jones_only;
    gradient &= plans[i]->k.gradient;
    ks.push_back(&plans[i]->k);
  }
  kn_batch* b = new (std::nothrow) kn_batch();
  if (!b) return KN_E_NOMEM;
  try {
    const int64_t nb = build_image_into(
        ks, [&](size_t bytes) { return b->image.allocate(bytes); }, nullptr);
    if (nb < 0) {
      delete b;
      return nb == -2 ? KN_E_NOMEM : KN_E_BUDGET;
    }
    b->precision = plans[0]->k.precision;
    b->jones_only = jones_only;
    b->gradient = gradient;
    int64_t off = 0;
    double flops = 0, bytes = 0;
    for (int32_t i = 0; i < n; ++i) {
      b->edge_offset.push_back(off);
      off += plans[i]->k.n_edges;
      flops += plans[i]->stats.flops;
      bytes += plans[i]->stats.bytes;
    }
    const ImgHeader& h = *reinterpret_cast<const ImgHeader*>(b->image.data());
    b->stats.workspace_bytes = (uint64_t)h.workspace_bytes;
    b->stats.image_bytes = (uint64_t)h.image_bytes;
    b->stats.n_tasks = h.n_tasks;
    b->stats.n_knots = n;
    b->stats.flops = flops;
    b->stats.bytes = bytes;
    b->stats.total_edges = off;
    b->stats.grid = 0;
  } catch (const std::bad_alloc&) {
    delete b;
    return KN_E_NOMEM;
  }
  *out = b;
  return KN_OK;
}

extern "C" kn_status kn_batch_info(const kn_batch* b, kn_batch_stats* out) {
  if (!b || !out) return KN_E_INVALID;
  *out = b->stats;
  int32_t grid = b->grid_override > 0 ? b->grid_override : 0;
  out->grid = grid;
  return KN_OK;
}

extern "C" kn_status kn_batch_edge_offset(const kn_batch* b, int32_t i, int64_t* off) {
  if (!b || !off || i < 0 || i >= (int32_t)b->edge_offset.size()) return KN_E_INVALID;
  *off = b->edge_offset[i];
  return KN_OK;
}

extern "C" kn_status kn_batch_upload(const kn_batch* b, void* workspace, size_t workspace_bytes,
                                     void* stream) {
  if (!b || !workspace) return KN_E_INVALID;
  if (!aligned256(workspace)) return KN_E_INVALID;
  const ImgHeader& h = *reinterpret_cast<const ImgHeader*>(b->image.data());
  if ((int64_t)workspace_bytes < h.workspace_bytes) return KN_E_BUDGET;
  if (hipMemcpyAsync(workspace, b->image.data(), (size_t)h.image_bytes, hipMemcpyHostToDevice,
                     reinterpret_cast<hipStream_t>(stream)) != hipSuccess)
    return KN_E_DEVICE;
  return KN_OK;
}

namespace {

kn_status contract_batch(const kn_batch* b, const double* J, void* workspace,
                         size_t workspace_bytes, void* stream, kn_scalar* z_dev, double* grad) {
  if (!b || !workspace || !z_dev) return KN_E_INVALID;
  if (J && b->jones_only) return KN_E_UNSUPPORTED;
  if (!aligned256(workspace)) return KN_E_INVALID;
  const ImgHeader& h = *reinterpret_cast<const ImgHeader*>(b->image.data());
  if ((int64_t)workspace_bytes < h.workspace_bytes) return KN_E_BUDGET;
  if (b->trace && b->trace_bytes < (size_t)h.n_tasks * sizeof(TraceRec)) return KN_E_BUDGET;
  return launch(h, reinterpret_cast<uint8_t*>(workspace), reinterpret_cast<hipStream_t>(stream), J,
                z_dev, grad, b->grid_override, reinterpret_cast<TraceRec*>(b->trace));
}

}  // namespace

extern "C" kn_status kn_batch_contract(const kn_batch* b, const double* J, void* workspace,
                                       size_t workspace_bytes, void* stream, kn_scalar* z_dev) {
  return contract_batch(b, J, workspace, workspace_bytes, stream, z_dev, nullptr);
}

extern "C" kn_status kn_batch_contract_backward(const kn_batch* b, const double* J,
                                                void* workspace, size_t workspace_bytes,
                                                void* stream, kn_scalar* z_dev, double* grad_dev) {
  if (!b || !grad_dev) return KN_E_INVALID;
  if (!b->gradient) return KN_E_UNSUPPORTED;
  return contract_batch(b, J, workspace, workspace_bytes, stream, z_dev, grad_dev);
}

extern "C" kn_status kn_batch_image(const kn_batch* b, const void** data, size_t* bytes) {
  if (!b || !data || !bytes) return KN_E_INVALID;
  *data = b->image.data();
  *bytes = b->image.size();
  return KN_OK;
}

extern "C" kn_status kn_batch_set_grid(kn_batch* b, int32_t grid) {
  if (!b || grid < 0) return KN_E_INVALID;
  b->grid_override = grid;
  return KN_OK;
}

extern "C" kn_status kn_batch_set_trace(kn_batch* b, void* trace_dev, size_t bytes) {
  if (!b) return KN_E_INVALID;
  b->trace = trace_dev;
  b->trace_bytes = trace_dev ? bytes : 0;
  return KN_OK;
}

extern "C" void kn_batch_free(kn_batch* b) { delete b; }

extern "C" kn_status kn_backward_workspace(const kn_plan* p, uint64_t* bytes) {
  if (!p || !bytes) return KN_E_INVALID;
  if (!p->k.gradient) return KN_E_UNSUPPORTED;
  *bytes = p->stats.workspace_bytes;
  return KN_OK;
}

extern "C" kn_status kn_contract_backward(const kn_plan* p, const double* J, void* workspace,
                                          size_t workspace_bytes, void* stream, kn_scalar* z_dev,
                                          double* grad_dev) {
  if (!p || !grad_dev) return KN_E_INVALID;
  if (!p->k.gradient) return KN_E_UNSUPPORTED;
  return contract_plan(p, J, workspace, workspace_bytes, stream, z_dev, grad_dev);
}

// ------------------------------------------------------------------ status

extern "C" int32_t kn_device_checks(void) { return kChecks ? 1 : 0; }

extern "C" kn_status kn_workspace_status(const void* workspace, void* stream, int32_t* status) {
  if (!workspace || !status) return KN_E_INVALID;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  ImgHeader h;
  int32_t w[CTRL_ERR_INFO + 1];
  if (hipMemcpyAsync(&h, workspace, sizeof(h), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return KN_E_DEVICE;
  if (h.magic != kMagic) return KN_E_INVALID;
  if (hipMemcpyAsync(w, reinterpret_cast<const uint8_t*>(workspace) + h.state_off, sizeof(w),
                     hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return KN_E_DEVICE;
  status[0] = w[CTRL_ERROR];
  status[1] = w[CTRL_ERR_TASK];
  status[2] = w[CTRL_ERR_STEP];
  status[3] = w[CTRL_ERR_INFO];
  return KN_OK;
}
