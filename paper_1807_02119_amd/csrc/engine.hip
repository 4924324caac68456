// engine.hip -- GPU contraction of PACI tensor networks (Sec. III of
// arXiv:1807.02119) for CDNA4 (gfx950).
//
// One persistent kernel executes the task list of a device program (see
// program.h).  Workgroups take tasks in list order from a global ticket; a
// task first waits until the tensors it reads are complete (per-tensor
// completion counters, acquire at device scope), runs, then publishes what it
// wrote (release at device scope) and bumps the counters of the tensors it
// produced.  Because tasks are handed out in an order in which every
// dependency precedes its consumer, the earliest unfinished task always has
// its inputs and the queue cannot deadlock, whatever the grid size.
//
// Work done by tasks:
//   setup   edge weights x_e = e^{J_e} (or the Jones couplings -t^{-eps_e},
//           Sec. II), merged weights x_m = prod x_e over parallel edges, and
//           every vertex tensor F_v(s_v, s_w...) = prod_j T_{v wj}(s_v, s_wj)
//           with T = 1 + (x - 1) delta (Eqs. 3, 5); a vertex spin private to
//           its tensor is summed here.
//   step    C[b,m,n] = sum_k A[b,m,k] B[b,k,n] (one pairwise contraction of
//           Eq. 6).  Operands are gathered through per-step offset tables, so
//           the permutation that brings A and B into GEMM order is fused into
//           the loads and never materialised.  Each tensor is stored as a raw
//           mantissa array R with an int64 exponent e (true = R 2^e) and a
//           shift s = frexp exponent of max(|Re|,|Im|) over R; the consumer
//           multiplies by 2^-(sA+sB) while accumulating, so every product
//           stays bounded by the contracted extent and Z never overflows.
//   final   Z = prod over components of (scalar R 2^e) times the
//           simplification factors (loops x_e, spikes x_m + q - 1) and q per
//           isolated spin, renormalised after every product.
#include <hip/hip_runtime.h>

#include <climits>
#include <cstdint>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>

#include "internal.h"

namespace kn {

template <class T>
struct alignas(2 * sizeof(T)) Cx {
  T re, im;
};

struct DevProg {
  const ImgHeader* h;
  const TaskDesc* tasks;
  const int32_t* deps;
  const KnotDesc* knots;
  const TensorDesc* tens;
  const StepDesc* steps;
  const VtxDesc* vtx;
  const int32_t* vslot;
  const MEdge* medges;
  const int32_t* members;
  const Factor* factors;
  const int32_t* tables;
  const int8_t* eps;
  const int32_t* comps;
  TensorState* ts;
  Cx<double>* weights;  // x_e (n_edges) then x_m (n_medges)
  int32_t* ctrl;        // [0] ticket, [1] error
};

__device__ inline DevProg make_prog(const uint8_t* img, uint8_t* state) {
  DevProg p;
  p.h = reinterpret_cast<const ImgHeader*>(img);
  const ImgHeader& h = *p.h;
  p.tasks = reinterpret_cast<const TaskDesc*>(img + h.o_tasks);
  p.deps = reinterpret_cast<const int32_t*>(img + h.o_deps);
  p.knots = reinterpret_cast<const KnotDesc*>(img + h.o_knots);
  p.tens = reinterpret_cast<const TensorDesc*>(img + h.o_tensors);
  p.steps = reinterpret_cast<const StepDesc*>(img + h.o_steps);
  p.vtx = reinterpret_cast<const VtxDesc*>(img + h.o_vtx);
  p.vslot = reinterpret_cast<const int32_t*>(img + h.o_vslot);
  p.medges = reinterpret_cast<const MEdge*>(img + h.o_medges);
  p.members = reinterpret_cast<const int32_t*>(img + h.o_members);
  p.factors = reinterpret_cast<const Factor*>(img + h.o_factors);
  p.tables = reinterpret_cast<const int32_t*>(img + h.o_tables);
  p.eps = reinterpret_cast<const int8_t*>(img + h.o_eps);
  p.comps = reinterpret_cast<const int32_t*>(img + h.o_comps);
  p.ctrl = reinterpret_cast<int32_t*>(state);
  p.ts = reinterpret_cast<TensorState*>(state + h.o_tstate);
  p.weights = reinterpret_cast<Cx<double>*>(state + h.o_weights);
  return p;
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
  __syncthreads();
  if (lane == 0) red[wv] = v;
  __syncthreads();
  T r = red[0];
#pragma unroll
  for (int i = 1; i < kBlock / 64; ++i) r = fmax(r, red[i]);
  return r;
}

// ------------------------------------------------------------------ setup

template <class T>
__device__ void knot_setup(const DevProg& p, const KnotDesc& kd, Cx<T>* arena, const double* J) {
  const int tid = threadIdx.x;
  const ImgHeader& h = *p.h;
  Cx<double>* xe = p.weights + kd.edge_off;
  Cx<double>* xm = p.weights + h.n_edges + kd.medge_off;
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
    for (int i = 0; i < me.n_members; ++i) x = cmul(x, xe[p.members[me.member_off + i]]);
    xm[m] = x;
  }
  __syncthreads();
  // vertex tensors: one wavefront per tensor
  const int lane = tid & 63, wv = tid >> 6;
  const int q = kd.q;
  for (int v = wv; v < kd.n_vtx; v += kBlock / 64) {
    const VtxDesc vd = p.vtx[kd.vtx_off + v];
    const TensorDesc td = p.tens[vd.tensor];
    Cx<T>* out = arena + td.off;
    for (int i = lane; i < td.size; i += 64) {
      // digits: last neighbour slot fastest; the kept centre is the leading index
      int rem = i;
      int dig[8];
      for (int j = vd.n_slots - 1; j >= 0; --j) {
        dig[j] = rem % q;
        rem /= q;
      }
      Cx<double> acc{0.0, 0.0};
      const int a_lo = vd.keep_center ? rem : 0;
      const int a_hi = vd.keep_center ? rem + 1 : q;
      for (int a = a_lo; a < a_hi; ++a) {
        Cx<double> prod{1.0, 0.0};
        for (int j = 0; j < vd.n_slots; ++j)
          if (dig[j] == a) prod = cmul(prod, xm[p.vslot[vd.slot_off + j]]);
        acc.re += prod.re;
        acc.im += prod.im;
      }
      out[i] = Cx<T>{(T)acc.re, (T)acc.im};
    }
    if (lane == 0) {
      p.ts[vd.tensor].shift = 0;  // entries are products of <= 8 weights: no scaling needed
      p.ts[vd.tensor].exp2 = 0;
    }
  }
}

// ------------------------------------------------------------------ step

// Computes outputs [o_begin, o_end) of step s; returns this thread's max |.|.
template <class T>
__device__ T step_outputs(const DevProg& p, const StepDesc& s, Cx<T>* arena, int64_t o_begin,
                          int64_t o_end, T scale) {
  const TensorDesc A = p.tens[s.a], B = p.tens[s.b], C = p.tens[s.c];
  const int32_t* tAb = p.tables + s.tab;
  const int32_t* tAm = tAb + s.nb;
  const int32_t* tAk = tAm + s.nm;
  const int32_t* tBb = tAk + s.nk;
  const int32_t* tBk = tBb + s.nb;
  const int32_t* tBn = tBk + s.nk;
  const Cx<T>* pa = arena + A.off;
  const Cx<T>* pb = arena + B.off;
  Cx<T>* pc = arena + C.off;
  const int32_t nn = s.nn, mn = s.nm * s.nn, nk = s.nk;
  T lmax = 0;
  for (int64_t o = o_begin + threadIdx.x; o < o_end; o += kBlock) {
    const int32_t oi = (int32_t)o;
    const int32_t b = oi / mn;
    const int32_t r = oi - b * mn;
    const int32_t m = r / nn;
    const int32_t n = r - m * nn;
    const Cx<T>* ra = pa + tAb[b] + tAm[m];
    const Cx<T>* rb = pb + tBb[b] + tBn[n];
    T cr = 0, ci = 0;
    for (int32_t k = 0; k < nk; ++k) {
      const Cx<T> x = ra[tAk[k]];
      const Cx<T> y = rb[tBk[k]];
      cr = fma(x.re, y.re, cr);
      cr = fma(-x.im, y.im, cr);
      ci = fma(x.re, y.im, ci);
      ci = fma(x.im, y.re, ci);
    }
    cr *= scale;
    ci *= scale;
    pc[oi] = Cx<T>{cr, ci};
    lmax = fmax(lmax, fmax(fabs(cr), fabs(ci)));
  }
  return lmax;
}

template <class T>
__device__ inline T step_scale(const DevProg& p, const StepDesc& s, int64_t& e_out) {
  const TensorState sa = p.ts[s.a], sb = p.ts[s.b];
  const int32_t sh = shift_of(sa.shift) + shift_of(sb.shift);
  e_out = sa.exp2 + sb.exp2 + sh;
  return (T)ldexp(1.0, -sh);
}

template <class T>
__device__ inline int32_t frexp_shift(T m) {
  if (!(m > 0)) return kShiftNone;
  int s;
  frexp((double)m, &s);
  return s;
}

// ------------------------------------------------------------------ final

template <class T>
__device__ void knot_final(const DevProg& p, const KnotDesc& kd, const Cx<T>* arena,
                           kn_scalar* zout) {
  if (threadIdx.x != 0) return;
  const ImgHeader& h = *p.h;
  const Cx<double>* xe = p.weights + kd.edge_off;
  const Cx<double>* xm = p.weights + h.n_edges + kd.medge_off;
  Cx<double> z{1.0, 0.0};
  int64_t e = 0;
  for (int i = 0; i < kd.n_comps; ++i) {
    const int32_t t = p.comps[kd.comp_off + i];
    const Cx<T> r = arena[p.tens[t].off];
    e += p.ts[t].exp2;
    acc_mul(z, e, Cx<double>{(double)r.re, (double)r.im});
  }
  for (int i = 0; i < kd.n_factors; ++i) {
    const Factor f = p.factors[kd.factor_off + i];
    Cx<double> x = f.kind == FAC_LOOP ? xe[f.id] : xm[f.id];
    if (f.kind == FAC_LEAF) x.re += (double)(kd.q - 1);
    acc_mul(z, e, x);
  }
  for (int i = 0; i < kd.n_iso; ++i) acc_mul(z, e, Cx<double>{(double)kd.q, 0.0});
  kn_scalar out;
  if (__hip_atomic_load(&p.ctrl[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
    out.re = out.im = __builtin_nan("");
    out.exp2 = 0;
  } else {
    out.re = z.re;
    out.im = z.im;
    out.exp2 = (z.re == 0.0 && z.im == 0.0) ? 0 : e;
  }
  zout[kd.out_slot] = out;
}

// ------------------------------------------------------------------ kernels

__global__ void clear_state(uint8_t* state, int32_t n_tensors, int64_t o_tstate) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < 64) reinterpret_cast<int32_t*>(state)[i] = 0;
  TensorState* ts = reinterpret_cast<TensorState*>(state + o_tstate);
  if (i < n_tensors) {
    ts[i].shift = kShiftNone;
    ts[i].done = 0;
    ts[i].exp2 = 0;
  }
}

// Bound on the wait for one dependency (sleep iterations, ~0.3 us each): a
// dependency that is never satisfied (a planner bug) ends the task with the
// error flag set instead of hanging the device.
constexpr int32_t kSpinLimit = 1 << 24;

template <class T>
__global__ __launch_bounds__(kBlock) void engine(const uint8_t* __restrict__ img,
                                                 uint8_t* __restrict__ state,
                                                 Cx<T>* __restrict__ arena,
                                                 const double* __restrict__ J,
                                                 kn_scalar* __restrict__ zout) {
  __shared__ int32_t s_task;
  __shared__ T s_red[kBlock / 64];
  const DevProg p = make_prog(img, state);
  const int32_t n_tasks = p.h->n_tasks;
  const int tid = threadIdx.x;
  for (;;) {
    if (tid == 0) s_task = atomicAdd(&p.ctrl[0], 1);
    __syncthreads();
    const int32_t ti = s_task;
    __syncthreads();
    if (ti >= n_tasks) break;
    const TaskDesc td = p.tasks[ti];
    // ---- wait for inputs
    if (tid == 0) {
      for (int i = 0; i < td.n_deps; ++i) {
        const int32_t d = p.deps[td.dep_off + i];
        const int32_t target = p.tens[d].target;
        int32_t spins = 0;
        while (__hip_atomic_load(&p.ts[d].done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) <
               target) {
          __builtin_amdgcn_s_sleep(8);
          if (++spins > kSpinLimit) {
            __hip_atomic_store(&p.ctrl[1], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            break;
          }
        }
      }
    }
    __syncthreads();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    const KnotDesc kd = p.knots[td.knot];
    if (td.kind == TASK_SERIAL) {
      if (td.flags & TF_SETUP) {
        knot_setup<T>(p, kd, arena, J);
        __syncthreads();
      }
      for (int32_t si = td.first; si < td.first + td.count; ++si) {
        const StepDesc s = p.steps[si];
        int64_t ec;
        const T scale = step_scale<T>(p, s, ec);
        const int64_t outs = (int64_t)s.nb * s.nm * s.nn;
        T lm = step_outputs<T>(p, s, arena, 0, outs, scale);
        lm = block_max<T>(lm, s_red);
        if (tid == 0) {
          p.ts[s.c].shift = frexp_shift<T>(lm);
          p.ts[s.c].exp2 = ec;
        }
        __syncthreads();
      }
      if (td.flags & TF_FINAL) knot_final<T>(p, kd, arena, zout);
    } else {
      const StepDesc s = p.steps[td.first];
      int64_t ec;
      const T scale = step_scale<T>(p, s, ec);
      const int64_t outs = (int64_t)s.nb * s.nm * s.nn;
      const int64_t o0 = (int64_t)td.count * s.tile;
      const int64_t o1 = o0 + s.tile < outs ? o0 + s.tile : outs;
      T lm = step_outputs<T>(p, s, arena, o0, o1, scale);
      lm = block_max<T>(lm, s_red);
      if (tid == 0) {
        const int32_t sh = frexp_shift<T>(lm);
        if (sh != kShiftNone)
          __hip_atomic_fetch_max(&p.ts[s.c].shift, sh, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (td.count == 0) p.ts[s.c].exp2 = ec;
      }
    }
    // ---- publish
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    for (int i = tid; i < td.n_sig; i += kBlock)
      __hip_atomic_fetch_add(&p.ts[p.deps[td.sig_off + i]].done, 1, __ATOMIC_RELEASE,
                             __HIP_MEMORY_SCOPE_AGENT);
  }
}

// ------------------------------------------------------------------ host side

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

kn_status launch(const ImgHeader& h, uint8_t* ws, hipStream_t st, const double* J,
                 kn_scalar* z, int32_t grid_override) {
  uint8_t* state = ws + h.state_off;
  const int32_t n_clear = h.n_tensors > 64 ? h.n_tensors : 64;
  hipLaunchKernelGGL(clear_state, dim3((n_clear + 255) / 256), dim3(256), 0, st, state,
                     h.n_tensors, h.o_tstate);
  if (hipGetLastError() != hipSuccess) return KN_E_DEVICE;
  int32_t grid = grid_override > 0 ? grid_override : device_cus() * 4;
  if (grid > h.n_tasks) grid = h.n_tasks;
  if (grid < 1) grid = 1;
  if (h.precision == 1) {
    hipLaunchKernelGGL(engine<float>, dim3(grid), dim3(kBlock), 0, st, ws, state,
                       reinterpret_cast<Cx<float>*>(ws + h.arena_off), J, z);
  } else {
    hipLaunchKernelGGL(engine<double>, dim3(grid), dim3(kBlock), 0, st, ws, state,
                       reinterpret_cast<Cx<double>*>(ws + h.arena_off), J, z);
  }
  if (hipGetLastError() != hipSuccess) return KN_E_DEVICE;
  return KN_OK;
}

bool aligned256(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 255) == 0; }

}  // namespace
}  // namespace kn

using namespace kn;

extern "C" kn_status kn_contract(const kn_plan* p, const double* J, void* workspace,
                                 size_t workspace_bytes, void* stream, kn_scalar* z_dev) {
  if (!p || !workspace || !z_dev) return KN_E_INVALID;
  if (p->image.empty()) return KN_E_BUDGET;
  if (J && p->k.jones_only) return KN_E_UNSUPPORTED;
  if (!aligned256(workspace)) return KN_E_INVALID;
  const ImgHeader& h = *reinterpret_cast<const ImgHeader*>(p->image.data());
  if ((int64_t)workspace_bytes < h.workspace_bytes) return KN_E_BUDGET;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  if (hipMemcpyAsync(workspace, p->image.data(), (size_t)h.image_bytes, hipMemcpyHostToDevice, st) !=
      hipSuccess)
    return KN_E_DEVICE;
  return launch(h, reinterpret_cast<uint8_t*>(workspace), st, J, z_dev, 0);
}

extern "C" kn_status kn_batch_create(const kn_plan* const* plans, int32_t n, kn_batch** out) {
  if (!out) return KN_E_INVALID;
  *out = nullptr;
  if (!plans || n <= 0) return KN_E_INVALID;
  std::vector<const PlanKnot*> ks;
  bool jones_only = false;
  for (int32_t i = 0; i < n; ++i) {
    if (!plans[i] || plans[i]->image.empty()) return KN_E_INVALID;
    if (plans[i]->k.precision != plans[0]->k.precision) return KN_E_INVALID;
    jones_only |= plans[i]->k.jones_only;
    ks.push_back(&plans[i]->k);
  }
  kn_batch* b = new (std::nothrow) kn_batch();
  if (!b) return KN_E_NOMEM;
  try {
    b->image = build_image(ks);
    b->precision = plans[0]->k.precision;
    b->jones_only = jones_only;
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

extern "C" kn_status kn_batch_contract(const kn_batch* b, const double* J, void* workspace,
                                       size_t workspace_bytes, void* stream, kn_scalar* z_dev) {
  if (!b || !workspace || !z_dev) return KN_E_INVALID;
  if (J && b->jones_only) return KN_E_UNSUPPORTED;
  if (!aligned256(workspace)) return KN_E_INVALID;
  const ImgHeader& h = *reinterpret_cast<const ImgHeader*>(b->image.data());
  if ((int64_t)workspace_bytes < h.workspace_bytes) return KN_E_BUDGET;
  return launch(h, reinterpret_cast<uint8_t*>(workspace), reinterpret_cast<hipStream_t>(stream), J,
                z_dev, b->grid_override);
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

extern "C" void kn_batch_free(kn_batch* b) { delete b; }

extern "C" kn_status kn_backward_workspace(const kn_plan* p, uint64_t* bytes) {
  if (!p || !bytes) return KN_E_INVALID;
  return KN_E_UNSUPPORTED;
}

extern "C" kn_status kn_contract_backward(const kn_plan* p, const double* J, void* workspace,
                                          size_t workspace_bytes, void* stream, kn_scalar* z_dev,
                                          double* grad_dev) {
  (void)J; (void)workspace; (void)workspace_bytes; (void)stream; (void)z_dev; (void)grad_dev;
  if (!p) return KN_E_INVALID;
  return KN_E_UNSUPPORTED;
}
