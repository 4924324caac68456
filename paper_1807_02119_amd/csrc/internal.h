// internal.h -- host-side objects behind the opaque handles of kn.h.
#pragma once
#include <stdint.h>

#include <algorithm>
#include <complex>
#include <cstring>
#include <functional>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <utility>
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

// Allocator whose value-less construct leaves elements uninitialised, so that
// a buffer about to be overwritten in full is not zero-filled first.
template <class T>
struct DefaultInit : std::allocator<T> {
  template <class U>
  struct rebind {
    using other = DefaultInit<U>;
  };
  DefaultInit() = default;
  template <class U>
  DefaultInit(const DefaultInit<U>&) noexcept {}
  template <class U>
  void construct(U* p) noexcept {
    ::new (static_cast<void*>(p)) U;
  }
  template <class U, class... A>
  void construct(U* p, A&&... a) {
    ::new (static_cast<void*>(p)) U(std::forward<A>(a)...);
  }
};
using Bytes = std::vector<uint8_t, DefaultInit<uint8_t>>;

// A short list of spin ids.  Tensors of a plan have low rank, so up to kIn ids
// are stored inline and only longer lists go to the heap; this keeps the
// planner's thousands of small lists out of the allocator.
class SpinList {
 public:
  static constexpr int32_t kIn = 10;
  SpinList() = default;
  SpinList(const SpinList& o) { copy_from(o); }
  SpinList(SpinList&& o) noexcept { move_from(o); }
  SpinList& operator=(const SpinList& o) {
    if (this != &o) {
      n_ = 0;
      copy_from(o);
    }
    return *this;
  }
  SpinList& operator=(SpinList&& o) noexcept {
    if (this != &o) {
      release();
      move_from(o);
    }
    return *this;
  }
  ~SpinList() { release(); }
  int32_t size() const { return n_; }
  bool empty() const { return n_ == 0; }
  const int32_t* begin() const { return p_; }
  const int32_t* end() const { return p_ + n_; }
  int32_t operator[](int32_t i) const { return p_[i]; }
  void reserve(int32_t c) {
    if (c > cap_) grow(c);
  }
  void push_back(int32_t x) {
    if (n_ == cap_) grow(2 * cap_);
    p_[n_++] = x;
  }
  // in-place edits: entries [0, size) writable, shrink to the first k
  int32_t* mut() { return p_; }
  void truncate(int32_t k) {
    if (k < n_) n_ = k;
  }

 private:
  bool inline_() const { return p_ == in_; }
  void grow(int32_t c) {
    int32_t* np = new int32_t[c];
    std::memcpy(np, p_, sizeof(int32_t) * (size_t)n_);
    if (!inline_()) delete[] p_;
    p_ = np;
    cap_ = c;
  }
  void release() {
    if (!inline_()) delete[] p_;
    p_ = in_;
    cap_ = kIn;
    n_ = 0;
  }
  void copy_from(const SpinList& o) {
    reserve(o.n_);
    std::memcpy(p_, o.p_, sizeof(int32_t) * (size_t)o.n_);
    n_ = o.n_;
  }
  void move_from(SpinList& o) {
    n_ = o.n_;
    if (o.inline_()) {
      std::memcpy(in_, o.in_, sizeof(in_));
      p_ = in_;
      cap_ = kIn;
    } else {
      p_ = o.p_;
      cap_ = o.cap_;
    }
    o.p_ = o.in_;
    o.cap_ = kIn;
    o.n_ = 0;
  }
  int32_t* p_ = in_;
  int32_t n_ = 0;
  int32_t cap_ = kIn;
  int32_t in_[kIn];
};

// One knot's part of a device program with knot-local ids and offsets; an
// image is the concatenation of sections with the ids shifted (build_image).
// make_section fills a SectionBuild; the Section kept with the plan holds the
// same arrays in one allocation (a batch frees hundreds of plans at once).
struct SectionBuild {
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
  std::vector<int32_t> pins;        // (merged edge, sliced spin) pairs of the vertices
  std::vector<double> consts;       // complex constants (re, im), plan-local ids
  std::vector<TaskDesc> tasks;      // group, first, state_lo knot-local
  std::vector<GroupDesc> groups;    // first_task, next knot-local
  double est = 0;                   // estimated chain time (start priority)
  int32_t lds_used = 0;             // bytes of LDS arena the knot needs
  int64_t arena_elems = 0;
};

// A read-only array inside a Section's block.
template <class T>
struct SecArr {
  const T* p = nullptr;
  size_t n = 0;
  size_t size() const { return n; }
  bool empty() const { return n == 0; }
  const T* data() const { return p; }
  const T& operator[](size_t i) const { return p[i]; }
  const T* begin() const { return p; }
  const T* end() const { return p + n; }
};

struct Section {
  KnotDesc kd;
  SecArr<TensorDesc> td;
  SecArr<StepDesc> sd;
  SecArr<VtxDesc> vd;
  SecArr<int32_t> vslot;
  SecArr<MEdge> md;
  SecArr<int32_t> members;
  SecArr<Factor> fac;
  SecArr<int32_t> strides;
  SecArr<int32_t> comps;
  SecArr<int32_t> pins;
  SecArr<double> consts;
  SecArr<TaskDesc> tasks;
  SecArr<GroupDesc> groups;
  double est = 0;
  int32_t lds_used = 0;
  int64_t arena_elems = 0;
  std::unique_ptr<uint64_t[]> block;  // every array above, 8-byte aligned

  // Copy a built section into one block (replacing what was held).
  void assign(const SectionBuild& b);
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
  int32_t level = 0;    // serial steps: dependency level inside its run (from 1)
  // serial steps of a forked run: the concurrent task (0, 1, ...) whose
  // subtrees hold the step, or kForkTop for the steps above them; -1: the
  // run is not forked
  int32_t part = -1;
};

constexpr int32_t kForkTop = 1 << 30;

// One pairwise contraction C = A . B over spin groups.
struct PStep {
  int32_t a, b, c;
  SpinList bs, ms, ns, ks;  // batch, rows (A only), cols (B only), contracted
};

struct PTensor {
  SpinList spins;  // storage order, first = most significant
  int64_t off = 0;             // arena offset (entries), knot-local
  int64_t size = 1;            // q^rank
};

struct PVertex {
  int32_t tensor;
  int32_t center;               // spin of the vertex itself
  bool keep_center;
  bool seed = false;            // reverse-pass seed: the scalar 1, no spins
  int32_t adjoint = -1;         // gradient plans: tensor id of dS/dF_v
  int32_t comp = 0;             // gradient plans: component index
  SpinList nbr;                 // neighbour spins, slot order
  SpinList medge;               // merged edge per slot (knot-local)
  SpinList pin_medge, pin_slice;  // slices: edges to sliced spins (merged edge, sliced spin)
};

// Everything about one knot's contraction, in knot-local ids.
struct PlanKnot {
  int32_t q = 3;
  double t_re = 0, t_im = 0;
  int32_t precision = 0;
  bool jones_only = true;
  bool gradient = false;                        // reverse pass appended
  int32_t n_slice_spins = 0;                    // spins fixed by slicing
  int32_t n_slices = 1;                         // q^n_slice_spins slices
  int32_t slice_chains = 1;                     // slices run as this many chains
  int32_t n_edges = 0;                          // original Tait edges
  std::vector<int8_t> eps;                      // original Tait signs
  // merged edge m: original edges medge_mem[medge_off[m] .. medge_off[m + 1]),
  // or, when medge_const[m] >= 0, none: x_m is the constant consts[medge_const[m]]
  std::vector<int32_t> medge_off{0}, medge_mem, medge_const;
  std::vector<std::complex<double>> consts;     // derived edges, FAC_CONST factors
  std::vector<Factor> factors;                  // simplification factors
  int32_t n_iso = 0;                            // isolated spins
  std::vector<PTensor> tensors;                 // vertex tensors, then step outputs
  std::vector<PVertex> vtx;
  std::vector<PStep> steps;
  std::vector<int32_t> comps;                   // final scalar tensor per component
  int64_t arena_elems = 0;
  int32_t tile = 256;
  int32_t big_log2 = 16;
  int32_t big_outs_log2 = 12;
  int32_t lds_bytes = 32768;
  double split_est = 1024;                      // serial runs estimated at least this
                                                // long run level by level
  double fork_est = 1e30;                       // ... or at least this long: forked into
                                                // concurrent subtree tasks
  std::vector<PTiling> tiling;                  // per step: how it is executed
  Section sec;  // device-program section (make_section)

  // Once the section is made, images need only it, the Tait signs and the
  // slice counts: the planning structures are freed on the planning thread.
  void release_planning() {
    std::vector<PTensor>().swap(tensors);
    std::vector<PVertex>().swap(vtx);
    std::vector<PStep>().swap(steps);
    std::vector<PTiling>().swap(tiling);
    std::vector<int32_t>().swap(comps);
    std::vector<Factor>().swap(factors);
    std::vector<int32_t>().swap(medge_off);
    std::vector<int32_t>().swap(medge_mem);
    std::vector<int32_t>().swap(medge_const);
    std::vector<std::complex<double>>().swap(consts);
  }
};

// Adjacent steps i and i + 1 may run concurrently: both serial and of the
// same level of one task (runs of serial steps are separated by tiled steps,
// and levels ascend inside a task), or both in the concurrent tasks of a
// forked run (each of which runs on its own workgroup, all at once).
inline bool same_level(const PlanKnot& k, size_t i) {
  const PTiling& a = k.tiling[i];
  const PTiling& b = k.tiling[i + 1];
  if (a.mode != STEP_SERIAL || b.mode != STEP_SERIAL) return false;
  if (a.part >= 0 && a.part != kForkTop && b.part >= 0 && b.part != kForkTop) return true;
  return a.part == b.part && a.level == b.level;
}

// First-fit allocator over [0, cap) entries, sizes rounded up to `align`
// entries, free blocks kept in a sorted vector; alloc returns -1 when the
// request does not fit.
struct FitAlloc {
  struct Blk {
    int64_t off, len;
  };
  int64_t cap, align;
  int64_t top = 0;
  std::vector<Blk> free_blk;  // sorted by offset
  FitAlloc(int64_t c, int64_t a) : cap(c), align(a) {}
  int64_t round(int64_t len) const { return (len + align - 1) / align * align; }
  int64_t alloc(int64_t len) {
    len = round(len);
    for (size_t i = 0; i < free_blk.size(); ++i)
      if (free_blk[i].len >= len) {
        int64_t off = free_blk[i].off;
        free_blk[i].off += len;
        free_blk[i].len -= len;
        if (free_blk[i].len == 0) free_blk.erase(free_blk.begin() + i);
        return off;
      }
    if (!free_blk.empty() && free_blk.back().off + free_blk.back().len == top &&
        free_blk.back().off + len <= cap) {
      int64_t off = free_blk.back().off;
      free_blk.pop_back();
      top = off + len;
      return off;
    }
    if (top + len > cap) return -1;
    int64_t off = top;
    top += len;
    return off;
  }
  void release(int64_t off, int64_t len) {
    len = round(len);
    size_t i = (size_t)(std::lower_bound(free_blk.begin(), free_blk.end(), off,
                                         [](const Blk& b, int64_t o) { return b.off < o; }) -
                        free_blk.begin());
    free_blk.insert(free_blk.begin() + i, Blk{off, len});
    if (i + 1 < free_blk.size() && free_blk[i].off + free_blk[i].len == free_blk[i + 1].off) {
      free_blk[i].len += free_blk[i + 1].len;
      free_blk.erase(free_blk.begin() + i + 1);
    }
    if (i > 0 && free_blk[i - 1].off + free_blk[i - 1].len == free_blk[i].off) {
      free_blk[i - 1].len += free_blk[i].len;
      free_blk.erase(free_blk.begin() + i);
    }
  }
};

// Run f() on the calling thread and on up to n_threads - 1 threads of a
// persistent host pool, returning when every call has returned (f pulls work
// items itself, e.g. from an atomic counter).  Concurrent callers, and
// callers in a process forked after the pool started, get threads of their
// own for the call.
void parallel_run(int32_t n_threads, const std::function<void()>& f);
// f on up to n_threads threads of the pool (the caller's among them) when no
// other call holds it; otherwise false, with f not run (the caller runs it
// alone rather than adding threads to cores the other call keeps busy).
bool parallel_run_idle(int32_t n_threads, const std::function<void()>& f);

// CPUs this process may run on (its affinity mask), at least 1.
int32_t usable_cpus();

// Lay the knot's plan out as a relocatable device-program section.
void make_section(PlanKnot& k);

// Build the device image for a list of knots (a batch of one or more) by
// concatenating their sections.  out_slot of knot i is i.  With header_only
// the result is just the ImgHeader (every size and offset, nothing written).
// Empty when the arena does not fit int32 offsets.
Bytes build_image(const std::vector<const PlanKnot*>& knots, bool header_only = false);

// The same image written into a buffer that buffer(bytes) provides (the image
// is not zero-filled beyond what it writes: every array and all padding are
// written).  Returns the image size, -1 when the arena does not fit int32
// offsets, -2 when buffer returned null.  header (may be null) receives the
// header.  With a null buffer only the header is computed.
int64_t build_image_into(const std::vector<const PlanKnot*>& knots,
                         const std::function<uint8_t*(size_t)>& buffer, ImgHeader* header);

// Host buffers for batch images, page-locked when the HIP runtime can provide
// them (uploads are then plain DMA), kept in a pool for reuse.  host_buf_get
// returns at least `bytes` bytes and its capacity; host_buf_put takes it back.
uint8_t* host_buf_get(size_t bytes, size_t* capacity, bool* pinned);
void host_buf_put(uint8_t* p, size_t capacity, bool pinned);

// Move-only owner of a host_buf_get buffer.
class HostBuf {
 public:
  HostBuf() = default;
  HostBuf(const HostBuf&) = delete;
  HostBuf& operator=(const HostBuf&) = delete;
  HostBuf(HostBuf&& o) noexcept { swap(o); }
  HostBuf& operator=(HostBuf&& o) noexcept {
    if (this != &o) {
      reset();
      swap(o);
    }
    return *this;
  }
  ~HostBuf() { reset(); }
  // a buffer of `bytes` (nullptr when out of memory)
  uint8_t* allocate(size_t bytes) {
    reset();
    p_ = host_buf_get(bytes, &cap_, &pinned_);
    n_ = p_ ? bytes : 0;
    return p_;
  }
  void reset() {
    if (p_) host_buf_put(p_, cap_, pinned_);
    p_ = nullptr;
    n_ = cap_ = 0;
    pinned_ = false;
  }
  uint8_t* data() const { return p_; }
  size_t size() const { return n_; }
  bool empty() const { return n_ == 0; }

 private:
  void swap(HostBuf& o) {
    std::swap(p_, o.p_);
    std::swap(n_, o.n_);
    std::swap(cap_, o.cap_);
    std::swap(pinned_, o.pinned_);
  }
  uint8_t* p_ = nullptr;
  size_t n_ = 0, cap_ = 0;
  bool pinned_ = false;
};

int64_t elem_bytes(int32_t precision);

// Nested-dissection ranks of the n spins of a graph (compressed rows off, nb;
// symmetric, no self-loops): recursive vertex separators down to parts of at
// most `leaf` spins, `trials` search roots per split, roots after the first
// drawn from `seed`.  rank[v] = height of v's node in the hierarchy.
void separator_ranks(int32_t n, const std::vector<int32_t>& off, const std::vector<int32_t>& nb,
                     int32_t leaf, int32_t trials, uint64_t seed, std::vector<int32_t>& rank);

}  // namespace kn

struct kn_plan {
  kn::PlanKnot k;
  kn_plan_stats stats{};
  bool laid_out = false;  // the single-knot image fits (its header was built)
  uint64_t bwd_workspace = 0;
  // single-knot device image, built on first use (plans planned for a batch
  // never need it); guarded for concurrent users of one plan
  mutable std::mutex image_mu;
  mutable kn::Bytes image;
};

namespace kn {
// The plan's single-knot image (empty when it does not fit).
const Bytes& plan_image(const kn_plan* p);
}  // namespace kn

struct kn_batch {
  kn::HostBuf image;  // page-locked when possible: uploaded by DMA
  kn_batch_stats stats{};
  std::vector<int64_t> edge_offset;
  int32_t precision = 0;
  bool jones_only = false;
  bool gradient = false;  // every plan carries the reverse pass
  int32_t grid_override = 0;
  void* trace = nullptr;
  size_t trace_bytes = 0;
};
