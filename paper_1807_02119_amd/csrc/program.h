// program.h -- layout of the device program ("image") that the host planner
// writes and the persistent contraction kernel reads.
//
// An image describes the full contraction of one or more tensor networks G_T
// (one per knot, Sec. III of arXiv:1807.02119): the vertex tensors built from
// absorbed edge matrices, the pairwise contraction steps, and the tasks that
// perform them.  Tasks are organised in groups; the groups of one knot form a
// chain (group g+1 starts when every task of group g has finished).  A group
// is either one serial task (a run of small steps done by one workgroup, with
// the knot's setup and/or final reduction) or the tiles of one large step.
// Everything is plain old data addressed by byte offsets from the start of
// the image, so the image is copied to the device verbatim.
//
// Workspace layout (device): [ image | runtime state | tensor arena ], each
// part 256-byte aligned; offsets are recorded in the header.
#pragma once
#include <stdint.h>

namespace kn {

constexpr int32_t kMagic = 0x4b4e4732;  // "KNG2"
constexpr int32_t kBlock = 256;         // threads per workgroup of the engine
// Fixed LDS areas of a workgroup (the tensor arena follows them):
constexpr int32_t kTabBuf = 3072;   // gather-table entries generated per chunk of serial steps
constexpr int32_t kDescBuf = 64;    // step descriptors staged per chunk
constexpr int32_t kStateCap = 768;  // tensor states cached for the running serial task

enum TaskKind : int32_t {
  // One workgroup runs, in order: the knot's setup (edge weights + vertex
  // tensors) if flags & TF_SETUP, steps [first, first+count) entirely, and
  // the knot's final reduction to Z if flags & TF_FINAL.
  TASK_SERIAL = 0,
  // Tile `count` of step `first` (see StepDesc.mode).
  TASK_TILE = 1,
  // Sum the n_ks partial results of split step `first` into outputs
  // [count * kReduceChunk, (count + 1) * kReduceChunk) of its output.
  TASK_REDUCE = 2,
};

enum StepMode : int32_t {
  STEP_SERIAL = 0,  // done inside a serial task
  STEP_TILES = 1,   // tiles of `tile` consecutive outputs (all L lanes per output)
  STEP_GEMM = 2,    // 32 x 32 output blocks per batch index, LDS-staged, 2x2 per thread
  STEP_GEMM64 = 3,  // 64 x 64 output blocks, LDS-staged, 4x4 per thread
};
constexpr int32_t kGemmBlock = 32;  // rows and columns of a STEP_GEMM tile
constexpr int32_t kGemmChunk = 16;  // contracted entries staged per LDS round
constexpr int32_t kReduceChunk = 8192;  // outputs per task of a split step's reduction

enum TaskFlags : int32_t { TF_SETUP = 1, TF_FINAL = 2 };

enum FactorKind : int32_t {
  FAC_LOOP = 0,  // loop edge e: factor x_e (original edge id)
  FAC_LEAF = 1,  // degree-1 vertex on merged edge m: factor x_m + q - 1
  FAC_PAIR = 2,  // merged edge m between sliced spins a and b: x_m if their
                 // fixed values are equal, else 1
  FAC_CONST = 3,  // constant id of the plan (series reduction at known couplings)
};

struct ImgHeader {
  int32_t magic;
  int32_t precision;  // 0 complex128, 1 complex64
  int32_t n_tasks, n_knots, n_tensors, n_steps;
  int32_t n_vtx, n_medges, n_members, n_factors;
  int32_t n_strides, n_groups;
  int32_t n_edges;    // original edges over all knots (couplings J, gradients)
  int32_t n_roots;    // first groups of the knots, in start-priority order
  int32_t lds_bytes;  // per-workgroup LDS arena for serial tasks (bytes)
  int32_t n_pins;
  int32_t n_wslots;   // complex weight slots over all knots (x_e then x_m per knot)
  int32_t n_outputs;  // entries of the output scalar array
  int32_t sliced;     // 1: some knots are slices; their sums are formed after the launch
  int32_t n_consts;   // complex128 constants over all plans
  int32_t n_queue;    // task executions (queue slots): a sliced unit runs its tasks
                      // once per slice of its chain
  int32_t n_zslice;   // slice results over all sliced plans
  int64_t o_tasks, o_groups, o_roots, o_knots, o_tensors, o_steps, o_vtx, o_vslot;
  int64_t o_medges, o_members, o_factors, o_strides, o_eps, o_comps, o_pins, o_consts;
  int64_t image_bytes;
  // runtime state (relative to the workspace base)
  int64_t state_off, state_bytes;
  int64_t o_queue;    // int32[n_queue] ready queue (-1 = slot not yet written)
  int64_t o_pending;  // int32[n_groups] unfinished predecessor tasks
  int64_t o_tstate;   // TensorState[n_tensors]
  int64_t o_weights;  // complex128 x_e per original edge, then x_m per merged edge
  int64_t o_mgrad;    // complex128 d log Z / d J per merged edge (gradient plans)
  int64_t o_zslice;   // kn_scalar per slice of every sliced plan
  int64_t o_uslice;   // int32 per knot descriptor: the slice it is running
  // tensor arena (relative to the workspace base), in complex entries
  int64_t arena_off, arena_elems;
  int64_t workspace_bytes;
  int64_t guard_off;  // guard zone after the arena (relative to the workspace base)
};

struct TaskDesc {
  int32_t kind, knot, group;
  int32_t first, count;
  int32_t flags;
  // serial tasks: tensor ids [state_lo, state_lo + state_len) are produced by
  // this task (its vertex tensors and step outputs, consecutive ids); their
  // states are kept in LDS while it runs
  int32_t state_lo, state_len;
};

struct GroupDesc {
  int32_t knot;
  int32_t first_task, n_tasks;
  int32_t next;    // next group of the same knot, -1 for the last
  int32_t n_pred;  // tasks of the previous group (0 for a knot's first group)
};

struct KnotDesc {
  double t_re, t_im;        // Jones variable t(q) (Eq. 1)
  int32_t q;
  int32_t edge_off, n_edges;      // original edges (global index range)
  int32_t medge_off, n_medges;    // merged edges
  int32_t vtx_off, n_vtx;         // vertex tensors
  int32_t factor_off, n_factors;  // simplification factors
  int32_t comp_off, n_comps;      // final (scalar) tensor of each component
  int32_t n_iso;                  // isolated vertices: factor q each
  int32_t out_slot;               // index into the kn_scalar output array
  int32_t step_off, n_steps;
  int32_t grad;  // 1: the steps include the reverse pass; the final task
                 // writes d log Z / d J_e for every original edge
  // Slicing: the network of one plan with n_slice_spins spins fixed.  This
  // descriptor is one chain of slice_step chains: it runs slices slice,
  // slice + slice_step, ... < n_slices one after another (the slice running
  // now is in the runtime state; digit j of a slice number in base q is the
  // value of sliced spin j).  Slice s writes its Z to entry out_slot + s of
  // the slice array, and the sum over slices goes to output plan_slot.
  // n_slices == 1: not sliced (out_slot indexes the outputs).
  int32_t slice, n_slices, n_slice_spins, plan_slot, slice_step;
  // this descriptor's groups and tensors (reset between its slices)
  int32_t group_off, n_groups, tensor_off, n_tensors;
  int32_t w_off;  // this knot's weight slots: x_e at w_off, x_m at w_off + n_edges
  int32_t const_off;  // this plan's constants (derived merged edges, FAC_CONST)
  int32_t pad;        // explicit: no implicit padding, so images are byte-reproducible
};

static_assert(sizeof(KnotDesc) == 16 + 28 * 4, "KnotDesc has no implicit padding");

struct TensorDesc {
  int64_t off;      // complex entries from the arena base (global home)
  int32_t size;     // entries
  int32_t lds_off;  // complex entries into the workgroup's LDS arena; -1 = global
};

// A pairwise step C[b,m,n] = sum_k A[b,m,k] B[b,k,n].  Each of the four spin
// groups (batch b, rows m, contracted k, columns n) is a list of spins, most
// significant first; an operand entry's offset is the sum over the group's
// spins of (digit of the group index) x (element stride of that spin in the
// operand's storage order).  The strides are stored, the offset tables are
// generated on the device.
struct StepDesc {
  int32_t a, b, c;          // tensor ids: C = A . B
  int32_t nb, nm, nn, nk;   // batch, rows, cols, contracted extents (powers of q)
  int32_t str;              // strides: A_b[rb] A_m[rm] A_k[rk] B_b[rb] B_k[rk] B_n[rn]
  int32_t ranks;            // rb | rm << 8 | rk << 16 | rn << 24
  int32_t n_tiles;          // 0 for steps run inside a serial task
  int32_t tile;             // STEP_TILES: outputs per tile; STEP_GEMM: blocks per task
  // where A, B, C live: >= 0 global arena offset (complex entries),
  // < 0 LDS arena offset -1 - value (serial steps only)
  int32_t home_a, home_b, home_c;
  int32_t mode;             // StepMode
  int32_t n_mb, n_nb;       // STEP_GEMM: row and column blocks
  int32_t n_ks, kseg;       // contracted-index splits and entries per split
  int32_t partial;          // n_ks > 1: arena offset of the partial sums [ks][output]
  // serial steps: dependency level inside the task's run of steps; adjacent
  // steps of equal level are independent and run concurrently
  int32_t lvl;
};

struct VtxDesc {
  int32_t tensor;      // tensor id
  int32_t n_slots;     // neighbour spins (absorbed edges)
  int32_t slot_off;    // merged-edge id (knot-local) per neighbour slot
  int32_t keep_center; // 1: the vertex's own spin is the leading index;
                       // 0: it is private to this tensor and summed at build;
                       // -1: not a vertex but a reverse-pass seed, the scalar 1
  int32_t adjoint;     // gradient plans: tensor id of dS/dF_v (-1: none)
  int32_t comp;        // gradient plans: index of the vertex's component
  int32_t adj_str;     // gradient plans: offset into the stride table of the
                       // element strides, in the adjoint's storage, of the
                       // kept centre (if any) and then of each slot's spin
  int32_t pin_off, n_pins;  // slices: pins (merged edge, sliced spin) of the
                            // vertex's own spin, a factor x_m where it equals
                            // the sliced spin's value
};

struct MEdge {
  // original edge ids (knot-local); n_members == -1: a derived edge whose x
  // is the plan's constant member_off (series-parallel reduction)
  int32_t member_off, n_members;
};

struct Factor {
  int32_t kind, id;
  int32_t a, b;  // FAC_PAIR: the two sliced spins (indices into the slice digits)
};

// Per-tensor runtime state.
struct TensorState {
  int32_t shift;  // frexp exponent of max(|re|,|im|) over the raw entries
                  // (kShiftNone until written / for an all-zero tensor)
  int32_t pad;
  int64_t exp2;   // true tensor = raw * 2^exp2
};

// Optional per-task trace record (device clock ticks, 100 MHz).
struct TraceRec {
  int64_t t_claim;  // slot claimed
  int64_t t_start;  // task available, execution starts
  int64_t t_end;    // execution finished
  int32_t task;
  int32_t wg;
  // serial tasks: time in setup, in staging descriptors and generating
  // tables, in the step products, in reductions and barriers; tile tasks:
  // from the start to the end of tables and operand states (descriptor loads
  // included), the products, the publish of C's shift (0 for reduce tasks)
  int64_t ph[4];
};

constexpr int32_t kShiftNone = (-2147483647 - 1);

// Byte offsets of the LDS areas; the tensor arena starts at kLdsArena.
constexpr int32_t kLdsTab = 0;
constexpr int32_t kLdsDesc = kLdsTab + kTabBuf * 4;
constexpr int32_t kLdsShift = kLdsDesc + kDescBuf * (int32_t)sizeof(StepDesc);
constexpr int32_t kLdsExp = (kLdsShift + kStateCap * 4 + 7) / 8 * 8;
constexpr int32_t kLdsExt = (kLdsExp + kStateCap * 8 + 15) / 16 * 16;  // operand states
constexpr int32_t kLdsArena = kLdsExt + 2 * kDescBuf * (int32_t)sizeof(TensorState);
// Dynamic LDS the engine may use, and the staging area after the tensor arena
// (lds_bytes of it): global operands of a serial step that the whole
// workgroup computes are copied there when they fit, so that the step's
// gathers read LDS.  Up to kStageMax bytes, within kLdsLimit (the 160 KiB
// of a CU less 2 KiB for the engine's static shared variables).
constexpr int32_t kLdsLimit = 160 * 1024 - 2048;
constexpr int32_t kStageMax = 64 * 1024;
constexpr int32_t stage_bytes(int32_t lds_bytes) {
  return kLdsLimit - kLdsArena - lds_bytes >= kStageMax
             ? kStageMax
             : (kLdsLimit - kLdsArena - lds_bytes > 0 ? (kLdsLimit - kLdsArena - lds_bytes) / 256 * 256
                                                      : 0);
}

// control words at the start of the runtime state
// (CTRL_ERROR: first error code, CTRL_ERR_*: the task, step and detail of it)
enum Ctrl : int32_t {
  CTRL_HEAD = 0,
  CTRL_TAIL = 1,
  CTRL_ERROR = 2,
  CTRL_ERR_TASK = 3,
  CTRL_ERR_STEP = 4,
  CTRL_ERR_INFO = 5,
  CTRL_WORDS = 64
};

inline int64_t align256(int64_t x) { return (x + 255) & ~int64_t(255); }

}  // namespace kn
