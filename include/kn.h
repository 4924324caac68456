/*
 * kn.h -- C ABI of libkn: exact evaluation of the Jones polynomial V_K(t(q))
 * by contracting the tensor network of the q-state Potts model with
 * anisotropic complex interactions (PACI) on the signed Tait graph of a knot
 * diagram (Meichanetzidis & Kourtis, arXiv:1807.02119).
 *
 * Pipeline and where each call sits in the paper:
 *   kn_build_tait      diagram -> bicoloured regions -> signed Tait graph G,
 *                      writhe w, Tait number tau                    (Sec. II)
 *   kn_plan_create     Reidemeister-I/II simplification (Sec. III.A), the
 *                      tensor network G_T with the q x q interaction matrices
 *                      absorbed into the vertex COPY tensors (Sec. III, Eq. 5),
 *                      and a greedy pairwise contraction order (Sec. III)
 *   kn_contract        full contraction of G_T on the GPU -> Z(q)
 *                      (Eqs. 2-3, Eq. 6)
 *   kn_contract_backward  d log Z / d J_e for every edge coupling
 *   kn_jones           V = A(q) Z (Eq. 4)
 *   kn_batch_*         many knots (and q values) in one persistent launch
 *
 * Conventions shared by every call:
 *   - Status codes: every call returns kn_status; nothing aborts or throws.
 *     Validation failures return KN_E_INVALID and leave *out == NULL.
 *   - Input arrays are borrowed for the duration of the call only.
 *   - Handles (kn_tait, kn_plan, kn_batch) are host objects owned by the
 *     caller and released with their *_free; *_free(NULL) is a no-op.
 *     Plans and batches are immutable after creation and may be shared by
 *     threads and streams.
 *   - Device buffers (workspace, couplings, outputs) are caller-owned device
 *     memory on the current HIP device; "stream" is a hipStream_t passed as
 *     void* (NULL = the null stream).  Device calls are asynchronous on that
 *     stream; HIP launch/copy failures return KN_E_DEVICE.
 *   - Complex numbers are interleaved (re, im) doubles.
 *   - q must be in [2, 8]; other values return KN_E_UNSUPPORTED.
 */
#ifndef KN_H
#define KN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  KN_OK = 0,
  KN_E_INVALID = -1,     /* malformed argument or diagram */
  KN_E_NOMEM = -2,       /* host allocation failed */
  KN_E_BUDGET = -3,      /* plan exceeds the memory budget / workspace too small */
  KN_E_DEVICE = -4,      /* HIP runtime error */
  KN_E_NUMERIC = -5,     /* non-finite input or result */
  KN_E_UNSUPPORTED = -6  /* q out of range, or plan/call combination not supported */
} kn_status;

typedef struct kn_tait kn_tait;
typedef struct kn_plan kn_plan;
typedef struct kn_batch kn_batch;

/* A complex number with a separate power-of-two exponent:
   value = (re + i*im) * 2^exp2.  Results are normalised so that
   max(|re|, |im|) lies in [0.5, 1) unless the value is zero. */
typedef struct {
  double re, im;
  int64_t exp2;
} kn_scalar;

/* ------------------------------------------------------------------ Sec. II
 * kn_build_tait: signed Tait graph of a knot diagram given as a PD code.
 *   n      number of crossings (n == 0: the crossingless unknot).
 *   pd     int32[4n]; pd[4i..4i+3] = (a, b, c, d): the arcs at crossing i
 *          counter-clockwise from the incoming under-arc a.  Arcs are labelled
 *          0..2n-1 consecutively along the orientation (arc k runs from the
 *          k-th to the (k+1)-th crossing visit), so c == a+1 (mod 2n), and the
 *          over-strand satisfies b == d+1 (positive crossing) or d == b+1
 *          (negative crossing).
 *   signs  int8[n] twist signs (+1 right-handed) or NULL to read them from
 *          the labels; required when n == 1 (the labels are ambiguous).
 *   outer_arc, outer_side
 *          the region taken as unbounded (coloured white, Sec. II): the region
 *          on the left (outer_side 0) or right (1) of arc outer_arc where it
 *          leaves its crossing.  outer_arc < 0 selects arc 0, left.  Either
 *          choice gives the same V (the two Tait graphs are planar duals).
 * Errors: KN_E_INVALID for labels out of range / not used exactly twice,
 * labels inconsistent with one oriented closed curve, or a non-planar code
 * (region count != n + 2).
 */
kn_status kn_build_tait(int32_t n, const int32_t* pd, const int8_t* signs,
                        int32_t outer_arc, int32_t outer_side, kn_tait** out);
/* n_vertices = black regions (n_v), n_edges = crossings, writhe w = sum of
   twist signs, tait_number tau = sum of Tait signs (Sec. II).  Any pointer may
   be NULL. */
kn_status kn_tait_info(const kn_tait* g, int32_t* n_vertices, int32_t* n_edges,
                       int32_t* writhe, int32_t* tait_number);
/* Edge k is crossing k: uv[2k], uv[2k+1] are its black regions (equal for a
   loop), eps[k] its Tait sign.  uv: int32[2*n_edges], eps: int8[n_edges]. */
kn_status kn_tait_edges(const kn_tait* g, int32_t* uv, int8_t* eps);
void kn_tait_free(kn_tait* g);

/* ------------------------------------------------------------------ Sec. III
 * Planning: simplification, absorption, contraction order, memory layout.
 *
 * strategy   0: greedy pairwise order minimising size(C) - size(A) - size(B)
 *               over tensors indexed by spins;
 *            1: greedy by the rank of the result (the paper's "cheapest
 *               contraction in terms of the resulting degree");
 *            2: variable elimination in min-fill order, each spin's holders
 *               contracted pairwise, smallest first;
 *            3: auto (default) -- plan 2; when it has at least 1e8 flops
 *               plan 0 is built too, when it has at least 1e11 flops the
 *               plans of strategy 4 too, and the one with the smallest
 *               modelled time (per step max(flops/peak, bytes/HBM
 *               bandwidth) plus a fixed per-step latency) is kept;
 *            4: separator hierarchy (the paper's METIS alternative to the
 *               greedy order): the spin graph is split recursively by small
 *               vertex separators into parts of comparable size, and spins
 *               are eliminated part by part, a separator after the parts it
 *               splits (least fill first among spins of one level).
 *               order_trials hierarchies (seeds, leaf sizes 8, 24, 64 in
 *               turn; 0 = default 12) are built and the plan with the
 *               smallest modelled time is kept;
 * precision  0: complex128 (FP64) tensors; 1: complex64 (FP32) tensors with
 *               FP32 accumulation, exponents and normalisation kept in
 *               int64 / FP64.
 * simplify   bit 0: Reidemeister I (loops and degree-1 vertices);
 *            bit 1: Reidemeister II (parallel edges of opposite Tait sign;
 *                   only valid for the Jones couplings);
 *            bit 2: exact series-parallel reduction at the Jones couplings
 *                   (their values are known when planning): a degree-2 spin
 *                   between edges x1, x2 is summed out into one edge
 *                   x' = (x1 x2 + q - 1) / (x1 + x2 + q - 2) times the
 *                   constant x1 + x2 + q - 2, spikes give x + q - 1, and
 *                   new parallel edges multiply, until every spin left has
 *                   degree three or more.  It removes about a fifth of the
 *                   spins of lattice knots, but the contraction order found
 *                   on the reduced graph is better for some knots and worse
 *                   for others (on a 256-knot q = 3 batch the total work
 *                   grew by a third), so it is not in the default.
 *            Parallel edges are always merged into one q x q matrix
 *            (elementwise product).  Default (opts == NULL): 3.
 * jones_only 1: the plan may only be contracted with the Jones couplings
 *               (J == NULL); required for simplify bits 1 and 2.  0: any
 *               couplings.
 * mem_budget_bytes  0 = no limit; otherwise a plan whose workspace exceeds it
 *               returns KN_E_BUDGET (and still fills *out so that its
 *               statistics can be read, see kn_plan_info).
 * tile_outputs      outputs per tile for steps split across workgroups
 *               (0 = default); big_step_macs_log2: log2 of the complex
 *               multiply-adds above which a step is split into tiles
 *               (0 = default 16); tile_macs_log2: log2 of the multiply-adds a
 *               tile of outputs aims at when tile_outputs is 0 (0 = default
 *               15).  These are the knobs the autotuner searches.
 * slice_log2_budget  0: no slicing.  Otherwise spins are fixed one at a time
 *               (each time the spin held by most of the plan's largest
 *               tensors) until the largest tensor has at most 2^budget
 *               entries, 24 spins are fixed or one more would exceed 2^24
 *               slices.  The plan then covers q^k
 *               slices, each the same network with those spins at fixed
 *               values: an edge to a fixed spin becomes a diagonal factor on
 *               its other end, an edge between two fixed spins a constant, and
 *               Z is the sum of the slices' values (formed on the device).
 *               Slices run as chains (at most 64, as many as mem_budget_bytes,
 *               default 16 GiB of arena, allows): one copy of the knot's
 *               device program per chain, whose final task starts the chain's
 *               next slice on the device.  Not combinable with gradient.
 * split_serial_log2  a run of small steps whose estimated time (one unit
 *               per step plus one per 512 multiply-adds) is at least
 *               2^split_serial_log2 is not executed by one workgroup but level
 *               by level: the independent steps of each dependency level are
 *               shared out to several workgroups, the levels one after
 *               another (with vertex-tensor setup and the final product as
 *               tasks of their own).  This shortens the longest knots' chains
 *               at the price of more tasks.  0 = default 40 (never).
 * gemm_tasks_log2  a step computed in output blocks over workgroups with
 *               more than 2^gemm_tasks_log2 blocks gives each task several
 *               blocks (at most 32 of 32 x 32 or 8 of 64 x 64), which saves
 *               per-task scheduling work.
 *               0 = default 5; 30 = one block per task.
 * gemm64_pct    a step computed in blocks uses 64 x 64 blocks instead of
 *               32 x 32 when both its output sides are at least 64 and the
 *               64-blocks' padded output count is at most gemm64_pct percent
 *               of the 32-blocks' (0 = default 300; 1 = never).  A 64-block
 *               does four times the multiply-adds per staged chunk, which
 *               hides the operand loads better, and needs 2 x 16 x 65 entries
 *               of LDS (33 KiB in complex128; the launch grows to fit).
 * big_step_outs_log2  a step with at least 2^big_step_outs_log2 outputs is
 *               split into tiles over workgroups too, whatever its
 *               multiply-add count: with a short contracted index its time on
 *               one workgroup is set by rounds of gathered loads, one round
 *               per 512 outputs (0 = default 12; 31 = by multiply-adds only).
 * tile_outs_log2  most outputs one tile of a tiled step computes, 2^value
 *               (0 = default 10).
 * bucket        per intermediate-size bucket overrides of the tile shape: a
 *               step whose output C has at most 2^8, 2^12, 2^16, 2^20 or more
 *               entries takes bucket 0, 1, 2, 3 or 4, and any non-zero field
 *               of that bucket replaces the plan-wide value (tile_macs_log2,
 *               tile_outs_log2, gemm64_pct, gemm_tasks_log2).  The autotuner
 *               searches them per workload.
 * order_trials  separator hierarchies tried by strategies 3 and 4 (0 =
 *               default 12, at most 4096).
 * fork_serial_log2  a run of small steps whose estimated time (as for
 *               split_serial_log2) is at least 2^fork_serial_log2 is forked:
 *               its steps form a forest (every intermediate is read once), so
 *               its heaviest subtrees are split at their roots until each
 *               weighs at most 1/8 of the run, and the subtrees run as up to 8
 *               concurrent tasks on their own workgroups, between a task for
 *               the knot's vertex tensors (if the run starts the knot) and
 *               one for the steps above them.  Not applied to gradient plans
 *               (their tensors are read twice).  0 = default 10; 40 = never.
 * split_min_log2  a step split into tiles over workgroups whose tiles are
 *               few (fewer than 256) while its contracted index is long has
 *               that index split as well: each split computes partial sums
 *               over one segment and a reduce task adds them in split order.
 *               An index of nk entries has at most nk / 2^split_min_log2
 *               segments, rounded up (and at most 256), of equal length.
 *               Every task costs a few microseconds
 *               of claiming, descriptor loads and release whatever its size,
 *               so short segments make many tasks that each do little.
 *               0 = default 12.
 * paper_stats   1: also compute delta_h_paper (costs about as much as the
 *               plan itself); 0: delta_h_paper = -1.
 * lds_bytes     per-workgroup LDS for tensors that live inside one serial task
 *               (0 = default 24 KiB, at most 128 KiB: with the engine's own
 *               28 KiB of tables and descriptors one workgroup then fills a
 *               compute unit's 160 KiB).  All plans of a batch are launched
 *               with the largest value any of them uses.
 * gradient      1: the plan also carries the reverse pass of the contraction
 *               (for kn_contract_backward): after the forward steps, the
 *               adjoint of every intermediate is contracted back to the vertex
 *               tensors (for C = A.B: dS/dA = dS/dC . B, dS/dB = A . dS/dC),
 *               and every intermediate is kept until its reverse step.  With
 *               mem_budget_bytes set, forward intermediates from the largest
 *               rank down are dropped after their forward use and computed
 *               again from their operands just before the reverse step that
 *               needs them, in chains of at most 1, 2, 4 or 8 such steps
 *               (shallow first), until the plan's arena fits the budget
 *               (stats: n_recompute_steps; the flops include the recompute).
 *               Requires simplify without bits 1 and 2 (they drop edges
 *               whose derivative is not zero).  kn_contract on such a plan
 *               computes Z and runs the reverse steps without writing them out.
 */
#define KN_N_BUCKETS 5
typedef struct {
  int32_t tile_macs_log2;
  int32_t tile_outs_log2;
  int32_t gemm64_pct;
  int32_t gemm_tasks_log2;
} kn_bucket_opts;
typedef struct {
  int32_t strategy;
  int32_t precision;
  int32_t simplify;
  int32_t jones_only;
  uint64_t mem_budget_bytes;
  int32_t tile_outputs;
  int32_t big_step_macs_log2;
  int32_t paper_stats;
  int32_t lds_bytes;
  int32_t gradient;
  int32_t tile_macs_log2;
  int32_t slice_log2_budget;
  int32_t split_serial_log2;
  int32_t gemm_tasks_log2;
  int32_t gemm64_pct;
  int32_t big_step_outs_log2;
  int32_t tile_outs_log2;
  kn_bucket_opts bucket[KN_N_BUCKETS];
  int32_t order_trials;
  int32_t fork_serial_log2;
  int32_t split_min_log2;
} kn_plan_opts;

/* Statistics of a plan (algorithmic, from the plan itself).
 *   n_steps            pairwise contractions
 *   n_vertex_tensors   tensors built from absorbed edge matrices
 *   log2_max_entries   log2 of the largest tensor (entries)
 *   flops              8 * sum over steps of |batch|*|M|*|N|*|K| (complex MAC = 8)
 *   bytes              sum over steps of s*(|A| + |B| + |C|), s = 16 (c128) or 8 (c64)
 *   workspace_bytes    device workspace kn_contract needs
 *   delta_h_paper      max vertex degree over the graph minors of the paper's
 *                      edge-contraction greedy on the simplified graph (Sec. III)
 *   n_edges_simplified edges left after simplification and merging
 *   n_vertices_simplified */
typedef struct {
  int32_t n_steps;
  int32_t n_vertex_tensors;
  double log2_max_entries;
  double flops;
  double bytes;
  uint64_t workspace_bytes;
  uint64_t image_bytes;
  int32_t delta_h_paper;
  int32_t n_edges_simplified;
  int32_t n_vertices_simplified;
  int32_t n_tasks;
  int32_t n_components;
  int32_t max_rank;
  int32_t n_slices;       /* q^(fixed spins); flops and bytes cover all slices */
  int32_t slice_chains;   /* slices run as this many concurrent chains */
  int32_t n_recompute_steps; /* gradient plans: forward steps run again in the reverse
                                pass for tensors dropped to fit mem_budget_bytes */
} kn_plan_stats;

/* Build a plan for q.  opts == NULL selects the defaults above (Jones-only,
   full simplification, complex128, auto order). */
kn_status kn_plan_create(const kn_tait* g, int32_t q, const kn_plan_opts* opts, kn_plan** out);
kn_status kn_plan_info(const kn_plan* p, kn_plan_stats* out);
void kn_plan_free(kn_plan* p);
/* Read-only view of the plan's device image (the bytes kn_contract copies to
   the device; layout private to this library version), for inspection tools
   and tests.  *data stays valid until kn_plan_free. */
kn_status kn_plan_image(const kn_plan* p, const void** data, size_t* bytes);
/* The plan's contraction order, for inspection: step k contracts tensors
   ab[2k], ab[2k+1] (ids: 0..n_vertex_tensors-1 are vertex tensors, id
   n_vertex_tensors + k is the result of step k).  ab: int32[2*n_steps]. */
kn_status kn_plan_steps(const kn_plan* p, int32_t* ab);

/* ------------------------------------------------------------------ Eqs. 2-3, 6
 * kn_contract: Z(q) of the plan's knot, computed on the GPU.
 *   J          device array of 2*n_edges doubles: complex coupling J_e for every
 *              ORIGINAL Tait edge (edge order of kn_tait_edges), interaction
 *              matrix T_e = 1 + (exp(J_e) - 1) * delta.  NULL = the Jones
 *              couplings exp(J_e) = -t(q)^(-eps_e) (Sec. II).  Non-NULL with a
 *              jones_only plan returns KN_E_UNSUPPORTED.
 *   workspace  device memory of at least plan workspace_bytes, 256-byte
 *              aligned; its contents on entry do not matter and are
 *              overwritten (the plan's device image is copied into it).
 *   z_dev      device pointer to one kn_scalar receiving Z.  On an internal
 *              device error Z is written as NaN.
 * The call enqueues a host-to-device copy of the plan image, one clear kernel
 * and one persistent contraction kernel on `stream` and returns. */
kn_status kn_contract(const kn_plan* p, const double* J, void* workspace,
                      size_t workspace_bytes, void* stream, kn_scalar* z_dev);

/* kn_contract without a workspace argument and without any device allocation,
 * for callers that cannot allocate device memory (code under stream capture,
 * tight serving loops, harnesses that forbid hipMalloc).  The workspace is a
 * library-owned array of KN_NOALLOC_MAX_BYTES in device memory, one per
 * device, held until the process ends; the call uploads the plan's image
 * there and launches the same kernels as kn_contract (same results, bit for
 * bit).  Every call on one device shares that device's array and leaves its
 * contents behind (the kernels reset the state they need), so calls that
 * overlap on one device -- on different streams, or from different host
 * threads without ordering -- race and give undefined results.
 *   J, stream, z_dev  as in kn_contract.
 * Errors: KN_E_BUDGET when the plan's workspace_bytes exceeds
 * KN_NOALLOC_MAX_BYTES (or the plan has no image); KN_E_DEVICE when the
 * array's device address cannot be obtained. */
#define KN_NOALLOC_MAX_BYTES ((size_t)64 << 20)
kn_status kn_contract_noalloc(const kn_plan* p, const double* J, void* stream, kn_scalar* z_dev);

/* ------------------------------------------------------------------ checking
 * Error state of the last launch in a workspace (of a plan or a batch):
 * status[0] the first error code, status[1] the task, status[2] the step,
 * status[3] a detail (-1 where it does not apply).  Codes:
 *   0 none
 *   1 a ready-queue slot stayed empty past the engine's time limit (20 s):
 *     the launch gave up, unfinished knots read NaN
 *   checking build only (kn_device_checks() == 1), the task was skipped:
 *   2 a task record out of range (kind, knot, group, steps, tile id)
 *   3 a tensor outside the global or the LDS arena
 *   4 spin-group extents disagree with their ranks or outputs with C's size
 *   5 the largest offset a gather can form leaves its operand
 *   6 a serial step's gather tables exceed the LDS table buffer
 *   7 the guard zone after the arena (the last 4 KiB of every workspace) was
 *     overwritten; status[3] is the first word found changed
 * The call waits for `stream` and copies the error words to the host
 * (synchronous).  workspace: the device workspace of a finished launch. */
kn_status kn_workspace_status(const void* workspace, void* stream, int32_t* status);
/* 1 when this library is the checking build (every task checked on the device
 * before it runs, the guard zone checked after each launch), else 0. */
int32_t kn_device_checks(void);
/* The same checks on the host over a device image (kn_plan_image or
 * kn_batch_image bytes, 8-byte aligned): every section inside the image and
 * every task and step consistent.  status as in kn_workspace_status (0 = the
 * image passes).  KN_E_INVALID when the header itself is unusable. */
kn_status kn_image_check(const void* image, size_t bytes, int32_t* status);

/* d log Z / d J_e (holomorphic derivative, dT_e/dJ_e = e^{J_e} delta) for
 * every ORIGINAL edge, written to grad_dev (device, 2*n_edges doubles, re/im
 * interleaved, edge order of kn_tait_edges).  One launch runs the forward
 * sweep and the reverse sweep (nothing from a previous kn_contract is
 * needed); z_dev receives Z as in kn_contract.  Edges removed by
 * simplification get their closed forms: a loop 1, an edge of a merged spike
 * m: x_m / (x_m + q - 1) with x_m the product of its members' e^{J}.
 * Requires a plan created with opts.gradient = 1 (else KN_E_UNSUPPORTED);
 * J as in kn_contract.  kn_backward_workspace gives the workspace size (the
 * plan's workspace_bytes). */
kn_status kn_backward_workspace(const kn_plan* p, uint64_t* bytes);
kn_status kn_contract_backward(const kn_plan* p, const double* J, void* workspace,
                               size_t workspace_bytes, void* stream,
                               kn_scalar* z_dev, double* grad_dev);

/* ------------------------------------------------------------------ Eq. 4
 * V = A(q) Z with A(q) = (-t^{1/2} - t^{-1/2})^{-n_v-1} (-t^{3/4})^{w} t^{tau/4},
 * all fractional powers taken from the principal fourth root of t (Eq. 1).
 * n_v, w and tau are those of the ORIGINAL Tait graph `g`.  Outputs are host
 * scalars; v_re/v_im overflow to +-inf when |V| exceeds double range, in which
 * case log2_abs_v (nullable) and arg_v (nullable) still carry V exactly. */
kn_status kn_jones(int32_t q, const kn_tait* g, const kn_scalar* z_host, double* v_re,
                   double* v_im, double* log2_abs_v, double* arg_v);
/* t(q) of Eq. 1 with principal square roots. */
kn_status kn_jones_variable(int32_t q, double* t_re, double* t_im);

/* ------------------------------------------------------------------ host runtime
 * kn_plan_many: kn_build_tait + kn_plan_create for many knots on a pool of
 * host threads (n_threads <= 0: one per CPU in the process affinity mask).  Knot i has
 * n_crossings[i] crossings; its PD code starts at pd + 4*s_i and its signs
 * (optional, NULL for all knots) at signs + s_i, s_i = sum of n_crossings[j]
 * for j < i.  q[i] in [2, 8].  taits[i] / plans[i] receive handles owned by
 * the caller (NULL where that knot failed; a plan over budget is still
 * returned, as with kn_plan_create); status[i] (nullable) its status.
 * Returns KN_OK if every knot succeeded, else the first failing status. */
kn_status kn_plan_many(int32_t n_knots, const int32_t* n_crossings, const int32_t* pd,
                       const int8_t* signs, const int32_t* q, const kn_plan_opts* opts,
                       int32_t n_threads, kn_tait** taits, kn_plan** plans, kn_status* status);
/* Free n Tait graphs and n plans (as returned by kn_plan_many; null entries
 * are skipped; either array may be NULL). */
void kn_free_many(int32_t n, kn_tait** taits, kn_plan** plans);
/* kn_jones for n knots: v (nullable) receives 2n doubles (re, im). */
kn_status kn_jones_many(int32_t n, const int32_t* q, const kn_tait* const* g,
                        const kn_scalar* z_host, double* v, double* log2_abs_v, double* arg_v);

/* ------------------------------------------------------------------ batches
 * A batch contracts many plans (any mix of knots, q and sizes) in one
 * persistent kernel launch.  All plans must share one precision.
 * kn_batch_create builds the combined task list on the host; kn_batch_upload
 * copies its device image into the workspace (once); kn_batch_contract only
 * launches kernels (a clear kernel and the persistent kernel), so it can be
 * captured in a hipGraph and replayed.
 *   J    NULL (Jones couplings for every knot) or a device array holding, for
 *        knot i, 2*n_edges(i) doubles at offset 2*edge_offset(i) (see
 *        kn_batch_edge_offset).  A non-NULL J needs no jones_only plans.
 *   z_dev  device array of n kn_scalar, one per plan, in input order. */
typedef struct {
  uint64_t workspace_bytes;
  uint64_t image_bytes;
  int32_t n_tasks;
  int32_t n_knots;
  double flops;
  double bytes;
  int64_t total_edges;
  int32_t grid;
} kn_batch_stats;
kn_status kn_batch_create(const kn_plan* const* plans, int32_t n, kn_batch** out);
kn_status kn_batch_info(const kn_batch* b, kn_batch_stats* out);
kn_status kn_batch_edge_offset(const kn_batch* b, int32_t i, int64_t* off);
kn_status kn_batch_upload(const kn_batch* b, void* workspace, size_t workspace_bytes, void* stream);
kn_status kn_batch_contract(const kn_batch* b, const double* J, void* workspace,
                            size_t workspace_bytes, void* stream, kn_scalar* z_dev);
/* kn_contract_backward for a batch of gradient plans: grad_dev receives, for
   knot i, 2*n_edges(i) doubles at offset 2*edge_offset(i).  KN_E_UNSUPPORTED
   unless every plan was created with opts.gradient = 1. */
kn_status kn_batch_contract_backward(const kn_batch* b, const double* J, void* workspace,
                                     size_t workspace_bytes, void* stream, kn_scalar* z_dev,
                                     double* grad_dev);
/* Read-only view of the batch's device image (see kn_plan_image). */
kn_status kn_batch_image(const kn_batch* b, const void** data, size_t* bytes);
/* Override the persistent grid size (workgroups) of later kn_batch_contract
   calls; 0 restores the default (one workgroup per compute unit, at most one
   per task). */
kn_status kn_batch_set_grid(kn_batch* b, int32_t grid);
/* Per-task timing of later kn_batch_contract calls: trace_dev (device, at
   least 64 * n_tasks bytes; NULL switches tracing off) receives for task i the
   record {int64 t_claim, t_start, t_end; int32 task, workgroup; int64 ph[4]}
   in device clock ticks (100 MHz): queue slot claimed, task available, task
   done; for serial tasks ph = time in setup, staging descriptors and
   tables, step products, reductions and barriers. */
kn_status kn_batch_set_trace(kn_batch* b, void* trace_dev, size_t bytes);
void kn_batch_free(kn_batch* b);

/* Human-readable name of a status code (static string). */
const char* kn_status_string(kn_status s);
/* Library version string (static). */
const char* kn_version(void);

#ifdef __cplusplus
}
#endif
#endif /* KN_H */
