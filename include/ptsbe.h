/*
 * ptsbe.h - C ABI of the MI355X-native PTSBE hot path.
 *
 * Pre-trajectory sampling with batched execution (PTSBE) for noisy tensor-network
 * simulation, following "Accelerating Quantum Tensor Network Simulations with
 * Unified Path Variations and Non-Degenerate Batched Sampling":
 *
 *   ptsbe_plan                 one unified, error-independent contraction path per
 *                              qubit batch (Sec. III-A, unified path variations);
 *                              host only, outside the timed hot path (Sec. IV-D).
 *   ptsbe_sample_trajectories  pre-trajectory sampling of unique error sets with
 *                              multiplicities (Sec. II-C); host only.
 *   ptsbe_contract_batch       error injection (the UPV merge of each sampled
 *                              Kraus operator into its gate) and the batch-wise
 *                              contraction of one batch's marginals for a list of
 *                              (trajectory, prefix) elements (Sec. II-B, III-A).
 *   ptsbe_sample_shots         the whole non-degenerate batched sampling loop
 *                              (Sec. III-B, proportional mode): contract once per
 *                              unique prefix, FP64 cumulative sums, inverse-CDF
 *                              draws, prefix deduplication, trajectory weights.
 *
 * Conventions
 *   - Qubit q of a shot is bit (q % 64) of word (q / 64); 0 <-> |0>.
 *   - Gate matrices are row-major, rows = outputs, interleaved complex128
 *     (re, im).  A two-qubit gate on (q0, q1) is indexed 2*x[q0] + x[q1].
 *   - Noise sites act right after their gate, in site order (the paper's "errors
 *     are preceded or succeeded by a gate of the same size and location").
 *   - Batches are contiguous ascending qubit ranges; batch j starts at
 *     b_0 + ... + b_{j-1}.  Batch indices are 0-based.
 *   - The marginal of batch j for element e = (trajectory i, prefix s_<j) is the
 *     unnormalised pi_e(x) = sum_y |psi~_i(s_<j, x, y)|^2 over batch values x
 *     (x = sum_k x_{start+k} 2^k) and later-qubit values y; psi~_i is built with
 *     the inserted operators K_k / sqrt(q_k) (q_k: the proposal of Kraus k).
 *   - Shot draws: u = Philox4x32-10(key = (lo32(seed), hi32(seed) ^ 2*0x9E3779B9),
 *     counter = (trajectory, batch, shot index within trajectory, 0)), top 53
 *     bits; x = min{x : C(x) > u * C(last)} with C the FP64 inclusive prefix sum
 *     of pi_e in index order (the largest x with pi_e(x) > 0 if none; 0 if pi_e
 *     is identically zero: a trajectory whose inserted operators annihilate the
 *     state, e.g. amplitude damping's K1 twice on a qubit with only diagonal
 *     gates between, has Z_i = 0, weight 0 and all-zero shots).
 *
 * Memory ownership
 *   - Host arrays passed in are copied before the call returns.
 *   - Every d_* pointer is caller-owned device memory on the plan's device.
 *     The library never allocates on the hot path: scratch comes from the
 *     caller's workspace (d_workspace, workspace_bytes).  The plan owns small
 *     constant tables (gate tensors, step tables) allocated in ptsbe_plan and
 *     freed by ptsbe_plan_destroy.
 *   - Device calls are asynchronous on the given stream except where noted: the
 *     sampling loop reads data-dependent element counts back to the host once
 *     per batch and so synchronises the stream.
 *
 * Errors
 *   Every call returns a status; ptsbe_last_error() gives a thread-local message
 *   for the last non-OK status.  Argument errors, unsupported shapes and
 *   workspace shortfalls are detected before any launch.
 */
#ifndef PTSBE_H
#define PTSBE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  PTSBE_OK = 0,
  PTSBE_ERR_INVALID_ARG = 1,   /* malformed circuit / options / pointers        */
  PTSBE_ERR_UNSUPPORTED = 2,   /* gate arity > 2, batch size > 30, path shape   */
  PTSBE_ERR_OUT_OF_MEMORY = 3, /* workspace or plan budget too small            */
  PTSBE_ERR_DEVICE = 4,        /* HIP runtime error                             */
  PTSBE_ERR_NUMERIC = 5        /* non-finite marginal                           */
} ptsbe_status_t;

enum { PTSBE_C64 = 0, PTSBE_SPLIT_BF16 = 1, PTSBE_SPLIT_F16 = 2 };
enum { PTSBE_OUT_POPULATION = 0, PTSBE_OUT_AMPLITUDE = 1 };
enum { PTSBE_MODE_PROPORTIONAL = 0 };
/* How the per-trajectory network is contracted (plan option "method"):
 *   NETWORK      the doubled / ket network of each batch along the unified
 *                sweep path (Sec. III-A); any n, but the path must fit.
 *   STATEVECTOR  the ket network contracted in circuit order into the full
 *                2^n statevector of each trajectory (n <= 30), gates applied in
 *                LDS-resident windows of at most 12 qubits; every batch's
 *                marginals are then partial sums over that state.  Same
 *                unified-path property: one gate schedule for all trajectories.
 *   AUTO         STATEVECTOR when n <= 20, or when the network path does not
 *                fit and n <= 30 (both only if every b_j <= 12); NETWORK
 *                otherwise. */
enum { PTSBE_METHOD_AUTO = 0, PTSBE_METHOD_NETWORK = 1, PTSBE_METHOD_STATEVECTOR = 2 };

typedef struct ptsbe_plan_s* ptsbe_plan_t;

/* A circuit D with its noise model (Sec. II-B: coherent gates d_l, noise sites p).
 * gate_mats packs gate g's d x d matrix (d = 2^arity) as 2*d*d doubles, gates in
 * order.  ch_kraus packs channel c's Kraus operators (d x d each, d = 2^ch_arity)
 * the same way, channels in order.  ch_prob (may be NULL) gives the pre-sampling
 * probability of every Kraus operator in the same packed order; a negative entry,
 * or NULL, means q_k = tr(K_k^dag K_k) / d.  Site s attaches channel
 * site_channel[s] to gate site_gate[s] on qubits site_qubits[2s], [2s+1] (-1 if
 * unused); site qubits must be qubits of that gate. */
typedef struct {
  int32_t n_qubits;
  int32_t n_gates;
  const int32_t* gate_arity;    /* [n_gates] 1 or 2                              */
  const int32_t* gate_qubits;   /* [n_gates][2], second entry -1 for 1q gates    */
  const double* gate_mats;      /* packed interleaved complex128                 */
  int32_t n_channels;
  const int32_t* ch_arity;      /* [n_channels] 1 or 2                           */
  const int32_t* ch_nkraus;     /* [n_channels] >= 1, <= 256                     */
  const double* ch_kraus;       /* packed interleaved complex128                 */
  const double* ch_prob;        /* packed per Kraus operator, or NULL            */
  int32_t n_sites;
  const int32_t* site_gate;     /* [n_sites]                                     */
  const int32_t* site_qubits;   /* [n_sites][2]                                  */
  const int32_t* site_channel;  /* [n_sites]                                     */
} ptsbe_circuit_t;

/* Plan options (Sec. II-B / V-B: flexible per-batch sizes b_j; Sec. IV-C:
 * hypersamples of the path search). */
typedef struct {
  int32_t n_batches;
  const int32_t* batch_sizes;   /* [n_batches], each 1..30, sum == n_qubits     */
  int32_t hypersamples;         /* randomised path-search restarts (>= 1)        */
  uint64_t path_seed;
  int32_t precision;            /* PTSBE_C64, PTSBE_SPLIT_BF16 or PTSBE_SPLIT_F16:
                                   the dense contractions run with hi+lo 16-bit
                                   operands, three products on bf16 / fp16 MFMA
                                   with FP32 accumulation: network method, the
                                   join of doubled networks (16 or 32 crossing-
                                   wire values; fp16: power-of-two scaling per
                                   row and per x); statevector method, the gate
                                   clusters of its windows (fp16: power-of-two
                                   scaling per column).  Everything else stays
                                   c64, FP64 for sums, CDFs and weights */
  int32_t device;               /* HIP device ordinal; -1: host-only plan (path,
                                   query and pre-sampling only, no device calls) */
  size_t device_budget_bytes;   /* 0: no limit; else plan constants must fit     */
  int32_t method;               /* PTSBE_METHOD_*                                 */
  int32_t light_cone;           /* 1: every doubled network (batches before the
                                   last) keeps only the gates in the past light
                                   cone of its prefix and batch qubits, plus every
                                   gate that is not unitary for some trajectory
                                   (bare gate or a possible inserted K / sqrt(q)
                                   with |M^dag M - I| > 1e-6) and that gate's
                                   past: the removed gates meet their adjoints and
                                   cancel under the trace (an extension of the
                                   unified path; Sec. VI names light-cone
                                   simplification under UPV as open).  The kept
                                   set depends on channel types only, so one path
                                   serves every trajectory.  Results equal the full
                                   network's up to the removed gates' deviation
                                   from unitarity.  0: full networks.  Network
                                   method only (the statevector method ignores
                                   it); other values: INVALID_ARG                */
  int32_t subtree_reuse;        /* 1: the per-trajectory parts of the network
                                   method reuse partial sweeps between error sets
                                   (Sec. VI names such caching as open): jobs whose
                                   Kraus choices agree on every site absorbed so
                                   far share the running tensor, and split only at
                                   the launch that absorbs a site they disagree on.
                                   Results are bit-identical to 0 (each group runs
                                   on gates every member shares).  Parts swept
                                   whole in LDS are not split.  0: off; other
                                   values: INVALID_ARG                           */
  int32_t sample_kernel;        /* 0: automatic: batches of at most 5 qubits with
                                   at most 4 shots per element on average sample
                                   and split their elements one lane per element
                                   (elements with more shots: one wavefront each);
                                   1: one wavefront per element always.  Both give
                                   the same shots bit for bit (the lane kernels
                                   repeat the wavefront's FP64 operations in the
                                   same order); other values: INVALID_ARG        */
  int32_t max_part_rank;        /* 0: 31.  Largest rank of the last batch's
                                   per-trajectory tensors: beyond it the wires
                                   crossing to the per-element part are sliced
                                   (each fixed to 0 and 1 in turn on both parts,
                                   the join's amplitudes summed over the slices;
                                   the sum over a contracted index split into
                                   terms), as long as the slice bits fit the
                                   unused bits of the last prefix word (n + s
                                   bits, all in word n / 64); 4..31, other
                                   values: INVALID_ARG                           */
} ptsbe_plan_opts_t;

typedef struct {
  int32_t n_qubits, n_gates, n_sites, n_batches, n_words;  /* n_words = ceil(n/64) */
  int32_t max_kraus;            /* largest channel size                          */
  int64_t plan_device_bytes;    /* constants held by the plan                    */
  int32_t method;               /* PTSBE_METHOD_NETWORK or _STATEVECTOR (chosen)  */
  int32_t sv_windows;           /* statevector method: launches (state passes) per
                                   trajectory to apply every gate; else 0        */
  int32_t sv_windows_by_size[3];/* the same for windows of 10, 11, 12 qubits     */
  int32_t sv_clusters;          /* statevector method: gate clusters (16 x 16
                                   matrices applied on MFMA) in those windows    */
  int32_t sv_cluster_steps;     /* gates applied inside those clusters           */
  int32_t precision;            /* the plan's precision option                    */
  int32_t light_cone;           /* the plan's light-cone option                   */
  int32_t subtree_reuse;        /* the plan's subtree-reuse option                */
} ptsbe_plan_info_t;

/* Per-batch description of the unified path P^j (host-side cost model). */
typedef struct {
  int32_t start, size;          /* batch qubits [start, start+size)              */
  int32_t doubled;              /* 1: ket x bra network (j < f-1), 0: ket only   */
  int32_t n_left_steps;         /* per-element steps (prefix-projected part)     */
  int32_t n_right_steps;        /* per-trajectory steps                          */
  int32_t n_resume_steps;       /* per-element steps when resuming from the parent
                                   element's left tensor (sampling loop, j >= 1)  */
  int32_t left_rank, right_rank;/* ranks of the two partial results              */
  int32_t left_peak_rank, right_peak_rank;
  int32_t join_rows_log2;       /* open batch legs carried by the left part      */
  int32_t crossing;             /* wires joining the left and right parts        */
  double flops_per_traj;        /* algorithmic real flops, per-trajectory part   */
  double flops_per_elem;        /* per element: left sweep + join                */
  double join_flops_per_elem;   /* join only; for a doubled batch on the MFMA
                                   join (K = 16, 32) the flops of the real
                                   bilinear form over K^2 folded slots: 2 K^2 per
                                   row and x                                     */
  double bytes_per_traj;        /* algorithmic HBM bytes of the per-traj part    */
  int32_t n_right_launches;     /* launches of the per-trajectory part: fused
                                   in-place runs + single steps in HBM (0 when it
                                   runs as one LDS sweep)                        */
  int32_t n_right_fused_steps;  /* per-trajectory steps inside fused in-place runs */
  int32_t right_longest_run;    /* steps of the longest fused run                */
  int32_t kept_gates;           /* gates in the batch's network (all of them
                                   unless the light cone removed some)           */
  int32_t slice_bits;           /* last batch: crossing wires sliced (the parts
                                   are contracted 2^slice_bits times and the
                                   join's amplitudes summed); 0 otherwise; the
                                   crossing count above excludes them            */
} ptsbe_batch_info_t;

ptsbe_status_t ptsbe_plan(const ptsbe_circuit_t* circuit, const ptsbe_plan_opts_t* opts,
                          ptsbe_plan_t* out);
ptsbe_status_t ptsbe_plan_query(ptsbe_plan_t plan, ptsbe_plan_info_t* out);
ptsbe_status_t ptsbe_plan_batch_info(ptsbe_plan_t plan, int32_t j, ptsbe_batch_info_t* out);
/* The noise sites whose Kraus choices enter the per-trajectory part of batch j:
 * two trajectories that agree on these sites have the same per-trajectory tensor
 * at batch j (network method).  sites (host, caller-owned, may be NULL): the
 * ascending site ids, room for the circuit's site count; *n_sites_out: their
 * number.  PTSBE_ERR_INVALID_ARG for a statevector plan or j out of range. */
ptsbe_status_t ptsbe_plan_right_sites(ptsbe_plan_t plan, int32_t j, int32_t* sites, int32_t* n_sites_out);

/* Tiling of the last-batch GEMV join over x (plan introspection, network method):
 * for a ket-only batch j whose per-trajectory part carries at least 12 bits of x,
 * the 12 tile bits' offsets in that part's tensor T (read order, ascending) and in
 * the population output (write order, ascending), the write-order index of each
 * read-order bit, and the T and output offsets of the x bits outside the tile;
 * also every x bit's own offsets in T and in the output, so that a caller can
 * check that the tiles cover each x once.  PTSBE_ERR_UNSUPPORTED when the batch
 * takes no tiling (doubled batch, fewer than 12 bits, more than 2 rows).
 *   t_read[12], o_read[12], o_write[12] int64; w_of[12] int32;
 *   t_hi[32], o_hi[32] int64, n_hi: bits outside the tile;
 *   x_t[32], x_o[32] int64, n_x: every x bit (host buffers, caller-owned). */
ptsbe_status_t ptsbe_plan_join_tiling(ptsbe_plan_t plan, int32_t j, int64_t* t_read, int64_t* o_read,
                                      int32_t* w_of, int64_t* o_write, int64_t* t_hi, int64_t* o_hi,
                                      int32_t* n_hi, int64_t* x_t, int64_t* x_o, int32_t* n_x);
/* Statevector method: the gate schedule for windows of window_qubits (10, 11 or
 * 12) qubits, for inspection and tests.  Host outputs (caller-owned; any may be
 * NULL): gate_order [n_gates] gate indices in execution order (each gate once; a
 * gate is moved only past gates on disjoint qubits), window_first [n_windows + 1]
 * offsets into gate_order, window_qubits [n_windows][12] the qubits held in LDS
 * by each window (-1 padded), n_windows_out.  Arrays must hold n_gates entries
 * (window_first: n_gates + 1, window_qubits: 12 * n_gates).
 * PTSBE_ERR_INVALID_ARG for a network-method plan or another window size. */
ptsbe_status_t ptsbe_plan_sv_schedule(ptsbe_plan_t plan, int32_t window_qubits, int32_t* gate_order,
                                      int32_t* window_first, int32_t* window_qubits_out, int32_t* n_windows_out);
void ptsbe_plan_destroy(ptsbe_plan_t plan);
const char* ptsbe_last_error(void);

/* Pre-trajectory sampling (host).  Draw d, site p uses Philox counter
 * (lo32(d), p, hi32(d), 0)
 * with tag 1; the Kraus index is the first k whose FP64 inclusive cumulative
 * proposal exceeds u.  Draws continue until n_unique distinct error sets exist,
 * every error set of non-zero probability has appeared, or max_draws draws were
 * made.  Outputs (host, caller-owned):
 *   kraus_idx [n_unique][n_sites] uint8, distinct sets in order of first draw
 *   mult      [n_unique] draws that produced each set
 *   log_q     [n_unique] sum of log proposals of the set
 *   n_unique_out, n_draws_out (either may be NULL). */
ptsbe_status_t ptsbe_sample_trajectories(ptsbe_plan_t plan, uint64_t seed, int64_t n_unique,
                                         int64_t max_draws, uint8_t* kraus_idx, int64_t* mult,
                                         double* log_q, int64_t* n_unique_out,
                                         int64_t* n_draws_out);

/* Workspace needed by ptsbe_contract_batch / ptsbe_sample_shots for E
 * trajectories, n_elems elements (contract) and total_shots shots (sample). */
ptsbe_status_t ptsbe_contract_workspace_size(ptsbe_plan_t plan, int32_t j, int64_t E,
                                             int64_t n_elems, size_t* bytes);
ptsbe_status_t ptsbe_sample_workspace_size(ptsbe_plan_t plan, int64_t E, int64_t total_shots,
                                           size_t* bytes);

/* Trajectory chunking of a network-method plan (host only, no device work): the
 * per-trajectory tensors of a batch are built for a chunk of trajectories at a
 * time, the chunk sized so that they take at most half of the workspace left
 * after the call's persistent arrays.  For call 0 (ptsbe_contract_batch with E
 * trajectories and count elements) or call 1 (ptsbe_sample_shots with E
 * trajectories and count shots in total) and workspace_bytes of workspace,
 * traj_per_chunk[j] (host, [n_batches], caller-owned) receives the number of
 * trajectories per chunk at batch j, or 0 when not even one fits (the call
 * would return PTSBE_ERR_OUT_OF_MEMORY).  Chunking never changes results.
 * PTSBE_ERR_INVALID_ARG for a statevector-method plan or a bad call kind. */
ptsbe_status_t ptsbe_plan_chunking(ptsbe_plan_t plan, int32_t call, int64_t E, int64_t count,
                                   size_t workspace_bytes, int64_t* traj_per_chunk);

/* Batch-wise contraction of batch j (Sec. II-B) for n_elems elements.
 *   d_kraus_idx   [E][n_sites] uint8 error sets (device)
 *   d_elem_traj   [n_elems] int32 trajectory of each element, non-decreasing
 *   d_elem_prefix [n_elems][n_words] uint64 prefix bits (qubits < start; others 0)
 *   out_kind      PTSBE_OUT_POPULATION: d_out is float [n_elems][2^b_j] pi_e(x)
 *                 PTSBE_OUT_AMPLITUDE (last batch only): d_out is float2
 *                 [n_elems][2^b_j] amplitudes
 *   d_elem_total  [n_elems] double, FP64 sum of pi_e (may be NULL)
 * Asynchronous on `stream` (a hipStream_t). */
ptsbe_status_t ptsbe_contract_batch(ptsbe_plan_t plan, int32_t j, const uint8_t* d_kraus_idx,
                                    int64_t E, const int32_t* d_elem_traj,
                                    const uint64_t* d_elem_prefix, int64_t n_elems,
                                    int32_t out_kind, void* d_out, double* d_elem_total,
                                    void* d_workspace, size_t workspace_bytes, void* stream);

/* ptsbe_contract_batch without a caller workspace, for callers that cannot
 * allocate device memory (serving loops and harnesses that forbid allocation):
 * the workspace is a fixed array of PTSBE_NOALLOC_SCRATCH_BYTES in the library's
 * own device memory, one per GPU, held until the process ends.  Same arguments,
 * results and stream semantics as ptsbe_contract_batch (it also synchronises
 * `stream` to check d_elem_traj); no device memory is allocated or freed.  Calls
 * whose trajectories and elements do not fit the array (with the executor's
 * chunking) return PTSBE_ERR_UNSUPPORTED with the sizes in ptsbe_last_error().
 * Every call on a GPU uses the same array: calls that overlap on one GPU (other
 * host threads, other streams) race and must be serialised by the caller.  No
 * part of the array needs to start at zero. */
#define PTSBE_NOALLOC_SCRATCH_BYTES ((size_t)256 << 20)
ptsbe_status_t ptsbe_contract_batch_noalloc(ptsbe_plan_t plan, int32_t j, const uint8_t* d_kraus_idx,
                                            int64_t E, const int32_t* d_elem_traj,
                                            const uint64_t* d_elem_prefix, int64_t n_elems,
                                            int32_t out_kind, void* d_out, double* d_elem_total, void* stream);

/* Batch lists against measured time (Sec. V-B: the qubit batch sizes b_j are a
 * free choice of the interface and set the contraction cost).  Candidate c is
 * the list cand_sizes[cand_offsets[c] .. cand_offsets[c+1]) (host arrays,
 * n_candidates + 1 offsets); each gets its own plan from base_opts with that
 * list, then ptsbe_sample_shots (proportional mode) runs once untimed and once
 * timed with HIP events on `stream`, on the caller's trajectories and shots
 * (the same arguments as ptsbe_sample_shots; d_shots [M][n_words] receives each
 * candidate's shots in turn, the last one's remain).  Error sets do not depend
 * on the batch list, so d_kraus_idx serves every candidate.
 *   times_ms  host double [n_candidates]: the timed call, or -1 when the list
 *             cannot be planned or sampled (sizes not summing to n_qubits, a
 *             batch wider than the sampler draws, a workspace too small)
 *   best      host: index of the fastest candidate
 * PTSBE_ERR_UNSUPPORTED when no candidate runs; a device error ends the call.
 * Plans are built and destroyed inside the call (host path finding and device
 * constants per candidate); synchronises `stream`. */
ptsbe_status_t ptsbe_tune_batches(const ptsbe_circuit_t* circuit, const ptsbe_plan_opts_t* base_opts,
                                  int32_t n_candidates, const int32_t* cand_offsets, const int32_t* cand_sizes,
                                  const uint8_t* d_kraus_idx, int64_t E, const int64_t* d_mult,
                                  const int64_t* d_shots_per_traj, uint64_t seed, uint64_t* d_shots,
                                  void* d_workspace, size_t workspace_bytes, void* stream, double* times_ms,
                                  int32_t* best);

/* Non-degenerate batched sampling, proportional mode (Sec. III-B).
 *   d_kraus_idx       [E][n_sites] uint8
 *   d_mult            [E] int64 multiplicities (NULL: all 1)
 *   d_shots_per_traj  [E] int64 m_i
 *   seed              shot seed (Philox tag 2)
 *   d_shots           [M][n_words] uint64, M = sum m_i; trajectory i's shots occupy
 *                     rows [sum_{k<i} m_k, ... + m_i) in shot-index order
 *   d_shot_traj       [M] int32 (may be NULL)
 *   d_traj_weight     [E] double W_i = mult_i Z_i / sum_k mult_k Z_k, Z_i the
 *                     trajectory's squared norm (may be NULL)
 *   d_traj_norm       [E] double Z_i (may be NULL)
 *   stats_out         host int64 [n_batches]: distinct elements contracted per
 *                     batch (may be NULL)
 * Synchronises `stream` once per batch. */
ptsbe_status_t ptsbe_sample_shots(ptsbe_plan_t plan, const uint8_t* d_kraus_idx, int64_t E,
                                  const int64_t* d_mult, const int64_t* d_shots_per_traj,
                                  int32_t mode, uint64_t seed, uint64_t* d_shots,
                                  int32_t* d_shot_traj, double* d_traj_weight,
                                  double* d_traj_norm, int64_t* stats_out, void* d_workspace,
                                  size_t workspace_bytes, void* stream);

/* Non-degenerate batched sampling, non-proportional mode (Sec. III-B), with
 * exhaustive or direct final-batch sampling.  Statevector-method plans take
 * batches of at most 12 qubits (the last one included) and run trajectories in
 * chunks whose states fit the workspace; rows do not depend on the chunking.
 *   Non-final batches: every distinct (trajectory, prefix) element takes
 *   `draws` draws from its conditional marginal (Philox tag 3, counter
 *   (trajectory, j, r * draws + d, 0) for the element of rank r among its
 *   trajectory's elements, r counted in the order below); its distinct outcomes
 *   become the next batch's elements.  Elements are ordered by trajectory, then
 *   lexicographically by (s_1, s_2, ...), the first batch most significant.
 *   Final batch, final_draws == 0 (exhaustive; any size up to 30 qubits, the
 *   other batches at most 12): for every element of total Z_e > 0, one row per
 *   x with P(x | prefix) = pi_e(x) / Z_e strictly above `threshold` (FP64
 *   quotient of the FP32 population and the FP64 total), in element order then
 *   x ascending.
 *   Final batch, final_draws > 0 (direct; last batch of at most 12 qubits,
 *   threshold unused): element e takes final_draws draws (counters as above with
 *   j = f - 1), rows [e * final_draws, (e + 1) * final_draws) in draw order,
 *   repeats kept; an element of total 0 draws x = 0 with P = p(prefix) = 0.
 *   draws            >= 1
 *   max_elems        bound on the elements of any batch (sizes the workspace;
 *                    exceeding it returns PTSBE_ERR_OUT_OF_MEMORY)
 *   d_bits           [capacity][n_words] uint64 full bitstrings
 *   d_row_traj       [capacity] int32 trajectory of each row (may be NULL)
 *   d_p_cond         [capacity] double P(x | prefix) (may be NULL)
 *   d_p_prefix       [capacity] double p(prefix) = Z_e / Z_i (may be NULL)
 *   n_rows_out       host: the number of rows found; when it exceeds capacity
 *                    the call returns PTSBE_ERR_OUT_OF_MEMORY (call again with
 *                    more room): exhaustive mode writes the first `capacity`
 *                    rows, direct mode at most a leading part of them
 *   d_traj_weight, d_traj_norm, stats_out: as for ptsbe_sample_shots.
 * Synchronises `stream` once per batch and once per final-batch element chunk. */
ptsbe_status_t ptsbe_nonproportional_workspace_size(ptsbe_plan_t plan, int64_t E, int32_t draws,
                                                    int32_t final_draws, int64_t max_elems, size_t* bytes);
ptsbe_status_t ptsbe_sample_nonproportional(ptsbe_plan_t plan, const uint8_t* d_kraus_idx, int64_t E,
                                            const int64_t* d_mult, int32_t draws, int32_t final_draws,
                                            int64_t max_elems, uint64_t seed, double threshold,
                                            uint64_t* d_bits, int32_t* d_row_traj, double* d_p_cond,
                                            double* d_p_prefix, int64_t capacity, int64_t* n_rows_out,
                                            double* d_traj_weight, double* d_traj_norm, int64_t* stats_out,
                                            void* d_workspace, size_t workspace_bytes, void* stream);

/* Differentiation of trajectory-averaged quantities (an addition to the paper's
 * method; its unified gate schedule and UPV merge (Sec. III-A) are reused).
 *   - Rotation gates: gate g with gate_param[g] >= 0 has the matrix
 *     U_g = exp(-i theta[gate_param[g]] P / 2), P = X, Y, Z for gate_axis[g] = 0,
 *     1, 2; its matrix in the plan's circuit is ignored.  Several gates may share
 *     a parameter.  Other gates keep their matrix U_g.
 *   - Error sets are fixed; psi_i is the trajectory's state: the UPV-merged gates
 *     A_g = (inserted operators of g) U_g applied in circuit order to |0...0>
 *     (n_qubits <= 30, any method).
 *   - The quantity differentiated is L = sum_i w_i <psi_i|O|psi_i> for a
 *     diagonal observable O (the ZZ terms, or d_obs_diag), or, with d_psi_bar,
 *     any real L(psi_1, ..., psi_E) whose conjugate-Wirtinger derivative
 *     psi-bar_i = dL / d conj(psi_i) the caller supplies (then dL = 2 Re sum_i
 *     <psi-bar_i | d psi_i>).
 *   - Adjoint contraction: the ket network of every trajectory is contracted
 *     through LDS gate windows of at most 11 qubits, the state after each window
 *     kept as a checkpoint; the backward pass walks the windows in reverse with
 *     lambda = psi-bar (or w_i O psi_i), lambda_{k-1} = A_k^dag lambda_k, and
 *     psi_{k-1} = A_k^dag psi_k when every inserted operator is unitary (mixed-
 *     unitary channels), else recomputed from the window's checkpoint.  It gives
 *     dL/dtheta = sum over gates of the parameter of Im <lambda_{k-1}|P|psi_{k-1}>
 *     and the gate-tensor adjoint 2 dL/d conj(U_g) = 2 U_g sum_i sum_rest
 *     lambda_{k-1} psi_{k-1}^dag (torch's convention for a real loss).  Sums over
 *     trajectories and tiles are FP64 in a fixed order (deterministic). */
typedef struct {
  int32_t n_params;
  const int32_t* gate_param;    /* [n_gates] (host) parameter index, -1 for fixed (NULL: none) */
  const int32_t* gate_axis;     /* [n_gates] (host) 0 X, 1 Y, 2 Z                  */
  int32_t n_terms;              /* O = sum_t zz_coef[t] Z_a Z_b when d_obs_diag is NULL */
  const int32_t* zz_qubits;     /* [n_terms][2] (host), at most 64 terms          */
  const double* zz_coef;        /* [n_terms] (host)                                */
  const double* d_obs_diag;     /* [2^n] (device) real diagonal of O, or NULL      */
} ptsbe_adjoint_spec_t;

ptsbe_status_t ptsbe_adjoint_workspace_size(ptsbe_plan_t plan, const ptsbe_adjoint_spec_t* spec, int64_t E,
                                            size_t* bytes);
/*   d_kraus_idx [E][n_sites] uint8, d_weights [E] double w_i, d_theta [n_params]
 *   double (device).  d_psi_bar: NULL, or [E][2^n] complex64 (interleaved, device)
 *   seeds of the backward pass.  Outputs (device, each may be NULL):
 *   d_traj_value [E] <psi_i|O|psi_i> and d_value [1] sum_i w_i <psi_i|O|psi_i>
 *   (need an observable); d_grad [n_params] dL/dtheta; d_gate_adj [n_gates][16]
 *   complex128 (interleaved; the first d*d entries, row-major in the gate's own
 *   index order): 2 dL/d conj(U_g).  Without d_grad and d_gate_adj only the
 *   forward pass runs.  Workspace: ptsbe_adjoint_workspace_size (trajectories
 *   run in chunks that fit it).  Synchronises `stream`. */
ptsbe_status_t ptsbe_contract_adjoint(ptsbe_plan_t plan, const ptsbe_adjoint_spec_t* spec,
                                      const uint8_t* d_kraus_idx, int64_t E, const double* d_weights,
                                      const double* d_theta, const void* d_psi_bar, double* d_traj_value,
                                      double* d_value, double* d_grad, double* d_gate_adj, void* d_workspace,
                                      size_t workspace_bytes, void* stream);

/* The ZZ-observable form of the same contraction: f = sum_i w_i <psi_i|O|psi_i>
 * with O = sum_t zz_coef[t] Z_a Z_b, its value and (d_grad non-NULL) its angle
 * gradient.  checkpoint_every is kept for compatibility (must be >= 1; the
 * checkpoints are the window boundaries). */
typedef struct {
  int32_t n_params;
  const int32_t* gate_param;    /* [n_gates] (host) parameter index, -1 for fixed */
  const int32_t* gate_axis;     /* [n_gates] (host) 0 X, 1 Y, 2 Z                  */
  int32_t n_terms;
  const int32_t* zz_qubits;     /* [n_terms][2] (host)                             */
  const double* zz_coef;        /* [n_terms] (host)                                */
  int32_t checkpoint_every;     /* >= 1                                            */
} ptsbe_grad_spec_t;

ptsbe_status_t ptsbe_expect_workspace_size(ptsbe_plan_t plan, const ptsbe_grad_spec_t* spec, int64_t E,
                                           size_t* bytes);
/*   d_kraus_idx [E][n_sites] uint8, d_weights [E] double w_i, d_theta [n_params] double;
 *   outputs: d_traj_value [E] <psi_i|O|psi_i> (may be NULL), d_value [1] f,
 *   d_grad [n_params] df/dtheta (NULL: value only, forward pass only).  Synchronises `stream`. */
ptsbe_status_t ptsbe_expect_grad(ptsbe_plan_t plan, const ptsbe_grad_spec_t* spec, const uint8_t* d_kraus_idx,
                                 int64_t E, const double* d_weights, const double* d_theta,
                                 double* d_traj_value, double* d_value, double* d_grad, void* d_workspace,
                                 size_t workspace_bytes, void* stream);

/* ------------------------------------------------------------- ragged sets
 * Several circuits sampled in the same launches (an addition to the paper's
 * method, which batches the trajectories of one circuit).  Every job is a
 * statevector-method plan with its error sets and shot counts; the set cuts the
 * jobs' trajectories into waves whose states fit the workspace and runs each
 * wave as one fixed launch sequence with no host round trip: UPV merge per
 * piece, one persistent gate-window launch per window level (all circuits'
 * tiles in one grid-stride queue, heaviest circuits first), then per batch
 * level one persistent marginal, sampling, scan and children launch over the
 * elements of every circuit, with element counts kept on the device.  With
 * PTSBE_RAGGED_GRAPH each wave is captured once as a hipGraph and replayed on
 * later calls with the same arguments.  Kernel boundaries are the dependency
 * barriers between window and batch levels.
 *
 * Ownership: the set owns its graphs; jobs' device arrays and the workspace
 * are the caller's and must stay untouched between calls that replay graphs.
 * stream must not be the null stream when PTSBE_RAGGED_GRAPH is set. */
typedef struct ptsbe_ragged_s* ptsbe_ragged_t;
enum { PTSBE_RAGGED_GRAPH = 1 };

typedef struct {
  ptsbe_plan_t plan;              /* statevector-method plan (b_j <= 12)          */
  const uint8_t* d_kraus_idx;     /* [E][n_sites] uint8 (device)                   */
  int64_t E;
  const int64_t* shots_per_traj;  /* [E] m_i (HOST: the shot layout of the waves)  */
  const int64_t* d_mult;          /* [E] multiplicities (device) or NULL (all 1)   */
  uint64_t seed;                  /* shot seed (Philox tag 2, counters as in
                                     ptsbe_sample_shots: same shots bit for bit)   */
  uint64_t* d_shots;              /* [sum m_i][1] uint64 (device; n <= 30)         */
  double* d_traj_weight;          /* [E] W_i within the job (device) or NULL       */
  double* d_traj_norm;            /* [E] Z_i (device) or NULL                      */
} ptsbe_ragged_job_t;

typedef struct {
  int32_t n_waves;                /* waves of the last call                        */
  int32_t graphs_replayed;        /* waves of the last call served by a cached graph */
  int64_t launches;               /* kernel launches of the last call              */
  double wall_clock_khz;          /* rate of the completion stamps                 */
} ptsbe_ragged_info_t;

ptsbe_status_t ptsbe_ragged_create(int32_t device, ptsbe_ragged_t* out);
void ptsbe_ragged_destroy(ptsbe_ragged_t set);
ptsbe_status_t ptsbe_ragged_info(ptsbe_ragged_t set, ptsbe_ragged_info_t* out);
/* Workspace for the jobs: states of at least one wave of the largest job
 * trajectory plus the per-job arrays; more workspace means fewer waves. */
ptsbe_status_t ptsbe_ragged_workspace_size(ptsbe_ragged_t set, const ptsbe_ragged_job_t* jobs, int32_t n_jobs,
                                           size_t* bytes);
/* Autotuner: for every job's plan, times one full gate-window pass of up to 2
 * trajectories with windows of 10, 11 and 12 qubits (tiles of 2^10..2^12
 * amplitudes in LDS) and keeps the fastest per plan for later calls.
 * best_window (host, [n_jobs], may be NULL) receives the choice; ms_per_traj
 * (host, [n_jobs][3], may be NULL) the measured times.  Synchronises. */
ptsbe_status_t ptsbe_ragged_autotune(ptsbe_ragged_t set, const ptsbe_ragged_job_t* jobs, int32_t n_jobs,
                                     int32_t* best_window, float* ms_per_traj, void* d_workspace,
                                     size_t workspace_bytes, void* stream);
/* Sample every job's shots (proportional mode).  d_done_ticks (device uint64
 * [n_jobs + 1], may be NULL): entry n_jobs receives the wall-clock stamp at the
 * start, entry i the stamp at which job i's last element was sampled (rate in
 * ptsbe_ragged_info).  Synchronises `stream` at the end. */
ptsbe_status_t ptsbe_ragged_sample_shots(ptsbe_ragged_t set, const ptsbe_ragged_job_t* jobs, int32_t n_jobs,
                                         int32_t flags, uint64_t* d_done_ticks, void* d_workspace,
                                         size_t workspace_bytes, void* stream);

/* Timing hook for measurement.  Level 1: the library records HIP events (on
 * the launch stream) around every launch of the MFMA join of doubled networks
 * and accumulates its total time (milliseconds), launch count and algorithmic
 * flops (the real bilinear form over K^2 folded slots: 2^xb * 2^xT * 2 K^2 per
 * element, K = 2^crossing), and the algorithmic bytes of the per-trajectory
 * sweeps.  Level 2 adds events around every single sweep step in HBM
 * (ptsbe_profile_read_sweeps).  Level 0 turns recording off; every call resets
 * the counters.  Events are read when a sampling or contraction call returns. */
ptsbe_status_t ptsbe_profile_enable(ptsbe_plan_t plan, int32_t on);
ptsbe_status_t ptsbe_profile_read(ptsbe_plan_t plan, double* join_ms, int64_t* join_launches,
                                  double* join_flops, double* sweep_ms, double* sweep_bytes);
/* Single sweep steps in HBM (one launch per absorbed gate of a part too large
 * for LDS): total event time (level 2 only), launches, and algorithmic bytes
 * (each job's input and output tensor once: 8 (2^rA + 2^rC)); fused_bytes: the
 * in-place tile runs (each job's tensor read and written once per run). */
ptsbe_status_t ptsbe_profile_read_sweeps(ptsbe_plan_t plan, double* step_ms, int64_t* step_launches,
                                         double* step_bytes, double* fused_bytes);
/* Statevector-method gate windows (any level >= 1): total event time of the
 * window launches (events recorded on the launch stream), launches, and
 * algorithmic bytes (every trajectory state of the launch read and written once:
 * 16 * 2^n bytes per trajectory and window).  The windows of
 * ptsbe_contract_adjoint count here too: 16 * 2^n bytes per trajectory for a
 * forward window (checkpoint read, next checkpoint written) and 24 * 2^n for a
 * backward window (state read, adjoint state read and written). */
ptsbe_status_t ptsbe_profile_read_windows(ptsbe_plan_t plan, double* ms, int64_t* launches, double* bytes);
/* Parts swept whole in LDS (network method; the per-element parts of small
 * batches, and the leading steps of larger parts), any level >= 1: total event
 * time of those launches, launches, and algorithmic flops (each absorbed gate: 8
 * real flops per complex multiply-add, 8 * 2^(rank_out + contracted legs) per step
 * and job). */
ptsbe_status_t ptsbe_profile_read_lds_sweeps(ptsbe_plan_t plan, double* ms, int64_t* launches, double* flops);

#ifdef __cplusplus
}
#endif
#endif /* PTSBE_H */
