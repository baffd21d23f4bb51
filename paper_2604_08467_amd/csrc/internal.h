// Internal structures shared by the planner (host C++), the executor and the
// HIP kernels of the PTSBE library.  Nothing here is part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <array>
#include <cstdint>
#include <string>
#include <vector>

#include "ptsbe.h"

namespace ptsbe {

// ---------------------------------------------------------------- host helpers
extern thread_local std::string g_last_error;
ptsbe_status_t fail(ptsbe_status_t s, const std::string& msg);

#define HIP_TRY(expr)                                                                         \
  do {                                                                                        \
    hipError_t e_ = (expr);                                                                   \
    if (e_ != hipSuccess)                                                                     \
      return ::ptsbe::fail(PTSBE_ERR_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

// bump allocator over the caller's workspace (256-byte aligned blocks)
struct Arena {
  char* base = nullptr;
  size_t cap = 0, used = 0;
  void* take(size_t bytes) {
    size_t off = (used + 255) & ~(size_t)255;
    if (off + bytes > cap) return nullptr;
    used = off + bytes;
    return base + off;
  }
  size_t left() const {
    size_t off = (used + 255) & ~(size_t)255;
    return off >= cap ? 0 : cap - off;
  }
};

constexpr int kMaxBatch = 30;       // largest b_j accepted
// An HSA dispatch counts its work-items in 32 bits: grids stay at most 2^20
// workgroups and the kernels walk larger ranges with grid- or block-stride loops.
constexpr int64_t kMaxGridBlocks = (int64_t)1 << 20;
inline unsigned grid_blocks(int64_t blocks) {
  return (unsigned)(blocks < 1 ? 1 : (blocks > kMaxGridBlocks ? kMaxGridBlocks : blocks));
}
constexpr int kMaxQubits = 1024;
constexpr int kSvMaxQubits = 30;   // statevector method and adjoint pass
constexpr int kVmMaxRank = 11;      // parts whose tensors fit 2^11 c64 run in LDS
constexpr int kMaxSlices = 4;

// ----------------------------------------------------------------------------
// One absorb step of a sweep: C = A (x) B where A is the running tensor of the
// part (rank rA; it starts as the scalar 1) and B is one (merged) gate tensor.
// Labels of A that B contracts sit at bit positions kpos[] of A (ascending);
// the remaining ("kept") labels keep their relative order in C; B's new labels
// are inserted into C at positions npos[] (ascending).  Hyper labels (kept, and
// also indexing B) are bits hm[] of the kept index.  The index into B's 4x4 (or
// 2x2) matrix is the sum of the leg weights of the set bits.
struct AbsorbStep {
  int32_t gate, conj;
  int32_t rA, rC, nK, nN, nH, nS;
  int32_t kpos[4], kw[4];
  int32_t npos[4], nw[4];
  int32_t hm[4], hw[4];
  int32_t sq[kMaxSlices], sw[kMaxSlices];   // prefix-sliced legs: qubit, weight
  // derived tables (filled by the planner): for every value k of the contracted
  // legs / n of the new legs, the offset into A / C and the index into B
  uint32_t koff[16], noff[16];
  int32_t kB[16], nB[16];
  // gate entries in the order the LDS sweep reads them: entry d of the staged
  // gate is entry (gperm[d / 8] >> 4 (d % 8)) & 15 of B.  For steps without
  // hyper or sliced legs d = n 2^nK + k (n-major, so a job's products read
  // consecutive entries at fixed offsets); the identity otherwise
  uint32_t gperm[2] = {0x76543210u, 0xFEDCBA98u};
};

// Local view of an in-place step (same bit positions in and out, rank
// unchanged) inside a fused tile of the tensor: positions are indices into the
// tile's position list P; hyper legs read their bit from the tile-local index
// (h_inP = 1) or from the tile's global base (h_inP = 0, h_pos a global position).
struct FusedStep {
  int32_t gate, conj, nK, nN, nH, nS;
  int32_t kloc[4];
  uint32_t koff[16], noff[16];
  int32_t kB[16], nB[16];
  int32_t h_inP[4], h_pos[4], hw[4];
  int32_t sq[kMaxSlices], sw[kMaxSlices];
  // gate cluster (statevector windows): on the first step of a cluster, cl_len > 0
  // consecutive plain steps act on the 4 distinct tile-local positions cl_pos and
  // are applied together as one 16 x 16 matrix on MFMA (matrix cl_id of the
  // window set's cluster table, built per trajectory beforehand); 0 elsewhere
  int32_t cl_len, cl_id;
  int32_t cl_pos[4];
};

// A gate cluster of a statevector window set: steps [first, first + len) of the
// plan's fused-step list on the tile-local positions pos.
struct ClusterDesc {
  int32_t first, len;
  int32_t pos[4];
};

// Compact op of a statevector gate window, read by the window kernel through the
// scalar cache: a plain one- or two-qubit gate applied in place on the LDS tile,
// or a gate cluster (a 16 x 16 matrix on four tile positions, applied on MFMA).
enum { kSvOpGate1 = 1, kSvOpGate2 = 2, kSvOpCluster = 3 };
struct SvOp {
  int8_t kind;
  int8_t p0, p1;            // gate: tile positions of local index bits 0 and 1
  int8_t conj;              // gate: use the complex conjugate of the merged matrix
  int8_t cpos[4];           // cluster: tile position of cluster-local bit i
  int32_t gate;             // gate: index into the trajectory's merged gates
  int32_t slot;             // gate: staged matrix slot; cluster: index within the window
  int8_t idx[16];           // gate: local entry (n, k), n * d + k, is merged entry idx[n * d + k]
};
static_assert(sizeof(SvOp) == 32, "SvOp is read as eight dwords");
// One window of a statevector schedule in compact form: ops [op_off, op_off + n_ops)
// on the tile positions P (|P| = np, P[0] == 0), n_plain staged gate matrices and
// the window set's clusters [cl_first, cl_first + n_cl).
struct SvWin {
  int32_t op_off, n_ops, n_plain, cl_first, n_cl, np;
  int32_t P[12];
  uint32_t other;           // bit mask of the state's qubits outside the window
};

// Op of an adjoint window (a plain gate in place on the tile): the gate's merged
// matrix entry idx[a * d + b] is local entry (a, b); axis >= 0 marks a rotation
// exp(-i theta P / 2) about P = X, Y, Z whose derivative is accumulated; nslot >= 0
// receives the gate-tensor adjoint N = sum lambda psi^dag.
struct AdjOp {
  int8_t kind, p0, p1, axis;
  int32_t gate, nslot;
  int32_t slot;                   // the op's index in its window (staged matrix slot)
  int8_t idx[16];
};
static_assert(sizeof(AdjOp) == 32, "AdjOp is read as eight dwords");
struct AdjWin {
  int32_t op_off, n_ops, np;
  int32_t P[12];
  int32_t group_off, n_groups;    // the window's op groups (build_adj_groups)
};
// A run of consecutive ops of a window (after regrouping) on at most two tile
// positions pa < pb (nq = 1: pa only), applied by a tile pass in registers.
constexpr int kAdjGroupMax = 8;
struct AdjGroup {
  int8_t nq, pa, pb, n;           // positions used, the group's tile positions, op count
  int32_t first;                  // index of the group's first op in the window
  uint32_t rot_mask;              // bit j: op first + j is a differentiated rotation
  int32_t pad;
};
static_assert(sizeof(AdjGroup) == 16, "AdjGroup is read as four dwords");
struct AdjArgs {
  int n, np, n_ops, n_nslots, G, want_n;
  int P[12];
  uint32_t other;                 // bit mask of the qubits outside the window
  int64_t n_jobs;
  int32_t traj_base;
  const float2* A;                // [E][G][16] merged gates
  const float2* Ad;               // [E][G][16] their adjoints
  const float2* psi_in;           // forward: input states; backward: states after (1) / before (2) the window
  float2* psi_out;                // forward: output states
  float2* lam;                    // backward: adjoint states, in place
  double* wg_acc;                 // backward: [grid][n_ops + 32 n_nslots] per-workgroup sums
  const AdjGroup* groups;         // the window's op groups (tile kernels)
  int n_groups;
};
struct AdjSeedArgs {
  const float2* psi;              // [n_jobs][2^n] final states
  float2* lam;                    // [n_jobs][2^n] seed out (null: values only)
  const float2* psi_bar;          // [E][2^n] caller's seed, or null (lambda = w O psi)
  const double* obs_diag;         // [2^n] diagonal of O (the caller's or the ZZ terms')
  const double* weights;          // [E]
  double* part;                   // [n_jobs][64] partial values (workspace)
  double* values;                 // [E] <psi|O|psi>, or null
  int n;
  int32_t traj_base;
};
size_t adj_window_lds_bytes(int mode, int np, int n_ops, int n_nslots);
int adj_window_grid(int mode, const AdjArgs& a, size_t lds);
hipError_t launch_adj_window(int mode, const AdjArgs& a, const AdjOp* d_ops, int grid, hipStream_t stream);
hipError_t launch_adj_seed(const AdjSeedArgs& s, int64_t n_jobs, hipStream_t stream);
hipError_t launch_adj_zz_diag(int n, const int32_t* zq, const double* zc, int n_terms, double* diag,
                              hipStream_t stream);
hipError_t launch_adj_reduce(const double* wg_acc, int n_wg, int width, double* tot, hipStream_t stream);

// A run of steps executed by one launch: either one absorb step, or a fused
// run of in-place steps whose positions lie in P (|P| = np <= kFuseMax).
constexpr int kFuseMax = 12;
constexpr int kGateChunkHost = 32;    // gate matrices staged per window pass (device: kGateChunk)
constexpr int kSvWindowMin = 10;      // smallest statevector window the autotuner tries
struct Segment {
  int first = 0, count = 1;
  bool fused = false;
  int np = 0, r = 0;
  int P[kFuseMax] = {0};
  int64_t fused_off = 0;            // index of the first FusedStep on the device
};
bool build_segments(const std::vector<AbsorbStep>& steps, std::vector<Segment>& segs,
                    std::vector<FusedStep>& fused);

struct PartPlan {
  std::vector<AbsorbStep> steps;
  std::vector<Segment> segs;        // launch grouping of the steps (global execution)
  std::vector<int> labels;          // final labels, bit order (bit 0 first)
  int peak = 0;                     // largest rank of any A or C
  double flops = 0, bytes = 0, cost = 0;
  std::string order_name;
};

// Offsets of a labelled result tensor used by the join: offset of a group of
// labels as a function of the group's index is a sum over set bits, stored as
// two tables (low / high halves of the group index).
struct SplitTable {
  int bits = 0, lo_bits = 0;
  std::vector<int64_t> lo, hi;
};

// Largest |M^dag M - I| entry for which a gate or an inserted operator counts as
// unitary in the light cone (complex64-rounded unitaries sit near 1e-7).
constexpr double kUnitaryTol = 1e-6;

struct BatchPlan {
  int start = 0, size = 0;
  bool doubled = false;
  PartPlan left, right;             // left: per element (ket, prefix projected)
  std::vector<int> lk, lb, xb, xT;  // join label groups
  std::vector<int> xb_qubits;       // qubit of each xb label
  std::vector<int> left_gates;      // gates of the left part
  // resume variant of the left part (j >= 1): starts from the parent element's
  // left tensor (rank resume_parent_rank) with the legs at resume_slice_pos sliced
  // to the element's bits of qubits resume_slice_q (initial rank resume_rank0)
  PartPlan left_resume;
  int resume_rank0 = 0, resume_parent_rank = 0;
  std::vector<int> resume_slice_pos, resume_slice_q;
  SplitTable v_row_r, v_col_r;
  // join tables
  SplitTable v_row, v_col;          // V[e]: rows over xb, cols over lk
  SplitTable t_x, t_k, t_b;         // T[t]: xT, lk, lb
  SplitTable o_x, o_b;              // output index: xT, xb
  double join_flops_per_elem = 0;
  int kept_gates = 0;               // gates in this batch's network (light cone applied)
  // last batch: crossing wires fixed to each of their 2^slice_bits values in
  // turn (sliced legs read bit n + i of the job's prefix words for wire i),
  // so that the per-trajectory tensor stays within max_part_rank; the join's
  // amplitudes are summed over the slices
  int slice_bits = 0;
  std::vector<int> slice_labels;
};

struct RgWindow;

// Per-gate tensor data uploaded at plan time.
struct DeviceGate {
  float2 def[16];                   // default-branch merged matrix (all sites k=0)
  float2 raw[16];                   // bare gate matrix
  int32_t site_begin, site_end;     // range into the gate-site list
  int32_t arity, pad;
};

struct Plan {
  int device = 0;
  int precision = PTSBE_C64;
  int n = 0, G = 0, S = 0, NW = 1, max_kraus = 1;
  int n_user_gates = 0;                           // gates of the caller's circuit (identities follow)
  std::vector<int> arity;
  std::vector<std::array<int, 2>> qubits;
  std::vector<std::array<double, 32>> mats;       // complex128, 4x4 or 2x2 row-major
  std::vector<int> site_gate, site_channel;
  std::vector<std::array<int, 2>> site_qubits;
  std::vector<std::vector<std::array<double, 32>>> ch_ops;  // per channel, inserted K/sqrt(q)
  std::vector<std::vector<double>> ch_q;          // proposals
  std::vector<std::vector<int>> gate_sites;       // per gate, sites in order
  std::vector<int> batch_sizes;
  std::vector<BatchPlan> batches;
  int hypersamples = 1;
  uint64_t path_seed = 0;

  // device constants
  DeviceGate* d_gates = nullptr;
  int32_t* d_gate_site_list = nullptr;            // site ids ordered by gate
  float2* d_site_ops = nullptr;                   // [S][max_kraus][16] embedded K/sqrt(q)
  AbsorbStep* d_steps = nullptr;                  // all parts' steps, concatenated
  int64_t* d_tables = nullptr;                    // all join tables, concatenated
  std::vector<int64_t> part_step_off;             // per batch: left, right, resumed-left offsets
  struct JoinDev { int64_t vr_lo, vr_hi, vc_lo, vc_hi, tx_lo, tx_hi, tk_lo, tk_hi, tb_lo, tb_hi, ox_lo, ox_hi, ob_lo, ob_hi; };
  std::vector<JoinDev> join_dev;
  std::vector<JoinDev> join_dev_r;                // same with the resumed left part's V tables
  int64_t device_bytes = 0;

  // statevector schedule (qubit q = bit q, gates in circuit order, in place)
  std::vector<AbsorbStep> sv_steps;
  AbsorbStep* d_sv_steps = nullptr;
  // statevector method: the same steps regrouped into LDS windows (sv_run holds
  // them in execution order; every segment of sv_segs is one fused window)
  int method = PTSBE_METHOD_NETWORK;
  std::vector<AbsorbStep> sv_run;
  std::vector<Segment> sv_segs;                   // windows of kFuseMax qubits (the default)
  // window schedules for every tile size the ragged autotuner may pick:
  // sv_win[i] holds windows of at most kSvWindowMin + i qubits
  std::vector<Segment> sv_win[3];
  RgWindow* d_rg_win[3] = {nullptr, nullptr, nullptr};   // the same windows on the device
  std::vector<ClusterDesc> sv_cl[3];              // gate clusters of each window set
  ClusterDesc* d_sv_cl[3] = {nullptr, nullptr, nullptr};
  // the same windows as compact ops (empty when a window holds a step that is not
  // a plain in-place gate: then the generic fused pass runs it)
  std::vector<SvWin> sv_wins[3];
  std::vector<SvOp> sv_ops[3];
  SvOp* d_sv_ops[3] = {nullptr, nullptr, nullptr};
  // the same windows with every step a plain op (ragged sets), on the device
  std::vector<SvWin> sv_wins_plain[3];
  std::vector<SvOp> sv_ops_plain[3];
  SvWin* d_sv_wins_plain[3] = {nullptr, nullptr, nullptr};
  SvOp* d_sv_ops_plain[3] = {nullptr, nullptr, nullptr};
  // fused in-place steps of every part and of the statevector schedule
  std::vector<FusedStep> fused;
  FusedStep* d_fused = nullptr;
  bool inserted_unitary = true;                   // every inserted operator K / sqrt(q) is unitary
  // light cone of doubled networks: gate_unitary[g] when the bare gate and every
  // operator its sites may insert are unitary (to kUnitaryTol)
  bool light_cone = false;
  int max_part_rank = 31;              // last batch's per-trajectory tensor rank before slicing
  std::vector<char> gate_unitary;
  // subtree reuse in the per-trajectory parts (launches shared by jobs that agree
  // on the sites absorbed so far)
  bool subtree_reuse = false;
  int sample_kernel = 0;               // 0: automatic lane-per-element sampling, 1: wavefront per element

  // measurement
  int profile = 0;                                // 1: time the MFMA join; 2: also single HBM sweep steps
  double join_ms = 0, sweep_ms = 0, join_flops = 0, sweep_bytes = 0, fused_bytes = 0;
  int64_t join_launches = 0, sweep_launches = 0;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> sweep_evs;   // recorded, not yet read
  // whole parts swept in LDS (part_vm_kernel): event time, launches, algorithmic flops
  double vm_ms = 0, vm_flops = 0;
  int64_t vm_launches = 0;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> vm_evs;      // recorded, not yet read
  // statevector gate windows (any profile level): event time, launches, algorithmic bytes
  double win_ms = 0, win_bytes = 0;
  int64_t win_launches = 0;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> win_evs;     // recorded, not yet read
};
// Reads and destroys the recorded window events (the stream has been synchronised).
ptsbe_status_t collect_window_events(Plan& p);

// planner.cpp
bool build_batch_plans(Plan& p, std::string& err);
// Batch table without network parts (statevector method).
void build_sv_batches(Plan& p);
// Gate windows of the statevector method: gates are packed greedily into
// windows of at most kFuseMax qubits (qubits 0..3 always included, so that the
// window's tile rows are 128-byte runs), a gate joining a window only when no
// earlier gate left out of it touches its qubits (so it commutes with all of
// them).  Fills p.sv_run, p.sv_segs, p.sv_win[*] and appends to p.fused.
void build_sv_schedule(Plan& p);
// Compact ops of every statevector window set (p.sv_wins, p.sv_ops), from the
// fused steps and clusters that build_sv_schedule made.
void build_sv_ops(Plan& p);
// Windows of at most wmax qubits and max_ops steps for the adjoint pass: the
// statevector schedule's steps packed as in build_sv_schedule, in circuit order,
// every step a plain op.
// Gate windows of at most wmax qubits the statevector schedule needs (needs sv_steps).
int count_sv_windows(const Plan& p, int wmax);
void build_adj_windows(const Plan& p, int wmax, int max_ops, std::vector<AdjWin>& wins, std::vector<AdjOp>& ops);
// Reorders each window's ops into groups of at most kAdjGroupMax ops on at most two
// tile positions (an op only moves past ops on other positions) and fills the
// windows' group ranges; slots follow the new order.
void build_adj_groups(std::vector<AdjWin>& wins, std::vector<AdjOp>& ops, std::vector<AdjGroup>& groups);

// kernels.hip: launchers (all asynchronous on `stream`)
struct GateCtx {
  const DeviceGate* gates;
  const int32_t* gate_site_list;
  const float2* site_ops;
  const uint8_t* kraus;     // [E][S]
  int32_t S, max_kraus;
  const float2* merged;     // [E][G][16] merged gates of every trajectory
  int32_t G;
};
// UPV merge (error injection) of every (trajectory, gate): merged[t][g] =
// (prod of the inserted operators of g's sites) . d_g, the shared default when
// all of g's sites take Kraus index 0.
hipError_t launch_upv_merge(GateCtx g, int64_t E, float2* merged, hipStream_t stream);

// Initial tensor of a resumed part: the parent element's tensor with some legs
// sliced to the job's prefix bits (Vprev == null: the scalar 1).
struct InitArgs {
  const float2* Vprev = nullptr;
  int64_t stride = 1;                 // entries per parent tensor
  const int32_t* parent = nullptr;    // [job] parent index into Vprev
  int r0 = 0;                         // rank of the initial tensor
  int nsl = 0;
  int pos[8] = {0, 0, 0, 0, 0, 0, 0, 0};   // sliced positions in the parent tensor (ascending)
  int q[8] = {0, 0, 0, 0, 0, 0, 0, 0};     // qubit whose prefix bit fixes each
};
// Run all steps of one part in LDS, up to 64 jobs per workgroup.
// jobs: traj of job = job_traj ? job_traj[job] : job0 + job; prefix words of job.
// peak: largest rank held in LDS; direct = 1: the last step (contracted legs <= 1,
// more new legs than contracted) writes its output to `out` in HBM, its rank may
// exceed peak.
hipError_t launch_part_vm(const AbsorbStep* d_steps, int n_steps, int peak, GateCtx g,
                          int64_t n_jobs, const int32_t* job_traj, int32_t traj_base,
                          const uint64_t* job_prefix, int NW, const InitArgs& init, float2* out,
                          int out_rank, int direct, hipStream_t stream);
hipError_t launch_init_gather(const InitArgs& init, int64_t n_jobs, const uint64_t* job_prefix, int NW,
                              float2* out, hipStream_t stream);
// One absorb step over all jobs in global memory.
hipError_t launch_absorb_global(const AbsorbStep& st, const AbsorbStep* d_st, GateCtx g,
                                int64_t n_jobs, const int32_t* job_traj, int32_t traj_base,
                                const uint64_t* job_prefix, int NW, const float2* A,
                                float2* C, hipStream_t stream);
hipError_t launch_fill_one(float2* buf, int64_t n, hipStream_t stream);
// A fused run of in-place steps on every job's tensor (rank seg.r), in place.
hipError_t launch_fused(const Segment& seg, const FusedStep* d_fs, GateCtx g, int64_t n_jobs,
                        const int32_t* job_traj, int32_t traj_base, const uint64_t* job_prefix, int NW,
                        float2* A, hipStream_t stream,
                        const float2* Ucl = nullptr, int n_cl = 0);
// Gate-cluster matrices of a window set for n_jobs trajectories: Ucl[job][c][16 x 16]
// = the product of cluster c's gates (merged operands of the job's trajectory).
hipError_t launch_cluster_build(const ClusterDesc* d_cl, int n_cl, const FusedStep* d_fused, GateCtx g, int64_t n_jobs,
                                const int32_t* job_traj, int32_t traj_base, float2* Ucl, hipStream_t stream);

struct JoinArgs {
  const float2* V; int64_t v_stride;     // per element
  const float2* T; int64_t t_stride;     // per trajectory (indexed traj - traj_base, or its slot)
  const int32_t* elem_traj; int32_t traj_base;
  const int32_t* tslot;                  // slot of T of each trajectory (traj - traj_base), or null
  int64_t n_elems;
  int xb_bits, lk_bits, xT_bits;
  const int64_t* tab;                    // plan table base
  Plan::JoinDev jd;
  int b;                                 // output has 2^b entries per element
  int doubled;
  float* pop;                            // [n_elems][2^b] (population out) or null
  float2* amp;                           // [n_elems][2^b] (amplitude out) or null
};
hipError_t launch_join(const JoinArgs& a, hipStream_t stream);
// Last-batch join as an HBM-bound GEMV on the right part's own layout (no
// canonical copy): for elements of at most 4 rows and at least 256 values of x.
inline bool ketjoin_gemv_supported(int xb_bits, int lk_bits, int xT_bits) {
  // ketjoin_gemv_kernel (k <= 64), or the tiled kernel (k in LDS chunks, x >= 2^12)
  return (xb_bits <= 2 && lk_bits <= 6 && xT_bits >= 8) || (xb_bits <= 1 && lk_bits <= 12 && xT_bits >= 12);
}
hipError_t launch_ketjoin_gemv(const JoinArgs& a, hipStream_t stream);
// Tiling of the GEMV join over x when T's x bits are scattered (xT >= 12): a
// workgroup takes 4096 values of x spanned by 12 tile bits, chosen as the x bits
// of smallest offset in T (reads) together with those of smallest offset in the
// output (writes); the remaining x bits enumerate the tiles.
struct GemvTiling {
  int64_t t_off[12];     // T offset of tile bit s, s in read order (ascending T offset)
  int32_t w_of[12];      // write-order index of tile bit s
  int64_t o_off[12];     // output offset of tile bit q, q in write order (ascending output offset)
  int64_t o_read[12];    // output offset of tile bit s, s in read order
  int32_t n_hi;          // x bits outside the tile
  int64_t t_hi[32], o_hi[32];
};
bool make_gemv_tiling(const BatchPlan& bp, GemvTiling& g);
// GEMV join when the lowest T offsets belong to crossing wires (k): the 6 bits
// of smallest T offset, x or k, go on the lanes of a wavefront (its reads are
// then contiguous), each lane sums its k values over the k bits off the lanes,
// and the lanes of one x are summed by shuffles.  A wavefront takes one value
// of the x bits off the lanes at a time.
struct GemvLanes {
  int64_t lane_toff[6];  // T offset of lane bit i (the six smallest offsets)
  int64_t lane_ooff[6];  // output offset of lane bit i when it is an x bit, else 0
  int32_t lane_kbit[6];  // k value of lane bit i when it is a k bit, else 0
  int32_t lane_is_k[6];
  int32_t n_hx, n_hk;    // x and k bits off the lanes
  int64_t hx_toff[32], hx_ooff[32];
  int64_t hk_toff[12];
  int32_t hk_kbit[12];
};
// false unless a k bit has the smallest T offset (the tiled GEMV serves the rest)
bool make_gemv_lanes(const BatchPlan& bp, GemvLanes& g);
hipError_t launch_ketjoin_gemv_lanes(const JoinArgs& a, const GemvLanes& g, hipStream_t stream);
hipError_t launch_ketjoin_gemv_tiled(const JoinArgs& a, const GemvTiling& g, hipStream_t stream);
struct QformArgs {
  const float2* V; int64_t v_stride; int64_t v_base;   // V rows of elements [v_base, ...)
  const float2* Tc;                                     // canonical [traj][x][k][k'] (split join, ket join)
  const float* Th;                                      // Theta [traj][x][K^2] (FP32), or its bf16 hi plane
  int64_t th_plane;                                     // split join: 16-bit elements from the hi to the lo plane
  const int32_t* th_scale;                              // fp16 split: Theta exponent per (trajectory slot, x)
  int32_t traj_base;                                    // Tc index = traj - traj_base (or its slot)
  const int32_t* tslot;                                 // slot of each trajectory's Tc / Theta, or null
  int32_t traj0;                                        // trajectory of grid.y == 0
  const int32_t* first;                                 // [E+1] first element of each trajectory
  int64_t e_lo, e_hi;                                   // element range of this launch
  int xb_bits, lk_bits, xT_bits, b;
  const int64_t* tab; Plan::JoinDev jd;
  float* pop;                                           // [elements - v_base][2^b] or null
  float2* amp;                                          // ket join only: amplitudes or null
};
hipError_t launch_permute_T(const float2* T, int64_t t_stride, int64_t n_traj, const int64_t* tab,
                            const Plan::JoinDev& jd, int xT_bits, int lk_bits, int lb_bits, float2* Tc,
                            hipStream_t stream);
bool qform_supported(int lk_bits);
// Theta layout of the doubled join (FP32 MFMA path): bytes per trajectory
size_t qform_theta_bytes(int xT_bits, int lk_bits);
hipError_t launch_theta_T(const float2* T, int64_t t_stride, int64_t n_traj, const int64_t* tab,
                          const Plan::JoinDev& jd, int xT_bits, int lk_bits, float* Th, int split,
                          hipStream_t stream);
bool ketjoin_supported(int lk_bits);
bool qform_split_supported(int lk_bits);
// split-precision slot GEMM (bf16 hi + lo, three products, FP32 accumulate) of the doubled join
hipError_t launch_qform_split(const QformArgs& a, int n_traj, int max_rows, bool f16, hipStream_t stream);
hipError_t launch_qform(const QformArgs& a, int n_traj, int max_rows, hipStream_t stream);
hipError_t launch_ketjoin(const QformArgs& a, int n_traj, int max_rows, hipStream_t stream);
hipError_t launch_row_totals(const float* pop, int64_t n_elems, int b, double* totals,
                             hipStream_t stream);

struct SampleArgs {
  const float* pop; int b; int start; int NW;
  int64_t n_elems;
  const int32_t* elem_traj;
  const int32_t* elem_shot_off; const int32_t* elem_shot_cnt;
  const int32_t* shot_ids;               // shots grouped by element (global rows)
  const int64_t* traj_shot_base;         // [E] first global row of each trajectory
  uint64_t seed; int j;
  uint64_t* shots;                       // [M][NW]
  int32_t* shot_x;                       // [M] batch value of each shot (by row)
  double* elem_total;                    // [n_elems]
  int32_t* child_cnt;                    // [n_elems] or null
  int32_t* bad_flag;                     // set to 1 on a zero / non-finite total
  uint32_t tag = 2u;                     // Philox stream: 2 shot draws, 3 non-proportional draws
  double* p_cond = nullptr;              // [rows] P(x | prefix) of each draw (direct final batch), or null
  int lane_path = 0;                     // b <= 5 and about one shot per element: one lane per element
};
hipError_t launch_sample(const SampleArgs& a, hipStream_t stream);

// Sliced last batch: dst[i] = src[i] (zero when src is null) with `bits` OR'ed
// into word wi of each of the n rows of NW words; acc[i] += amp[i]; pop[i] = |acc[i]|^2.
hipError_t launch_prefix_or(const uint64_t* src, uint64_t* dst, int64_t n, int NW, int wi, uint64_t bits,
                            hipStream_t stream);
hipError_t launch_amp_accumulate(float2* acc, const float2* amp, int64_t n, hipStream_t stream);
hipError_t launch_amp_population(const float2* acc, float* pop, int64_t n, hipStream_t stream);

// Non-proportional NBS (Sec. III-B): element e of a non-final batch takes
// `draws` fresh draws on the rows [e * draws, (e + 1) * draws); traj_base[t] is
// the first row of trajectory t's elements, so a draw's Philox counter is the
// element's rank within its trajectory times `draws` plus the draw index.
// Elements of a trajectory range [t0, t0 + count): one per trajectory, empty prefix.
hipError_t launch_np_init(int64_t count, int64_t t0, int32_t* elem_traj, uint64_t* elem_prefix, int NW,
                          hipStream_t stream);
// Direct final-batch sampling: rows [e * draws, (e + 1) * draws) start as element
// e's prefix bits (the draw ORs its batch bits in) with its trajectory; after the
// draws, p(prefix) = Z_e / Z_t (1 without traj_norm; 0 for Z_e = 0).
hipError_t launch_np_direct_rows(int64_t n_elems, int draws, const int32_t* elem_traj, const uint64_t* elem_prefix,
                                 int NW, uint64_t* bits, int32_t* row_traj, hipStream_t stream);
hipError_t launch_np_direct_prefix_p(int64_t n_elems, int draws, const int32_t* elem_traj, const double* elem_total,
                                     const double* traj_norm, double* p_prefix, hipStream_t stream);
hipError_t launch_np_rows(int64_t n_elems, int draws, const int32_t* elem_traj, int32_t* shot_off,
                          int32_t* shot_cnt, int32_t* shot_ids, int64_t* traj_base, hipStream_t stream);

// Exhaustive final-batch sampling (Sec. III-B): one row for every x whose
// conditional P(x | prefix) = pop(x) / Z_e is strictly above the threshold, in
// element order then x ascending.  Work unit: (element, tile of kExhTile values).
constexpr int kExhTile = 4096;
struct ExhArgs {
  const float* pop; int b; int start; int NW;
  int64_t n_elems;
  const int32_t* elem_traj; const uint64_t* elem_prefix;
  const double* elem_total;              // [n_elems] Z_e
  const double* traj_norm;               // [E] squared norm of each trajectory
  double threshold;
  int32_t* tile_cnt;                     // [n_elems << tile_bits] rows per tile
  const int32_t* tile_off;               // exclusive scan of tile_cnt
  int tile_bits;                         // log2 tiles per element
  int64_t row_base, capacity;            // rows at or beyond capacity are not written
  double* totals_out;                    // [n_elems] copy of Z_e (null: none)
  uint64_t* bits; int32_t* row_traj; double* p_cond; double* p_prefix;   // any of the last three may be null
};
hipError_t launch_exh_count(const ExhArgs& a, hipStream_t stream);
hipError_t launch_exh_write(const ExhArgs& a, hipStream_t stream);

struct ChildArgs {
  int32_t* out_parent;                   // [children] index of the parent element
  int64_t n_elems; int b; int start; int NW;
  const int32_t* elem_traj; const uint64_t* elem_prefix;
  const int32_t* elem_shot_off; const int32_t* elem_shot_cnt;
  const int32_t* shot_ids; const int32_t* shot_x;
  const int32_t* child_off;
  int32_t* out_traj; uint64_t* out_prefix; int32_t* out_shot_off; int32_t* out_shot_cnt;
  int32_t* out_shot_ids;
  int lane_path = 0;                     // b <= 5 and about one shot per element: one lane per element
};
hipError_t launch_children(const ChildArgs& a, hipStream_t stream);

// exclusive scan of n int32 values into int32 out, total written to *d_total
hipError_t launch_scan_i32(const int32_t* in, int32_t* out, int64_t n, int32_t* d_total,
                           int32_t* d_scratch, hipStream_t stream);
size_t scan_scratch_bytes(int64_t n);

struct WeightArgs {
  const double* norms; const int64_t* mult; int64_t E;
  double* weights; double* norm_out;
};
hipError_t launch_weights(const WeightArgs& a, hipStream_t stream);
hipError_t launch_init_elements(int64_t E, const int64_t* shots_per_traj, int32_t* elem_traj,
                                uint64_t* elem_prefix, int NW, int32_t* shot_off,
                                int32_t* shot_cnt, int64_t* traj_shot_base, int32_t* shot_ids,
                                int32_t* shot_traj, uint64_t* shots, int64_t M,
                                hipStream_t stream);
// Shot rows only: ids = identity, shots zeroed, row -> trajectory.
hipError_t launch_init_shots(int64_t M, int64_t E, const int64_t* traj_shot_base, int32_t* shot_ids,
                             int32_t* shot_traj, uint64_t* shots, int NW, hipStream_t stream);
hipError_t launch_traj_ranges(const int32_t* elem_traj, int64_t n_elems, int64_t E,
                              int32_t* traj_first, hipStream_t stream);

// ---------------------------------------------------------------- adjoint pass
struct GradGateArgs {
  GateCtx g;
  int64_t E;
  const int32_t* gate_param;   // [G] parameter index or -1
  const int32_t* gate_axis;    // [G]
  const int32_t* gate_slot;    // [G] index among parameterised gates or -1
  int n_slots;
  const double* theta;
  float2* merged;              // [E][G][16] A = S . U
  float2* dagger;              // [E][G][16] A^dag
  float2* dmerged;             // [E][n_slots][16] S . dU/dtheta
};
hipError_t launch_grad_gates(const GradGateArgs& a, hipStream_t stream);
hipError_t launch_state_init(float2* psi, int64_t n_jobs, int n, hipStream_t stream);
// One statevector gate window on the n-qubit states of n_jobs trajectories
// (trajectory traj_base + job), in place: every 2^np tile is loaded into LDS,
// the window's ops are applied there and the tile is written back.  Gate
// matrices come from merged ([E][G][16]); cluster matrices from
// Ucl[job][n_cl_total][256].  precision: PTSBE_C64 (FP32 MFMA for clusters) or
// PTSBE_SPLIT_BF16 / _F16 (clusters with hi + lo 16-bit operands, three products,
// FP32 accumulation).
hipError_t launch_sv_window(const SvWin& w, const SvOp* d_ops, const float2* merged, int G, const float2* Ucl,
                            int n_cl_total, int64_t n_jobs, int32_t traj_base, float2* psi, int n, int precision,
                            hipStream_t stream);
// LDS bytes the window kernel needs for a window (0 if it cannot take it).
size_t sv_window_lds_bytes(const SvWin& w);
hipError_t launch_copy(const float2* src, float2* dst, int64_t n, hipStream_t stream);
// dst row j (2^row_bits entries) = src row idx[j], for n_rows rows.
hipError_t launch_gather_rows(const float2* src, const int32_t* idx, float2* dst, int64_t n_rows, int row_bits,
                              hipStream_t stream);
hipError_t launch_value_sum(const double* vals, const double* w, int64_t E, double* out, hipStream_t stream);

// ---------------------------------------------------------- statevector method
// Marginal of batch qubits [start, start + b) of each element (trajectory,
// prefix bits of qubits < start) from its trajectory's statevector:
// part[e][s][x] = sum over later-qubit values y in slice s of |psi(y, x, prefix)|^2
// (FP64 sums), then pop[e][x] = sum_s part[e][s][x] in slice order (FP32 out).
struct SvMargArgs {
  const float2* psi;                 // [traj - traj_base][2^n]
  int n, start, b, NW;
  int64_t n_elems;
  const int32_t* elem_traj; int32_t traj_base;
  const uint64_t* elem_prefix;       // [n_elems][NW] (bits of qubits < start used)
  int log_split;                     // later-qubit values split into 2^log_split slices
  double* part;                      // [n_elems][2^log_split][2^b]
  int64_t part_rows = 0;             // capacity of part in rows of 2^b (checked at launch)
  float* pop;                        // [n_elems][2^b]
};
hipError_t launch_sv_marginal(const SvMargArgs& a, hipStream_t stream);
// Amplitudes of the last batch: amp[e][x] = psi(x, prefix) (no later qubits).
hipError_t launch_sv_amplitudes(const SvMargArgs& a, float2* amp, hipStream_t stream);
// Elements of a trajectory range [t0, t0 + count): one element per trajectory.
// statevector method drivers (sv.cpp)
ptsbe_status_t sv_evolve(Plan& p, const GateCtx& g, int64_t t0, int64_t nj, float2* psi, float2* Ucl,
                         hipStream_t s);
size_t sv_sample_workspace(const Plan& p, int64_t E, int64_t M);
size_t sv_np_workspace(const Plan& p, int64_t E, int64_t cap, int32_t rows_per_elem);
ptsbe_status_t sv_sample_nonproportional(Plan& p, const uint8_t* d_kraus, int64_t E, const int64_t* d_mult,
                                         int32_t draws, int32_t final_draws, int64_t cap, uint64_t seed,
                                         double threshold, uint64_t* d_bits, int32_t* d_row_traj, double* d_p_cond,
                                         double* d_p_prefix, int64_t capacity, int64_t* n_rows_out, double* d_w,
                                         double* d_norm, int64_t* stats, void* d_workspace, size_t workspace_bytes,
                                         hipStream_t s);
size_t sv_contract_workspace(const Plan& p, int j, int64_t E, int64_t n_elems);
ptsbe_status_t sv_sample_shots(Plan& p, const uint8_t* d_kraus, int64_t E, const int64_t* d_mult,
                               const int64_t* d_m, uint64_t seed, uint64_t* d_shots, int32_t* d_shot_traj,
                               double* d_w, double* d_norm, int64_t* stats, void* d_workspace,
                               size_t workspace_bytes, hipStream_t s);
ptsbe_status_t sv_contract_batch(Plan& p, int j, const uint8_t* d_kraus, int64_t E, const int32_t* d_elem_traj,
                                 const uint64_t* d_elem_prefix, int64_t n_elems, int32_t out_kind, void* d_out,
                                 double* d_elem_total, void* d_workspace, size_t workspace_bytes, hipStream_t s);
hipError_t launch_init_traj_range(int64_t t0, int64_t count, const int64_t* shots_per_traj,
                                  const int64_t* traj_shot_base, int32_t* elem_traj, uint64_t* elem_prefix,
                                  int NW, int32_t* shot_off, int32_t* shot_cnt, hipStream_t stream);

// ------------------------------------------------------------------ ragged sets
constexpr int kRgMaxBatches = kSvMaxQubits;
constexpr int kRgThreads = 256;
struct RgWindow {                    // one gate window of a statevector plan
  int32_t np, n_fs;
  int32_t P[kFuseMax];
  int64_t fused_off;
};
struct RgPiece {                     // trajectories [t0, t0 + nj) of one job inside a wave
  GateCtx g;                         // kraus / merged of the piece (local trajectory index)
  const RgWindow* win;               // the plan's windows (device)
  const SvWin* swin;                 // the same windows as plain compact ops (device), or null
  const SvOp* sops;
  const FusedStep* fused;            // the plan's fused steps (device)
  float2* psi;                       // [nj][2^n]
  uint64_t* shots;                   // the job's shot rows (device, one word per row)
  double* norms;                     // [E] the job's squared norms (workspace)
  int64_t row0;                      // first wave row of the piece
  int64_t job_row0;                  // the same row in the job's shot array
  int64_t part_off;                  // first-batch partial sums: first row
  uint64_t seed;
  int32_t job, n, f, n_win;
  int32_t t0, nj, traj_off;          // job trajectory range, first wave trajectory
  int32_t log_split0;                // slices per trajectory of the first-batch marginal
  int32_t start[kRgMaxBatches], b[kRgMaxBatches];
};
struct RgWave {                      // device arrays of one wave (all in the workspace)
  const RgPiece* pieces; int32_t n_pieces;
  const int32_t* traj_piece;         // [T] piece of every wave trajectory
  const int64_t* traj_row0;          // [T + 1] first wave row of every trajectory
  int32_t T; int64_t R;              // trajectories, shot rows
  int32_t xbits;                     // populations are stored with stride 2^xbits
  int32_t* el_wt[2]; uint64_t* el_prefix[2]; int32_t* el_off[2]; int32_t* el_cnt[2];
  int32_t* ids[2]; int32_t* shot_x;
  int32_t* child_cnt; int32_t* child_off; int32_t* scan_sums;
  int32_t* counts;                   // [kRgMaxBatches + 1] elements per batch level (device)
  int64_t cap;                       // element capacity
  float* pop; double* part;
  const int64_t* m0_start;           // [n_pieces + 1] first-batch marginal tasks per piece
  uint64_t* done;                    // [n_jobs + 1] completion stamps or null
  int32_t* bad_flag;
  int32_t n_jobs;
};
// window level l: entries (piece, first task) of the pieces with more than l windows
struct RgLevel { const int32_t* piece; const int64_t* start; int32_t n; int64_t tasks; int32_t max_ops; };
hipError_t launch_rg_start(const RgWave& w, hipStream_t s);
hipError_t launch_rg_prepare(const RgWave& w, int grid, hipStream_t s);
// grid: n_cu times the kernel's occupancy per CU
hipError_t launch_rg_window(const RgWave& w, const RgLevel& lv, int level, int n_cu, hipStream_t s);
hipError_t launch_rg_marginal0(const RgWave& w, int64_t tasks, int grid, hipStream_t s);
hipError_t launch_rg_marginal(const RgWave& w, int j, int cur, int grid, hipStream_t s);
hipError_t launch_rg_sample(const RgWave& w, int j, int cur, int grid, hipStream_t s);
hipError_t launch_rg_scan(const RgWave& w, int j, hipStream_t s);
hipError_t launch_rg_children(const RgWave& w, int j, int cur, int grid, hipStream_t s);

}  // namespace ptsbe
