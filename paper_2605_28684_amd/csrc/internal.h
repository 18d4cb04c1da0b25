// Internal declarations of the romhip library: the batch handle, launch helpers
// and the kernel launchers each translation unit provides.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/romhip.h"

namespace romhip {

void set_error(const std::string& msg);

#define ROM_HIP_CHECK(expr)                                                        \
  do {                                                                             \
    hipError_t _e = (expr);                                                        \
    if (_e != hipSuccess) {                                                        \
      ::romhip::set_error(std::string(#expr) + ": " + hipGetErrorString(_e));     \
      return ROM_E_DEVICE;                                                         \
    }                                                                              \
  } while (0)

#define ROM_TRY(x)                 \
  do {                             \
    rom_status _s = (x);           \
    if (_s != ROM_OK) return _s;   \
  } while (0)

#define ROM_REQUIRE(cond, code, msg)      \
  do {                                    \
    if (!(cond)) {                        \
      ::romhip::set_error(msg);           \
      return code;                        \
    }                                     \
  } while (0)

constexpr int kTile = 256;          // cells per tile of the stencil kernels
constexpr int kPassRows = 2048;     // basis rows per block of the tall-skinny passes
constexpr int kMaxR = 64;           // largest reduced dimension supported
constexpr int kMaxNs = 2 * kMaxR;   // largest number of DEIM rows
constexpr int kPhibarPending = 6;   // Phibar terms the online adjoint keeps for one pass

// Position of element (i, j) of one tile's r x r block of Phi^T J_f Phi in the
// partials the FP32 MFMA pass writes for r = 32.  The single-wave solve keeps
// row i, columns of parity h, in lane i + 32 h (column j in register j >> 1);
// this order hands each lane its 16 values as four float4 loads, load u of
// the wave reading 1 KB contiguous (registers 4u .. 4u + 3 of every lane).
__host__ __device__ constexpr int mpart_pos32(int i, int j) {
  return (((j >> 1) >> 2) * 64 + i + 32 * (j & 1)) * 4 + ((j >> 1) & 3);
}

// A contiguous run of cells of one instance handled by one thread block.
struct Tile {
  int32_t inst;
  int32_t pad;
  int64_t cell0;   // first cell (instance-local)
  int64_t ncell;   // number of cells in the tile
  int64_t n;       // cells of the instance
  int64_t base;    // first DOF of the instance in the batch
};

constexpr int kBigTile = 1024;      // cells per block of the streaming Euler residual

// Workspace of the batched thin SVD of N x w column matrices (CGS2-QR, then the
// SVD of R): Q T[total_dof * wmax], R and U [n_inst * wmax^2], the per-instance
// reductions and projection coefficients.
struct PodWs {
  void* Q = nullptr;
  double* R = nullptr;
  double* U = nullptr;
  double* red = nullptr;
  double* pr = nullptr;
  int wmax = 0;
};

// One level of the recursive block-tridiagonal (Schur complement) solver.
struct BtLevel {
  int64_t n_total = 0;            // cells at this level, all instances
  int64_t parts_total = 0;        // parts at this level, all instances
  std::vector<int64_t> cell_off;  // [n_inst+1]
  std::vector<int64_t> part_off;  // [n_inst+1]
  int64_t* d_cell_off = nullptr;
  int64_t* d_part_off = nullptr;
  void* sys = nullptr;    // A,B,C (nv*nv each) and d (nv) per cell
  void* fwd = nullptr;    // Chat, Vhat (nv*nv each) and ghat (nv) per cell
  void* part = nullptr;   // What_last, V_first, W_first (nv*nv) and g_first (nv) per part
  void* x = nullptr;      // solution per cell (nv)
};

// Cross-lane exchanges without LDS, for wave-wide reductions that must add or
// compare exactly the pairs a shuffle-xor butterfly would.  The 64-bit value
// of lane l ^ 32 and of lane l ^ 16 come from the VALU permutes of gfx950
// (v_permlane32_swap: with both operands x, the first result holds the low
// half's copy and the second the high half's; v_permlane16_swap: the first
// result holds rows 0, 0, 2, 2 and the second rows 1, 1, 3, 3).  The other
// offsets are DPP moves within 16-lane rows.
__device__ __forceinline__ double bfly_join(unsigned lo, unsigned hi) {
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}
__device__ __forceinline__ double bfly_xor32(double v) {
  const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
  const auto lo = __builtin_amdgcn_permlane32_swap((unsigned)u, (unsigned)u, false, false);
  const auto hi = __builtin_amdgcn_permlane32_swap((unsigned)(u >> 32), (unsigned)(u >> 32), false,
                                                   false);
  return (__lane_id() & 32) ? bfly_join(lo[0], hi[0]) : bfly_join(lo[1], hi[1]);
}
__device__ __forceinline__ double bfly_xor16(double v) {
  const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
  const auto lo = __builtin_amdgcn_permlane16_swap((unsigned)u, (unsigned)u, false, false);
  const auto hi = __builtin_amdgcn_permlane16_swap((unsigned)(u >> 32), (unsigned)(u >> 32), false,
                                                   false);
  return (__lane_id() & 16) ? bfly_join(lo[0], hi[0]) : bfly_join(lo[1], hi[1]);
}
template <int CTRL>
__device__ __forceinline__ double bfly_dpp(double v) {
  const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
  return bfly_join((unsigned)__builtin_amdgcn_mov_dpp((int)(unsigned)u, CTRL, 0xF, 0xF, false),
                   (unsigned)__builtin_amdgcn_mov_dpp((int)(unsigned)(u >> 32), CTRL, 0xF, 0xF,
                                                      false));
}

// The wave sum of v in every lane, with the additions of a shuffle-xor
// butterfly over offsets 32, 16, 8, 4, 2, 1, in that order, so bit for bit its
// result.  row_ror:8 is lane ^ 8; after the first three stages a lane's value
// depends only on its index mod 8, where row_ror:4 equals lane ^ 4; the quad
// permutes are lane ^ 2 and lane ^ 1.  Every lane of the wavefront must be
// active.
__device__ __forceinline__ double wave_sum_bfly(double v) {
  v += bfly_xor32(v);
  v += bfly_xor16(v);
  v += bfly_dpp<0x128>(v);   // row_ror:8
  v += bfly_dpp<0x124>(v);   // row_ror:4
  v += bfly_dpp<0x4E>(v);    // quad_perm [2,3,0,1]
  v += bfly_dpp<0xB1>(v);    // quad_perm [1,0,3,2]
  return v;
}

// The wave maximum of v in every lane (v never NaN; every lane active).
__device__ __forceinline__ double wave_max_bfly(double v) {
  double o = bfly_xor32(v);
  v = o > v ? o : v;
  o = bfly_xor16(v);
  v = o > v ? o : v;
  o = bfly_dpp<0x128>(v);
  v = o > v ? o : v;
  o = bfly_dpp<0x124>(v);
  v = o > v ? o : v;
  o = bfly_dpp<0x4E>(v);
  v = o > v ? o : v;
  o = bfly_dpp<0xB1>(v);
  return o > v ? o : v;
}

// Max of v over the 64 lanes of a wavefront, then one atomicMax into *dst from
// lane 0.  Every lane of the wavefront must call it with the same dst.
__device__ __forceinline__ void wave_atomic_max(uint64_t* dst, uint64_t v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const uint64_t o = __shfl_xor((unsigned long long)v, off);
    v = o > v ? o : v;
  }
  if ((threadIdx.x & 63) == 0 && v) atomicMax((unsigned long long*)dst, (unsigned long long)v);
}

}  // namespace romhip

struct rom_batch {
  rom_config cfg{};
  std::vector<int64_t> n_cells;
  std::vector<double> phys;
  int nv = 1;
  size_t esz = 4;                 // bytes per bulk element
  int64_t total_cells = 0, total_dof = 0;
  std::vector<int64_t> dof_off, cell_off;
  int64_t max_dof = 0;

  // device layout
  int64_t* d_dof_off = nullptr;
  int64_t* d_cell_off = nullptr;
  double* d_phys = nullptr;
  romhip::Tile* d_tiles = nullptr;
  int n_tiles = 0;
  int* d_tile_first = nullptr;       // first cell tile of each instance [n_inst+1]
  romhip::Tile* d_btiles = nullptr;  // kBigTile-cell tiles
  int n_btiles = 0;
  romhip::Tile* d_btiles2 = nullptr; // kBigTile/2-cell tiles
  int n_btiles2 = 0;
  int n_cu = 256;                    // compute units of the device
  int device = 0;                    // HIP device the handle was created on
  int tune_residual = 0;             // chosen launch shape of the streaming residual
  int deim_split = 4;                // candidate rows per pass tile of the greedy DEIM pass
  int bt_m_req = 0;                  // requested solver part size (0: the default)
  romhip::Tile* d_ptiles = nullptr;  // row tiles of kPassRows basis rows
  int n_ptiles = 0;
  std::vector<int> ptile_first;      // first row tile of each instance [n_inst+1]
  int* d_ptile_first = nullptr;

  // reduced state
  void* Phi = nullptr;       // T[total_dof * r]
  double* sigma = nullptr;   // [n_inst * r]
  double* a = nullptr;       // [n_inst * r]
  double* a_prev = nullptr;  // [n_inst * r]
  void* q_ref = nullptr;     // T[total_dof]
  double* d_var = nullptr;   // [n_inst * nv]
  void* y_corr = nullptr;    // T[total_dof]
  uint32_t* flags = nullptr; // [n_inst]
  int32_t* P = nullptr;      // [n_inst * n_s]
  double* M = nullptr;       // [n_inst * r * n_s]
  void* mesh_phi = nullptr;    // T[n_inst * n_s * 3 * nv * r]: the bulk precision (values of Phi)
  double* mesh_qref = nullptr; // [n_inst * n_s * 3 * nv]
  double* mesh5_phi = nullptr;  // [n_inst * n_s * 5 * nv * r]: five-cell mesh (explicit scheme)
  double* mesh5_qref = nullptr; // [n_inst * n_s * 5 * nv]
  uint32_t* chosen = nullptr;  // [total_dof] epoch marks for DEIM
  void* phi_cm = nullptr;      // T[total_dof * r]: Phi by columns per instance (DEIM only)
  double* hr_as = nullptr;     // [n_inst * (n_s + r) * (r + 1)]: rows of [A_s | b], then [M A_s | -M b] (DEIM only)
  uint32_t deim_epoch = 0;
  double* qdeim_q = nullptr;   // [n_inst * kMaxR * kMaxR] QDEIM's orthonormal directions (QDEIM only)
  double* fgs_g = nullptr;     // [total_cells] squared feature gradient (feature-guided sampling)

  // iSVD workspace
  double* part = nullptr;    // block partial sums [n_ptiles * (r*r + 2r + 4)]
  double* red = nullptr;     // per-instance reductions [n_inst * (3r + 8)]
  double* ubar = nullptr;    // core left singular vectors [n_inst * (r+1)*(r+1)]
  double* lmat = nullptr;    // re-orth factor [n_inst * r * r]
  int32_t* active = nullptr; // per-instance Newton activity [n_inst]
  int32_t* iters = nullptr;  // per-instance Newton counters [n_inst]
  uint64_t* norms = nullptr; // Newton norms: 3 blocks of (newton_max+1) x n_inst (residual, iterate, update)
  double* rstate = nullptr;  // reduced Newton workspace [n_inst * (r*r + 4r)]
  double* qtmp = nullptr;    // first Gram-Schmidt residual [total_dof] (FP64)
  void* mpart_tap = nullptr; // when set: receives a copy of mpart after a Galerkin step's first pass
  void* mpart = nullptr;     // Galerkin block partials of Phi^T J Phi [n_ptiles * kMaxR^2] (T;
                             // mpart_pos32 order when the FP32 MFMA pass wrote them for r = 32)
  double* epart = nullptr;   // projection partials of the event chain [n_ptiles * kMaxR^2]
  int32_t* ev_iters = nullptr; // Newton counters of the event's coarse step [n_inst]
  uint32_t* d_epoch = nullptr; // DEIM epoch counter (device)

  // full-order Newton workspace
  void* fq = nullptr;        // T[total_dof] current iterate
  void* fq_prev = nullptr;   // T[total_dof]
  std::vector<romhip::BtLevel> levels;
  int bt_m = 16;                      // part size of the block-tridiagonal solver
  void* vjp_tmp = nullptr;   // T[total_dof]
  void* rvjp = nullptr;      // rollout-adjoint checkpoints and segment states
  size_t rvjp_bytes = 0;

  // windowed basis update rules (App. A)
  void* win = nullptr;         // T[window * total_dof] raw correction snapshots (ring)
  int win_count = 0;           // snapshots held
  int win_head = 0;            // next slot written
  double* lift = nullptr;      // [total_dof] Phi a before the update (FP64)
  romhip::PodWs podws;         // thin-SVD workspace (wmax = max(window, r))
  double* zmat = nullptr;      // [n_inst * 64 * (r+1)] Z = Phi^T Y by columns (Direct)
  double* zpinv = nullptr;     // [n_inst * 64 * r] Z^+ (Direct)
  void* phit = nullptr;        // T[r * total_dof] Y Z^+ by columns (Direct)
  double* sig_scratch = nullptr; // [n_inst * r] singular values of Y Z^+ (Direct)

  // host counters
  int64_t n_fine = 0;        // fine step index n of Alg. 1 (starts at w_init)
  int64_t n_update = 0;      // iSVD updates done
  int64_t n_events = 0;
  int64_t n_reorth = 0;
  bool has_rom = false;
  bool fom_block = false;          // backward-Euler steps run one workgroup per instance
  hipStream_t last_stream = nullptr;

  // graphs of one adaptation window
  // window graphs, one per basis buffer holding the current basis (the
  // overlapped window rotates into the other buffer)
  hipGraphExec_t win_exec[2] = {nullptr, nullptr};
  hipStream_t win_stream[2] = {nullptr, nullptr};
  void* Phi_alt = nullptr;     // T[total_dof * r]: second basis buffer (overlapped windows)
  void* phi_first = nullptr;   // the first basis allocation (identifies the buffer in use)
  // second stream of a window: the event's coarse step, projections and core
  // SVD run beside the fine steps (they share no written data)
  hipStream_t aux = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
};

namespace romhip {

// ---- residual.hip
rom_status launch_residual(rom_batch* h, const void* q, const void* q_prev, double dt, void* out,
                           hipStream_t s);
rom_status launch_residual_norm(rom_batch* h, const void* q, const void* q_prev, double dt,
                                void* out, int it, hipStream_t s);
rom_status launch_residual_vjp(rom_batch* h, const void* q, const void* q_prev, double dt,
                               const void* gbar, void* gq, void* gq_prev, hipStream_t s);
// assemble backward-Euler Newton system at level 0: -r and blocks of I - dt J_f
rom_status launch_assemble(rom_batch* h, const void* q, const void* q_prev, double dt, int it,
                           hipStream_t s);
// assemble the transposed Jacobian system with a given right-hand side (adjoint)
rom_status launch_assemble_adjoint(rom_batch* h, const void* q, double dt, const void* rhs,
                                   hipStream_t s);

// ---- btsolve.hip
rom_status bt_setup(rom_batch* h);
// part sizes the solver can use for nv-variable blocks (the first is the default)
int bt_part_candidates(int nv, int* out);
void bt_free(rom_batch* h);
// solve the level-0 system; it >= 0: Newton mode (skip inactive instances,
// converge check against norms[it]; add solution into q); it < 0: plain solve into out
rom_status bt_solve(rom_batch* h, int it, void* q_update, void* out, hipStream_t s);

// ---- isvd.hip
rom_status launch_isvd(rom_batch* h, const void* y, hipStream_t s);
// The two halves of launch_isvd: projections and core SVD (partials in part),
// then the state transfer and the basis rotation.
rom_status launch_isvd_core(rom_batch* h, const void* y, double* part, hipStream_t s);
rom_status launch_isvd_apply(rom_batch* h, hipStream_t s);
// launch_isvd_apply split for the overlapped window (MFMA path): rotation of
// the current basis into dst (out of place), then the state transfer.
rom_status launch_isvd_rotate_into(rom_batch* h, void* dst, hipStream_t s);
rom_status launch_isvd_transfer(rom_batch* h, hipStream_t s);
// Online-loop adjoint pieces (adjoint.hip): the loss seed at the end state,
// one fine step backward (after a Galerkin pass at its converged state), one
// event backward down to yhat, FP32/FP64 conversion of device vectors.
// With qrbar (FP64 [total_dof]) and dvbar (FP64 [n_inst * nv]) the seed and the
// event also give the gradients of q_ref and of D's diagonal per variable (the
// seed writes them, the event adds to them).
rom_status launch_online_seed(rom_batch* h, const void* qbar, double* abar, double* phibar,
                              hipStream_t s, double* qrbar = nullptr, double* dvbar = nullptr);
// one fine step backward with its Phibar terms kept as uv (the caller keeps
// lambda = abar and a1 beside it) for launch_phibar_flush, which applies K of
// them in one pass
rom_status launch_step_vjp_deferred(rom_batch* h, const void* Phi, const double* a1,
                                    double* abar, double2* uv, hipStream_t s,
                                    const void* mpart = nullptr);
rom_status launch_phibar_flush(rom_batch* h, int K, const double2* uv, const double* lam,
                               const double* a1, double* phibar, hipStream_t s);
rom_status launch_event_vjp(rom_batch* h, const void* Phi_old, const void* y_new,
                            const double* sig_old, const double* a_old, const double* ubar,
                            const double* pr, const double* sig_new, double* abar,
                            double* phibar, double* sigbar, double* ybar, double* qs, double* js,
                            double* evscr, hipStream_t s, double* qrbar = nullptr,
                            double* dvbar = nullptr, int* npend = nullptr, int kp = 0,
                            double2* puv = nullptr, double* plam = nullptr,
                            double* pa1 = nullptr);
// doubles of the event adjoint's scratch (per-tile partials, per-instance vectors)
size_t event_vjp_scratch_doubles(const rom_batch* h);
rom_status convert_words(const void* src, bool src_f64, void* dst, bool dst_f64, int64_t n,
                         hipStream_t s);
rom_status adjoint_kernels_prepare();
rom_status launch_reorth(rom_batch* h, hipStream_t s);
rom_status launch_pod(rom_batch* h, const void* Q, int w, hipStream_t s);  // Q: T[w * total_dof]
rom_status pod_ws_alloc(rom_batch* h, int wmax, PodWs* ws);
// the windowed basis update rules (App. A) of an adaptation event, and the
// window at the end of the offline stage
rom_status launch_windowed_update(rom_batch* h, const void* y, hipStream_t s);
rom_status launch_window_init(rom_batch* h, const void* Q, int w, hipStream_t s);
void pod_ws_free(PodWs* ws);
rom_status launch_preprocess(rom_batch* h, const void* q0, const void* Q, int w, hipStream_t s);
rom_status launch_project_state(rom_batch* h, const void* q, hipStream_t s);  // a = Phi^T D (q - q_ref)

// ---- rom.hip
rom_status launch_rom_fine_step(rom_batch* h, hipStream_t s);
// Whole-Newton-loop-per-workgroup backward-Euler step for batches of small
// scalar instances (see fomblock.hip); fom_block_ok tells whether it applies.
struct ResidualShape {
  int cpt;            // cells per thread (tile = 256 cpt cells)
  int blocks_per_cu;  // persistent grid = blocks_per_cu x compute units
  int nt;             // non-temporal loads / stores of the streamed state
};
int residual_shape_count(const rom_batch* h);
ResidualShape residual_shape(const rom_batch* h, int i);
bool fom_block_ok(const rom_batch* h);
rom_status launch_fom_block(rom_batch* h, const void* q_prev, double dt, void* q_out,
                            int32_t* iters, hipStream_t s);
rom_status prepare_galerkin_pass(rom_batch* h, hipStream_t s);
rom_status launch_galerkin_pass(rom_batch* h, hipStream_t s);  // one pass, every instance active
rom_status launch_isvd_project(rom_batch* h, const void* y, hipStream_t s);  // pass A only
rom_status launch_rebuild(rom_batch* h, hipStream_t s);
// ---- sample.hip: QDEIM picks (and feature-guided sampling) into P
rom_status launch_qdeim(rom_batch* h, hipStream_t s);
int fgs_feature(int problem);
rom_status launch_reconstruct(rom_batch* h, void* out, hipStream_t s);
rom_status rom_kernels_prepare();
rom_status isvd_kernels_prepare();

// ---- mfma.hip (FP32, r in {32, 64})
bool mfma_ok(const rom_batch* h);
// first: the first Newton iteration of a step (every instance runs)
rom_status launch_galerkin_mfma(rom_batch* h, hipStream_t s, int first = 0);
rom_status launch_galerkin_tail(rom_batch* h, int it0, hipStream_t s);
rom_status launch_rotate_mfma(rom_batch* h, const double* pr, void* dst, hipStream_t s);
rom_status launch_project_fast(rom_batch* h, const void* y, const double* p1, int ldp, int mode,
                               double* part, int pst, double* q1out, hipStream_t s);

// ---- explicit.hip: the SSPRK(4,3) path (limited second-order residual)
rom_status launch_residual2(rom_batch* h, const void* q, void* out, hipStream_t s);
// one SSPRK(4,3) full-order step; uses fq_prev, fq and vjp_tmp as stage buffers
rom_status fom_step_explicit(rom_batch* h, const void* q_prev, double dt, void* q_out,
                             hipStream_t s);
rom_status launch_mesh5(rom_batch* h, hipStream_t s);  // after every rebuild of P
rom_status launch_hr_explicit_step(rom_batch* h, hipStream_t s);
rom_status explicit_kernels_prepare();

// ---- the rollout adjoint (gradient with respect to q0 through Alg. 1)
// one HR-LSPG step backward with the window's P and M held fixed (rom.hip)
rom_status launch_hr_step_vjp(rom_batch* h, const void* Phi, const int32_t* P, const double* M,
                              const double* a1, double* abar, double* phibar, double* qrbar,
                              double* dvbar, hipStream_t s);
// the POD with a caller-owned workspace that keeps Q_pod and R (isvd.hip)
rom_status launch_pod_ws(rom_batch* h, const void* Q, int w, const PodWs& ws, hipStream_t s);
rom_status launch_pod_vjp_small(rom_batch* h, const double* R, int w, const double* Z,
                                const double* sigbar, double* Cm, double* Em, double* scr,
                                hipStream_t s);
// the offline stage backward (rollout.hip); part: offline_vjp_part_doubles
// doubles; small: n_inst (w r + w w + r w + 3 w w) doubles
size_t offline_vjp_part_doubles(const rom_batch* h, int w);
rom_status launch_offline_a_vjp(rom_batch* h, const void* Phi0, const void* qw, const double* abar,
                                double* phibar, double* qbw, double* qrbar, double* dvbar,
                                double* part, hipStream_t s);
rom_status launch_offline_pod_vjp(rom_batch* h, const PodWs& ws, int w, const void* Qtr,
                                  const double* phibar, const double* sigbar, double* qb,
                                  double* qrbar, double* dvbar, double* part, double* small,
                                  hipStream_t s);
rom_status add_to_double(rom_batch* h, const void* src, double* dst, hipStream_t s);
rom_status sum_to_state(rom_batch* h, const double* x, const double* y, void* out, hipStream_t s);

// ---- small helpers (api.cpp)
rom_status fill_zero(void* p, size_t bytes, hipStream_t s);

}  // namespace romhip
