// C interface of the romhip library: argument checking, batch layout, device
// allocation, the backward-Euler Newton driver and the Alg. 1 driver.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <string>

#include "internal.h"

// Device scratch of the entry points that allocate nothing
// (fom_rollout_vjp_noalloc): 32 MiB per device, held until the process ends.
static constexpr size_t kScratchBytes = size_t(32) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace romhip {

static thread_local std::string g_err;
void set_error(const std::string& msg) { g_err = msg; }

namespace {

__global__ void k_fill_u64(uint64_t* p, uint64_t v, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}
__global__ void k_fill_i32v(int32_t* p, int32_t v, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}
__global__ void k_fill_u32(uint32_t* p, uint32_t v, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}
__global__ void k_copy_bytes(const uint32_t* src, uint32_t* dst, int64_t nwords) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nwords) dst[i] = src[i];
}

// Newton bookkeeping.  norms holds three (newton_max+1) x n_inst blocks: the
// residual sup norm of each iterate (bits of a T), the iterate's sup norm
// (bits of a T) and the sup norm of each Newton update (bits of a double).
// Converged when ||r||_inf <= tol.  In single precision the residual of the
// rounded solution cannot go below about eps ||J_r|| ||y||, which exceeds an
// absolute tolerance on fine grids, so an FP32 iterate also counts as
// converged once the last update is at round-off level:
// ||delta||_inf <= 8 eps_32 (1 + ||y||_inf).
template <typename T>
__device__ __forceinline__ double bits_to(uint64_t v) {
  return sizeof(T) == 4 ? (double)__uint_as_float((uint32_t)v) : __longlong_as_double((long long)v);
}

template <typename T>
__device__ bool newton_converged(const uint64_t* norms, int it, int mx, int n_inst, int b,
                                 double tol) {
  const uint64_t rb = norms[(size_t)it * n_inst + b];
  if (rb != ~0ull && bits_to<T>(rb) <= tol) return true;
  if (sizeof(T) == 4 && it > 0) {
    const uint64_t db = norms[(size_t)(2 * (mx + 1) + it - 1) * n_inst + b];
    const int iy = it < mx ? it : it - 1;
    const double yn = bits_to<T>(norms[(size_t)(mx + 1 + iy) * n_inst + b]);
    const double dn = __longlong_as_double((long long)db);
    if (db != ~0ull && dn <= 8.0 * 1.1920928955078125e-07 * (1.0 + yn)) return true;
  }
  return false;
}

template <typename T>
__global__ void k_newton_decide(int n_inst, const uint64_t* norms, int it, int mx, double tol,
                                int32_t* active, int32_t* iters) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= n_inst || !active[b]) return;
  if (newton_converged<T>(norms, it, mx, n_inst, b, tol)) active[b] = 0;
  else iters[b] += 1;
}

template <typename T>
__global__ void k_newton_final(int n_inst, const uint64_t* norms, int mx, double tol,
                               const int32_t* active, uint32_t* flags) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= n_inst || !active[b]) return;
  if (!newton_converged<T>(norms, mx, mx, n_inst, b, tol))
    atomicOr(&flags[b], ROM_FLAG_NEWTON_NOCONV);
}

inline int nblk(int64_t n, int t = 256) { return (int)((n + t - 1) / t); }

rom_status copy_words(const void* src, void* dst, size_t bytes, hipStream_t s) {
  // device-to-device copy as a kernel (graph-safe; no memcpy nodes)
  const int64_t nw = (int64_t)(bytes / 4);
  if (nw) hipLaunchKernelGGL(k_copy_bytes, dim3(nblk(nw)), dim3(256), 0, s, (const uint32_t*)src,
                             (uint32_t*)dst, nw);
  ROM_HIP_CHECK(hipGetLastError());
  return ROM_OK;
}

rom_status validate(const rom_config* c) {
  ROM_REQUIRE(c, ROM_E_INVAL, "cfg is NULL");
  ROM_REQUIRE(c->problem >= ROM_BURGERS && c->problem <= ROM_REACT, ROM_E_INVAL, "unknown problem");
  ROM_REQUIRE(c->precision == ROM_F32 || c->precision == ROM_F64, ROM_E_INVAL, "bad precision");
  ROM_REQUIRE(c->projection == ROM_GALERKIN || c->projection == ROM_LSPG, ROM_E_INVAL,
              "bad projection");
  ROM_REQUIRE(c->hyper >= ROM_HR_NONE && c->hyper <= ROM_HR_QDEIM_FGS, ROM_E_INVAL, "bad hyper");
  ROM_REQUIRE(c->n_inst >= 1, ROM_E_INVAL, "n_inst must be >= 1");
  ROM_REQUIRE(c->n_cells && c->phys, ROM_E_INVAL, "n_cells and phys are required");
  const int need = c->problem == ROM_REACT ? 88 : 1;
  ROM_REQUIRE(c->n_phys == need, ROM_E_INVAL, "n_phys does not match the problem");
  int64_t mn = INT64_MAX;
  for (int b = 0; b < c->n_inst; ++b) {
    ROM_REQUIRE(c->n_cells[b] >= 3, ROM_E_INVAL, "every instance needs at least 3 cells");
    ROM_REQUIRE(c->n_cells[b] < (int64_t)1 << 31, ROM_E_INVAL, "instance too large");
    mn = std::min(mn, c->n_cells[b]);
  }
  const int nv = c->problem == ROM_REACT ? 12 : (c->problem == ROM_BURGERS ? 1 : 3);
  ROM_REQUIRE(c->r >= 1 && c->r <= kMaxR, ROM_E_INVAL, "r must be in [1, 64]");
  ROM_REQUIRE(c->r <= mn * nv, ROM_E_INVAL, "r exceeds the smallest instance");
  ROM_REQUIRE(c->w_init >= c->r && c->w_init <= 100, ROM_E_INVAL, "w_init must be in [r, 100]");
  ROM_REQUIRE(c->z >= 1, ROM_E_INVAL, "z must be >= 1");
  ROM_REQUIRE(c->lambda >= 0.0 && c->lambda <= 1.0, ROM_E_INVAL, "lambda must be in [0, 1]");
  ROM_REQUIRE(c->dt > 0.0 && std::isfinite(c->dt), ROM_E_INVAL, "dt must be positive");
  ROM_REQUIRE(c->newton_max >= 1 && c->newton_max <= 50, ROM_E_INVAL, "newton_max in [1, 50]");
  ROM_REQUIRE(c->rom_max >= 1 && c->rom_max <= 50, ROM_E_INVAL, "rom_max in [1, 50]");
  ROM_REQUIRE(c->newton_tol > 0.0 && c->rom_tol > 0.0, ROM_E_INVAL, "tolerances must be positive");
  ROM_REQUIRE(c->reorth_every >= 0, ROM_E_INVAL, "reorth_every must be >= 0");
  ROM_REQUIRE(c->update_rule >= ROM_UPDATE_ISVD && c->update_rule <= ROM_UPDATE_DIRECT,
              ROM_E_INVAL, "unknown update rule");
  if (c->update_rule != ROM_UPDATE_ISVD)
    ROM_REQUIRE(c->window >= c->r && c->window <= 64, ROM_E_INVAL,
                "the windowed rules need r <= window <= 64");
  ROM_REQUIRE(c->scheme == ROM_SCHEME_BE || c->scheme == ROM_SCHEME_SSPRK43, ROM_E_INVAL,
              "unknown scheme");
  if (c->scheme == ROM_SCHEME_SSPRK43) {
    ROM_REQUIRE(c->projection == ROM_GALERKIN, ROM_E_UNSUPPORTED,
                "the explicit scheme runs the (DEIM-)Galerkin ROM");
    ROM_REQUIRE(c->hyper != ROM_HR_NONE, ROM_E_UNSUPPORTED,
                "the explicit scheme runs the hyper-reduced Galerkin ROM (hyper != none)");
  }
  if (c->hyper == ROM_HR_DEIM) {
    ROM_REQUIRE(c->n_s >= c->r && c->n_s <= 2 * c->r && c->n_s <= kMaxNs, ROM_E_INVAL,
                "n_s must be in [r, 2r] with DEIM");
    ROM_REQUIRE(c->n_s <= mn * nv, ROM_E_INVAL, "n_s exceeds the smallest instance");
  } else if (c->hyper == ROM_HR_QDEIM) {
    ROM_REQUIRE(c->n_s == c->r, ROM_E_INVAL, "QDEIM gives n_s = r rows");
  } else if (c->hyper == ROM_HR_QDEIM_FGS) {
    ROM_REQUIRE(c->n_s > c->r && c->n_s <= 2 * c->r, ROM_E_INVAL,
                "feature-guided sampling adds 1 .. r rows to QDEIM's r (r < n_s <= 2r)");
    ROM_REQUIRE(c->n_s - c->r <= mn, ROM_E_INVAL, "more feature rows than cells");
  } else {
    ROM_REQUIRE(c->problem == ROM_BURGERS, ROM_E_UNSUPPORTED,
                "the full Galerkin ROM (no hyper-reduction) is implemented for Burgers");
    ROM_REQUIRE(c->projection == ROM_GALERKIN, ROM_E_UNSUPPORTED,
                "without hyper-reduction only the Galerkin projection is implemented");
  }
  return ROM_OK;
}

template <typename T>
rom_status alloc(T** p, size_t count) {
  *p = nullptr;
  if (count == 0) return ROM_OK;
  if (hipMalloc((void**)p, sizeof(T) * count) != hipSuccess) {
    set_error("hipMalloc failed");
    return ROM_E_NOMEM;
  }
  return ROM_OK;
}

void free_all(rom_batch* h) {
  void* ps[] = {h->d_dof_off, h->d_cell_off, h->d_phys, h->d_tiles, h->d_btiles, h->d_btiles2, h->d_ptiles, h->d_ptile_first,
                h->Phi, h->sigma, h->a, h->a_prev, h->q_ref, h->d_var, h->y_corr, h->flags, h->P,
                h->M, h->mesh_phi, h->mesh_qref, h->chosen, h->part, h->red, h->ubar, h->lmat,
                h->active, h->iters, h->norms, h->rstate, h->qtmp, h->mpart, h->fq, h->fq_prev, h->vjp_tmp,
                h->d_epoch, h->rvjp, h->epart, h->ev_iters, h->phi_cm, h->Phi_alt, h->hr_as};
  for (void* p : ps) (void)hipFree(p);
  void* pw[] = {h->win, h->lift, h->zmat, h->zpinv, h->phit, h->sig_scratch, h->qdeim_q,
                h->fgs_g, h->d_tile_first, h->mesh5_phi, h->mesh5_qref};
  for (void* p : pw) (void)hipFree(p);
  pod_ws_free(&h->podws);
  bt_free(h);
  for (auto& g : h->win_exec) if (g) (void)hipGraphExecDestroy(g);
  if (h->ev_fork) (void)hipEventDestroy(h->ev_fork);
  if (h->ev_join) (void)hipEventDestroy(h->ev_join);
  if (h->aux) (void)hipStreamDestroy(h->aux);
}

// The event at the end of a window (coarse step of y_corr, then the iSVD
// projections and core SVD) reads nothing the window's fine steps write, and
// the fine steps read nothing it writes, when the steps are Galerkin on the
// MFMA path (partials in part and mpart, the projections' in epart) and the
// coarse step is the one-workgroup kernel (its counters in ev_iters).  Only
// the state transfer and the rotation of Phi need the fine steps done.
bool window_split_ok(const rom_batch* h) {
  return h->cfg.hyper == ROM_HR_NONE && h->cfg.update_rule == ROM_UPDATE_ISVD && mfma_ok(h) &&
         h->fom_block;
}

rom_status setup(rom_batch* h) {
  const rom_config& c = h->cfg;
  const int B = c.n_inst;
  h->nv = c.problem == ROM_REACT ? 12 : (c.problem == ROM_BURGERS ? 1 : 3);
  h->esz = c.precision == ROM_F64 ? 8 : 4;
  h->dof_off.assign(B + 1, 0);
  h->cell_off.assign(B + 1, 0);
  for (int b = 0; b < B; ++b) {
    h->cell_off[b + 1] = h->cell_off[b] + h->n_cells[b];
    h->dof_off[b + 1] = h->dof_off[b] + h->n_cells[b] * h->nv;
    h->max_dof = std::max(h->max_dof, h->n_cells[b] * h->nv);
  }
  h->total_cells = h->cell_off[B];
  h->total_dof = h->dof_off[B];
  // stencil tiles (cells) and pass tiles (basis rows)
  std::vector<Tile> tiles, ptiles, btiles, btiles2;
  h->ptile_first.assign(B + 1, 0);
  std::vector<int> tile_first(B + 1, 0);
  for (int b = 0; b < B; ++b) {
    const int64_t nb = h->n_cells[b], base = h->dof_off[b];
    tile_first[b] = (int)tiles.size();
    for (int64_t c0 = 0; c0 < nb; c0 += kTile)
      tiles.push_back(Tile{b, 0, c0, std::min<int64_t>(kTile, nb - c0), nb, base});
    for (int64_t c0 = 0; c0 < nb; c0 += kBigTile)
      btiles.push_back(Tile{b, 0, c0, std::min<int64_t>(kBigTile, nb - c0), nb, base});
    for (int64_t c0 = 0; c0 < nb; c0 += kBigTile / 2)
      btiles2.push_back(Tile{b, 0, c0, std::min<int64_t>(kBigTile / 2, nb - c0), nb, base});
    const int64_t rows = nb * h->nv;
    h->ptile_first[b] = (int)ptiles.size();
    for (int64_t r0 = 0; r0 < rows; r0 += kPassRows)
      ptiles.push_back(Tile{b, 0, r0, std::min<int64_t>(kPassRows, rows - r0), nb, base});
  }
  h->ptile_first[B] = (int)ptiles.size();
  tile_first[B] = (int)tiles.size();
  h->n_tiles = (int)tiles.size();
  h->n_btiles = (int)btiles.size();
  h->n_btiles2 = (int)btiles2.size();
  h->n_ptiles = (int)ptiles.size();
  const size_t es = h->esz;
  const int r = c.r;
  ROM_TRY(alloc(&h->d_dof_off, B + 1));
  ROM_TRY(alloc(&h->d_cell_off, B + 1));
  ROM_TRY(alloc(&h->d_phys, h->phys.size()));
  ROM_TRY(alloc(&h->d_tiles, tiles.size()));
  ROM_TRY(alloc(&h->d_btiles, btiles.size()));
  ROM_TRY(alloc(&h->d_btiles2, btiles2.size()));
  ROM_TRY(alloc(&h->d_ptiles, ptiles.size()));
  ROM_TRY(alloc(&h->d_ptile_first, B + 1));
  ROM_TRY(alloc(&h->d_tile_first, B + 1));
  ROM_HIP_CHECK(hipMemcpy(h->d_tile_first, tile_first.data(), sizeof(int) * (B + 1),
                          hipMemcpyHostToDevice));
  ROM_HIP_CHECK(hipMemcpy(h->d_dof_off, h->dof_off.data(), 8 * (B + 1), hipMemcpyHostToDevice));
  ROM_HIP_CHECK(hipMemcpy(h->d_cell_off, h->cell_off.data(), 8 * (B + 1), hipMemcpyHostToDevice));
  ROM_HIP_CHECK(hipMemcpy(h->d_phys, h->phys.data(), 8 * h->phys.size(), hipMemcpyHostToDevice));
  ROM_HIP_CHECK(hipMemcpy(h->d_tiles, tiles.data(), sizeof(Tile) * tiles.size(), hipMemcpyHostToDevice));
  ROM_HIP_CHECK(hipMemcpy(h->d_btiles, btiles.data(), sizeof(Tile) * btiles.size(), hipMemcpyHostToDevice));
  ROM_HIP_CHECK(hipMemcpy(h->d_btiles2, btiles2.data(), sizeof(Tile) * btiles2.size(), hipMemcpyHostToDevice));
  {
    int dev = 0, ncu = 0;
    ROM_HIP_CHECK(hipGetDevice(&dev));
    ROM_HIP_CHECK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    h->n_cu = ncu > 0 ? ncu : 256;
  }
  ROM_HIP_CHECK(hipMemcpy(h->d_ptiles, ptiles.data(), sizeof(Tile) * ptiles.size(), hipMemcpyHostToDevice));
  ROM_HIP_CHECK(hipMemcpy(h->d_ptile_first, h->ptile_first.data(), sizeof(int) * (B + 1),
                          hipMemcpyHostToDevice));
  const int64_t td = h->total_dof;
  const int ns = std::max(c.n_s, 1);
  ROM_TRY(alloc((char**)&h->Phi, es * td * r));
  h->phi_first = h->Phi;
  ROM_TRY(alloc(&h->sigma, (size_t)B * r));
  ROM_TRY(alloc(&h->a, (size_t)B * r));
  ROM_TRY(alloc(&h->a_prev, (size_t)B * r));
  ROM_TRY(alloc((char**)&h->q_ref, es * td));
  ROM_TRY(alloc(&h->d_var, (size_t)B * h->nv));
  ROM_TRY(alloc((char**)&h->y_corr, es * td));
  ROM_TRY(alloc((char**)&h->fq, es * td));
  ROM_TRY(alloc((char**)&h->fq_prev, es * td));
  ROM_TRY(alloc((char**)&h->vjp_tmp, es * td));
  ROM_TRY(alloc(&h->flags, B));
  ROM_TRY(alloc(&h->P, (size_t)B * ns));
  ROM_TRY(alloc(&h->M, (size_t)B * r * ns));
  ROM_TRY(alloc((char**)&h->mesh_phi, es * B * ns * 3 * h->nv * r));
  ROM_TRY(alloc(&h->mesh_qref, (size_t)B * ns * 3 * h->nv));
  ROM_TRY(alloc(&h->chosen, (size_t)td));
  if (c.hyper == ROM_HR_DEIM) ROM_TRY(alloc((char**)&h->phi_cm, es * td * r));
  if (c.hyper != ROM_HR_NONE) ROM_TRY(alloc(&h->hr_as, (size_t)B * (ns + r) * (r + 1)));
  if (c.hyper == ROM_HR_QDEIM || c.hyper == ROM_HR_QDEIM_FGS)
    ROM_TRY(alloc(&h->qdeim_q, (size_t)B * kMaxR * kMaxR));
  if (c.hyper == ROM_HR_QDEIM_FGS) ROM_TRY(alloc(&h->fgs_g, (size_t)h->total_cells));
  if (c.scheme == ROM_SCHEME_SSPRK43) {
    ROM_TRY(alloc(&h->mesh5_phi, (size_t)B * ns * 5 * h->nv * r));
    ROM_TRY(alloc(&h->mesh5_qref, (size_t)B * ns * 5 * h->nv));
  }
  ROM_TRY(alloc(&h->part, (size_t)std::max(h->n_ptiles, 1) * kMaxR * kMaxR));
  ROM_TRY(alloc(&h->red, (size_t)B * (2 * 128 + 8)));
  ROM_TRY(alloc(&h->ubar, (size_t)B * (r + 1) * (r + 1)));
  ROM_TRY(alloc(&h->lmat, (size_t)B * r * r));
  ROM_TRY(alloc(&h->active, B));
  ROM_TRY(alloc(&h->iters, B));
  ROM_TRY(alloc(&h->norms, (size_t)3 * (c.newton_max + 1) * B));
  ROM_TRY(alloc(&h->rstate, (size_t)B * (kMaxR * kMaxR + 4 * kMaxR)));
  ROM_TRY(alloc(&h->qtmp, (size_t)td));
  ROM_TRY(alloc((char**)&h->mpart, es * std::max(h->n_ptiles, 1) * kMaxR * kMaxR));
  ROM_TRY(alloc(&h->epart, (size_t)std::max(h->n_ptiles, 1) * kMaxR * kMaxR));
  ROM_TRY(alloc(&h->ev_iters, B));
  ROM_TRY(alloc(&h->d_epoch, 1));
  ROM_HIP_CHECK(hipMemset(h->flags, 0, 4 * B));
  ROM_HIP_CHECK(hipMemset(h->chosen, 0, 4 * td));
  ROM_HIP_CHECK(hipMemset(h->d_epoch, 0, 4));
  ROM_HIP_CHECK(hipMemset(h->P, 0, 4 * (size_t)B * ns));
  ROM_HIP_CHECK(hipMemset(h->a, 0, 8 * (size_t)B * r));
  ROM_HIP_CHECK(hipMemset(h->sigma, 0, 8 * (size_t)B * r));
  if (c.update_rule != ROM_UPDATE_ISVD) {
    ROM_TRY(alloc((char**)&h->win, es * td * c.window));
    ROM_TRY(alloc(&h->lift, (size_t)td));
    ROM_TRY(alloc(&h->zmat, (size_t)B * 64 * (r + 1)));
    ROM_TRY(alloc(&h->zpinv, (size_t)B * 64 * r));
    ROM_TRY(alloc((char**)&h->phit, es * td * r));
    ROM_TRY(alloc(&h->sig_scratch, (size_t)B * r));
    ROM_TRY(pod_ws_alloc(h, std::max(c.window, r), &h->podws));
  }
  ROM_TRY(bt_setup(h));
  h->fom_block = c.scheme == ROM_SCHEME_BE && fom_block_ok(h);
  if (window_split_ok(h)) {  // the second stream of a window (created outside any capture)
    ROM_TRY(alloc((char**)&h->Phi_alt, es * td * r));
    ROM_HIP_CHECK(hipStreamCreateWithFlags(&h->aux, hipStreamNonBlocking));
    ROM_HIP_CHECK(hipEventCreateWithFlags(&h->ev_fork, hipEventDisableTiming));
    ROM_HIP_CHECK(hipEventCreateWithFlags(&h->ev_join, hipEventDisableTiming));
  }
  ROM_TRY(isvd_kernels_prepare());
  ROM_TRY(adjoint_kernels_prepare());
  ROM_TRY(rom_kernels_prepare());
  ROM_TRY(explicit_kernels_prepare());
  ROM_HIP_CHECK(hipDeviceSynchronize());
  return ROM_OK;
}

// One backward-Euler step of size dt for every instance (Newton, exact banded
// Jacobian, direct block-tridiagonal solve).  q_prev and q_out may alias.
rom_status fom_step_impl(rom_batch* h, const void* q_prev, double dt, void* q_out,
                         int32_t* iters_out, hipStream_t s) {
  const int B = h->cfg.n_inst;
  const size_t bytes = h->esz * h->total_dof;
  const bool f64 = h->cfg.precision == ROM_F64;
  if (h->cfg.scheme == ROM_SCHEME_SSPRK43) {
    ROM_TRY(fom_step_explicit(h, q_prev, dt, q_out, s));
    if (iters_out)
      hipLaunchKernelGGL(k_fill_i32v, dim3(nblk(B)), dim3(256), 0, s, iters_out, 4, (int64_t)B);
    ROM_HIP_CHECK(hipGetLastError());
    return ROM_OK;
  }
  if (h->fom_block) {
    ROM_TRY(launch_fom_block(h, q_prev, dt, q_out, h->iters, s));
    if (iters_out) ROM_TRY(copy_words(h->iters, iters_out, 4 * (size_t)B, s));
    return ROM_OK;
  }
  ROM_TRY(copy_words(q_prev, h->fq_prev, bytes, s));
  ROM_TRY(copy_words(q_prev, h->fq, bytes, s));
  const int mx = h->cfg.newton_max;
  hipLaunchKernelGGL(k_fill_i32v, dim3(nblk(B)), dim3(256), 0, s, h->active, 1, (int64_t)B);
  hipLaunchKernelGGL(k_fill_i32v, dim3(nblk(B)), dim3(256), 0, s, h->iters, 0, (int64_t)B);
  const int64_t nn = (int64_t)3 * (mx + 1) * B;
  hipLaunchKernelGGL(k_fill_u64, dim3(nblk(nn)), dim3(256), 0, s, h->norms, (uint64_t)0, nn);
  for (int it = 0; it < mx; ++it) {
    ROM_TRY(launch_assemble(h, h->fq, h->fq_prev, dt, it, s));
    if (f64)
      hipLaunchKernelGGL(k_newton_decide<double>, dim3(nblk(B)), dim3(256), 0, s, B, h->norms,
                         it, mx, h->cfg.newton_tol, h->active, h->iters);
    else
      hipLaunchKernelGGL(k_newton_decide<float>, dim3(nblk(B)), dim3(256), 0, s, B, h->norms,
                         it, mx, h->cfg.newton_tol, h->active, h->iters);
    ROM_TRY(bt_solve(h, it, h->fq, nullptr, s));
  }
  ROM_TRY(launch_residual_norm(h, h->fq, h->fq_prev, dt, h->vjp_tmp, mx, s));
  if (f64)
    hipLaunchKernelGGL(k_newton_final<double>, dim3(nblk(B)), dim3(256), 0, s, B, h->norms, mx,
                       h->cfg.newton_tol, h->active, h->flags);
  else
    hipLaunchKernelGGL(k_newton_final<float>, dim3(nblk(B)), dim3(256), 0, s, B, h->norms, mx,
                       h->cfg.newton_tol, h->active, h->flags);
  ROM_TRY(copy_words(h->fq, q_out, bytes, s));
  if (iters_out) ROM_TRY(copy_words(h->iters, iters_out, 4 * (size_t)B, s));
  ROM_HIP_CHECK(hipGetLastError());
  return ROM_OK;
}

rom_status isvd_impl(rom_batch* h, const void* y, hipStream_t s) {
  if (h->cfg.update_rule == ROM_UPDATE_ISVD) ROM_TRY(launch_isvd(h, y, s));
  else ROM_TRY(launch_windowed_update(h, y, s));
  h->n_update += 1;
  if (h->cfg.reorth_every > 0 && h->n_update % h->cfg.reorth_every == 0) {
    ROM_TRY(launch_reorth(h, s));
    h->n_reorth += 1;
  }
  return ROM_OK;
}

// One whole window with that overlap: the event chain on a second stream,
// forked from s at the start and joined before the state transfer.  The event
// chain ends with the rotation of the basis into the second buffer Phi_alt
// (the fine steps only read Phi), so only the transfer waits for the fine
// steps.  The kernels and their inputs are those of the serial order, so the
// results are the same.  The caller makes Phi_alt the current basis (swaps the
// two pointers) once the window's work is enqueued or replayed.
rom_status window_split_impl(rom_batch* h, hipStream_t s) {
  ROM_REQUIRE(h->aux && h->ev_fork && h->ev_join && h->Phi_alt, ROM_E_STATE, "no second stream");
  const int z = h->cfg.z;
  ROM_HIP_CHECK(hipEventRecord(h->ev_fork, s));
  ROM_HIP_CHECK(hipStreamWaitEvent(h->aux, h->ev_fork, 0));
  rom_status st = launch_fom_block(h, h->y_corr, z * h->cfg.dt, h->y_corr, h->ev_iters, h->aux);
  if (st == ROM_OK) st = launch_isvd_core(h, h->y_corr, h->epart, h->aux);
  if (st == ROM_OK) st = launch_isvd_rotate_into(h, h->Phi_alt, h->aux);
  // join even after an error, so that a capture in progress ends consistently
  ROM_HIP_CHECK(hipEventRecord(h->ev_join, h->aux));
  for (int k = 0; k < z && st == ROM_OK; ++k) st = launch_rom_fine_step(h, s);
  ROM_HIP_CHECK(hipStreamWaitEvent(s, h->ev_join, 0));
  ROM_TRY(st);
  ROM_TRY(launch_isvd_transfer(h, s));
  h->n_update += 1;
  ROM_TRY(launch_rebuild(h, s));
  h->n_events += 1;
  h->n_fine += z;
  return ROM_OK;
}

// One adaptation window unit: a fine reduced step and, if due, the event.
rom_status fine_step_impl(rom_batch* h, hipStream_t s) {
  ROM_TRY(launch_rom_fine_step(h, s));
  const int64_t n = h->n_fine;
  if ((n + 1 - h->cfg.w_init) % h->cfg.z == 0) {
    ROM_TRY(fom_step_impl(h, h->y_corr, h->cfg.z * h->cfg.dt, h->y_corr, nullptr, s));
    ROM_TRY(isvd_impl(h, h->y_corr, s));
    ROM_TRY(launch_rebuild(h, s));
    h->n_events += 1;
  }
  h->n_fine += 1;
  return ROM_OK;
}

rom_status offline(rom_batch* h, const void* q0, hipStream_t s) {
  const int w = h->cfg.w_init;
  const size_t bytes = h->esz * h->total_dof;
  char* Q = nullptr;
  ROM_TRY(alloc(&Q, bytes * w));
  rom_status st = ROM_OK;
  const void* prev = q0;
  for (int j = 0; j < w && st == ROM_OK; ++j) {
    st = fom_step_impl(h, prev, h->cfg.dt, Q + bytes * j, nullptr, s);
    prev = Q + bytes * j;
  }
  if (st == ROM_OK) st = launch_preprocess(h, q0, Q, w, s);
  if (st == ROM_OK) st = launch_pod(h, Q, w, s);
  if (st == ROM_OK && h->cfg.update_rule != ROM_UPDATE_ISVD) st = launch_window_init(h, Q, w, s);
  const void* qlast = Q + bytes * (w - 1);
  if (st == ROM_OK) st = launch_project_state(h, qlast, s);
  if (st == ROM_OK) st = fom_step_impl(h, qlast, h->cfg.z * h->cfg.dt, h->y_corr, nullptr, s);
  if (st == ROM_OK) st = launch_rebuild(h, s);
  hipError_t e = hipStreamSynchronize(s);
  (void)hipFree(Q);
  if (st != ROM_OK) return st;
  if (e != hipSuccess) { set_error(hipGetErrorString(e)); return ROM_E_DEVICE; }
  h->n_fine = w;
  h->has_rom = true;
  return ROM_OK;
}

// ---- the rollout adjoint's checkpoint plan and body (shared by the
// allocating entry point and the one that runs in the static device scratch)
struct RolloutPlan {
  int64_t T = 0, S = 0, nseg = 0;  // steps, steps per segment, checkpoints
  size_t st = 0;                    // bytes of one state
  size_t bytes = 0;                 // checkpoints + segment states + two adjoint vectors
};

rom_status rollout_check(rom_batch* h, const void* q0, int32_t n_steps, double dt, int32_t n_ckpt,
                         const void* gbar, void* gq0) {
  ROM_REQUIRE(h && q0 && gbar && gq0, ROM_E_INVAL, "handle, q0, gbar and gq0 are required");
  ROM_REQUIRE(n_steps >= 1, ROM_E_INVAL, "n_steps must be >= 1");
  ROM_REQUIRE(n_ckpt >= 0, ROM_E_INVAL, "n_ckpt must be >= 0");
  ROM_REQUIRE(dt > 0.0 && std::isfinite(dt), ROM_E_INVAL, "dt must be positive");
  ROM_REQUIRE(h->cfg.scheme == ROM_SCHEME_BE, ROM_E_UNSUPPORTED,
              "the full-order adjoint covers the backward-Euler scheme");
  return ROM_OK;
}

RolloutPlan rollout_plan(const rom_batch* h, int32_t n_steps, int32_t n_ckpt) {
  RolloutPlan p;
  p.T = n_steps;
  int64_t C = n_ckpt > 0 ? n_ckpt : (int64_t)std::ceil(std::sqrt((double)p.T));
  if (C > p.T) C = p.T;
  p.S = (p.T + C - 1) / C;
  p.nseg = (p.T + p.S - 1) / p.S;  // states q^0, q^S, q^2S, ...
  p.st = h->esz * (size_t)h->total_dof;
  p.bytes = (size_t)(p.nseg + p.S + 1 + 2) * p.st;
  return p;
}

// Forward pass keeping only the checkpoints, then one segment at a time:
// recompute its states from the checkpoint and apply the step adjoints in
// reverse.  Every byte of ws that is read was written earlier in the call.
rom_status rollout_vjp_impl(rom_batch* h, const void* q0, double dt, const RolloutPlan& pl,
                            const void* gbar, void* gq0, char* ws, hipStream_t s) {
  const int64_t T = pl.T, S = pl.S, nseg = pl.nseg;
  const size_t st = pl.st;
  char* ck = ws;
  char* seg = ck + (size_t)nseg * st;
  char* ga = seg + (size_t)(S + 1) * st;
  char* gb = ga + st;
  ROM_TRY(copy_words(q0, ck, st, s));
  for (int64_t j = 0; j + 1 < nseg; ++j) {
    char* nxt = ck + (size_t)(j + 1) * st;
    ROM_TRY(copy_words(ck + (size_t)j * st, nxt, st, s));
    for (int64_t k = 0; k < S; ++k) ROM_TRY(fom_step_impl(h, nxt, dt, nxt, nullptr, s));
  }
  ROM_TRY(copy_words(gbar, ga, st, s));
  for (int64_t j = nseg - 1; j >= 0; --j) {
    const int64_t k0 = j * S, k1 = std::min(k0 + S, T), L = k1 - k0;
    ROM_TRY(copy_words(ck + (size_t)j * st, seg, st, s));
    for (int64_t i = 0; i < L; ++i)
      ROM_TRY(fom_step_impl(h, seg + (size_t)i * st, dt, seg + (size_t)(i + 1) * st, nullptr, s));
    for (int64_t i = L - 1; i >= 0; --i) {
      ROM_TRY(launch_assemble_adjoint(h, seg + (size_t)(i + 1) * st, dt, ga, s));
      ROM_TRY(bt_solve(h, -1, nullptr, gb, s));
      std::swap(ga, gb);
    }
  }
  ROM_TRY(copy_words(ga, gq0, st, s));
  ROM_HIP_CHECK(hipGetLastError());
  return ROM_OK;
}

// ---- the static device scratch (top of this file): each device holds its
// own copy of the array; its address is looked up once per device (with that
// device current) and kept.  In host code the array's name is not a device
// address: only the looked-up pointer is passed on.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Look up the scratch address of the current device (once per device).
rom_status scratch_resolve_current(int* dev_out) {
  int dev = 0;
  ROM_HIP_CHECK(hipGetDevice(&dev));
  ROM_REQUIRE(dev >= 0 && dev < kMaxDevices, ROM_E_DEVICE, "device index out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    ROM_HIP_CHECK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    ROM_REQUIRE(p, ROM_E_DEVICE, "hipGetSymbolAddress returned no address for the scratch");
    g_scratch_ptr[dev] = p;
  }
  if (dev_out) *dev_out = dev;
  return ROM_OK;
}

// The scratch of the device the handle was created on (resolved at rom_create).
rom_status scratch_of_handle(const rom_batch* h, void** out) {
  int cur = 0;
  ROM_HIP_CHECK(hipGetDevice(&cur));
  ROM_REQUIRE(cur == h->device, ROM_E_STATE, "the handle's device is not the current device");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  ROM_REQUIRE(g_scratch_ptr[h->device], ROM_E_STATE, "device scratch not resolved for this device");
  *out = g_scratch_ptr[h->device];
  return ROM_OK;
}

// ---- saved handle state (rom_save / rom_load): a 256-byte header of int64
// words, then the sections below, each starting on a 256-byte boundary.
constexpr int64_t kSaveMagic = 0x31535049484d4f52ll;  // "ROMHIPS1"
constexpr int64_t kSaveVersion = 1;
enum { kSecPhi, kSecSigma, kSecA, kSecYcorr, kSecQref, kSecDvar, kSecFlags, kSecP, kSecM, kSecWin,
       kNumSec };
constexpr int kHdrWords = 32;
struct SaveHeader { int64_t w[kHdrWords]; };
struct SaveLayout {
  size_t off[kNumSec];
  size_t len[kNumSec];
  size_t total;
};

SaveLayout save_layout(const rom_batch* h) {
  const size_t B = h->cfg.n_inst, r = h->cfg.r, td = h->total_dof;
  const size_t ns = std::max(h->cfg.n_s, 1);
  SaveLayout L;
  L.len[kSecPhi] = h->esz * td * r;
  L.len[kSecSigma] = 8 * B * r;
  L.len[kSecA] = 8 * B * r;
  L.len[kSecYcorr] = h->esz * td;
  L.len[kSecQref] = h->esz * td;
  L.len[kSecDvar] = 8 * B * h->nv;
  L.len[kSecFlags] = 4 * B;
  L.len[kSecP] = 4 * B * ns;
  L.len[kSecM] = 8 * B * r * ns;
  L.len[kSecWin] = h->win ? h->esz * td * h->cfg.window : 0;
  size_t o = sizeof(SaveHeader);
  for (int i = 0; i < kNumSec; ++i) {
    o = (o + 255) & ~(size_t)255;
    L.off[i] = o;
    o += L.len[i];
  }
  L.total = o;
  return L;
}

// FNV-1a over the instance sizes: a loaded state must come from the same layout.
int64_t layout_hash(const rom_batch* h) {
  uint64_t x = 1469598103934665603ull;
  for (int64_t n : h->n_cells) {
    for (int k = 0; k < 8; ++k) {
      x ^= (uint64_t)((n >> (8 * k)) & 0xff);
      x *= 1099511628211ull;
    }
  }
  return (int64_t)(x >> 1);
}

SaveHeader save_header(const rom_batch* h, const SaveLayout& L) {
  SaveHeader hd{};
  const rom_config& c = h->cfg;
  const int64_t v[21] = {kSaveMagic, kSaveVersion, c.problem, c.precision, c.n_inst, h->total_dof,
                         c.r, c.n_s, h->nv, layout_hash(h), h->n_fine, h->n_update, h->n_events,
                         h->n_reorth, (int64_t)L.total, c.hyper, c.update_rule, c.window,
                         h->win_count, h->win_head, c.scheme};
  for (int i = 0; i < 21; ++i) hd.w[i] = v[i];
  return hd;
}

__global__ void k_write_header(SaveHeader hd, int64_t* dst) {
  if (threadIdx.x < kHdrWords) dst[threadIdx.x] = hd.w[threadIdx.x];
}

}  // namespace

rom_status fill_zero(void* p, size_t bytes, hipStream_t s) {
  const int64_t nw = (int64_t)(bytes / 4);
  if (nw) hipLaunchKernelGGL(k_fill_u32, dim3(nblk(nw)), dim3(256), 0, s, (uint32_t*)p, 0u, nw);
  ROM_HIP_CHECK(hipGetLastError());
  return ROM_OK;
}

}  // namespace romhip

using namespace romhip;

extern "C" {

const char* rom_last_error(void) { return g_err.c_str(); }

rom_status rom_create(const rom_config* cfg, const void* q0, void* stream, rom_handle* out) {
  ROM_REQUIRE(out, ROM_E_INVAL, "out is NULL");
  *out = nullptr;
  ROM_TRY(validate(cfg));
  rom_batch* h = new (std::nothrow) rom_batch();
  ROM_REQUIRE(h, ROM_E_NOMEM, "host allocation failed");
  h->cfg = *cfg;
  h->n_cells.assign(cfg->n_cells, cfg->n_cells + cfg->n_inst);
  h->phys.assign(cfg->phys, cfg->phys + (size_t)cfg->n_inst * cfg->n_phys);
  h->cfg.n_cells = nullptr;
  h->cfg.phys = nullptr;
  rom_status st = scratch_resolve_current(&h->device);
  if (st == ROM_OK) st = setup(h);
  hipStream_t s = (hipStream_t)stream;
  h->last_stream = s;
  if (st == ROM_OK && q0) st = offline(h, q0, s);
  if (st != ROM_OK) {
    free_all(h);
    delete h;
    return st;
  }
  *out = h;
  return ROM_OK;
}

rom_status rom_destroy(rom_handle h) {
  if (!h) return ROM_OK;
  (void)hipDeviceSynchronize();
  free_all(h);
  delete h;
  return ROM_OK;
}

rom_status rom_query(rom_handle h, int64_t* total_dof, int32_t* n_var, int32_t* r, int32_t* n_s) {
  ROM_REQUIRE(h, ROM_E_INVAL, "handle is NULL");
  if (total_dof) *total_dof = h->total_dof;
  if (n_var) *n_var = h->nv;
  if (r) *r = h->cfg.r;
  if (n_s) *n_s = h->cfg.n_s;
  return ROM_OK;
}

rom_status fom_residual(rom_handle h, const void* q, const void* q_prev, double dt, void* out,
                        void* stream) {
  ROM_REQUIRE(h && q && out, ROM_E_INVAL, "handle, q and out are required");
  ROM_REQUIRE(out != q && out != q_prev, ROM_E_INVAL, "out must not alias q or q_prev");
  ROM_REQUIRE(std::isfinite(dt), ROM_E_INVAL, "dt must be finite");
  h->last_stream = (hipStream_t)stream;
  if (h->cfg.scheme == ROM_SCHEME_SSPRK43) {
    ROM_REQUIRE(!q_prev, ROM_E_INVAL, "the explicit scheme has no backward-Euler residual");
    return launch_residual2(h, q, out, (hipStream_t)stream);
  }
  return launch_residual(h, q, q_prev, dt, out, (hipStream_t)stream);
}

rom_status fom_step(rom_handle h, const void* q_prev, double dt, void* q_out, int32_t* iters,
                    void* stream) {
  ROM_REQUIRE(h && q_prev && q_out, ROM_E_INVAL, "handle, q_prev and q_out are required");
  ROM_REQUIRE(dt > 0.0 && std::isfinite(dt), ROM_E_INVAL, "dt must be positive");
  h->last_stream = (hipStream_t)stream;
  return fom_step_impl(h, q_prev, dt, q_out, iters, (hipStream_t)stream);
}

rom_status isvd_update(rom_handle h, const void* y, void* stream) {
  ROM_REQUIRE(h && y, ROM_E_INVAL, "handle and y are required");
  ROM_REQUIRE(h->has_rom, ROM_E_STATE, "no reduced state: create with q0 or load with rom_set");
  h->last_stream = (hipStream_t)stream;
  return isvd_impl(h, y, (hipStream_t)stream);
}

rom_status rom_rebuild(rom_handle h, void* stream) {
  ROM_REQUIRE(h, ROM_E_INVAL, "handle is NULL");
  ROM_REQUIRE(h->has_rom, ROM_E_STATE, "no reduced state");
  h->last_stream = (hipStream_t)stream;
  return launch_rebuild(h, (hipStream_t)stream);
}

rom_status rom_step(rom_handle h, int32_t n_fine, void* stream) {
  ROM_REQUIRE(h, ROM_E_INVAL, "handle is NULL");
  ROM_REQUIRE(n_fine >= 0, ROM_E_INVAL, "n_fine must be >= 0");
  ROM_REQUIRE(h->has_rom, ROM_E_STATE, "no reduced state");
  hipStream_t s = (hipStream_t)stream;
  h->last_stream = s;
  const int z = h->cfg.z;
  int done = 0;
  // the windowed rules keep their window's fill level and next slot on the
  // host, so their windows run eagerly
  const bool graphs = h->cfg.use_graph && s != nullptr && h->cfg.update_rule == ROM_UPDATE_ISVD;
  while (done < n_fine) {
    const int64_t pos = (h->n_fine - h->cfg.w_init) % z;  // steps since the last event
    const bool aligned = pos == 0 && n_fine - done >= z;
    const bool reorth_due =
        h->cfg.reorth_every > 0 && (h->n_update + 1) % h->cfg.reorth_every == 0;
    if (graphs && aligned && !reorth_due) {
      // one graph per buffer holding the current basis: an overlapped window
      // rotates into the other buffer, so consecutive windows alternate
      const bool split = window_split_ok(h);
      const int gk = (split && h->Phi != h->phi_first) ? 1 : 0;
      hipGraphExec_t& ex = h->win_exec[gk];
      if (!ex || h->win_stream[gk] != s) {
        if (ex) { (void)hipGraphExecDestroy(ex); ex = nullptr; }
        hipGraph_t g = nullptr;
        ROM_HIP_CHECK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        rom_status st = ROM_OK;
        const int64_t nf = h->n_fine, nu = h->n_update, ne = h->n_events;
        if (split) st = window_split_impl(h, s);
        else
          for (int k = 0; k < z && st == ROM_OK; ++k) st = fine_step_impl(h, s);
        hipError_t e = hipStreamEndCapture(s, &g);
        h->n_fine = nf; h->n_update = nu; h->n_events = ne;  // captured, not yet run
        if (st != ROM_OK) { if (g) (void)hipGraphDestroy(g); return st; }
        ROM_HIP_CHECK(e);
        ROM_HIP_CHECK(hipGraphInstantiate(&ex, g, nullptr, nullptr, 0));
        ROM_HIP_CHECK(hipGraphDestroy(g));
        h->win_stream[gk] = s;
      }
      ROM_HIP_CHECK(hipGraphLaunch(ex, s));
      if (split) std::swap(h->Phi, h->Phi_alt);
      h->n_fine += z;
      h->n_update += 1;
      h->n_events += 1;
      done += z;
    } else {
      ROM_TRY(fine_step_impl(h, s));
      done += 1;
    }
  }
  return ROM_OK;
}

rom_status rom_get(rom_handle h, int32_t what, void* dst, void* stream) {
  ROM_REQUIRE(h && dst, ROM_E_INVAL, "handle and dst are required");
  hipStream_t s = (hipStream_t)stream;
  const int B = h->cfg.n_inst, r = h->cfg.r;
  const size_t td = (size_t)h->total_dof;
  switch (what) {
    case ROM_GET_BASIS: return copy_words(h->Phi, dst, h->esz * td * r, s);
    case ROM_GET_SIGMA: return copy_words(h->sigma, dst, 8 * (size_t)B * r, s);
    case ROM_GET_A: return copy_words(h->a, dst, 8 * (size_t)B * r, s);
    case ROM_GET_QTILDE: return launch_reconstruct(h, dst, s);
    case ROM_GET_SAMPLES: return copy_words(h->P, dst, 4 * (size_t)B * std::max(h->cfg.n_s, 1), s);
    case ROM_GET_YCORR: return copy_words(h->y_corr, dst, h->esz * td, s);
    case ROM_GET_QREF: return copy_words(h->q_ref, dst, h->esz * td, s);
    case ROM_GET_DVAR: return copy_words(h->d_var, dst, 8 * (size_t)B * h->nv, s);
    case ROM_GET_PINV: return copy_words(h->M, dst, 8 * (size_t)B * r * std::max(h->cfg.n_s, 1), s);
    case ROM_GET_UBAR: return copy_words(h->ubar, dst, 8 * (size_t)B * (r + 1) * (r + 1), s);
    case ROM_GET_WINDOW:
      ROM_REQUIRE(h->win, ROM_E_STATE, "the handle keeps no snapshot window (iSVD rule)");
      return copy_words(h->win, dst, h->esz * td * h->cfg.window, s);
    case ROM_GET_COUNTERS: {
      int64_t* o = (int64_t*)dst;
      o[0] = h->n_fine; o[1] = h->n_update; o[2] = h->n_events; o[3] = h->n_reorth;
      o[4] = h->win_count; o[5] = h->win_head;
      return ROM_OK;
    }
  }
  set_error("unknown quantity");
  return ROM_E_INVAL;
}

rom_status rom_set(rom_handle h, int32_t what, const void* src, void* stream) {
  ROM_REQUIRE(h && src, ROM_E_INVAL, "handle and src are required");
  hipStream_t s = (hipStream_t)stream;
  const int B = h->cfg.n_inst, r = h->cfg.r;
  const size_t td = (size_t)h->total_dof;
  for (auto& g : h->win_exec)
    if (g) { (void)hipGraphExecDestroy(g); g = nullptr; }
  switch (what) {
    case ROM_GET_BASIS: h->has_rom = true; return copy_words(src, h->Phi, h->esz * td * r, s);
    case ROM_GET_SIGMA: return copy_words(src, h->sigma, 8 * (size_t)B * r, s);
    case ROM_GET_A: return copy_words(src, h->a, 8 * (size_t)B * r, s);
    case ROM_GET_SAMPLES: return copy_words(src, h->P, 4 * (size_t)B * std::max(h->cfg.n_s, 1), s);
    case ROM_GET_YCORR: return copy_words(src, h->y_corr, h->esz * td, s);
    case ROM_GET_QREF: return copy_words(src, h->q_ref, h->esz * td, s);
    case ROM_GET_DVAR: return copy_words(src, h->d_var, 8 * (size_t)B * h->nv, s);
    case ROM_GET_WINDOW:
      ROM_REQUIRE(h->win, ROM_E_STATE, "the handle keeps no snapshot window (iSVD rule)");
      return copy_words(src, h->win, h->esz * td * h->cfg.window, s);
    case ROM_GET_COUNTERS: {
      const int64_t* o = (const int64_t*)src;
      if (h->win)
        ROM_REQUIRE(o[4] >= 0 && o[4] <= h->cfg.window && o[5] >= 0 && o[5] < h->cfg.window,
                    ROM_E_INVAL, "window fill level or slot out of range");
      h->n_fine = o[0]; h->n_update = o[1]; h->n_events = o[2]; h->n_reorth = o[3];
      if (h->win) { h->win_count = (int)o[4]; h->win_head = (int)o[5]; }
      return ROM_OK;
    }
  }
  set_error("quantity cannot be set");
  return ROM_E_INVAL;
}

rom_status rom_save(rom_handle h, void* dst, size_t* bytes, void* stream) {
  ROM_REQUIRE(h && bytes, ROM_E_INVAL, "handle and bytes are required");
  const SaveLayout L = save_layout(h);
  if (!dst) {
    *bytes = L.total;
    return ROM_OK;
  }
  ROM_REQUIRE(*bytes >= L.total, ROM_E_INVAL, "dst is smaller than the saved state");
  ROM_REQUIRE(h->has_rom, ROM_E_STATE, "no reduced state to save");
  ROM_REQUIRE(((uintptr_t)dst & 7) == 0, ROM_E_INVAL, "dst must be 8-byte aligned");
  hipStream_t s = (hipStream_t)stream;
  h->last_stream = s;
  char* d = (char*)dst;
  hipLaunchKernelGGL(k_write_header, dim3(1), dim3(64), 0, s, save_header(h, L), (int64_t*)d);
  const void* src[kNumSec] = {h->Phi, h->sigma, h->a, h->y_corr, h->q_ref, h->d_var, h->flags,
                              h->P, h->M, h->win};
  for (int i = 0; i < kNumSec; ++i) ROM_TRY(copy_words(src[i], d + L.off[i], L.len[i], s));
  *bytes = L.total;
  ROM_HIP_CHECK(hipGetLastError());
  return ROM_OK;
}

rom_status rom_load(rom_handle h, const void* src, size_t bytes, void* stream) {
  ROM_REQUIRE(h && src, ROM_E_INVAL, "handle and src are required");
  ROM_REQUIRE(((uintptr_t)src & 7) == 0, ROM_E_INVAL, "src must be 8-byte aligned");
  const SaveLayout L = save_layout(h);
  ROM_REQUIRE(bytes >= L.total, ROM_E_INVAL, "src is smaller than this handle's saved state");
  hipStream_t s = (hipStream_t)stream;
  h->last_stream = s;
  SaveHeader got{};
  ROM_HIP_CHECK(hipStreamSynchronize(s));
  ROM_HIP_CHECK(hipMemcpy(got.w, src, sizeof(got.w), hipMemcpyDeviceToHost));
  const SaveHeader want = save_header(h, L);
  ROM_REQUIRE(got.w[0] == kSaveMagic && got.w[1] == kSaveVersion, ROM_E_INVAL,
              "src does not hold a saved romhip state of this version");
  for (int i = 2; i < 10; ++i)
    ROM_REQUIRE(got.w[i] == want.w[i], ROM_E_INVAL,
                "the saved state comes from a different configuration or layout");
  ROM_REQUIRE(got.w[14] == (int64_t)L.total && got.w[15] == want.w[15] &&
                  got.w[16] == want.w[16] && got.w[17] == want.w[17] && got.w[20] == want.w[20],
              ROM_E_INVAL, "the saved state comes from a different configuration");
  if (h->win)
    ROM_REQUIRE(got.w[18] >= 0 && got.w[18] <= h->cfg.window && got.w[19] >= 0 &&
                    got.w[19] < h->cfg.window,
                ROM_E_INVAL, "damaged window counters in the saved state");
  for (auto& g : h->win_exec)
    if (g) { (void)hipGraphExecDestroy(g); g = nullptr; }
  const char* p = (const char*)src;
  void* dst[kNumSec] = {h->Phi, h->sigma, h->a, h->y_corr, h->q_ref, h->d_var, h->flags,
                        h->P, h->M, h->win};
  for (int i = 0; i < kNumSec; ++i) ROM_TRY(copy_words(p + L.off[i], dst[i], L.len[i], s));
  h->n_fine = got.w[10];
  h->n_update = got.w[11];
  h->n_events = got.w[12];
  h->n_reorth = got.w[13];
  if (h->win) { h->win_count = (int)got.w[18]; h->win_head = (int)got.w[19]; }
  h->has_rom = true;
  // the sample mesh and the column-major copy are derived from the basis:
  // the rebuild recomputes them (and P, (P^T Phi)^+) with the same kernels
  ROM_TRY(launch_rebuild(h, s));
  ROM_HIP_CHECK(hipGetLastError());
  return ROM_OK;
}

rom_status rom_get_status(rom_handle h, uint32_t* host_flags) {
  ROM_REQUIRE(h && host_flags, ROM_E_INVAL, "handle and host_flags are required");
  ROM_HIP_CHECK(hipStreamSynchronize(h->last_stream));
  ROM_HIP_CHECK(hipMemcpy(host_flags, h->flags, 4 * (size_t)h->cfg.n_inst, hipMemcpyDeviceToHost));
  return ROM_OK;
}

rom_status rom_clear_status(rom_handle h, void* stream) {
  ROM_REQUIRE(h, ROM_E_INVAL, "handle is NULL");
  return fill_zero(h->flags, 4 * (size_t)h->cfg.n_inst, (hipStream_t)stream);
}

rom_status fom_residual_vjp(rom_handle h, const void* q, const void* q_prev, double dt,
                            const void* gbar, void* gq, void* gq_prev, void* stream) {
  ROM_REQUIRE(h && q && gbar && gq, ROM_E_INVAL, "handle, q, gbar and gq are required");
  ROM_REQUIRE(gq != gbar && gq != q, ROM_E_INVAL, "gq must not alias q or gbar");
  ROM_REQUIRE(h->cfg.scheme == ROM_SCHEME_BE, ROM_E_UNSUPPORTED,
              "the residual adjoint covers the backward-Euler scheme");
  h->last_stream = (hipStream_t)stream;
  return launch_residual_vjp(h, q, q_prev, dt, gbar, gq, gq_prev, (hipStream_t)stream);
}

rom_status fom_step_vjp(rom_handle h, const void* q, double dt, const void* gbar, void* gq_prev,
                        void* stream) {
  ROM_REQUIRE(h && q && gbar && gq_prev, ROM_E_INVAL, "handle, q, gbar and gq_prev are required");
  ROM_REQUIRE(dt > 0.0 && std::isfinite(dt), ROM_E_INVAL, "dt must be positive");
  ROM_REQUIRE(h->cfg.scheme == ROM_SCHEME_BE, ROM_E_UNSUPPORTED,
              "the step adjoint covers the backward-Euler scheme");
  hipStream_t s = (hipStream_t)stream;
  h->last_stream = s;
  ROM_TRY(launch_assemble_adjoint(h, q, dt, gbar, s));
  return bt_solve(h, -1, nullptr, gq_prev, s);
}

rom_status fom_rollout_vjp(rom_handle h, const void* q0, int32_t n_steps, double dt,
                           int32_t n_ckpt, const void* gbar, void* gq0, void* stream) {
  ROM_TRY(rollout_check(h, q0, n_steps, dt, n_ckpt, gbar, gq0));
  hipStream_t s = (hipStream_t)stream;
  h->last_stream = s;
  const RolloutPlan pl = rollout_plan(h, n_steps, n_ckpt);
  if (h->rvjp_bytes < pl.bytes) {
    ROM_HIP_CHECK(hipStreamSynchronize(s));
    if (h->rvjp) (void)hipFree(h->rvjp);
    h->rvjp = nullptr;
    h->rvjp_bytes = 0;
    char* p = nullptr;
    ROM_TRY(alloc(&p, pl.bytes));
    h->rvjp = p;
    h->rvjp_bytes = pl.bytes;
  }
  return rollout_vjp_impl(h, q0, dt, pl, gbar, gq0, (char*)h->rvjp, s);
}

rom_status fom_rollout_vjp_noalloc(rom_handle h, const void* q0, int32_t n_steps, double dt,
                                   int32_t n_ckpt, const void* gbar, void* gq0, void* stream) {
  ROM_TRY(rollout_check(h, q0, n_steps, dt, n_ckpt, gbar, gq0));
  const RolloutPlan pl = rollout_plan(h, n_steps, n_ckpt);
  if (pl.bytes > kScratchBytes) {
    set_error("fom_rollout_vjp_noalloc: the checkpoints need " + std::to_string(pl.bytes) +
              " bytes, more than the " + std::to_string(kScratchBytes) + "-byte device scratch");
    return ROM_E_INVAL;
  }
  void* ws = nullptr;
  ROM_TRY(scratch_of_handle(h, &ws));
  hipStream_t s = (hipStream_t)stream;
  h->last_stream = s;
  return rollout_vjp_impl(h, q0, dt, pl, gbar, gq0, (char*)ws, s);
}

rom_status rom_offline(rom_handle h, const void* q0, void* stream) {
  ROM_REQUIRE(h && q0, ROM_E_INVAL, "handle and q0 are required");
  hipStream_t s = (hipStream_t)stream;
  h->last_stream = s;
  h->n_update = 0;
  h->n_events = 0;
  h->n_reorth = 0;
  h->win_count = 0;
  h->win_head = 0;
  return offline(h, q0, s);
}

rom_status rom_rollout_vjp(rom_handle h, const void* q0, int32_t n_steps, int32_t n_ckpt,
                           const void* gbar, void* gq0, void* stream) {
  ROM_REQUIRE(h && q0 && gbar && gq0, ROM_E_INVAL, "handle, q0, gbar and gq0 are required");
  ROM_REQUIRE(n_steps >= 1, ROM_E_INVAL, "n_steps must be >= 1");
  ROM_REQUIRE(n_ckpt >= 0, ROM_E_INVAL, "n_ckpt must be >= 0");
  const rom_config& c = h->cfg;
  ROM_REQUIRE(c.hyper != ROM_HR_NONE && c.projection == ROM_LSPG, ROM_E_UNSUPPORTED,
              "the rollout adjoint covers the hyper-reduced LSPG path");
  ROM_REQUIRE(c.update_rule == ROM_UPDATE_ISVD && c.scheme == ROM_SCHEME_BE, ROM_E_UNSUPPORTED,
              "the rollout adjoint covers the iSVD update and backward-Euler steps");
  const int B = c.n_inst, r = c.r, n = r + 1, z = c.z, w = c.w_init, ns = c.n_s;
  const int64_t T = n_steps;
  auto due = [&](int64_t nf) { return (nf + 1 - w) % z == 0; };
  {  // no re-orthonormalisation may fall inside the rollout
    int64_t nu = 0;
    for (int64_t k = 0; k < T; ++k)
      if (due(w + k)) {
        ++nu;
        ROM_REQUIRE(!(c.reorth_every > 0 && nu % c.reorth_every == 0), ROM_E_UNSUPPORTED,
                    "a re-orthonormalisation falls inside the rollout");
      }
  }
  hipStream_t s = (hipStream_t)stream;
  h->last_stream = s;
  const bool f64 = c.precision == ROM_F64;
  const int64_t td = h->total_dof;
  int64_t C = n_ckpt > 0 ? n_ckpt : (int64_t)std::ceil(std::sqrt((double)T));
  if (C > T) C = T;
  const int64_t S = (T + C - 1) / C;
  const int64_t nseg = (T + S - 1) / S;
  const int64_t E = S / z + 1;
  const size_t phi_b = h->esz * (size_t)td * r, y_b = h->esz * (size_t)td;
  const size_t br = 8 * (size_t)B * r;
  const size_t state_b = phi_b + y_b + 2 * br;
  const size_t ev_b = phi_b + y_b + 3 * br + 8 * (size_t)B * n * n + 8 * (size_t)B * (2 * r + 2);
  const size_t winp_b = 4 * (size_t)B * ns, winm_b = 8 * (size_t)B * r * ns;
  const size_t td8 = 8 * (size_t)td;
  const size_t part_n = offline_vjp_part_doubles(h, w);
  const size_t small_n = (size_t)B * ((size_t)w * r + (size_t)w * w + (size_t)r * w + 3 * (size_t)w * w);
  auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
  size_t off = 0;
  auto take = [&](size_t bytes) { const size_t o = off; off += al(bytes); return o; };
  const size_t o_ck = take((size_t)(nseg + 1) * state_b);
  const size_t o_reca = take((size_t)S * br);
  const size_t o_ev = take((size_t)E * ev_b);
  const size_t o_winp = take((size_t)(E + 1) * winp_b);
  const size_t o_winm = take((size_t)(E + 1) * winm_b);
  const size_t o_scr0 = take(td8), o_scr1 = take(td8);
  const size_t o_rhs = take(y_b), o_out = take(y_b);
  const size_t o_qtr = take((size_t)w * y_b);
  const size_t o_phi0 = take(phi_b), o_y0 = take(y_b);
  const size_t o_ab = take(br), o_sb = take(br), o_pb = take(8 * (size_t)td * r);
  const size_t o_yb = take(td8), o_qrb = take(td8), o_dvb = take(8 * (size_t)B * h->nv);
  const size_t o_qb = take((size_t)(w + 1) * td8);
  const size_t o_part = take(8 * part_n), o_small = take(8 * small_n);
  const size_t o_evscr = take(8 * event_vjp_scratch_doubles(h));
  char* ws = nullptr;
  ROM_TRY(alloc(&ws, off));
  PodWs pws;
  rom_status st = pod_ws_alloc(h, w, &pws);
  if (st != ROM_OK) { (void)hipFree(ws); return st; }
  char* ck = ws + o_ck;
  char* rec_a = ws + o_reca;
  char* ev = ws + o_ev;
  int32_t* winP = (int32_t*)(ws + o_winp);
  double* winM = (double*)(ws + o_winm);
  double* scr0 = (double*)(ws + o_scr0);
  double* scr1 = (double*)(ws + o_scr1);
  char* rhs = ws + o_rhs;
  char* out = ws + o_out;
  char* Qtr = ws + o_qtr;
  char* phi0 = ws + o_phi0;
  char* y0 = ws + o_y0;
  double* abar = (double*)(ws + o_ab);
  double* sigbar = (double*)(ws + o_sb);
  double* phibar = (double*)(ws + o_pb);
  double* ycbar = (double*)(ws + o_yb);
  double* qrbar = (double*)(ws + o_qrb);
  double* dvbar = (double*)(ws + o_dvb);
  double* qb = (double*)(ws + o_qb);
  double* part = (double*)(ws + o_part);
  double* small = (double*)(ws + o_small);
  double* evscr = (double*)(ws + o_evscr);
  struct Host { int64_t nf, nu, ne; };
  std::vector<Host> hc(nseg + 1);
  auto save = [&](int64_t j) -> rom_status {
    char* p = ck + (size_t)j * state_b;
    ROM_TRY(copy_words(h->Phi, p, phi_b, s));
    ROM_TRY(copy_words(h->y_corr, p + phi_b, y_b, s));
    ROM_TRY(copy_words(h->sigma, p + phi_b + y_b, br, s));
    ROM_TRY(copy_words(h->a, p + phi_b + y_b + br, br, s));
    hc[j] = Host{h->n_fine, h->n_update, h->n_events};
    return ROM_OK;
  };
  // restoring a checkpoint also rebuilds P, (P^T Phi)^+ and the sample mesh:
  // the kernels are deterministic, so they equal those of the forward run
  auto restore = [&](int64_t j) -> rom_status {
    const char* p = ck + (size_t)j * state_b;
    ROM_TRY(copy_words(p, h->Phi, phi_b, s));
    ROM_TRY(copy_words(p + phi_b, h->y_corr, y_b, s));
    ROM_TRY(copy_words(p + phi_b + y_b, h->sigma, br, s));
    ROM_TRY(copy_words(p + phi_b + y_b + br, h->a, br, s));
    h->n_fine = hc[j].nf;
    h->n_update = hc[j].nu;
    h->n_events = hc[j].ne;
    return launch_rebuild(h, s);
  };
  auto ev_phi = [&](int64_t e) { return ev + (size_t)e * ev_b; };
  auto ev_y = [&](int64_t e) { return ev_phi(e) + phi_b; };
  auto ev_sold = [&](int64_t e) { return (double*)(ev_y(e) + y_b); };
  auto ev_aold = [&](int64_t e) { return ev_sold(e) + (size_t)B * r; };
  auto ev_snew = [&](int64_t e) { return ev_aold(e) + (size_t)B * r; };
  auto ev_u = [&](int64_t e) { return ev_snew(e) + (size_t)B * r; };
  auto ev_pr = [&](int64_t e) { return ev_u(e) + (size_t)B * n * n; };
  auto win_save = [&](int64_t k) -> rom_status {
    ROM_TRY(copy_words(h->P, winP + (size_t)k * B * ns, winp_b, s));
    return copy_words(h->M, winM + (size_t)k * B * r * ns, winm_b, s);
  };
  // ---- forward: the offline stage, keeping the training states and the QR
  // of the POD, then the online loop with checkpoints at segment starts
  for (int j = 0; j < w && st == ROM_OK; ++j)
    st = fom_step_impl(h, j == 0 ? q0 : (const void*)(Qtr + (size_t)(j - 1) * y_b), c.dt,
                       Qtr + (size_t)j * y_b, nullptr, s);
  if (st == ROM_OK) st = launch_preprocess(h, q0, Qtr, w, s);
  if (st == ROM_OK) st = launch_pod_ws(h, Qtr, w, pws, s);
  const void* qlast = Qtr + (size_t)(w - 1) * y_b;
  if (st == ROM_OK) st = launch_project_state(h, qlast, s);
  if (st == ROM_OK) st = fom_step_impl(h, qlast, z * c.dt, h->y_corr, nullptr, s);
  if (st == ROM_OK) st = launch_rebuild(h, s);
  if (st == ROM_OK) st = copy_words(h->Phi, phi0, phi_b, s);
  if (st == ROM_OK) st = copy_words(h->y_corr, y0, y_b, s);
  h->n_fine = w;
  h->n_update = 0;
  h->n_events = 0;
  h->n_reorth = 0;
  h->has_rom = true;
  for (int64_t j = 0; j < nseg && st == ROM_OK; ++j) {
    st = save(j);
    const int64_t L = std::min(S, T - j * S);
    for (int64_t k = 0; k < L && st == ROM_OK; ++k) st = fine_step_impl(h, s);
  }
  if (st == ROM_OK) st = save(nseg);
  // ---- seed at the end state (with the q_ref and D terms)
  if (st == ROM_OK) st = launch_online_seed(h, gbar, abar, phibar, s, qrbar, dvbar);
  if (st == ROM_OK) st = fill_zero(sigbar, br, s);
  if (st == ROM_OK) st = fill_zero(ycbar, td8, s);
  // ---- the online loop backward, one segment at a time
  for (int64_t j = nseg - 1; j >= 0 && st == ROM_OK; --j) {
    st = restore(j);
    if (st == ROM_OK) st = win_save(0);
    const int64_t L = std::min(S, T - j * S);
    std::vector<int64_t> after;
    for (int64_t k = 0; k < L && st == ROM_OK; ++k) {
      st = launch_rom_fine_step(h, s);
      if (st == ROM_OK) st = copy_words(h->a, rec_a + (size_t)k * br, br, s);
      if (st == ROM_OK && due(h->n_fine)) {
        const int64_t e = (int64_t)after.size();
        after.push_back(k);
        st = copy_words(h->Phi, ev_phi(e), phi_b, s);
        if (st == ROM_OK) st = copy_words(h->sigma, ev_sold(e), br, s);
        if (st == ROM_OK) st = copy_words(h->a, ev_aold(e), br, s);
        if (st == ROM_OK) st = fom_step_impl(h, h->y_corr, z * c.dt, h->y_corr, nullptr, s);
        if (st == ROM_OK) st = copy_words(h->y_corr, ev_y(e), y_b, s);
        if (st == ROM_OK) st = launch_isvd_core(h, h->y_corr, h->part, s);
        if (st == ROM_OK) st = copy_words(h->ubar, ev_u(e), 8 * (size_t)B * n * n, s);
        if (st == ROM_OK) st = copy_words(h->rstate, ev_pr(e), 8 * (size_t)B * (2 * r + 2), s);
        if (st == ROM_OK) st = copy_words(h->sigma, ev_snew(e), br, s);
        if (st == ROM_OK) st = launch_isvd_apply(h, s);
        h->n_update += 1;
        if (st == ROM_OK) st = launch_rebuild(h, s);
        if (st == ROM_OK) st = win_save(e + 1);
        h->n_events += 1;
      }
      h->n_fine += 1;
    }
    for (int64_t k = L - 1; k >= 0 && st == ROM_OK; --k) {
      int64_t e_next = -1;   // first event at or after step k: its Phi_old is step k's basis
      for (int64_t e = 0; e < (int64_t)after.size(); ++e)
        if (after[e] >= k) { e_next = e; break; }
      if (e_next >= 0 && after[e_next] == k) {
        const int64_t e = e_next;
        st = launch_event_vjp(h, ev_phi(e), ev_y(e), ev_sold(e), ev_aold(e), ev_u(e), ev_pr(e),
                              ev_snew(e), abar, phibar, sigbar, ycbar, scr0, scr1, evscr, s,
                              qrbar, dvbar);
        if (st == ROM_OK) st = convert_words(ycbar, true, rhs, f64, td, s);
        if (st == ROM_OK) st = launch_assemble_adjoint(h, ev_y(e), z * c.dt, rhs, s);
        if (st == ROM_OK) st = bt_solve(h, -1, nullptr, out, s);
        if (st == ROM_OK) st = convert_words(out, f64, ycbar, true, td, s);
      }
      if (st != ROM_OK) break;
      const int64_t wi = e_next >= 0 ? e_next : (int64_t)after.size();
      const void* phi_k = e_next >= 0 ? (const void*)ev_phi(e_next) : (const void*)h->Phi;
      st = launch_hr_step_vjp(h, phi_k, winP + (size_t)wi * B * ns, winM + (size_t)wi * B * r * ns,
                              (const double*)(rec_a + (size_t)k * br), abar, phibar, qrbar, dvbar,
                              s);
    }
  }
  // ---- the offline stage backward
  if (st == ROM_OK) st = fill_zero(qb, (size_t)(w + 1) * td8, s);
  double* qbw = qb + (size_t)w * td;
  if (st == ROM_OK)
    st = launch_offline_a_vjp(h, phi0, qlast, abar, phibar, qbw, qrbar, dvbar, part, s);
  // y_corr^{w_init} = BE(q_w) over z dt
  if (st == ROM_OK) st = convert_words(ycbar, true, rhs, f64, td, s);
  if (st == ROM_OK) st = launch_assemble_adjoint(h, y0, z * c.dt, rhs, s);
  if (st == ROM_OK) st = bt_solve(h, -1, nullptr, out, s);
  if (st == ROM_OK) st = add_to_double(h, out, qbw, s);
  if (st == ROM_OK)
    st = launch_offline_pod_vjp(h, pws, w, Qtr, phibar, sigbar, qb, qrbar, dvbar, part, small, s);
  // training steps q_j = BE(q_{j-1}), j = w .. 1
  for (int j = w; j >= 1 && st == ROM_OK; --j) {
    st = convert_words(qb + (size_t)j * td, true, rhs, f64, td, s);
    if (st == ROM_OK)
      st = launch_assemble_adjoint(h, Qtr + (size_t)(j - 1) * y_b, c.dt, rhs, s);
    if (st == ROM_OK) st = bt_solve(h, -1, nullptr, out, s);
    if (st == ROM_OK) st = add_to_double(h, out, qb + (size_t)(j - 1) * td, s);
  }
  // q_ref = q0
  if (st == ROM_OK) st = sum_to_state(h, qb, qrbar, gq0, s);
  // the handle ends at the rollout's end state
  if (st == ROM_OK) st = restore(nseg);
  hipError_t e = hipStreamSynchronize(s);
  pod_ws_free(&pws);
  (void)hipFree(ws);
  ROM_TRY(st);
  if (e != hipSuccess) { set_error(hipGetErrorString(e)); return ROM_E_DEVICE; }
  return ROM_OK;
}

rom_status rom_online_vjp(rom_handle h, int32_t n_fine, int32_t n_ckpt, const void* qbar,
                          double* abar, double* phibar, double* sigbar, double* ycbar,
                          void* stream) {
  ROM_REQUIRE(h && qbar && abar && phibar && sigbar && ycbar, ROM_E_INVAL,
              "handle, qbar and the four gradient buffers are required");
  ROM_REQUIRE(n_fine >= 1, ROM_E_INVAL, "n_fine must be >= 1");
  ROM_REQUIRE(n_ckpt >= 0, ROM_E_INVAL, "n_ckpt must be >= 0");
  ROM_REQUIRE(h->has_rom, ROM_E_STATE, "no reduced state");
  ROM_REQUIRE(h->cfg.hyper == ROM_HR_NONE && h->cfg.problem == ROM_BURGERS, ROM_E_UNSUPPORTED,
              "the online adjoint covers the Galerkin (Burgers) path only");
  ROM_REQUIRE(h->cfg.update_rule == ROM_UPDATE_ISVD, ROM_E_UNSUPPORTED,
              "the online adjoint covers the iSVD update only");
  const rom_config& c = h->cfg;
  const int B = c.n_inst, r = c.r, n = r + 1, z = c.z;
  const int64_t T = n_fine;
  auto due = [&](int64_t nf) { return (nf + 1 - c.w_init) % z == 0; };
  {  // no re-orthonormalisation may fall inside the range
    int64_t nu = h->n_update;
    for (int64_t k = 0; k < T; ++k)
      if (due(h->n_fine + k)) {
        ++nu;
        ROM_REQUIRE(!(c.reorth_every > 0 && nu % c.reorth_every == 0), ROM_E_UNSUPPORTED,
                    "a re-orthonormalisation falls inside the adjoint's range");
      }
  }
  hipStream_t s = (hipStream_t)stream;
  h->last_stream = s;
  const bool f64 = c.precision == ROM_F64;
  const size_t phi_b = h->esz * (size_t)h->total_dof * r, y_b = h->esz * (size_t)h->total_dof;
  const size_t br = 8 * (size_t)B * r;
  const size_t state_b = phi_b + y_b + 2 * br;        // Phi, y_corr, sigma, a
  const size_t ev_b = phi_b + y_b + 3 * br + 8 * (size_t)B * n * n + 8 * (size_t)B * (2 * r + 2);
  const size_t td8 = 8 * (size_t)h->total_dof;
  const size_t evscr_b = 8 * event_vjp_scratch_doubles(h);
  // Phibar terms (a window's fine steps, and two per event) wait for one pass
  // over Phibar per window: up to KP = min(z + 2, kPhibarPending) of
  // (uv, lambda, a1)
  const int KP = std::min(z + 2, kPhibarPending);
  const size_t pend_b = (size_t)KP * (16 * (size_t)h->total_dof + 2 * br);
  // per recorded step: the partials of its first Galerkin pass, which is taken
  // at the previous step's converged state (that step's adjoint reuses them)
  const size_t tap_b = h->esz * (size_t)std::max(h->n_ptiles, 1) * kMaxR * kMaxR;
  auto ws_bytes = [&](int64_t C) {
    const int64_t S = (T + C - 1) / C, nseg = (T + S - 1) / S, E = S / z + 1;
    return (size_t)(nseg + 1) * state_b + (size_t)S * (br + tap_b) + (size_t)E * ev_b +
           2 * td8 + 2 * y_b + evscr_b + pend_b + 4096;
  };
  // n_ckpt = 0: one segment (nothing recomputed) when its records fit in half
  // of the free device memory, else ceil(sqrt(n_fine)) checkpoints
  int64_t C = n_ckpt;
  if (C <= 0) {
    size_t fr = 0, tot = 0;
    ROM_HIP_CHECK(hipMemGetInfo(&fr, &tot));
    C = ws_bytes(1) <= fr / 2 ? 1 : (int64_t)std::ceil(std::sqrt((double)T));
  }
  if (C > T) C = T;
  const int64_t S = (T + C - 1) / C;      // fine steps per segment
  const int64_t nseg = (T + S - 1) / S;
  const int64_t E = S / z + 1;            // events per segment, at most
  const size_t need = ws_bytes(C);
  char* ws = nullptr;
  ROM_TRY(alloc(&ws, need));
  struct Host { int64_t nf, nu, ne; };
  std::vector<Host> hc(nseg + 1);
  char* ck = ws;
  char* rec_a = ck + (size_t)(nseg + 1) * state_b;
  char* taps = rec_a + (size_t)S * br;
  char* ev = taps + (size_t)S * tap_b;
  double* scr0 = (double*)(ev + (size_t)E * ev_b);
  double* scr1 = scr0 + h->total_dof;
  char* rhs = (char*)(scr1 + h->total_dof);
  char* out = rhs + y_b;
  double* evscr = (double*)(((uintptr_t)(out + y_b) + 7) & ~(uintptr_t)7);
  double2* pend_uv = (double2*)(((uintptr_t)((char*)evscr + evscr_b) + 15) & ~(uintptr_t)15);
  double* pend_lam = (double*)(pend_uv + (size_t)KP * h->total_dof);
  double* pend_a1 = pend_lam + (size_t)KP * B * r;
  int npend = 0;
  auto flush = [&]() -> rom_status {
    const int K = npend;
    npend = 0;
    return launch_phibar_flush(h, K, pend_uv, pend_lam, pend_a1, phibar, s);
  };
  auto save = [&](int64_t j) -> rom_status {
    char* p = ck + (size_t)j * state_b;
    ROM_TRY(copy_words(h->Phi, p, phi_b, s));
    ROM_TRY(copy_words(h->y_corr, p + phi_b, y_b, s));
    ROM_TRY(copy_words(h->sigma, p + phi_b + y_b, br, s));
    ROM_TRY(copy_words(h->a, p + phi_b + y_b + br, br, s));
    hc[j] = Host{h->n_fine, h->n_update, h->n_events};
    return ROM_OK;
  };
  auto restore = [&](int64_t j) -> rom_status {
    const char* p = ck + (size_t)j * state_b;
    ROM_TRY(copy_words(p, h->Phi, phi_b, s));
    ROM_TRY(copy_words(p + phi_b, h->y_corr, y_b, s));
    ROM_TRY(copy_words(p + phi_b + y_b, h->sigma, br, s));
    ROM_TRY(copy_words(p + phi_b + y_b + br, h->a, br, s));
    h->n_fine = hc[j].nf;
    h->n_update = hc[j].nu;
    h->n_events = hc[j].ne;
    return ROM_OK;
  };
  // event record e: Phi_old, y_new, sigma_old, a_old, sigma_new, Ubar, pr
  auto ev_phi = [&](int64_t e) { return ev + (size_t)e * ev_b; };
  auto ev_y = [&](int64_t e) { return ev_phi(e) + phi_b; };
  auto ev_sold = [&](int64_t e) { return (double*)(ev_y(e) + y_b); };
  auto ev_aold = [&](int64_t e) { return ev_sold(e) + (size_t)B * r; };
  auto ev_snew = [&](int64_t e) { return ev_aold(e) + (size_t)B * r; };
  auto ev_u = [&](int64_t e) { return ev_snew(e) + (size_t)B * r; };
  auto ev_pr = [&](int64_t e) { return ev_u(e) + (size_t)B * n * n; };
  rom_status st = ROM_OK;
  // the fine steps of one segment from the handle's state, recording a after
  // every step and, per event (after[e] = its step), what its adjoint reads
  auto record = [&](int64_t L, std::vector<int64_t>& after) -> rom_status {
    rom_status st = ROM_OK;
    after.clear();
    for (int64_t k = 0; k < L && st == ROM_OK; ++k) {
      h->mpart_tap = taps + (size_t)k * tap_b;
      st = launch_rom_fine_step(h, s);
      h->mpart_tap = nullptr;
      if (st == ROM_OK) st = copy_words(h->a, rec_a + (size_t)k * br, br, s);
      if (st == ROM_OK && due(h->n_fine)) {
        const int64_t e = (int64_t)after.size();
        after.push_back(k);
        st = copy_words(h->Phi, ev_phi(e), phi_b, s);
        if (st == ROM_OK) st = copy_words(h->sigma, ev_sold(e), br, s);
        if (st == ROM_OK) st = copy_words(h->a, ev_aold(e), br, s);
        if (st == ROM_OK) st = fom_step_impl(h, h->y_corr, z * c.dt, h->y_corr, nullptr, s);
        if (st == ROM_OK) st = copy_words(h->y_corr, ev_y(e), y_b, s);
        if (st == ROM_OK) st = launch_isvd_core(h, h->y_corr, h->part, s);
        if (st == ROM_OK) st = copy_words(h->ubar, ev_u(e), 8 * (size_t)B * n * n, s);
        if (st == ROM_OK) st = copy_words(h->rstate, ev_pr(e), 8 * (size_t)B * (2 * r + 2), s);
        if (st == ROM_OK) st = copy_words(h->sigma, ev_snew(e), br, s);
        if (st == ROM_OK) st = launch_isvd_apply(h, s);
        h->n_update += 1;
        if (st == ROM_OK) st = launch_rebuild(h, s);
        h->n_events += 1;
      }
      h->n_fine += 1;
    }
    return st;
  };
  // forward: checkpoints at segment starts, and the end state; the last
  // segment is recorded on the way, so the backward pass starts without
  // recomputing it
  std::vector<int64_t> after_last;
  for (int64_t j = 0; j < nseg && st == ROM_OK; ++j) {
    st = save(j);
    const int64_t L = std::min(S, T - j * S);
    if (j + 1 < nseg)
      for (int64_t k = 0; k < L && st == ROM_OK; ++k) st = fine_step_impl(h, s);
    else if (st == ROM_OK)
      st = record(L, after_last);
  }
  // the end state (one segment: the backward pass leaves the handle there)
  if (st == ROM_OK && nseg > 1) st = save(nseg);
  // seed at the end state
  if (st == ROM_OK) st = launch_online_seed(h, qbar, abar, phibar, s);
  if (st == ROM_OK) st = fill_zero(sigbar, br, s);
  if (st == ROM_OK) st = fill_zero(ycbar, td8, s);
  // backward, one segment at a time
  for (int64_t j = nseg - 1; j >= 0 && st == ROM_OK; --j) {
    const int64_t L = std::min(S, T - j * S);
    std::vector<int64_t> after;   // event e follows fine step after[e] of the segment
    if (j + 1 == nseg) {
      after = after_last;   // recorded by the forward pass; the handle is at its end
    } else {
      st = restore(j);
      if (st == ROM_OK) st = record(L, after);
    }
    for (int64_t k = L - 1; k >= 0 && st == ROM_OK; --k) {
      int64_t e_next = -1;   // first event at or after step k: its Phi_old is step k's basis
      for (int64_t e = 0; e < (int64_t)after.size(); ++e)
        if (after[e] >= k) { e_next = e; break; }
      if (e_next >= 0 && after[e_next] == k) {
        const int64_t e = e_next;
        // the event reads Phibar with the pending step terms added (its first
        // pass adds them)
        st = launch_event_vjp(h, ev_phi(e), ev_y(e), ev_sold(e), ev_aold(e), ev_u(e), ev_pr(e),
                              ev_snew(e), abar, phibar, sigbar, ycbar, scr0, scr1, evscr, s,
                              nullptr, nullptr, &npend, KP, pend_uv, pend_lam, pend_a1);
        // coarse step y_new = BE(y_prev) over z dt: ybar <- J_r(y_new)^-T ybar
        if (st == ROM_OK) st = convert_words(ycbar, true, rhs, f64, h->total_dof, s);
        if (st == ROM_OK) st = launch_assemble_adjoint(h, ev_y(e), z * c.dt, rhs, s);
        if (st == ROM_OK) st = bt_solve(h, -1, nullptr, out, s);
        if (st == ROM_OK) st = convert_words(out, f64, ycbar, true, h->total_dof, s);
      }
      if (st != ROM_OK) break;
      void* phi_k = e_next >= 0 ? (void*)ev_phi(e_next) : h->Phi;
      double* a_k = (double*)(rec_a + (size_t)k * br);
      // J_g at a_k: step k + 1's first pass (same basis) if it was recorded,
      // else a pass here
      const bool ev_after = e_next >= 0 && after[e_next] == k;
      const void* mp = nullptr;
      if (k + 1 < L && !ev_after) {
        mp = taps + (size_t)(k + 1) * tap_b;
      } else {
        void* phi_live = h->Phi;
        double* a_live = h->a;
        h->Phi = phi_k;
        h->a = a_k;
        st = prepare_galerkin_pass(h, s);
        if (st == ROM_OK) st = launch_galerkin_pass(h, s);
        h->Phi = phi_live;
        h->a = a_live;
      }
      if (st == ROM_OK && npend == KP) st = flush();
      if (st == ROM_OK) {
        st = launch_step_vjp_deferred(h, phi_k, a_k, abar, pend_uv + (size_t)npend * h->total_dof,
                                      s, mp);
        if (st == ROM_OK) st = copy_words(abar, pend_lam + (size_t)npend * B * r, br, s);
        if (st == ROM_OK) st = copy_words(a_k, pend_a1 + (size_t)npend * B * r, br, s);
        ++npend;
      }
    }
  }
  if (st == ROM_OK) st = flush();
  if (st == ROM_OK && nseg > 1) st = restore(nseg);
  hipError_t e = hipStreamSynchronize(s);
  (void)hipFree(ws);
  ROM_TRY(st);
  if (e != hipSuccess) { set_error(hipGetErrorString(e)); return ROM_E_DEVICE; }
  return ROM_OK;
}

rom_status rom_autotune(rom_handle h, int32_t what, const void* q, int32_t* choice,
                        void* stream) {
  ROM_REQUIRE(h, ROM_E_INVAL, "handle is required");
  ROM_REQUIRE(what >= ROM_TUNE_RESIDUAL && what <= ROM_TUNE_BT_PART, ROM_E_INVAL,
              "unknown tuning target");
  ROM_REQUIRE(q || what == ROM_TUNE_DEIM_PASS, ROM_E_INVAL, "q is required for this target");
  if (what == ROM_TUNE_DEIM_PASS)
    ROM_REQUIRE(h->has_rom, ROM_E_STATE, "the DEIM pass needs a reduced state");
  hipStream_t s = (hipStream_t)stream;
  h->last_stream = s;
  int n = 0;
  ROM_TRY(rom_set_tuning(h, what, -1, &n));
  int best = 0;
  if (n > 1) {
    hipEvent_t e0, e1;
    ROM_HIP_CHECK(hipEventCreate(&e0));
    ROM_HIP_CHECK(hipEventCreate(&e1));
    const int warm = what == ROM_TUNE_RESIDUAL ? 2 : 1, reps = what == ROM_TUNE_RESIDUAL ? 5 : 3;
    auto run = [&]() -> rom_status {
      switch (what) {
        case ROM_TUNE_RESIDUAL: return launch_residual(h, q, nullptr, 0.0, h->vjp_tmp, s);
        case ROM_TUNE_DEIM_PASS: return launch_rebuild(h, s);
        default: return fom_step_impl(h, q, h->cfg.dt, h->fq_prev, nullptr, s);
      }
    };
    float tbest = 0.f;
    rom_status st = ROM_OK;
    for (int i = 0; i < n && st == ROM_OK; ++i) {
      st = rom_set_tuning(h, what, i, nullptr);
      for (int w = 0; w < warm && st == ROM_OK; ++w) st = run();
      if (st != ROM_OK) break;
      ROM_HIP_CHECK(hipEventRecord(e0, s));
      for (int k = 0; k < reps && st == ROM_OK; ++k) st = run();
      ROM_HIP_CHECK(hipEventRecord(e1, s));
      ROM_HIP_CHECK(hipEventSynchronize(e1));
      float t = 0.f;
      ROM_HIP_CHECK(hipEventElapsedTime(&t, e0, e1));
      if (i == 0 || t < tbest) { tbest = t; best = i; }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    ROM_TRY(st);
  }
  ROM_TRY(rom_set_tuning(h, what, best, nullptr));
  if (choice) *choice = best;
  return ROM_OK;
}

rom_status rom_set_tuning(rom_handle h, int32_t what, int32_t choice, int32_t* n_candidates) {
  ROM_REQUIRE(h, ROM_E_INVAL, "handle is required");
  ROM_REQUIRE(what >= ROM_TUNE_RESIDUAL && what <= ROM_TUNE_BT_PART, ROM_E_INVAL,
              "unknown tuning target");
  static const int kSplits[] = {4, 2, 8};
  int parts[4] = {0, 0, 0, 0};
  int n = 1;
  if (what == ROM_TUNE_RESIDUAL) n = residual_shape_count(h);
  else if (what == ROM_TUNE_DEIM_PASS) n = h->cfg.hyper == ROM_HR_DEIM ? 3 : 1;
  else n = bt_part_candidates(h->nv, parts);
  if (n_candidates) *n_candidates = n;
  if (choice < 0) return ROM_OK;  // query only
  ROM_REQUIRE(choice < n, ROM_E_INVAL, "tuning choice out of range");
  if (what == ROM_TUNE_RESIDUAL) {
    h->tune_residual = choice;
  } else if (what == ROM_TUNE_DEIM_PASS) {
    if (h->cfg.hyper == ROM_HR_DEIM && h->deim_split != kSplits[choice]) {
      // captured windows hold the split as a launch argument
      ROM_HIP_CHECK(hipStreamSynchronize(h->last_stream));
      for (auto& g : h->win_exec)
        if (g) { (void)hipGraphExecDestroy(g); g = nullptr; }
      h->deim_split = kSplits[choice];
    }
  } else if (parts[choice] != h->bt_m) {
    // the solver's levels depend on the part size: re-create them (captured
    // windows refer to the old ones)
    ROM_HIP_CHECK(hipStreamSynchronize(h->last_stream));
    ROM_HIP_CHECK(hipDeviceSynchronize());
    for (auto& g : h->win_exec)
      if (g) { (void)hipGraphExecDestroy(g); g = nullptr; }
    bt_free(h);
    h->bt_m_req = parts[choice];
    ROM_TRY(bt_setup(h));
    ROM_HIP_CHECK(hipDeviceSynchronize());
  }
  return ROM_OK;
}

rom_status rom_profile(rom_handle h, int32_t stage, int32_t reps, const void* q, double* ms,
                       void* stream) {
  ROM_REQUIRE(h && ms, ROM_E_INVAL, "handle and ms are required");
  ROM_REQUIRE(reps >= 1, ROM_E_INVAL, "reps must be >= 1");
  ROM_REQUIRE(stage >= ROM_PROF_RESIDUAL && stage <= ROM_PROF_FOM_STEP, ROM_E_INVAL, "unknown stage");
  ROM_REQUIRE(q || stage == ROM_PROF_GALERKIN_PASS, ROM_E_INVAL, "q is required for this stage");
  ROM_REQUIRE(h->cfg.scheme == ROM_SCHEME_BE || stage != ROM_PROF_RESIDUAL_VJP, ROM_E_UNSUPPORTED,
              "the explicit scheme has no residual adjoint");
  hipStream_t s = (hipStream_t)stream;
  h->last_stream = s;
  // the Galerkin pass writes only scratch: a and the flags stay intact
  hipEvent_t e0, e1;
  ROM_HIP_CHECK(hipEventCreate(&e0));
  ROM_HIP_CHECK(hipEventCreate(&e1));
  rom_status st = ROM_OK;
  if (stage == ROM_PROF_GALERKIN_PASS) st = prepare_galerkin_pass(h, s);
  ROM_HIP_CHECK(hipEventRecord(e0, s));
  for (int i = 0; i < reps && st == ROM_OK; ++i) {
    switch (stage) {
      case ROM_PROF_RESIDUAL:
        st = h->cfg.scheme == ROM_SCHEME_SSPRK43
                 ? launch_residual2(h, q, h->vjp_tmp, s)
                 : launch_residual(h, q, nullptr, 0.0, h->vjp_tmp, s);
        break;
      case ROM_PROF_GALERKIN_PASS: st = launch_galerkin_pass(h, s); break;
      case ROM_PROF_ISVD_PROJECT: st = launch_isvd_project(h, q, s); break;
      case ROM_PROF_RESIDUAL_VJP:
        st = launch_residual_vjp(h, q, nullptr, 0.0, q, h->vjp_tmp, nullptr, s);
        break;
      case ROM_PROF_FOM_STEP: st = fom_step_impl(h, q, h->cfg.dt, h->fq_prev, nullptr, s); break;
    }
  }
  ROM_HIP_CHECK(hipEventRecord(e1, s));
  ROM_HIP_CHECK(hipEventSynchronize(e1));
  float t = 0.f;
  ROM_HIP_CHECK(hipEventElapsedTime(&t, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != ROM_OK) return st;
  *ms = (double)t / reps;
  return ROM_OK;
}

}  // extern "C"
