// Sampling rules of the hyper-reduced ROM besides greedy DEIM (Sec. 3.2):
// QDEIM, the pivots of the column-pivoted QR factorisation of Phi^T
// (eq. qdeim_qr), and feature-guided sampling, QDEIM plus the cells where the
// gradient of a feature of the estimated future state is largest
// (eq. fgs_selection).
//
// QDEIM on the device.  Pivoted QR of Phi^T picks, at step k, the column of
// largest norm in the trailing block, i.e. the row phi_i of Phi farthest from
// the span of the rows already chosen.  Each instance keeps an orthonormal
// basis q_0 .. q_{k-1} of that span (FP64, r-vectors) and every row its
// squared distance nu_i = |phi_i|^2 - sum_j (q_j . phi_i)^2 (FP64), so a pick
// costs one pass over the basis: the pass subtracts the newest direction's
// share from every nu_i and proposes each tile's largest (lowest row on ties),
// then one block per instance takes the winner, marks it and
// orthonormalises it against the earlier directions (classical Gram-Schmidt,
// twice).  Feature-guided sampling then takes, n_s - r times, the cell of
// largest squared feature gradient whose feature row is not yet chosen.
#include <algorithm>

#include "internal.h"

namespace romhip {
namespace {

#define DEV __device__ __forceinline__

constexpr int kPassThreads = 256;
constexpr int kParts = 4;          // candidates per pass tile

DEV void better(double v, int64_t i, double& bv, int64_t& bi) {
  if (i >= 0 && (bi < 0 || v > bv || (v == bv && i < bi))) { bv = v; bi = i; }
}

// the block's best (value, index) from per-thread candidates; result in bv[0], bi[0]
DEV void block_best(double* bv, int64_t* bi) {
  for (int st = blockDim.x / 2; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) {
      double v = bv[threadIdx.x];
      int64_t i = bi[threadIdx.x];
      better(bv[threadIdx.x + st], bi[threadIdx.x + st], v, i);
      bv[threadIdx.x] = v;
      bi[threadIdx.x] = i;
    }
    __syncthreads();
  }
}

// One QDEIM pass over the rows of part `part` of a pass tile: k == 0 sets
// nu_i = |phi_i|^2; k > 0 subtracts (q_{k-1} . phi_i)^2.  Candidates: the
// largest nu_i among rows not chosen in this rebuild.
template <typename T>
__global__ __launch_bounds__(kPassThreads) void k_qdeim_pass(
    const Tile* __restrict__ tiles, const int64_t* __restrict__ dof_off,
    const T* __restrict__ Phi, int r, int k, const double* __restrict__ qs,
    double* __restrict__ nu, const uint32_t* __restrict__ chosen,
    const uint32_t* __restrict__ epoch_p, double* __restrict__ tval, int64_t* __restrict__ tidx) {
  __shared__ double sq[kMaxR];
  __shared__ double bv[kPassThreads];
  __shared__ int64_t bi[kPassThreads];
  const Tile t = tiles[blockIdx.x / kParts];
  const int part = blockIdx.x % kParts;
  const int b = t.inst, tid = threadIdx.x;
  const int64_t base = dof_off[b];
  const int64_t len = (t.ncell + kParts - 1) / kParts;
  const int64_t lo = t.cell0 + part * len;
  const int64_t hi = t.cell0 + ((part + 1) * len < t.ncell ? (part + 1) * len : t.ncell);
  const uint32_t epoch = *epoch_p;
  if (k > 0)
    for (int c = tid; c < r; c += blockDim.x) sq[c] = qs[((size_t)b * kMaxR + (k - 1)) * kMaxR + c];
  __syncthreads();
  double best = -1.0;
  int64_t bidx = -1;
  for (int64_t l = lo + tid; l < hi; l += blockDim.x) {
    const T* row = Phi + (base + l) * r;
    double v;
    if (k == 0) {
      v = 0.0;
      for (int c = 0; c < r; ++c) { const double x = (double)row[c]; v += x * x; }
    } else {
      double d = 0.0;
      for (int c = 0; c < r; ++c) d += (double)row[c] * sq[c];
      v = nu[base + l] - d * d;
    }
    nu[base + l] = v;
    if (chosen[base + l] != epoch) better(v, l, best, bidx);
  }
  bv[tid] = best;
  bi[tid] = bidx;
  __syncthreads();
  block_best(bv, bi);
  if (tid == 0) {
    tval[blockIdx.x] = bv[0];
    tidx[blockIdx.x] = bi[0];
  }
}

// Pick t of QDEIM: the instance's winner among its tiles' candidates, then the
// new direction q_t = normalised residual of phi_{p_t} against q_0 .. q_{t-1}.
template <typename T>
__global__ __launch_bounds__(kPassThreads) void k_qdeim_select(
    const int* __restrict__ tfirst, const double* __restrict__ tval,
    const int64_t* __restrict__ tidx, const int64_t* __restrict__ dof_off,
    const T* __restrict__ Phi, int r, int ns, int t, int32_t* __restrict__ P,
    uint32_t* __restrict__ chosen, const uint32_t* __restrict__ epoch_p,
    double* __restrict__ qs, uint32_t* flags) {
  __shared__ double bv[kPassThreads];
  __shared__ int64_t bi[kPassThreads];
  __shared__ double v[kMaxR];
  __shared__ double pc[kMaxR];
  __shared__ double nrm;
  const int b = blockIdx.x, tid = threadIdx.x;
  double best = -1.0;
  int64_t bidx = -1;
  for (int tt = tfirst[b] * kParts + tid; tt < tfirst[b + 1] * kParts; tt += blockDim.x)
    better(tval[tt], tidx[tt], best, bidx);
  bv[tid] = best;
  bi[tid] = bidx;
  __syncthreads();
  block_best(bv, bi);
  int64_t w = bi[0];
  if (tid == 0) {
    if (w < 0 || !(bv[0] > 0.0)) atomicOr(&flags[b], ROM_FLAG_SINGULAR);
    if (w < 0) w = 0;
    P[(size_t)b * ns + t] = (int32_t)w;
    chosen[dof_off[b] + w] = *epoch_p;
  }
  if (w < 0) w = 0;
  if (t + 1 >= r) return;          // no later QDEIM pass needs q_t
  double* Qb = qs + (size_t)b * kMaxR * kMaxR;
  for (int c = tid; c < r; c += blockDim.x) v[c] = (double)Phi[(dof_off[b] + w) * r + c];
  __syncthreads();
  for (int pass = 0; pass < 2; ++pass) {
    for (int j = tid; j < t; j += blockDim.x) {
      double d = 0.0;
      for (int c = 0; c < r; ++c) d += Qb[j * kMaxR + c] * v[c];
      pc[j] = d;
    }
    __syncthreads();
    for (int c = tid; c < r; c += blockDim.x) {
      double d = v[c];
      for (int j = 0; j < t; ++j) d -= Qb[j * kMaxR + c] * pc[j];
      v[c] = d;
    }
    __syncthreads();
  }
  if (tid == 0) {
    double s = 0.0;
    for (int c = 0; c < r; ++c) s += v[c] * v[c];
    nrm = sqrt(s);
  }
  __syncthreads();
  const double inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
  for (int c = tid; c < r; c += blockDim.x) Qb[t * kMaxR + c] = v[c] * inv;
}

// ||grad theta||^2 per cell, theta = variable `feat` of the estimated future
// state, centred differences on the unit interval (periodic wrap, or the
// zero-gradient ghosts of the walls)
template <typename T>
__global__ __launch_bounds__(256) void k_fgs_grad(const Tile* __restrict__ tiles,
                                                  const int64_t* __restrict__ dof_off,
                                                  const int64_t* __restrict__ cell_off,
                                                  const T* __restrict__ y, int nv, int feat,
                                                  int periodic, double* __restrict__ g) {
  const Tile t = tiles[blockIdx.x];
  const int b = t.inst;
  const int64_t base = dof_off[b], n = t.n;
  for (int64_t cc = threadIdx.x; cc < t.ncell; cc += blockDim.x) {
    const int64_t c = t.cell0 + cc;
    int64_t cp = c + 1, cm = c - 1;
    if (periodic) { cp = cp == n ? 0 : cp; cm = cm < 0 ? n - 1 : cm; }
    else { cp = cp == n ? n - 1 : cp; cm = cm < 0 ? 0 : cm; }
    const double d = ((double)y[base + cp * nv + feat] - (double)y[base + cm * nv + feat]) *
                     ((double)n * 0.5);
    g[cell_off[b] + c] = d * d;
  }
}

// candidates of one FGS pick: the largest g among cells whose feature row is
// not chosen (lowest cell on ties), one per cell tile
__global__ __launch_bounds__(256) void k_fgs_argmax(const Tile* __restrict__ tiles,
                                                    const int64_t* __restrict__ dof_off,
                                                    const int64_t* __restrict__ cell_off,
                                                    const double* __restrict__ g, int nv, int feat,
                                                    const uint32_t* __restrict__ chosen,
                                                    const uint32_t* __restrict__ epoch_p,
                                                    double* __restrict__ tval,
                                                    int64_t* __restrict__ tidx) {
  __shared__ double bv[256];
  __shared__ int64_t bi[256];
  const Tile t = tiles[blockIdx.x];
  const int b = t.inst, tid = threadIdx.x;
  const uint32_t epoch = *epoch_p;
  double best = -1.0;
  int64_t bidx = -1;
  for (int64_t cc = tid; cc < t.ncell; cc += blockDim.x) {
    const int64_t c = t.cell0 + cc;
    if (chosen[dof_off[b] + c * nv + feat] != epoch) better(g[cell_off[b] + c], c, best, bidx);
  }
  bv[tid] = best;
  bi[tid] = bidx;
  __syncthreads();
  block_best(bv, bi);
  if (tid == 0) {
    tval[blockIdx.x] = bv[0];
    tidx[blockIdx.x] = bi[0];
  }
}

// FGS pick t: the instance's best cell over its tiles [tfirst[b], tfirst[b+1])
__global__ __launch_bounds__(256) void k_fgs_select(const int* __restrict__ tfirst,
                                                    const double* __restrict__ tval,
                                                    const int64_t* __restrict__ tidx,
                                                    const int64_t* __restrict__ dof_off, int nv,
                                                    int feat, int ns, int t,
                                                    int32_t* __restrict__ P,
                                                    uint32_t* __restrict__ chosen,
                                                    const uint32_t* __restrict__ epoch_p,
                                                    uint32_t* flags) {
  __shared__ double bv[256];
  __shared__ int64_t bi[256];
  const int b = blockIdx.x, tid = threadIdx.x;
  double best = -1.0;
  int64_t bidx = -1;
  for (int tt = tfirst[b] + tid; tt < tfirst[b + 1]; tt += blockDim.x)
    better(tval[tt], tidx[tt], best, bidx);
  bv[tid] = best;
  bi[tid] = bidx;
  __syncthreads();
  block_best(bv, bi);
  if (tid == 0) {
    int64_t c = bi[0];
    if (c < 0) { c = 0; atomicOr(&flags[b], ROM_FLAG_SINGULAR); }
    const int64_t row = c * nv + feat;
    P[(size_t)b * ns + t] = (int32_t)row;
    chosen[dof_off[b] + row] = *epoch_p;
  }
}

__global__ void k_bump_epoch(uint32_t* e) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *e = *e + 1u;
}

}  // namespace

int fgs_feature(int problem) { return problem == ROM_REACT ? 10 : 0; }

template <typename T>
static rom_status qdeim_t(rom_batch* h, hipStream_t s) {
  const int r = h->cfg.r, ns = h->cfg.n_s, B = h->cfg.n_inst;
  hipLaunchKernelGGL(k_bump_epoch, dim3(1), dim3(64), 0, s, h->d_epoch);
  double* tval = h->part;
  int64_t* tidx = (int64_t*)(h->part + std::max((size_t)kParts * h->n_ptiles, (size_t)h->n_tiles));
  double* nu = h->qtmp;
  for (int k = 0; k < r; ++k) {
    hipLaunchKernelGGL((k_qdeim_pass<T>), dim3(h->n_ptiles * kParts), dim3(kPassThreads), 0, s,
                       h->d_ptiles, h->d_dof_off, (const T*)h->Phi, r, k, h->qdeim_q, nu,
                       h->chosen, h->d_epoch, tval, tidx);
    hipLaunchKernelGGL((k_qdeim_select<T>), dim3(B), dim3(kPassThreads), 0, s, h->d_ptile_first,
                       tval, tidx, h->d_dof_off, (const T*)h->Phi, r, ns, k, h->P, h->chosen,
                       h->d_epoch, h->qdeim_q, h->flags);
  }
  if (h->cfg.hyper == ROM_HR_QDEIM_FGS && ns > r) {
    const int feat = fgs_feature(h->cfg.problem);
    const int periodic = (h->cfg.problem == ROM_BURGERS || h->cfg.problem == ROM_REACT) ? 1 : 0;
    hipLaunchKernelGGL((k_fgs_grad<T>), dim3(h->n_tiles), dim3(256), 0, s, h->d_tiles,
                       h->d_dof_off, h->d_cell_off, (const T*)h->y_corr, h->nv, feat, periodic,
                       h->fgs_g);
    for (int t = r; t < ns; ++t) {
      hipLaunchKernelGGL(k_fgs_argmax, dim3(h->n_tiles), dim3(256), 0, s, h->d_tiles,
                         h->d_dof_off, h->d_cell_off, h->fgs_g, h->nv, feat, h->chosen,
                         h->d_epoch, tval, tidx);
      hipLaunchKernelGGL(k_fgs_select, dim3(B), dim3(256), 0, s, h->d_tile_first, tval, tidx,
                         h->d_dof_off, h->nv, feat, ns, t, h->P, h->chosen, h->d_epoch, h->flags);
    }
  }
  ROM_HIP_CHECK(hipGetLastError());
  return ROM_OK;
}

rom_status launch_qdeim(rom_batch* h, hipStream_t s) {
  return h->cfg.precision == ROM_F64 ? qdeim_t<double>(h, s) : qdeim_t<float>(h, s);
}

}  // namespace romhip
