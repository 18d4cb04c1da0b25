// Reverse mode of Alg. 1's offline stage (an extension; the paper has no
// adjoint), the last part of the gradient of a final-state loss with respect
// to the initial state q0 through the whole method.  Given the adjoints of the
// state the online loop starts from (abar of a^{w_init}, Phibar of the POD
// basis, sigbar of its singular values, ybar of the first correction state)
// and the accumulated adjoints of q_ref and of D's diagonal:
//
//  * a^{w_init} = Phi^T D (q_w - q_ref): Phibar += D (q_w - q_ref) abar^T,
//    with t = Phi abar: Qbar_w += D t, qrbar -= D t, dvbar[v] += sum t (q_w - q_ref);
//  * (Phi, sigma) = the leading r left singular vectors and values of the
//    preprocessed training matrix X = D (Q - q_ref 1^T) = Q_pod R (the CGS2 QR
//    of the forward POD), X = U S V^T with U = Q_pod U_R and V = R^T U_R S^-1:
//    Xbar = U (F o (U^T Ubar - Ubar^T U) S + diag(sbar)) V^T + (I - U U^T) Ubar S^-1 V^T
//    (Ubar = [Phibar, 0], sbar = [sigbar, 0], F_ij = 1/(s_j^2 - s_i^2)), formed
//    as Xbar = Q_pod C + Phibar E with the small matrices
//    C = U_R G V^T - Z S_r^-1 V_r^T, E = S_r^-1 V_r^T, Z = Q_pod^T Phibar;
//    then Qbar_j += D Xbar_j, qrbar -= sum_j D Xbar_j, dvbar[v] += sum Xbar (Q - q_ref);
//  * d_v = 1 / phi_v with phi_v the mean square of (Q - q_ref) over the cells
//    and snapshots of variable v: phibar_v = -dvbar_v d_v^2, and
//    Qbar_j += 2 phibar_v (Q_j - q_ref) / (n_cell w), qrbar -= the sum over j.
//
// The coarse step and the training BE steps are transposed banded solves done
// by the caller.  Per-tile partial sums are reduced per instance in tile order,
// so every result is independent of scheduling.
#include "internal.h"
#include "physics.h"

namespace romhip {
namespace {

constexpr int kRT = 256;   // threads per pass tile block

// dvbar partials of one tile: per thread one sum per variable, then a block
// reduction per variable into part[tile * 12 + v]
DEV void tile_dv(double (&dva)[12], int nv, double* red, double* part) {
  const int tid = threadIdx.x;
  for (int v = 0; v < nv; ++v) {
    double x = dva[v];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off);
    __syncthreads();
    if ((tid & 63) == 0) red[tid >> 6] = x;
    __syncthreads();
    if (tid == 0) {
      double s = 0.0;
      for (int q = 0; q < (int)(blockDim.x >> 6); ++q) s += red[q];
      part[(size_t)blockIdx.x * 12 + v] = s;
    }
  }
}

DEV void dv_add(double (&dva)[12], int v, double x) {
#pragma unroll
  for (int u = 0; u < 12; ++u)
    if (u == v) dva[u] += x;
}

// a^{w_init} = Phi^T D (q_w - q_ref) backward, over pass tiles
template <typename T>
__global__ __launch_bounds__(kRT) void k_offline_a_vjp(
    const Tile* __restrict__ tiles, const int64_t* __restrict__ dof_off, int r, int nv,
    const double* __restrict__ dvar, const T* __restrict__ Phi, const T* __restrict__ qw,
    const T* __restrict__ qref, const double* __restrict__ abar, double* __restrict__ phibar,
    double* __restrict__ qbw, double* __restrict__ qrbar, double* __restrict__ part) {
  __shared__ double sab[kMaxR];
  __shared__ double red[kRT / 64];
  const Tile t = tiles[blockIdx.x];
  const int b = t.inst, tid = threadIdx.x;
  const int64_t base = dof_off[b];
  const double* dvb = dvar + (size_t)b * nv;
  for (int c = tid; c < r; c += kRT) sab[c] = abar[(size_t)b * r + c];
  __syncthreads();
  double dva[12];
  for (int v = 0; v < 12; ++v) dva[v] = 0.0;
  for (int64_t rr = tid; rr < t.ncell; rr += kRT) {
    const int64_t lr = t.cell0 + rr, g = base + lr;
    const int v = (int)(lr % nv);
    const double d = dvb[v];
    const double x = (double)qw[g] - (double)qref[g];
    double tt = 0.0;
    for (int c = 0; c < r; ++c) {
      tt += (double)Phi[g * r + c] * sab[c];
      phibar[g * r + c] += d * x * sab[c];
    }
    qbw[g] += d * tt;
    qrbar[g] -= d * tt;
    dv_add(dva, v, tt * x);
  }
  tile_dv(dva, nv, red, part);
}

// Z = Q_pod^T Phibar per tile (w x r partials, row-major)
template <typename T>
__global__ __launch_bounds__(kRT) void k_offline_qtz(const Tile* __restrict__ tiles,
                                                     const int64_t* __restrict__ dof_off, int r,
                                                     int w, const T* __restrict__ Qp,
                                                     const double* __restrict__ phibar,
                                                     double* __restrict__ zpart) {
  const Tile t = tiles[blockIdx.x];
  const int b = t.inst, tid = threadIdx.x;
  const int64_t base = dof_off[b];
  double* out = zpart + (size_t)blockIdx.x * w * r;
  // one thread per (k, c) entry, rows in order
  for (int e = tid; e < w * r; e += kRT) {
    const int k = e / r, c = e - k * r;
    double s = 0.0;
    for (int64_t rr = 0; rr < t.ncell; ++rr) {
      const int64_t g = base + t.cell0 + rr;
      s += (double)Qp[g * w + k] * phibar[g * r + c];
    }
    out[e] = s;
  }
}

// per instance: dst[b][e] = sum over the instance's tiles (in order) of part[tile][e]
__global__ void k_tile_sum(const int* __restrict__ tfirst, const double* __restrict__ part,
                           int ne, int ldp, double* __restrict__ dst, int add) {
  const int b = blockIdx.x;
  for (int e = threadIdx.x; e < ne; e += blockDim.x) {
    double s = 0.0;
    for (int tt = tfirst[b]; tt < tfirst[b + 1]; ++tt) s += part[(size_t)tt * ldp + e];
    if (add) dst[(size_t)b * ne + e] += s;
    else dst[(size_t)b * ne + e] = s;
  }
}

// Xbar rows = Q_pod C + Phibar E; its terms into Qbar_1..w, qrbar and dvbar
template <typename T>
__global__ __launch_bounds__(kRT) void k_offline_xbar(
    const Tile* __restrict__ tiles, const int64_t* __restrict__ dof_off, int64_t total, int r,
    int w, int nv, const double* __restrict__ dvar, const T* __restrict__ Qp,
    const double* __restrict__ phibar, const double* __restrict__ Cm,
    const double* __restrict__ Em, const T* __restrict__ Qtr, const T* __restrict__ qref,
    double* __restrict__ qb, double* __restrict__ qrbar, double* __restrict__ part) {
  __shared__ double red[kRT / 64];
  const Tile t = tiles[blockIdx.x];
  const int b = t.inst, tid = threadIdx.x;
  const int64_t base = dof_off[b];
  const double* dvb = dvar + (size_t)b * nv;
  const double* C = Cm + (size_t)b * w * w;
  const double* E = Em + (size_t)b * r * w;
  double dva[12];
  for (int v = 0; v < 12; ++v) dva[v] = 0.0;
  for (int64_t rr = tid; rr < t.ncell; rr += kRT) {
    const int64_t lr = t.cell0 + rr, g = base + lr;
    const int v = (int)(lr % nv);
    const double d = dvb[v];
    const double qr = (double)qref[g];
    double srow = 0.0, sdv = 0.0;
    for (int j = 0; j < w; ++j) {
      double x = 0.0;
      for (int k = 0; k < w; ++k) x += (double)Qp[g * w + k] * C[k * w + j];
      for (int c = 0; c < r; ++c) x += phibar[g * r + c] * E[c * w + j];
      qb[(size_t)(j + 1) * total + g] += d * x;
      srow += d * x;
      sdv += x * ((double)Qtr[(size_t)j * total + g] - qr);
    }
    qrbar[g] -= srow;
    dv_add(dva, v, sdv);
  }
  tile_dv(dva, nv, red, part);
}

// the preprocessing scale: phibar_v = -dvbar_v d_v^2 and the mean square's terms
template <typename T>
__global__ __launch_bounds__(kRT) void k_offline_scale(
    const Tile* __restrict__ tiles, const int64_t* __restrict__ dof_off, int64_t total, int w,
    int nv, const double* __restrict__ dvar, const double* __restrict__ dvbar,
    const T* __restrict__ Qtr, const T* __restrict__ qref, double* __restrict__ qb,
    double* __restrict__ qrbar) {
  const Tile t = tiles[blockIdx.x];
  const int b = t.inst, tid = threadIdx.x;
  const int64_t base = dof_off[b];
  const double ncell = (double)(t.n);
  for (int64_t rr = tid; rr < t.ncell; rr += kRT) {
    const int64_t lr = t.cell0 + rr, g = base + lr;
    const int v = (int)(lr % nv);
    const double d = dvar[(size_t)b * nv + v];
    const double fb = -dvbar[(size_t)b * nv + v] * d * d;
    const double cf = 2.0 * fb / (ncell * (double)w);
    const double qr = (double)qref[g];
    double srow = 0.0;
    for (int j = 0; j < w; ++j) {
      const double x = cf * ((double)Qtr[(size_t)j * total + g] - qr);
      qb[(size_t)(j + 1) * total + g] += x;
      srow += x;
    }
    qrbar[g] -= srow;
  }
}

// dst (FP64) += src (T), or dst (T) = a + b (FP64)
template <typename T>
__global__ __launch_bounds__(256) void k_add_to_double(int64_t n, const T* __restrict__ src,
                                                        double* __restrict__ dst) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] += (double)src[i];
}

template <typename T>
__global__ __launch_bounds__(256) void k_sum_to(int64_t n, const double* __restrict__ x,
                                                const double* __restrict__ y, T* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = (T)(x[i] + y[i]);
}

template <class X> struct TagT { using type = X; };

}  // namespace

size_t offline_vjp_part_doubles(const rom_batch* h, int w) {
  const size_t nt = (size_t)std::max(h->n_ptiles, 1);
  return std::max(nt * 12, nt * (size_t)w * h->cfg.r);
}

rom_status launch_offline_a_vjp(rom_batch* h, const void* Phi0, const void* qw, const double* abar,
                                double* phibar, double* qbw, double* qrbar, double* dvbar,
                                double* part, hipStream_t s) {
  const int B = h->cfg.n_inst, r = h->cfg.r, nv = h->nv;
  auto go = [&](auto tag) {
    using T = typename decltype(tag)::type;
    hipLaunchKernelGGL((k_offline_a_vjp<T>), dim3(h->n_ptiles), dim3(kRT), 0, s, h->d_ptiles,
                       h->d_dof_off, r, nv, h->d_var, (const T*)Phi0, (const T*)qw,
                       (const T*)h->q_ref, abar, phibar, qbw, qrbar, part);
  };
  if (h->cfg.precision == ROM_F64) go(TagT<double>{});
  else go(TagT<float>{});
  hipLaunchKernelGGL(k_tile_sum, dim3(B), dim3(64), 0, s, h->d_ptile_first, part, nv, 12, dvbar, 1);
  ROM_HIP_CHECK(hipGetLastError());
  return ROM_OK;
}

// POD backward: Z = Q_pod^T Phibar, the small matrices (isvd.hip), then the
// Xbar terms; finally the preprocessing scale (dvbar complete by then)
rom_status launch_offline_pod_vjp(rom_batch* h, const PodWs& ws, int w, const void* Qtr,
                                  const double* phibar, const double* sigbar, double* qb,
                                  double* qrbar, double* dvbar, double* part, double* small,
                                  hipStream_t s) {
  const int B = h->cfg.n_inst, r = h->cfg.r, nv = h->nv;
  double* Z = small;                           // [B][w][r]
  double* Cm = Z + (size_t)B * w * r;          // [B][w][w]
  double* Em = Cm + (size_t)B * w * w;         // [B][r][w]
  double* scr = Em + (size_t)B * r * w;        // [B][3 w w]: U_R, V, G V^T
  auto go = [&](auto tag) -> rom_status {
    using T = typename decltype(tag)::type;
    hipLaunchKernelGGL((k_offline_qtz<T>), dim3(h->n_ptiles), dim3(kRT), 0, s, h->d_ptiles,
                       h->d_dof_off, r, w, (const T*)ws.Q, phibar, part);
    hipLaunchKernelGGL(k_tile_sum, dim3(B), dim3(256), 0, s, h->d_ptile_first, part, w * r,
                       w * r, Z, 0);
    ROM_TRY(launch_pod_vjp_small(h, ws.R, w, Z, sigbar, Cm, Em, scr, s));
    hipLaunchKernelGGL((k_offline_xbar<T>), dim3(h->n_ptiles), dim3(kRT), 0, s, h->d_ptiles,
                       h->d_dof_off, h->total_dof, r, w, nv, h->d_var, (const T*)ws.Q, phibar,
                       Cm, Em, (const T*)Qtr, (const T*)h->q_ref, qb, qrbar, part);
    hipLaunchKernelGGL(k_tile_sum, dim3(B), dim3(64), 0, s, h->d_ptile_first, part, nv, 12,
                       dvbar, 1);
    hipLaunchKernelGGL((k_offline_scale<T>), dim3(h->n_ptiles), dim3(kRT), 0, s, h->d_ptiles,
                       h->d_dof_off, h->total_dof, w, nv, h->d_var, dvbar, (const T*)Qtr,
                       (const T*)h->q_ref, qb, qrbar);
    ROM_HIP_CHECK(hipGetLastError());
    return ROM_OK;
  };
  if (h->cfg.precision == ROM_F64) return go(TagT<double>{});
  return go(TagT<float>{});
}

rom_status add_to_double(rom_batch* h, const void* src, double* dst, hipStream_t s) {
  const int64_t n = h->total_dof;
  const unsigned grid = (unsigned)((n + 255) / 256);
  if (h->cfg.precision == ROM_F64)
    hipLaunchKernelGGL((k_add_to_double<double>), dim3(grid), dim3(256), 0, s, n,
                       (const double*)src, dst);
  else
    hipLaunchKernelGGL((k_add_to_double<float>), dim3(grid), dim3(256), 0, s, n,
                       (const float*)src, dst);
  ROM_HIP_CHECK(hipGetLastError());
  return ROM_OK;
}

rom_status sum_to_state(rom_batch* h, const double* x, const double* y, void* out, hipStream_t s) {
  const int64_t n = h->total_dof;
  const unsigned grid = (unsigned)((n + 255) / 256);
  if (h->cfg.precision == ROM_F64)
    hipLaunchKernelGGL((k_sum_to<double>), dim3(grid), dim3(256), 0, s, n, x, y, (double*)out);
  else
    hipLaunchKernelGGL((k_sum_to<float>), dim3(grid), dim3(256), 0, s, n, x, y, (float*)out);
  ROM_HIP_CHECK(hipGetLastError());
  return ROM_OK;
}

}  // namespace romhip
