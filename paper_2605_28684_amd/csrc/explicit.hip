// The explicit path of the detonation case's ROM structure (Sec. 5.3: a
// Galerkin ROM because the full-order solver is explicit; App. D: four-stage
// third-order SSP Runge-Kutta, a cell-centred second-order finite volume
// discretisation with a Barth-Jespersen limiter).
//
//  * k_residual2: f of the second-order discretisation.  Each face takes the
//    limited linear reconstructions of its two cells, q_i +- psi_i s_i / 2 with
//    the centred slope s_i = (q_{i+1} - q_{i-1}) / 2 and the Barth-Jespersen
//    factor psi_i = min(1, min(dmax_i, -dmin_i) / (|s_i| / 2)) (dmax, dmin:
//    the largest and smallest neighbour differences; psi = 1 where s_i = 0),
//    and the model's two-point flux; diffusion and sources are the first-order
//    model's.  Tiles of kTile cells with two halo cells on each side (wrap for
//    periodic models, copies of the end cell at zero-gradient walls).
//  * SSPRK(4,3) (Spiteri and Ruuth): y1 = y + dt/2 L(y), y2 = y1 + dt/2 L(y1),
//    y3 = 2/3 y + 1/3 y2 + dt/6 L(y2), y+ = y3 + dt/2 L(y3): the full-order
//    step (four residual launches and four stage combinations in FP64) and
//    the DEIM-Galerkin step of eq. deim_galerkin_rom, da/dt = (P^T Phi)^+ P^T D
//    f(q_ref + D^-1 Phi a), one block per instance: every stage rebuilds the
//    state on the five-cell mesh of each sampled row (the cell and two on each
//    side, gathered after each rebuild), evaluates that row's limited residual
//    in FP64, and applies (P^T Phi)^+.
#pragma clang fp contract(off)

#include "internal.h"
#include "physics.h"

namespace romhip {
namespace {

// the limited right-face (sgn = +1) or left-face (sgn = -1) state of a cell
// from its value c and its neighbours m (left) and p (right)
template <typename T>
DEV T limited(T m, T c, T p, T sgn) {
  const T s = T(0.5) * (p - m);
  const T mx = (m > c ? m : c) > p ? (m > c ? m : c) : p;
  const T mn = (m < c ? m : c) < p ? (m < c ? m : c) : p;
  const T dmax = mx - c, dmin = mn - c;
  const T e = T(0.5) * (s >= T(0) ? s : -s);
  T psi = T(1);
  if (e > T(0)) {
    const T lim = (dmax < -dmin ? dmax : -dmin) / e;
    psi = lim < T(1) ? lim : T(1);
  }
  return c + sgn * (T(0.5) * psi * s);
}

template <class Mdl, typename T>
__global__ __launch_bounds__(kTile) void k_residual2(
    const Tile* __restrict__ tiles, const int64_t* __restrict__ dof_off,
    const int64_t* __restrict__ cell_off, const double* __restrict__ phys, int nphys,
    const T* __restrict__ q, T* __restrict__ out, uint32_t* flags) {
  constexpr int NV = Mdl::NV;
  __shared__ T sq[(kTile + 4) * NV];
  __shared__ T sH[(kTile + 1) * NV];
  const Tile t = tiles[blockIdx.x];
  const int b = t.inst;
  const int64_t n = cell_off[b + 1] - cell_off[b];
  const int nt = (int)t.ncell;
  const int64_t base = dof_off[b];
  Mdl m(phys + (size_t)b * nphys);
  for (int e = threadIdx.x; e < (nt + 4) * NV; e += blockDim.x) {
    const int lc = e / NV, v = e - lc * NV;
    int64_t c = t.cell0 - 2 + lc;
    if (Mdl::periodic) { c = c < 0 ? c + n : (c >= n ? c - n : c); }
    else { c = c < 0 ? 0 : (c >= n ? n - 1 : c); }
    sq[e] = q[base + c * NV + v];
  }
  __syncthreads();
  unsigned fl = 0;
  // face k (k = 0 .. nt) between tile cells k-1 and k: LDS cell j sits at slot j+2
  for (int k = threadIdx.x; k <= nt; k += blockDim.x) {
    T L[NV], R[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      L[v] = limited(sq[(k + 0) * NV + v], sq[(k + 1) * NV + v], sq[(k + 2) * NV + v], T(1));
      R[v] = limited(sq[(k + 1) * NV + v], sq[(k + 2) * NV + v], sq[(k + 3) * NV + v], T(-1));
    }
    m.face(L, R, &sH[k * NV], fl);
  }
  __syncthreads();
  T f[NV];
  const int i = threadIdx.x;
  const T inv = T(n), inv2 = T(n) * T(n);
  if (i < nt) {
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const T qm = sq[(i + 1) * NV + v], q0 = sq[(i + 2) * NV + v], qp = sq[(i + 3) * NV + v];
      f[v] = -(sH[(i + 1) * NV + v] - sH[i * NV + v]) * inv;
      const T kap = m.kappa(v);
      if (kap != T(0)) f[v] += kap * ((qp - q0) - (q0 - qm)) * inv2;
    }
    if (Mdl::has_source) {
      T S[NV];
      const double x = ((double)(t.cell0 + i) + 0.5) / (double)n;
      m.source(&sq[(i + 2) * NV], x, S, fl);
#pragma unroll
      for (int v = 0; v < NV; ++v) f[v] += S[v];
    }
  }
  __syncthreads();
  if (i < nt) {
#pragma unroll
    for (int v = 0; v < NV; ++v) sH[i * NV + v] = f[v];
  }
  __syncthreads();
  const int64_t o = base + t.cell0 * NV;
  for (int e = threadIdx.x; e < nt * NV; e += blockDim.x) {
    const T val = sH[e];
    if (!isfinite(val)) fl |= ROM_FLAG_NONFINITE;
    out[o + e] = val;
  }
  if (fl) atomicOr(&flags[b], fl);
}

// out = (ca x + cb y) + cc f, formed in FP64 (the stages of SSPRK(4,3)); out may
// alias x or y (one element per thread)
template <typename T>
__global__ __launch_bounds__(256) void k_ssp_combine(int64_t n, const T* x, const T* y,
                                                     const T* f, double ca, double cb, double cc,
                                                     T* out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double v = ca * (double)x[i];
  if (y) v = v + cb * (double)y[i];
  out[i] = (T)(v + cc * (double)f[i]);
}

// five-cell sample mesh: basis rows and q_ref of cells c-2 .. c+2 of every
// sampled row, FP64: phi5[((b ns + s) 5 + k) nv + v][r], qref5[(b ns + s) 5 + k) nv + v]
template <typename T>
__global__ __launch_bounds__(256) void k_mesh5(int r, int ns, int nv, int periodic,
                                               const int64_t* __restrict__ dof_off,
                                               const int64_t* __restrict__ cell_off,
                                               const T* __restrict__ Phi,
                                               const T* __restrict__ qref,
                                               const int32_t* __restrict__ P,
                                               double* __restrict__ phi5,
                                               double* __restrict__ qref5) {
  const int b = blockIdx.x;
  const int64_t base = dof_off[b], n = cell_off[b + 1] - cell_off[b];
  const int rows = ns * 5 * nv;
  for (int e = threadIdx.x; e < rows; e += blockDim.x) {
    const int s = e / (5 * nv), rem = e % (5 * nv), k = rem / nv, v = rem % nv;
    int64_t c = P[(size_t)b * ns + s] / nv + k - 2;
    if (periodic) { c = c < 0 ? c + n : (c >= n ? c - n : c); }
    else { c = c < 0 ? 0 : (c >= n ? n - 1 : c); }
    const int64_t g = base + c * nv + v;
    const size_t o = (size_t)b * rows + e;
    qref5[o] = (double)qref[g];
    for (int j = 0; j < r; ++j) phi5[o * r + j] = (double)Phi[g * r + j];
  }
}

// One SSPRK(4,3) step of the DEIM-Galerkin ROM per instance (one block each).
template <class Mdl>
__global__ __launch_bounds__(256) void k_hr_explicit_step(
    int r, int ns, const int64_t* __restrict__ cell_off, const double* __restrict__ phys,
    int nphys, const double* __restrict__ dvar, const int32_t* __restrict__ P,
    const double* __restrict__ M, const double* __restrict__ phi5,
    const double* __restrict__ qref5, double dt, double* __restrict__ a, uint32_t* flags) {
  constexpr int NV = Mdl::NV;
  extern __shared__ double sm[];
  const int b = blockIdx.x, tid = threadIdx.x;
  const int rows = ns * 5 * NV;
  double* qm = sm;                 // rows: the state on the sample mesh
  double* fs = qm + rows;          // ns: D f at the sampled rows
  double* x = fs + ns;             // r: the stage's reduced state
  double* a0 = x + r;              // r: a at the step start
  double* y = a0 + r;              // r: the running stage value
  const int64_t n = cell_off[b + 1] - cell_off[b];
  Mdl m(phys + (size_t)b * nphys);
  const double* dv = dvar + (size_t)b * NV;
  const double* Pb5 = phi5 + (size_t)b * rows * r;
  const double* Qb5 = qref5 + (size_t)b * rows;
  const double* Mb = M + (size_t)b * r * ns;
  for (int c = tid; c < r; c += blockDim.x) { a0[c] = a[(size_t)b * r + c]; x[c] = a0[c]; }
  __syncthreads();
  unsigned fl = 0;
  const double h = 0.5 * dt;
  for (int stage = 0; stage < 4; ++stage) {
    for (int e = tid; e < rows; e += blockDim.x) {
      double s = 0.0;
      for (int j = 0; j < r; ++j) s += Pb5[(size_t)e * r + j] * x[j];
      qm[e] = Qb5[e] + s / dv[e % NV];
    }
    __syncthreads();
    for (int si = tid; si < ns; si += blockDim.x) {
      const int row = P[(size_t)b * ns + si], v = row % NV;
      const double* q5 = qm + (size_t)si * 5 * NV;  // cells c-2 .. c+2
      double L[NV], R[NV], Hm[NV], Hp[NV];
#pragma unroll
      for (int w = 0; w < NV; ++w) {
        L[w] = limited(q5[0 * NV + w], q5[1 * NV + w], q5[2 * NV + w], 1.0);
        R[w] = limited(q5[1 * NV + w], q5[2 * NV + w], q5[3 * NV + w], -1.0);
      }
      m.face(L, R, Hm, fl);
#pragma unroll
      for (int w = 0; w < NV; ++w) {
        L[w] = limited(q5[1 * NV + w], q5[2 * NV + w], q5[3 * NV + w], 1.0);
        R[w] = limited(q5[2 * NV + w], q5[3 * NV + w], q5[4 * NV + w], -1.0);
      }
      m.face(L, R, Hp, fl);
      double f = -(Hp[v] - Hm[v]) * (double)n;
      const double kap = m.kappa(v);
      const double qmv = q5[1 * NV + v], q0 = q5[2 * NV + v], qpv = q5[3 * NV + v];
      if (kap != 0.0) f += kap * ((qpv - q0) - (q0 - qmv)) * ((double)n * (double)n);
      if (Mdl::has_source) {
        double S[NV];
        const double xc = ((double)(row / NV) + 0.5) / (double)n;
        m.source(q5 + 2 * NV, xc, S, fl);
        f += S[v];
      }
      if (!isfinite(f)) fl |= ROM_FLAG_NONFINITE;
      fs[si] = dv[v] * f;
    }
    __syncthreads();
    for (int i = tid; i < r; i += blockDim.x) {
      double Lr = 0.0;
      for (int si = 0; si < ns; ++si) Lr += Mb[(size_t)i * ns + si] * fs[si];
      double nx;
      if (stage == 0) nx = a0[i] + h * Lr;
      else if (stage == 1) nx = x[i] + h * Lr;
      else if (stage == 2) nx = ((2.0 / 3.0) * a0[i] + (1.0 / 3.0) * x[i]) + (dt / 6.0) * Lr;
      else nx = x[i] + h * Lr;
      y[i] = nx;
    }
    __syncthreads();
    for (int i = tid; i < r; i += blockDim.x) x[i] = y[i];
    __syncthreads();
  }
  for (int i = tid; i < r; i += blockDim.x) a[(size_t)b * r + i] = x[i];
  if (fl) atomicOr(&flags[b], fl);
}

template <class M> struct Tag2 { using type = M; };

template <typename T, class Fn>
rom_status with_model2(const rom_batch* h, Fn&& fn) {
  switch (h->cfg.problem) {
    case ROM_BURGERS: return fn(Tag2<BurgersModel<T>>{});
    case ROM_EULER_RUSANOV: return fn(Tag2<EulerModel<T, false>>{});
    case ROM_EULER_HLLC: return fn(Tag2<EulerModel<T, true>>{});
    case ROM_REACT: return fn(Tag2<ReactModel<T>>{});
  }
  set_error("unknown problem");
  return ROM_E_INVAL;
}

size_t explicit_step_shm(const rom_batch* h) {
  return sizeof(double) * ((size_t)h->cfg.n_s * 5 * h->nv + h->cfg.n_s + 3 * (size_t)h->cfg.r);
}

}  // namespace

rom_status launch_residual2(rom_batch* h, const void* q, void* out, hipStream_t s) {
  auto go = [&](auto tagT) -> rom_status {
    using T = typename decltype(tagT)::type;
    return with_model2<T>(h, [&](auto tag) -> rom_status {
      using Mdl = typename decltype(tag)::type;
      hipLaunchKernelGGL((k_residual2<Mdl, T>), dim3(h->n_tiles), dim3(kTile), 0, s, h->d_tiles,
                         h->d_dof_off, h->d_cell_off, h->d_phys, h->cfg.n_phys, (const T*)q,
                         (T*)out, h->flags);
      ROM_HIP_CHECK(hipGetLastError());
      return ROM_OK;
    });
  };
  return h->cfg.precision == ROM_F64 ? go(Tag2<double>{}) : go(Tag2<float>{});
}

// one SSPRK(4,3) step of size dt of the limited full-order model; q_prev and
// q_out may alias
rom_status fom_step_explicit(rom_batch* h, const void* q_prev, double dt, void* q_out,
                             hipStream_t s) {
  const int64_t n = h->total_dof;
  const unsigned grid = (unsigned)((n + 255) / 256);
  auto go = [&](auto tagT) -> rom_status {
    using T = typename decltype(tagT)::type;
    T* y = (T*)h->fq_prev;   // the step's start
    T* st = (T*)h->fq;       // the running stage
    T* f = (T*)h->vjp_tmp;   // L of the stage
    if ((const void*)y != q_prev)
      ROM_HIP_CHECK(hipMemcpyAsync(y, q_prev, sizeof(T) * (size_t)n, hipMemcpyDeviceToDevice, s));
    const double h2 = 0.5 * dt;
    ROM_TRY(launch_residual2(h, y, f, s));
    hipLaunchKernelGGL((k_ssp_combine<T>), dim3(grid), dim3(256), 0, s, n, (const T*)y,
                       (const T*)nullptr, (const T*)f, 1.0, 0.0, h2, st);
    ROM_TRY(launch_residual2(h, st, f, s));
    hipLaunchKernelGGL((k_ssp_combine<T>), dim3(grid), dim3(256), 0, s, n, (const T*)st,
                       (const T*)nullptr, (const T*)f, 1.0, 0.0, h2, st);
    ROM_TRY(launch_residual2(h, st, f, s));
    hipLaunchKernelGGL((k_ssp_combine<T>), dim3(grid), dim3(256), 0, s, n, (const T*)y,
                       (const T*)st, (const T*)f, 2.0 / 3.0, 1.0 / 3.0, dt / 6.0, st);
    ROM_TRY(launch_residual2(h, st, f, s));
    hipLaunchKernelGGL((k_ssp_combine<T>), dim3(grid), dim3(256), 0, s, n, (const T*)st,
                       (const T*)nullptr, (const T*)f, 1.0, 0.0, h2, (T*)q_out);
    ROM_HIP_CHECK(hipGetLastError());
    return ROM_OK;
  };
  return h->cfg.precision == ROM_F64 ? go(Tag2<double>{}) : go(Tag2<float>{});
}

rom_status launch_mesh5(rom_batch* h, hipStream_t s) {
  const int periodic = (h->cfg.problem == ROM_BURGERS || h->cfg.problem == ROM_REACT) ? 1 : 0;
  auto go = [&](auto tagT) -> rom_status {
    using T = typename decltype(tagT)::type;
    hipLaunchKernelGGL((k_mesh5<T>), dim3(h->cfg.n_inst), dim3(256), 0, s, h->cfg.r, h->cfg.n_s,
                       h->nv, periodic, h->d_dof_off, h->d_cell_off, (const T*)h->Phi,
                       (const T*)h->q_ref, h->P, h->mesh5_phi, h->mesh5_qref);
    ROM_HIP_CHECK(hipGetLastError());
    return ROM_OK;
  };
  return h->cfg.precision == ROM_F64 ? go(Tag2<double>{}) : go(Tag2<float>{});
}

rom_status launch_hr_explicit_step(rom_batch* h, hipStream_t s) {
  return with_model2<double>(h, [&](auto tag) -> rom_status {
    using Mdl = typename decltype(tag)::type;
    hipLaunchKernelGGL((k_hr_explicit_step<Mdl>), dim3(h->cfg.n_inst), dim3(256),
                       explicit_step_shm(h), s, h->cfg.r, h->cfg.n_s, h->d_cell_off, h->d_phys,
                       h->cfg.n_phys, h->d_var, h->P, h->M, h->mesh5_phi, h->mesh5_qref,
                       h->cfg.dt, h->a, h->flags);
    ROM_HIP_CHECK(hipGetLastError());
    return ROM_OK;
  });
}

rom_status explicit_kernels_prepare() {
  const int big = 160 * 1024 - 1024;
  ROM_HIP_CHECK(hipFuncSetAttribute((const void*)k_hr_explicit_step<BurgersModel<double>>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, big));
  ROM_HIP_CHECK(hipFuncSetAttribute((const void*)k_hr_explicit_step<EulerModel<double, false>>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, big));
  ROM_HIP_CHECK(hipFuncSetAttribute((const void*)k_hr_explicit_step<EulerModel<double, true>>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, big));
  ROM_HIP_CHECK(hipFuncSetAttribute((const void*)k_hr_explicit_step<ReactModel<double>>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, big));
  return ROM_OK;
}

}  // namespace romhip
