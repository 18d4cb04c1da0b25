// Reverse mode of Alg. 1's online loop (an extension; the paper has no
// adjoint): Galerkin fine steps (Burgers), adaptation events with the coarse
// backward-Euler step, the Brand update (Alg. 2) and the closed-form state
// transfer.  FP64 throughout; the basis and the states are read in the
// storage precision T.
//
//  * k_online_seed: the loss seed at the end, q~ = q_ref + D^-1 Phi a:
//    abar = Phi^T D^-1 qbar, Phibar = D^-1 qbar a^T.
//  * k_step_vjp_solve + k_step_vjp_uv: one fine step a_{n+1} = G(a_n, Phi) with
//    g(a) = a - a_n - dt Phi^T D f(q_ref + D^-1 Phi a) = 0, differentiated by
//    the implicit-function theorem at the converged a_{n+1}:
//    J_g^T lambda = abar, abar_n = lambda and
//    Phibar += dt (D f) lambda^T + dt D^-1 J_f^T (D Phi lambda) a_{n+1}^T.
//    J_g = I - dt Phi^T J_f Phi comes from the Galerkin pass's tile partials;
//    the r x r solve runs per instance; the Phibar terms are kept per row and
//    k_phibar_flush applies a window's steps in one pass over Phibar.
//  * k_ev_a, k_ev_core, k_ev_b, k_ev_c, k_ev_d: one event from the transfer back
//    to yhat = D (y - q_ref):
//    transfer a' = Ubar[:r, :r]^T a, rotation Phi' = [Phi, q / rho] Ubar[:, :r],
//    truncation sigma' = Sbar[:r], the SVD of the core K (distinct singular
//    values: Kbar = Ubar G Vbar^T with G_ii = sbar_i and
//    G_ij = s_j (M_ij - M_ji) / (s_j^2 - s_i^2), M = Ubar^T Ubarbar), the core's
//    entries lambda sigma, p = p1 + p2 and rho = |q|, and the two classical
//    Gram-Schmidt passes: four passes over the rows by pass tiles, with the
//    per-instance work between them.  The coarse step's transposed solve is
//    done by the banded solver outside.
#include "internal.h"
#include "linalg.h"
#include "physics.h"

#define DEV_HOST_INLINE __host__ __device__ inline

namespace romhip {

namespace {

constexpr int kAT = 1024;  // threads per instance (seed and step adjoints)

// Block-wide sum of one double per thread (all threads call; result in all).
DEV double block_sum(double v, double* red) {
  const int tid = threadIdx.x;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  __syncthreads();
  if ((tid & 63) == 0) red[tid >> 6] = v;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += red[w];
  __syncthreads();
  return s;
}

// Burgers on the periodic unit grid: f_i, its diagonal derivative and the two
// off-diagonal entries of column i of J_f (d f_{i+1} / d u_i, d f_{i-1} / d u_i).
DEV void burgers_col(double um, double u0, double up, double nu, double inv, double inv2,
                     double& f, double& be, double& al_next, double& ga_prev) {
  double dla, dlb, dra, drb;
  const double FL = godunov(um, u0, dla, dlb);
  const double FR = godunov(u0, up, dra, drb);
  f = -(FR - FL) * inv + nu * ((up - u0) - (u0 - um)) * inv2;
  be = (dlb - dra) * inv - 2.0 * nu * inv2;
  al_next = dra * inv + nu * inv2;    // f_{i+1} through its left face (u_i, u_{i+1})
  ga_prev = -dlb * inv + nu * inv2;   // f_{i-1} through its right face (u_{i-1}, u_i)
}

DEV int64_t wrap(int64_t c, int64_t n) { return c < 0 ? c + n : (c >= n ? c - n : c); }

constexpr int kSC = 64;   // rows of a staged chunk in the seed adjoint
constexpr int kEV = 256;  // threads of the seed's and the event adjoint's tile kernels

template <typename T>
__global__ __launch_bounds__(kAT) void k_online_seed(
    int r, const int64_t* __restrict__ dof_off, const double* __restrict__ dvar,
    const T* __restrict__ Phi, const double* __restrict__ a, const T* __restrict__ qbar,
    double* __restrict__ abar, double* __restrict__ phibar, int nv, double* __restrict__ qrbar,
    double* __restrict__ dvbar) {
  __shared__ double cP[kSC * kMaxR];
  __shared__ double cq[kSC];
  __shared__ double red[kAT / 64];
  const int b = blockIdx.x, tid = threadIdx.x;
  const int64_t base = dof_off[b], n = dof_off[b + 1] - base;
  const double* dvb = dvar + (size_t)b * nv;
  double dva[12];
  for (int v = 0; v < 12; ++v) dva[v] = 0.0;
  // (Phi^T qbar)_c: G row groups of r threads, their sums added in group order
  const int G = kAT / r, gq = tid / r, gc = tid - (tid / r) * r;
  double acc = 0.0;
  for (int64_t r0 = 0; r0 < n; r0 += kSC) {
    const int nr = (int)(n - r0 < kSC ? n - r0 : kSC);
    for (int e = tid; e < nr * r; e += kAT) cP[e] = (double)Phi[(base + r0) * r + e];
    // cq holds D^-1 qbar
    for (int k = tid; k < nr; k += kAT)
      cq[k] = (double)qbar[base + r0 + k] / dvb[(r0 + k) % nv];
    __syncthreads();
    if (gq < G)
      for (int k = gq; k < nr; k += G) acc += cP[k * r + gc] * cq[k];
    for (int e = tid; e < nr * r; e += kAT)
      phibar[(base + r0) * r + e] = cq[e / r] * a[(size_t)b * r + e % r];
    // q_ref and D terms: qrbar = qbar, dvbar[v] -= sum qbar (Phi a) / d^2
    if (qrbar)
      for (int k = tid; k < nr; k += kAT) {
        const int v = (int)((r0 + k) % nv);
        double pa = 0.0;
        for (int c = 0; c < r; ++c) pa += cP[k * r + c] * a[(size_t)b * r + c];
        qrbar[base + r0 + k] = (double)qbar[base + r0 + k];
        for (int u = 0; u < 12; ++u)
          if (u == v) dva[u] -= cq[k] * pa / dvb[v];
      }
    __syncthreads();
  }
  if (gq < G) cP[gq * r + gc] = acc;
  __syncthreads();
  if (tid < r) {
    double s = 0.0;
    for (int g = 0; g < G; ++g) s += cP[g * r + tid];
    abar[(size_t)b * r + tid] = s;
  }
  if (qrbar) {
    for (int v = 0; v < nv; ++v) {
      const double sv_ = block_sum(dva[v], red);
      if (tid == 0) dvbar[(size_t)b * nv + v] = sv_;
    }
  }
}

// The seed without the q_ref and D terms, by pass tiles: Phibar = D^-1 qbar a^T
// for the tile's rows and the tile's partial of Phi^T D^-1 qbar (G = kEV / r
// row groups of r threads, thread (g, c) always on column c, so the loads and
// stores of consecutive threads are consecutive elements); k_seed_abar adds
// the partials of an instance's tiles in tile order.
template <typename T>
__global__ __launch_bounds__(kEV) void k_seed_tile(
    const Tile* __restrict__ tiles, int r, const int64_t* __restrict__ dof_off,
    const double* __restrict__ dvar, int nv, const T* __restrict__ Phi,
    const double* __restrict__ a, const T* __restrict__ qbar, double* __restrict__ phibar,
    double* __restrict__ part) {
  __shared__ double sa[kMaxR], red[kEV];
  const Tile t = tiles[blockIdx.x];
  const int b = t.inst, tid = threadIdx.x;
  const int G = kEV / r, gc = tid % r;
  const bool on = tid < G * r;
  for (int c = tid; c < r; c += kEV) sa[c] = a[(size_t)b * r + c];
  __syncthreads();
  const int64_t g0 = dof_off[b] + t.cell0;
  const double* dvb = dvar + (size_t)b * nv;
  if (r % 2 == 0 && kEV % (r / 2) == 0) {
    // column pairs: thread (g, c) always on columns 2c, 2c + 1 of every row of
    // group g; the pair sums are added over the groups in order as above
    const int hr = r / 2, G2 = kEV / hr, c2 = tid % hr;
    const int64_t ne2 = t.ncell * hr;
    double ax = 0.0, ay = 0.0;
    double2* pb = reinterpret_cast<double2*>(phibar + g0 * r);
#pragma unroll 4
    for (int64_t e = tid; e < ne2; e += kEV) {
      const int64_t k = e / hr;
      const double cq = (double)qbar[g0 + k] / dvb[(t.cell0 + k) % nv];
      const T* pp = Phi + g0 * r + 2 * e;
      ax += (double)pp[0] * cq;
      ay += (double)pp[1] * cq;
      pb[e] = make_double2(cq * sa[2 * c2], cq * sa[2 * c2 + 1]);
    }
    red[tid] = ax;
    __syncthreads();
    double sx = 0.0;
    if (tid < hr)
      for (int g = 0; g < G2; ++g) sx += red[g * hr + tid];
    __syncthreads();
    red[tid] = ay;
    __syncthreads();
    if (tid < hr) {
      double sy = 0.0;
      for (int g = 0; g < G2; ++g) sy += red[g * hr + tid];
      part[(size_t)blockIdx.x * r + 2 * tid] = sx;
      part[(size_t)blockIdx.x * r + 2 * tid + 1] = sy;
    }
    return;
  }
  const int64_t ne = t.ncell * r, step = (int64_t)G * r;
  double acc = 0.0;
  if (on) {
#pragma unroll 4
    for (int64_t e = tid; e < ne; e += step) {
      const int64_t k = e / r;
      const double cq = (double)qbar[g0 + k] / dvb[(t.cell0 + k) % nv];
      acc += (double)Phi[g0 * r + e] * cq;
      phibar[g0 * r + e] = cq * sa[gc];
    }
  }
  red[tid] = acc;
  __syncthreads();
  if (tid < r) {
    double sum = 0.0;
    for (int g = 0; g < G; ++g) sum += red[g * r + tid];
    part[(size_t)blockIdx.x * r + tid] = sum;
  }
}

__global__ void k_seed_abar(int r, const int* __restrict__ tfirst, const double* __restrict__ part,
                            double* __restrict__ abar) {
  const int b = blockIdx.x;
  for (int c = threadIdx.x; c < r; c += blockDim.x) {
    double sum = 0.0;
    for (int tt = tfirst[b]; tt < tfirst[b + 1]; ++tt) sum += part[(size_t)tt * r + c];
    abar[(size_t)b * r + c] = sum;
  }
}

// One fine step backward, in two launches.  k_step_vjp_solve (a workgroup per
// instance): lambda = J_g^-T abar with J_g = I - dt M, M = Phi^T J_f Phi at a1
// (= a_{n+1}) summed from the Galerkin pass's tile partials in tile order;
// abar is replaced by lambda.  Then k_step_vjp_uv keeps the step's Phibar
// terms (below).
template <typename T>
__global__ __launch_bounds__(kAT) void k_step_vjp_solve(int r, double dt,
                                                        const int* __restrict__ tfirst,
                                                        const T* __restrict__ mpart, int pos32,
                                                        double* __restrict__ abar,
                                                        uint32_t* flags) {
  __shared__ double A[kMaxR * (kMaxR + 1)];
  __shared__ double lam[kMaxR];
  const int b = blockIdx.x, tid = threadIdx.x;
  const int ld = r + 1;
  const int t0 = tfirst[b], t1 = tfirst[b + 1];
  for (int e = tid; e < r * r; e += kAT) {
    const int i = e / r, j = e % r;
    const int pe = pos32 ? mpart_pos32(i, j) : e;   // the partials' order (see mpart)
    double s = 0.0;
    for (int tt = t0; tt < t1; tt += 8) {   // eight tiles' loads in flight, summed in order
      T v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u)
        v[u] = tt + u < t1 ? mpart[(size_t)(tt + u) * kMaxR * kMaxR + pe] : T(0);
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (tt + u < t1) s += (double)v[u];
    }
    A[j * ld + i] = (i == j ? 1.0 : 0.0) - dt * s;
  }
  for (int c = tid; c < r; c += kAT) lam[c] = abar[(size_t)b * r + c];
  __syncthreads();
  const int ok = block_lu_solve(A, ld, lam, r);
  if (!ok && tid == 0) atomicOr(&flags[b], ROM_FLAG_SINGULAR);
  for (int c = tid; c < r; c += kAT) abar[(size_t)b * r + c] = lam[c];
}

constexpr int kRT = 256;   // threads of k_step_vjp_uv and k_phibar_flush
constexpr int kSL = 8;     // lanes per row (each holds kSL-strided columns)

// k_step_vjp_uv (a workgroup per pass tile): the step's Phibar terms
//   Phibar += dt d f lambda^T + dt (J_f^T Phi lambda) a1^T
// kept as two numbers per row, uv[i] = (dt d f_i, dt v_i) with v = J_f^T w,
// w = Phi lambda, and q~ = q_ref + D^-1 Phi a1 of the rows and their two
// neighbours in LDS (the neighbours are recomputed by each tile);
// k_phibar_flush applies the terms of several steps in one pass over Phibar.
template <typename T>
__global__ __launch_bounds__(kRT) void k_step_vjp_uv(
    const Tile* __restrict__ tiles, int r, double dt, const int64_t* __restrict__ dof_off,
    const double* __restrict__ phys, int nphys, const double* __restrict__ dvar,
    const T* __restrict__ Phi, const T* __restrict__ qref, const double* __restrict__ a1,
    const double* __restrict__ lambda, double2* __restrict__ uv) {
  __shared__ double sq[kPassRows + 2], sw[kPassRows + 2];
  __shared__ double lam[kMaxR], sa[kMaxR];
  const Tile t = tiles[blockIdx.x];
  const int b = t.inst, tid = threadIdx.x;
  const int64_t base = dof_off[b], n = dof_off[b + 1] - base;
  const int nt = (int)t.ncell;
  const double d = dvar[b], dinv = 1.0 / d;
  const double nu = phys[(size_t)b * nphys];
  const double inv = (double)n, inv2 = (double)n * (double)n;
  for (int c = tid; c < r; c += kRT) {
    lam[c] = lambda[(size_t)b * r + c];
    sa[c] = a1[(size_t)b * r + c];
  }
  __syncthreads();
  if (sizeof(T) == 4 && r == 32) {
    // FP32 basis, r = 32: four lanes per row, eight columns (two float4) each
    const int q = tid & 3;
#pragma unroll 2
    for (int rr = tid >> 2; rr < nt + 2; rr += kRT / 4) {
      const int64_t i = wrap(t.cell0 - 1 + rr, n);
      const float4* pr = reinterpret_cast<const float4*>(Phi + (base + i) * 32 + 8 * q);
      const float4 u0 = pr[0], u1 = pr[1];
      const float pv[8] = {u0.x, u0.y, u0.z, u0.w, u1.x, u1.y, u1.z, u1.w};
      double sqv = 0.0, swv = 0.0;
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        sqv += (double)pv[c] * sa[8 * q + c];
        swv += (double)pv[c] * lam[8 * q + c];
      }
      sqv += __shfl_xor(sqv, 1);
      swv += __shfl_xor(swv, 1);
      sqv += __shfl_xor(sqv, 2);
      swv += __shfl_xor(swv, 2);
      if (q == 0) {
        sq[rr] = (double)qref[base + i] + sqv * dinv;
        sw[rr] = swv;
      }
    }
  } else {
    const int sub = tid % kSL;
    for (int rr = tid / kSL; rr < nt + 2; rr += kRT / kSL) {
      const int64_t i = wrap(t.cell0 - 1 + rr, n);
      const T* pr = Phi + (base + i) * r;
      double sqv = 0.0, swv = 0.0;
      for (int c = sub; c < r; c += kSL) {
        const double p = (double)pr[c];
        sqv += p * sa[c];
        swv += p * lam[c];
      }
#pragma unroll
      for (int off = kSL / 2; off > 0; off >>= 1) {
        sqv += __shfl_xor(sqv, off);
        swv += __shfl_xor(swv, off);
      }
      if (sub == 0) {
        sq[rr] = (double)qref[base + i] + sqv * dinv;
        sw[rr] = swv;
      }
    }
  }
  __syncthreads();
  for (int rr = tid; rr < nt; rr += kRT) {
    double f, be, al_next, ga_prev;
    burgers_col(sq[rr], sq[rr + 1], sq[rr + 2], nu, inv, inv2, f, be, al_next, ga_prev);
    const double v = al_next * sw[rr + 2] + be * sw[rr + 1] + ga_prev * sw[rr];
    uv[base + t.cell0 + rr] = make_double2(dt * d * f, dt * v);
  }
}

// Phibar[i, :] += uv_k[i].x lambda_k + uv_k[i].y a1_k for the pending steps k =
// 0 .. K-1 in order (the order in which the steps' adjoints ran): one pass
// over Phibar for all of them.  uv: K slots of total_dof double2; lam, a1: K
// slots of n_inst * r doubles.
__global__ __launch_bounds__(kRT) void k_phibar_flush(
    const Tile* __restrict__ tiles, int r, const int64_t* __restrict__ dof_off, int K,
    int64_t total, const double2* __restrict__ uv, const double* __restrict__ lam,
    const double* __restrict__ a1, int64_t n_inst, double* __restrict__ phibar) {
  constexpr int KM = kPhibarPending;
  __shared__ double sl[KM][kMaxR], sa[KM][kMaxR];
  const Tile t = tiles[blockIdx.x];
  const int b = t.inst, tid = threadIdx.x;
  for (int e = tid; e < K * r; e += kRT) {
    const int k = e / r, c = e - k * r;
    sl[k][c] = lam[((size_t)k * n_inst + b) * r + c];
    sa[k][c] = a1[((size_t)k * n_inst + b) * r + c];
  }
  __syncthreads();
  const int64_t g0 = dof_off[b] + t.cell0;
  if (r % 8 == 0) {
    // four threads per row, r / 4 contiguous columns each (double2 accesses);
    // a row's K uv pairs are loaded once per thread
    const int q = tid & 3, w4 = r / 4;
    for (int64_t i = tid >> 2; i < t.ncell; i += kRT / 4) {
      double2 wk[KM];
#pragma unroll
      for (int k = 0; k < KM; ++k)
        wk[k] = k < K ? uv[(size_t)k * total + g0 + i] : make_double2(0.0, 0.0);
      double2* pb = reinterpret_cast<double2*>(phibar + (g0 + i) * r + q * w4);
      for (int m = 0; m < w4 / 2; ++m) {
        double2 p = pb[m];
        const int c = q * w4 + 2 * m;
#pragma unroll
        for (int k = 0; k < KM; ++k) {
          if (k < K) {
            p.x += wk[k].x * sl[k][c] + wk[k].y * sa[k][c];
            p.y += wk[k].x * sl[k][c + 1] + wk[k].y * sa[k][c + 1];
          }
        }
        pb[m] = p;
      }
    }
    return;
  }
  const int64_t ne = t.ncell * r;
  for (int64_t e = tid; e < ne; e += kRT) {
    const int64_t i = e / r;
    const int c = (int)(e - i * r);
    double p = phibar[g0 * r + e];
    for (int k = 0; k < K; ++k) {
      const double2 w = uv[(size_t)k * total + g0 + i];
      p += w.x * sl[k][c] + w.y * sa[k][c];
    }
    phibar[g0 * r + e] = p;
  }
}

// ---- one event backward over pass tiles.  The passes over the rows of an
// instance (A: the transfer and rotation adjoints and the Ubar partials; B:
// Phi^T qbar; C: the second Gram-Schmidt pass; D: the first pass and yhat) run
// one block per pass tile and write per-tile partial sums; between them a
// block per instance sums the partials in tile order and does the small work
// (the core SVD's adjoint, pbar, p2bar, p1bar).  Rows are staged through LDS in
// chunks of rows padded to r + 1 (as many as the LDS budget kEVLds holds).
constexpr int kEC = 32;    // rows of a staged chunk, at least
constexpr int kETI = 4, kETJ = 4;   // register tile of the Ubar partials
constexpr int kEVLds = 4352;    // doubles of LDS for the staged chunks (34 KB)

// rows of a staged chunk: as many as kEVLds holds (two row arrays padded to
// r + 1 and three per-row scalars), at most one per thread
DEV_HOST_INLINE int ev_chunk(int r) {
  int c = kEVLds / (2 * (r + 1) + 3);
  c = c > kEV ? kEV : c;
  return c < kEC ? kEC : c;
}

// per-instance vector between the passes: pbar[0..r), rhobar, p2bar[0..r), p1bar[0..r)
DEV_HOST_INLINE int evs_ld(int r) { return 3 * r + 2; }
// partial sums per pass tile
DEV_HOST_INLINE int evp_ld(int r) { return (r + 1) * r + 1 > 12 ? (r + 1) * r + 1 : 12; }
DEV_HOST_INLINE int ev_ntl(int r) {
  return ((r + 1 + kETI - 1) / kETI) * ((r + kETJ - 1) / kETJ);
}

// Stage nr rows of Phi (and of phibar) into LDS: each thread issues a batch of
// eight loads before it writes any of them, so loads overlap.
template <typename T>
DEV void ev_stage(const T* __restrict__ Phi, const double* __restrict__ pb, int64_t g0, int nr,
                  int r, double* cP, double* cB) {
  constexpr int NB = 8;
  const int LDR = r + 1, ne = nr * r, tid = threadIdx.x;
  for (int e0 = 0; e0 < ne; e0 += NB * kEV) {
    double vp[NB], vb[NB];
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      const int e = e0 + u * kEV + tid;
      if (e < ne) {
        vp[u] = (double)Phi[g0 * r + e];
        if (cB) vb[u] = pb[g0 * r + e];
      }
    }
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      const int e = e0 + u * kEV + tid;
      if (e < ne) {
        const int k = e / r, c = e - k * r;
        cP[k * LDR + c] = vp[u];
        if (cB) cB[k * LDR + c] = vb[u];
      }
    }
  }
}

// column sums over the chunk rows by G = kEV / r row groups of r threads;
// acc holds the thread's running sum
DEV void ev_colsum(const double* cP, const double* w, int nr, int r, double& acc) {
  const int G = kEV / r, tid = threadIdx.x;
  const int gq = tid / r, gc = tid - (tid / r) * r;
  if (gq < G)
    for (int k = gq; k < nr; k += G) acc += cP[k * (r + 1) + gc] * w[k];
}

// the groups' sums, added in group order, into out[0..r)
DEV void ev_colsum_out(double acc, int r, double* scratch, double* out) {
  const int G = kEV / r, tid = threadIdx.x;
  const int gq = tid / r, gc = tid - (tid / r) * r;
  __syncthreads();
  if (gq < G) scratch[gq * r + gc] = acc;
  __syncthreads();
  if (tid < r) {
    double s = 0.0;
    for (int g = 0; g < G; ++g) s += scratch[g * r + tid];
    out[tid] = s;
  }
}

// Pass A: q = yhat - Phi (p1 + p2) (into qs); the rows of Phibar_old =
// Phibar' U[:r, :r]^T and jbar = Phibar' U[r, :r]^T (into js); partials of
// Ubar[:r, :r] += Phi^T Phibar', Ubar[r, :r] += (q / rho)^T Phibar' and of
// jq = jbar . q.  Dynamic LDS: n^2 + max(CH (2 (r + 1) + 1), 16 max(kEV, NTL)).
template <typename T>
__global__ __launch_bounds__(kEV) void k_ev_a(
    const Tile* __restrict__ tiles, const int64_t* __restrict__ dof_off, int r, int nv,
    const double* __restrict__ dvar, const T* __restrict__ Phi, const T* __restrict__ ynew,
    const T* __restrict__ qref, const double* __restrict__ ubar, const double* __restrict__ prs,
    double* __restrict__ phibar, double* __restrict__ qs, double* __restrict__ js,
    double* __restrict__ part) {
  extern __shared__ double sm[];
  __shared__ double red[kEV / 64];
  __shared__ double sp[kMaxR];
  const int n = r + 1, LDR = r + 1, tid = threadIdx.x;
  const Tile t = tiles[blockIdx.x];
  const int b = t.inst;
  const double* pr = prs + (size_t)b * (2 * r + 2);
  const double irho = pr[2 * r];
  if (irho == 0.0) return;   // rho = 0: the instance is flagged and skipped
  const int CH = ev_chunk(r);
  double* U = sm;
  double* cP = U + n * n;
  double* cB = cP + CH * LDR;
  double* c0 = cB + CH * LDR;
  double* tp = cP;           // the threads' Ubar tile sums, after the last chunk
  for (int e = tid; e < n * n; e += kEV) U[e] = ubar[(size_t)b * n * n + e];
  for (int c = tid; c < r; c += kEV) sp[c] = pr[c] + pr[r + c];
  const int64_t base = dof_off[b];
  const double* dvb = dvar + (size_t)b * nv;
  const int NJ = (r + kETJ - 1) / kETJ, NTL = ev_ntl(r);
  const int nslot = (NTL + kEV - 1) / kEV;            // 1, or 2 for the widest bases
  const int KS = nslot == 1 ? kEV / NTL : 1;          // row groups per tile
  const int ks = nslot == 1 ? tid / NTL : 0;
  const bool tl_on = nslot == 1 ? tid < KS * NTL : true;
  double ta[2][kETI][kETJ];
#pragma unroll
  for (int m = 0; m < 2; ++m)
#pragma unroll
    for (int a = 0; a < kETI; ++a)
#pragma unroll
      for (int c = 0; c < kETJ; ++c) ta[m][a][c] = 0.0;
  double jq = 0.0;
  for (int64_t r0 = 0; r0 < t.ncell; r0 += CH) {
    const int nr = (int)(t.ncell - r0 < CH ? t.ncell - r0 : CH);
    const int64_t g0 = base + t.cell0 + r0;
    __syncthreads();
    ev_stage(Phi, phibar, g0, nr, r, cP, cB);
    __syncthreads();
    for (int k = tid; k < nr; k += kEV) {
      const int64_t g = g0 + k;
      double q = dvb[(t.cell0 + r0 + k) % nv] * ((double)ynew[g] - (double)qref[g]);
      for (int c = 0; c < r; ++c) q -= cP[k * LDR + c] * sp[c];
      c0[k] = q;
      qs[g] = q;
    }
    __syncthreads();
    if (tl_on) {
#pragma unroll
      for (int m = 0; m < 2; ++m) {
        if (m >= nslot) continue;
        const int tt = nslot == 1 ? tid - ks * NTL : tid + m * kEV;
        if (tt >= NTL) continue;
        const int i0 = (tt / NJ) * kETI, j0 = (tt - (tt / NJ) * NJ) * kETJ;
        for (int k = ks; k < nr; k += KS) {
          double av[kETI], bv[kETJ];
#pragma unroll
          for (int a = 0; a < kETI; ++a) {
            const int i = i0 + a;
            av[a] = i < r ? cP[k * LDR + i] : (i == r ? c0[k] * irho : 0.0);
          }
#pragma unroll
          for (int c = 0; c < kETJ; ++c) bv[c] = j0 + c < r ? cB[k * LDR + j0 + c] : 0.0;
#pragma unroll
          for (int a = 0; a < kETI; ++a)
#pragma unroll
            for (int c = 0; c < kETJ; ++c) ta[m][a][c] += av[a] * bv[c];
        }
      }
    }
    // rows of Phibar_old and jbar in 4 x 3 register tiles (each output summed
    // over m in order by one thread)
    {
      constexpr int TR = 4, TC = 3;
      const int NR = (nr + TR - 1) / TR, NC = (n + TC - 1) / TC;
      for (int e = tid; e < NR * NC; e += kEV) {
        const int k0 = (e / NC) * TR, ct = (e - (e / NC) * NC) * TC;
        double o[TR][TC];
#pragma unroll
        for (int a = 0; a < TR; ++a)
#pragma unroll
          for (int c = 0; c < TC; ++c) o[a][c] = 0.0;
        for (int m = 0; m < r; ++m) {
          double bv[TR], uv[TC];
#pragma unroll
          for (int a = 0; a < TR; ++a) bv[a] = k0 + a < nr ? cB[(k0 + a) * LDR + m] : 0.0;
#pragma unroll
          for (int c = 0; c < TC; ++c) uv[c] = ct + c < n ? U[(ct + c) * n + m] : 0.0;
#pragma unroll
          for (int a = 0; a < TR; ++a)
#pragma unroll
            for (int c = 0; c < TC; ++c) o[a][c] += bv[a] * uv[c];
        }
#pragma unroll
        for (int a = 0; a < TR; ++a) {
          const int k = k0 + a;
          if (k >= nr) continue;
#pragma unroll
          for (int c = 0; c < TC; ++c) {
            const int cc = ct + c;
            if (cc < r) phibar[(g0 + k) * r + cc] = o[a][c];
            else if (cc == r) {
              js[g0 + k] = o[a][c];
              jq += o[a][c] * c0[k];
            }
          }
        }
      }
    }
  }
  __syncthreads();
  // the tile's partials: Ubar entries summed over the row groups in order, then jq
  if (tl_on) {
#pragma unroll
    for (int m = 0; m < 2; ++m) {
      if (m >= nslot) continue;
      const int tt = nslot == 1 ? tid - ks * NTL : tid + m * kEV;
      if (tt >= NTL) continue;
      const int slot = nslot == 1 ? ks * NTL + tt : tt;
#pragma unroll
      for (int a = 0; a < kETI; ++a)
#pragma unroll
        for (int c = 0; c < kETJ; ++c) tp[(size_t)slot * (kETI * kETJ) + a * kETJ + c] = ta[m][a][c];
    }
  }
  __syncthreads();
  double* out = part + (size_t)blockIdx.x * evp_ld(r);
  for (int e = tid; e < n * r; e += kEV) {
    const int i = e / r, j = e % r;
    const int t2 = (i / kETI) * NJ + j / kETJ, w = (i % kETI) * kETJ + j % kETJ;
    double s = 0.0;
    for (int g = 0; g < KS; ++g) s += tp[((size_t)g * NTL + t2) * (kETI * kETJ) + w];
    out[e] = s;
  }
  jq = block_sum(jq, red);
  if (tid == 0) out[n * r] = jq;
}

// Pass A for r = 32 on the FP64 matrix cores (v_mfma_f64_16x16x4f64; lane l
// supplies A[l % 16][l / 16] and B[l / 16][l % 16], accumulator element v is
// D[4 v + l / 16][l % 16], checked on the device).  The same quantities as k_ev_a, by one wave per
// 16-row block of the tile (blocks w, w + 4, ... for wave w), staged through
// the wave's own LDS slice:
//   * q = D (yhat - q_ref) - Phi sp and jbar = Phibar' U[r, :r]^T, four lanes
//     per row with a quad reduction, into qs and js, and jq += jbar q;
//   * Ubar[:r, :r] partials Phi^T Phibar' as 2 x 2 accumulator tiles over the
//     wave's rows (four rows per product), Ubar[r, :r] += (q / rho)^T Phibar'
//     by lane sums;
//   * Phibar_old = Phibar' U[:r, :r]^T as two 16 x 16 tiles per block (eight
//     products over m), written over the block's rows of phibar.
// The four waves' partials are added in wave order; no block barrier inside
// the row loop.  Phibar' is first completed by the K pending fine-step terms
// (those k_phibar_flush would add; K = 0: none).
typedef double d4_t __attribute__((ext_vector_type(4)));
constexpr int kEA = 32;        // r of the matrix-core pass A
constexpr int kEAL = kEA + 1;  // padded row of the staged blocks (doubles)

DEV void ev_wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <typename T>
__global__ __launch_bounds__(kEV) __attribute__((amdgpu_waves_per_eu(3))) void k_ev_a_mfma(
    const Tile* __restrict__ tiles, const int64_t* __restrict__ dof_off, int nv,
    const double* __restrict__ dvar, const T* __restrict__ Phi, const T* __restrict__ ynew,
    const T* __restrict__ qref, const double* __restrict__ ubar, const double* __restrict__ prs,
    double* __restrict__ phibar, double* __restrict__ qs, double* __restrict__ js,
    double* __restrict__ part, int K, int64_t total, const double2* __restrict__ puv,
    const double* __restrict__ plam, const double* __restrict__ pa1, int n_inst) {
  constexpr int r = kEA, n = kEA + 1, NW = kEV / 64;
  __shared__ double pl[kPhibarPending][kEA], pa[kPhibarPending][kEA];
  __shared__ double2 wU[kEV / 64][kPhibarPending][16];   // the block rows' pending uv
  __shared__ double U[n * n];                    // U[c][m], row c of Ubar
  __shared__ double sp[r];
  __shared__ double wB[NW][16 * kEAL];           // the wave's Phibar' rows
  __shared__ double wP[NW][16 * kEAL];           // the wave's Phi rows (FP64)
  __shared__ double wq[NW][16];                  // q of those rows
  __shared__ double red[kEV / 64];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const Tile t = tiles[blockIdx.x];
  const int b = t.inst;
  const double* pr = prs + (size_t)b * (2 * r + 2);
  const double irho = pr[2 * r];
  for (int e = tid; e < K * r; e += kEV) {
    const int k = e / r, c = e - k * r;
    pl[k][c] = plam[((size_t)k * n_inst + b) * r + c];
    pa[k][c] = pa1[((size_t)k * n_inst + b) * r + c];
  }
  const int64_t base = dof_off[b] + t.cell0;
  if (irho == 0.0) {   // rho = 0: flagged and skipped; the pending terms still land
    __syncthreads();
    for (int64_t e = tid; e < t.ncell * r; e += kEV) {
      const int64_t k = e / r;
      const int c = (int)(e - k * r);
      double p = phibar[base * r + e];
      for (int kk = 0; kk < K; ++kk) {
        const double2 w = puv[(size_t)kk * total + base + k];
        p += w.x * pl[kk][c] + w.y * pa[kk][c];
      }
      phibar[base * r + e] = p;
    }
    return;
  }
  for (int e = tid; e < n * n; e += kEV) U[e] = ubar[(size_t)b * n * n + e];
  for (int c = tid; c < r; c += kEV) sp[c] = pr[c] + pr[r + c];
  __syncthreads();
  const double* dvb = dvar + (size_t)b * nv;
  double* cB = wB[wave];
  double* cP = wP[wave];
  double* cq = wq[wave];
  const int l16 = lane & 15, lk = lane >> 4;     // MFMA row / column and k slot
  const int qr = lane >> 2, qc = lane & 3;       // row and quarter of the row sums
  d4_t acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int c = 0; c < 2; ++c) acc[a][c] = d4_t{0.0, 0.0, 0.0, 0.0};
  double ub = 0.0;   // Ubar[r][lane & 31] over the rows of half lane >> 5
  double jq = 0.0;
  const int nblk = (int)((t.ncell + 15) / 16);
  for (int kb = wave; kb < nblk; kb += NW) {
    const int64_t r0 = (int64_t)kb * 16;
    const int nr = (int)(t.ncell - r0 < 16 ? t.ncell - r0 : 16);
    const int64_t g0 = base + r0;
    // stage 16 rows: eight elements of each array per lane, loads first (all
    // sixteen issued together: rows past the tile read its last row, then are
    // zeroed; a load under a condition would be waited for on its own)
    {
      double vb[8], vp[8];
      const int emax = nr * r - 1;
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = lane + 64 * u, ec = e < emax ? e : emax;
        vb[u] = phibar[g0 * r + ec];
        vp[u] = (double)Phi[g0 * r + ec];
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = lane + 64 * u;
        if ((e >> 5) >= nr) vb[u] = vp[u] = 0.0;
      }
      // the fine steps' pending Phibar terms, in the order k_phibar_flush adds
      // them; their uv values of the block's rows go through LDS first
      if (K > 0) {
        for (int idx = lane; idx < K * 16; idx += 64) {
          const int kk = idx >> 4, k = idx & 15;
          wU[wave][kk][k] = k < nr ? puv[(size_t)kk * total + g0 + k] : make_double2(0.0, 0.0);
        }
        ev_wave_sync();
        for (int kk = 0; kk < K; ++kk) {
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            const int e = lane + 64 * u, k = e >> 5, c = e & 31;
            const double2 w = wU[wave][kk][k];
            vb[u] += w.x * pl[kk][c] + w.y * pa[kk][c];
          }
        }
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = lane + 64 * u, k = e >> 5, c = e & 31;
        cB[k * kEAL + c] = vb[u];
        cP[k * kEAL + c] = vp[u];
      }
    }
    ev_wave_sync();
    // q and jbar of row qr: lanes 4 qr .. 4 qr + 3 take eight columns each
    {
      double sq = 0.0, sj = 0.0;
#pragma unroll
      for (int c = 8 * qc; c < 8 * qc + 8; ++c) {
        sq += cP[qr * kEAL + c] * sp[c];
        sj += cB[qr * kEAL + c] * U[r * n + c];
      }
      sq += __shfl_xor(sq, 1);
      sq += __shfl_xor(sq, 2);
      sj += __shfl_xor(sj, 1);
      sj += __shfl_xor(sj, 2);
      if (qc == 0) {
        double q = 0.0;
        if (qr < nr) {
          const int64_t g = g0 + qr;
          q = dvb[(t.cell0 + r0 + qr) % nv] * ((double)ynew[g] - (double)qref[g]) - sq;
          qs[g] = q;
          js[g] = sj;
          jq += sj * q;
        }
        cq[qr] = q;
      }
    }
    ev_wave_sync();
    // Ubar partials: four rows per product, 2 x 2 tiles
#pragma unroll
    for (int st = 0; st < 4; ++st) {
      const int k = 4 * st + lk;
      const double a0 = cP[k * kEAL + l16], a1 = cP[k * kEAL + 16 + l16];
      const double b0 = cB[k * kEAL + l16], b1 = cB[k * kEAL + 16 + l16];
      acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
    }
    // Ubar[r, :] += (q / rho)^T Phibar': column lane & 31, rows of half lane >> 5
    {
      const int c = lane & 31, h = lane >> 5;
#pragma unroll
      for (int k = 8 * h; k < 8 * h + 8; ++k) ub += (cq[k] * irho) * cB[k * kEAL + c];
    }
    // Phibar_old rows of the block: D[k][c] = sum_m Phibar'[k][m] U[c][m]
    {
      d4_t o0 = d4_t{0.0, 0.0, 0.0, 0.0}, o1 = d4_t{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int sm = 0; sm < 8; ++sm) {
        const int m = 4 * sm + lk;
        const double av = cB[l16 * kEAL + m];
        o0 = __builtin_amdgcn_mfma_f64_16x16x4f64(av, U[l16 * n + m], o0, 0, 0, 0);
        o1 = __builtin_amdgcn_mfma_f64_16x16x4f64(av, U[(16 + l16) * n + m], o1, 0, 0, 0);
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int k = 4 * v + lk;
        if (k < nr) {
          phibar[(g0 + k) * r + l16] = o0[v];
          phibar[(g0 + k) * r + 16 + l16] = o1[v];
        }
      }
    }
    ev_wave_sync();   // the block's rows are read before the next staging
  }
  // the tile's partials: the waves' sums added in wave order into wB[0]
  double* sum = &wB[0][0];   // 33 x 32 doubles (fits the 4 x 16 x 33 staging area)
  __syncthreads();
  for (int w = 0; w < NW; ++w) {
    if (wave == w) {
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int c = 0; c < 2; ++c)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int i = 16 * a + 4 * v + lk, j = 16 * c + l16;
            sum[i * r + j] = (w == 0 ? 0.0 : sum[i * r + j]) + acc[a][c][v];
          }
      // row r: the two halves of the wave (lanes c and c + 32), in half order
      const double uh = __shfl_xor(ub, 32);
      if (lane < 32) sum[r * r + lane] = (w == 0 ? 0.0 : sum[r * r + lane]) + (ub + uh);
    }
    __syncthreads();
  }
  double* out = part + (size_t)blockIdx.x * evp_ld(r);
  for (int e = tid; e < n * r; e += kEV) out[e] = sum[e];
  jq = block_sum(jq, red);
  if (tid == 0) out[n * r] = jq;
}

// After pass A, one block per instance: the transfer adjoint (abar <- U[:r, :r]
// abar, Ubar[:r, :r] += a_old abar^T), the tiles' Ubar partials in tile order,
// then the adjoint of the core SVD and of K's entries: sigbar, pbar, rhobar.
// Dynamic LDS: 4 n^2 + n doubles.
__global__ __launch_bounds__(kEV) void k_ev_core(
    int r, double lam_f, const int* __restrict__ tfirst, const double* __restrict__ part,
    const double* __restrict__ sig_old, const double* __restrict__ a_old,
    const double* __restrict__ ubar, const double* __restrict__ prs,
    const double* __restrict__ sig_new, double* __restrict__ abar,
    double* __restrict__ sigbar, double* __restrict__ evs, uint32_t* flags) {
  extern __shared__ double sm[];
  __shared__ double sv[kMaxR + 1], ab[kMaxR], p1[kMaxR], p2[kMaxR], wr[kMaxR + 1],
      pb[kMaxR + 1];
  __shared__ double jqs;
  const int n = r + 1, tid = threadIdx.x, b = blockIdx.x;
  const double* pr = prs + (size_t)b * (2 * r + 2);
  const double irho = pr[2 * r];
  if (irho == 0.0) {
    if (tid == 0) atomicOr(&flags[b], ROM_FLAG_SINGULAR);
    return;
  }
  const double rho = 1.0 / irho;
  double* U = sm;
  double* Ub = U + n * n;
  double* X = Ub + n * n;
  double* GVt = X + n * n;
  for (int e = tid; e < n * n; e += kEV) U[e] = ubar[(size_t)b * n * n + e];
  for (int c = tid; c < r; c += kEV) {
    ab[c] = abar[(size_t)b * r + c];
    p1[c] = pr[c];
    p2[c] = pr[r + c];
    sv[c] = sig_new[(size_t)b * r + c];
  }
  if (tid == 0) sv[r] = pr[2 * r + 1];
  __syncthreads();
  for (int c = tid; c < r; c += kEV) {
    double s = 0.0;
    for (int k = 0; k < r; ++k) s += U[c * n + k] * ab[k];
    abar[(size_t)b * r + c] = s;
  }
  const int ld = evp_ld(r);
  for (int e = tid; e < n * n; e += kEV) {
    const int i = e / n, j = e % n;
    double s = (i < r && j < r) ? a_old[(size_t)b * r + i] * ab[j] : 0.0;
    if (j < r)
      for (int tt = tfirst[b]; tt < tfirst[b + 1]; ++tt) s += part[(size_t)tt * ld + i * r + j];
    Ub[e] = s;
  }
  if (tid == 0) {
    double s = 0.0;
    for (int tt = tfirst[b]; tt < tfirst[b + 1]; ++tt) s += part[(size_t)tt * ld + n * r];
    jqs = s;
  }
  __syncthreads();
  // SVD of K: M = U^T Ub (in X), G (in Ub), V = K^T U / s (in X); the entries
  // of Kbar = U G V^T that K depends on: lambda sigma (diagonal), p (last column), rho
  for (int e = tid; e < n * n; e += kEV) {
    const int i = e / n, j = e % n;
    double s = 0.0;
    for (int k = 0; k < n; ++k) s += U[k * n + i] * Ub[k * n + j];
    X[e] = s;
  }
  __syncthreads();
  for (int e = tid; e < n * n; e += kEV) {
    const int i = e / n, j = e % n;
    double g;
    if (i == j) g = i < r ? sigbar[(size_t)b * r + i] : 0.0;
    else g = sv[j] > 0.0 ? sv[j] * (X[i * n + j] - X[j * n + i]) / ((sv[j] - sv[i]) * (sv[j] + sv[i]))
                         : 0.0;
    Ub[e] = g;
  }
  __syncthreads();
  for (int e = tid; e < n * n; e += kEV) {
    const int k = e / n, j = e % n;   // V[k][j]
    double v = 0.0;
    if (sv[j] > 0.0) {
      double t;
      if (k < r) {
        t = lam_f * sig_old[(size_t)b * r + k] * U[k * n + j];
      } else {
        t = rho * U[r * n + j];
        for (int i = 0; i < r; ++i) t += (p1[i] + p2[i]) * U[i * n + j];
      }
      v = t / sv[j];
    }
    X[e] = v;
  }
  __syncthreads();
  for (int k = tid; k < n; k += kEV) {   // wr = G V[r, :]^T
    double s = 0.0;
    for (int m = 0; m < n; ++m) s += Ub[k * n + m] * X[r * n + m];
    wr[k] = s;
  }
  for (int e = tid; e < n * n; e += kEV) {
    const int k = e / n, c = e - (e / n) * n;
    double gv = 0.0;
    for (int m = 0; m < n; ++m) gv += Ub[k * n + m] * X[c * n + m];
    GVt[e] = gv;
  }
  __syncthreads();
  for (int c = tid; c < n; c += kEV) {
    double kd = 0.0, kc = 0.0;
    for (int k = 0; k < n; ++k) {
      kd += U[c * n + k] * GVt[k * n + c];
      kc += U[c * n + k] * wr[k];
    }
    if (c < r) sigbar[(size_t)b * r + c] = lam_f * kd;
    pb[c] = kc;
  }
  __syncthreads();
  double* e_out = evs + (size_t)b * evs_ld(r);
  for (int c = tid; c < r; c += kEV) e_out[c] = pb[c];
  // j = q / rho, rho = |q|: qbar = (jbar + rhobar q) / rho
  if (tid == 0) e_out[r] = pb[r] - jqs * irho * irho;
}

// Pass B: partials of Phi^T qbar with qbar = (jbar + rhobar q) / rho.
template <typename T>
__global__ __launch_bounds__(kEV) void k_ev_b(const Tile* __restrict__ tiles,
                                              const int64_t* __restrict__ dof_off, int r,
                                              const T* __restrict__ Phi,
                                              const double* __restrict__ prs,
                                              const double* __restrict__ evs,
                                              const double* __restrict__ qs,
                                              const double* __restrict__ js,
                                              double* __restrict__ part) {
  extern __shared__ double sm[];
  const int LDR = r + 1, tid = threadIdx.x;
  const Tile t = tiles[blockIdx.x];
  const int b = t.inst;
  const double irho = prs[(size_t)b * (2 * r + 2) + 2 * r];
  if (irho == 0.0) return;
  const double rhob = evs[(size_t)b * evs_ld(r) + r];
  const int CH = ev_chunk(r);
  double* cP = sm;
  double* c0 = cP + CH * LDR;
  double* scr = c0 + CH;
  const int64_t base = dof_off[b];
  double acc = 0.0;
  for (int64_t r0 = 0; r0 < t.ncell; r0 += CH) {
    const int nr = (int)(t.ncell - r0 < CH ? t.ncell - r0 : CH);
    const int64_t g0 = base + t.cell0 + r0;
    __syncthreads();
    ev_stage(Phi, (const double*)nullptr, g0, nr, r, cP, nullptr);
    for (int k = tid; k < nr; k += kEV) c0[k] = (js[g0 + k] + rhob * qs[g0 + k]) * irho;
    __syncthreads();
    ev_colsum(cP, c0, nr, r, acc);
  }
  ev_colsum_out(acc, r, scr, part + (size_t)blockIdx.x * evp_ld(r));
}

// A kept Phibar term that adds nothing: zero rows of the tile and, by the
// instance's first tile, zero coefficients.
DEV void ev_pending_zero(const Tile& t, const int64_t* __restrict__ dof_off, int r,
                         double2* __restrict__ uv, double* __restrict__ ulam,
                         double* __restrict__ ua1) {
  const int64_t g0 = dof_off[t.inst] + t.cell0;
  for (int64_t k = threadIdx.x; k < t.ncell; k += blockDim.x) uv[g0 + k] = make_double2(0.0, 0.0);
  if (t.cell0 == 0)
    for (int c = threadIdx.x; c < r; c += blockDim.x) {
      ulam[(size_t)t.inst * r + c] = 0.0;
      ua1[(size_t)t.inst * r + c] = 0.0;
    }
}

// Pass C: q1 = yhat - Phi p1; q1bar = qbar + Phi p2bar (into js);
// Phibar_old += -qbar p2^T + q1 p2bar^T; partials of Phi^T q1bar.  With uv,
// the Phibar term is kept instead (uv = (-qbar, q1) per row, coefficients p2
// and p2bar) for a later pass over Phibar, and Phibar is not read.
template <typename T>
__global__ __launch_bounds__(kEV) void k_ev_c(
    const Tile* __restrict__ tiles, const int64_t* __restrict__ dof_off, int r, int nv,
    const double* __restrict__ dvar, const T* __restrict__ Phi, const T* __restrict__ ynew,
    const T* __restrict__ qref, const double* __restrict__ prs, const double* __restrict__ evs,
    const double* __restrict__ qs, double* __restrict__ js, double* __restrict__ phibar,
    double* __restrict__ part, double2* __restrict__ uv, double* __restrict__ ulam,
    double* __restrict__ ua1) {
  extern __shared__ double sm[];
  __shared__ double p1[kMaxR], p2[kMaxR], p2b[kMaxR];
  const int LDR = r + 1, tid = threadIdx.x;
  const Tile t = tiles[blockIdx.x];
  const int b = t.inst;
  const double* pr = prs + (size_t)b * (2 * r + 2);
  const double irho = pr[2 * r];
  if (irho == 0.0) {   // rho = 0: flagged and skipped; a kept term adds nothing
    if (uv) ev_pending_zero(t, dof_off, r, uv, ulam, ua1);
    return;
  }
  const double* e_in = evs + (size_t)b * evs_ld(r);
  const double rhob = e_in[r];
  for (int c = tid; c < r; c += kEV) {
    p1[c] = pr[c];
    p2[c] = pr[r + c];
    p2b[c] = e_in[r + 1 + c];
    if (uv && t.cell0 == 0) {   // the term's coefficients, by the instance's first tile
      ulam[(size_t)b * r + c] = pr[r + c];
      ua1[(size_t)b * r + c] = e_in[r + 1 + c];
    }
  }
  const int CH = ev_chunk(r);
  double* cP = sm;
  double* cB = cP + CH * LDR;
  double* c0 = cB + CH * LDR;
  double* c1 = c0 + CH;
  double* c2 = c1 + CH;
  double* scr = c2 + CH;
  const int64_t base = dof_off[b];
  const double* dvb = dvar + (size_t)b * nv;
  double acc = 0.0;
  for (int64_t r0 = 0; r0 < t.ncell; r0 += CH) {
    const int nr = (int)(t.ncell - r0 < CH ? t.ncell - r0 : CH);
    const int64_t g0 = base + t.cell0 + r0;
    __syncthreads();
    ev_stage(Phi, phibar, g0, nr, r, cP, uv ? nullptr : cB);
    __syncthreads();
    for (int k = tid; k < nr; k += kEV) {
      const int64_t g = g0 + k;
      double q1 = dvb[(t.cell0 + r0 + k) % nv] * ((double)ynew[g] - (double)qref[g]);
      double tt = 0.0;
      for (int c = 0; c < r; ++c) {
        q1 -= cP[k * LDR + c] * p1[c];
        tt += cP[k * LDR + c] * p2b[c];
      }
      const double qb = (js[g] + rhob * qs[g]) * irho;
      c0[k] = qb;
      c1[k] = q1;
      c2[k] = qb + tt;   // q1bar
      js[g] = qb + tt;
      if (uv) uv[g] = make_double2(-qb, q1);   // the Phibar term, kept
    }
    __syncthreads();
    if (!uv)
      for (int e = tid; e < nr * r; e += kEV) {
        const int k = e / r, c = e % r;
        phibar[g0 * r + e] = cB[k * LDR + c] - c0[k] * p2[c] + c1[k] * p2b[c];
      }
    ev_colsum(cP, c2, nr, r, acc);
  }
  ev_colsum_out(acc, r, scr, part + (size_t)blockIdx.x * evp_ld(r));
}

// Pass D: Phibar_old += -q1bar p1^T + yhat p1bar^T; yhatbar = q1bar + Phi p1bar;
// ybar += D yhatbar; with qrbar: qrbar -= D yhatbar and partials of
// sum yhatbar (y - q_ref) per variable.  With uv, the Phibar term is kept
// (uv = (-q1bar, yhat), coefficients p1 and p1bar).
template <typename T>
__global__ __launch_bounds__(kEV) void k_ev_d(
    const Tile* __restrict__ tiles, const int64_t* __restrict__ dof_off, int r, int nv,
    const double* __restrict__ dvar, const T* __restrict__ Phi, const T* __restrict__ ynew,
    const T* __restrict__ qref, const double* __restrict__ prs, const double* __restrict__ evs,
    const double* __restrict__ js, double* __restrict__ phibar, double* __restrict__ ybar,
    double* __restrict__ qrbar, double* __restrict__ part, double2* __restrict__ uv,
    double* __restrict__ ulam, double* __restrict__ ua1) {
  extern __shared__ double sm[];
  __shared__ double p1[kMaxR], p1b[kMaxR];
  __shared__ double red[kEV / 64];
  const int LDR = r + 1, tid = threadIdx.x;
  const Tile t = tiles[blockIdx.x];
  const int b = t.inst;
  const double* pr = prs + (size_t)b * (2 * r + 2);
  if (pr[2 * r] == 0.0) {
    if (uv) ev_pending_zero(t, dof_off, r, uv, ulam, ua1);
    return;
  }
  const double* e_in = evs + (size_t)b * evs_ld(r);
  for (int c = tid; c < r; c += kEV) {
    p1[c] = pr[c];
    p1b[c] = e_in[2 * r + 1 + c];
    if (uv && t.cell0 == 0) {
      ulam[(size_t)b * r + c] = pr[c];
      ua1[(size_t)b * r + c] = e_in[2 * r + 1 + c];
    }
  }
  const int CH = ev_chunk(r);
  double* cP = sm;
  double* cB = cP + CH * LDR;
  double* c0 = cB + CH * LDR;
  double* c1 = c0 + CH;
  const int64_t base = dof_off[b];
  const double* dvb = dvar + (size_t)b * nv;
  double dva[12];
  for (int v = 0; v < 12; ++v) dva[v] = 0.0;
  for (int64_t r0 = 0; r0 < t.ncell; r0 += CH) {
    const int nr = (int)(t.ncell - r0 < CH ? t.ncell - r0 : CH);
    const int64_t g0 = base + t.cell0 + r0;
    __syncthreads();
    ev_stage(Phi, phibar, g0, nr, r, cP, uv ? nullptr : cB);
    __syncthreads();
    for (int k = tid; k < nr; k += kEV) {
      const int64_t g = g0 + k;
      const int v = (int)((t.cell0 + r0 + k) % nv);
      const double d = dvb[v];
      const double dy = (double)ynew[g] - (double)qref[g];
      const double q1b = js[g];
      double tt = 0.0;
      for (int c = 0; c < r; ++c) tt += cP[k * LDR + c] * p1b[c];
      c0[k] = q1b;
      c1[k] = d * dy;
      if (uv) uv[g] = make_double2(-q1b, d * dy);   // the Phibar term, kept
      ybar[g] += d * (q1b + tt);
      if (qrbar) {
        qrbar[g] -= d * (q1b + tt);
        for (int u = 0; u < 12; ++u)
          if (u == v) dva[u] += (q1b + tt) * dy;
      }
    }
    __syncthreads();
    if (!uv)
      for (int e = tid; e < nr * r; e += kEV) {
        const int k = e / r, c = e % r;
        phibar[g0 * r + e] = cB[k * LDR + c] - c0[k] * p1[c] + c1[k] * p1b[c];
      }
  }
  if (qrbar) {
    double* out = part + (size_t)blockIdx.x * evp_ld(r);
    for (int v = 0; v < nv; ++v) {
      const double s = block_sum(dva[v], red);
      if (tid == 0) out[v] = s;
    }
  }
}

// Passes C and D for r = 32 with their Phibar terms kept (the online adjoint's
// layout): four lanes per row, eight columns each loaded straight from the
// basis, row dot products by a quad butterfly; no LDS staging.  Pass C also
// sums Phi^T q1bar per column: each lane keeps its eight columns' sums, and
// the 64 row groups' sums are added in group order at the end of the tile.
template <typename T>
DEV void ev_load8(const T* __restrict__ p, double (&v)[8]) {
  if constexpr (sizeof(T) == 4) {
    const float4 a = reinterpret_cast<const float4*>(p)[0], b = reinterpret_cast<const float4*>(p)[1];
    v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w; v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
  } else {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const double2 a = reinterpret_cast<const double2*>(p)[u];
      v[2 * u] = a.x;
      v[2 * u + 1] = a.y;
    }
  }
}

DEV double quad_sum(double x) {
  x += __shfl_xor(x, 1);
  return x + __shfl_xor(x, 2);
}

template <typename T>
__global__ __launch_bounds__(kEV) void k_ev_c32(
    const Tile* __restrict__ tiles, const int64_t* __restrict__ dof_off, int nv,
    const double* __restrict__ dvar, const T* __restrict__ Phi, const T* __restrict__ ynew,
    const T* __restrict__ qref, const double* __restrict__ prs, const double* __restrict__ evs,
    const double* __restrict__ qs, double* __restrict__ js, double* __restrict__ part,
    double2* __restrict__ uv, double* __restrict__ ulam, double* __restrict__ ua1) {
  constexpr int r = 32;
  __shared__ double p1[r], p2b[r];
  __shared__ double red[kEV / 4][r + 1];
  const int tid = threadIdx.x, q = tid & 3;
  const Tile t = tiles[blockIdx.x];
  const int b = t.inst;
  const double* pr = prs + (size_t)b * (2 * r + 2);
  const double irho = pr[2 * r];
  if (irho == 0.0) {
    ev_pending_zero(t, dof_off, r, uv, ulam, ua1);
    return;
  }
  const double* e_in = evs + (size_t)b * evs_ld(r);
  const double rhob = e_in[r];
  for (int c = tid; c < r; c += kEV) {
    p1[c] = pr[c];
    p2b[c] = e_in[r + 1 + c];
    if (t.cell0 == 0) {
      ulam[(size_t)b * r + c] = pr[r + c];
      ua1[(size_t)b * r + c] = e_in[r + 1 + c];
    }
  }
  __syncthreads();
  const int64_t g0 = dof_off[b] + t.cell0;
  const double* dvb = dvar + (size_t)b * nv;
  double acc[8];
#pragma unroll
  for (int u = 0; u < 8; ++u) acc[u] = 0.0;
  for (int64_t k = tid >> 2; k < t.ncell; k += kEV / 4) {
    const int64_t g = g0 + k;
    double v[8];
    ev_load8(Phi + g * r + 8 * q, v);
    double s1 = 0.0, s2 = 0.0;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      s1 += v[u] * p1[8 * q + u];
      s2 += v[u] * p2b[8 * q + u];
    }
    s1 = quad_sum(s1);
    s2 = quad_sum(s2);
    const double q1 = dvb[(t.cell0 + k) % nv] * ((double)ynew[g] - (double)qref[g]) - s1;
    const double qb = (js[g] + rhob * qs[g]) * irho;
    const double q1b = qb + s2;
#pragma unroll
    for (int u = 0; u < 8; ++u) acc[u] += v[u] * q1b;
    if (q == 0) {
      js[g] = q1b;
      uv[g] = make_double2(-qb, q1);
    }
  }
  // column sums: thread (row group rg, quarter q) holds columns 8 q .. 8 q + 7
#pragma unroll
  for (int u = 0; u < 8; ++u) red[tid >> 2][8 * q + u] = acc[u];
  __syncthreads();
  if (tid < r) {
    double sum = 0.0;
    for (int gq = 0; gq < kEV / 4; ++gq) sum += red[gq][tid];
    part[(size_t)blockIdx.x * evp_ld(r) + tid] = sum;
  }
}

// Pass B for r = 32 in the same layout: qbar per row, column sums of
// Phi^T qbar per lane, the row groups added in order.
template <typename T>
__global__ __launch_bounds__(kEV) void k_ev_b32(
    const Tile* __restrict__ tiles, const int64_t* __restrict__ dof_off,
    const T* __restrict__ Phi, const double* __restrict__ prs, const double* __restrict__ evs,
    const double* __restrict__ qs, const double* __restrict__ js, double* __restrict__ part) {
  constexpr int r = 32;
  __shared__ double red[kEV / 4][r + 1];
  const int tid = threadIdx.x, q = tid & 3;
  const Tile t = tiles[blockIdx.x];
  const int b = t.inst;
  const double irho = prs[(size_t)b * (2 * r + 2) + 2 * r];
  if (irho == 0.0) return;
  const double rhob = evs[(size_t)b * evs_ld(r) + r];
  const int64_t g0 = dof_off[b] + t.cell0;
  double acc[8];
#pragma unroll
  for (int u = 0; u < 8; ++u) acc[u] = 0.0;
  for (int64_t k = tid >> 2; k < t.ncell; k += kEV / 4) {
    const int64_t g = g0 + k;
    double v[8];
    ev_load8(Phi + g * r + 8 * q, v);
    const double qb = (js[g] + rhob * qs[g]) * irho;
#pragma unroll
    for (int u = 0; u < 8; ++u) acc[u] += v[u] * qb;
  }
#pragma unroll
  for (int u = 0; u < 8; ++u) red[tid >> 2][8 * q + u] = acc[u];
  __syncthreads();
  if (tid < r) {
    double sum = 0.0;
    for (int gq = 0; gq < kEV / 4; ++gq) sum += red[gq][tid];
    part[(size_t)blockIdx.x * evp_ld(r) + tid] = sum;
  }
}

template <typename T>
__global__ __launch_bounds__(kEV) void k_ev_d32(
    const Tile* __restrict__ tiles, const int64_t* __restrict__ dof_off, int nv,
    const double* __restrict__ dvar, const T* __restrict__ Phi, const T* __restrict__ ynew,
    const T* __restrict__ qref, const double* __restrict__ prs, const double* __restrict__ evs,
    const double* __restrict__ js, double* __restrict__ ybar, double2* __restrict__ uv,
    double* __restrict__ ulam, double* __restrict__ ua1) {
  constexpr int r = 32;
  __shared__ double p1b[r];
  const int tid = threadIdx.x, q = tid & 3;
  const Tile t = tiles[blockIdx.x];
  const int b = t.inst;
  const double* pr = prs + (size_t)b * (2 * r + 2);
  if (pr[2 * r] == 0.0) {
    ev_pending_zero(t, dof_off, r, uv, ulam, ua1);
    return;
  }
  const double* e_in = evs + (size_t)b * evs_ld(r);
  for (int c = tid; c < r; c += kEV) {
    p1b[c] = e_in[2 * r + 1 + c];
    if (t.cell0 == 0) {
      ulam[(size_t)b * r + c] = pr[c];
      ua1[(size_t)b * r + c] = e_in[2 * r + 1 + c];
    }
  }
  __syncthreads();
  const int64_t g0 = dof_off[b] + t.cell0;
  const double* dvb = dvar + (size_t)b * nv;
  for (int64_t k = tid >> 2; k < t.ncell; k += kEV / 4) {
    const int64_t g = g0 + k;
    double v[8];
    ev_load8(Phi + g * r + 8 * q, v);
    double s = 0.0;
#pragma unroll
    for (int u = 0; u < 8; ++u) s += v[u] * p1b[8 * q + u];
    s = quad_sum(s);
    if (q == 0) {
      const double d = dvb[(t.cell0 + k) % nv];
      const double dy = (double)ynew[g] - (double)qref[g];
      const double q1b = js[g];
      ybar[g] += d * (q1b + s);
      uv[g] = make_double2(-q1b, d * dy);
    }
  }
}

// Between the passes: dst[c] = pbar[c] - sum over the tiles (in order) of the
// partials; the last step adds the D partials to dvbar instead.
__global__ void k_ev_vec(int r, const int* __restrict__ tfirst, const double* __restrict__ prs,
                         const double* __restrict__ part, double* __restrict__ evs, int dst_off,
                         int nv, double* __restrict__ dvbar) {
  const int b = blockIdx.x;
  if (prs[(size_t)b * (2 * r + 2) + 2 * r] == 0.0) return;
  const int ld = evp_ld(r);
  double* e = evs + (size_t)b * evs_ld(r);
  if (dvbar) {
    for (int v = threadIdx.x; v < nv; v += blockDim.x) {
      double s = 0.0;
      for (int tt = tfirst[b]; tt < tfirst[b + 1]; ++tt) s += part[(size_t)tt * ld + v];
      dvbar[(size_t)b * nv + v] += s;
    }
    return;
  }
  for (int c = threadIdx.x; c < r; c += blockDim.x) {
    double s = 0.0;
    for (int tt = tfirst[b]; tt < tfirst[b + 1]; ++tt) s += part[(size_t)tt * ld + c];
    e[dst_off + c] = e[c] - s;
  }
}

__global__ void k_to_double(const float* __restrict__ x, double* __restrict__ y, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = (double)x[i];
}
__global__ void k_to_float(const double* __restrict__ x, float* __restrict__ y, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = (float)x[i];
}

}  // namespace

rom_status launch_online_seed(rom_batch* h, const void* qbar, double* abar, double* phibar,
                              hipStream_t s, double* qrbar, double* dvbar) {
  const int B = h->cfg.n_inst, r = h->cfg.r;
  if (!qrbar) {   // no q_ref / D terms: by pass tiles
    if (h->cfg.precision == ROM_F64)
      hipLaunchKernelGGL((k_seed_tile<double>), dim3(h->n_ptiles), dim3(kEV), 0, s, h->d_ptiles,
                         r, h->d_dof_off, h->d_var, h->nv, (const double*)h->Phi, h->a,
                         (const double*)qbar, phibar, h->part);
    else
      hipLaunchKernelGGL((k_seed_tile<float>), dim3(h->n_ptiles), dim3(kEV), 0, s, h->d_ptiles,
                         r, h->d_dof_off, h->d_var, h->nv, (const float*)h->Phi, h->a,
                         (const float*)qbar, phibar, h->part);
    hipLaunchKernelGGL(k_seed_abar, dim3(B), dim3(64), 0, s, r, h->d_ptile_first, h->part, abar);
    ROM_HIP_CHECK(hipGetLastError());
    return ROM_OK;
  }
  if (h->cfg.precision == ROM_F64)
    hipLaunchKernelGGL((k_online_seed<double>), dim3(B), dim3(kAT), 0, s, r, h->d_dof_off,
                       h->d_var, (const double*)h->Phi, h->a, (const double*)qbar, abar, phibar,
                       h->nv, qrbar, dvbar);
  else
    hipLaunchKernelGGL((k_online_seed<float>), dim3(B), dim3(kAT), 0, s, r, h->d_dof_off,
                       h->d_var, (const float*)h->Phi, h->a, (const float*)qbar, abar, phibar,
                       h->nv, qrbar, dvbar);
  ROM_HIP_CHECK(hipGetLastError());
  return ROM_OK;
}

size_t event_vjp_scratch_doubles(const rom_batch* h) {
  const int r = h->cfg.r;
  return (size_t)std::max(h->n_ptiles, 1) * evp_ld(r) + (size_t)h->cfg.n_inst * evs_ld(r);
}

rom_status launch_event_vjp(rom_batch* h, const void* Phi_old, const void* y_new,
                            const double* sig_old, const double* a_old, const double* ubar,
                            const double* pr, const double* sig_new, double* abar,
                            double* phibar, double* sigbar, double* ybar, double* qs, double* js,
                            double* evscr, hipStream_t s, double* qrbar, double* dvbar,
                            int* npend, int kp, double2* puv, double* plam, double* pa1) {
  const int B = h->cfg.n_inst, r = h->cfg.r, n = r + 1, nv = h->nv;
  // pending Phibar terms: pass A adds them (r = 32; else a flush first); passes
  // C and D keep theirs as two more while there is room
  int K = npend ? *npend : 0;
  if (r != kEA) {
    ROM_TRY(launch_phibar_flush(h, K, puv, plam, pa1, phibar, s));
    K = 0;
  }
  const int kA = K;
  K = 0;
  auto slot = [&](double2*& u, double*& l, double*& a1) {
    if (npend && K < kp) {
      u = puv + (size_t)K * h->total_dof;
      l = plam + (size_t)K * B * r;
      a1 = pa1 + (size_t)K * B * r;
      ++K;
    } else {
      u = nullptr;
      l = a1 = nullptr;
    }
  };
  double2 *uC, *uD;
  double *lC, *aC, *lD, *aD;
  slot(uC, lC, aC);
  slot(uD, lD, aD);
  if (npend) *npend = K;
  double* part = evscr;
  double* evs = evscr + (size_t)std::max(h->n_ptiles, 1) * evp_ld(r);
  const size_t ntl = (size_t)ev_ntl(r);
  const size_t ch = (size_t)ev_chunk(r);
  const size_t shm_a = sizeof(double) * ((size_t)n * n + std::max(ch * (2 * (r + 1) + 1),
                                                                   16 * std::max((size_t)kEV, ntl)));
  const size_t shm_core = sizeof(double) * 4 * (size_t)n * n;
  const size_t shm_b = sizeof(double) * (ch * (r + 1) + ch + kEV);
  const size_t shm_c = sizeof(double) * (2 * ch * (r + 1) + 3 * ch + kEV);
  const size_t shm_d = sizeof(double) * (2 * ch * (r + 1) + 2 * ch);
  const unsigned nt = (unsigned)h->n_ptiles;
  auto go = [&](auto tag) {
    using T = decltype(tag);
    if (r == kEA)
      hipLaunchKernelGGL((k_ev_a_mfma<T>), dim3(nt), dim3(kEV), 0, s, h->d_ptiles, h->d_dof_off,
                         nv, h->d_var, (const T*)Phi_old, (const T*)y_new, (const T*)h->q_ref,
                         ubar, pr, phibar, qs, js, part, kA, h->total_dof, puv, plam, pa1, B);
    else
      hipLaunchKernelGGL((k_ev_a<T>), dim3(nt), dim3(kEV), shm_a, s, h->d_ptiles, h->d_dof_off,
                         r, nv, h->d_var, (const T*)Phi_old, (const T*)y_new, (const T*)h->q_ref,
                         ubar, pr, phibar, qs, js, part);
    hipLaunchKernelGGL(k_ev_core, dim3(B), dim3(kEV), shm_core, s, r, h->cfg.lambda,
                       h->d_ptile_first, part, sig_old, a_old, ubar, pr, sig_new, abar, sigbar,
                       evs, h->flags);
    if (r == 32)
      hipLaunchKernelGGL((k_ev_b32<T>), dim3(nt), dim3(kEV), 0, s, h->d_ptiles, h->d_dof_off,
                         (const T*)Phi_old, pr, evs, qs, js, part);
    else
      hipLaunchKernelGGL((k_ev_b<T>), dim3(nt), dim3(kEV), shm_b, s, h->d_ptiles, h->d_dof_off,
                         r, (const T*)Phi_old, pr, evs, qs, js, part);
    hipLaunchKernelGGL(k_ev_vec, dim3(B), dim3(64), 0, s, r, h->d_ptile_first, pr, part, evs,
                       r + 1, nv, (double*)nullptr);
    if (r == 32 && uC)
      hipLaunchKernelGGL((k_ev_c32<T>), dim3(nt), dim3(kEV), 0, s, h->d_ptiles, h->d_dof_off, nv,
                         h->d_var, (const T*)Phi_old, (const T*)y_new, (const T*)h->q_ref, pr,
                         evs, qs, js, part, uC, lC, aC);
    else
      hipLaunchKernelGGL((k_ev_c<T>), dim3(nt), dim3(kEV), shm_c, s, h->d_ptiles, h->d_dof_off,
                         r, nv, h->d_var, (const T*)Phi_old, (const T*)y_new, (const T*)h->q_ref,
                         pr, evs, qs, js, phibar, part, uC, lC, aC);
    hipLaunchKernelGGL(k_ev_vec, dim3(B), dim3(64), 0, s, r, h->d_ptile_first, pr, part, evs,
                       2 * r + 1, nv, (double*)nullptr);
    if (r == 32 && uD && !qrbar)
      hipLaunchKernelGGL((k_ev_d32<T>), dim3(nt), dim3(kEV), 0, s, h->d_ptiles, h->d_dof_off, nv,
                         h->d_var, (const T*)Phi_old, (const T*)y_new, (const T*)h->q_ref, pr,
                         evs, js, ybar, uD, lD, aD);
    else
      hipLaunchKernelGGL((k_ev_d<T>), dim3(nt), dim3(kEV), shm_d, s, h->d_ptiles, h->d_dof_off, r,
                         nv, h->d_var, (const T*)Phi_old, (const T*)y_new, (const T*)h->q_ref, pr,
                         evs, js, phibar, ybar, qrbar, part, uD, lD, aD);
    if (qrbar)
      hipLaunchKernelGGL(k_ev_vec, dim3(B), dim3(64), 0, s, r, h->d_ptile_first, pr, part, evs,
                         0, nv, dvbar);
  };
  if (h->cfg.precision == ROM_F64) go(double{});
  else go(float{});
  ROM_HIP_CHECK(hipGetLastError());
  return ROM_OK;
}

rom_status launch_step_vjp_deferred(rom_batch* h, const void* Phi, const double* a1,
                                    double* abar, double2* uv, hipStream_t s,
                                    const void* mpart) {
  if (!mpart) mpart = h->mpart;
  const int B = h->cfg.n_inst, r = h->cfg.r;
  auto go = [&](auto tag) {
    using T = decltype(tag);
    hipLaunchKernelGGL((k_step_vjp_solve<T>), dim3(B), dim3(kAT), 0, s, r, h->cfg.dt,
                       h->d_ptile_first, (const T*)mpart, mfma_ok(h) && r == 32 ? 1 : 0,
                       abar, h->flags);
    hipLaunchKernelGGL((k_step_vjp_uv<T>), dim3(h->n_ptiles), dim3(kRT), 0, s, h->d_ptiles, r,
                       h->cfg.dt, h->d_dof_off, h->d_phys, h->cfg.n_phys, h->d_var,
                       (const T*)Phi, (const T*)h->q_ref, a1, abar, uv);
  };
  if (h->cfg.precision == ROM_F64) go(double{});
  else go(float{});
  ROM_HIP_CHECK(hipGetLastError());
  return ROM_OK;
}

rom_status launch_phibar_flush(rom_batch* h, int K, const double2* uv, const double* lam,
                               const double* a1, double* phibar, hipStream_t s) {
  ROM_REQUIRE(K >= 0 && K <= kPhibarPending, ROM_E_INVAL, "too many pending step terms");
  if (K == 0) return ROM_OK;
  hipLaunchKernelGGL(k_phibar_flush, dim3(h->n_ptiles), dim3(kRT), 0, s, h->d_ptiles,
                     h->cfg.r, h->d_dof_off, K, h->total_dof, uv, lam, a1,
                     (int64_t)h->cfg.n_inst, phibar);
  ROM_HIP_CHECK(hipGetLastError());
  return ROM_OK;
}

rom_status convert_words(const void* src, bool src_f64, void* dst, bool dst_f64, int64_t n,
                         hipStream_t s) {
  if (src_f64 == dst_f64) {
    ROM_HIP_CHECK(hipMemcpyAsync(dst, src, (size_t)n * (src_f64 ? 8 : 4), hipMemcpyDeviceToDevice, s));
    return ROM_OK;
  }
  const int64_t nb = (n + 255) / 256;
  if (nb > 0) {
    if (src_f64) hipLaunchKernelGGL(k_to_float, dim3(nb), dim3(256), 0, s, (const double*)src, (float*)dst, n);
    else hipLaunchKernelGGL(k_to_double, dim3(nb), dim3(256), 0, s, (const float*)src, (double*)dst, n);
  }
  ROM_HIP_CHECK(hipGetLastError());
  return ROM_OK;
}

rom_status adjoint_kernels_prepare() {
  // the largest dynamic LDS of each kernel (r = 64, n = 65)
  constexpr int n = kMaxR + 1;
  const int big_a = (int)(sizeof(double) * (n * n + std::max(kEVLds + 2 * kEC, 16 * 272)));
  const int big_c = (int)(sizeof(double) * (kEVLds + kEV));
  const int big_core = (int)(sizeof(double) * 4 * n * n);
  static_assert(((kMaxR + 1 + kETI - 1) / kETI) * ((kMaxR + kETJ - 1) / kETJ) <= 272,
                "tile count bound of the pass A partials");
  ROM_HIP_CHECK(hipFuncSetAttribute((const void*)k_ev_a<float>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, big_a));
  ROM_HIP_CHECK(hipFuncSetAttribute((const void*)k_ev_a<double>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, big_a));
  ROM_HIP_CHECK(hipFuncSetAttribute((const void*)k_ev_core,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, big_core));
  const void* chunked[] = {(const void*)k_ev_b<float>, (const void*)k_ev_b<double>,
                           (const void*)k_ev_c<float>, (const void*)k_ev_c<double>,
                           (const void*)k_ev_d<float>, (const void*)k_ev_d<double>};
  for (const void* f : chunked)
    ROM_HIP_CHECK(hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, big_c));
  return ROM_OK;
}

}  // namespace romhip
