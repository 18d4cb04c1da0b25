// Reverse mode of Alg. 1's online loop (an extension; the paper has no
// adjoint): Galerkin fine steps (Burgers), adaptation events with the coarse
// backward-Euler step, the Brand update (Alg. 2) and the closed-form state
// transfer.  FP64 throughout; the basis and the states are read in the
// storage precision T.
//
//  * k_online_seed: the loss seed at the end, q~ = q_ref + D^-1 Phi a:
//    abar = Phi^T D^-1 qbar, Phibar = D^-1 qbar a^T.
//  * k_step_vjp_solve + k_step_vjp_rows: one fine step a_{n+1} = G(a_n, Phi) with
//    g(a) = a - a_n - dt Phi^T D f(q_ref + D^-1 Phi a) = 0, differentiated by
//    the implicit-function theorem at the converged a_{n+1}:
//    J_g^T lambda = abar, abar_n = lambda and
//    Phibar += dt (D f) lambda^T + dt D^-1 J_f^T (D Phi lambda) a_{n+1}^T.
//    J_g = I - dt Phi^T J_f Phi comes from the Galerkin pass's tile partials;
//    the r x r solve runs per instance, the Phibar update per pass tile.
//  * k_event_vjp: one event from the transfer back to yhat = D (y - q_ref):
//    transfer a' = Ubar[:r, :r]^T a, rotation Phi' = [Phi, q / rho] Ubar[:, :r],
//    truncation sigma' = Sbar[:r], the SVD of the core K (distinct singular
//    values: Kbar = Ubar G Vbar^T with G_ii = sbar_i and
//    G_ij = s_j (M_ij - M_ji) / (s_j^2 - s_i^2), M = Ubar^T Ubarbar), the core's
//    entries lambda sigma, p = p1 + p2 and rho = |q|, and the two classical
//    Gram-Schmidt passes, one workgroup per instance.  The coarse step's
//    transposed solve is done by the banded solver outside.
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

// One fine step backward, in two launches.  k_step_vjp_solve (a workgroup per
// instance): lambda = J_g^-T abar with J_g = I - dt M, M = Phi^T J_f Phi at a1
// (= a_{n+1}) summed from the Galerkin pass's tile partials in tile order;
// abar is replaced by lambda.  k_step_vjp_rows (a workgroup per pass tile):
// Phibar += dt d f lambda^T + dt (J_f^T Phi lambda) a1^T over the tile's rows,
// with q~ = q_ref + D^-1 Phi a1 and w = Phi lambda of the rows and their two
// neighbours kept in LDS (the neighbours are recomputed by each tile).
template <typename T>
__global__ __launch_bounds__(kAT) void k_step_vjp_solve(int r, double dt,
                                                        const int* __restrict__ tfirst,
                                                        const T* __restrict__ mpart,
                                                        double* __restrict__ abar,
                                                        uint32_t* flags) {
  __shared__ double A[kMaxR * (kMaxR + 1)];
  __shared__ double lam[kMaxR];
  const int b = blockIdx.x, tid = threadIdx.x;
  const int ld = r + 1;
  const int t0 = tfirst[b], t1 = tfirst[b + 1];
  for (int e = tid; e < r * r; e += kAT) {
    double s = 0.0;
    for (int tt = t0; tt < t1; ++tt) s += (double)mpart[(size_t)tt * kMaxR * kMaxR + e];
    const int i = e / r, j = e % r;
    A[j * ld + i] = (i == j ? 1.0 : 0.0) - dt * s;
  }
  for (int c = tid; c < r; c += kAT) lam[c] = abar[(size_t)b * r + c];
  __syncthreads();
  const int ok = block_lu_solve(A, ld, lam, r);
  if (!ok && tid == 0) atomicOr(&flags[b], ROM_FLAG_SINGULAR);
  for (int c = tid; c < r; c += kAT) abar[(size_t)b * r + c] = lam[c];
}

constexpr int kRT = 256;   // threads of k_step_vjp_rows
constexpr int kSL = 8;     // lanes per row (each holds kSL-strided columns)

template <typename T>
__global__ __launch_bounds__(kRT) void k_step_vjp_rows(
    const Tile* __restrict__ tiles, int r, double dt, const int64_t* __restrict__ dof_off,
    const double* __restrict__ phys, int nphys, const double* __restrict__ dvar,
    const T* __restrict__ Phi, const T* __restrict__ qref, const double* __restrict__ a1,
    const double* __restrict__ lambda, double* __restrict__ phibar) {
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
  const int sub = tid % kSL;
  // q~ and w of rows cell0 - 1 .. cell0 + nt (periodic), each summed over its lanes
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
  __syncthreads();
  for (int rr = tid / kSL; rr < nt; rr += kRT / kSL) {
    const int64_t i = t.cell0 + rr;
    double f, be, al_next, ga_prev;
    burgers_col(sq[rr], sq[rr + 1], sq[rr + 2], nu, inv, inv2, f, be, al_next, ga_prev);
    const double v = al_next * sw[rr + 2] + be * sw[rr + 1] + ga_prev * sw[rr];
    double* pb = phibar + (base + i) * r;
    for (int c = sub; c < r; c += kSL) pb[c] += dt * d * f * lam[c] + dt * v * sa[c];
  }
}

constexpr int kET = 512;  // threads of the event adjoint

constexpr int kEChunk = 8192;   // elements of a staged chunk (rows x r), at most
constexpr int kELds = 19200;    // doubles of dynamic LDS, at most (150 KB)

// Rows of a staged chunk: as many as the LDS left after the three n x n core
// matrices holds (two rows x (r + 1) arrays, rows padded by one double so that
// lanes walking rows hit distinct banks, and four per-row scalars), at most
// 1024 rows and kEChunk elements.
DEV_HOST_INLINE int event_chunk_rows(int r) {
  const int n = r + 1;
  int c = (kELds - 3 * n * n - n) / (2 * (r + 1) + 4);
  if (c > kEChunk / r) c = kEChunk / r;
  return c > 1024 ? 1024 : c;
}

constexpr int kEPF = (kEChunk + kET - 1) / kET;   // chunk elements per thread

// Loads of one chunk (ne <= kEChunk elements from offset off) into registers, so that the
// next chunk is in flight while the current one is processed from LDS.
template <typename T>
DEV void chunk_fetch(const T* __restrict__ Phi, const double* __restrict__ pb, int64_t off, int ne,
                     bool with_b, double (&rp)[kEPF], double (&rb)[kEPF]) {
  const int tid = threadIdx.x;
#pragma unroll
  for (int u = 0; u < kEPF; ++u) {
    const int e = tid + u * kET;
    if (e < ne) {
      rp[u] = (double)Phi[off + e];
      if (with_b) rb[u] = pb[off + e];
    }
  }
}

// Element e = k r + c of the chunk goes to row k, column c of the padded LDS
// copy (row stride r + 1).
DEV void chunk_put(double* cP, double* cB, int ne, int r, bool with_b, const double (&rp)[kEPF],
                   const double (&rb)[kEPF]) {
  const int tid = threadIdx.x;
#pragma unroll
  for (int u = 0; u < kEPF; ++u) {
    const int e = tid + u * kET;
    if (e < ne) {
      const int k = e / r;
      const int o = e + k;   // k (r + 1) + (e - k r)
      cP[o] = rp[u];
      if (with_b) cB[o] = rb[u];
    }
  }
}

// One event backward, from the transfer down to yhat (the coarse step's
// transposed solve follows outside).  Inputs recorded in the forward pass:
// Phi_old, y_new (after the coarse step), sigma_old, a_old (before the
// transfer), Ubar (n x n), pr = (p1, p2, 1/rho, s_n).  abar, sigbar and the
// rows of phibar are replaced by the adjoints of the pre-event state; ybar
// receives D yhatbar.  Rows are streamed in chunks staged in LDS (Phi as FP64
// and the matching rows of phibar, rows padded to r + 1); dynamic LDS:
// 3 n^2 + 2 C (r + 1) + 4 C + n
// doubles for C = event_chunk_rows(r).
template <typename T>
__global__ __launch_bounds__(kET) void k_event_vjp(
    int r, double lam_f, const int64_t* __restrict__ dof_off, const double* __restrict__ dvar,
    const T* __restrict__ Phi, const T* __restrict__ ynew, const T* __restrict__ qref,
    const double* __restrict__ sig_old, const double* __restrict__ a_old,
    const double* __restrict__ ubar, const double* __restrict__ prs,
    const double* __restrict__ sig_new, double* __restrict__ abar,
    double* __restrict__ phibar, double* __restrict__ sigbar, double* __restrict__ ybar,
    double* __restrict__ qs, double* __restrict__ js, uint32_t* flags, int nv,
    double* __restrict__ qrbar, double* __restrict__ dvbar) {
  extern __shared__ double sm[];
  __shared__ double red[kET / 64];
  __shared__ double vr[7][kMaxR + 1];  // p1, p2, abar', pbar (rhobar in [r]), p1bar, p2bar, wr
  __shared__ double sv[kMaxR + 1];
  const int n = r + 1, tid = threadIdx.x, b = blockIdx.x;
  const int CH = event_chunk_rows(r);
  double* U = sm;               // Ubar
  double* Ub = U + n * n;       // its adjoint, then G
  double* X = Ub + n * n;       // U^T Ub, then V
  const int LDR = r + 1;         // padded row stride of the staged chunk
  double* cP = X + n * n;       // chunk of Phi rows (FP64)
  double* cB = cP + CH * LDR;   // the same rows of phibar
  double* c0 = cB + CH * LDR;   // per-row scalars of the chunk
  double* c1 = c0 + CH;
  double* c2 = c1 + CH;
  double* c3 = c2 + CH;
  double* p1 = vr[0];
  double* p2 = vr[1];
  double* ab = vr[2];
  double* pb = vr[3];
  double* p1b = vr[4];
  double* p2b = vr[5];
  double* wr = vr[6];
  const int64_t base = dof_off[b], nd = dof_off[b + 1] - base;
  const double* dvb = dvar + (size_t)b * nv;   // D per variable; row i has variable i mod nv
  const double* pr = prs + (size_t)b * (2 * r + 2);
  const double irho = pr[2 * r];
  if (irho == 0.0) {   // rho = 0: the update is not differentiable there
    if (tid == 0) atomicOr(&flags[b], ROM_FLAG_SINGULAR);
    return;
  }
  const double rho = 1.0 / irho;
  for (int e = tid; e < n * n; e += kET) {
    U[e] = ubar[(size_t)b * n * n + e];
    Ub[e] = 0.0;
  }
  for (int c = tid; c < r; c += kET) {
    p1[c] = pr[c];
    p2[c] = pr[r + c];
    ab[c] = abar[(size_t)b * r + c];
    sv[c] = sig_new[(size_t)b * r + c];
  }
  if (tid == 0) sv[r] = pr[2 * r + 1];
  __syncthreads();
  // transfer a' = U[:r, :r]^T a: abar_old = U[:r, :r] abar, Ubar[:r, :r] += a_old abar^T
  for (int c = tid; c < r; c += kET) {
    double s = 0.0;
    for (int k = 0; k < r; ++k) s += U[c * n + k] * ab[k];
    abar[(size_t)b * r + c] = s;
  }
  for (int e = tid; e < r * r; e += kET) {
    const int i = e / r, j = e % r;
    Ub[i * n + j] += a_old[(size_t)b * r + i] * ab[j];
  }
  __syncthreads();
  // pass A: q = yhat - Phi (p1 + p2); rotation adjoint Ubar[:r, :r] += Phi^T Phibar',
  // Ubar[r, :r] += (q / rho)^T Phibar'; rows Phibar_old = Phibar' U[:r, :r]^T and
  // jbar = Phibar' U[r, :r]^T; jq = jbar . q
  double jq = 0.0;
  double rp[kEPF], rb[kEPF];
  auto chunk_ne = [&](int64_t r0) { return (int)((nd - r0 < CH ? nd - r0 : CH) * r); };
  // Ubar rows 0..r (row r from q / rho) against the r columns of Phibar', in
  // 4 x 4 register tiles; KS thread groups split the rows of each chunk and
  // keep their sums over the whole pass, added in group order at the end
  constexpr int TI = 4, TJ = 4;
  const int NI = (n + TI - 1) / TI, NJ = (r + TJ - 1) / TJ, NTL = NI * NJ;
  int KS = kET / NTL;
  if (KS * NTL * TI * TJ > 2 * CH * LDR) KS = 2 * CH * LDR / (NTL * TI * TJ);
  if (KS < 1) KS = 1;
  const bool tl_on = tid < NTL * KS;
  const int ks = tid / NTL, tt = tid - (tid / NTL) * NTL;
  const int i0 = (tt / NJ) * TI, j0 = (tt - (tt / NJ) * NJ) * TJ;
  double ta[TI][TJ];
#pragma unroll
  for (int a = 0; a < TI; ++a)
#pragma unroll
    for (int c = 0; c < TJ; ++c) ta[a][c] = 0.0;
  if (nd > 0) chunk_fetch(Phi, phibar, base * r, chunk_ne(0), true, rp, rb);
  for (int64_t r0 = 0; r0 < nd; r0 += CH) {
    const int nr = (int)(nd - r0 < CH ? nd - r0 : CH);
    chunk_put(cP, cB, nr * r, r, true, rp, rb);
    __syncthreads();
    if (r0 + CH < nd) chunk_fetch(Phi, phibar, (base + r0 + CH) * r, chunk_ne(r0 + CH), true, rp, rb);
    for (int k = tid; k < nr; k += kET) {
      double q = dvb[(r0 + k) % nv] * ((double)ynew[base + r0 + k] - (double)qref[base + r0 + k]);
      for (int c = 0; c < r; ++c) q -= cP[k * LDR + c] * (p1[c] + p2[c]);
      c0[k] = q;
      qs[base + r0 + k] = q;
    }
    __syncthreads();
    if (tl_on) {
      for (int k = ks; k < nr; k += KS) {
        double av[TI], bv[TJ];
#pragma unroll
        for (int a = 0; a < TI; ++a) {
          const int i = i0 + a;
          av[a] = i < r ? cP[k * LDR + i] : (i == r ? c0[k] * irho : 0.0);
        }
#pragma unroll
        for (int c = 0; c < TJ; ++c) bv[c] = j0 + c < r ? cB[k * LDR + j0 + c] : 0.0;
#pragma unroll
        for (int a = 0; a < TI; ++a)
#pragma unroll
          for (int c = 0; c < TJ; ++c) ta[a][c] += av[a] * bv[c];
      }
    }
    // rows of Phibar_old = Phibar' U[:r, :r]^T and jbar = Phibar' U[r, :r]^T in 4 x 3
    // register tiles (each output summed over m in order by one thread)
    {
      constexpr int TR = 4, TC = 3;
      const int NR = (nr + TR - 1) / TR, NC = (n + TC - 1) / TC;
      for (int e = tid; e < NR * NC; e += kET) {
        const int k0 = (e / NC) * TR, c0t = (e - (e / NC) * NC) * TC;
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
          for (int c = 0; c < TC; ++c) uv[c] = c0t + c < n ? U[(c0t + c) * n + m] : 0.0;
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
            const int cc = c0t + c;
            if (cc < r) phibar[(base + r0 + k) * r + cc] = o[a][c];
            else if (cc == r) {
              js[base + r0 + k] = o[a][c];
              jq += o[a][c] * c0[k];
            }
          }
        }
      }
    }
    __syncthreads();
  }
  // the row groups' sums of the Ubar tiles, added in group order (the chunk area is free)
  {
    double* part = cP;
    if (tl_on) {
#pragma unroll
      for (int a = 0; a < TI; ++a)
#pragma unroll
        for (int c = 0; c < TJ; ++c) part[((size_t)ks * NTL + tt) * (TI * TJ) + a * TJ + c] = ta[a][c];
    }
    __syncthreads();
    for (int e = tid; e < n * r; e += kET) {
      const int i = e / r, j = e % r;
      const int t2 = (i / TI) * NJ + j / TJ, w = (i % TI) * TJ + j % TJ;
      double sacc = 0.0;
      for (int g = 0; g < KS; ++g) sacc += part[((size_t)g * NTL + t2) * (TI * TJ) + w];
      Ub[i * n + j] += sacc;
    }
    __syncthreads();
  }
  jq = block_sum(jq, red);
  // SVD of K: M = U^T Ub (in X), G (in Ub), V = K^T U / s (in X), then the entries of
  // Kbar = U G V^T that K depends on: lambda sigma (diagonal), p (last column), rho
  for (int e = tid; e < n * n; e += kET) {
    const int i = e / n, j = e % n;
    double s = 0.0;
    for (int k = 0; k < n; ++k) s += U[k * n + i] * Ub[k * n + j];
    X[e] = s;
  }
  __syncthreads();
  for (int e = tid; e < n * n; e += kET) {
    const int i = e / n, j = e % n;
    double g;
    if (i == j) g = i < r ? sigbar[(size_t)b * r + i] : 0.0;
    else g = sv[j] > 0.0 ? sv[j] * (X[i * n + j] - X[j * n + i]) / ((sv[j] - sv[i]) * (sv[j] + sv[i]))
                         : 0.0;
    Ub[e] = g;
  }
  __syncthreads();
  for (int e = tid; e < n * n; e += kET) {
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
  for (int k = tid; k < n; k += kET) {   // wr = G V[r, :]^T
    double s = 0.0;
    for (int m = 0; m < n; ++m) s += Ub[k * n + m] * X[r * n + m];
    wr[k] = s;
  }
  __syncthreads();
  double* GVt = cP;   // (G V^T)[k][c], in the chunk area (at least n^2 doubles)
  for (int e = tid; e < n * n; e += kET) {
    const int k = e / n, c = e - (e / n) * n;
    double gv = 0.0;
    for (int m = 0; m < n; ++m) gv += Ub[k * n + m] * X[c * n + m];
    GVt[e] = gv;
  }
  __syncthreads();
  for (int c = tid; c < n; c += kET) {
    double kd = 0.0, kc = 0.0;
    for (int k = 0; k < n; ++k) {
      kd += U[c * n + k] * GVt[k * n + c];
      kc += U[c * n + k] * wr[k];
    }
    if (c < r) {
      sigbar[(size_t)b * r + c] = lam_f * kd;
      pb[c] = kc;
    } else {
      pb[r] = kc;
    }
  }
  __syncthreads();
  // j = q / rho, rho = |q|: qbar = (jbar + rhobar q) / rho
  const double rhob = pb[r] - jq * irho * irho;
  // pass B: p2bar = pbar - Phi^T qbar (G row groups of r threads; their sums
  // are added in group order)
  const int G = kET / r;
  const int gq = tid / r, gc = tid - (tid / r) * r;
  auto group_sum = [&](double acc, double* out) {
    __syncthreads();
    if (gq < G) cP[gq * r + gc] = acc;
    __syncthreads();
    if (tid < r) {
      double sacc = 0.0;
      for (int g = 0; g < G; ++g) sacc += cP[g * r + tid];
      out[tid] = pb[tid] - sacc;
    }
    __syncthreads();
  };
  double acc = 0.0;
  if (nd > 0) chunk_fetch(Phi, phibar, base * r, chunk_ne(0), false, rp, rb);
  for (int64_t r0 = 0; r0 < nd; r0 += CH) {
    const int nr = (int)(nd - r0 < CH ? nd - r0 : CH);
    chunk_put(cP, cB, nr * r, r, false, rp, rb);
    if (r0 + CH < nd) chunk_fetch(Phi, phibar, (base + r0 + CH) * r, chunk_ne(r0 + CH), false, rp, rb);
    for (int k = tid; k < nr; k += kET)
      c0[k] = (js[base + r0 + k] + rhob * qs[base + r0 + k]) * irho;
    __syncthreads();
    if (gq < G)
      for (int k = gq; k < nr; k += G) acc += cP[k * LDR + gc] * c0[k];
    __syncthreads();
  }
  group_sum(acc, p2b);
  // pass C: q1 = yhat - Phi p1, q1bar = qbar + Phi p2bar (into js);
  // Phibar_old += -qbar p2^T + q1 p2bar^T; p1bar = pbar - Phi^T q1bar
  acc = 0.0;
  if (nd > 0) chunk_fetch(Phi, phibar, base * r, chunk_ne(0), true, rp, rb);
  for (int64_t r0 = 0; r0 < nd; r0 += CH) {
    const int nr = (int)(nd - r0 < CH ? nd - r0 : CH);
    chunk_put(cP, cB, nr * r, r, true, rp, rb);
    __syncthreads();
    if (r0 + CH < nd) chunk_fetch(Phi, phibar, (base + r0 + CH) * r, chunk_ne(r0 + CH), true, rp, rb);
    for (int k = tid; k < nr; k += kET) {
      const int64_t g = base + r0 + k;
      double q1 = dvb[(r0 + k) % nv] * ((double)ynew[g] - (double)qref[g]);
      double t = 0.0;
      for (int c = 0; c < r; ++c) {
        q1 -= cP[k * LDR + c] * p1[c];
        t += cP[k * LDR + c] * p2b[c];
      }
      const double qb = (js[g] + rhob * qs[g]) * irho;
      c0[k] = qb;
      c1[k] = q1;
      c2[k] = qb + t;   // q1bar
      js[g] = qb + t;
    }
    __syncthreads();
    for (int e = tid; e < nr * r; e += kET) {
      const int k = e / r, c = e % r;
      phibar[(base + r0) * r + e] = cB[k * LDR + c] - c0[k] * p2[c] + c1[k] * p2b[c];
    }
    if (gq < G)
      for (int k = gq; k < nr; k += G) acc += cP[k * LDR + gc] * c2[k];
    __syncthreads();
  }
  group_sum(acc, p1b);
  // pass D: Phibar_old += -q1bar p1^T + yhat p1bar^T; yhatbar = q1bar + Phi p1bar;
  // ybar += D yhatbar; with qrbar: qrbar -= D yhatbar, and dvbar[v] += the sum
  // of yhatbar (y - q_ref) over the rows of variable v
  double dva[12];
  for (int v = 0; v < 12; ++v) dva[v] = 0.0;
  if (nd > 0) chunk_fetch(Phi, phibar, base * r, chunk_ne(0), true, rp, rb);
  for (int64_t r0 = 0; r0 < nd; r0 += CH) {
    const int nr = (int)(nd - r0 < CH ? nd - r0 : CH);
    chunk_put(cP, cB, nr * r, r, true, rp, rb);
    __syncthreads();
    if (r0 + CH < nd) chunk_fetch(Phi, phibar, (base + r0 + CH) * r, chunk_ne(r0 + CH), true, rp, rb);
    for (int k = tid; k < nr; k += kET) {
      const int64_t g = base + r0 + k;
      const int v = (int)((r0 + k) % nv);
      const double d = dvb[v];
      const double dy = (double)ynew[g] - (double)qref[g];
      const double yh = d * dy;
      const double q1b = js[g];
      double t = 0.0;
      for (int c = 0; c < r; ++c) t += cP[k * LDR + c] * p1b[c];
      c0[k] = q1b;
      c1[k] = yh;
      ybar[g] += d * (q1b + t);
      if (qrbar) {
        qrbar[g] -= d * (q1b + t);
        for (int u = 0; u < 12; ++u)
          if (u == v) dva[u] += (q1b + t) * dy;
      }
    }
    __syncthreads();
    for (int e = tid; e < nr * r; e += kET) {
      const int k = e / r, c = e % r;
      phibar[(base + r0) * r + e] = cB[k * LDR + c] - c0[k] * p1[c] + c1[k] * p1b[c];
    }
    __syncthreads();
  }
  if (qrbar) {
    for (int v = 0; v < nv; ++v) {
      const double sv_ = block_sum(dva[v], red);
      if (tid == 0) dvbar[(size_t)b * nv + v] += sv_;
    }
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

rom_status launch_step_vjp(rom_batch* h, const void* Phi, const double* a1, double* abar,
                           double* phibar, hipStream_t s) {
  const int B = h->cfg.n_inst, r = h->cfg.r;
  auto go = [&](auto tag) {
    using T = decltype(tag);
    hipLaunchKernelGGL((k_step_vjp_solve<T>), dim3(B), dim3(kAT), 0, s, r, h->cfg.dt,
                       h->d_ptile_first, (const T*)h->mpart, abar, h->flags);
    hipLaunchKernelGGL((k_step_vjp_rows<T>), dim3(h->n_ptiles), dim3(kRT), 0, s, h->d_ptiles, r,
                       h->cfg.dt, h->d_dof_off, h->d_phys, h->cfg.n_phys, h->d_var,
                       (const T*)Phi, (const T*)h->q_ref, a1, abar, phibar);
  };
  if (h->cfg.precision == ROM_F64) go(double{});
  else go(float{});
  ROM_HIP_CHECK(hipGetLastError());
  return ROM_OK;
}

size_t event_vjp_shm(int r) {
  const size_t n = (size_t)r + 1, C = (size_t)event_chunk_rows(r);
  return sizeof(double) * (3 * n * n + 2 * C * (r + 1) + 4 * C + n);
}

rom_status launch_event_vjp(rom_batch* h, const void* Phi_old, const void* y_new,
                            const double* sig_old, const double* a_old, const double* ubar,
                            const double* pr, const double* sig_new, double* abar,
                            double* phibar, double* sigbar, double* ybar, double* qs, double* js,
                            hipStream_t s, double* qrbar, double* dvbar) {
  const int B = h->cfg.n_inst, r = h->cfg.r;
  const size_t shm = event_vjp_shm(r);
  if (h->cfg.precision == ROM_F64)
    hipLaunchKernelGGL((k_event_vjp<double>), dim3(B), dim3(kET), shm, s, r, h->cfg.lambda,
                       h->d_dof_off, h->d_var, (const double*)Phi_old, (const double*)y_new,
                       (const double*)h->q_ref, sig_old, a_old, ubar, pr, sig_new, abar, phibar,
                       sigbar, ybar, qs, js, h->flags, h->nv, qrbar, dvbar);
  else
    hipLaunchKernelGGL((k_event_vjp<float>), dim3(B), dim3(kET), shm, s, r, h->cfg.lambda,
                       h->d_dof_off, h->d_var, (const float*)Phi_old, (const float*)y_new,
                       (const float*)h->q_ref, sig_old, a_old, ubar, pr, sig_new, abar, phibar,
                       sigbar, ybar, qs, js, h->flags, h->nv, qrbar, dvbar);
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
  const int big = (int)(sizeof(double) * kELds);   // bound of event_vjp_shm(r) for every r
  ROM_HIP_CHECK(hipFuncSetAttribute((const void*)k_event_vjp<float>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, big));
  ROM_HIP_CHECK(hipFuncSetAttribute((const void*)k_event_vjp<double>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, big));
  return ROM_OK;
}

}  // namespace romhip
