#include <algorithm>
// Incremental SVD (Alg. 2) and the offline POD / preprocessing on the device.
//
// Tall-skinny passes: a block owns a row tile (<= kPassRows rows of one
// instance) and walks it in chunks of kChunk rows.  Each chunk of the
// row-major basis is staged through LDS with coalesced loads; the
// per-row scalar work (snapshot preprocessing y^ = D (y - q_ref), the row dot
// products of the second Gram-Schmidt pass) runs one row per thread, and the
// column reductions run one column per lane with FP64 accumulation.  Block
// partials are reduced per instance in a fixed order, so results do not
// depend on scheduling.
//
// The (r+1) x (r+1) core K = [[lambda diag(sigma), p], [0, rho]] is
// decomposed by one-sided (Hestenes) Jacobi on its rows in FP64, one
// workgroup per instance with both K and the accumulated rotations in LDS;
// rows are orthogonalised pairwise in round-robin order until every pair is
// orthogonal to 2 n eps relative.
#include "internal.h"
#include "linalg.h"
#include "physics.h"

namespace romhip {

constexpr int kChunk = 64;
constexpr int kMaxK = 128;          // widest matrix a pass handles (POD window)
constexpr int kPst = kMaxK + 4;     // partial-sum stride per tile

namespace {

template <typename T>
DEV double yhat_of(const T* y, const T* qref, const double* dvar, int nv, int64_t gdof,
                   int64_t ldof) {
  return dvar[ldof % nv] * ((double)y[gdof] - (double)qref[gdof]);
}

// mode 1: partial[c] = sum_i Phi_ic y^_i,  partial[k] = sum_i y^_i^2
// mode 2: q1_i = y^_i - Phi_i . p1 ; partial[c] = sum_i Phi_ic q1_i, partial[k] = sum q1_i^2;
//         q1 is also written to q1out (FP64) when given
// When qref == nullptr the snapshot is used as is (y^ = y).
template <typename T>
__global__ __launch_bounds__(256) void k_project(const Tile* __restrict__ tiles,
                                                 const int64_t* __restrict__ dof_off,
                                                 const T* __restrict__ Phi, int ld, int k,
                                                 const T* __restrict__ y, const T* __restrict__ qref,
                                                 const double* __restrict__ dvar, int nv,
                                                 const double* __restrict__ p1, int ldp, int mode,
                                                 double* __restrict__ part,
                                                 double* __restrict__ q1out, int split) {
  __shared__ T sP[kChunk][kMaxK + 1];
  __shared__ double sY[kChunk];
  __shared__ double sp[kMaxK];
  __shared__ double red[4][kMaxK + 1];
  // block blockIdx.x takes part blockIdx.x % split of tile blockIdx.x / split
  // and writes its own partial (an empty part writes zeros)
  Tile t = tiles[blockIdx.x / split];
  {
    const int pt = blockIdx.x % split;
    const int64_t len = (t.ncell + split - 1) / split;
    const int64_t lo = pt * len < t.ncell ? pt * len : t.ncell;
    t.cell0 += lo;
    t.ncell = t.ncell - lo < len ? t.ncell - lo : len;
  }
  const int b = t.inst;
  const int tid = threadIdx.x;
  const int64_t base = dof_off[b];
  const double* dv = dvar ? dvar + (size_t)b * nv : nullptr;
  if (mode == 2)
    for (int c = tid; c < k; c += blockDim.x) sp[c] = p1[(size_t)b * ldp + c];
  const int lane = tid & 63, grp = tid >> 6;
  double acc0 = 0.0, acc1 = 0.0, accn = 0.0;
  for (int64_t r0 = 0; r0 < t.ncell; r0 += kChunk) {
    const int nr = (int)(t.ncell - r0 < kChunk ? t.ncell - r0 : kChunk);
    const int64_t row0 = t.cell0 + r0;  // instance-local row of the chunk
    __syncthreads();
    {
      // eight loads per thread in flight (indices clamped into the chunk),
      // then the LDS stores
      const int ne = nr * k;
      for (int e0 = tid; e0 < ne; e0 += 256 * 8) {
        T v[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const int e = e0 + 256 * j < ne ? e0 + 256 * j : ne - 1;
          const int rr = e / k, c = e - rr * k;
          v[j] = Phi[(base + row0 + rr) * ld + c];
        }
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const int e = e0 + 256 * j;
          if (e < ne) {
            const int rr = e / k, c = e - rr * k;
            sP[rr][c] = v[j];
          }
        }
      }
    }
    if (tid < nr) {
      const int64_t g = base + row0 + tid;
      sY[tid] = qref ? yhat_of(y, qref, dv, nv, g, row0 + tid) : (double)y[g];
    }
    __syncthreads();
    if (mode == 2 && tid < nr) {
      double d = 0.0;
      for (int c = 0; c < k; ++c) d += (double)sP[tid][c] * sp[c];
      sY[tid] -= d;
      // the second Gram-Schmidt projection must act on this stored vector:
      // recomputing it elsewhere differs in the last bits, which for a
      // nearly dependent snapshot is the size of the residual itself
      if (q1out) q1out[base + row0 + tid] = sY[tid];
    }
    __syncthreads();
    for (int rr = grp; rr < nr; rr += 4) {
      const double yv = sY[rr];
      if (lane < k) acc0 += (double)sP[rr][lane] * yv;
      if (lane + 64 < k) acc1 += (double)sP[rr][lane + 64] * yv;
      if (lane == 0) accn += yv * yv;
    }
  }
  __syncthreads();
  if (lane < k) red[grp][lane] = acc0;
  if (lane + 64 < k) red[grp][lane + 64] = acc1;
  if (lane == 0) red[grp][kMaxK] = accn;
  __syncthreads();
  double* out = part + (size_t)blockIdx.x * kPst;
  for (int c = tid; c < k; c += blockDim.x) out[c] = red[0][c] + red[1][c] + red[2][c] + red[3][c];
  if (tid == 0) out[k] = red[0][kMaxK] + red[1][kMaxK] + red[2][kMaxK] + red[3][kMaxK];
}

// Sum the tile partials of each instance in tile order: dst[b*ldd + c], c <= k.
// With split > 1 each tile has split consecutive partials.
__global__ void k_reduce_tiles(const int* __restrict__ tfirst, const double* __restrict__ part, int k,
                               double* __restrict__ dst, int ldd, int split) {
  const int b = blockIdx.x;
  for (int c = threadIdx.x; c <= k; c += blockDim.x) {
    double s = 0.0;
    for (int tt = tfirst[b] * split; tt < tfirst[b + 1] * split; ++tt) s += part[(size_t)tt * kPst + c];
    dst[(size_t)b * ldd + c] = s;
  }
}

// ------------------------------------------------------------------ small SVD
DEV void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Rotation that orthogonalises two rows with squared norms al, be and inner
// product ga: tan(theta) = t with t the smaller root of t^2 + 2 zeta t - 1 = 0,
// zeta = (be - al) / (2 ga), written as t = 2 ga sign / (|be - al| +
// sqrt((be - al)^2 + 4 ga^2)) (one square root and one division on the
// critical path), cos = 1 / sqrt(1 + t^2), sin = t cos.
DEV void rotation(double al, double be, double ga, double& cs, double& sn) {
  const double dd = be - al;
  const double num = (dd * ga >= 0.0) ? fabs(2.0 * ga) : -fabs(2.0 * ga);
  const double tt = num / (fabs(dd) + sqrt(dd * dd + 4.0 * ga * ga));
  cs = rsqrt(1.0 + tt * tt);
  sn = cs * tt;
}

// One-sided Jacobi on the rows of the n x n matrix K (LDS, leading dim ld),
// run by a single wavefront (blockDim.x == 64, n <= 128): K <- G K with G
// orthogonal until the rows are mutually orthogonal.  Then sigma_i = ||row i||
// and row i of G is the left singular vector.  Pairs of a round (circle
// ordering) are independent, so each gets a lane group of TPP lanes and the
// rounds are separated by wave-level fences only.  On exit the sorted
// (descending, stable) vectors are the columns of U (n x n, row-major, global)
// with the sign convention "largest |entry| positive, first index on ties",
// and the sorted values are in sv.
DEV void jacobi_rows(double* K, double* G, int n, int ld, double* U, double* sv, double* norms,
                     int* rank) {
  const int lane = threadIdx.x;
  for (int e = lane; e < n * ld; e += 64) G[e] = ((e / ld) == (e % ld)) ? 1.0 : 0.0;
  wave_sync();
  const int np = n + (n & 1);
  const int npairs = np / 2;
  int TPP = 1;
  while (TPP * 2 * npairs <= 64) TPP *= 2;
  const int grp = lane / TPP, sub = lane % TPP, ngrp = 64 / TPP;
  // rows count as orthogonal below 2 n eps: below that the rounding of the
  // length-n dot products and of the rotations themselves dominates
  const double tol = 2.0 * n * 2.220446049250313e-16, tol2 = tol * tol;
  for (int sweep = 0; sweep < 30; ++sweep) {
    int rotated = 0;
    for (int rnd = 0; rnd < np - 1; ++rnd) {
      for (int pr = grp; pr < npairs; pr += ngrp) {
        // circle method: slot 0 fixed, the other np-1 slots rotate each round
        const int a = pr == 0 ? 0 : ((pr - 1 + rnd) % (np - 1)) + 1;
        const int c = ((np - 2 - pr + rnd) % (np - 1)) + 1;
        const int i = a < c ? a : c, j = a < c ? c : a;
        const bool live = j < n;
        double al = 0.0, be = 0.0, ga = 0.0;
        if (live) {
          for (int q = sub; q < n; q += TPP) {
            const double x = K[i * ld + q], z = K[j * ld + q];
            al += x * x; be += z * z; ga += x * z;
          }
        }
        for (int off = 1; off < TPP; off <<= 1) {
          al += __shfl_xor(al, off, TPP);
          be += __shfl_xor(be, off, TPP);
          ga += __shfl_xor(ga, off, TPP);
        }
        if (live && ga != 0.0 && ga * ga > tol2 * al * be) {
          double cs, sn;
          rotation(al, be, ga, cs, sn);
          for (int q = sub; q < n; q += TPP) {
            const double x = K[i * ld + q], z = K[j * ld + q];
            K[i * ld + q] = cs * x - sn * z;
            K[j * ld + q] = sn * x + cs * z;
            const double gx = G[i * ld + q], gz = G[j * ld + q];
            G[i * ld + q] = cs * gx - sn * gz;
            G[j * ld + q] = sn * gx + cs * gz;
          }
          rotated = 1;
        }
      }
      wave_sync();
    }
    if (!__any(rotated)) break;
  }
  for (int i = lane; i < n; i += 64) {
    double s = 0.0;
    for (int q = 0; q < n; ++q) s += K[i * ld + q] * K[i * ld + q];
    norms[i] = sqrt(s);
  }
  wave_sync();
  for (int i = lane; i < n; i += 64) {
    int rk = 0;
    for (int j = 0; j < n; ++j)
      if (norms[j] > norms[i] || (norms[j] == norms[i] && j < i)) ++rk;
    rank[i] = rk;
    sv[rk] = norms[i];
  }
  wave_sync();
  // sign convention per vector (row i of G), then scatter as column rank[i] of U
  for (int i = lane; i < n; i += 64) {
    int im = 0;
    double best = -1.0;
    for (int q = 0; q < n; ++q) {
      const double v = fabs(G[i * ld + q]);
      if (v > best) { best = v; im = q; }
    }
    const double sg = G[i * ld + im] < 0.0 ? -1.0 : 1.0;
    const int col = rank[i];
    for (int q = 0; q < n; ++q) U[q * n + col] = sg * G[i * ld + q];
  }
  __syncthreads();
}

// The same one-sided Jacobi for a compile-time size N (the online core, N = r + 1
// with r in {32, 64}), run by a whole 256-thread block: each pair of a round
// gets TPP lanes (8 for N = 33, 4 for N = 65), every lane loads its at most
// EPL elements of both K rows and both G rows at once, keeps the K values in
// registers for the rotation, and the rounds are separated by one block
// barrier.  Same pair order, test and conventions as jacobi_rows.
template <int N>
DEV void jacobi_rows_blk(double* K, double* G, double* U, double* sv, double* norms, int* rank) {
  constexpr int ld = N;
  constexpr int NP = N + (N & 1), NPAIRS = NP / 2;
  constexpr int TPP = NPAIRS * 16 <= 256 ? 16 : NPAIRS * 8 <= 256 ? 8 : NPAIRS * 4 <= 256 ? 4 : 2;
  constexpr int EPL = (N + TPP - 1) / TPP;
  static_assert(NPAIRS * TPP <= 256, "core too large for one block");
  const int tid = threadIdx.x, grp = tid / TPP, sub = tid % TPP;
  for (int e = tid; e < N * ld; e += 256) G[e] = ((e / ld) == (e % ld)) ? 1.0 : 0.0;
  __syncthreads();
  const double tol = 2.0 * N * 2.220446049250313e-16, tol2 = tol * tol;
  for (int sweep = 0; sweep < 30; ++sweep) {
    int rotated = 0;
    for (int rnd = 0; rnd < NP - 1; ++rnd) {
      if (grp < NPAIRS) {
        const int a = grp == 0 ? 0 : ((grp - 1 + rnd) % (NP - 1)) + 1;
        const int c = ((NP - 2 - grp + rnd) % (NP - 1)) + 1;
        const int i = a < c ? a : c, j = a < c ? c : a;
        if (j < N) {
          double x[EPL], z[EPL], gx[EPL], gz[EPL];
          double al = 0.0, be = 0.0, ga = 0.0;
#pragma unroll
          for (int e = 0; e < EPL; ++e) {
            const int q = sub + TPP * e;
            const bool in = q < N;
            x[e] = in ? K[i * ld + q] : 0.0;
            z[e] = in ? K[j * ld + q] : 0.0;
            gx[e] = in ? G[i * ld + q] : 0.0;
            gz[e] = in ? G[j * ld + q] : 0.0;
          }
#pragma unroll
          for (int e = 0; e < EPL; ++e) {
            al += x[e] * x[e];
            be += z[e] * z[e];
            ga += x[e] * z[e];
          }
#pragma unroll
          for (int off = 1; off < TPP; off <<= 1) {
            al += __shfl_xor(al, off, TPP);
            be += __shfl_xor(be, off, TPP);
            ga += __shfl_xor(ga, off, TPP);
          }
          if (ga != 0.0 && ga * ga > tol2 * al * be) {
            double cs, sn;
            rotation(al, be, ga, cs, sn);
#pragma unroll
            for (int e = 0; e < EPL; ++e) {
              const int q = sub + TPP * e;
              if (q < N) {
                K[i * ld + q] = cs * x[e] - sn * z[e];
                K[j * ld + q] = sn * x[e] + cs * z[e];
                G[i * ld + q] = cs * gx[e] - sn * gz[e];
                G[j * ld + q] = sn * gx[e] + cs * gz[e];
              }
            }
            rotated = 1;
          }
        }
      }
      __syncthreads();
    }
    if (!__syncthreads_or(rotated)) break;
  }
  if (tid < N) {
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < N; ++q) s += K[tid * ld + q] * K[tid * ld + q];
    norms[tid] = sqrt(s);
  }
  __syncthreads();
  if (tid < N) {
    int rk = 0;
    const double ni = norms[tid];
#pragma unroll
    for (int j = 0; j < N; ++j) {
      const double nj = norms[j];
      if (nj > ni || (nj == ni && j < tid)) ++rk;
    }
    rank[tid] = rk;
    sv[rk] = ni;
  }
  __syncthreads();
  // sign convention per vector (row i of G), then scatter as column rank[i] of U
  if (tid < N) {
    int im = 0;
    double best = -1.0;
#pragma unroll
    for (int q = 0; q < N; ++q) {
      const double v = fabs(G[tid * ld + q]);
      if (v > best) { best = v; im = q; }
    }
    const double sg = G[tid * ld + im] < 0.0 ? -1.0 : 1.0;
    const int col = rank[tid];
#pragma unroll 4
    for (int q = 0; q < N; ++q) U[q * N + col] = sg * G[tid * ld + q];
  }
  __syncthreads();
}

// ------------------------------------------------------------------ arrowhead SVD
// Left singular vectors and values of the core K = [[diag(d), p], [0, rho]]
// (d = lambda sigma, sorted descending) from the eigenproblem of
// K K^T = D^2 + z z^T, D = diag(d, 0), z = (p, rho): a rank-one change of a
// diagonal matrix (Brand's update core).  Steps, one wavefront per instance:
//  * scale by max(|d|, |z|);
//  * deflation: weights |z_i| <= 8 eps max(d_0, |z|) give the value d_i with
//    vector e_i; a pole within that tolerance of the previous kept pole is
//    removed by a plane rotation that moves its weight onto the kept one;
//  * the K remaining roots of the secular equation
//      1 + sum_i zeta_i^2 / (delta_i^2 - omega^2) = 0
//    one per lane, each in its interlacing interval, written as
//    omega = delta_o + tau with o the nearer pole so that every
//    delta_i - omega = (delta_i - delta_o) - tau is formed without
//    cancellation; iteration on a two-pole rational model of the secular
//    function (value and slope of the sums over the poles on each side) with a
//    bisection safeguard;
//  * weights recomputed from the roots by Loewner's formula
//      zhat_i^2 = prod_k (omega_k^2 - delta_i^2) / prod_{j != i} (delta_j^2 - delta_i^2),
//    which makes the vectors u_k ~ zhat / (delta^2 - omega_k^2) orthogonal to
//    working precision (Gu and Eisenstat);
//  * the deflation rotations undone, then the same stable descending sort and
//    sign convention as the Jacobi path.
// Returns false (nothing written) when d is not sorted descending.
DEV void sec_sums(int o, double x, int k, int K, const double* delta, const double* zeta2,
                  double& psi, double& dpsi, double& phi, double& dphi, double& dl, double& du) {
  const double dO = delta[o], w = dO + x;
  psi = dpsi = phi = dphi = 0.0;
  dl = du = 0.0;
  for (int i = 0; i < K; ++i) {
    const double den = ((delta[i] - dO) - x) * (delta[i] + w);   // delta_i^2 - omega^2
    const double inv = 1.0 / den;
    const double t = zeta2[i] * inv;
    if (i >= k) { psi += t; dpsi += t * inv; } else { phi += t; dphi += t * inv; }
    if (i == k) dl = den;
    if (i == k - 1) du = den;
  }
}

DEV void sec_root(int k, int K, const double* delta, const double* zeta2, double rho2, int& o,
                  double& tau) {
  const double eps = 2.220446049250313e-16;
  if (K == 1) {  // closed form: omega^2 = delta_0^2 + zeta_0^2
    o = 0;
    tau = zeta2[0] / (delta[0] + sqrt(delta[0] * delta[0] + zeta2[0]));
    return;
  }
  double lo, hi, psi, dpsi, phi, dphi, dl, du;
  if (k == 0) {
    o = 0;
    lo = 0.0;
    hi = rho2 / (delta[0] + sqrt(delta[0] * delta[0] + rho2));
  } else {
    const double a2 = (delta[k - 1] - delta[k]) * (delta[k - 1] + delta[k]);
    const double wm = sqrt(0.5 * (delta[k - 1] * delta[k - 1] + delta[k] * delta[k]));
    const double tm = 0.5 * a2 / (wm + delta[k]);
    sec_sums(k, tm, k, K, delta, zeta2, psi, dpsi, phi, dphi, dl, du);
    if (1.0 + psi + phi >= 0.0) { o = k; lo = 0.0; hi = tm; }
    else { o = k - 1; lo = -(0.5 * a2) / (delta[k - 1] + wm); hi = 0.0; }
  }
  const double dO = delta[o];
  double x = 0.5 * (lo + hi);
  for (int it = 0; it < 100; ++it) {
    sec_sums(o, x, k, K, delta, zeta2, psi, dpsi, phi, dphi, dl, du);
    const double g = 1.0 + psi + phi;
    if (g == 0.0) break;
    if (g < 0.0) lo = x; else hi = x;
    const double sl = dpsi * dl * dl;
    double c = 1.0 + (psi - sl / dl), eta;
    if (k == 0) {
      c += phi;
      eta = c != 0.0 ? dl + sl / c : NAN;
    } else {
      const double su = dphi * du * du;
      c += phi - su / du;
      const double B = c * (dl + du) + sl + su;
      const double disc = sqrt(fmax(B * B - 4.0 * c * dl * du * g, 0.0));
      eta = B > 0.0 ? 2.0 * dl * du * g / (B + disc) : (c != 0.0 ? (B - disc) / (2.0 * c) : NAN);
    }
    const double mu_rel = x * (2.0 * dO + x) + eta;             // omega'^2 - delta_o^2
    double xn = isfinite(eta) ? mu_rel / (sqrt(fmax(dO * dO + mu_rel, 0.0)) + dO) : NAN;
    if (isfinite(xn) && fabs(xn - x) <= 4.0 * eps * fabs(x)) {
      if (lo < xn && xn < hi) x = xn;
      break;
    }
    if (!(lo < xn && xn < hi)) xn = 0.5 * (lo + hi);
    if (hi - lo <= 2.0 * eps * fmax(fabs(lo), fabs(hi))) { x = xn; break; }
    x = xn;
  }
  tau = x;
}

// K: the core in LDS (N x N, row-major); Uc: LDS N x N scratch (column c at
// Uc + c N); U: output N x N (row-major, columns = sorted vectors); sv: LDS N.
DEV bool arrow_svd_wave(const int N, const double* K, double* Uc, double* U, double* sv, double* ws,
                        int* iw) {
  const int lane = threadIdx.x & 63;
  const double eps = 2.220446049250313e-16;
  double* d = ws;            // N
  double* z = d + N;         // N
  double* delta = z + N;     // N
  double* zeta2 = delta + N; // N
  double* zsgn = zeta2 + N;  // N
  double* tau = zsgn + N;    // N
  double* omg = tau + N;     // N
  double* zhat = omg + N;    // N
  double* vals = zhat + N;   // N
  double* rc = vals + N;     // N
  double* rsn = rc + N;      // N
  double* scal = rsn + N;    // [0] scale, [1] rho2
  int* L = iw;               // N: kept poles
  int* orig = L + N;         // N
  int* ri = orig + N;        // N
  int* rj = ri + N;          // N
  int* key = rj + N;         // N
  int* rnk = key + N;        // N
  int* dfl = rnk + N;        // N: deflated indices in order
  int* cnt = dfl + N;        // [0] K, [1] nrot, [2] ndefl
  double m = 0.0;
  int sorted = 1;
  for (int i = lane; i < N; i += 64) {
    d[i] = i < N - 1 ? K[i * N + i] : 0.0;
    z[i] = K[i * N + N - 1];
    m = fmax(m, fmax(fabs(d[i]), fabs(z[i])));
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off));
  lds_wave_sync();
  for (int i = lane; i + 1 < N; i += 64)
    if (!(d[i] >= d[i + 1])) sorted = 0;
  if (!__all(sorted)) return false;
  const double scale = m;
  if (scale == 0.0) {
    for (int e = lane; e < N * N; e += 64) U[e] = (e / N == e % N) ? 1.0 : 0.0;
    for (int i = lane; i < N; i += 64) sv[i] = 0.0;
    lds_wave_sync();
    return true;
  }
  for (int i = lane; i < N; i += 64) { d[i] /= scale; z[i] /= scale; }
  lds_wave_sync();
  if (lane == 0) {  // deflation (at most N entries; sequential)
    double zn2 = 0.0;
    for (int i = 0; i < N; ++i) zn2 += z[i] * z[i];
    const double tol = 8.0 * eps * fmax(d[0], sqrt(zn2));
    int nrot = 0, nd = 0, prev = -1;
    for (int j = 0; j < N; ++j) {
      if (fabs(z[j]) <= tol) { z[j] = 0.0; dfl[nd++] = j; continue; }
      if (prev >= 0 && d[prev] - d[j] <= tol) {
        const double h = hypot(z[prev], z[j]);
        const double c = z[prev] / h, sn = z[j] / h;
        z[prev] = h;
        z[j] = 0.0;
        ri[nrot] = prev; rj[nrot] = j; rc[nrot] = c; rsn[nrot] = sn;
        ++nrot;
        dfl[nd++] = j;
        continue;
      }
      prev = j;
    }
    int Kk = 0;
    double rho2 = 0.0;
    for (int j = 0; j < N; ++j) {
      if (z[j] == 0.0) continue;
      L[Kk] = j;
      delta[Kk] = d[j];
      zeta2[Kk] = z[j] * z[j];
      zsgn[Kk] = z[j] < 0.0 ? -1.0 : 1.0;
      rho2 += zeta2[Kk];
      ++Kk;
    }
    cnt[0] = Kk; cnt[1] = nrot; cnt[2] = nd;
    scal[1] = rho2;
  }
  lds_wave_sync();
  const int Kk = cnt[0], nrot = cnt[1], nd = cnt[2];
  const double rho2 = scal[1];
  for (int k = lane; k < Kk; k += 64) {
    int o;
    double t;
    sec_root(k, Kk, delta, zeta2, rho2, o, t);
    orig[k] = o;
    tau[k] = t;
    omg[k] = delta[o] + t;
  }
  lds_wave_sync();
  for (int mm = lane; mm < Kk; mm += 64) {  // Loewner weights
    const double dm = delta[mm];
    double p = ((delta[orig[mm]] - dm) + tau[mm]) * (omg[mm] + dm);
    for (int k = 0; k < Kk; ++k) {
      if (k == mm) continue;
      const double wd = (delta[orig[k]] - dm) + tau[k];
      p *= (wd * (omg[k] + dm)) / ((delta[k] - dm) * (delta[k] + dm));
    }
    zhat[mm] = zsgn[mm] * sqrt(fabs(p));
  }
  for (int e = lane; e < N * N; e += 64) Uc[e] = 0.0;
  lds_wave_sync();
  for (int k = lane; k < Kk; k += 64) {  // vectors of the kept poles
    const int o = orig[k];
    double nn = 0.0;
    for (int mm = 0; mm < Kk; ++mm) {
      const double v = zhat[mm] / (((delta[mm] - delta[o]) - tau[k]) * (delta[mm] + omg[k]));
      Uc[k * N + L[mm]] = v;
      nn += v * v;
    }
    const double inv = 1.0 / sqrt(nn);
    for (int mm = 0; mm < Kk; ++mm) Uc[k * N + L[mm]] *= inv;
    vals[k] = omg[k] * scale;
    key[k] = L[k];
  }
  for (int t = lane; t < nd; t += 64) {  // deflated: e_j with value d_j
    const int j = dfl[t];
    Uc[(Kk + t) * N + j] = 1.0;
    vals[Kk + t] = d[j] * scale;
    key[Kk + t] = j;
  }
  lds_wave_sync();
  for (int c = lane; c < N; c += 64) {   // undo the deflation rotations, last first
    double* col = Uc + c * N;
    for (int t = nrot - 1; t >= 0; --t) {
      const int i = ri[t], j = rj[t];
      const double vi = col[i], vj = col[j];
      col[i] = rc[t] * vi - rsn[t] * vj;
      col[j] = rsn[t] * vi + rc[t] * vj;
    }
  }
  lds_wave_sync();
  for (int c = lane; c < N; c += 64) {   // stable descending rank
    int rk = 0;
    const double vc = vals[c];
    for (int c2 = 0; c2 < N; ++c2) {
      const double v2 = vals[c2];
      if (v2 > vc || (v2 == vc && key[c2] < key[c])) ++rk;
    }
    rnk[c] = rk;
    sv[rk] = vc;
  }
  lds_wave_sync();
  for (int c = lane; c < N; c += 64) {   // sign convention, scatter as column rank
    const double* col = Uc + c * N;
    int im = 0;
    double best = -1.0;
    for (int q = 0; q < N; ++q) {
      const double v = fabs(col[q]);
      if (v > best) { best = v; im = q; }
    }
    const double sg = col[im] < 0.0 ? -1.0 : 1.0;
    const int dst = rnk[c];
    for (int q = 0; q < N; ++q) U[q * N + dst] = sg * col[q];
  }
  lds_wave_sync();
  return true;
}

// Core of Alg. 2: K from lambda, sigma, p, rho; SVD; sigma' and the transfer of a.
// red layout per instance: [0..r) p1, r: |y^|^2, [r+1..2r+1) p2, 2r+1: |q1|^2
// One wavefront per instance: the arrowhead SVD (arrow_svd_wave), with the
// one-sided Jacobi SVD (jacobi_rows) when sigma is not sorted (ARROW), or
// Jacobi alone (!ARROW).
template <bool ARROW>
__global__ __launch_bounds__(64) void k_isvd_core(int r, double lambda, double tau_rho,
                                                  const double* __restrict__ red, int ldr,
                                                  double* __restrict__ sigma,
                                                  double* __restrict__ ubar, double* __restrict__ pr,
                                                  uint32_t* flags) {
  extern __shared__ double sm[];
  const int n = r + 1, ld = n;
  double* K = sm;
  double* G = K + n * ld;
  double* nrm = G + n * ld;
  double* sv = nrm + n;
  double* ta = sv + n;
  int* rank = (int*)(ta + n);
  __shared__ double rho_s;
  const int b = blockIdx.x, tid = threadIdx.x;
  const double* R = red + (size_t)b * ldr;
  double* U = ubar + (size_t)b * n * n;
  if (tid == 0) {
    double yy = R[r], s1 = R[2 * r + 1], p2n = 0.0;
    for (int c = 0; c < r; ++c) p2n += R[r + 1 + c] * R[r + 1 + c];
    double rho2 = s1 - p2n;
    double rho = rho2 > 0.0 ? sqrt(rho2) : 0.0;
    if (!(rho > tau_rho * sqrt(yy))) {
      rho = 0.0;
      atomicOr(&flags[b], ROM_FLAG_RHO_ZERO);
    }
    rho_s = rho;
  }
  __syncthreads();
  for (int e = tid; e < n * ld; e += blockDim.x) {
    const int i = e / ld, j = e % ld;
    double v = 0.0;
    if (i < r && j < r) v = i == j ? lambda * sigma[(size_t)b * r + i] : 0.0;
    else if (i < r && j == r) v = R[i] + R[r + 1 + i];  // p = p1 + p2
    else if (i == r && j == r) v = rho_s;
    K[e] = v;
  }
  __syncthreads();
  if constexpr (!ARROW) {
    jacobi_rows(K, G, n, ld, U, sv, nrm, rank);
  } else {
    // arrowhead SVD (one wavefront); Jacobi when sigma is not sorted
    double* ws = reinterpret_cast<double*>(rank + n + (n & 1));
    int* iw = reinterpret_cast<int*>(ws + 13 * n);
    if (!arrow_svd_wave(n, K, G, U, sv, ws, iw)) jacobi_rows(K, G, n, ld, U, sv, nrm, rank);
    __syncthreads();
  }
  for (int c = tid; c < r; c += blockDim.x) sigma[(size_t)b * r + c] = sv[c];
  // p1, p2 (kept apart: the rotation subtracts them one after the other), 1/rho and
  // the (r+1)-th singular value
  for (int c = tid; c < r; c += blockDim.x) {
    pr[(size_t)b * (2 * r + 2) + c] = R[c];
    pr[(size_t)b * (2 * r + 2) + r + c] = R[r + 1 + c];
  }
  if (tid == 0) {
    pr[(size_t)b * (2 * r + 2) + 2 * r] = rho_s > 0.0 ? 1.0 / rho_s : 0.0;
    pr[(size_t)b * (2 * r + 2) + 2 * r + 1] = sv[r];   // the truncated singular value
  }
}

// Closed-form state transfer of an iSVD update: a <- Ubar[:r, :r]^T a (the new
// direction is orthogonal to Phi, so its coefficient is zero).  One 64-thread
// block per instance.
__global__ __launch_bounds__(64) void k_isvd_transfer(int r, const double* __restrict__ ubar,
                                                      double* __restrict__ a) {
  __shared__ double sU[kMaxR * (kMaxR + 1)];  // rows 0 .. r-1 of Ubar (row length n)
  __shared__ double sa[kMaxR];
  const int b = blockIdx.x, tid = threadIdx.x, n = r + 1;
  const double* U = ubar + (size_t)b * n * n;
  for (int e = tid; e < r * n; e += blockDim.x) sU[e] = U[e];   // all loads in flight at once
  for (int k = tid; k < r; k += blockDim.x) sa[k] = a[(size_t)b * r + k];
  __syncthreads();
  for (int c = tid; c < r; c += blockDim.x) {
    double s = 0.0;
    for (int k = 0; k < r; ++k) s += sU[k * n + c] * sa[k];
    a[(size_t)b * r + c] = s;
  }
}

// Phi_out[i, j] = sum_{c<kin} Phi_in[i, c] U[c, j] (+ s_i U[kin, j]),  j < kout,
// with s_i = (q1_i - Phi_in[i,:] p2) / rho for the iSVD update (mode 1), q1 the
// first-pass residual stored by the second projection pass, and no extra term
// otherwise (mode 0).  pr holds (p1, p2, 1/rho) per instance (stride ldpr).
// U is (kin+1) x ldu per instance (FP64).
// enable (optional): instances with enable[b] == 0 are left untouched.
template <typename T>
__global__ __launch_bounds__(256) void k_rotate(const Tile* __restrict__ tiles,
                                                const int64_t* __restrict__ dof_off,
                                                const T* Phi_in, int ld_in, int kin, T* Phi_out,
                                                int ld_out, int kout, const double* __restrict__ U,
                                                int ldu, size_t ustride, int mode,
                                                const double* __restrict__ q1,
                                                const double* __restrict__ pr, int ldpr,
                                                const int32_t* __restrict__ enable, int split) {
  __shared__ T sP[kChunk][kMaxK + 1];
  __shared__ double sS[kChunk];
  __shared__ double sU[(kMaxK + 1) * 64];
  __shared__ double sp[2 * kMaxR + 1];
  // block blockIdx.x takes part blockIdx.x % split of tile blockIdx.x / split
  // (few tiles, as for one large instance, still fill the chip)
  Tile t = tiles[blockIdx.x / split];
  {
    const int part = blockIdx.x % split;
    const int64_t len = (t.ncell + split - 1) / split;
    const int64_t lo = part * len;
    if (lo >= t.ncell) return;
    t.cell0 += lo;
    t.ncell = t.ncell - lo < len ? t.ncell - lo : len;
  }
  const int b = t.inst;
  if (enable && !enable[b]) return;
  const int tid = threadIdx.x;
  const int64_t base = dof_off[b];
  const double* Ub = U + (size_t)b * ustride;
  const int krow = mode == 1 ? kin + 1 : kin;
  for (int e = tid; e < krow * kout; e += blockDim.x) {
    const int c = e / kout, j = e % kout;
    sU[c * 64 + j] = Ub[c * ldu + j];
  }
  if (mode == 1)
    for (int c = tid; c <= 2 * kin; c += blockDim.x) sp[c] = pr[(size_t)b * ldpr + c];
  const int lane = tid & 63, grp = tid >> 6;
  for (int64_t r0 = 0; r0 < t.ncell; r0 += kChunk) {
    const int nr = (int)(t.ncell - r0 < kChunk ? t.ncell - r0 : kChunk);
    const int64_t row0 = t.cell0 + r0;
    __syncthreads();
    {
      // eight loads per thread in flight (indices clamped into the chunk),
      // then the LDS stores
      const int ne = nr * kin;
      for (int e0 = tid; e0 < ne; e0 += 256 * 8) {
        T v[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const int e = e0 + 256 * j < ne ? e0 + 256 * j : ne - 1;
          const int rr = e / kin, c = e - rr * kin;
          v[j] = Phi_in[(base + row0 + rr) * ld_in + c];
        }
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const int e = e0 + 256 * j;
          if (e < ne) {
            const int rr = e / kin, c = e - rr * kin;
            sP[rr][c] = v[j];
          }
        }
      }
    }
    __syncthreads();
    if (mode == 1 && tid < nr) {
      double d2 = 0.0;
      for (int c = 0; c < kin; ++c) d2 += (double)sP[tid][c] * sp[kin + c];
      sS[tid] = (q1[base + row0 + tid] - d2) * sp[2 * kin];
    }
    __syncthreads();
    if (lane < kout) {
      // four rows per wave at a time (rows grp + 4 j), four independent sums,
      // each over the columns in order
      for (int rb = grp; rb < nr; rb += 16) {
        double acc[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int rr = rb + 4 * j < nr ? rb + 4 * j : rb;
          acc[j] = mode == 1 ? sS[rr] * sU[kin * 64 + lane] : 0.0;
        }
        for (int c = 0; c < kin; ++c) {
          const double u = sU[c * 64 + lane];
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const int rr = rb + 4 * j < nr ? rb + 4 * j : rb;
            acc[j] += (double)sP[rr][c] * u;
          }
        }
#pragma unroll
        for (int j = 0; j < 4; ++j)
          if (rb + 4 * j < nr) Phi_out[(base + row0 + rb + 4 * j) * ld_out + lane] = (T)acc[j];
      }
    }
  }
}

// The same projection and rotation for narrow matrices (k, kin, kout <= 16):
// one row per thread with the row and its sums in registers, so every lane
// works (the generic kernels above keep one lane per column).  Rows of a tile
// are visited in the same order by every launch, and the per-column sums are
// reduced by wavefront shuffles and then over the block's waves in order.
constexpr int kNarrow = 16;

template <typename T>
__global__ __launch_bounds__(256) void k_project_small(const Tile* __restrict__ tiles,
                                                       const int64_t* __restrict__ dof_off,
                                                       const T* __restrict__ Phi, int ld, int k,
                                                       const T* __restrict__ y,
                                                       const T* __restrict__ qref,
                                                       const double* __restrict__ dvar, int nv,
                                                       const double* __restrict__ p1, int ldp,
                                                       int mode, double* __restrict__ part,
                                                       double* __restrict__ q1out) {
  __shared__ double red[4][kNarrow + 1];
  __shared__ double sp[kNarrow];
  __shared__ T sIn[256 * kNarrow];   // the chunk's rows, loaded contiguously
  const Tile t = tiles[blockIdx.x];
  const int b = t.inst, tid = threadIdx.x;
  const int64_t base = dof_off[b];
  const double* dv = dvar ? dvar + (size_t)b * nv : nullptr;
  if (mode == 2 && tid < k) sp[tid] = p1[(size_t)b * ldp + tid];
  double acc[kNarrow + 1];
#pragma unroll
  for (int c = 0; c <= kNarrow; ++c) acc[c] = 0.0;
  for (int64_t r0 = 0; r0 < t.ncell; r0 += 256) {
    const int nr = (int)(t.ncell - r0 < 256 ? t.ncell - r0 : 256);
    const int64_t g0 = base + t.cell0 + r0;
    __syncthreads();
    {
      T v[kNarrow];   // all loads of the chunk in flight before the LDS writes
#pragma unroll
      for (int u = 0; u < kNarrow; ++u) {
        const int e = u * 256 + tid < nr * k ? u * 256 + tid : 0;   // unconditional load
        const int rr = e / k;
        v[u] = Phi[(g0 + rr) * ld + (e - rr * k)];
      }
#pragma unroll
      for (int u = 0; u < kNarrow; ++u)
        if (u * 256 + tid < nr * k) sIn[u * 256 + tid] = v[u];
    }
    __syncthreads();
    if (tid < nr) {
      const int64_t lr = t.cell0 + r0 + tid, g = g0 + tid;
      double row[kNarrow];
#pragma unroll
      for (int c = 0; c < kNarrow; ++c) row[c] = c < k ? (double)sIn[tid * k + c] : 0.0;
      double yv = qref ? yhat_of(y, qref, dv, nv, g, lr) : (double)y[g];
      if (mode == 2) {
        double d = 0.0;
#pragma unroll
        for (int c = 0; c < kNarrow; ++c)
          if (c < k) d += row[c] * sp[c];
        yv -= d;
        if (q1out) q1out[g] = yv;
      }
#pragma unroll
      for (int c = 0; c < kNarrow; ++c)
        if (c < k) acc[c] += row[c] * yv;
      acc[kNarrow] += yv * yv;
    }
  }
  const int lane = tid & 63, wv = tid >> 6;
#pragma unroll
  for (int c = 0; c <= kNarrow; ++c) {
    const double v = wave_sum_bfly(acc[c]);
    if (lane == 0) red[wv][c] = v;
  }
  __syncthreads();
  double* out = part + (size_t)blockIdx.x * kPst;
  if (tid < k) out[tid] = red[0][tid] + red[1][tid] + red[2][tid] + red[3][tid];
  if (tid == 0)
    out[k] = red[0][kNarrow] + red[1][kNarrow] + red[2][kNarrow] + red[3][kNarrow];
}

// mode 0: out_row = in_row U; mode 1: out_row = [in_row, s_row] U with
// s_row = (q1_row - in_row . p2) / rho (the new direction).  Rows are dense
// (ld_in = kin, ld_out = kout); a chunk of 256 rows is loaded contiguously,
// rotated one row per thread, and stored contiguously, all of its loads
// before any of its stores, so Phi_in may equal Phi_out.
template <typename T>
__global__ __launch_bounds__(256) void k_rotate_small(const Tile* __restrict__ tiles,
                                                      const int64_t* __restrict__ dof_off,
                                                      const T* Phi_in, int kin, T* Phi_out,
                                                      int kout, const double* __restrict__ U,
                                                      int ldu, size_t ustride, int mode,
                                                      const double* __restrict__ q1,
                                                      const double* __restrict__ pr, int ldpr,
                                                      const int32_t* __restrict__ enable) {
  __shared__ double sU[(kNarrow + 1) * kNarrow];
  __shared__ double sp[2 * kNarrow + 1];
  __shared__ T sIn[256 * kNarrow];
  __shared__ T sOut[256 * kNarrow];
  const Tile t = tiles[blockIdx.x];
  const int b = t.inst;
  if (enable && !enable[b]) return;
  const int tid = threadIdx.x;
  const int64_t base = dof_off[b];
  const double* Ub = U + (size_t)b * ustride;
  const int krow = mode == 1 ? kin + 1 : kin;
  for (int e = tid; e < krow * kout; e += blockDim.x) {
    const int c = e / kout, j = e % kout;
    sU[c * kNarrow + j] = Ub[c * ldu + j];
  }
  if (mode == 1)
    for (int c = tid; c <= 2 * kin; c += blockDim.x) sp[c] = pr[(size_t)b * ldpr + c];
  for (int64_t r0 = 0; r0 < t.ncell; r0 += 256) {
    const int nr = (int)(t.ncell - r0 < 256 ? t.ncell - r0 : 256);
    const int64_t g0 = base + t.cell0 + r0;
    __syncthreads();
    {
      T v[kNarrow];   // all loads of the chunk in flight before the LDS writes
#pragma unroll
      for (int u = 0; u < kNarrow; ++u)
        if (u * 256 + tid < nr * kin) v[u] = Phi_in[g0 * kin + u * 256 + tid];
#pragma unroll
      for (int u = 0; u < kNarrow; ++u)
        if (u * 256 + tid < nr * kin) sIn[u * 256 + tid] = v[u];
    }
    __syncthreads();
    if (tid < nr) {
      double row[kNarrow];
#pragma unroll
      for (int c = 0; c < kNarrow; ++c) row[c] = c < kin ? (double)sIn[tid * kin + c] : 0.0;
      double sv = 0.0;
      if (mode == 1) {
        double d2 = 0.0;
#pragma unroll
        for (int c = 0; c < kNarrow; ++c)
          if (c < kin) d2 += row[c] * sp[kin + c];
        sv = (q1[g0 + tid] - d2) * sp[2 * kin];
      }
#pragma unroll 1
      for (int j = 0; j < kout; ++j) {
        double acc = mode == 1 ? sv * sU[kin * kNarrow + j] : 0.0;
#pragma unroll
        for (int c = 0; c < kNarrow; ++c)
          if (c < kin) acc += row[c] * sU[c * kNarrow + j];
        sOut[tid * kout + j] = (T)acc;
      }
    }
    __syncthreads();
    for (int e = tid; e < nr * kout; e += 256) Phi_out[g0 * kout + e] = sOut[e];
  }
}

// Gram partials G = Phi^T Phi per tile (FP64), lane j accumulates column j.
template <typename T>
__global__ __launch_bounds__(256) void k_gram(const Tile* __restrict__ tiles,
                                              const int64_t* __restrict__ dof_off,
                                              const T* __restrict__ Phi, int r,
                                              double* __restrict__ part) {
  __shared__ T sP[kChunk][kMaxR + 1];
  __shared__ double red[4][kMaxR];
  const Tile t = tiles[blockIdx.x];
  const int b = t.inst, tid = threadIdx.x, lane = tid & 63, grp = tid >> 6;
  const int64_t base = dof_off[b];
  double acc[kMaxR];
#pragma unroll
  for (int c = 0; c < kMaxR; ++c) acc[c] = 0.0;
  for (int64_t r0 = 0; r0 < t.ncell; r0 += kChunk) {
    const int nr = (int)(t.ncell - r0 < kChunk ? t.ncell - r0 : kChunk);
    __syncthreads();
    for (int e = tid; e < nr * r; e += blockDim.x) {
      const int rr = e / r, c = e - rr * r;
      sP[rr][c] = Phi[(base + t.cell0 + r0 + rr) * r + c];
    }
    __syncthreads();
    if (lane < r) {
      for (int rr = grp; rr < nr; rr += 4) {
        const double pj = (double)sP[rr][lane];
#pragma unroll
        for (int c = 0; c < kMaxR; ++c)
          if (c < r) acc[c] += (double)sP[rr][c] * pj;
      }
    }
  }
  double* out = part + (size_t)blockIdx.x * (kMaxR * kMaxR);
#pragma unroll
  for (int c = 0; c < kMaxR; ++c) {
    if (c < r) {
      __syncthreads();
      if (lane < r) red[grp][lane] = acc[c];
      __syncthreads();
      if (tid < r) out[c * r + tid] = red[0][tid] + red[1][tid] + red[2][tid] + red[3][tid];
    }
  }
}

// Per instance: G = sum of partials; if max|G - I| > tau: Cholesky G = L L^T,
// store Linv^T (so that Phi <- Phi Linv^T) and a <- L^T a; enable[b] = 1.
__global__ __launch_bounds__(256) void k_reorth_decide(const int* __restrict__ tfirst,
                                                       const double* __restrict__ part, int r,
                                                       double tau, double* __restrict__ lmat,
                                                       double* __restrict__ a,
                                                       int32_t* __restrict__ enable,
                                                       uint32_t* flags) {
  __shared__ double G[kMaxR * kMaxR];
  __shared__ double Li[kMaxR * kMaxR];
  __shared__ double dev;
  __shared__ double ta[kMaxR];
  const int b = blockIdx.x, tid = threadIdx.x;
  for (int e = tid; e < r * r; e += blockDim.x) {
    double s = 0.0;
    for (int tt = tfirst[b]; tt < tfirst[b + 1]; ++tt) s += part[(size_t)tt * (kMaxR * kMaxR) + e];
    G[e] = s;
  }
  __syncthreads();
  if (tid == 0) {
    double m = 0.0;
    for (int i = 0; i < r; ++i)
      for (int j = 0; j < r; ++j) {
        const double v = fabs(G[i * r + j] - (i == j ? 1.0 : 0.0));
        m = v > m ? v : m;
      }
    dev = m;
  }
  __syncthreads();
  const bool go = dev > tau;
  if (tid == 0) enable[b] = go ? 1 : 0;
  if (!go) return;
  if (tid == 0) {
    atomicOr(&flags[b], ROM_FLAG_REORTH);
    // Cholesky in place (lower), G = L L^T
    for (int j = 0; j < r; ++j) {
      double s = G[j * r + j];
      for (int k = 0; k < j; ++k) s -= G[j * r + k] * G[j * r + k];
      const double d = sqrt(s > 0.0 ? s : 1e-300);
      G[j * r + j] = d;
      for (int i = j + 1; i < r; ++i) {
        double t2 = G[i * r + j];
        for (int k = 0; k < j; ++k) t2 -= G[i * r + k] * G[j * r + k];
        G[i * r + j] = t2 / d;
      }
      for (int k = j + 1; k < r; ++k) G[j * r + k] = 0.0;
    }
    // Li = L^{-1} (lower) by forward substitution on the identity
    for (int c = 0; c < r; ++c)
      for (int i = 0; i < r; ++i) {
        double s = (i == c) ? 1.0 : 0.0;
        for (int k = 0; k < i; ++k) s -= G[i * r + k] * Li[k * r + c];
        Li[i * r + c] = s / G[i * r + i];
      }
  }
  __syncthreads();
  // Phi_new = Phi Li^T : U[c][j] = Li[j][c]
  for (int e = tid; e < r * r; e += blockDim.x) {
    const int c = e / r, j = e % r;
    lmat[(size_t)b * r * r + c * r + j] = Li[j * r + c];
  }
  // a_new = L^T a
  for (int j = tid; j < r; j += blockDim.x) {
    double s = 0.0;
    for (int i = j; i < r; ++i) s += G[i * r + j] * a[(size_t)b * r + i];
    ta[j] = s;
  }
  __syncthreads();
  for (int j = tid; j < r; j += blockDim.x) a[(size_t)b * r + j] = ta[j];
}

// POD helpers -------------------------------------------------------------
// Column k of the CGS2 QR of X = D (Q_train - q_ref 1^T): red holds p1 (+ |x|^2)
// at [0..k] and p2 (+ |q1|^2) at [kMaxK+1 ..].  Writes R[0..k-1][k] = p and pr = p.
__global__ void k_pod_column(int k, int w, const double* __restrict__ red, int ldr,
                             double* __restrict__ R, double* __restrict__ pr, int ldpr) {
  const int b = blockIdx.x, tid = threadIdx.x;
  const double* X = red + (size_t)b * ldr;
  double* Rb = R + (size_t)b * w * w;
  for (int c = tid; c < k; c += blockDim.x) {
    Rb[c * w + k] = X[c] + X[kMaxK + 1 + c];
    pr[(size_t)b * ldpr + c] = X[c];
    pr[(size_t)b * ldpr + kMaxK + c] = X[kMaxK + 1 + c];
  }
}

// Q[:, k] = q1 - Q[:, :k] p2 with q1 the stored first-pass residual (x itself
// for k = 0), not yet normalised; per-tile partial of |q|^2.
// The norm is taken of the computed vector itself: with nearly dependent
// training columns, the Pythagorean |q1|^2 - |p2|^2 loses the orthonormality
// of Q and the error cascades into later columns.
template <typename T>
__global__ __launch_bounds__(256) void k_pod_write(const Tile* __restrict__ tiles,
                                                   const int64_t* __restrict__ dof_off, T* Q, int w,
                                                   int k, const T* __restrict__ y,
                                                   const T* __restrict__ qref,
                                                   const double* __restrict__ dvar, int nv,
                                                   const double* __restrict__ pr, int ldpr,
                                                   const double* __restrict__ q1,
                                                   double* __restrict__ part) {
  __shared__ double red[256];
  const Tile t = tiles[blockIdx.x];
  const int b = t.inst, tid = threadIdx.x;
  const int64_t base = dof_off[b];
  const double* p = pr + (size_t)b * ldpr;
  double acc = 0.0;
  for (int64_t rr = tid; rr < t.ncell; rr += blockDim.x) {
    const int64_t lr = t.cell0 + rr, g = base + lr;
    double v;
    if (k == 0) {
      v = qref ? yhat_of(y, qref, dvar + (size_t)b * nv, nv, g, lr) : (double)y[g];
    } else {
      double d2 = 0.0;
      for (int c = 0; c < k; ++c) d2 += (double)Q[g * w + c] * p[kMaxK + c];
      v = q1[g] - d2;
    }
    const T vt = (T)v;
    Q[g * w + k] = vt;
    acc += (double)vt * (double)vt;
  }
  red[tid] = acc;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (tid < st) red[tid] += red[tid + st];
    __syncthreads();
  }
  if (tid == 0) part[(size_t)blockIdx.x * kPst] = red[0];
}

// rho = |q| (from the reduced partials in red[b*ldr]); R[k][k] = rho; pr[kMaxK] = 1/rho
__global__ void k_pod_rho(int k, int w, const double* __restrict__ red, int ldr,
                          double* __restrict__ R, double* __restrict__ pr, int ldpr) {
  const int b = blockIdx.x;
  if (threadIdx.x != 0) return;
  const double rho = sqrt(red[(size_t)b * ldr]);
  R[(size_t)b * w * w + k * w + k] = rho;
  pr[(size_t)b * ldpr + 2 * kMaxK] = rho > 0.0 ? 1.0 / rho : 0.0;
}

template <typename T>
__global__ __launch_bounds__(256) void k_pod_scale(const Tile* __restrict__ tiles,
                                                   const int64_t* __restrict__ dof_off, T* Q, int w,
                                                   int k, const double* __restrict__ pr, int ldpr) {
  const Tile t = tiles[blockIdx.x];
  const int b = t.inst;
  const double s = pr[(size_t)b * ldpr + 2 * kMaxK];
  const int64_t base = dof_off[b];
  for (int64_t rr = threadIdx.x; rr < t.ncell; rr += blockDim.x) {
    const int64_t g = base + t.cell0 + rr;
    Q[g * w + k] = (T)((double)Q[g * w + k] * s);
  }
}

__global__ __launch_bounds__(64) void k_pod_svd(int w, int r, const double* __restrict__ R,
                                                double* __restrict__ U, double* __restrict__ sigma,
                                                int use_lds) {
  extern __shared__ double sm[];
  const int b = blockIdx.x, tid = threadIdx.x;
  const int n = w, ld = w;
  double* K = sm;
  double* G = K + n * ld;
  double* nrm = G + n * ld;
  double* sv = nrm + n;
  int* rank = (int*)(sv + n);
  for (int e = tid; e < n * n; e += blockDim.x) K[e] = R[(size_t)b * n * n + e];
  __syncthreads();
  jacobi_rows(K, G, n, ld, U + (size_t)b * n * n, sv, nrm, rank);
  for (int c = tid; c < r; c += blockDim.x) sigma[(size_t)b * r + c] = sv[c];
  (void)use_lds;
}

// The small matrices of the POD's backward pass (see rollout.hip), one
// wavefront per instance: the SVD of R again (the same kernel path as the
// forward, so U_R and the singular values are the forward's), then
// V = R^T U_R S^-1, Mm = U_R^T Z (Z = Q_pod^T Phibar, w x r),
// G = F o (Mm_pad - Mm_pad^T) S + diag(sbar_pad), C = U_R G V^T - Z S_r^-1 V_r^T
// and E = S_r^-1 V_r^T.  Zero singular values carry no gradient.
// scr: [B][3 w w] global scratch (U_R, V, G V^T).
__global__ __launch_bounds__(64) void k_pod_vjp_small(int w, int r, const double* __restrict__ R,
                                                      const double* __restrict__ Z,
                                                      const double* __restrict__ sigbar,
                                                      double* __restrict__ Cm,
                                                      double* __restrict__ Em,
                                                      double* __restrict__ scr) {
  extern __shared__ double sm[];
  const int b = blockIdx.x, tid = threadIdx.x;
  const int n = w, ld = w;
  double* K = sm;
  double* G = K + n * ld;
  double* nrm = G + n * ld;
  double* sv = nrm + n;
  int* rank = (int*)(sv + n);
  double* U = scr + (size_t)b * 3 * w * w;
  double* V = U + w * w;
  double* GV = V + w * w;
  const double* Rb = R + (size_t)b * w * w;
  const double* Zb = Z + (size_t)b * w * r;
  for (int e = tid; e < n * n; e += blockDim.x) K[e] = Rb[e];
  __syncthreads();
  jacobi_rows(K, G, n, ld, U, sv, nrm, rank);
  __threadfence_block();
  __syncthreads();
  auto inv = [&](int j) { return sv[j] > 0.0 ? 1.0 / sv[j] : 0.0; };
  // V[i][j] = sum_k R[k][i] U[k][j] / s_j
  for (int e = tid; e < w * w; e += blockDim.x) {
    const int i = e / w, j = e % w;
    double acc = 0.0;
    for (int k = 0; k < w; ++k) acc += Rb[k * w + i] * U[k * w + j];
    V[e] = acc * inv(j);
  }
  // G (into K): Mm_ij = (U^T Z)_ij for j < r
  for (int e = tid; e < w * w; e += blockDim.x) {
    const int i = e / w, j = e % w;
    double g = 0.0;
    if (i == j) {
      g = i < r ? sigbar[(size_t)b * r + i] : 0.0;
    } else {
      double mij = 0.0, mji = 0.0;
      if (j < r)
        for (int k = 0; k < w; ++k) mij += U[k * w + i] * Zb[k * r + j];
      if (i < r)
        for (int k = 0; k < w; ++k) mji += U[k * w + j] * Zb[k * r + i];
      const double den = sv[j] * sv[j] - sv[i] * sv[i];
      if (sv[j] > 0.0 && den != 0.0) g = (mij - mji) * sv[j] / den;
    }
    K[e] = g;
  }
  __threadfence_block();
  __syncthreads();
  // GV = G V^T
  for (int e = tid; e < w * w; e += blockDim.x) {
    const int i = e / w, j = e % w;
    double acc = 0.0;
    for (int l = 0; l < w; ++l) acc += K[i * w + l] * V[j * w + l];
    GV[e] = acc;
  }
  __threadfence_block();
  __syncthreads();
  // C = U_R GV - Z S_r^-1 V_r^T; E = S_r^-1 V_r^T
  double* Cb = Cm + (size_t)b * w * w;
  for (int e = tid; e < w * w; e += blockDim.x) {
    const int k = e / w, j = e % w;
    double acc = 0.0;
    for (int i = 0; i < w; ++i) acc += U[k * w + i] * GV[i * w + j];
    double t = 0.0;
    for (int c = 0; c < r; ++c) t += Zb[k * r + c] * V[j * w + c] * inv(c);
    Cb[e] = acc - t;
  }
  double* Eb = Em + (size_t)b * r * w;
  for (int e = tid; e < r * w; e += blockDim.x) {
    const int c = e / w, j = e % w;
    Eb[e] = V[j * w + c] * inv(c);
  }
}

// preprocessing: sum over cells and snapshots of (Q - q_ref)^2 per variable
template <typename T>
__global__ __launch_bounds__(256) void k_sqdev(const Tile* __restrict__ tiles,
                                               const int64_t* __restrict__ dof_off,
                                               const T* __restrict__ Q, int w, int64_t total,
                                               const T* __restrict__ qref, int nv,
                                               double* __restrict__ part) {
  __shared__ double red[256][12];
  const Tile t = tiles[blockIdx.x];
  const int b = t.inst, tid = threadIdx.x;
  const int64_t base = dof_off[b];
  double acc[12];
  for (int v = 0; v < 12; ++v) acc[v] = 0.0;
  for (int64_t rr = tid; rr < t.ncell; rr += blockDim.x) {
    const int64_t lr = t.cell0 + rr, g = base + lr;
    const double q0 = (double)qref[g];
    double s = 0.0;
    for (int j = 0; j < w; ++j) {
      const double d = (double)Q[(size_t)j * total + g] - q0;
      s += d * d;
    }
    const int v = (int)(lr % nv);
    for (int u = 0; u < 12; ++u) acc[u] += (u == v) ? s : 0.0;
  }
  for (int v = 0; v < nv; ++v) red[tid][v] = acc[v];
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (tid < st)
      for (int v = 0; v < nv; ++v) red[tid][v] += red[tid + st][v];
    __syncthreads();
  }
  if (tid < nv) part[(size_t)blockIdx.x * kPst + tid] = red[0][tid];
}

__global__ void k_dvar(const int* __restrict__ tfirst, const double* __restrict__ part, int nv,
                       const int64_t* __restrict__ cell_off, int w, double* __restrict__ dvar) {
  const int b = blockIdx.x;
  const int v = threadIdx.x;
  if (v >= nv) return;
  double s = 0.0;
  for (int tt = tfirst[b]; tt < tfirst[b + 1]; ++tt) s += part[(size_t)tt * kPst + v];
  const double cnt = (double)(cell_off[b + 1] - cell_off[b]) * (double)w;
  const double phi = s / cnt;
  dvar[(size_t)b * nv + v] = phi == 0.0 ? 1.0 : 1.0 / phi;
}

// Phi_out = [Phi_in (, new direction)] U over the pass tiles: the narrow kernel
// when every dimension fits in registers, the generic one otherwise
template <typename T>
void rotate_t(rom_batch* h, const T* Phi_in, int ld_in, int kin, T* Phi_out, int ld_out, int kout,
              const double* U, int ldu, size_t ustride, int mode, const double* q1,
              const double* pr, int ldpr, const int32_t* enable, hipStream_t s) {
  if (kin <= kNarrow && kout <= kNarrow && ld_in == kin && ld_out == kout)
    hipLaunchKernelGGL((k_rotate_small<T>), dim3(h->n_ptiles), dim3(256), 0, s, h->d_ptiles,
                       h->d_dof_off, Phi_in, kin, Phi_out, kout, U, ldu, ustride, mode, q1, pr,
                       ldpr, enable);
  else {
    const int split = std::max(1, std::min(8, 2 * h->n_cu / std::max(h->n_ptiles, 1)));
    hipLaunchKernelGGL((k_rotate<T>), dim3(h->n_ptiles * split), dim3(256), 0, s, h->d_ptiles,
                       h->d_dof_off, Phi_in, ld_in, kin, Phi_out, ld_out, kout, U, ldu, ustride,
                       mode, q1, pr, ldpr, enable, split);
  }
}

template <typename T>
rom_status project_t(rom_batch* h, const void* Phi, int ld, int k, const void* y, const void* qref,
                     const double* p1, int ldp, int mode, double* dst, int ldd, hipStream_t s,
                     double* q1out = nullptr) {
  if (k <= kNarrow)
    hipLaunchKernelGGL((k_project_small<T>), dim3(h->n_ptiles), dim3(256), 0, s, h->d_ptiles,
                       h->d_dof_off, (const T*)Phi, ld, k, (const T*)y, (const T*)qref, h->d_var,
                       h->nv, p1, ldp, mode, h->part, q1out);
  int split = 1;
  if (k > kNarrow) {
    split = std::max(1, std::min(8, 2 * h->n_cu / std::max(h->n_ptiles, 1)));
    hipLaunchKernelGGL((k_project<T>), dim3(h->n_ptiles * split), dim3(256), 0, s, h->d_ptiles,
                       h->d_dof_off, (const T*)Phi, ld, k, (const T*)y, (const T*)qref, h->d_var,
                       h->nv, p1, ldp, mode, h->part, q1out, split);
  }
  hipLaunchKernelGGL(k_reduce_tiles, dim3(h->cfg.n_inst), dim3(128), 0, s, h->d_ptile_first,
                     h->part, k, dst, ldd, split);
  return ROM_OK;
}

// pass A / pass B of the projection, through the fast kernel when it applies;
// the fast kernel's per-tile partials go to part (h->part when null), the
// generic kernel always uses h->part
template <typename T>
rom_status projection_pass(rom_batch* h, const void* y, const double* p1, int ldp, int mode,
                           double* dst, int ldd, double* q1out, hipStream_t s,
                           double* part = nullptr) {
  const int r = h->cfg.r;
  if (mfma_ok(h)) {
    double* pp = part ? part : h->part;
    rom_status st = launch_project_fast(h, y, p1, ldp, mode, pp, kPst, q1out, s);
    if (st != ROM_OK) return st;
    hipLaunchKernelGGL(k_reduce_tiles, dim3(h->cfg.n_inst), dim3(128), 0, s, h->d_ptile_first,
                       pp, r, dst, ldd, 1);
    return ROM_OK;
  }
  return project_t<T>(h, h->Phi, r, r, y, h->q_ref, p1, ldp, mode, dst, ldd, s, q1out);
}

// Projections and core SVD of one iSVD update (Alg. 2): reads Phi and y,
// writes sigma, Ubar and (p1, p2, 1/rho); a and Phi are left alone.
template <typename T>
rom_status isvd_core_t(rom_batch* h, const void* y, double* part, hipStream_t s) {
  const int r = h->cfg.r, B = h->cfg.n_inst;
  const int ldr = 2 * r + 4;
  double* red = h->red;
  // pass A: p1 = Phi^T y^, |y^|^2 ; pass B: p2 = Phi^T q1, |q1|^2 (q1 stored)
  rom_status st = projection_pass<T>(h, y, nullptr, 0, 1, red, ldr, nullptr, s, part);
  if (st != ROM_OK) return st;
  st = projection_pass<T>(h, y, red, ldr, 2, red + r + 1, ldr, h->qtmp, s, part);
  if (st != ROM_OK) return st;
  const int n = r + 1;
  const size_t shm = sizeof(double) * (2 * n * n + 3 * n) + sizeof(int) * n;
  double* pr = h->rstate;  // (p1, p2, 1/rho) per instance, stride 2r + 2
  // the arrowhead path adds 13 N doubles and 8 N + 3 ints of workspace
  const size_t shm_arrow = shm + sizeof(double) * (13 * n + 2) + sizeof(int) * (8 * n + 3 + 2);
  (void)shm;
  hipLaunchKernelGGL(k_isvd_core<true>, dim3(B), dim3(64), shm_arrow, s, r, h->cfg.lambda,
                     h->cfg.tau_rho, red, ldr, h->sigma, h->ubar, pr, h->flags);
  ROM_HIP_CHECK(hipGetLastError());
  return ROM_OK;
}

// The rest of the update: the closed-form transfer of a, then the rotation of
// Phi by Ubar (with the new direction).
template <typename T>
rom_status isvd_apply_t(rom_batch* h, hipStream_t s) {
  const int r = h->cfg.r, B = h->cfg.n_inst, n = r + 1;
  double* pr = h->rstate;
  hipLaunchKernelGGL(k_isvd_transfer, dim3(B), dim3(64), 0, s, r, h->ubar, h->a);
  if (mfma_ok(h)) return launch_rotate_mfma(h, pr, h->Phi, s);
  rotate_t<T>(h, (const T*)h->Phi, r, r, (T*)h->Phi, r, r, h->ubar, n, (size_t)n * n, 1,
              h->qtmp, pr, 2 * r + 2, nullptr, s);
  ROM_HIP_CHECK(hipGetLastError());
  return ROM_OK;
}

template <typename T>
rom_status isvd_t(rom_batch* h, const void* y, hipStream_t s) {
  rom_status st = isvd_core_t<T>(h, y, h->part, s);
  if (st != ROM_OK) return st;
  return isvd_apply_t<T>(h, s);
}

template <typename T>
rom_status reorth_t(rom_batch* h, hipStream_t s) {
  const int r = h->cfg.r, B = h->cfg.n_inst;
  hipLaunchKernelGGL((k_gram<T>), dim3(h->n_ptiles), dim3(256), 0, s, h->d_ptiles, h->d_dof_off,
                     (const T*)h->Phi, r, h->part);
  hipLaunchKernelGGL(k_reorth_decide, dim3(B), dim3(256), 0, s, h->d_ptile_first, h->part, r,
                     h->cfg.tau_orth, h->lmat, h->a, h->active, h->flags);
  rotate_t<T>(h, (const T*)h->Phi, r, r, (T*)h->Phi, r, r, h->lmat, r, (size_t)r * r, 0,
              nullptr, nullptr, 0, h->active, s);
  ROM_HIP_CHECK(hipGetLastError());
  return ROM_OK;
}

}  // namespace

rom_status pod_ws_alloc(rom_batch* h, int wmax, PodWs* ws) {
  const size_t B = h->cfg.n_inst;
  *ws = PodWs{};
  ws->wmax = wmax;
  const size_t ldr = 2 * kMaxK + 4, ldpr = 2 * kMaxK + 2;
  if (hipMalloc(&ws->Q, h->esz * (size_t)h->total_dof * wmax) != hipSuccess ||
      hipMalloc((void**)&ws->R, sizeof(double) * B * wmax * wmax) != hipSuccess ||
      hipMalloc((void**)&ws->U, sizeof(double) * B * wmax * wmax) != hipSuccess ||
      hipMalloc((void**)&ws->red, sizeof(double) * B * ldr) != hipSuccess ||
      hipMalloc((void**)&ws->pr, sizeof(double) * B * ldpr) != hipSuccess) {
    pod_ws_free(ws);
    set_error("hipMalloc failed (thin-SVD workspace)");
    return ROM_E_NOMEM;
  }
  return ROM_OK;
}

void pod_ws_free(PodWs* ws) {
  (void)hipFree(ws->Q);
  (void)hipFree(ws->R);
  (void)hipFree(ws->U);
  (void)hipFree(ws->red);
  (void)hipFree(ws->pr);
  *ws = PodWs{};
}

namespace {

template <typename T>
__global__ __launch_bounds__(256) void k_copy_t(const T* __restrict__ src, T* __restrict__ dst,
                                                int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

// Left singular vectors of a batch of N x w column matrices by CGS2-QR (FP64
// norms and the stored first-pass residual), then the Jacobi SVD of R and
// the rotation Q U[:, :r] into phi_out, leading singular values into sigma_out
// (reading R1).  Without svd (w == r) the Gram-Schmidt basis Q itself is the
// result (R has a positive diagonal).  cols: T[w * total_dof], column j of every instance at
// j * total_dof + dof_off[b]; with pre the columns are preprocessed on the
// fly (D (y - q_ref)), otherwise taken as they are.  Kernels only (no
// allocation, no memset, no synchronisation): usable inside a captured graph.
template <typename T>
rom_status pod_core_t(rom_batch* h, const void* cols, int w, bool pre, bool svd, const PodWs& ws,
                      double* sigma_out, void* phi_out, hipStream_t s) {
  const int r = h->cfg.r, B = h->cfg.n_inst;
  const int64_t tot = h->total_dof;
  T* Q = (T*)ws.Q;
  double* R = ws.R;
  double* U = ws.U;
  double* redp = ws.red;
  double* prp = ws.pr;
  const int ldr = 2 * kMaxK + 4;
  const T* qref = pre ? (const T*)h->q_ref : nullptr;
  ROM_TRY(fill_zero(R, sizeof(double) * B * w * w, s));
  for (int k = 0; k < w; ++k) {
    const T* yk = (const T*)cols + (size_t)k * tot;
    if (k > 0) {
      project_t<T>(h, Q, w, k, yk, qref, nullptr, 0, 1, redp, ldr, s);
      project_t<T>(h, Q, w, k, yk, qref, redp, ldr, 2, redp + kMaxK + 1, ldr, s, h->qtmp);
    } else {
      project_t<T>(h, Q, w, 0, yk, qref, nullptr, 0, 1, redp, ldr, s);
    }
    hipLaunchKernelGGL(k_pod_column, dim3(B), dim3(128), 0, s, k, w, redp, ldr, R, prp,
                       2 * kMaxK + 2);
    hipLaunchKernelGGL((k_pod_write<T>), dim3(h->n_ptiles), dim3(256), 0, s, h->d_ptiles,
                       h->d_dof_off, Q, w, k, yk, qref, h->d_var, h->nv, prp,
                       2 * kMaxK + 2, h->qtmp, h->part);
    hipLaunchKernelGGL(k_reduce_tiles, dim3(B), dim3(128), 0, s, h->d_ptile_first, h->part, 0,
                       redp, ldr, 1);
    hipLaunchKernelGGL(k_pod_rho, dim3(B), dim3(64), 0, s, k, w, redp, ldr, R, prp, 2 * kMaxK + 2);
    hipLaunchKernelGGL((k_pod_scale<T>), dim3(h->n_ptiles), dim3(256), 0, s, h->d_ptiles,
                       h->d_dof_off, Q, w, k, prp, 2 * kMaxK + 2);
  }
  if (!svd) {   // the Gram-Schmidt basis itself (w == r columns, same row layout)
    hipLaunchKernelGGL((k_copy_t<T>), dim3((unsigned)((tot * w + 255) / 256)), dim3(256), 0, s,
                       (const T*)Q, (T*)phi_out, tot * w);
    ROM_HIP_CHECK(hipGetLastError());
    return ROM_OK;
  }
  const size_t shm = sizeof(double) * (2 * w * w + 2 * w) + sizeof(int) * w;
  hipLaunchKernelGGL(k_pod_svd, dim3(B), dim3(64), shm, s, w, r, R, U, sigma_out, 1);
  rotate_t<T>(h, (const T*)Q, w, w, (T*)phi_out, r, r, U, w, (size_t)w * w, 0, nullptr,
              nullptr, 0, nullptr, s);
  ROM_HIP_CHECK(hipGetLastError());
  return ROM_OK;
}

// ------------------------------------------------------------------ windowed rules
// (App. A: the windowed SVD of Alg. A.1 and the Direct rule of Alg. A.2)
constexpr int kMaxWin = 64;   // widest snapshot window

// v = Phi a in FP64, row by row (the lifted state before the basis changes)
template <typename T>
__global__ __launch_bounds__(256) void k_lift(const Tile* __restrict__ tiles,
                                              const int64_t* __restrict__ dof_off,
                                              const T* __restrict__ Phi, int r,
                                              const double* __restrict__ a,
                                              double* __restrict__ v) {
  const Tile t = tiles[blockIdx.x];
  const int b = t.inst;
  const int64_t base = dof_off[b];
  const double* ab = a + (size_t)b * r;
  for (int64_t rr = threadIdx.x; rr < t.ncell; rr += blockDim.x) {
    const int64_t g = base + t.cell0 + rr;
    double s = 0.0;
    for (int c = 0; c < r; ++c) s += (double)Phi[g * r + c] * ab[c];
    v[g] = s;
  }
}

// per-tile partials of Phi^T v (v FP64), same lane layout and summation order
// as the projection pass: four row groups, lanes over columns
template <typename T>
__global__ __launch_bounds__(256) void k_project_vec(const Tile* __restrict__ tiles,
                                                     const int64_t* __restrict__ dof_off,
                                                     const T* __restrict__ Phi, int r,
                                                     const double* __restrict__ v,
                                                     double* __restrict__ part) {
  __shared__ double red[4][kMaxR];
  const Tile t = tiles[blockIdx.x];
  const int b = t.inst, tid = threadIdx.x, lane = tid & 63, grp = tid >> 6;
  const int64_t base = dof_off[b];
  double acc = 0.0;
  for (int64_t rr = grp; rr < t.ncell; rr += 4) {
    const int64_t g = base + t.cell0 + rr;
    if (lane < r) acc += (double)Phi[g * r + lane] * v[g];
  }
  if (lane < r) red[grp][lane] = acc;
  __syncthreads();
  for (int c = tid; c < r; c += blockDim.x)
    part[(size_t)blockIdx.x * kPst + c] = red[0][c] + red[1][c] + red[2][c] + red[3][c];
}

// Z^+ (m x r) of Z = Phi^T Y (r x m, column j of instance b at
// Z[(b * ldz + j) * (r + 1) + c]) by one-sided Jacobi on the rows of the
// zero-padded m x m matrix [Z; 0]: after the sweeps G [Z; 0] has orthogonal
// rows g_i with norms s_i, and Z^+ = sum_i g_i^T G[i, :r] / s_i^2 over the
// values above 1e-15 of the largest.  One wavefront per instance.
__global__ __launch_bounds__(64) void k_direct_pinv(int r, int m, const double* __restrict__ Z,
                                                    int ldz, double* __restrict__ Zp,
                                                    double* __restrict__ Uscr) {
  extern __shared__ double sm[];
  const int b = blockIdx.x, tid = threadIdx.x, n = m, ld = m;
  double* K = sm;
  double* G = K + n * ld;
  double* nrm = G + n * ld;
  double* sv = nrm + n;
  int* rank = (int*)(sv + n);
  for (int e = tid; e < n * ld; e += 64) {
    const int i = e / ld, j = e % ld;
    K[e] = i < r ? Z[((size_t)b * ldz + j) * (r + 1) + i] : 0.0;
  }
  __syncthreads();
  jacobi_rows(K, G, n, ld, Uscr + (size_t)b * n * n, sv, nrm, rank);
  double smax = 0.0;
  for (int i = 0; i < n; ++i) smax = fmax(smax, nrm[i]);
  const double cut = 1e-15 * smax;
  for (int e = tid; e < m * r; e += 64) {
    const int j = e / r, c = e % r;
    double acc = 0.0;
    for (int i = 0; i < n; ++i)
      if (nrm[i] > cut) acc += K[i * ld + j] * G[i * ld + c] / (nrm[i] * nrm[i]);
    Zp[((size_t)b * ldz + j) * r + c] = acc;
  }
}

// Phi~ = Y Z^+ with Y the preprocessed window (slot j of instance b's rows at
// j * total + g), written column-major: out[c * total + g]
template <typename T>
__global__ __launch_bounds__(256) void k_direct_combine(
    const Tile* __restrict__ tiles, const int64_t* __restrict__ dof_off,
    const T* __restrict__ win, int64_t total, int m, const T* __restrict__ qref,
    const double* __restrict__ dvar, int nv, const double* __restrict__ Zp, int ldz, int r,
    T* __restrict__ out) {
  const Tile t = tiles[blockIdx.x];
  const int b = t.inst;
  const int64_t base = dof_off[b];
  const double* Zb = Zp + (size_t)b * ldz * r;
  for (int64_t rr = threadIdx.x; rr < t.ncell; rr += blockDim.x) {
    const int64_t lr = t.cell0 + rr, g = base + lr;
    double yh[kMaxWin];
#pragma unroll
    for (int j = 0; j < kMaxWin; ++j)
      yh[j] = j < m ? yhat_of(win + (size_t)j * total, qref, dvar + (size_t)b * nv, nv, g, lr)
                    : 0.0;
    for (int c = 0; c < r; ++c) {
      double acc = 0.0;
#pragma unroll
      for (int j = 0; j < kMaxWin; ++j)
        if (j < m) acc += yh[j] * Zb[j * r + c];
      out[(size_t)c * total + g] = (T)acc;
    }
  }
}

template <typename T>
rom_status pod_t(rom_batch* h, const void* Qtrain, int w, hipStream_t s) {
  PodWs ws;
  rom_status st = pod_ws_alloc(h, w, &ws);
  if (st == ROM_OK) st = pod_core_t<T>(h, Qtrain, w, true, true, ws, h->sigma, h->Phi, s);
  hipError_t e = hipStreamSynchronize(s);
  pod_ws_free(&ws);
  if (st != ROM_OK) return st;
  ROM_HIP_CHECK(e);
  return ROM_OK;
}

}  // namespace

rom_status launch_pod_ws(rom_batch* h, const void* Q, int w, const PodWs& ws, hipStream_t s) {
  if (h->cfg.precision == ROM_F64)
    return pod_core_t<double>(h, Q, w, true, true, ws, h->sigma, h->Phi, s);
  return pod_core_t<float>(h, Q, w, true, true, ws, h->sigma, h->Phi, s);
}

rom_status launch_pod_vjp_small(rom_batch* h, const double* R, int w, const double* Z,
                                const double* sigbar, double* Cm, double* Em, double* scr,
                                hipStream_t s) {
  const size_t shm = sizeof(double) * (2 * w * w + 2 * w) + sizeof(int) * w;
  hipLaunchKernelGGL(k_pod_vjp_small, dim3(h->cfg.n_inst), dim3(64), shm, s, w, h->cfg.r, R, Z,
                     sigbar, Cm, Em, scr);
  ROM_HIP_CHECK(hipGetLastError());
  return ROM_OK;
}

namespace {

// One windowed basis update (App. A): the raw snapshot y joins the window
// (replacing the oldest once it holds `window`), the lifted state v = Phi a is
// kept in FP64, the basis is rebuilt by the rule, and a = Phi_new^T v.
template <typename T>
rom_status windowed_t(rom_batch* h, const void* y, hipStream_t s) {
  const int r = h->cfg.r, B = h->cfg.n_inst, w = h->cfg.window;
  const int64_t tot = h->total_dof;
  T* win = (T*)h->win;
  hipLaunchKernelGGL((k_copy_t<T>), dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s,
                     (const T*)y, win + (size_t)h->win_head * tot, tot);
  h->win_head = (h->win_head + 1) % w;
  h->win_count = h->win_count < w ? h->win_count + 1 : w;
  const int m = h->win_count;
  hipLaunchKernelGGL((k_lift<T>), dim3(h->n_ptiles), dim3(256), 0, s, h->d_ptiles,
                     h->d_dof_off, (const T*)h->Phi, r, h->a, h->lift);
  if (h->cfg.update_rule == ROM_UPDATE_WSVD) {
    ROM_TRY(pod_core_t<T>(h, win, m, true, true, h->podws, h->sigma, h->Phi, s));
  } else {
    const int ldz = kMaxWin;
    for (int j = 0; j < m; ++j)
      project_t<T>(h, h->Phi, r, r, win + (size_t)j * tot, h->q_ref, nullptr, 0, 1,
                   h->zmat + (size_t)j * (r + 1), ldz * (r + 1), s);
    const size_t shm = sizeof(double) * (2 * m * m + 2 * m) + sizeof(int) * m;
    hipLaunchKernelGGL(k_direct_pinv, dim3(B), dim3(64), shm, s, r, m, h->zmat, ldz, h->zpinv,
                       h->podws.U);
    hipLaunchKernelGGL((k_direct_combine<T>), dim3(h->n_ptiles), dim3(256), 0, s, h->d_ptiles,
                       h->d_dof_off, (const T*)win, tot, m, (const T*)h->q_ref, h->d_var, h->nv,
                       h->zpinv, ldz, r, (T*)h->phit);
    ROM_TRY(pod_core_t<T>(h, h->phit, r, false, false, h->podws, h->sig_scratch, h->Phi, s));
  }
  hipLaunchKernelGGL((k_project_vec<T>), dim3(h->n_ptiles), dim3(256), 0, s, h->d_ptiles,
                     h->d_dof_off, (const T*)h->Phi, r, h->lift, h->part);
  hipLaunchKernelGGL(k_reduce_tiles, dim3(B), dim3(128), 0, s, h->d_ptile_first, h->part, r - 1,
                     h->a, r, 1);
  ROM_HIP_CHECK(hipGetLastError());
  return ROM_OK;
}

// The window at the end of the offline stage: the last min(window, w) training
// snapshots (Q: T[w * total_dof]), oldest first.
template <typename T>
rom_status window_init_t(rom_batch* h, const void* Q, int w, hipStream_t s) {
  const int64_t tot = h->total_dof;
  const int m = std::min(h->cfg.window, w);
  const T* src = (const T*)Q + (size_t)(w - m) * tot;
  hipLaunchKernelGGL((k_copy_t<T>), dim3((unsigned)((tot * m + 255) / 256)), dim3(256), 0, s, src,
                     (T*)h->win, tot * m);
  h->win_count = m;
  h->win_head = m % h->cfg.window;
  ROM_HIP_CHECK(hipGetLastError());
  return ROM_OK;
}

template <typename T>
rom_status preprocess_t(rom_batch* h, const void* q0, const void* Qtrain, int w, hipStream_t s) {
  ROM_HIP_CHECK(hipMemcpyAsync(h->q_ref, q0, sizeof(T) * h->total_dof, hipMemcpyDeviceToDevice, s));
  hipLaunchKernelGGL((k_sqdev<T>), dim3(h->n_ptiles), dim3(256), 0, s, h->d_ptiles, h->d_dof_off,
                     (const T*)Qtrain, w, h->total_dof, (const T*)h->q_ref, h->nv, h->part);
  hipLaunchKernelGGL(k_dvar, dim3(h->cfg.n_inst), dim3(64), 0, s, h->d_ptile_first, h->part,
                     h->nv, h->d_cell_off, w, h->d_var);
  ROM_HIP_CHECK(hipGetLastError());
  return ROM_OK;
}

__global__ void k_copy_cols(const double* src, int lds, int k, double* dst) {
  const int b = blockIdx.x;
  for (int c = threadIdx.x; c < k; c += blockDim.x) dst[(size_t)b * k + c] = src[(size_t)b * lds + c];
}

template <typename T>
rom_status project_state_t(rom_batch* h, const void* q, hipStream_t s) {
  const int r = h->cfg.r;
  // a[b*r + c] = Phi^T D (q - q_ref); the squared norm lands in red scratch
  rom_status st = projection_pass<T>(h, q, nullptr, 0, 1, h->red, 2 * r + 4, nullptr, s);
  if (st != ROM_OK) return st;
  hipLaunchKernelGGL(k_copy_cols, dim3(h->cfg.n_inst), dim3(64), 0, s, h->red, 2 * r + 4, r, h->a);
  return ROM_OK;
}

}  // namespace

rom_status isvd_kernels_prepare() {
  const int big = 160 * 1024 - 1024;
  ROM_HIP_CHECK(hipFuncSetAttribute((const void*)k_isvd_core<true>, hipFuncAttributeMaxDynamicSharedMemorySize, big));
  ROM_HIP_CHECK(hipFuncSetAttribute((const void*)k_pod_svd, hipFuncAttributeMaxDynamicSharedMemorySize, big));
  ROM_HIP_CHECK(hipFuncSetAttribute((const void*)k_pod_vjp_small, hipFuncAttributeMaxDynamicSharedMemorySize, big));
  ROM_HIP_CHECK(hipFuncSetAttribute((const void*)k_direct_pinv, hipFuncAttributeMaxDynamicSharedMemorySize, big));
  return ROM_OK;
}

rom_status launch_isvd(rom_batch* h, const void* y, hipStream_t s) {
  return h->cfg.precision == ROM_F64 ? isvd_t<double>(h, y, s) : isvd_t<float>(h, y, s);
}
rom_status launch_isvd_core(rom_batch* h, const void* y, double* part, hipStream_t s) {
  return h->cfg.precision == ROM_F64 ? isvd_core_t<double>(h, y, part, s)
                                     : isvd_core_t<float>(h, y, part, s);
}
rom_status launch_isvd_apply(rom_batch* h, hipStream_t s) {
  return h->cfg.precision == ROM_F64 ? isvd_apply_t<double>(h, s) : isvd_apply_t<float>(h, s);
}
// The two halves of launch_isvd_apply for the overlapped window (MFMA path):
// the rotation of the current basis into dst, and the state transfer.
rom_status launch_isvd_rotate_into(rom_batch* h, void* dst, hipStream_t s) {
  if (!mfma_ok(h)) {
    set_error("the rotation into a second buffer needs the MFMA path");
    return ROM_E_UNSUPPORTED;
  }
  return launch_rotate_mfma(h, h->rstate, dst, s);
}
rom_status launch_isvd_transfer(rom_batch* h, hipStream_t s) {
  hipLaunchKernelGGL(k_isvd_transfer, dim3(h->cfg.n_inst), dim3(64), 0, s, h->cfg.r, h->ubar, h->a);
  ROM_HIP_CHECK(hipGetLastError());
  return ROM_OK;
}
rom_status launch_isvd_project(rom_batch* h, const void* y, hipStream_t s) {
  const int r = h->cfg.r;
  return h->cfg.precision == ROM_F64
             ? projection_pass<double>(h, y, nullptr, 0, 1, h->red, 2 * r + 4, nullptr, s)
             : projection_pass<float>(h, y, nullptr, 0, 1, h->red, 2 * r + 4, nullptr, s);
}

rom_status launch_reorth(rom_batch* h, hipStream_t s) {
  return h->cfg.precision == ROM_F64 ? reorth_t<double>(h, s) : reorth_t<float>(h, s);
}
rom_status launch_pod(rom_batch* h, const void* Q, int w, hipStream_t s) {
  return h->cfg.precision == ROM_F64 ? pod_t<double>(h, Q, w, s) : pod_t<float>(h, Q, w, s);
}
rom_status launch_preprocess(rom_batch* h, const void* q0, const void* Q, int w, hipStream_t s) {
  return h->cfg.precision == ROM_F64 ? preprocess_t<double>(h, q0, Q, w, s)
                                     : preprocess_t<float>(h, q0, Q, w, s);
}
rom_status launch_windowed_update(rom_batch* h, const void* y, hipStream_t s) {
  return h->cfg.precision == ROM_F64 ? windowed_t<double>(h, y, s) : windowed_t<float>(h, y, s);
}
rom_status launch_window_init(rom_batch* h, const void* Q, int w, hipStream_t s) {
  return h->cfg.precision == ROM_F64 ? window_init_t<double>(h, Q, w, s)
                                     : window_init_t<float>(h, Q, w, s);
}
rom_status launch_project_state(rom_batch* h, const void* q, hipStream_t s) {
  return h->cfg.precision == ROM_F64 ? project_state_t<double>(h, q, s)
                                     : project_state_t<float>(h, q, s);
}

}  // namespace romhip
