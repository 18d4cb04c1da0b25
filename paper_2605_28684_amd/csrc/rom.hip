// Reduced steps, sampling and rebuild.
//
//  * Galerkin backward-Euler step (eq. galerkin_continuous_rom discretised by
//    backward Euler): Newton on g(a) = a - a_prev - dt Phi^T D f(q~(a)) with
//    J_g = I - dt Phi^T D J_f D^-1 Phi.  One fused pass over the basis per
//    Newton iteration: reconstruct q~ on a chunk (+ halo), evaluate f and the
//    three Jacobian diagonals per row, form (J_f Phi) rows on the fly and
//    accumulate Phi^T f (FP64) and Phi^T (J_f Phi) per block; a second
//    launch reduces the block partials in fixed order and solves the r x r
//    system in FP64 (partial-pivoting LU), one workgroup per instance.
//  * Hyper-reduced LSPG step (eqs. hyperreduced_lspg,
//    hyperreduced_lspg_stationarity): Gauss-Newton on the sampled residual
//    M P^T D r with M = (P^T Phi)^+, evaluated on the sample mesh only (each
//    sampled row needs its cell and the two neighbours), in FP64; each
//    iteration evaluates the sampled rows over many blocks per instance, then
//    reduces M A_s, M b and solves the r x r system per instance.
//  * Greedy DEIM with oversampling (interpolation-residual argmax, then a
//    least-squares round) and the (P^T Phi)^+ rebuild by Householder QR.
#include "internal.h"
#include "linalg.h"
#include "physics.h"

namespace romhip {

namespace {

constexpr int kGC = 64;  // rows per Galerkin chunk

template <class M>
struct Tag { using type = M; };

// ------------------------------------------------------------------ Galerkin pass
template <typename T>
__global__ __launch_bounds__(256) void k_galerkin_pass(
    const Tile* __restrict__ tiles, const int64_t* __restrict__ dof_off,
    const int64_t* __restrict__ cell_off, const double* __restrict__ phys, int nphys,
    const T* __restrict__ Phi, int r, const T* __restrict__ qref, const double* __restrict__ dvar,
    const double* __restrict__ a, const int32_t* __restrict__ active, double* __restrict__ gpart,
    T* __restrict__ mpart) {
  __shared__ T sP[kGC + 2][kMaxR + 1];
  __shared__ double sQ[kGC + 2];
  __shared__ double sF[kGC], sA[kGC], sB[kGC], sC[kGC];
  __shared__ double sa[kMaxR];
  __shared__ T red[4][kMaxR];
  __shared__ double redg[4][kMaxR];
  const Tile t = tiles[blockIdx.x];
  const int b = t.inst;
  if (!active[b]) return;
  const int tid = threadIdx.x, lane = tid & 63, grp = tid >> 6;
  const int64_t n = cell_off[b + 1] - cell_off[b];
  const int64_t base = dof_off[b];
  const double nu = phys[(size_t)b * nphys];
  const double dinv = 1.0 / dvar[b];
  const double inv = (double)n, inv2 = (double)n * (double)n;
  for (int c = tid; c < r; c += blockDim.x) sa[c] = a[(size_t)b * r + c];
  T acc[kMaxR];
#pragma unroll
  for (int c = 0; c < kMaxR; ++c) acc[c] = T(0);
  double accg = 0.0;
  for (int64_t r0 = 0; r0 < t.ncell; r0 += kGC) {
    const int nr = (int)(t.ncell - r0 < kGC ? t.ncell - r0 : kGC);
    const int64_t c0 = t.cell0 + r0;
    __syncthreads();
    for (int e = tid; e < (nr + 2) * r; e += blockDim.x) {
      const int rr = e / r, c = e - rr * r;
      int64_t cell = c0 - 1 + rr;
      cell = cell < 0 ? cell + n : (cell >= n ? cell - n : cell);
      sP[rr][c] = Phi[(base + cell) * r + c];
    }
    __syncthreads();
    if (tid < nr + 2) {
      int64_t cell = c0 - 1 + tid;
      cell = cell < 0 ? cell + n : (cell >= n ? cell - n : cell);
      double s = 0.0;
      for (int c = 0; c < r; ++c) s += (double)sP[tid][c] * sa[c];
      sQ[tid] = (double)qref[base + cell] + s * dinv;
    }
    __syncthreads();
    if (tid < nr) {
      const double um = sQ[tid], u0 = sQ[tid + 1], up = sQ[tid + 2];
      double dla, dlb, dra, drb;
      const double FL = godunov(um, u0, dla, dlb);
      const double FR = godunov(u0, up, dra, drb);
      sF[tid] = -(FR - FL) * inv + nu * ((up - u0) - (u0 - um)) * inv2;
      sA[tid] = dla * inv + nu * inv2;
      sB[tid] = (dlb - dra) * inv - 2.0 * nu * inv2;
      sC[tid] = -drb * inv + nu * inv2;
    }
    __syncthreads();
    if (lane < r) {
      for (int rr = grp; rr < nr; rr += 4) {
        const double z = sA[rr] * (double)sP[rr][lane] + sB[rr] * (double)sP[rr + 1][lane] +
                         sC[rr] * (double)sP[rr + 2][lane];
        accg += (double)sP[rr + 1][lane] * sF[rr];
        const T zt = (T)z;
#pragma unroll
        for (int c = 0; c < kMaxR; ++c)
          if (c < r) acc[c] += sP[rr + 1][c] * zt;
      }
    }
  }
  // reduce the four row groups; M[c][lane] = sum_i Phi_ic (J Phi)_i,lane
  T* mo = mpart + (size_t)blockIdx.x * kMaxR * kMaxR;
#pragma unroll
  for (int c = 0; c < kMaxR; ++c) {
    if (c < r) {
      __syncthreads();
      if (lane < r) red[grp][lane] = acc[c];
      __syncthreads();
      if (tid < r) mo[c * r + tid] = red[0][tid] + red[1][tid] + red[2][tid] + red[3][tid];
    }
  }
  __syncthreads();
  if (lane < r) redg[grp][lane] = accg;
  __syncthreads();
  if (tid < r) gpart[(size_t)blockIdx.x * kMaxR + tid] = redg[0][tid] + redg[1][tid] + redg[2][tid] + redg[3][tid];
}

// LU with partial pivoting on an n x n FP64 matrix in LDS (row-major, ld n),
// solving A x = b in place of b.  Single-thread pivot search, row updates by
// the whole block.  Returns false (via *ok) if a pivot vanishes.
// Block-level wrapper (A row-major, leading dimension ld); *ok is written for
// the whole block.
DEV void lu_solve_block(double* A, int ld, double* bvec, int n, int* ok) {
  const int r = block_lu_solve(A, ld, bvec, n);
  if (threadIdx.x == 0) *ok = r;
  __syncthreads();
}

template <typename T>
__global__ __launch_bounds__(256) void k_galerkin_solve(
    const int* __restrict__ tfirst, const double* __restrict__ gpart, const T* __restrict__ mpart,
    int r, double dt, const double* __restrict__ dvar, double* __restrict__ a,
    double* __restrict__ a_prev, int32_t* __restrict__ active, int32_t* __restrict__ iters,
    double tol, uint32_t* flags, int first) {
  __shared__ double J[kMaxR * (kMaxR + 1)];
  __shared__ double g[kMaxR];
  __shared__ int ok;
  const int b = blockIdx.x, tid = threadIdx.x;
  if (!first && !active[b]) return;
  const int ld = r + 1;
  const double d = dvar[b];
  // tile partials summed in tile order; the loads of 8 tiles are issued together
  const int t0 = tfirst[b], t1 = tfirst[b + 1];
  for (int e = tid; e < r * r; e += blockDim.x) {
    double s = 0.0;
    for (int tt = t0; tt < t1; tt += 8) {
      T v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u)
        v[u] = tt + u < t1 ? mpart[(size_t)(tt + u) * kMaxR * kMaxR + e] : T(0);
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (tt + u < t1) s += (double)v[u];
    }
    const int i = e / r, j = e % r;
    J[i * ld + j] = (i == j ? 1.0 : 0.0) - dt * s;
  }
  for (int c = tid; c < r; c += blockDim.x) {
    double s = 0.0;
    for (int tt = t0; tt < t1; tt += 8) {
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = tt + u < t1 ? gpart[(size_t)(tt + u) * kMaxR + c] : 0.0;
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (tt + u < t1) s += v[u];
    }
    // the first iteration of a step starts from a_prev = a (and records it)
    const double ac = a[(size_t)b * r + c];
    if (first) a_prev[(size_t)b * r + c] = ac;
    g[c] = -(ac - (first ? ac : a_prev[(size_t)b * r + c]) - dt * d * s);
  }
  __syncthreads();
  lu_solve_block(J, ld, g, r, &ok);
  // a += delta, one lane per component (r <= 64), then the stopping test
  if (tid < 64) {
    double dm = 0.0, am = 0.0;
    int fin = 1;
    if (tid < r) {
      const double an = a[(size_t)b * r + tid] + g[tid];
      a[(size_t)b * r + tid] = an;
      dm = fabs(g[tid]);
      am = fabs(an);
      fin = isfinite(an) ? 1 : 0;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      dm = fmax(dm, __shfl_xor(dm, off));
      am = fmax(am, __shfl_xor(am, off));
      fin &= __shfl_xor(fin, off);
    }
    if (tid == 0) {
      iters[b] = first ? 1 : iters[b] + 1;
      if (!ok) atomicOr(&flags[b], ROM_FLAG_SINGULAR);
      if (!fin) atomicOr(&flags[b], ROM_FLAG_NONFINITE);
      active[b] = (dm <= tol * (1.0 + am) || !fin) ? 0 : 1;
    }
  }
}

// The value a DPP move with source CTRL brings to each lane: lanes in the
// rows of ROWMASK receive it, the other lanes keep their own value.
template <int CTRL, int ROWMASK>
DEV double dpp_move_d(double v) {
  const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
  const int lo = (int)(unsigned)u, hi = (int)(unsigned)(u >> 32);
  int olo, ohi;
  if (ROWMASK == 0xF) {
    olo = __builtin_amdgcn_mov_dpp(lo, CTRL, 0xF, 0xF, false);
    ohi = __builtin_amdgcn_mov_dpp(hi, CTRL, 0xF, 0xF, false);
  } else {
    olo = __builtin_amdgcn_update_dpp(lo, lo, CTRL, ROWMASK, 0xF, false);
    ohi = __builtin_amdgcn_update_dpp(hi, hi, CTRL, ROWMASK, 0xF, false);
  }
  return __builtin_bit_cast(double, ((unsigned long long)(unsigned)ohi << 32) |
                                        (unsigned long long)(unsigned)olo);
}

// One exchange of a wave max of v: a compare and select, so a NaN never
// replaces a number, and the maximum of numbers is exact.
template <int CTRL, int ROWMASK>
DEV double max_dpp(double v) {
  const double o = dpp_move_d<CTRL, ROWMASK>(v);
  return o > v ? o : v;
}

DEV double readlane_d(double x, int l) {
  const unsigned long long u = __builtin_bit_cast(unsigned long long, x);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)u, l);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u >> 32), l);
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// fmax over the wave, by DPP moves only (no LDS): each 16-lane row, then rows
// 1 and 3 take rows 0 and 2, then row 3 takes row 1; lane 63 ends with it.
DEV double wave_fmax_d(double v) {
  v = fmax(v, dpp_move_d<0xB1, 0xF>(v));    // quad_perm [1,0,3,2]
  v = fmax(v, dpp_move_d<0x4E, 0xF>(v));    // quad_perm [2,3,0,1]
  v = fmax(v, dpp_move_d<0x141, 0xF>(v));   // row_half_mirror
  v = fmax(v, dpp_move_d<0x140, 0xF>(v));   // row_mirror
  v = fmax(v, dpp_move_d<0x142, 0xA>(v));   // row_bcast:15 into rows 1, 3
  v = fmax(v, dpp_move_d<0x143, 0xC>(v));   // row_bcast:31 into rows 2, 3
  return readlane_d(v, 63);
}

// The value that lane (l & 31) + 32 H holds, for every lane l (H = 0 or 1):
// v_permlane32_swap with both operands x returns the half-0 copy in its first
// and the half-1 copy in its second result.
template <int H>
DEV double half_value(double x) {
  const unsigned long long u = __builtin_bit_cast(unsigned long long, x);
  const auto lo = __builtin_amdgcn_permlane32_swap((unsigned)u, (unsigned)u, false, false);
  const auto hi = __builtin_amdgcn_permlane32_swap((unsigned)(u >> 32), (unsigned)(u >> 32), false, false);
  return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi[H] << 32) | (unsigned)lo[H]);
}

// The same reduced Newton step for r = 32 (the FP32 MFMA path), by one
// wavefront with no LDS and no barriers.  Lane l holds row l & 31 of J_g,
// the even columns in lanes 0-31 and the odd ones in lanes 32-63, summed
// from the tile partials into registers; the right-hand side is kept in both
// halves.  LU with partial pivoting runs on the register rows: the pivot of
// column k is the lowest remaining row attaining max |J_g[:, k]| (a DPP max
// inside the half that holds column k, then a ballot), each row's
// column-k entry reaches the other half by a cross-half lane swap, each lane
// reads its columns of the pivot row from lanes p and p + 32 (lane reads,
// not LDS permutes), and every remaining row is eliminated
// with the pivot's reciprocal.  No rows move; the pivot order is recorded.
// Back-substitution walks the pivot order from the last column, each half
// summing the products of its own columns.
template <int RT>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(1, 2)))
void k_galerkin_solve_w(
    const int* __restrict__ tfirst, const double* __restrict__ gpart,
    const float* __restrict__ mpart, double dt, const double* __restrict__ dvar,
    double* __restrict__ a, double* __restrict__ a_prev, int32_t* __restrict__ active,
    int32_t* __restrict__ iters, double tol, uint32_t* flags, int first) {
  static_assert(RT == 32, "two columns per lane pair, 32 rows");
  constexpr int NL = RT / 2;   // columns per lane
  __builtin_amdgcn_s_setprio(3);   // critical path of the window (see k_galerkin_mfma)
  const int b = blockIdx.x, lane = threadIdx.x;
  if (!first && !active[b]) return;
  const int i = lane & 31, h = lane >> 5;
  const int t0 = tfirst[b], t1 = tfirst[b + 1];
  // Sum the tile partials of Phi^T J_f Phi and Phi^T f.  The pass stores each
  // tile's block in the order of this kernel's registers (mpart_pos32), so
  // every lane reads its row half as four float4 loads (1 KB contiguous per
  // load of the wave), up to kTG tiles in flight at once; every element is
  // summed over the tiles in order in FP64.  No LDS anywhere in the kernel:
  // the solve shares its compute unit with LDS-heavy kernels of the event
  // chain and must not queue behind them.
  // The loads are issued unconditionally (tile indices clamped to the last
  // tile) so that a group's loads are in flight together; the state, a_prev
  // and d of the instance are loaded first, beside them.
  constexpr int kTG = 2;
  const double ai = a[(size_t)b * RT + i];
  const double api = first ? ai : a_prev[(size_t)b * RT + i];
  const double dvb = dvar[b];
  double A[NL];
#pragma unroll
  for (int jj = 0; jj < NL; ++jj) A[jj] = 0.0;
  double gs = 0.0;
  for (int tt = t0; tt < t1; tt += kTG) {
    float4 v[kTG][4];
    double gv[kTG];
#pragma unroll
    for (int g = 0; g < kTG; ++g) {
      const int tg = tt + g < t1 ? tt + g : t1 - 1;
      const float4* src = reinterpret_cast<const float4*>(mpart + (size_t)tg * kMaxR * kMaxR);
#pragma unroll
      for (int u = 0; u < 4; ++u) v[g][u] = src[lane + 64 * u];
      gv[g] = gpart[(size_t)tg * kMaxR + i];
    }
#pragma unroll
    for (int g = 0; g < kTG; ++g) {
      if (tt + g < t1) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          A[4 * u + 0] += (double)v[g][u].x;
          A[4 * u + 1] += (double)v[g][u].y;
          A[4 * u + 2] += (double)v[g][u].z;
          A[4 * u + 3] += (double)v[g][u].w;
        }
        gs += gv[g];
      }
    }
  }
  // register jj of lane (i, h) holds column 2 jj + h of row i
#pragma unroll
  for (int jj = 0; jj < NL; ++jj) A[jj] = (2 * jj + h == i ? 1.0 : 0.0) - dt * A[jj];
  // the first iteration of a step starts from a_prev = a (and records it)
  if (first && h == 0) a_prev[(size_t)b * RT + i] = ai;
  double bi = -(ai - api - dt * dvb * gs);
  bool used = false;
  int ord = -1;
  int pivl = 0;       // lane k: the pivot row of column k
  double myr = 0.0;   // pivot rows: the reciprocal of their pivot
#pragma unroll
  for (int k = 0; k < RT; ++k) {
    const int hk = k & 1, kk = k >> 1;
    const double cand = used ? -1.0 : fabs(A[kk]);
    double v = max_dpp<0xB1, 0xF>(cand);   // quad_perm [1,0,3,2]
    v = max_dpp<0x4E, 0xF>(v);              // quad_perm [2,3,0,1]
    v = max_dpp<0x141, 0xF>(v);             // row_half_mirror
    v = max_dpp<0x140, 0xF>(v);             // row_mirror: each 16-lane row holds its max
    v = max_dpp<0x142, 0xA>(v);             // row_bcast:15 into rows 1, 3
    const double vmax = readlane_d(v, hk ? 63 : 31);  // max of the half holding column k
    // the pivot: the lowest row of that half attaining the max (any remaining
    // row if the column holds no number)
    unsigned long long m = __ballot((cand == vmax) & (h == hk));
    if (m == 0) m = __ballot(!used & (h == hk));
    const int p = (__ffsll((long long)m) - 1) & 31;   // pivot row
    const double ck = hk ? half_value<1>(A[kk]) : half_value<0>(A[kk]);  // row's column-k entry
    const double pk = readlane_d(A[kk], p + 32 * hk);
    const double rp = pk != 0.0 ? 1.0 / pk : 0.0;
    if (lane == k) pivl = p;
    // rows already pivoted and the pivot row itself keep their values (f = 0)
    const double f = (used || i == p) ? 0.0 : ck * rp;
    if (i == p) {
      used = true;
      ord = k;
      myr = rp;
    }
    // the pivot row's copy of this lane's columns: lane p holds the even
    // ones, lane p + 32 the odd ones
#pragma unroll
    for (int jj = kk; jj < NL; ++jj) {
      const double e0 = readlane_d(A[jj], p), e1 = readlane_d(A[jj], p + 32);
      A[jj] -= f * (h ? e1 : e0);
    }
    bi -= f * readlane_d(bi, p);
  }
  // a zero pivot leaves a zero reciprocal on its row
  const int ok = __ballot((h == 0) & (myr == 0.0)) == 0ull;
  // back-substitution: x_k = (c_q - s0_q - s1_q) / U_qk for the pivot row q of
  // column k, where s0 and s1 are the products already subtracted by the even
  // and odd columns
  double sh = 0.0, del = 0.0;
#pragma unroll
  for (int k = RT - 1; k >= 0; --k) {
    const int hk = k & 1, kk = k >> 1;
    const double st = half_value<0>(sh) + half_value<1>(sh);
    const double xk = readlane_d((bi - st) * myr, __builtin_amdgcn_readlane(pivl, k));
    if (h == hk) sh += A[kk] * xk;
    if (i == k) del = xk;
  }
  double dm = 0.0, am = 0.0;
  int fin = 1;
  if (h == 0) {
    const double an = ai + del;
    a[(size_t)b * RT + i] = an;
    dm = fabs(del);
    am = fabs(an);
    fin = isfinite(an) ? 1 : 0;
  }
  dm = wave_fmax_d(dm);
  am = wave_fmax_d(am);
  fin = __ballot(fin == 0) == 0ull ? 1 : 0;
  if (lane == 0) {
    iters[b] = first ? 1 : iters[b] + 1;
    if (!ok) atomicOr(&flags[b], ROM_FLAG_SINGULAR);
    if (!fin) atomicOr(&flags[b], ROM_FLAG_NONFINITE);
    active[b] = (dm <= tol * (1.0 + am) || !fin) ? 0 : 1;
  }
}

__global__ void k_rom_finalize(int n_inst, const int32_t* active, uint32_t* flags) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < n_inst && active[b]) atomicOr(&flags[b], ROM_FLAG_ROM_NOCONV);
}

// Solves A x = b (n x n, n <= kMaxR, A row-major in LDS with leading dimension
// ld) on the first wavefront of the block, with no barrier: lane i keeps row i
// of [A | b] in registers.  Partial pivoting chooses rows without moving them
// (the largest magnitude, lowest lane on ties); the elimination and the
// multipliers are those of row-pivoted LU, and back-substitution reads each
// column's pivot row by its lane.  x overwrites b; *ok is 0 if a pivot vanishes.
// The caller synchronises the block afterwards.
// NM >= n bounds the columns kept per lane (up to kMaxR; columns n .. NM - 1 cost
// work, so the instances are sized to the configurations' r).
template <int NM>
DEV void wave_lu_solve(const double* A, int ld, double* bvec, int n, int* ok) {
  static_assert(NM <= kMaxR && NM <= 64, "one row per lane");
  const int lane = threadIdx.x & 63;
  double row[NM + 1];   // columns beyond n stay zero and are updated harmlessly
#pragma unroll
  for (int c = 0; c < NM; ++c) row[c] = (lane < n && c < n) ? A[lane * ld + c] : 0.0;
  row[NM] = lane < n ? bvec[lane] : 0.0;
  bool used = lane >= n, good = true;
  int pivl = 0;        // lane k: the pivot row (lane) of column k
  double myr = 0.0;    // pivot rows: the reciprocal of their pivot
#pragma unroll
  for (int k = 0; k < NM; ++k) {
    if (k < n) {
      const double a = row[k];
      // the pivot: the lowest lane holding the largest key (keys are never NaN;
      // an unused row with lane < n exists, so the maximum is at least 0)
      const double key = used ? -1.0 : (isnan(a) ? (double)INFINITY : fabs(a));
      const double kmax = wave_fmax_d(key);
      const int p = __builtin_amdgcn_readfirstlane(__builtin_ctzll(__ballot(key == kmax)));
      const double pk = readlane_d(a, p);
      const double rp = pk != 0.0 ? 1.0 / pk : 0.0;
      if (!(pk != 0.0)) good = false;
      if (lane == k) pivl = p;
      const double f = (used || lane == p) ? 0.0 : a * rp;
      if (lane == p) { used = true; myr = rp; }
#pragma unroll
      for (int c = k + 1; c <= NM; ++c) row[c] -= f * readlane_d(row[c], p);
    }
  }
  double sh = 0.0, xm = 0.0;   // sh: sum over the solved columns of row * x
#pragma unroll
  for (int k = NM - 1; k >= 0; --k) {
    if (k < n) {
      const int q = __builtin_amdgcn_readlane(pivl, k);
      const double xk = readlane_d((row[NM] - sh) * myr, q);
      sh += row[k] * xk;
      if (lane == k) xm = xk;
    }
  }
  if (lane < n) bvec[lane] = xm;
  if (lane == 0) *ok = good ? 1 : 0;
}

// ------------------------------------------------------------------ HR-LSPG step
// f_v and row v of the three Jacobian blocks (cells c-1, c, c+1) of J_f at a
// sampled row (cell c, variable v) of an instance of n cells, from the three
// stencil states q3 (FP64).  Walls fold the ghost's column into the centre
// block.  Shared by the HR-LSPG step and its adjoint.
template <class Mdl>
DEV void hr_row(const Mdl& m, const double* q3, int64_t c, int v, int64_t n, double& fv,
                double* jm, double* j0, double* jp, unsigned& fl) {
  constexpr int NV = Mdl::NV;
  constexpr int NN = NV * NV;
  const bool lw = !Mdl::periodic && c == 0, rw = !Mdl::periodic && c == n - 1;
  const double inv = (double)n, inv2 = (double)n * (double)n;
  if constexpr (NV >= 8) {
    // large blocks: only row v is formed (the model's row methods)
    double hl, hr, dll[NV], drl[NV], dlr[NV], drr[NV];
    m.face_jac_row(&q3[0], &q3[NV], v, hl, dll, drl);
    m.face_jac_row(&q3[NV], &q3[2 * NV], v, hr, dlr, drr);
    fv = -(hr - hl) * inv;
    for (int w = 0; w < NV; ++w) {
      jm[w] = dll[w] * inv; j0[w] = (drl[w] - dlr[w]) * inv; jp[w] = -drr[w] * inv;
    }
    if (lw) for (int w = 0; w < NV; ++w) { j0[w] += jm[w]; jm[w] = 0.0; }
    if (rw) for (int w = 0; w < NV; ++w) { j0[w] += jp[w]; jp[w] = 0.0; }
    const double kap = m.kappa(v);
    if (kap != 0.0) {
      fv += kap * ((q3[2 * NV + v] - q3[NV + v]) - (q3[NV + v] - q3[v])) * inv2;
      const double cc = kap * inv2;
      for (int w = 0; w < NV; ++w)
        if (w == v) {
          jm[w] += lw ? 0.0 : cc;
          jp[w] += rw ? 0.0 : cc;
          j0[w] += -2.0 * cc + (lw ? cc : 0.0) + (rw ? cc : 0.0);
        }
    }
    if (Mdl::has_source) {
      double sv_, ds[NV];
      m.source_jac_row(&q3[NV], ((double)c + 0.5) / (double)n, v, sv_, ds, fl);
      fv += sv_;
      for (int w = 0; w < NV; ++w) j0[w] += ds[w];
    }
  } else {
    double f[NV], Jm[NN], J0[NN], Jp[NN];
    {
      // cell_jacobian for one cell (FP64), inlined to avoid a cross-file template
      double HL[NV], HR[NV], DLl[NN], DRl[NN], DLr[NN], DRr[NN];
      m.face_jac(&q3[0], &q3[NV], HL, DLl, DRl, fl);
      m.face_jac(&q3[NV], &q3[2 * NV], HR, DLr, DRr, fl);
      for (int w = 0; w < NV; ++w) f[w] = -(HR[w] - HL[w]) * inv;
      for (int e = 0; e < NN; ++e) {
        Jm[e] = DLl[e] * inv; J0[e] = (DRl[e] - DLr[e]) * inv; Jp[e] = -DRr[e] * inv;
      }
      if (lw) for (int e = 0; e < NN; ++e) { J0[e] += Jm[e]; Jm[e] = 0.0; }
      if (rw) for (int e = 0; e < NN; ++e) { J0[e] += Jp[e]; Jp[e] = 0.0; }
      for (int w = 0; w < NV; ++w) {
        const double kap = m.kappa(w);
        if (kap != 0.0) {
          f[w] += kap * ((q3[2 * NV + w] - q3[NV + w]) - (q3[NV + w] - q3[w])) * inv2;
          const double cc = kap * inv2;
          Jm[w * NV + w] += lw ? 0.0 : cc;
          Jp[w * NV + w] += rw ? 0.0 : cc;
          J0[w * NV + w] += -2.0 * cc + (lw ? cc : 0.0) + (rw ? cc : 0.0);
        }
      }
      if (Mdl::has_source) {
        double S[NV], DS[NN];
        m.source_jac(&q3[NV], ((double)c + 0.5) / (double)n, S, DS, fl);
        for (int w = 0; w < NV; ++w) f[w] += S[w];
        for (int e = 0; e < NN; ++e) J0[e] += DS[e];
      }
    }
    fv = f[v];
    for (int w = 0; w < NV; ++w) {
      jm[w] = Jm[v * NV + w]; j0[w] = J0[v * NV + w]; jp[w] = Jp[v * NV + w];
    }
  }
}

// One Gauss-Newton iteration is three launches: k_hr_eval spreads the sampled
// rows of every instance over blocks of kHrRows rows (stencil states, the
// sampled Jacobian rows, the rows of A_s and b); k_hr_reduce forms M A_s and
// M b over blocks of rows of M, and k_hr_solve solves each instance's r x r
// system on one wavefront and updates a.  Instances that have
// converged skip both.
constexpr int kHrRows = 8;            // sampled rows per evaluation block
constexpr int kHrEvalThreads = 128;
// mesh_phi[b][s][o][w][k] (bulk precision), o in {0,1,2} = cells c-1, c, c+1 of the
// sampled row's cell.
// hr_as[b][s][0..r) = row s of A_s, hr_as[b][s][r] = b_s.
template <class Mdl, typename TM>
__global__ __launch_bounds__(kHrEvalThreads) void k_hr_eval(
    int r, int ns, int gpi, const int64_t* __restrict__ cell_off, const double* __restrict__ phys,
    int nphys, const int32_t* __restrict__ P, const TM* __restrict__ mphi,
    const double* __restrict__ mqref, const double* __restrict__ dvar, const double* __restrict__ a,
    const double* __restrict__ a_prev, double dt, const int32_t* __restrict__ active,
    double* __restrict__ hr_as, uint32_t* flags) {
  constexpr int NV = Mdl::NV;
  constexpr int NN = NV * NV;
  constexpr int E3 = 3 * NV;       // entries of a sampled row's three-cell stencil
  static_assert(kMaxR <= 64, "eight columns per lane");
  __shared__ double sa[kMaxR], sap[kMaxR];
  __shared__ double sq3[kHrRows * E3];   // reconstructed states of the block's stencils
  __shared__ double sjr[kHrRows * E3];   // sampled Jacobian rows scaled by 1 / d
  __shared__ int sv[kHrRows];            // variable of each sampled row
  __shared__ double sdd[kHrRows];        // dt d_v of each sampled row
  __shared__ unsigned flacc;
  const int b = blockIdx.x / gpi, g = blockIdx.x - b * gpi, tid = threadIdx.x;
  if (!active[b]) return;
  const int s0 = g * kHrRows;
  const int nr = ns - s0 < kHrRows ? ns - s0 : kHrRows;
  const int64_t n = cell_off[b + 1] - cell_off[b];
  Mdl m(phys + (size_t)b * nphys);
  const double* dv = dvar + (size_t)b * NV;
  const TM* mph = mphi + ((size_t)b * ns + s0) * E3 * r;   // the block's stencil rows
  double* out = hr_as + ((size_t)b * ns + s0) * (r + 1);
  for (int c = tid; c < r; c += blockDim.x) {
    sa[c] = a[(size_t)b * r + c];
    sap[c] = a_prev[(size_t)b * r + c];
  }
  if (tid == 0) flacc = 0;
  __syncthreads();
  // stencil states q = q_ref + D^-1 Phi a: eight lanes per entry, each summing
  // every eighth basis column; all of a lane's loads (at most eight per entry,
  // two entries) are issued before its sums
  {
    const int l8 = tid & 7;
    const int nq = nr * E3, step = blockDim.x >> 3;
    for (int idx0 = tid >> 3; idx0 < nq; idx0 += 2 * step) {
      double v[2][8];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int idx = idx0 + h * step < nq ? idx0 + h * step : idx0;
        const TM* Ph = mph + (size_t)idx * r;
#pragma unroll
        for (int u = 0; u < 8; ++u) v[h][u] = (double)Ph[l8 + 8 * u < r ? l8 + 8 * u : 0];
      }
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int idx = idx0 + h * step;
        double acc = 0.0;
#pragma unroll
        for (int u = 0; u < 8; ++u)
          if (l8 + 8 * u < r) acc += v[h][u] * sa[l8 + 8 * u];
        acc += __shfl_xor(acc, 1, 8);
        acc += __shfl_xor(acc, 2, 8);
        acc += __shfl_xor(acc, 4, 8);
        if (l8 == 0 && idx < nq) {
          const int s = idx / E3, e = idx - s * E3;
          sq3[idx] = mqref[((size_t)b * ns + s0 + s) * E3 + e] + acc / dv[e % NV];
        }
      }
    }
  }
  __syncthreads();
  // sampled rows of P^T D r and of the Jacobian P^T D J_r D^-1 (one row per thread)
  for (int s = tid; s < nr; s += blockDim.x) {
    const TM* Ph = mph + (size_t)s * E3 * r;
    const int p = P[(size_t)b * ns + s0 + s];
    const int64_t c = p / NV;
    const int v = p % NV;
    const double* q3 = sq3 + s * E3;
    double fv, jm[NV], j0[NV], jp[NV];   // f_v and row v of the three Jacobian blocks
    unsigned fl = 0;
    hr_row(m, q3, c, v, n, fv, jm, j0, jp, fl);
    if (fl) atomicOr(&flacc, fl);
    const double dp = dv[v];
    double bsum = 0.0;
    for (int k = 0; k < r; ++k) bsum += (double)Ph[(NV + v) * r + k] * (sa[k] - sap[k]);
    out[(size_t)s * (r + 1) + r] = bsum - dt * dp * fv;
    for (int w = 0; w < NV; ++w) {
      const double id = 1.0 / dv[w];
      sjr[s * E3 + w] = jm[w] * id;
      sjr[s * E3 + NV + w] = j0[w] * id;
      sjr[s * E3 + 2 * NV + w] = jp[w] * id;
    }
    sv[s] = v;
    sdd[s] = dt * dp;
  }
  __syncthreads();
  // rows of A_s = P^T Phi - dt P^T D J_r D^-1 Phi, one entry per thread
  // (consecutive threads take consecutive basis columns), two per thread
  for (int idx0 = tid; idx0 < nr * r; idx0 += 2 * blockDim.x) {
    double acc[2] = {0.0, 0.0};
    const TM* Ph[2];
    int sx[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int idx = idx0 + h * blockDim.x < nr * r ? idx0 + h * blockDim.x : idx0;
      const int s = idx / r, k = idx - s * r;
      sx[h] = s;
      Ph[h] = mph + (size_t)s * E3 * r + k;
    }
#pragma unroll
    for (int w = 0; w < NV; ++w)
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const double* jr = sjr + sx[h] * E3;
        acc[h] += jr[w] * (double)Ph[h][w * r];
        acc[h] += jr[NV + w] * (double)Ph[h][(NV + w) * r];
        acc[h] += jr[2 * NV + w] * (double)Ph[h][(2 * NV + w) * r];
      }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int idx = idx0 + h * blockDim.x;
      if (idx < nr * r) {
        const int s = sx[h], k = idx - s * r;
        out[(size_t)s * (r + 1) + k] = (double)Ph[h][(NV + sv[s]) * r] - sdd[s] * acc[h];
      }
    }
  }
  if (tid == 0 && flacc) atomicOr(&flags[b], flacc);
}

// A_red = M A_s and rho = -M b: one block per instance and group of kHrRedRows
// rows of M, into hr_ar[b] (r rows of r + 1: A_red | rho).  The block copies
// its rows of M (sample-major) and the instance's [A_s | b] into LDS with
// every thread's loads in flight together, then thread (column c, half h)
// sums rows 4h .. 4h+3 of column c over the samples in order (FP64).
// k_hr_solve then solves the system; the launch boundary between them
// publishes the rows.
constexpr int kHrRedRows = 8;
constexpr int kHrRedThreads = 256;
__global__ __launch_bounds__(kHrRedThreads) void k_hr_reduce(
    int r, int ns, int gpr, const double* __restrict__ Mp, const double* __restrict__ hr_as,
    const int32_t* __restrict__ active, double* __restrict__ hr_ar) {
  extern __shared__ double shr[];
  const int b = blockIdx.x / gpr, g = blockIdx.x - b * gpr, tid = threadIdx.x;
  if (!active[b]) return;
  const int ld = r + 1;
  const int i0 = g * kHrRedRows;
  const int ni = r - i0 < kHrRedRows ? r - i0 : kHrRedRows;
  double* sMt = shr;                      // [ns][kHrRedRows]: M[i0 + u][s] at s*8 + u
  double* sA = shr + kHrRedRows * ns;     // [ns][ld]
  {
    // loads are issued unconditionally (indices clamped into range) so that a
    // batch of eight is in flight together; the guards apply to the stores
    const double* Mg = Mp + (size_t)b * r * ns + (size_t)i0 * ns;
    const double* Ag = hr_as + (size_t)b * ns * ld;
    const int nm = ni * ns, na = ns * ld;
    for (int e0 = tid; e0 < nm + na; e0 += kHrRedThreads * 8) {
      double v[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int e = e0 + kHrRedThreads * j;
        const double* src = e < nm ? Mg + e : Ag + (e < nm + na ? e - nm : na - 1);
        v[j] = *src;
      }
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int e = e0 + kHrRedThreads * j;
        if (e < nm) {
          const int u = e / ns;
          sMt[(e - u * ns) * kHrRedRows + u] = v[j];
        } else if (e < nm + na) {
          sA[e - nm] = v[j];
        }
      }
    }
  }
  __syncthreads();
  const int c = tid % ld, h = tid / ld;
  if (h < 2) {
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int s0 = 0; s0 < ns; ++s0) {
      const double av = sA[s0 * ld + c];
      const double* m = sMt + s0 * kHrRedRows + 4 * h;
#pragma unroll
      for (int u = 0; u < 4; ++u) acc[u] += m[u] * av;
    }
    double* out = hr_ar + (size_t)b * r * ld;
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (4 * h + u < ni) out[(size_t)(i0 + 4 * h + u) * ld + c] = c < r ? acc[u] : -acc[u];
  }
}

size_t hr_reduce_shm(int r, int ns) {
  return sizeof(double) * ((size_t)kHrRedRows * ns + (size_t)ns * (r + 1));
}

// The r x r solve of one instance (rows of hr_ar loaded by the block, solved by
// its first wavefront) and the update of a.
template <int NM>
__global__ __launch_bounds__(256) void k_hr_solve(int r, const double* __restrict__ hr_ar,
                                                  int32_t* __restrict__ active,
                                                  double* __restrict__ a,
                                                  int32_t* __restrict__ iters, double tol,
                                                  uint32_t* flags) {
  __shared__ double Ar[kMaxR * (kMaxR + 1)];
  __shared__ double rh[kMaxR];
  __shared__ int ok;
  const int b = blockIdx.x, k = threadIdx.x;
  if (!active[b]) return;
  const int ld = r + 1;
  const double* out = hr_ar + (size_t)b * r * ld;
  for (int e0 = k; e0 < r * ld; e0 += 256 * 8) {
    double v[8];   // eight loads in flight per thread
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] = out[e0 + 256 * j < r * ld ? e0 + 256 * j : r * ld - 1];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int e = e0 + 256 * j;
      if (e < r * ld) {
        const int i = e / ld, c = e - i * ld;
        if (c < r) Ar[e] = v[j]; else rh[i] = v[j];
      }
    }
  }
  __syncthreads();
  if (k >= 64) return;
  wave_lu_solve<NM>(Ar, ld, rh, r, &ok);
  // the update: lane c takes a_c (its own entry of rh); maxima by a wavefront
  // reduction
  const int lane = k;
  double dm = 0.0, am = 0.0;
  int fin = 1;
  if (lane < r) {
    const double an = a[(size_t)b * r + lane] + rh[lane];
    a[(size_t)b * r + lane] = an;
    dm = fabs(rh[lane]);
    am = fabs(an);
    fin = isfinite(an) ? 1 : 0;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    dm = fmax(dm, __shfl_xor(dm, off));
    am = fmax(am, __shfl_xor(am, off));
    fin &= __shfl_xor(fin, off);
  }
  if (lane == 0) {
    unsigned fl = 0;
    if (!ok) fl |= ROM_FLAG_SINGULAR;
    if (!fin) fl |= ROM_FLAG_NONFINITE;
    if (fl) atomicOr(&flags[b], fl);
    iters[b] += 1;
    active[b] = (dm <= tol * (1.0 + am) || !fin) ? 0 : 1;
  }
}

// ------------------------------------------------------------------ DEIM
// The greedy picks read the leading columns of every row of the basis, one
// column more per pick.  They read a column-major copy (per instance, column c
// of instance b at phi_cm + dof_off[b] r + c n_b with n_b its row count), so
// that a wavefront's loads of one column are contiguous and each pass moves
// only the columns it uses.
constexpr int kCmRows = 64;   // rows per step of the transposition

// phi_cm <- Phi by columns, one pass tile per block: 64-row slabs are read
// row-major into LDS and written out a column at a time.
template <typename T>
__global__ __launch_bounds__(256) void k_cols_transpose(const Tile* __restrict__ tiles,
                                                        const int64_t* __restrict__ dof_off,
                                                        const T* __restrict__ Phi, int r,
                                                        T* __restrict__ phi_cm) {
  __shared__ T sl[kCmRows][kMaxR + 1];
  const Tile t = tiles[blockIdx.x];
  const int b = t.inst, tid = threadIdx.x;
  const int64_t base = dof_off[b], nb = dof_off[b + 1] - base;
  const T* src = Phi + base * r;
  T* dst = phi_cm + base * r;
  for (int64_t r0 = t.cell0; r0 < t.cell0 + t.ncell; r0 += kCmRows) {
    const int nr = (int)(t.cell0 + t.ncell - r0 < kCmRows ? t.cell0 + t.ncell - r0 : kCmRows);
    __syncthreads();
    for (int e = tid; e < nr * r; e += blockDim.x) sl[e / r][e % r] = src[r0 * r + e];
    __syncthreads();
    for (int e = tid; e < nr * r; e += blockDim.x) {
      const int c = e / nr, i = e % nr;
      dst[(int64_t)c * nb + r0 + i] = sl[i][c];
    }
  }
}

// Residual of column j after fitting columns 0..j-1 with coef, and the argmax
// of |res| over the rows not yet chosen (lowest row on ties) in one of the S
// equal parts of a pass tile; block tt * S + s writes the candidate of part s
// of tile tt (value -1 and row -1 when the part has no free row).  The sum
// runs over the columns in increasing order in FP64.
template <typename T, int RPT>
__global__ __launch_bounds__(256) void k_deim_argmax(const Tile* __restrict__ tiles,
                                                     const int64_t* __restrict__ dof_off,
                                                     const T* __restrict__ phi_cm, int r, int j,
                                                     const double* __restrict__ coef, int ldc,
                                                     const uint32_t* __restrict__ chosen,
                                                     const uint32_t* __restrict__ epoch_p,
                                                     int S, double* __restrict__ tval,
                                                     int64_t* __restrict__ tidx) {
  __shared__ double sc[kMaxR];
  __shared__ double bv[256];
  __shared__ int64_t bi[256];
  const Tile t = tiles[blockIdx.x / S];
  const int part = blockIdx.x % S;
  const int b = t.inst, tid = threadIdx.x;
  const int64_t base = dof_off[b], nb = dof_off[b + 1] - base;
  const int64_t len = (t.ncell + S - 1) / S;
  const int64_t lo = t.cell0 + part * len;
  const int64_t hi = t.cell0 + ((part + 1) * len < t.ncell ? (part + 1) * len : t.ncell);
  const uint32_t epoch = *epoch_p;
  const T* cols = phi_cm + base * r;
  for (int c = tid; c < j; c += blockDim.x) sc[c] = coef[(size_t)b * ldc + c];
  __syncthreads();
  double best = -1.0;
  int64_t bidx = -1;
  for (int64_t r0 = lo; r0 < hi; r0 += 256 * RPT) {
    int64_t lr[RPT];
    bool ok[RPT];
    double res[RPT];
#pragma unroll
    for (int u = 0; u < RPT; ++u) {
      lr[u] = r0 + tid + 256 * u;
      ok[u] = lr[u] < hi;
      res[u] = ok[u] ? (double)cols[(int64_t)j * nb + lr[u]] : 0.0;
    }
    for (int c = 0; c < j; ++c) {
      const double w = sc[c];
      const T* col = cols + (int64_t)c * nb;
#pragma unroll
      for (int u = 0; u < RPT; ++u)
        if (ok[u]) res[u] -= (double)col[lr[u]] * w;
    }
#pragma unroll
    for (int u = 0; u < RPT; ++u) {
      if (!ok[u] || chosen[base + lr[u]] == epoch) continue;
      const double v = fabs(res[u]);
      if (v > best || (v == best && lr[u] < bidx)) { best = v; bidx = lr[u]; }
    }
  }
  bv[tid] = best;
  bi[tid] = bidx;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (tid < st) {
      const double v2 = bv[tid + st];
      const int64_t i2 = bi[tid + st];
      if (i2 >= 0 && (v2 > bv[tid] || (v2 == bv[tid] && (bi[tid] < 0 || i2 < bi[tid])))) {
        bv[tid] = v2; bi[tid] = i2;
      }
    }
    __syncthreads();
  }
  if (tid == 0) { tval[blockIdx.x] = bv[0]; tidx[blockIdx.x] = bi[0]; }
}

// The same pass for an FP32 basis with four consecutive rows per lane: each
// column is read as one 16-byte load per lane where the lane's rows are 16-byte
// aligned (scalar loads otherwise), with the per-row arithmetic of
// k_deim_argmax.
__global__ __launch_bounds__(128) void k_deim_argmax_v4(const Tile* __restrict__ tiles,
                                                        const int64_t* __restrict__ dof_off,
                                                        const float* __restrict__ phi_cm, int r,
                                                        int j, const double* __restrict__ coef,
                                                        int ldc, const uint32_t* __restrict__ chosen,
                                                        const uint32_t* __restrict__ epoch_p, int S,
                                                        double* __restrict__ tval,
                                                        int64_t* __restrict__ tidx) {
  constexpr int NT = 128;
  __shared__ double sc[kMaxR];
  __shared__ double bv[NT];
  __shared__ int64_t bi[NT];
  const Tile t = tiles[blockIdx.x / S];
  const int part = blockIdx.x % S;
  const int b = t.inst, tid = threadIdx.x;
  const int64_t base = dof_off[b], nb = dof_off[b + 1] - base;
  const int64_t len = (t.ncell + S - 1) / S;
  const int64_t lo = t.cell0 + part * len;
  const int64_t hi = t.cell0 + ((part + 1) * len < t.ncell ? (part + 1) * len : t.ncell);
  const uint32_t epoch = *epoch_p;
  const float* cols = phi_cm + base * r;
  for (int c = tid; c < j; c += blockDim.x) sc[c] = coef[(size_t)b * ldc + c];
  __syncthreads();
  double best = -1.0;
  int64_t bidx = -1;
  for (int64_t r0 = lo; r0 < hi; r0 += NT * 4) {
    const int64_t l0 = r0 + 4 * tid;
    bool ok[4];
    double res[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) ok[u] = l0 + u < hi;
    // all four rows in range and every column's four rows 16-byte aligned
    const bool vec = l0 + 4 <= hi && (nb & 3) == 0 &&
                     (reinterpret_cast<uintptr_t>(cols + l0) & 15) == 0;
    if (vec) {
      const float4 v0 = *reinterpret_cast<const float4*>(cols + (int64_t)j * nb + l0);
      res[0] = (double)v0.x; res[1] = (double)v0.y; res[2] = (double)v0.z; res[3] = (double)v0.w;
      for (int c = 0; c < j; ++c) {
        const double w = sc[c];
        const float4 v = *reinterpret_cast<const float4*>(cols + (int64_t)c * nb + l0);
        res[0] -= (double)v.x * w;
        res[1] -= (double)v.y * w;
        res[2] -= (double)v.z * w;
        res[3] -= (double)v.w * w;
      }
    } else {
#pragma unroll
      for (int u = 0; u < 4; ++u) res[u] = ok[u] ? (double)cols[(int64_t)j * nb + l0 + u] : 0.0;
      for (int c = 0; c < j; ++c) {
        const double w = sc[c];
#pragma unroll
        for (int u = 0; u < 4; ++u)
          if (ok[u]) res[u] -= (double)cols[(int64_t)c * nb + l0 + u] * w;
      }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (!ok[u] || chosen[base + l0 + u] == epoch) continue;
      const double v = fabs(res[u]);
      if (v > best || (v == best && l0 + u < bidx)) { best = v; bidx = l0 + u; }
    }
  }
  bv[tid] = best;
  bi[tid] = bidx;
  __syncthreads();
  for (int st = NT / 2; st > 0; st >>= 1) {
    if (tid < st) {
      const double v2 = bv[tid + st];
      const int64_t i2 = bi[tid + st];
      if (i2 >= 0 && (v2 > bv[tid] || (v2 == bv[tid] && (bi[tid] < 0 || i2 < bi[tid])))) {
        bv[tid] = v2; bi[tid] = i2;
      }
    }
    __syncthreads();
  }
  if (tid == 0) { tval[blockIdx.x] = bv[0]; tidx[blockIdx.x] = bi[0]; }
}

// Householder QR least squares on an m x nc FP64 matrix in LDS (row-major,
// ld = kMaxR + 1, m <= 128): overwrites x[0..nc) with argmin ||A x - rhs||.
// Four wavefronts (blockDim.x == 256) keep the columns in registers: wavefront
// w holds columns w, w + 4, ... (the rhs is column nc), lane l rows l and
// l + 64.  The owner of column k forms its reflector (squared norm by a wave
// sum, the head from row k) as soon as step k - 1 has updated that column,
// and publishes v and beta through LDS (double-buffered, one barrier per
// column); every wavefront then applies it to its own later columns with one
// wave sum per column.  R and the rotated rhs go back to LDS for the
// back-substitution.
DEV void qr_lstsq(double* A, int m, int nc, double* rhs, double* x) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  constexpr int ld = kMaxR + 1;
  constexpr int NQ = (kMaxR + 1 + 3) / 4;   // columns per wavefront, the rhs included
  static_assert(kMaxNs <= 128, "two rows per lane");
  __shared__ double sv[2][128];
  __shared__ double sbeta[2];
  __shared__ double salpha[kMaxR];    // R's diagonal
  const int r0 = lane, r1 = lane + 64;
  double c0[NQ], c1[NQ];   // rows r0 and r1 of columns wave + 4 q
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int c = wave + 4 * q;
    const double* src = c < nc ? A + c : rhs;
    const int cs = c < nc ? ld : 1;
    c0[q] = (c <= nc && r0 < m) ? src[r0 * cs] : 0.0;
    c1[q] = (c <= nc && r1 < m) ? src[r1 * cs] : 0.0;
  }
  // The reflector of column k from that column's rows (a0, a1) as all earlier
  // reflectors left them, by its owner: v and beta to LDS buffer k & 1, R's
  // diagonal entry alpha to salpha[k].
  auto reflector = [&](int k, double a0, double a1) {
    const double t0 = r0 >= k ? a0 : 0.0, t1 = r1 >= k ? a1 : 0.0;   // rows >= m hold 0
    const double s = wave_sum_bfly(t0 * t0 + t1 * t1);
    const double akk = readlane_d(k < 64 ? a0 : a1, k & 63);
    const double nrm = sqrt(s);
    const double alpha = akk >= 0.0 ? -nrm : nrm;
    // v = x - alpha e1 in column k (rows k..m-1); v^T v = s - akk^2 + (akk - alpha)^2
    const double vk = akk - alpha;
    const double vv = (s - akk * akk) + vk * vk;
    sv[k & 1][r0] = r0 == k ? vk : t0;
    sv[k & 1][r1] = r1 == k ? vk : t1;
    if (lane == 0) {
      sbeta[k & 1] = vv > 0.0 ? 2.0 / vv : 0.0;
      salpha[k] = alpha;
    }
  };
  if (wave == 0) reflector(0, c0[0], c1[0]);
  for (int k = 0; k < nc; ++k) {
    __syncthreads();
    const int buf = k & 1;
    const double v0 = sv[buf][r0], v1 = sv[buf][r1], beta = sbeta[buf];
    // each wavefront applies reflector k to its later columns; the owner of
    // column k + 1 updates it first and forms the next reflector at once, so
    // that its chain overlaps the remaining updates of every wavefront
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int c = wave + 4 * q;
      if (c > k && c <= nc) {   // uniform over the wavefront
        const double d = beta * wave_sum_bfly(v0 * c0[q] + v1 * c1[q]);
        c0[q] -= d * v0;
        c1[q] -= d * v1;
        if (c == k + 1 && c < nc) reflector(k + 1, c0[q], c1[q]);
      }
    }
  }
  // R and the rotated rhs back to LDS
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int c = wave + 4 * q;
    if (c <= nc) {
      double* dst = c < nc ? A + c : rhs;
      const int cs = c < nc ? ld : 1;
      // R's column c: the rows above c as updated, alpha on the diagonal
      // (the register copy of column c stopped at step c)
      const double d0 = c < nc && r0 == c ? salpha[c] : c0[q];
      const double d1 = c < nc && r1 == c ? salpha[c] : c1[q];
      if (r0 < m) dst[r0 * cs] = d0;
      if (r1 < m) dst[r1 * cs] = d1;
    }
  }
  __syncthreads();
  // back substitution R x = rhs[0..nc), column-oriented by the first wavefront
  if (wave == 0) {
    for (int i = nc - 1; i >= 0; --i) {
      const double d = A[i * ld + i];
      const double xi = d != 0.0 ? rhs[i] / d : 0.0;
      if (lane == 0) x[i] = xi;
      for (int j = lane; j < i; j += 64) rhs[j] -= A[j * ld + i] * xi;
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
  }
  __syncthreads();
}

// select pick t (reduce tile candidates), record it, and fit the coefficients
// of pick t+1 on the t+1 rows chosen so far.
template <typename T>
__global__ __launch_bounds__(256) void k_deim_select(const int* __restrict__ tfirst, int S,
                                                     const double* __restrict__ tval,
                                                     const int64_t* __restrict__ tidx,
                                                     const int64_t* __restrict__ dof_off,
                                                     const T* __restrict__ Phi, int r, int ns, int t,
                                                     int32_t* __restrict__ P,
                                                     uint32_t* __restrict__ chosen,
                                                     const uint32_t* __restrict__ epoch_p,
                                                     double* __restrict__ coef, int ldc,
                                                     uint32_t* flags) {
  __shared__ double A[kMaxNs * (kMaxR + 1)];
  __shared__ double rhs[kMaxNs];
  __shared__ double x[kMaxR];
  __shared__ double bv[256];
  __shared__ int64_t bix[256];
  const int b = blockIdx.x, tid = threadIdx.x;
  {  // argmax over the instance's tile winners (largest value, lowest row on ties)
    double best = -1.0;
    int64_t bi = -1;
    for (int tt = tfirst[b] * S + tid; tt < tfirst[b + 1] * S; tt += blockDim.x) {
      const double v = tval[tt];
      const int64_t i = tidx[tt];
      if (i >= 0 && (bi < 0 || v > best || (v == best && i < bi))) { best = v; bi = i; }
    }
    bv[tid] = best;
    bix[tid] = bi;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
      if (tid < st) {
        const double v2 = bv[tid + st];
        const int64_t i2 = bix[tid + st];
        if (i2 >= 0 && (bix[tid] < 0 || v2 > bv[tid] || (v2 == bv[tid] && i2 < bix[tid]))) {
          bv[tid] = v2;
          bix[tid] = i2;
        }
      }
      __syncthreads();
    }
    if (tid == 0) {
      int64_t w = bix[0];
      if (w < 0) { w = 0; atomicOr(&flags[b], ROM_FLAG_SINGULAR); }
      P[(size_t)b * ns + t] = (int32_t)w;
      chosen[dof_off[b] + w] = *epoch_p;
    }
    __syncthreads();
  }
  const int tn = t + 1;           // next pick
  if (tn >= ns) return;
  const int jn = tn < r ? tn : tn - r;   // column of the next pick
  const int m = tn;                     // rows available
  if (jn == 0) return;                  // no fit for the first column of a round
  const T* Pb = Phi + dof_off[b] * r;
  __shared__ int64_t srow[kMaxNs];   // offsets of the chosen rows
  for (int i = tid; i < m; i += blockDim.x) srow[i] = (int64_t)P[(size_t)b * ns + i] * r;
  __syncthreads();
  {
    // the gather of A (m x jn) and rhs (column jn): eight loads per thread in
    // flight together (indices clamped into range), then the LDS stores
    const int ne = m * jn, nt = ne + m;
    for (int e0 = tid; e0 < nt; e0 += 256 * 8) {
      T v[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int e = e0 + 256 * j < nt ? e0 + 256 * j : nt - 1;
        const int i = e < ne ? e / jn : e - ne;
        const int c = e < ne ? e - i * jn : jn;
        v[j] = Pb[srow[i] + c];
      }
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int e = e0 + 256 * j;
        if (e < ne) {
          const int i = e / jn;
          A[i * (kMaxR + 1) + (e - i * jn)] = (double)v[j];
        } else if (e < nt) {
          rhs[e - ne] = (double)v[j];
        }
      }
    }
  }
  __syncthreads();
  qr_lstsq(A, m, jn, rhs, x);
  for (int c = tid; c < jn; c += blockDim.x) coef[(size_t)b * ldc + c] = x[c];
}

// (P^T Phi)^+ by Householder QR (A = Q R, A^+ = R^-1 Q^T) and the sample-mesh gathers.
template <typename T>
__global__ __launch_bounds__(256) void k_rebuild(int r, int ns, int nv, int periodic,
                                                 const int64_t* __restrict__ dof_off,
                                                 const int64_t* __restrict__ cell_off,
                                                 const T* __restrict__ Phi, const T* __restrict__ qref,
                                                 const int32_t* __restrict__ P, double* __restrict__ Mout,
                                                 T* __restrict__ mphi, double* __restrict__ mqref,
                                                 uint32_t* flags) {
  extern __shared__ double sm[];
  constexpr int ld = kMaxR + 1;
  double* A = sm;                    // ns x ld : R above the diagonal, reflectors below
  double* Q = A + kMaxNs * ld;       // ns x r  : first r columns of Q (row stride ld)
  double* vd = Q + kMaxNs * ld;      // reflector heads
  double* bt = vd + kMaxR;           // reflector scales
  __shared__ double alpha_s;   // alpha of the current column
  const int b = blockIdx.x, tid = threadIdx.x;
  const int64_t base = dof_off[b];
  const int64_t n = cell_off[b + 1] - cell_off[b];
  const T* Pb = Phi + base * r;
  // gathers: mesh cells c-1, c, c+1 of every sampled row (wrap or wall copy)
  for (int e = tid; e < ns * 3 * nv; e += blockDim.x) {
    const int s = e / (3 * nv), rem = e % (3 * nv), o = rem / nv, w = rem % nv;
    const int64_t c = P[(size_t)b * ns + s] / nv;
    int64_t cc = c - 1 + o;
    if (periodic) cc = (cc % n + n) % n;
    else cc = cc < 0 ? 0 : (cc >= n ? n - 1 : cc);
    const int64_t row = cc * nv + w;
    mqref[((size_t)b * ns + s) * 3 * nv + rem] = (double)qref[base + row];
    for (int k = 0; k < r; ++k)
      mphi[(((size_t)b * ns + s) * 3 * nv + rem) * r + k] = Pb[row * r + k];
  }
  for (int e = tid; e < ns * r; e += blockDim.x) {
    const int i = e / r, c = e % r;
    A[i * ld + c] = (double)Pb[(int64_t)P[(size_t)b * ns + i] * r + c];
  }
  __syncthreads();
  // Householder QR: column k reflector v = x - alpha e_k, H = I - beta v v^T
  // (the squared norms are summed by the first wavefront, lanes over rows)
  const int lane = tid & 63;
  for (int k = 0; k < r; ++k) {
    if (tid < 64) {
      double s2 = 0.0;
      for (int i = k + lane; i < ns; i += 64) s2 += A[i * ld + k] * A[i * ld + k];
      s2 = wave_sum_bfly(s2);
      const double akk = A[k * ld + k];
      const double alpha = akk >= 0.0 ? -sqrt(s2) : sqrt(s2);
      // v = x - alpha e_k; v^T v = s2 - akk^2 + (akk - alpha)^2
      const double vk = akk - alpha;
      const double vv = (s2 - akk * akk) + vk * vk;
      if (lane == 0) {
        alpha_s = alpha;
        A[k * ld + k] = vk;
        bt[k] = vv > 0.0 ? 2.0 / vv : 0.0;
        vd[k] = vk;
      }
    }
    __syncthreads();
    const double alpha = alpha_s;
    for (int c = k + 1 + tid; c < r; c += blockDim.x) {
      double s2 = 0.0;
      for (int i = k; i < ns; ++i) s2 += A[i * ld + k] * A[i * ld + c];
      s2 *= bt[k];
      for (int i = k; i < ns; ++i) A[i * ld + c] -= s2 * A[i * ld + k];
    }
    __syncthreads();
    if (tid == 0) A[k * ld + k] = alpha;
    __syncthreads();
  }
  // Q[:, :r] = H_0 H_1 ... H_{r-1} [I; 0]
  for (int e = tid; e < ns * r; e += blockDim.x) {
    const int i = e / r, c = e - i * r;
    Q[i * ld + c] = i == c ? 1.0 : 0.0;
  }
  __syncthreads();
  for (int k = r - 1; k >= 0; --k) {
    for (int c = tid; c < r; c += blockDim.x) {
      double s2 = vd[k] * Q[k * ld + c];
      for (int i = k + 1; i < ns; ++i) s2 += A[i * ld + k] * Q[i * ld + c];
      s2 *= bt[k];
      Q[k * ld + c] -= s2 * vd[k];
      for (int i = k + 1; i < ns; ++i) Q[i * ld + c] -= s2 * A[i * ld + k];
    }
    __syncthreads();
  }
  // M[:, s] = R^-1 Q[s, :]^T, one column per thread, computed in place over
  // row s of Q in LDS (the odd row stride keeps the threads' rows on distinct
  // banks), then stored coalesced
  for (int s = tid; s < ns; s += blockDim.x) {
    double* qs = Q + s * ld;
    for (int i = r - 1; i >= 0; --i) {
      double acc = qs[i];
      for (int c = i + 1; c < r; ++c) acc -= A[i * ld + c] * qs[c];
      qs[i] = A[i * ld + i] != 0.0 ? acc / A[i * ld + i] : 0.0;
    }
  }
  __syncthreads();
  {
    double* Mb = Mout + (size_t)b * r * ns;
    for (int e = tid; e < r * ns; e += blockDim.x) {
      const int i = e / ns, s2 = e - i * ns;
      Mb[e] = Q[s2 * ld + i];
    }
  }
  if (tid == 0) {
    double mx = 0.0, mn = 1e300;
    for (int c = 0; c < r; ++c) {
      const double d = fabs(A[c * ld + c]);
      mx = fmax(mx, d); mn = fmin(mn, d);
    }
    if (!(mn > 1e-13 * mx)) atomicOr(&flags[b], ROM_FLAG_SINGULAR);
  }
}

size_t rebuild_shm() {
  return sizeof(double) * (2 * kMaxNs * (kMaxR + 1) + 2 * kMaxR);
}

template <typename T>
__global__ __launch_bounds__(256) void k_reconstruct(const Tile* __restrict__ tiles,
                                                     const int64_t* __restrict__ dof_off,
                                                     const T* __restrict__ Phi, int r,
                                                     const T* __restrict__ qref,
                                                     const double* __restrict__ dvar, int nv,
                                                     const double* __restrict__ a, T* __restrict__ out) {
  const Tile t = tiles[blockIdx.x];
  const int b = t.inst;
  const int64_t base = dof_off[b];
  for (int64_t rr = threadIdx.x; rr < t.ncell; rr += blockDim.x) {
    const int64_t lr = t.cell0 + rr, g = base + lr;
    double s = 0.0;
    for (int c = 0; c < r; ++c) s += (double)Phi[g * r + c] * a[(size_t)b * r + c];
    out[g] = (T)((double)qref[g] + s / dvar[(size_t)b * nv + lr % nv]);
  }
}

__global__ void k_bump(uint32_t* e) { if (threadIdx.x == 0 && blockIdx.x == 0) *e = *e + 1u; }

__global__ void k_copy_f64(const double* src, double* dst, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[i];
}
__global__ void k_fill_i32(int32_t* dst, int32_t v, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = v;
}

// a_prev <- a, active <- 1, iters <- 0 for every instance (one launch).
__global__ void k_rom_step_setup(int n_inst, int r, const double* __restrict__ a,
                                 double* __restrict__ a_prev, int32_t* __restrict__ active,
                                 int32_t* __restrict__ iters) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < (int64_t)n_inst * r) a_prev[i] = a[i];
  if (i < n_inst) { active[i] = 1; iters[i] = 0; }
}

// Grid-wide Newton iterations of the Galerkin step kept in the captured launch
// sequence when the MFMA pass applies; later iterations (rare) run in
// k_galerkin_tail, one block per instance that has not converged.
constexpr int kGridNewton = 2;

// the first pass of a step evaluates at the previous step's converged state:
// its partials are what that step's adjoint needs (taken only on request)
rom_status tap_mpart(rom_batch* h, hipStream_t s) {
  ROM_HIP_CHECK(hipMemcpyAsync(h->mpart_tap, h->mpart,
                               h->esz * (size_t)std::max(h->n_ptiles, 1) * kMaxR * kMaxR,
                               hipMemcpyDeviceToDevice, s));
  return ROM_OK;
}

template <typename T>
rom_status galerkin_step_t(rom_batch* h, hipStream_t s) {
  const int r = h->cfg.r, B = h->cfg.n_inst;
  const int64_t nr = (int64_t)B * r;
  const int64_t nset = std::max<int64_t>(nr, B);
  double* gpart = h->part;
  if (mfma_ok(h)) {
    // the first iteration's kernels do the step's set-up (a_prev, active, iters)
    const int ng = std::min(kGridNewton, h->cfg.rom_max);
    for (int it = 0; it < ng; ++it) {
      const int first = it == 0 ? 1 : 0;
      rom_status st = launch_galerkin_mfma(h, s, first);
      if (st != ROM_OK) return st;
      if (first && h->mpart_tap) ROM_TRY(tap_mpart(h, s));
      if (r == 32)  // register-resident single-wave solve (r = 64 rows do not fit)
        hipLaunchKernelGGL(k_galerkin_solve_w<32>, dim3(B), dim3(64), 0, s, h->d_ptile_first,
                           gpart, (const float*)h->mpart, h->cfg.dt, h->d_var, h->a, h->a_prev,
                           h->active, h->iters, h->cfg.rom_tol, h->flags, first);
      else
        hipLaunchKernelGGL((k_galerkin_solve<float>), dim3(B), dim3(256), 0, s,
                           h->d_ptile_first, gpart, (const float*)h->mpart, r, h->cfg.dt,
                           h->d_var, h->a, h->a_prev, h->active, h->iters, h->cfg.rom_tol,
                           h->flags, first);
    }
    // remaining iterations and the non-convergence flag
    return launch_galerkin_tail(h, ng, s);
  }
  hipLaunchKernelGGL(k_rom_step_setup, dim3((nset + 255) / 256), dim3(256), 0, s, B, r, h->a,
                     h->a_prev, h->active, h->iters);
  for (int it = 0; it < h->cfg.rom_max; ++it) {
    hipLaunchKernelGGL((k_galerkin_pass<T>), dim3(h->n_ptiles), dim3(256), 0, s, h->d_ptiles,
                       h->d_dof_off, h->d_cell_off, h->d_phys, h->cfg.n_phys, (const T*)h->Phi,
                       r, (const T*)h->q_ref, h->d_var, h->a, h->active, gpart, (T*)h->mpart);
    if (it == 0 && h->mpart_tap) ROM_TRY(tap_mpart(h, s));
    hipLaunchKernelGGL((k_galerkin_solve<T>), dim3(B), dim3(256), 0, s, h->d_ptile_first, gpart,
                       (const T*)h->mpart, r, h->cfg.dt, h->d_var, h->a, h->a_prev, h->active,
                       h->iters, h->cfg.rom_tol, h->flags, 0);
  }
  hipLaunchKernelGGL(k_rom_finalize, dim3((B + 255) / 256), dim3(256), 0, s, B, h->active, h->flags);
  ROM_HIP_CHECK(hipGetLastError());
  return ROM_OK;
}


// ------------------------------------------------------------------ HR-LSPG step adjoint
// One HR-LSPG step backward (the sample rows P and M = (P^T Phi)^+ of its
// window held fixed).  At the converged a1 = a_{n+1} the weighted residual
// b(a) = M P^T D r(q~(a)) vanishes, and since M P^T Phi = I it equals
// (a - a_n) - dt M g(a) with g = P^T D f(q~).  The implicit-function theorem
// gives lambda = J_b^-T abar with the Gauss-Newton matrix J_b = M A_s,
// A_s = P^T D J_r D^-1 Phi; abar_n = lambda, and Phi, q_ref and D receive
// dt (d(M g)/d theta)^T lambda:
//   through M:  Abar = -M^T Mbar M^T + (I - A M) Mbar^T M M^T with Mbar = dt lambda g^T
//               and A = P^T Phi, i.e. dt (-(M^T lambda)(M g)^T + (g - A M g)(M M^T lambda)^T)
//               on the sampled rows of Phibar;
//   through g:  gbar = dt M^T lambda; dvbar[v_s] += gbar_s f_s; fbar_s = gbar_s d_s,
//               q~bar = J_f^T fbar on the three-cell mesh of each sampled row, and
//               q~ = q_ref + D^-1 Phi a1 gives qrbar += q~bar,
//               Phibar += D^-1 q~bar a1^T, dvbar[v] -= sum q~bar (Phi a1) / d^2.
// One block per instance.  Every mesh row is updated by one thread, which sums
// the contributions of the sampled rows in their order, so the result does
// not depend on scheduling.  as_ws: FP64 [n_inst][ns][r] scratch for A_s.
// Dynamic LDS: 2 ns 3 NV + r^2 + 4 ns + 3 r doubles.
template <class Mdl, typename T>
__global__ __launch_bounds__(256) void k_hr_step_vjp(
    int r, int ns, const int64_t* __restrict__ dof_off, const int64_t* __restrict__ cell_off,
    const double* __restrict__ phys, int nphys, const double* __restrict__ dvar,
    const T* __restrict__ Phi, const T* __restrict__ qref, const int32_t* __restrict__ P,
    const double* __restrict__ M, const double* __restrict__ a1, double dt,
    double* __restrict__ abar, double* __restrict__ phibar, double* __restrict__ qrbar,
    double* __restrict__ dvbar, double* __restrict__ as_ws, uint32_t* flags) {
  constexpr int NV = Mdl::NV;
  constexpr int E3 = 3 * NV;
  extern __shared__ double sm[];
  __shared__ double sa[kMaxR], red[4];
  __shared__ unsigned flacc;
  double* sq3 = sm;                 // mesh states
  double* sj = sq3 + ns * E3;       // J_f row entries of each sampled row
  double* Jt = sj + ns * E3;        // J_b^T, r x r
  double* sf = Jt + r * r;          // f at the sampled rows
  double* su = sf + ns;             // M^T lambda
  double* se = su + ns;             // g - A M g
  double* sg = se + ns;             // g = d f
  double* lam = sg + ns;            // lambda
  double* mg = lam + r;             // M g
  double* wv = mg + r;              // M M^T lambda
  const int b = blockIdx.x, tid = threadIdx.x, nt = blockDim.x;
  const int64_t base = dof_off[b];
  const int64_t n = cell_off[b + 1] - cell_off[b];
  Mdl m(phys + (size_t)b * nphys);
  const double* dv = dvar + (size_t)b * NV;
  const int32_t* Pb = P + (size_t)b * ns;
  const double* Mb = M + (size_t)b * r * ns;
  double* Ab = as_ws + (size_t)b * ns * r;
  auto mesh_cell = [&](int s_, int o) -> int64_t {
    int64_t c = Pb[s_] / NV - 1 + o;
    if (Mdl::periodic) c = c < 0 ? c + n : (c >= n ? c - n : c);
    else c = c < 0 ? 0 : (c >= n ? n - 1 : c);
    return c;
  };
  for (int k = tid; k < r; k += nt) sa[k] = a1[(size_t)b * r + k];
  if (tid == 0) flacc = 0;
  __syncthreads();
  // mesh states q~ = q_ref + D^-1 Phi a1
  for (int idx = tid; idx < ns * E3; idx += nt) {
    const int s_ = idx / E3, e = idx - s_ * E3, o = e / NV, w = e - o * NV;
    const int64_t g = base + mesh_cell(s_, o) * NV + w;
    double acc = 0.0;
    for (int k = 0; k < r; ++k) acc += (double)Phi[g * r + k] * sa[k];
    sq3[idx] = (double)qref[g] + acc / dv[w];
  }
  __syncthreads();
  // f and the J_f row of each sampled row
  for (int s_ = tid; s_ < ns; s_ += nt) {
    const int p = Pb[s_];
    double fv, jm[NV], j0[NV], jp[NV];
    unsigned fl = 0;
    hr_row(m, sq3 + s_ * E3, (int64_t)(p / NV), p % NV, n, fv, jm, j0, jp, fl);
    if (fl) atomicOr(&flacc, fl);
    sf[s_] = fv;
    sg[s_] = dv[p % NV] * fv;
    for (int w = 0; w < NV; ++w) {
      sj[s_ * E3 + w] = jm[w];
      sj[s_ * E3 + NV + w] = j0[w];
      sj[s_ * E3 + 2 * NV + w] = jp[w];
    }
  }
  __syncthreads();
  // A_s = P^T Phi - dt P^T D J_f D^-1 Phi (rows of the mesh)
  for (int idx = tid; idx < ns * r; idx += nt) {
    const int s_ = idx / r, k = idx - s_ * r;
    const int p = Pb[s_];
    double acc = 0.0;
    for (int o = 0; o < 3; ++o) {
      const int64_t g0 = base + mesh_cell(s_, o) * NV;
      for (int w = 0; w < NV; ++w)
        acc += sj[s_ * E3 + o * NV + w] * ((double)Phi[(g0 + w) * r + k] / dv[w]);
    }
    Ab[idx] = (double)Phi[(base + p) * r + k] - dt * dv[p % NV] * acc;
  }
  __syncthreads();
  // J_b^T = (M A_s)^T, lambda = J_b^-T abar
  for (int idx = tid; idx < r * r; idx += nt) {
    const int i = idx / r, k = idx - i * r;
    double acc = 0.0;
    for (int s_ = 0; s_ < ns; ++s_) acc += Mb[(size_t)i * ns + s_] * Ab[(size_t)s_ * r + k];
    Jt[k * r + i] = acc;
  }
  for (int k = tid; k < r; k += nt) lam[k] = abar[(size_t)b * r + k];
  __syncthreads();
  const int ok = block_lu_solve(Jt, r, lam, r);
  if (!ok && tid == 0) atomicOr(&flacc, (unsigned)ROM_FLAG_SINGULAR);
  // M g, M^T lambda, g - A M g, M M^T lambda
  for (int i = tid; i < r; i += nt) {
    double acc = 0.0;
    for (int s_ = 0; s_ < ns; ++s_) acc += Mb[(size_t)i * ns + s_] * sg[s_];
    mg[i] = acc;
  }
  for (int s_ = tid; s_ < ns; s_ += nt) {
    double acc = 0.0;
    for (int i = 0; i < r; ++i) acc += Mb[(size_t)i * ns + s_] * lam[i];
    su[s_] = acc;
  }
  __syncthreads();
  for (int s_ = tid; s_ < ns; s_ += nt) {
    const int64_t g = base + Pb[s_];
    double acc = 0.0;
    for (int k = 0; k < r; ++k) acc += (double)Phi[g * r + k] * mg[k];
    se[s_] = sg[s_] - acc;
  }
  for (int i = tid; i < r; i += nt) {
    double acc = 0.0;
    for (int s_ = 0; s_ < ns; ++s_) acc += Mb[(size_t)i * ns + s_] * su[s_];
    wv[i] = acc;
  }
  __syncthreads();
  // the mesh rows: each distinct mesh cell (its first occurrence in sampled-row,
  // slot order) is handled by one thread, over its NV rows
  double dva[12];
  for (int w = 0; w < 12; ++w) dva[w] = 0.0;
  for (int j = tid; j < ns * 3; j += nt) {
    const int sj0 = j / 3, oj = j - sj0 * 3;
    const int64_t cell = mesh_cell(sj0, oj);
    bool first = true;
    for (int i = 0; i < j && first; ++i)
      if (mesh_cell(i / 3, i - (i / 3) * 3) == cell) first = false;
    if (!first) continue;
    for (int w = 0; w < NV; ++w) {
      const int64_t lr = cell * NV + w, g = base + lr;
      double coef = 0.0;     // q~bar of this row
      int own = -1;          // the sampled row at this DOF, if any
      for (int s_ = 0; s_ < ns; ++s_) {
        const double fb = dt * su[s_] * dv[Pb[s_] % NV];
        for (int o = 0; o < 3; ++o)
          if (mesh_cell(s_, o) == cell) coef += fb * sj[s_ * E3 + o * NV + w];
        if (Pb[s_] == lr) own = s_;
      }
      double pa = 0.0;
      for (int k = 0; k < r; ++k) pa += (double)Phi[g * r + k] * sa[k];
      qrbar[g] += coef;
      for (int u = 0; u < 12; ++u)
        if (u == w) dva[u] -= coef * pa / (dv[w] * dv[w]);
      const double cd = coef / dv[w];
      for (int k = 0; k < r; ++k) {
        double add = cd * sa[k];
        if (own >= 0) add += dt * (-su[own] * mg[k] + se[own] * wv[k]);
        phibar[g * r + k] += add;
      }
      if (own >= 0)
        for (int u = 0; u < 12; ++u)
          if (u == w) dva[u] += dt * su[own] * sf[own];
    }
  }
  for (int w = 0; w < NV; ++w) {
    const double v = wave_sum_bfly(dva[w]);
    __syncthreads();
    if ((tid & 63) == 0) red[tid >> 6] = v;
    __syncthreads();
    if (tid == 0) {
      double s2 = 0.0;
      for (int q = 0; q < (nt >> 6); ++q) s2 += red[q];
      dvbar[(size_t)b * NV + w] += s2;
    }
  }
  for (int k = tid; k < r; k += nt) abar[(size_t)b * r + k] = lam[k];
  if (tid == 0 && flacc) atomicOr(&flags[b], flacc);
}

size_t hr_step_vjp_shm(int r, int ns, int nv) {
  return sizeof(double) * ((size_t)2 * ns * 3 * nv + (size_t)r * r + 4 * (size_t)ns + 3 * (size_t)r);
}

rom_status hr_step(rom_batch* h, hipStream_t s) {
  const int B = h->cfg.n_inst, r = h->cfg.r, ns = h->cfg.n_s;
  const int gpi = (ns + kHrRows - 1) / kHrRows;         // evaluation blocks per instance
  const int gpr = (r + kHrRedRows - 1) / kHrRedRows;    // reduction blocks per instance
  double* hr_ar = h->hr_as + (size_t)B * ns * (r + 1);
  const int nset = B * r > B ? B * r : B;
  hipLaunchKernelGGL(k_rom_step_setup, dim3((nset + 255) / 256), dim3(256), 0, s, B, r, h->a,
                     h->a_prev, h->active, h->iters);
  auto go = [&](auto tag) -> rom_status {
    using M = typename decltype(tag)::type;
    for (int it = 0; it < h->cfg.rom_max; ++it) {
      // the sampled-mesh basis is stored in the bulk precision
      if (h->cfg.precision == ROM_F32)
        hipLaunchKernelGGL((k_hr_eval<M, float>), dim3(B * gpi), dim3(kHrEvalThreads), 0, s, r,
                           ns, gpi, h->d_cell_off, h->d_phys, h->cfg.n_phys, h->P,
                           (const float*)h->mesh_phi, h->mesh_qref, h->d_var, h->a, h->a_prev,
                           h->cfg.dt, h->active, h->hr_as, h->flags);
      else
        hipLaunchKernelGGL((k_hr_eval<M, double>), dim3(B * gpi), dim3(kHrEvalThreads), 0, s, r,
                           ns, gpi, h->d_cell_off, h->d_phys, h->cfg.n_phys, h->P,
                           (const double*)h->mesh_phi, h->mesh_qref, h->d_var, h->a, h->a_prev,
                           h->cfg.dt, h->active, h->hr_as, h->flags);
      // register rows of the solve sized to r rounded up to 16 (40 for r = 33..40)
      hipLaunchKernelGGL(k_hr_reduce, dim3(B * gpr), dim3(kHrRedThreads), hr_reduce_shm(r, ns), s,
                         r, ns, gpr, h->M, h->hr_as, h->active, hr_ar);
      auto rsolve = r <= 16 ? k_hr_solve<16> : r <= 32 ? k_hr_solve<32>
                  : r <= 40 ? k_hr_solve<40> : r <= 48 ? k_hr_solve<48> : k_hr_solve<64>;
      hipLaunchKernelGGL(rsolve, dim3(B), dim3(256), 0, s, r, hr_ar, h->active, h->a, h->iters,
                         h->cfg.rom_tol, h->flags);
    }
    hipLaunchKernelGGL(k_rom_finalize, dim3((B + 255) / 256), dim3(256), 0, s, B, h->active,
                       h->flags);
    return ROM_OK;
  };
  rom_status st;
  switch (h->cfg.problem) {
    case ROM_BURGERS: st = go(Tag<BurgersModel<double>>{}); break;
    case ROM_EULER_RUSANOV: st = go(Tag<EulerModel<double, false>>{}); break;
    case ROM_EULER_HLLC: st = go(Tag<EulerModel<double, true>>{}); break;
    default: st = go(Tag<ReactModel<double>>{}); break;
  }
  ROM_HIP_CHECK(hipGetLastError());
  return st;
}

template <typename T>
rom_status rebuild_t(rom_batch* h, hipStream_t s) {
  const int r = h->cfg.r, ns = h->cfg.n_s, B = h->cfg.n_inst;
  if (h->cfg.hyper == ROM_HR_NONE) return ROM_OK;
  if (h->cfg.hyper != ROM_HR_DEIM) {   // QDEIM (and feature-guided sampling) in sample.hip
    ROM_TRY(launch_qdeim(h, s));
    hipLaunchKernelGGL((k_rebuild<T>), dim3(B), dim3(256), rebuild_shm(), s, r, ns, h->nv,
                       (h->cfg.problem == ROM_BURGERS || h->cfg.problem == ROM_REACT) ? 1 : 0,
                       h->d_dof_off, h->d_cell_off, (const T*)h->Phi, (const T*)h->q_ref, h->P,
                       h->M, (T*)h->mesh_phi, h->mesh_qref, h->flags);
    ROM_HIP_CHECK(hipGetLastError());
    return ROM_OK;
  }
  hipLaunchKernelGGL(k_bump, dim3(1), dim3(64), 0, s, h->d_epoch);
  hipLaunchKernelGGL((k_cols_transpose<T>), dim3(h->n_ptiles), dim3(256), 0, s, h->d_ptiles,
                     h->d_dof_off, (const T*)h->Phi, r, (T*)h->phi_cm);
  // S candidates per pass tile (the tuned split; 4 by default: 512 rows per block)
  const int S = h->deim_split;
  double* tval = h->part;
  int64_t* tidx = (int64_t*)(h->part + (size_t)S * h->n_ptiles);
  double* coef = h->rstate;  // per instance kMaxR coefficients
  for (int t = 0; t < ns; ++t) {
    const int j = t < r ? t : t - r;
    if constexpr (sizeof(T) == 4) {
      hipLaunchKernelGGL(k_deim_argmax_v4, dim3(h->n_ptiles * S), dim3(128), 0, s, h->d_ptiles,
                         h->d_dof_off, (const float*)h->phi_cm, r, j, coef, kMaxR, h->chosen,
                         h->d_epoch, S, tval, tidx);
    } else {
      hipLaunchKernelGGL((k_deim_argmax<T, 2>), dim3(h->n_ptiles * S), dim3(256), 0, s,
                         h->d_ptiles, h->d_dof_off, (const T*)h->phi_cm, r, j, coef, kMaxR,
                         h->chosen, h->d_epoch, S, tval, tidx);
    }
    hipLaunchKernelGGL((k_deim_select<T>), dim3(B), dim3(256), 0, s, h->d_ptile_first, S, tval, tidx,
                       h->d_dof_off, (const T*)h->Phi, r, ns, t, h->P, h->chosen, h->d_epoch, coef,
                       kMaxR, h->flags);
  }
  hipLaunchKernelGGL((k_rebuild<T>), dim3(B), dim3(256), rebuild_shm(), s, r, ns, h->nv,
                     (h->cfg.problem == ROM_BURGERS || h->cfg.problem == ROM_REACT) ? 1 : 0,
                     h->d_dof_off, h->d_cell_off, (const T*)h->Phi, (const T*)h->q_ref, h->P, h->M,
                     (T*)h->mesh_phi, h->mesh_qref, h->flags);
  ROM_HIP_CHECK(hipGetLastError());
  return ROM_OK;
}

template <typename T>
rom_status reconstruct_t(rom_batch* h, void* out, hipStream_t s) {
  hipLaunchKernelGGL((k_reconstruct<T>), dim3(h->n_ptiles), dim3(256), 0, s, h->d_ptiles,
                     h->d_dof_off, (const T*)h->Phi, h->cfg.r, (const T*)h->q_ref, h->d_var, h->nv,
                     h->a, (T*)out);
  ROM_HIP_CHECK(hipGetLastError());
  return ROM_OK;
}

}  // namespace

rom_status rom_kernels_prepare() {
  const int big = 160 * 1024 - 1024;
  auto vjp_attr = [&](const void* f) {
    return hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, big);
  };
  ROM_HIP_CHECK(vjp_attr((const void*)k_hr_step_vjp<BurgersModel<double>, float>));
  ROM_HIP_CHECK(vjp_attr((const void*)k_hr_step_vjp<BurgersModel<double>, double>));
  ROM_HIP_CHECK(vjp_attr((const void*)k_hr_step_vjp<EulerModel<double, false>, float>));
  ROM_HIP_CHECK(vjp_attr((const void*)k_hr_step_vjp<EulerModel<double, false>, double>));
  ROM_HIP_CHECK(vjp_attr((const void*)k_hr_step_vjp<EulerModel<double, true>, float>));
  ROM_HIP_CHECK(vjp_attr((const void*)k_hr_step_vjp<EulerModel<double, true>, double>));
  ROM_HIP_CHECK(vjp_attr((const void*)k_hr_step_vjp<ReactModel<double>, float>));
  ROM_HIP_CHECK(vjp_attr((const void*)k_hr_step_vjp<ReactModel<double>, double>));
  ROM_HIP_CHECK(hipFuncSetAttribute((const void*)k_rebuild<float>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)rebuild_shm()));
  ROM_HIP_CHECK(hipFuncSetAttribute((const void*)k_hr_reduce, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)hr_reduce_shm(kMaxR, kMaxNs)));
  ROM_HIP_CHECK(hipFuncSetAttribute((const void*)k_rebuild<double>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)rebuild_shm()));
  return ROM_OK;
}

rom_status launch_hr_step_vjp(rom_batch* h, const void* Phi, const int32_t* P, const double* M,
                              const double* a1, double* abar, double* phibar, double* qrbar,
                              double* dvbar, hipStream_t s) {
  const int B = h->cfg.n_inst, r = h->cfg.r, ns = h->cfg.n_s;
  const size_t shm = hr_step_vjp_shm(r, ns, h->nv);
  auto go = [&](auto tagT) -> rom_status {
    using T = typename decltype(tagT)::type;
    auto run = [&](auto tag) {
      using Mdl = typename decltype(tag)::type;
      hipLaunchKernelGGL((k_hr_step_vjp<Mdl, T>), dim3(B), dim3(256), shm, s, r, ns,
                         h->d_dof_off, h->d_cell_off, h->d_phys, h->cfg.n_phys, h->d_var,
                         (const T*)Phi, (const T*)h->q_ref, P, M, a1, h->cfg.dt, abar, phibar,
                         qrbar, dvbar, h->hr_as, h->flags);
    };
    switch (h->cfg.problem) {
      case ROM_BURGERS: run(Tag<BurgersModel<double>>{}); break;
      case ROM_EULER_RUSANOV: run(Tag<EulerModel<double, false>>{}); break;
      case ROM_EULER_HLLC: run(Tag<EulerModel<double, true>>{}); break;
      default: run(Tag<ReactModel<double>>{}); break;
    }
    ROM_HIP_CHECK(hipGetLastError());
    return ROM_OK;
  };
  if (h->cfg.precision == ROM_F64) return go(Tag<double>{});
  return go(Tag<float>{});
}

rom_status launch_rom_fine_step(rom_batch* h, hipStream_t s) {
  if (h->cfg.scheme == ROM_SCHEME_SSPRK43) return launch_hr_explicit_step(h, s);
  if (h->cfg.hyper != ROM_HR_NONE) return hr_step(h, s);
  if (h->cfg.problem != ROM_BURGERS) {
    set_error("the full (non-hyper-reduced) Galerkin step is implemented for Burgers only");
    return ROM_E_UNSUPPORTED;
  }
  return h->cfg.precision == ROM_F64 ? galerkin_step_t<double>(h, s) : galerkin_step_t<float>(h, s);
}

rom_status prepare_galerkin_pass(rom_batch* h, hipStream_t s) {
  const int B = h->cfg.n_inst;
  if (h->cfg.problem != ROM_BURGERS) return ROM_E_UNSUPPORTED;
  hipLaunchKernelGGL(k_fill_i32, dim3((B + 255) / 256), dim3(256), 0, s, h->active, 1, (int64_t)B);
  ROM_HIP_CHECK(hipGetLastError());
  return ROM_OK;
}

// One Galerkin pass over the basis (block partials only: no reduced state
// changes); prepare_galerkin_pass must have marked the instances active.
rom_status launch_galerkin_pass(rom_batch* h, hipStream_t s) {
  const int r = h->cfg.r;
  if (h->cfg.problem != ROM_BURGERS) return ROM_E_UNSUPPORTED;
  if (mfma_ok(h)) return launch_galerkin_mfma(h, s);
  if (h->cfg.precision == ROM_F64)
    hipLaunchKernelGGL((k_galerkin_pass<double>), dim3(h->n_ptiles), dim3(256), 0, s, h->d_ptiles,
                       h->d_dof_off, h->d_cell_off, h->d_phys, h->cfg.n_phys, (const double*)h->Phi,
                       r, (const double*)h->q_ref, h->d_var, h->a, h->active, h->part,
                       (double*)h->mpart);
  else
    hipLaunchKernelGGL((k_galerkin_pass<float>), dim3(h->n_ptiles), dim3(256), 0, s, h->d_ptiles,
                       h->d_dof_off, h->d_cell_off, h->d_phys, h->cfg.n_phys, (const float*)h->Phi,
                       r, (const float*)h->q_ref, h->d_var, h->a, h->active, h->part,
                       (float*)h->mpart);
  ROM_HIP_CHECK(hipGetLastError());
  return ROM_OK;
}

rom_status launch_rebuild(rom_batch* h, hipStream_t s) {
  ROM_TRY(h->cfg.precision == ROM_F64 ? rebuild_t<double>(h, s) : rebuild_t<float>(h, s));
  if (h->cfg.scheme == ROM_SCHEME_SSPRK43) ROM_TRY(launch_mesh5(h, s));
  return ROM_OK;
}

rom_status launch_reconstruct(rom_batch* h, void* out, hipStream_t s) {
  return h->cfg.precision == ROM_F64 ? reconstruct_t<double>(h, out, s)
                                     : reconstruct_t<float>(h, out, s);
}

}  // namespace romhip
