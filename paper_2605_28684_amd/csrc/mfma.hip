// MFMA (gfx950 matrix core) and wave-level kernels for the FP32 tall-skinny
// passes over the basis when r equals the tile width RT (32 or 64).
//
//  * Galerkin pass: per Newton iteration of the Galerkin step, one stream over
//    Phi computing Phi^T f (FP64) and Phi^T (J_f Phi) (FP32 MFMA,
//    v_mfma_f32_32x32x2f32).  J_f Phi is formed row by row from the three
//    Jacobian diagonals, never stored.
//  * iSVD rotation: Phi' = Phi Ubar[:r, :r] + s Ubar[r, :] with s the
//    normalised residual, as an MFMA product of 32-row tiles by Ubar.
//  * Projection pass: p = Phi^T y^ (and the second Gram-Schmidt pass) with
//    float4 loads, lanes mapped to columns, FP64 accumulation.
//
// Each wave owns a contiguous row range of its block's tile and its own LDS
// slice, so waves synchronise among their own lanes only (wave barrier with
// wavefront-scope fences); block barriers appear only in the final reduction of
// the four waves, which runs in a fixed order (bitwise reproducible results).
//
// MFMA 32x32x2 f32 operand layout (checked on the device): lane l supplies
// A[l % 32][l / 32] and B[l / 32][l % 32]; accumulator element v of lane l is
// D[(v / 4) * 8 + (l / 32) * 4 + v % 4][l % 32].
#include "internal.h"
#include "linalg.h"
#include "physics.h"

namespace romhip {

typedef float f32x16 __attribute__((ext_vector_type(16)));

namespace {

DEV void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

constexpr int kCh = 32;  // rows per wave chunk

// A wave-uniform double moved to scalar registers (frees two vector registers
// in loops that only read it).
DEV double uniform_d(double x) {
  const unsigned long long u = __builtin_bit_cast(unsigned long long, x);
  const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)u);
  const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(u >> 32));
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

DEV int64_t wrap_cell(int64_t c, int64_t n) { return c < 0 ? c + n : (c >= n ? c - n : c); }

// ------------------------------------------------------------------ Galerkin pass
constexpr int kGW = 4;  // waves per Galerkin block

// LDS of one Galerkin block (8 waves).  Basis rows are padded to RT + 4 floats:
// 16-byte aligned stores, and the row-wise reads of the reconstruction hit
// distinct banks.
template <int RT>
struct GalerkinLds {
  float sP[kGW][kCh + 2][RT + 4];  // basis rows of the wave's window (see galerkin_tile)
  double sQ[kGW][kCh + 2];         // q~ of those rows
  float4 sJ[kGW][kCh];             // (alpha, beta, gamma, 0) of the 32 output rows
  double sF[kGW][kCh];             // f of the 32 output rows
  double sa[RT];                   // the reduced state a (set by the caller)
  float redM[RT * RT];             // Phi^T J_f Phi of the tile
  double redG[RT];                 // Phi^T f of the tile
};

// Prefetch of one window of 32 basis rows (stream rows 32 j + 2 .. 32 j + 33
// of the wave, zero outside 0 .. m + 1) and of q_ref of those rows (lanes < 32).
// Cell indices are instance-local (below 2^31).
template <int RT, int NPF>
DEV void galerkin_fetch(const float* __restrict__ Pb, const float* __restrict__ qb, int s_cell,
                        int n, int m, int j, int lane, float4 (&pf)[NPF], float& pq) {
  constexpr int NQ = RT / 4;
  const int s0 = kCh * j + 2;
  const int c0 = s_cell + s0;
  if (s0 >= 0 && s0 + kCh - 1 <= m + 1 && c0 >= 0 && c0 + kCh - 1 < n) {
    // the usual case: all 32 rows present and contiguous (no wrap-around)
    const float4* src = reinterpret_cast<const float4*>(Pb + (int64_t)c0 * RT);
#pragma unroll
    for (int u = 0; u < NPF; ++u) pf[u] = src[lane + 64 * u];
    pq = qb[c0 + (lane & 31)];
    return;
  }
#pragma unroll
  for (int u = 0; u < NPF; ++u) {
    const int e = lane + 64 * u;
    const int s = s0 + e / NQ;
    float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
    if (s >= 0 && s <= m + 1) {
      int c = s_cell + s;
      c = c < 0 ? c + n : (c >= n ? c - n : c);
      v = *reinterpret_cast<const float4*>(Pb + (int64_t)c * RT + 4 * (e % NQ));
    }
    pf[u] = v;
  }
  const int s = s0 + (lane & 31);
  int c = s_cell + s;
  c = c < 0 ? c + n : (c >= n ? c - n : c);
  pq = (s >= 0 && s <= m + 1) ? qb[c] : 0.f;
}

// One block's share of a Galerkin pass: the rows of tile t (cells of one
// instance).  Each wave owns m consecutive output rows and streams the m + 2
// basis rows around them (its "stream": row s is cell lo - 1 + s) in windows
// of 32: the LDS window holds stream rows 32 j .. 32 j + 33, the first two
// carried over from the previous window, the other 32 prefetched into
// registers while the previous window is processed.  Per window: q~ = q_ref +
// Phi a / d in FP64 (two lanes per row), f(q~) and the three diagonals of J_f
// for the 32 output rows 32 j + 1 .. 32 j + 32, then Phi^T f (FP64) and
// Phi^T J_f Phi (v_mfma_f32_32x32x2f32, two rows per instruction).  Output
// rows past m get zero coefficients and add nothing.  The waves' sums are
// added in a fixed order into L.redM / L.redG.  L.sa must hold a; ends with a
// block barrier.
template <int RT>
DEV void galerkin_tile(const Tile& t, const double* __restrict__ phys, int nphys,
                       const float* __restrict__ Phi, const float* __restrict__ qref,
                       const double* __restrict__ dvar, GalerkinLds<RT>& L) {
  constexpr int NCB = RT / 32;
  constexpr int NQ = RT / 4;            // float4 per basis row
  constexpr int NPF = kCh * NQ / 64;    // float4 per lane per window
  constexpr int HC = RT / 2;            // columns per lane in the reconstruction
  constexpr int NT = 64 * kGW;
  const int b = t.inst;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int n = (int)t.n;
  const float* __restrict__ Pb = Phi + t.base * RT;
  const float* __restrict__ qb = qref + t.base;
  // per-instance constants, uniform over the block: kept in scalar registers
  const double nu = uniform_d(phys[(size_t)b * nphys]);
  const double dinv = uniform_d(1.0 / dvar[b]);
  const double inv = uniform_d((double)n), inv2 = uniform_d((double)n * (double)n);
  for (int c = tid; c < RT; c += NT) L.redG[c] = 0.0;
  for (int e = tid; e < RT * RT; e += NT) L.redM[e] = 0.f;
  __syncthreads();
  // this wave's output rows of the tile
  const int64_t per = ((t.ncell + kGW * kCh - 1) / (kGW * kCh)) * kCh;
  const int64_t lo = wave * per;
  const int m = (int)((lo + per < t.ncell ? lo + per : t.ncell) - lo);
  const int s_cell = (int)(t.cell0 + lo - 1);
  const int nwin = m > 0 ? (m + kCh - 1) / kCh : 0;
  const int par = lane >> 5, cl = lane & 31;
  f32x16 acc[NCB][NCB];
#pragma unroll
  for (int i = 0; i < NCB; ++i)
#pragma unroll
    for (int j = 0; j < NCB; ++j)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[i][j][v] = 0.f;
  double gacc[NCB];
#pragma unroll
  for (int i = 0; i < NCB; ++i) gacc[i] = 0.0;
  float(*P)[RT + 4] = L.sP[wave];
  double* Q = L.sQ[wave];
  float4 pf[NPF];
  float pq = 0.f;
  // window -1 brings stream rows 0 and 1 (into LDS rows 32, 33)
  if (nwin > 0) galerkin_fetch<RT, NPF>(Pb, qb, s_cell, n, m, -1, lane, pf, pq);
  for (int j = -1; j < nwin; ++j) {
    wave_sync();
    // carry rows 32, 33 to 0, 1, then store the prefetched rows into 2 .. 33
#pragma unroll
    for (int v = 0; v < 2 * RT / 64; ++v) {
      const int e = lane + 64 * v;
      const float x = P[kCh + e / RT][e % RT];
      P[e / RT][e % RT] = x;
    }
    if (lane < 2) Q[lane] = Q[kCh + lane];
#pragma unroll
    for (int u = 0; u < NPF; ++u) {
      const int e = lane + 64 * u;
      *reinterpret_cast<float4*>(&P[2 + e / NQ][4 * (e % NQ)]) = pf[u];
    }
    const float qr = pq;
    wave_sync();
    if (j + 1 < nwin) galerkin_fetch<RT, NPF>(Pb, qb, s_cell, n, m, j + 1, lane, pf, pq);
    // q~ of rows 2 .. 33: lanes r and r + 32 take the two halves of row 2 + r
    {
      const float* pr = &P[2 + cl][par * HC];
      const double* ar = &L.sa[par * HC];
      double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
#pragma unroll
      for (int c = 0; c < HC; c += 4) {
        const float4 p = *reinterpret_cast<const float4*>(pr + c);
        s0 += (double)p.x * ar[c];
        s1 += (double)p.y * ar[c + 1];
        s2 += (double)p.z * ar[c + 2];
        s3 += (double)p.w * ar[c + 3];
      }
      double s = (s0 + s1) + (s2 + s3);
      s += __shfl_xor(s, 32);
      if (par == 0) Q[2 + cl] = (double)qr + s * dinv;
    }
    wave_sync();
    if (j < 0) continue;
    // f and the Jacobian diagonals of output rows 1 .. 32 (stream 32 j + 1 ..)
    if (lane < kCh) {
      const int i = lane + 1;
      double f = 0.0, al = 0.0, be = 0.0, ga = 0.0;
      if (kCh * j + i <= m) {
        const double um = Q[i - 1], u0 = Q[i], up = Q[i + 1];
        double dla, dlb, dra, drb;
        const double FL = godunov(um, u0, dla, dlb);
        const double FR = godunov(u0, up, dra, drb);
        f = -(FR - FL) * inv + nu * ((up - u0) - (u0 - um)) * inv2;
        al = dla * inv + nu * inv2;
        be = (dlb - dra) * inv - 2.0 * nu * inv2;
        ga = -drb * inv + nu * inv2;
      }
      L.sF[wave][lane] = f;
      L.sJ[wave][lane] = make_float4((float)al, (float)be, (float)ga, 0.f);
    }
    wave_sync();
    // output row i = 2 k + 1 + par: A = Phi row i, Z = (J_f Phi) row i
    float pm[NCB];
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) pm[cb] = P[par][cb * 32 + cl];
#pragma unroll 4
    for (int k = 0; k < kCh / 2; ++k) {
      const int i = 2 * k + 1 + par;
      const float4 J = L.sJ[wave][i - 1];
      const double fr = L.sF[wave][i - 1];
      float A[NCB], Z[NCB];
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb) {
        const int col = cb * 32 + cl;
        const float p0 = P[i][col], pp = P[i + 1][col];
        A[cb] = p0;
        Z[cb] = J.x * pm[cb] + J.y * p0 + J.z * pp;
        gacc[cb] += (double)p0 * fr;
        pm[cb] = pp;
      }
#pragma unroll
      for (int ca = 0; ca < NCB; ++ca)
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb)
          acc[ca][cb] = __builtin_amdgcn_mfma_f32_32x32x2f32(A[ca], Z[cb], acc[ca][cb], 0, 0, 0);
    }
  }
  // combine the two row parities of Phi^T f, then the waves in order
#pragma unroll
  for (int cb = 0; cb < NCB; ++cb) gacc[cb] += __shfl_xor(gacc[cb], 32);
  for (int w = 0; w < kGW; ++w) {
    if (wave == w) {
#pragma unroll
      for (int ca = 0; ca < NCB; ++ca)
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
          for (int v = 0; v < 16; ++v) {
            const int i = ca * 32 + (v >> 2) * 8 + par * 4 + (v & 3);
            const int j = cb * 32 + cl;
            L.redM[i * RT + j] += acc[ca][cb][v];
          }
      if (par == 0) {
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) L.redG[cb * 32 + cl] += gacc[cb];
      }
    }
    __syncthreads();
  }
}

// r = 32: four blocks of four waves (16 waves) per CU, within the LDS and the
// 128-register budget, so the 2048-row tiles of the batched configuration fit
// in one round of the grid; r = 64: two blocks per CU (LDS).
template <int RT>
__global__ __launch_bounds__(64 * kGW)
__attribute__((amdgpu_waves_per_eu(RT == 32 ? 4 : 1))) void k_galerkin_mfma(
    const Tile* __restrict__ tiles, const int64_t* __restrict__ dof_off,
    const int64_t* __restrict__ cell_off, const double* __restrict__ phys, int nphys,
    const float* __restrict__ Phi, const float* __restrict__ qref,
    const double* __restrict__ dvar, const double* __restrict__ a,
    const int32_t* __restrict__ active, double* __restrict__ gpart, float* __restrict__ mpart,
    int first) {
  constexpr int NT = 64 * kGW;
  __shared__ GalerkinLds<RT> L;
  // the fine steps are the window's critical path: their waves win issue
  // arbitration against the event chain running beside them
  __builtin_amdgcn_s_setprio(3);
  const Tile t = tiles[blockIdx.x];
  const int b = t.inst;
  if (!first && !active[b]) return;   // the first iteration of a step runs every instance
  const int tid = threadIdx.x;
  for (int c = tid; c < RT; c += NT) L.sa[c] = a[(size_t)b * RT + c];
  galerkin_tile<RT>(t, phys, nphys, Phi, qref, dvar, L);
  float* mo = mpart + (size_t)blockIdx.x * kMaxR * kMaxR;
  if (RT == 32) {
    // in the order of the single-wave solve (mpart_pos32), written contiguously
    for (int d = tid; d < RT * RT; d += NT) {
      const int ln = (d >> 2) & 63, jj = 4 * (d >> 8) + (d & 3);
      mo[d] = L.redM[(ln & 31) * RT + 2 * jj + (ln >> 5)];
    }
  } else {
    for (int e = tid; e < RT * RT; e += NT) mo[e] = L.redM[e];
  }
  for (int c = tid; c < RT; c += NT) gpart[(size_t)blockIdx.x * kMaxR + c] = L.redG[c];
}

// Newton iterations it0 .. max_it-1 of the reduced backward-Euler step for the
// instances still active after the grid-wide iterations: one block per
// instance streams all of its rows (galerkin_tile on the whole instance),
// solves J_g delta = -g in FP64 (block LU with partial pivoting) and repeats
// until ||delta||_inf <= tol (1 + ||a||_inf) or max_it; a is kept in LDS and
// written back at the end.  Instances still unconverged get the ROM
// non-convergence flag.  Converged instances exit at once, so in the common
// case this is one cheap launch in place of the remaining iterations.
template <int RT>
__global__ __launch_bounds__(64 * kGW) void k_galerkin_tail(
    const int64_t* __restrict__ cell_off, const int64_t* __restrict__ dof_off,
    const double* __restrict__ phys, int nphys, const float* __restrict__ Phi,
    const float* __restrict__ qref, const double* __restrict__ dvar, double* __restrict__ a,
    const double* __restrict__ a_prev, int32_t* __restrict__ active, int32_t* __restrict__ iters,
    double dt, double tol, int it0, int max_it, uint32_t* __restrict__ flags) {
  constexpr int NT = 64 * kGW;
  constexpr int LDJ = RT + 1;
  __shared__ GalerkinLds<RT> L;
  __shared__ double J[RT * LDJ];
  __shared__ double g[RT], ap[RT];
  __shared__ int stop, nit;
  const int b = blockIdx.x, tid = threadIdx.x;
  if (!active[b]) return;
  Tile t;
  t.inst = b;
  t.pad = 0;
  t.cell0 = 0;
  t.ncell = cell_off[b + 1] - cell_off[b];
  t.n = t.ncell;
  t.base = dof_off[b];
  for (int c = tid; c < RT; c += NT) {
    L.sa[c] = a[(size_t)b * RT + c];
    ap[c] = a_prev[(size_t)b * RT + c];
  }
  if (tid == 0) { stop = 0; nit = 0; }
  const double dd = dvar[b];
  unsigned fl = 0;
  for (int it = it0; it < max_it; ++it) {
    galerkin_tile<RT>(t, phys, nphys, Phi, qref, dvar, L);
    for (int e = tid; e < RT * RT; e += NT) {
      const int i = e / RT, j = e % RT;
      J[i * LDJ + j] = (i == j ? 1.0 : 0.0) - dt * (double)L.redM[e];
    }
    for (int c = tid; c < RT; c += NT) g[c] = -(L.sa[c] - ap[c] - dt * dd * L.redG[c]);
    __syncthreads();
    const int ok = block_lu_solve(J, LDJ, g, RT);
    if (tid < 64) {
      double dm = 0.0, am = 0.0;
      int fin = 1;
      if (tid < RT) {
        const double an = L.sa[tid] + g[tid];
        L.sa[tid] = an;
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
        nit += 1;
        if (!ok) fl |= ROM_FLAG_SINGULAR;
        if (!fin) fl |= ROM_FLAG_NONFINITE;
        stop = (dm <= tol * (1.0 + am) || !fin) ? 1 : 0;
      }
    }
    __syncthreads();
    if (stop) break;
  }
  for (int c = tid; c < RT; c += NT) a[(size_t)b * RT + c] = L.sa[c];
  if (tid == 0) {
    iters[b] += nit;
    if (!stop) fl |= ROM_FLAG_ROM_NOCONV;
    else active[b] = 0;
    if (fl) atomicOr(&flags[b], fl);
  }
}

// ------------------------------------------------------------------ iSVD rotation
// dst[i, :] <- Phi[i, :] U[:r, :r] + s_i U[r, :],  s_i = (q1_i - Phi[i, :] p2) / rho;
// dst may be Phi (in place: every row is read before it is written, by the same
// wave).  pr holds (p1, p2, 1/rho) per instance with stride 2r + 2.
template <int RT>
__global__ __launch_bounds__(256) void k_rotate_mfma(const Tile* __restrict__ tiles,
                                                     const int64_t* __restrict__ dof_off,
                                                     const float* Phi, float* dst,
                                                     const double* __restrict__ U,
                                                     const double* __restrict__ q1,
                                                     const double* __restrict__ pr) {
  constexpr int NCB = RT / 32;
  constexpr int LDP = RT + 1;
  constexpr int n = RT + 1;           // core size
  __shared__ float sP[4][kCh][LDP];
  __shared__ float sS[4][kCh];
  __shared__ float sU[n][RT];
  __shared__ double sp2[RT];
  __shared__ double irho;
  const Tile t = tiles[blockIdx.x];
  const int b = t.inst;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int64_t base = dof_off[b];
  const double* Ub = U + (size_t)b * n * n;
  for (int e = tid; e < n * RT; e += 256) sU[e / RT][e % RT] = (float)Ub[(e / RT) * n + (e % RT)];
  for (int c = tid; c < RT; c += 256) sp2[c] = pr[(size_t)b * (2 * RT + 2) + RT + c];
  if (tid == 0) irho = pr[(size_t)b * (2 * RT + 2) + 2 * RT];
  __syncthreads();
  const int64_t per = ((t.ncell + 4 * kCh - 1) / (4 * kCh)) * kCh;
  const int64_t lo = wave * per;
  const int64_t hi = lo + per < t.ncell ? lo + per : t.ncell;
  const int par = lane >> 5, cl = lane & 31;
  float(*P)[LDP] = sP[wave];
  for (int64_t r0 = lo; r0 < hi; r0 += kCh) {
    const int nr = (int)(hi - r0 < kCh ? hi - r0 : kCh);
    const int64_t g0 = base + t.cell0 + r0;
    for (int e4 = lane; e4 < kCh * (RT / 4); e4 += 64) {
      const int row = e4 / (RT / 4), col = (e4 % (RT / 4)) * 4;
      float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
      if (row < nr) v = *reinterpret_cast<const float4*>(Phi + (g0 + row) * RT + col);
      P[row][col] = v.x; P[row][col + 1] = v.y; P[row][col + 2] = v.z; P[row][col + 3] = v.w;
    }
    wave_sync();
    if (lane < kCh) {
      float sv = 0.f;
      if (lane < nr) {
        double d2 = 0.0;
#pragma unroll 8
        for (int c = 0; c < RT; ++c) d2 += (double)P[lane][c] * sp2[c];
        sv = (float)((q1[g0 + lane] - d2) * irho);
      }
      sS[wave][lane] = sv;
    }
    wave_sync();
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) {
      f32x16 acc;
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int i = (v >> 2) * 8 + par * 4 + (v & 3);
        acc[v] = sS[wave][i] * sU[RT][cb * 32 + cl];
      }
#pragma unroll 4
      for (int k0 = 0; k0 < RT; k0 += 2) {
        const float av = P[cl][k0 + par];               // A[i = row][k]
        const float bv = sU[k0 + par][cb * 32 + cl];    // B[k][j = col]
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(av, bv, acc, 0, 0, 0);
      }
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int i = (v >> 2) * 8 + par * 4 + (v & 3);
        if (i < nr) dst[(g0 + i) * RT + cb * 32 + cl] = acc[v];
      }
    }
    wave_sync();
  }
}

// The same rotation for r = 32 with no LDS: since Phi U[:r, :r] + s U[r, :]
// with s = (q1 - Phi p2) / rho equals Phi U' + (q1 / rho) U[r, :] for
// U' = U[:r, :r] - p2 U[r, :] / rho, each wave keeps its share of U' in
// registers (formed once in FP64, rounded to FP32) and feeds the basis rows
// straight from HBM to the matrix cores.  The MFMA's reduction index (the
// basis column) is ordered so that lane (c, h) of a 32-row chunk supplies row
// c, columns 16 h .. 16 h + 15: four float4 loads per lane (the other waves of
// the SIMD keep memory busy meanwhile; at most 80 registers, so that the
// fine steps' single-wave solve still finds room beside four of these waves
// on every SIMD while the rotation runs beside them).  A 17th product adds the
// rank-one term: lane (c, 0) supplies q1 / rho of row c against U[r, :], lane
// (c, 1) zero.  dst may be Phi (each wave reads a chunk's rows before it
// writes them and never touches another wave's rows).
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(6)))
void k_rotate_mfma_reg(const Tile* __restrict__ tiles,
                                                         const int64_t* __restrict__ dof_off,
                                                         const float* Phi, float* dst,
                                                         const double* __restrict__ U,
                                                         const double* __restrict__ q1,
                                                         const double* __restrict__ pr) {
  constexpr int RT = 32;
  constexpr int n = RT + 1;   // core size
  const Tile t = tiles[blockIdx.x];
  const int b = t.inst;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int par = lane >> 5, cl = lane & 31;
  const int64_t base = dof_off[b];
  const double* Ub = U + (size_t)b * n * n;
  const double* p2 = pr + (size_t)b * (2 * RT + 2) + RT;
  const double irho = pr[(size_t)b * (2 * RT + 2) + 2 * RT];
  // B operands: U'[16 par + s][cl] for s = 0 .. 15, and U[r][cl] for the
  // rank-one step (lane (c, 1) supplies the zero row)
  const double ur = Ub[RT * n + cl];
  float bU[16];
#pragma unroll
  for (int s2 = 0; s2 < 16; ++s2) {
    const int k = 16 * par + s2;
    bU[s2] = (float)(Ub[k * n + cl] - p2[k] * irho * ur);
  }
  const float bR = par == 0 ? (float)ur : 0.f;
  const int64_t per = ((t.ncell + 4 * kCh - 1) / (4 * kCh)) * kCh;
  const int64_t lo = wave * per;
  const int64_t hi = lo + per < t.ncell ? lo + per : t.ncell;
  if (lo >= hi) return;
  const float* src = Phi + (base + t.cell0) * RT;
  const double* q1b = q1 + base + t.cell0;
  float* out = dst + (base + t.cell0) * RT;
  // one chunk's operands of this lane: row lo + 32 j + cl, columns 16 par ..
  auto fetch = [&](int64_t r0, float4 (&v)[4], double& q) {
    const int64_t row = r0 + cl;
    if (row < hi) {
      const float4* p = reinterpret_cast<const float4*>(src + row * RT + 16 * par);
#pragma unroll
      for (int u = 0; u < 4; ++u) v[u] = p[u];
      q = par == 0 ? q1b[row] : 0.0;
    } else {
#pragma unroll
      for (int u = 0; u < 4; ++u) v[u] = make_float4(0.f, 0.f, 0.f, 0.f);
      q = 0.0;
    }
  };
  for (int64_t r0 = lo; r0 < hi; r0 += kCh) {
    float4 cur[4];
    double qc;
    fetch(r0, cur, qc);
    f32x16 acc;
#pragma unroll
    for (int v = 0; v < 16; ++v) acc[v] = 0.f;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      acc = __builtin_amdgcn_mfma_f32_32x32x2f32(cur[u].x, bU[4 * u + 0], acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_32x32x2f32(cur[u].y, bU[4 * u + 1], acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_32x32x2f32(cur[u].z, bU[4 * u + 2], acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_32x32x2f32(cur[u].w, bU[4 * u + 3], acc, 0, 0, 0);
    }
    acc = __builtin_amdgcn_mfma_f32_32x32x2f32((float)(qc * irho), bR, acc, 0, 0, 0);
    const int nr = (int)(hi - r0 < kCh ? hi - r0 : kCh);
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int i = (v >> 2) * 8 + par * 4 + (v & 3);
      if (i < nr) out[(r0 + i) * RT + cl] = acc[v];
    }
  }
}

// ------------------------------------------------------------------ projection pass
// mode 1: part[c] = sum_i Phi_ic y^_i, part[RT] = |y^|^2
// mode 2: q1_i = y^_i - Phi_i . p1 (stored to q1out); part[c] = sum Phi_ic q1_i, part[RT] = |q1|^2
template <int RT>
__global__ __launch_bounds__(256) void k_project_fast(
    const Tile* __restrict__ tiles, const int64_t* __restrict__ dof_off,
    const float* __restrict__ Phi, const float* __restrict__ y, const float* __restrict__ qref,
    const double* __restrict__ dvar, int nv, const double* __restrict__ p1, int ldp, int mode,
    double* __restrict__ part, int pst, double* __restrict__ q1out) {
  constexpr int LPR = RT / 4;          // lanes per row (float4 each)
  constexpr int RPW = 64 / LPR;        // rows per wave load
  __shared__ double red[4][RT + 1];
  const Tile t = tiles[blockIdx.x];
  const int b = t.inst;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int64_t base = dof_off[b];
  const double* dv = dvar + (size_t)b * nv;
  const int sub = lane % LPR, rsub = lane / LPR;
  double pc[4] = {0.0, 0.0, 0.0, 0.0};
  if (mode == 2) {
#pragma unroll
    for (int q = 0; q < 4; ++q) pc[q] = p1[(size_t)b * ldp + sub * 4 + q];
  }
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  double accn = 0.0;
  const int64_t per = ((t.ncell + 4 * RPW - 1) / (4 * RPW)) * RPW;
  const int64_t lo = wave * per;
  const int64_t hi = lo + per < t.ncell ? lo + per : t.ncell;
  for (int64_t r0 = lo; r0 < hi; r0 += RPW) {
    const int64_t lr = t.cell0 + r0 + rsub;      // instance-local row of this lane
    const bool live = r0 + rsub < hi;
    float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
    double yh = 0.0;
    if (live) {
      const int64_t g = base + lr;
      v = *reinterpret_cast<const float4*>(Phi + g * RT + sub * 4);
      yh = dv[lr % nv] * ((double)y[g] - (double)qref[g]);
    }
    const double ph[4] = {(double)v.x, (double)v.y, (double)v.z, (double)v.w};
    if (mode == 2) {
      double d = ph[0] * pc[0] + ph[1] * pc[1] + ph[2] * pc[2] + ph[3] * pc[3];
#pragma unroll
      for (int off = 1; off < LPR; off <<= 1) d += __shfl_xor(d, off);
      yh -= d;
      if (live && sub == 0) q1out[base + lr] = yh;
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[q] += ph[q] * yh;
    if (sub == 0) accn += yh * yh;
  }
  // lanes with the same column group: xor over the row-subgroup bits
#pragma unroll
  for (int off = LPR; off < 64; off <<= 1) {
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[q] += __shfl_xor(acc[q], off);
    accn += __shfl_xor(accn, off);
  }
  if (lane < LPR) {
#pragma unroll
    for (int q = 0; q < 4; ++q) red[wave][lane * 4 + q] = acc[q];
  }
  // accn: only sub == 0 lanes accumulated; the xor tree summed them into every lane
  if (lane == 0) red[wave][RT] = accn;
  __syncthreads();
  double* out = part + (size_t)blockIdx.x * pst;
  for (int c = tid; c <= RT; c += 256) out[c] = red[0][c] + red[1][c] + red[2][c] + red[3][c];
}

}  // namespace

bool mfma_ok(const rom_batch* h) {
  return h->cfg.precision == ROM_F32 && (h->cfg.r == 32 || h->cfg.r == 64);
}

rom_status launch_galerkin_mfma(rom_batch* h, hipStream_t s, int first) {
  if (h->cfg.r == 32)
    hipLaunchKernelGGL((k_galerkin_mfma<32>), dim3(h->n_ptiles), dim3(64 * kGW), 0, s, h->d_ptiles,
                       h->d_dof_off, h->d_cell_off, h->d_phys, h->cfg.n_phys, (const float*)h->Phi,
                       (const float*)h->q_ref, h->d_var, h->a, h->active, h->part,
                       (float*)h->mpart, first);
  else
    hipLaunchKernelGGL((k_galerkin_mfma<64>), dim3(h->n_ptiles), dim3(64 * kGW), 0, s, h->d_ptiles,
                       h->d_dof_off, h->d_cell_off, h->d_phys, h->cfg.n_phys, (const float*)h->Phi,
                       (const float*)h->q_ref, h->d_var, h->a, h->active, h->part,
                       (float*)h->mpart, first);
  ROM_HIP_CHECK(hipGetLastError());
  return ROM_OK;
}

rom_status launch_galerkin_tail(rom_batch* h, int it0, hipStream_t s) {
  auto go = [&](auto kern) {
    hipLaunchKernelGGL(kern, dim3(h->cfg.n_inst), dim3(64 * kGW), 0, s, h->d_cell_off,
                       h->d_dof_off, h->d_phys, h->cfg.n_phys, (const float*)h->Phi,
                       (const float*)h->q_ref, h->d_var, h->a, h->a_prev, h->active, h->iters,
                       h->cfg.dt, h->cfg.rom_tol, it0, h->cfg.rom_max, h->flags);
  };
  if (h->cfg.r == 32) go(k_galerkin_tail<32>);
  else go(k_galerkin_tail<64>);
  ROM_HIP_CHECK(hipGetLastError());
  return ROM_OK;
}

rom_status launch_rotate_mfma(rom_batch* h, const double* pr, void* dst, hipStream_t s) {
  if (h->cfg.r == 32)
    hipLaunchKernelGGL(k_rotate_mfma_reg, dim3(h->n_ptiles), dim3(256), 0, s, h->d_ptiles,
                       h->d_dof_off, (const float*)h->Phi, (float*)dst, h->ubar, h->qtmp, pr);
  else
    hipLaunchKernelGGL((k_rotate_mfma<64>), dim3(h->n_ptiles), dim3(256), 0, s, h->d_ptiles,
                       h->d_dof_off, (const float*)h->Phi, (float*)dst, h->ubar, h->qtmp, pr);
  ROM_HIP_CHECK(hipGetLastError());
  return ROM_OK;
}

rom_status launch_project_fast(rom_batch* h, const void* y, const double* p1, int ldp, int mode,
                               double* part, int pst, double* q1out, hipStream_t s) {
  if (h->cfg.r == 32)
    hipLaunchKernelGGL((k_project_fast<32>), dim3(h->n_ptiles), dim3(256), 0, s, h->d_ptiles,
                       h->d_dof_off, (const float*)h->Phi, (const float*)y, (const float*)h->q_ref,
                       h->d_var, h->nv, p1, ldp, mode, part, pst, q1out);
  else
    hipLaunchKernelGGL((k_project_fast<64>), dim3(h->n_ptiles), dim3(256), 0, s, h->d_ptiles,
                       h->d_dof_off, (const float*)h->Phi, (const float*)y, (const float*)h->q_ref,
                       h->d_var, h->nv, p1, ldp, mode, part, pst, q1out);
  ROM_HIP_CHECK(hipGetLastError());
  return ROM_OK;
}

}  // namespace romhip
