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

DEV int64_t wrap_cell(int64_t c, int64_t n) { return c < 0 ? c + n : (c >= n ? c - n : c); }

// ------------------------------------------------------------------ Galerkin pass
constexpr int kGW = 8;  // waves per Galerkin block

// LDS of one Galerkin block (8 waves).
template <int RT>
struct GalerkinLds {
  float sP[kGW][kCh + 2][RT + 1];
  double sQ[kGW][kCh + 2];
  double sF[kGW][kCh];
  float sAl[kGW][kCh], sBe[kGW][kCh], sGa[kGW][kCh];
  double sa[RT];        // the reduced state a (set by the caller)
  float redM[RT * RT];  // Phi^T J_f Phi of the tile
  double redG[RT];      // Phi^T f of the tile
};

// One block's share of a Galerkin pass: the rows of tile t (cells of one
// instance).  Each wave streams its row range in 32-row chunks (next chunk
// prefetched into registers, staged through LDS): q~ = q_ref + Phi a / d in
// FP64, f(q~) and the three diagonals of J_f, then Phi^T f (FP64) and
// Phi^T J_f Phi (v_mfma_f32_32x32x2f32).  The waves' sums are added in a fixed
// order into L.redM / L.redG.  L.sa must hold a; ends with a block barrier.
template <int RT>
DEV void galerkin_tile(const Tile& t, const double* __restrict__ phys, int nphys,
                       const float* __restrict__ Phi, const float* __restrict__ qref,
                       const double* __restrict__ dvar, GalerkinLds<RT>& L) {
  constexpr int NCB = RT / 32;
  constexpr int LDP = RT + 1;
  constexpr int NV4 = (kCh + 2) * (RT / 4);       // float4 per chunk (with halo)
  constexpr int NPF = (NV4 + 63) / 64;            // float4 per lane
  constexpr int NT = 64 * kGW;
  const int b = t.inst;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int64_t n = t.n;
  const int64_t base = t.base;
  const double nu = phys[(size_t)b * nphys];
  const double dinv = 1.0 / dvar[b];
  const double inv = (double)n, inv2 = (double)n * (double)n;
  for (int c = tid; c < RT; c += NT) L.redG[c] = 0.0;
  for (int e = tid; e < RT * RT; e += NT) L.redM[e] = 0.f;
  for (int e = tid; e < kGW * (kCh + 2) * LDP; e += NT) (&L.sP[0][0][0])[e] = 0.f;
  __syncthreads();
  // this wave's rows of the tile
  const int64_t per = ((t.ncell + kGW * kCh - 1) / (kGW * kCh)) * kCh;
  const int64_t lo = wave * per;
  const int64_t hi = lo + per < t.ncell ? lo + per : t.ncell;
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
  float(*P)[LDP] = L.sP[wave];
  // register prefetch of one chunk: basis rows c0-1 .. c0+nr and q_ref of those rows
  float4 pf[NPF];
  float pq = 0.f;
  auto fetch = [&](int64_t r0) {
    const int nr = (int)(hi - r0 < kCh ? hi - r0 : kCh);
    const int64_t c0 = t.cell0 + r0;
#pragma unroll
    for (int u = 0; u < NPF; ++u) {
      const int e4 = lane + 64 * u;
      if (e4 < (nr + 2) * (RT / 4)) {
        const int row = e4 / (RT / 4), col = (e4 % (RT / 4)) * 4;
        const int64_t cell = wrap_cell(c0 - 1 + row, n);
        pf[u] = *reinterpret_cast<const float4*>(Phi + (base + cell) * RT + col);
      }
    }
    if (lane < nr + 2) pq = qref[base + wrap_cell(c0 - 1 + lane, n)];
  };
  if (lo < hi) fetch(lo);
  for (int64_t r0 = lo; r0 < hi; r0 += kCh) {
    const int nr = (int)(hi - r0 < kCh ? hi - r0 : kCh);
#pragma unroll
    for (int u = 0; u < NPF; ++u) {
      const int e4 = lane + 64 * u;
      if (e4 < (nr + 2) * (RT / 4)) {
        const int row = e4 / (RT / 4), col = (e4 % (RT / 4)) * 4;
        P[row][col] = pf[u].x; P[row][col + 1] = pf[u].y;
        P[row][col + 2] = pf[u].z; P[row][col + 3] = pf[u].w;
      }
    }
    const double qr = (double)pq;
    wave_sync();
    if (r0 + kCh < hi) fetch(r0 + kCh);     // overlaps the compute below
    if (lane < nr + 2) {
      double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
#pragma unroll 2
      for (int c = 0; c < RT; c += 4) {
        s0 += (double)P[lane][c] * L.sa[c];
        s1 += (double)P[lane][c + 1] * L.sa[c + 1];
        s2 += (double)P[lane][c + 2] * L.sa[c + 2];
        s3 += (double)P[lane][c + 3] * L.sa[c + 3];
      }
      L.sQ[wave][lane] = qr + ((s0 + s1) + (s2 + s3)) * dinv;
    }
    wave_sync();
    if (lane < kCh) {
      double f = 0.0, al = 0.0, be = 0.0, ga = 0.0;
      if (lane < nr) {
        const double um = L.sQ[wave][lane], u0 = L.sQ[wave][lane + 1], up = L.sQ[wave][lane + 2];
        double dla, dlb, dra, drb;
        const double FL = godunov(um, u0, dla, dlb);
        const double FR = godunov(u0, up, dra, drb);
        f = -(FR - FL) * inv + nu * ((up - u0) - (u0 - um)) * inv2;
        al = dla * inv + nu * inv2;
        be = (dlb - dra) * inv - 2.0 * nu * inv2;
        ga = -drb * inv + nu * inv2;
      }
      L.sF[wave][lane] = f;
      L.sAl[wave][lane] = (float)al;
      L.sBe[wave][lane] = (float)be;
      L.sGa[wave][lane] = (float)ga;
    }
    wave_sync();
#pragma unroll 4
    for (int k = 0; k < kCh / 2; ++k) {
      const int row = 2 * k + par;
      const bool live = row < nr;
      const float al = L.sAl[wave][row], be = L.sBe[wave][row], ga = L.sGa[wave][row];
      const double fr = L.sF[wave][row];
      float A[NCB], Z[NCB];
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb) {
        const int col = cb * 32 + cl;
        const float p0 = P[row + 1][col];
        A[cb] = live ? p0 : 0.f;
        Z[cb] = live ? (al * P[row][col] + be * p0 + ga * P[row + 2][col]) : 0.f;
        gacc[cb] += (double)A[cb] * fr;
      }
#pragma unroll
      for (int ca = 0; ca < NCB; ++ca)
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb)
          acc[ca][cb] = __builtin_amdgcn_mfma_f32_32x32x2f32(A[ca], Z[cb], acc[ca][cb], 0, 0, 0);
    }
    wave_sync();
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

template <int RT>
__global__ __launch_bounds__(64 * kGW) void k_galerkin_mfma(
    const Tile* __restrict__ tiles, const int64_t* __restrict__ dof_off,
    const int64_t* __restrict__ cell_off, const double* __restrict__ phys, int nphys,
    const float* __restrict__ Phi, const float* __restrict__ qref,
    const double* __restrict__ dvar, const double* __restrict__ a,
    const int32_t* __restrict__ active, double* __restrict__ gpart, float* __restrict__ mpart) {
  constexpr int NT = 64 * kGW;
  __shared__ GalerkinLds<RT> L;
  const Tile t = tiles[blockIdx.x];
  const int b = t.inst;
  if (!active[b]) return;
  const int tid = threadIdx.x;
  for (int c = tid; c < RT; c += NT) L.sa[c] = a[(size_t)b * RT + c];
  galerkin_tile<RT>(t, phys, nphys, Phi, qref, dvar, L);
  float* mo = mpart + (size_t)blockIdx.x * kMaxR * kMaxR;
  for (int e = tid; e < RT * RT; e += NT) mo[e] = L.redM[e];
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
// Phi[i, :] <- Phi[i, :] U[:r, :r] + s_i U[r, :],  s_i = (q1_i - Phi[i, :] p2) / rho,
// in place.  pr holds (p1, p2, 1/rho) per instance with stride 2r + 2.
template <int RT>
__global__ __launch_bounds__(256) void k_rotate_mfma(const Tile* __restrict__ tiles,
                                                     const int64_t* __restrict__ dof_off,
                                                     float* Phi, const double* __restrict__ U,
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
        if (i < nr) Phi[(g0 + i) * RT + cb * 32 + cl] = acc[v];
      }
    }
    wave_sync();
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

rom_status launch_galerkin_mfma(rom_batch* h, hipStream_t s) {
  if (h->cfg.r == 32)
    hipLaunchKernelGGL((k_galerkin_mfma<32>), dim3(h->n_ptiles), dim3(64 * kGW), 0, s, h->d_ptiles,
                       h->d_dof_off, h->d_cell_off, h->d_phys, h->cfg.n_phys, (const float*)h->Phi,
                       (const float*)h->q_ref, h->d_var, h->a, h->active, h->part,
                       (float*)h->mpart);
  else
    hipLaunchKernelGGL((k_galerkin_mfma<64>), dim3(h->n_ptiles), dim3(64 * kGW), 0, s, h->d_ptiles,
                       h->d_dof_off, h->d_cell_off, h->d_phys, h->cfg.n_phys, (const float*)h->Phi,
                       (const float*)h->q_ref, h->d_var, h->a, h->active, h->part,
                       (float*)h->mpart);
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

rom_status launch_rotate_mfma(rom_batch* h, const double* pr, hipStream_t s) {
  if (h->cfg.r == 32)
    hipLaunchKernelGGL((k_rotate_mfma<32>), dim3(h->n_ptiles), dim3(256), 0, s, h->d_ptiles,
                       h->d_dof_off, (float*)h->Phi, h->ubar, h->qtmp, pr);
  else
    hipLaunchKernelGGL((k_rotate_mfma<64>), dim3(h->n_ptiles), dim3(256), 0, s, h->d_ptiles,
                       h->d_dof_off, (float*)h->Phi, h->ubar, h->qtmp, pr);
  ROM_HIP_CHECK(hipGetLastError());
  return ROM_OK;
}

rom_status launch_project_fast(rom_batch* h, const void* y, const double* p1, int ldp, int mode,
                               int pst, double* q1out, hipStream_t s) {
  if (h->cfg.r == 32)
    hipLaunchKernelGGL((k_project_fast<32>), dim3(h->n_ptiles), dim3(256), 0, s, h->d_ptiles,
                       h->d_dof_off, (const float*)h->Phi, (const float*)y, (const float*)h->q_ref,
                       h->d_var, h->nv, p1, ldp, mode, h->part, pst, q1out);
  else
    hipLaunchKernelGGL((k_project_fast<64>), dim3(h->n_ptiles), dim3(256), 0, s, h->d_ptiles,
                       h->d_dof_off, (const float*)h->Phi, (const float*)y, (const float*)h->q_ref,
                       h->d_var, h->nv, p1, ldp, mode, h->part, pst, q1out);
  ROM_HIP_CHECK(hipGetLastError());
  return ROM_OK;
}

}  // namespace romhip
