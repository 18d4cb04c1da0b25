// Direct solver for the block-tridiagonal Newton systems of the backward-Euler
// full-order step (periodic models give cyclic systems, walls give plain ones):
//     A_i x_{i-1} + B_i x_i + C_i x_{i+1} = d_i,   i = 0..n-1 (indices cyclic),
// with NV x NV blocks; for wall problems A_0 = C_{n-1} = 0.
//
// Method: recursive Schur complement on part separators.  Each instance is cut
// into parts of m consecutive cells whose last cell is a separator.  One thread
// eliminates the m-1 interior cells of its part by block Thomas, expressing
// them as x_j = g_j - V_j x_{sep left} - W_j x_{sep right} (the first interior
// cell's expression is accumulated during the same forward sweep).  Substituting the
// first/last interior expressions into the separator rows gives a system of the
// same block-tridiagonal (cyclic) form over the separators, which is solved the
// same way until one cell per instance remains; back-substitution then walks the
// levels down.  Work is O(n NV^3); every level is one launch over all instances.
#include <algorithm>

#include "internal.h"
#include "physics.h"

namespace romhip {

namespace {

template <typename T, int NV>
DEV void mm(const T* A, const T* B, T* C) {  // C = A B
#pragma unroll
  for (int i = 0; i < NV; ++i)
#pragma unroll
    for (int j = 0; j < NV; ++j) {
      T s = T(0);
#pragma unroll
      for (int k = 0; k < NV; ++k) s += A[i * NV + k] * B[k * NV + j];
      C[i * NV + j] = s;
    }
}
template <typename T, int NV>
DEV void mv(const T* A, const T* x, T* y) {  // y = A x
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    T s = T(0);
#pragma unroll
    for (int k = 0; k < NV; ++k) s += A[i * NV + k] * x[k];
    y[i] = s;
  }
}

// Gauss-Jordan inverse with partial pivoting; returns false if singular.
template <typename T, int NV>
DEV bool inv_block(const T* A, T* X) {
  T a[NV * NV];
#pragma unroll
  for (int e = 0; e < NV * NV; ++e) { a[e] = A[e]; X[e] = (e % (NV + 1)) == 0 ? T(1) : T(0); }
  bool ok = true;
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    int p = k;
    T best = fabs(a[k * NV + k]);
#pragma unroll
    for (int i = k + 1; i < NV; ++i) {
      const T v = fabs(a[i * NV + k]);
      if (v > best) { best = v; p = i; }
    }
#pragma unroll
    for (int i = k + 1; i < NV; ++i) {
      if (i == p) {
#pragma unroll
        for (int j = 0; j < NV; ++j) {
          T t = a[k * NV + j]; a[k * NV + j] = a[i * NV + j]; a[i * NV + j] = t;
          t = X[k * NV + j]; X[k * NV + j] = X[i * NV + j]; X[i * NV + j] = t;
        }
      }
    }
    const T piv = a[k * NV + k];
    if (!(piv != T(0))) ok = false;
    const T ip = ok ? T(1) / piv : T(0);
#pragma unroll
    for (int j = 0; j < NV; ++j) { a[k * NV + j] *= ip; X[k * NV + j] *= ip; }
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      if (i == k) continue;
      const T fct = a[i * NV + k];
#pragma unroll
      for (int j = 0; j < NV; ++j) {
        a[i * NV + j] -= fct * a[k * NV + j];
        X[i * NV + j] -= fct * X[k * NV + j];
      }
    }
  }
  return ok;
}

// v from another lane by one DPP control (whole rows, every bank), for 32- and
// 64-bit types.
template <int CTRL, typename T>
DEV T dpp_mov(T v) {
  if constexpr (sizeof(T) == 4) {
    return __builtin_bit_cast(T, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), CTRL, 0xF,
                                                          0xF, false));
  } else {
    const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
    const int lo = __builtin_amdgcn_mov_dpp((int)(unsigned)u, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp((int)(unsigned)(u >> 32), CTRL, 0xF, 0xF, false);
    return __builtin_bit_cast(T, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
  }
}

// The largest v over each 16-lane row of the wavefront, in every lane of the
// row (v never NaN): the quad, then the other quad of the half row (mirrored
// within 8 lanes), then the other half (mirrored within 16).
template <typename T>
DEV T row16_max(T v) {
  T o = dpp_mov<0xB1>(v);   // quad_perm [1,0,3,2]
  v = o > v ? o : v;
  o = dpp_mov<0x4E>(v);     // quad_perm [2,3,0,1]
  v = o > v ? o : v;
  o = dpp_mov<0x141>(v);    // row_half_mirror
  v = o > v ? o : v;
  o = dpp_mov<0x140>(v);    // row_mirror
  return o > v ? o : v;
}

DEV int find_inst(const int64_t* off, int n_inst, int64_t g) {
  int lo = 0, hi = n_inst;  // off[lo] <= g < off[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (off[mid] <= g) lo = mid; else hi = mid;
  }
  return lo;
}

template <typename T, int NV>
struct Lay {
  static constexpr int NN = NV * NV;
  static constexpr int SYS = 3 * NN + NV;   // A, B, C, d
  static constexpr int FWD = 2 * NN + NV;   // Chat, Vhat, ghat
  static constexpr int PRT = 3 * NN + NV;   // What_last, V_first, W_first, g_first
};

// Forward elimination of the interior of each part and the affine expression of
// its first interior cell.
template <typename T, int NV>
__global__ __launch_bounds__(256) void k_bt_factor(int n_inst, const int64_t* __restrict__ cell_off,
                                                   const int64_t* __restrict__ part_off, int m,
                                                   const T* __restrict__ sys, T* __restrict__ fwd,
                                                   T* __restrict__ prt, const int32_t* active,
                                                   uint32_t* flags) {
  using L = Lay<T, NV>;
  constexpr int NN = L::NN;
  const int64_t gp = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gp >= part_off[n_inst]) return;
  const int b = find_inst(part_off, n_inst, gp);
  if (active && !active[b]) return;
  const int64_t k = gp - part_off[b];
  const int64_t n = cell_off[b + 1] - cell_off[b];
  const int64_t first = k * m;
  const int64_t s = (first + m < n ? first + m : n) - 1;
  const int64_t len = s - first;  // interior cells
  if (len <= 0) return;
  const int64_t base = cell_off[b];
  T Ch[NN], Vh[NN], gh[NV], Bt[NN], Bi[NN], tmp[NN], tv[NV], Pm[NN], ga[NV], Va[NN];
  bool ok = true;
#pragma unroll
  for (int e = 0; e < NN; ++e) { Pm[e] = (e % (NV + 1)) == 0 ? T(1) : T(0); Va[e] = T(0); }
#pragma unroll
  for (int v = 0; v < NV; ++v) ga[v] = T(0);
  // the next cell's row blocks are loaded while the current cell is
  // eliminated (the loads do not depend on the recursion)
  T A[NN], B[NN], C[NN], d[NV], nx[3 * NN + NV];
  auto load_cell = [&](int64_t jj) {
    const T* S = sys + (base + jj) * L::SYS;
#pragma unroll
    for (int e = 0; e < 3 * NN + NV; ++e) nx[e] = S[e];
  };
  load_cell(first);
  for (int64_t j = first; j < s; ++j) {
#pragma unroll
    for (int e = 0; e < NN; ++e) { A[e] = nx[e]; B[e] = nx[NN + e]; C[e] = nx[2 * NN + e]; }
#pragma unroll
    for (int v = 0; v < NV; ++v) d[v] = nx[3 * NN + v];
    if (j + 1 < s) load_cell(j + 1);
    if (j == first) {
#pragma unroll
      for (int e = 0; e < NN; ++e) Bt[e] = B[e];
      ok &= inv_block<T, NV>(Bt, Bi);
      mv<T, NV>(Bi, d, gh);
      mm<T, NV>(Bi, A, Vh);
    } else {
      mm<T, NV>(A, Ch, tmp);
#pragma unroll
      for (int e = 0; e < NN; ++e) Bt[e] = B[e] - tmp[e];
      ok &= inv_block<T, NV>(Bt, Bi);
      mv<T, NV>(A, gh, tv);
#pragma unroll
      for (int v = 0; v < NV; ++v) tv[v] = d[v] - tv[v];
      mv<T, NV>(Bi, tv, gh);
      mm<T, NV>(A, Vh, tmp);
      mm<T, NV>(Bi, tmp, Vh);
#pragma unroll
      for (int e = 0; e < NN; ++e) Vh[e] = -Vh[e];
    }
    mm<T, NV>(Bi, C, Ch);  // Chat_j, or What_last at the last interior cell
    T* F = fwd + (base + j) * L::FWD;
#pragma unroll
    for (int e = 0; e < NN; ++e) { F[e] = Ch[e]; F[NN + e] = Vh[e]; }
#pragma unroll
    for (int v = 0; v < NV; ++v) F[2 * NN + v] = gh[v];
    // the first interior cell's expression, accumulated on the way forward:
    // x_first = sum_j P_j (ghat_j - Vhat_j x_L) + P_len x_R with P_0 = I and
    // P_{j+1} = -P_j Chat_j (Chat of the last interior cell is What_last)
    mv<T, NV>(Pm, gh, tv);
#pragma unroll
    for (int v = 0; v < NV; ++v) ga[v] += tv[v];
    mm<T, NV>(Pm, Vh, tmp);
#pragma unroll
    for (int e = 0; e < NN; ++e) Va[e] += tmp[e];
    mm<T, NV>(Pm, Ch, tmp);
#pragma unroll
    for (int e = 0; e < NN; ++e) Pm[e] = -tmp[e];
  }
  T* Pp = prt + (part_off[b] + k) * L::PRT;
#pragma unroll
  for (int e = 0; e < NN; ++e) {
    Pp[e] = Ch[e];            // What_last
    Pp[NN + e] = Va[e];       // V_first
    Pp[2 * NN + e] = -Pm[e];  // W_first
  }
#pragma unroll
  for (int v = 0; v < NV; ++v) Pp[3 * NN + v] = ga[v];   // g_first
  if (!ok) atomicOr(&flags[b], ROM_FLAG_SINGULAR);
}

// The same elimination for large blocks, where one thread's state (several NV x NV
// blocks) would not fit in registers.  A group of 16 lanes eliminates one part:
// lane i owns row i of every block, and whole blocks are shared through LDS.  At
// each cell the group forms the augmented rows [B - A Chat | C | A Vhat | d - A ghat]
// (at the first cell [B | C | A | d]) and reduces them by Gauss-Jordan with
// partial pivoting, which leaves Chat, -Vhat (+Vhat at the first cell) and ghat in
// the right-hand columns.  Pivot rows stay with the lane that holds them, so after
// the reduction lane i holds the row of the solution numbered by the step at which
// it was chosen.  The loops run the longest part's trip count on every group, so
// control flow, and every barrier, is uniform across the block.
template <typename T, int NV>
__global__ __launch_bounds__(64) void k_bt_factor_rows(int n_inst, const int64_t* __restrict__ cell_off,
                                                       const int64_t* __restrict__ part_off, int m,
                                                       const T* __restrict__ sys, T* __restrict__ fwd,
                                                       T* __restrict__ prt, const int32_t* active,
                                                       uint32_t* flags) {
  static_assert(NV <= 16, "one row per lane of a 16-lane group");
  using L = Lay<T, NV>;
  constexpr int NN = L::NN;
  constexpr int NA = 3 * NV + 1;   // augmented row: [Bt | C | X | y]
  constexpr int GP = 4;            // parts (16-lane groups) per block
  __shared__ T sC[GP][NN];         // Chat of the last cell (W in the backward sweep)
  __shared__ T sV[GP][NN];         // Vhat of the last cell (V in the backward sweep)
  __shared__ T sg[GP][NV];         // ghat of the last cell (g in the backward sweep)
  __shared__ T sp[GP][2][NA];      // scaled pivot row, double-buffered
  const int grp = threadIdx.x >> 4;
  const int i = threadIdx.x & 15;
  const bool row = i < NV;
  const int64_t gp = (int64_t)blockIdx.x * GP + grp;
  bool live = gp < part_off[n_inst];
  int b = 0;
  int64_t k = 0, first = 0, len = 0, base = 0;
  if (live) {
    b = find_inst(part_off, n_inst, gp);
    live = !(active && !active[b]);
  }
  if (live) {
    k = gp - part_off[b];
    const int64_t n = cell_off[b + 1] - cell_off[b];
    first = k * m;
    const int64_t s = (first + m < n ? first + m : n) - 1;
    len = s - first;
    base = cell_off[b];
    live = len > 0;
  }
  T* Pp = prt + (live ? (part_off[b] + k) * L::PRT : 0);
  bool ok = true;
  for (int t = 0; t < m - 1; ++t) {
    const bool act = live && t < len;
    const bool mine = act && row;
    T aug[NA], arow[NV];
#pragma unroll
    for (int e = 0; e < NA; ++e) aug[e] = T(0);
#pragma unroll
    for (int c = 0; c < NV; ++c) arow[c] = T(0);
    if (mine) {
      const T* S = sys + (base + first + t) * L::SYS;
#pragma unroll
      for (int c = 0; c < NV; ++c) {
        arow[c] = S[i * NV + c];
        aug[c] = S[NN + i * NV + c];
        aug[NV + c] = S[2 * NN + i * NV + c];
      }
      aug[3 * NV] = S[3 * NN + i];
    }
    if (t == 0) {
#pragma unroll
      for (int c = 0; c < NV; ++c) aug[2 * NV + c] = arow[c];
    } else {
      // rows of the previous cell's Chat, Vhat, ghat were written to LDS and a
      // barrier followed
#pragma unroll
      for (int c = 0; c < NV; ++c) {
        T s1 = T(0), s2 = T(0);
#pragma unroll
        for (int q = 0; q < NV; ++q) {
          s1 += arow[q] * sC[grp][q * NV + c];
          s2 += arow[q] * sV[grp][q * NV + c];
        }
        aug[c] -= s1;
        aug[2 * NV + c] = s2;
      }
      T s3 = T(0);
#pragma unroll
      for (int q = 0; q < NV; ++q) s3 += arow[q] * sg[grp][q];
      aug[3 * NV] -= s3;
    }
    // Gauss-Jordan over the group's rows
    bool done = !row;
    int myrow = 0;
#pragma unroll
    for (int kk = 0; kk < NV; ++kk) {
      const T a = aug[kk];
      // the pivot: the group's lowest lane holding its largest key (a group
      // is one 16-lane DPP row; an unchosen row always has key >= 0)
      const T key = done ? T(-1) : (isnan(a) ? T(INFINITY) : fabs(a));
      const T kmax = row16_max(key);
      const int kl = __builtin_ctz((unsigned)(__ballot(key == kmax) >> (16 * grp)) & 0xFFFFu);
      if (act && !(kmax != T(0))) ok = false;
      if (i == kl) {
        const T ip = a != T(0) ? T(1) / a : T(0);
#pragma unroll
        for (int c = kk + 1; c < NA; ++c) {
          aug[c] *= ip;
          sp[grp][kk & 1][c] = aug[c];
        }
        done = true;
        myrow = kk;
      }
      __syncthreads();
      if (i != kl) {
#pragma unroll
        for (int c = kk + 1; c < NA; ++c) aug[c] -= a * sp[grp][kk & 1][c];
      }
    }
    const T sgn = t == 0 ? T(1) : T(-1);
    if (mine) {
      T* F = fwd + (base + first + t) * L::FWD;
#pragma unroll
      for (int c = 0; c < NV; ++c) {
        F[myrow * NV + c] = aug[NV + c];
        F[NN + myrow * NV + c] = sgn * aug[2 * NV + c];
        sC[grp][myrow * NV + c] = aug[NV + c];
        sV[grp][myrow * NV + c] = sgn * aug[2 * NV + c];
      }
      F[2 * NN + myrow] = aug[3 * NV];
      sg[grp][myrow] = aug[3 * NV];
      if (t == len - 1) {
#pragma unroll
        for (int c = 0; c < NV; ++c) Pp[myrow * NV + c] = aug[NV + c];   // What of the last cell
      }
    }
    __syncthreads();
  }
  // Backward sweep for the first interior cell, starting from the last cell's
  // (Vhat, Chat, ghat): g = ghat_j - Chat_j g, V = Vhat_j - Chat_j V, W = -Chat_j W.
  for (int t = m - 3; t >= 0; --t) {
    const bool mine = live && row && t <= len - 2;
    T vn[NV], wn[NV], gn = T(0);
    if (mine) {
      const T* F = fwd + (base + first + t) * L::FWD;
      T crow[NV];
#pragma unroll
      for (int q = 0; q < NV; ++q) crow[q] = F[i * NV + q];
#pragma unroll
      for (int c = 0; c < NV; ++c) {
        T s1 = T(0), s2 = T(0);
#pragma unroll
        for (int q = 0; q < NV; ++q) {
          s1 += crow[q] * sV[grp][q * NV + c];
          s2 += crow[q] * sC[grp][q * NV + c];
        }
        vn[c] = F[NN + i * NV + c] - s1;
        wn[c] = -s2;
      }
      T s3 = T(0);
#pragma unroll
      for (int q = 0; q < NV; ++q) s3 += crow[q] * sg[grp][q];
      gn = F[2 * NN + i] - s3;
    }
    __syncthreads();
    if (mine) {
#pragma unroll
      for (int c = 0; c < NV; ++c) {
        sV[grp][i * NV + c] = vn[c];
        sC[grp][i * NV + c] = wn[c];
      }
      sg[grp][i] = gn;
    }
    __syncthreads();
  }
  if (live && row) {
#pragma unroll
    for (int c = 0; c < NV; ++c) {
      Pp[NN + i * NV + c] = sV[grp][i * NV + c];
      Pp[2 * NN + i * NV + c] = sC[grp][i * NV + c];
    }
    Pp[3 * NN + i] = sg[grp][i];
    if (!ok) atomicOr(&flags[b], ROM_FLAG_SINGULAR);
  }
}

// Separator rows -> next level's system.
template <typename T, int NV>
__global__ __launch_bounds__(256) void k_bt_reduce(int n_inst, const int64_t* __restrict__ cell_off,
                                                   const int64_t* __restrict__ part_off, int m,
                                                   const T* __restrict__ sys, const T* __restrict__ fwd,
                                                   const T* __restrict__ prt,
                                                   const int64_t* __restrict__ next_off,
                                                   T* __restrict__ nsys, const int32_t* active) {
  using L = Lay<T, NV>;
  constexpr int NN = L::NN;
  const int64_t gp = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gp >= part_off[n_inst]) return;
  const int b = find_inst(part_off, n_inst, gp);
  if (active && !active[b]) return;
  const int64_t k = gp - part_off[b];
  const int64_t P = part_off[b + 1] - part_off[b];
  const int64_t n = cell_off[b + 1] - cell_off[b];
  const int64_t base = cell_off[b];
  const int64_t first = k * m;
  const int64_t s = (first + m < n ? first + m : n) - 1;
  const T* S = sys + (base + s) * L::SYS;
  const T* As = S;
  const T* Bs = S + NN;
  const T* Cs = S + 2 * NN;
  const T* ds = S + 3 * NN;
  T Ah[NN], Bh[NN], Chh[NN], dh[NV], tmp[NN], tv[NV];
#pragma unroll
  for (int e = 0; e < NN; ++e) Bh[e] = Bs[e];
#pragma unroll
  for (int v = 0; v < NV; ++v) dh[v] = ds[v];
  // left neighbour x_{s-1}: last interior of this part, or the previous separator
  if (s > first) {
    const T* F = fwd + (base + s - 1) * L::FWD;          // ghat_l, Vhat_l
    const T* Pp = prt + (part_off[b] + k) * L::PRT;       // What_l
    mm<T, NV>(As, F + NN, tmp);
#pragma unroll
    for (int e = 0; e < NN; ++e) Ah[e] = -tmp[e];
    mm<T, NV>(As, Pp, tmp);
#pragma unroll
    for (int e = 0; e < NN; ++e) Bh[e] -= tmp[e];
    mv<T, NV>(As, F + 2 * NN, tv);
#pragma unroll
    for (int v = 0; v < NV; ++v) dh[v] -= tv[v];
  } else {
#pragma unroll
    for (int e = 0; e < NN; ++e) Ah[e] = As[e];
  }
  // right neighbour x_{s+1}: first interior of the next part, or the next separator
  const int64_t k1 = (k + 1) % P;
  const int64_t f1 = k1 * m;
  const int64_t s1 = (f1 + m < n ? f1 + m : n) - 1;
  if (s1 > f1) {
    const T* Pn = prt + (part_off[b] + k1) * L::PRT;      // V_first, W_first, g_first
    mm<T, NV>(Cs, Pn + NN, tmp);
#pragma unroll
    for (int e = 0; e < NN; ++e) Bh[e] -= tmp[e];
    mm<T, NV>(Cs, Pn + 2 * NN, tmp);
#pragma unroll
    for (int e = 0; e < NN; ++e) Chh[e] = -tmp[e];
    mv<T, NV>(Cs, Pn + 3 * NN, tv);
#pragma unroll
    for (int v = 0; v < NV; ++v) dh[v] -= tv[v];
  } else {
#pragma unroll
    for (int e = 0; e < NN; ++e) Chh[e] = Cs[e];
  }
  T* O = nsys + (next_off[b] + k) * L::SYS;
#pragma unroll
  for (int e = 0; e < NN; ++e) { O[e] = Ah[e]; O[NN + e] = Bh[e]; O[2 * NN + e] = Chh[e]; }
#pragma unroll
  for (int v = 0; v < NV; ++v) O[3 * NN + v] = dh[v];
}

// One cell per instance: (A + B + C) x = d (its neighbours are itself).
template <typename T, int NV>
__global__ void k_bt_top(int n_inst, const int64_t* __restrict__ cell_off, const T* __restrict__ sys,
                         T* __restrict__ x, const int32_t* active, uint32_t* flags) {
  using L = Lay<T, NV>;
  constexpr int NN = L::NN;
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= n_inst) return;
  if (active && !active[b]) return;
  const T* S = sys + cell_off[b] * L::SYS;
  T M[NN], Mi[NN];
#pragma unroll
  for (int e = 0; e < NN; ++e) M[e] = S[e] + S[NN + e] + S[2 * NN + e];
  if (!inv_block<T, NV>(M, Mi)) atomicOr(&flags[b], ROM_FLAG_SINGULAR);
  mv<T, NV>(Mi, S + 3 * NN, x + cell_off[b] * NV);
}

// Back-substitution of one level given the separator values (next level's x).
// mode 0: write x; mode 1: add x into upd (level 0 of a Newton step).
template <typename T, int NV>
__global__ __launch_bounds__(256) void k_bt_back(int n_inst, const int64_t* __restrict__ cell_off,
                                                 const int64_t* __restrict__ part_off, int m,
                                                 const T* __restrict__ fwd, const T* __restrict__ prt,
                                                 const int64_t* __restrict__ next_off,
                                                 const T* __restrict__ xs, T* __restrict__ x,
                                                 const int64_t* __restrict__ dof_off, T* upd, int mode,
                                                 const int32_t* active, uint64_t* dnorm) {
  using L = Lay<T, NV>;
  constexpr int NN = L::NN;
  const int64_t gp = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  // no early return: the update norm is reduced across the wavefront below
  const bool inb = gp < part_off[n_inst];
  const int b = inb ? find_inst(part_off, n_inst, gp) : -1;
  const bool live = inb && !(active && !active[b]);
  double dmax = 0.0;
  if (live) {
  const int64_t k = gp - part_off[b];
  const int64_t P = part_off[b + 1] - part_off[b];
  const int64_t n = cell_off[b + 1] - cell_off[b];
  const int64_t base = cell_off[b];
  const int64_t first = k * m;
  const int64_t s = (first + m < n ? first + m : n) - 1;
  T xl[NV], xr[NV], xn[NV], tv[NV], tw[NV];
  const int64_t kl = k == 0 ? P - 1 : k - 1;
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    xl[v] = xs[(next_off[b] + kl) * NV + v];
    xr[v] = xs[(next_off[b] + k) * NV + v];
  }
  auto emit = [&](int64_t j, const T* val) {
    if (mode == 0) {
#pragma unroll
      for (int v = 0; v < NV; ++v) x[(base + j) * NV + v] = val[v];
    } else {
      T* u = upd + dof_off[b] + j * NV;
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        u[v] += val[v];
        dmax = fmax(dmax, fabs((double)val[v]));
      }
    }
  };
  emit(s, xr);
  if (s > first) {
    const T* Pp = prt + (part_off[b] + k) * L::PRT;
    const T* F = fwd + (base + s - 1) * L::FWD;
    // x_l = ghat_l - Vhat_l xl - What_l xr
    mv<T, NV>(F + NN, xl, tv);
    mv<T, NV>(Pp, xr, tw);
#pragma unroll
    for (int v = 0; v < NV; ++v) xn[v] = F[2 * NN + v] - tv[v] - tw[v];
    emit(s - 1, xn);
    if constexpr (NV <= 3) {
      // the next cell's forward factors (and, in update mode, its old values)
      // are loaded while the current cell is solved: they do not depend on it
      T g[L::FWD], ng[L::FWD], uo[NV], nu[NV];
      auto load_cell = [&](int64_t jj) {
        const T* G = fwd + (base + jj) * L::FWD;
#pragma unroll
        for (int e = 0; e < L::FWD; ++e) ng[e] = G[e];
        if (mode != 0) {
          const T* u = upd + dof_off[b] + jj * NV;
#pragma unroll
          for (int v = 0; v < NV; ++v) nu[v] = u[v];
        }
      };
      if (s - 2 >= first) load_cell(s - 2);
      for (int64_t j = s - 2; j >= first; --j) {
#pragma unroll
        for (int e = 0; e < L::FWD; ++e) g[e] = ng[e];
#pragma unroll
        for (int v = 0; v < NV; ++v) uo[v] = nu[v];
        if (j - 1 >= first) load_cell(j - 1);
        mv<T, NV>(g + NN, xl, tv);
        mv<T, NV>(g, xn, tw);
#pragma unroll
        for (int v = 0; v < NV; ++v) xn[v] = g[2 * NN + v] - tv[v] - tw[v];
        if (mode == 0) {
#pragma unroll
          for (int v = 0; v < NV; ++v) x[(base + j) * NV + v] = xn[v];
        } else {
          T* u = upd + dof_off[b] + j * NV;
#pragma unroll
          for (int v = 0; v < NV; ++v) {
            u[v] = uo[v] + xn[v];
            dmax = fmax(dmax, fabs((double)xn[v]));
          }
        }
      }
    } else {
      for (int64_t j = s - 2; j >= first; --j) {
        const T* G = fwd + (base + j) * L::FWD;
        mv<T, NV>(G + NN, xl, tv);
        mv<T, NV>(G, xn, tw);
#pragma unroll
        for (int v = 0; v < NV; ++v) xn[v] = G[2 * NN + v] - tv[v] - tw[v];
        emit(j, xn);
      }
    }
  }
  }
  if (dnorm && mode == 1) {
    const uint64_t bits = !live ? 0ull
                          : isfinite(dmax) ? (uint64_t)__double_as_longlong(dmax) : ~0ull;
    // one atomic per wavefront when all its live lanes belong to one instance
    const int b0 = __builtin_amdgcn_readfirstlane(b);
    if (__all(!live || b == b0) && b0 >= 0) wave_atomic_max(&dnorm[b0], bits);
    else if (live) atomicMax((unsigned long long*)&dnorm[b], (unsigned long long)bits);
  }
}

template <typename T>
size_t esz() { return sizeof(T); }

// Cells per part.  The part size trades the parallelism of a level against the
// work of the upper levels: 16 for small blocks (one thread per part); 8 for the
// 12 x 12 blocks, whose parts are eliminated by 16-lane groups.
int bt_part_size(int nv) { return nv >= 8 ? 8 : 16; }

template <typename T, int NV>
rom_status bt_solve_t(rom_batch* h, int it, void* upd, void* out, hipStream_t s) {
  using L = Lay<T, NV>;
  const int B = h->cfg.n_inst;
  const int32_t* act = it >= 0 ? h->active : nullptr;
  const int nl = (int)h->levels.size();
  for (int l = 0; l + 1 < nl; ++l) {
    auto& lv = h->levels[l];
    auto& nx = h->levels[l + 1];
    const int nb = (int)((lv.parts_total + 255) / 256);
    if constexpr (NV >= 8) {
      const int ng = (int)((lv.parts_total + 3) / 4);
      hipLaunchKernelGGL((k_bt_factor_rows<T, NV>), dim3(ng), dim3(64), 0, s, B, lv.d_cell_off,
                         lv.d_part_off, h->bt_m, (const T*)lv.sys, (T*)lv.fwd, (T*)lv.part, act,
                         h->flags);
    } else {
      hipLaunchKernelGGL((k_bt_factor<T, NV>), dim3(nb), dim3(256), 0, s, B, lv.d_cell_off,
                         lv.d_part_off, h->bt_m, (const T*)lv.sys, (T*)lv.fwd, (T*)lv.part, act,
                         h->flags);
    }
    hipLaunchKernelGGL((k_bt_reduce<T, NV>), dim3(nb), dim3(256), 0, s, B, lv.d_cell_off,
                       lv.d_part_off, h->bt_m, (const T*)lv.sys, (const T*)lv.fwd,
                       (const T*)lv.part, nx.d_cell_off, (T*)nx.sys, act);
  }
  auto& top = h->levels[nl - 1];
  hipLaunchKernelGGL((k_bt_top<T, NV>), dim3((B + 63) / 64), dim3(64), 0, s, B, top.d_cell_off,
                     (const T*)top.sys, (T*)top.x, act, h->flags);
  for (int l = nl - 2; l >= 0; --l) {
    auto& lv = h->levels[l];
    auto& nx = h->levels[l + 1];
    const int nb = (int)((lv.parts_total + 255) / 256);
    const bool last = l == 0;
    T* xout = last && out ? (T*)out : (T*)lv.x;
    const int mode = last && upd ? 1 : 0;
    if (last && !upd && out) {
      // the plain solve writes the solution in the state layout (cell-major == level-0 layout
      // only when offsets coincide, which holds because level 0 uses the DOF ordering)
    }
    uint64_t* dn = (last && it >= 0)
                       ? h->norms + (size_t)(2 * (h->cfg.newton_max + 1) + it) * B
                       : nullptr;
    hipLaunchKernelGGL((k_bt_back<T, NV>), dim3(nb), dim3(256), 0, s, B, lv.d_cell_off,
                       lv.d_part_off, h->bt_m, (const T*)lv.fwd, (const T*)lv.part,
                       nx.d_cell_off, (const T*)nx.x, xout, h->d_dof_off, (T*)upd, mode, act, dn);
  }
  (void)sizeof(L);
  ROM_HIP_CHECK(hipGetLastError());
  return ROM_OK;
}

}  // namespace

int bt_part_candidates(int nv, int* out) {
  if (nv >= 8) {   // the 16-lane row elimination of the 12-variable blocks uses 8
    out[0] = 8;
    return 1;
  }
  out[0] = 16;
  out[1] = 8;
  out[2] = 32;
  return 3;
}

rom_status bt_setup(rom_batch* h) {
  const int B = h->cfg.n_inst;
  const size_t es = h->esz;
  const int NV = h->nv;
  const int NN = NV * NV;
  const int pm = h->bt_m = h->bt_m_req > 0 ? h->bt_m_req : bt_part_size(NV);
  std::vector<int64_t> n(h->n_cells);
  h->levels.clear();
  while (true) {
    BtLevel lv;
    lv.cell_off.assign(B + 1, 0);
    lv.part_off.assign(B + 1, 0);
    int64_t mx = 0;
    for (int b = 0; b < B; ++b) {
      lv.cell_off[b + 1] = lv.cell_off[b] + n[b];
      lv.part_off[b + 1] = lv.part_off[b] + (n[b] + pm - 1) / pm;
      mx = std::max(mx, n[b]);
    }
    lv.n_total = lv.cell_off[B];
    lv.parts_total = lv.part_off[B];
    ROM_HIP_CHECK(hipMalloc(&lv.d_cell_off, sizeof(int64_t) * (B + 1)));
    ROM_HIP_CHECK(hipMalloc(&lv.d_part_off, sizeof(int64_t) * (B + 1)));
    ROM_HIP_CHECK(hipMemcpy(lv.d_cell_off, lv.cell_off.data(), sizeof(int64_t) * (B + 1),
                            hipMemcpyHostToDevice));
    ROM_HIP_CHECK(hipMemcpy(lv.d_part_off, lv.part_off.data(), sizeof(int64_t) * (B + 1),
                            hipMemcpyHostToDevice));
    ROM_HIP_CHECK(hipMalloc(&lv.sys, es * lv.n_total * (3 * NN + NV)));
    ROM_HIP_CHECK(hipMalloc(&lv.x, es * lv.n_total * NV));
    const bool top = mx == 1;
    if (!top) {
      ROM_HIP_CHECK(hipMalloc(&lv.fwd, es * lv.n_total * (2 * NN + NV)));
      ROM_HIP_CHECK(hipMalloc(&lv.part, es * lv.parts_total * (3 * NN + NV)));
    }
    h->levels.push_back(std::move(lv));
    if (top) break;
    for (int b = 0; b < B; ++b) n[b] = (n[b] + pm - 1) / pm;
  }
  return ROM_OK;
}

void bt_free(rom_batch* h) {
  for (auto& lv : h->levels) {
    (void)hipFree(lv.d_cell_off);
    (void)hipFree(lv.d_part_off);
    (void)hipFree(lv.sys);
    (void)hipFree(lv.fwd);
    (void)hipFree(lv.part);
    (void)hipFree(lv.x);
  }
  h->levels.clear();
}

rom_status bt_solve(rom_batch* h, int it, void* upd, void* out, hipStream_t s) {
  const bool f64 = h->cfg.precision == ROM_F64;
  switch (h->nv) {
    case 1: return f64 ? bt_solve_t<double, 1>(h, it, upd, out, s) : bt_solve_t<float, 1>(h, it, upd, out, s);
    case 3: return f64 ? bt_solve_t<double, 3>(h, it, upd, out, s) : bt_solve_t<float, 3>(h, it, upd, out, s);
    case 12: return f64 ? bt_solve_t<double, 12>(h, it, upd, out, s) : bt_solve_t<float, 12>(h, it, upd, out, s);
  }
  set_error("unsupported block size");
  return ROM_E_UNSUPPORTED;
}

}  // namespace romhip
