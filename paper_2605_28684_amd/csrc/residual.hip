// Full-order residual kernels: f(q), the backward-Euler residual, the Newton
// system of a backward-Euler step (block-tridiagonal I - dt J_f and -r), and
// the vector-Jacobian products.
//
// One thread block handles a tile of up to kTile consecutive cells of one
// instance.  The tile and its two halo cells are staged through LDS with
// coalesced element loads (the halo wraps for periodic models and copies the
// end cell for zero-gradient walls), face fluxes are computed once per face
// into LDS, and results are staged back through LDS for coalesced stores.
// No multiply-add contraction: every product and sum is rounded on its own, so
// every launch shape and template instance of a kernel performs the same IEEE
// operations (the autotuner relies on bitwise-identical results; the compiler
// may otherwise fuse or not fuse a multiply-add differently per instance).
#pragma clang fp contract(off)

#include <algorithm>
#include <type_traits>

#include "internal.h"
#include "physics.h"

namespace romhip {

namespace {

template <class Mdl, typename T>
DEV void load_tile(T* sq, const T* qb, int64_t c0, int nt, int64_t n) {
  constexpr int NV = Mdl::NV;
  for (int e = threadIdx.x; e < (nt + 2) * NV; e += blockDim.x) {
    const int lc = e / NV, v = e - (e / NV) * NV;
    int64_t c = c0 - 1 + lc;
    if (c < 0) c = Mdl::periodic ? c + n : 0;
    else if (c >= n) c = Mdl::periodic ? c - n : n - 1;
    sq[e] = qb[c * NV + v];
  }
}

template <typename T>
DEV void flag_or(uint32_t* flags, int b, unsigned fl) {
  if (fl) atomicOr(&flags[b], fl);
}

// Max of a and of b over the whole block (kTile threads), then one atomicMax
// each from thread 0 (none for a zero).  Per-instance sup norms gathered this
// way cost one atomic per block instead of one per wavefront: with 1024 tiles
// per instance the per-wavefront atomics on one address serialise.  Every
// thread of the block must call it.
DEV void block_atomic_max2(uint64_t* da, uint64_t a, uint64_t* db, uint64_t b) {
  __shared__ uint64_t ra[kTile / 64], rb[kTile / 64];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const uint64_t oa = __shfl_xor((unsigned long long)a, off);
    const uint64_t ob = __shfl_xor((unsigned long long)b, off);
    a = oa > a ? oa : a;
    b = ob > b ? ob : b;
  }
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) { ra[w] = a; rb[w] = b; }
  __syncthreads();
  if (threadIdx.x == 0) {
    uint64_t ma = 0, mb = 0;
    for (int k = 0; k < (int)(blockDim.x >> 6); ++k) {
      ma = ra[k] > ma ? ra[k] : ma;
      mb = rb[k] > mb ? rb[k] : mb;
    }
    if (da && ma) atomicMax((unsigned long long*)da, (unsigned long long)ma);
    if (db && mb) atomicMax((unsigned long long*)db, (unsigned long long)mb);
  }
}

DEV uint64_t norm_bits(float x) { return (uint64_t)__float_as_uint(fabsf(x)); }
DEV uint64_t norm_bits(double x) { return (uint64_t)__double_as_longlong(fabs(x)); }

// f(q) (be = 0) or q - q_prev - dt f(q) (be = 1); optional per-instance sup norm
template <class Mdl, typename T>
__global__ __launch_bounds__(kTile) void k_residual(
    const Tile* __restrict__ tiles, const int64_t* __restrict__ dof_off,
    const int64_t* __restrict__ cell_off, const double* __restrict__ phys, int nphys,
    const T* __restrict__ q, const T* __restrict__ qprev, T dt, T* __restrict__ out,
    uint32_t* flags, uint64_t* norms, const int32_t* active) {
  constexpr int NV = Mdl::NV;
  __shared__ T sq[(kTile + 2) * NV];
  __shared__ T sH[(kTile + 1) * NV];
  const Tile t = tiles[blockIdx.x];
  const int b = t.inst;
  if (active && !active[b]) return;
  const int64_t n = cell_off[b + 1] - cell_off[b];
  const int nt = (int)t.ncell;
  const int64_t base = dof_off[b];
  Mdl m(phys + (size_t)b * nphys);
  load_tile<Mdl>(sq, q + base, t.cell0, nt, n);
  __syncthreads();
  unsigned fl = 0;
  for (int k = threadIdx.x; k <= nt; k += blockDim.x)
    m.face(&sq[k * NV], &sq[(k + 1) * NV], &sH[k * NV], fl);
  __syncthreads();
  T f[NV];
  const int i = threadIdx.x;
  const T inv = T(n), inv2 = T(n) * T(n);
  if (i < nt) {
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const T qm = sq[i * NV + v], q0 = sq[(i + 1) * NV + v], qp = sq[(i + 2) * NV + v];
      f[v] = -(sH[(i + 1) * NV + v] - sH[i * NV + v]) * inv;
      const T kap = m.kappa(v);
      if (kap != T(0)) f[v] += kap * ((qp - q0) - (q0 - qm)) * inv2;
    }
    if (Mdl::has_source) {
      T S[NV];
      const double x = ((double)(t.cell0 + i) + 0.5) / (double)n;
      m.source(&sq[(i + 1) * NV], x, S, fl);
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
  uint64_t nb = 0;
  for (int e = threadIdx.x; e < nt * NV; e += blockDim.x) {
    T val = sH[e];
    if (qprev) val = q[o + e] - qprev[o + e] - dt * val;
    if (!isfinite(val)) fl |= ROM_FLAG_NONFINITE;
    out[o + e] = val;
    const uint64_t bits = isfinite(val) ? norm_bits(val) : ~0ull;
    nb = bits > nb ? bits : nb;
  }
  if (norms) block_atomic_max2(&norms[b], nb, nullptr, 0);
  flag_or<T>(flags, b, fl);
}

// Euler residual, persistent and register-resident: a block of 256 threads
// walks tiles of 256 CPT cells (tile += gridDim.x); thread t owns cells t,
// t+256, ... of a tile, loads each cell's three conserved values with one
// 12-byte load straight into registers, and computes the cell's primitives
// there (floored density, velocity, pressure, sound speed, flux terms).  LDS
// only exchanges what neighbours need (structure-of-arrays, conflict-free):
// the primitives of every cell, then the face fluxes.  The next tile's states
// are prefetched into registers while the current tile computes, so memory
// traffic overlaps the arithmetic.  Faces follow App. B eqs.
// sod_rusanov_flux / sod_rusanov_speed (Rusanov) or Toro's HLLC with Davis
// speeds.  Same contract as k_residual.
constexpr int kEulerThreads = 256;

template <typename T>
struct Cell3 { T v[3]; };

// Reciprocal and square root of the streaming Euler residual with a fixed
// instruction choice: in FP32 the hardware v_rcp_f32 / v_sqrt_f32 (1 ulp; the
// arguments are normal numbers: densities and pressures are floored at 1e-10),
// in FP64 correctly rounded.  Left to the compiler, the FP32 lowering of a
// division depends on the surrounding code, which would make results differ
// between launch shapes.
DEV float rcp_s(float x) { return __builtin_amdgcn_rcpf(x); }
DEV double rcp_s(double x) { return 1.0 / x; }
DEV float sqrt_s(float x) { return __builtin_amdgcn_sqrtf(x); }
DEV double sqrt_s(double x) { return sqrt(x); }

// One cell's three conserved values; NT = non-temporal (streamed, not kept in
// the caches) for data that is touched exactly once.
template <bool NT, typename T>
DEV Cell3<T> load3(const T* p) {
  if constexpr (NT) {
    Cell3<T> c;
#pragma unroll
    for (int v = 0; v < 3; ++v) c.v[v] = __builtin_nontemporal_load(p + v);
    return c;
  } else {
    return *reinterpret_cast<const Cell3<T>*>(p);
  }
}
template <bool NT, typename T>
DEV void store3(T* p, const Cell3<T>& c) {
  if constexpr (NT) {
#pragma unroll
    for (int v = 0; v < 3; ++v) __builtin_nontemporal_store(c.v[v], p + v);
  } else {
    *reinterpret_cast<Cell3<T>*>(p) = c;
  }
}

template <typename T, bool HLLC, int CPT, bool NT>
__global__ __launch_bounds__(kEulerThreads) void k_residual_euler(
    const Tile* __restrict__ tiles, int n_tiles, const double* __restrict__ phys, int nphys,
    const T* __restrict__ q, const T* __restrict__ qprev, T dt, T* __restrict__ out,
    uint32_t* flags, uint64_t* norms, const int32_t* active) {
  constexpr int NA = 8;  // rho, m, E, rf, u, p, c, (F1 or 1/rf)
  constexpr int kCellsPerThread = CPT, TILE = kEulerThreads * CPT;
  constexpr int LA = TILE + 2, LH = TILE + 1;
  __shared__ T sa[NA * LA];
  __shared__ T sH[3 * LH];
  const int tid = threadIdx.x;
  // registers: this thread's cells of the current / next tile (+ halo cells for two threads)
  Cell3<T> cur[kCellsPerThread], nxt[kCellsPerThread];
  Cell3<T> hcur, hnxt;  // halo cell: thread 0 -> left, thread 1 -> right
  // Every load is issued unconditionally (cells past the tile read its last
  // cell, threads other than 0 and 1 read the tile's first cell as their
  // "halo"; those values are never used), so that all of them are in flight
  // together: a load under a condition is waited for before the branch joins.
  auto fetch = [&](int ti, Cell3<T>* dst, Cell3<T>& hd) {
    const Tile t = tiles[ti];
    const int64_t n = t.n;
    const int last = (int)t.ncell - 1;
#pragma unroll
    for (int j = 0; j < kCellsPerThread; ++j) {
      const int lc = tid + kEulerThreads * j;
      dst[j] = load3<NT>(q + t.base + (t.cell0 + (lc < last ? lc : last)) * 3);
    }
    int64_t c = tid == 0 ? t.cell0 - 1 : (tid == 1 ? t.cell0 + t.ncell : t.cell0);
    c = c < 0 ? 0 : (c >= n ? n - 1 : c);   // zero-gradient ghosts
    hd = *reinterpret_cast<const Cell3<T>*>(q + t.base + c * 3);
  };
  int ti = blockIdx.x;
  if (ti < n_tiles) fetch(ti, cur, hcur);
  unsigned fl = 0;
  for (; ti < n_tiles; ti += gridDim.x) {
    const Tile t = tiles[ti];
    const int b = t.inst;
    const bool skip = active && !active[b];
    const int64_t n = t.n;
    const int nt = (int)t.ncell;
    const T gamma = T(phys[(size_t)b * nphys]);
    const int tn = ti + gridDim.x;
    // primitives of owned cells (LDS slot lc + 1) and of the halo cells
    auto prim = [&](const Cell3<T>& c3, int slot) {
      const T rho = c3.v[0], m = c3.v[1], E = c3.v[2];
      if (rho < T(kRhoMin)) fl |= ROM_FLAG_FLOOR;
      const T rf = rho >= T(kRhoMin) ? rho : T(kRhoMin);
      const T ir = rcp_s(rf);
      const T u = m * ir;
      const T pe = (gamma - T(1)) * (E - T(0.5) * m * u);
      if (pe < T(kPMin)) fl |= ROM_FLAG_FLOOR;
      const T p = pe >= T(kPMin) ? pe : T(kPMin);
      sa[slot] = rho; sa[LA + slot] = m; sa[2 * LA + slot] = E; sa[3 * LA + slot] = rf;
      sa[4 * LA + slot] = u; sa[5 * LA + slot] = p; sa[6 * LA + slot] = sqrt_s(gamma * p * ir);
      sa[7 * LA + slot] = HLLC ? ir : m * u + p;
    };
    if (!skip) {
#pragma unroll
      for (int j = 0; j < kCellsPerThread; ++j) {
        const int lc = tid + kEulerThreads * j;
        if (lc < nt) prim(cur[j], lc + 1);
      }
      if (tid == 0) prim(hcur, 0);
      if (tid == 1) prim(hcur, nt + 1);
    }
    // the next tile's loads overlap everything below
    if (tn < n_tiles) fetch(tn, nxt, hnxt);
    __syncthreads();
    if (!skip) {
      for (int k = tid; k <= nt; k += kEulerThreads) {
        T L[NA], R[NA], H[3];
#pragma unroll
        for (int v = 0; v < NA; ++v) { L[v] = sa[v * LA + k]; R[v] = sa[v * LA + k + 1]; }
        if (!HLLC) {
          const T uL = L[4], uR = R[4];
          const T aL = (uL >= T(0) ? uL : -uL) + L[6], aR = (uR >= T(0) ? uR : -uR) + R[6];
          const T s = aL >= aR ? aL : aR;
          const T h = T(0.5);
          H[0] = h * (L[1] + R[1]) - h * s * (R[0] - L[0]);
          H[1] = h * (L[7] + R[7]) - h * s * (R[1] - L[1]);
          H[2] = h * (uL * (L[2] + L[5]) + uR * (R[2] + R[5])) - h * s * (R[2] - L[2]);
        } else {
          const T rL = L[3], uL = L[4], pL = L[5], cL = L[6];
          const T rR = R[3], uR = R[4], pR = R[5], cR = R[6];
          const T SL = (uL - cL) <= (uR - cR) ? (uL - cL) : (uR - cR);
          const T SR = (uL + cL) >= (uR + cR) ? (uL + cL) : (uR + cR);
          if (SL >= T(0)) {
            H[0] = L[1]; H[1] = L[1] * uL + pL; H[2] = uL * (L[2] + pL);
          } else {
            const T num = pR - pL + rL * uL * (SL - uL) - rR * uR * (SR - uR);
            const T den = rL * (SL - uL) - rR * (SR - uR);
            const T Ss = num * rcp_s(den);
            if (Ss >= T(0)) {
              const T fac = rL * (SL - uL) * rcp_s(SL - Ss);
              const T e = L[2] * L[7] + (Ss - uL) * (Ss + pL * rcp_s(rL * (SL - uL)));
              H[0] = L[1] + SL * (fac - L[0]);
              H[1] = L[1] * uL + pL + SL * (fac * Ss - L[1]);
              H[2] = uL * (L[2] + pL) + SL * (fac * e - L[2]);
            } else if (SR >= T(0)) {
              const T fac = rR * (SR - uR) * rcp_s(SR - Ss);
              const T e = R[2] * R[7] + (Ss - uR) * (Ss + pR * rcp_s(rR * (SR - uR)));
              H[0] = R[1] + SR * (fac - R[0]);
              H[1] = R[1] * uR + pR + SR * (fac * Ss - R[1]);
              H[2] = uR * (R[2] + pR) + SR * (fac * e - R[2]);
            } else {
              H[0] = R[1]; H[1] = R[1] * uR + pR; H[2] = uR * (R[2] + pR);
            }
          }
        }
        sH[k] = H[0]; sH[LH + k] = H[1]; sH[2 * LH + k] = H[2];
      }
    }
    __syncthreads();
    if (!skip) {
      const T nn = T(n);
      uint64_t nb = 0;
      // with q_prev, its loads are waited for here, and with them the next
      // tile's (issued earlier); without it no load stands before the stores
      auto emit = [&](auto with_prev) {
        constexpr bool WP = decltype(with_prev)::value;
#pragma unroll
        for (int j = 0; j < kCellsPerThread; ++j) {
          const int lc = tid + kEulerThreads * j;
          if (lc < nt) {
            const int64_t g = t.base + (t.cell0 + lc) * 3;
            Cell3<T> o;
            Cell3<T> pv;
            if constexpr (WP) pv = load3<NT>(qprev + g);
#pragma unroll
            for (int v = 0; v < 3; ++v) {
              T val = -(sH[v * LH + lc + 1] - sH[v * LH + lc]) * nn;
              if constexpr (WP) val = cur[j].v[v] - pv.v[v] - dt * val;
              if (!isfinite(val)) fl |= ROM_FLAG_NONFINITE;
              o.v[v] = val;
              const uint64_t bits = isfinite(val) ? norm_bits(val) : ~0ull;
              nb = bits > nb ? bits : nb;
            }
            store3<NT>(out + g, o);
          }
        }
      };
      if (qprev) emit(std::true_type{});
      else emit(std::false_type{});
      if (norms) wave_atomic_max(&norms[b], nb);
      flag_or<T>(flags, b, fl);
      fl = 0;
    }
#pragma unroll
    for (int j = 0; j < kCellsPerThread; ++j) cur[j] = nxt[j];
    hcur = hnxt;
    __syncthreads();   // LDS is rewritten by the next tile
  }
}

// Newton system of r(q) = q - q_prev - dt f(q): per cell A = -dt Jm,
// B = I - dt J0, C = -dt Jp, d = -r; plus the sup norm of r.
template <class Mdl, typename T>
__global__ __launch_bounds__(kTile) void k_assemble(
    const Tile* __restrict__ tiles, const int64_t* __restrict__ dof_off,
    const int64_t* __restrict__ cell_off, const double* __restrict__ phys, int nphys,
    const T* __restrict__ q, const T* __restrict__ qprev, T dt, T* __restrict__ sys,
    uint32_t* flags, uint64_t* norms, uint64_t* ynorms, const int32_t* active) {
  constexpr int NV = Mdl::NV;
  constexpr int NN = NV * NV;
  constexpr int SYS = 3 * NN + NV;
  __shared__ T sq[(kTile + 2) * NV];
  const Tile t = tiles[blockIdx.x];
  const int b = t.inst;
  if (active && !active[b]) return;
  const int64_t n = cell_off[b + 1] - cell_off[b];
  const int nt = (int)t.ncell;
  const int64_t base = dof_off[b];
  Mdl m(phys + (size_t)b * nphys);
  load_tile<Mdl>(sq, q + base, t.cell0, nt, n);
  __syncthreads();
  const int i = threadIdx.x;
  unsigned fl = 0;
  uint64_t nb = 0, yb = 0;
  if (i < nt) {
    const int64_t c = t.cell0 + i;
    const bool lw = !Mdl::periodic && c == 0;
    const bool rw = !Mdl::periodic && c == n - 1;
    T f[NV], Jm[NN], J0[NN], Jp[NN];
    const double x = ((double)c + 0.5) / (double)n;
    cell_jacobian(m, &sq[i * NV], &sq[(i + 1) * NV], &sq[(i + 2) * NV], lw, rw, T(n),
                  T(n) * T(n), x, f, Jm, J0, Jp, fl);
    T* o = sys + (cell_off[b] + c) * SYS;
#pragma unroll
    for (int e = 0; e < NN; ++e) {
      o[e] = -dt * Jm[e];
      o[NN + e] = -dt * J0[e] + ((e % (NV + 1)) == 0 ? T(1) : T(0));
      o[2 * NN + e] = -dt * Jp[e];
    }
    const int64_t g = base + c * NV;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const T r = q[g + v] - qprev[g + v] - dt * f[v];
      o[3 * NN + v] = -r;
      if (!isfinite(r)) fl |= ROM_FLAG_NONFINITE;
      const uint64_t bits = isfinite(r) ? norm_bits(r) : ~0ull;
      nb = bits > nb ? bits : nb;
      const uint64_t yv = norm_bits(q[g + v]);
      yb = yv > yb ? yv : yb;
    }
  }
  block_atomic_max2(norms ? &norms[b] : nullptr, nb, ynorms ? &ynorms[b] : nullptr, yb);
  flag_or<T>(flags, b, fl);
}

// A face quantity in LDS: word w of face k at p[w * st] (structure of arrays).
template <typename T>
struct FaceView {
  const T* p;
  int st;
  DEV T operator[](int w) const { return p[w * st]; }
};

// The same Newton system for models of at most three variables (Burgers,
// Euler), with each face's flux Jacobian evaluated once: a thread per face
// (nt + 1 faces) into LDS, then a thread per cell combines its two faces
// exactly as cell_jacobian does (bitwise the same blocks), and the tile's
// rows of sys, contiguous in memory, are written from LDS with coalesced
// stores.
template <class Mdl, typename T>
__global__ __launch_bounds__(kTile) void k_assemble_faces(
    const Tile* __restrict__ tiles, const int64_t* __restrict__ dof_off,
    const int64_t* __restrict__ cell_off, const double* __restrict__ phys, int nphys,
    const T* __restrict__ q, const T* __restrict__ qprev, T dt, T* __restrict__ sys,
    uint32_t* flags, uint64_t* norms, uint64_t* ynorms, const int32_t* active) {
  constexpr int NV = Mdl::NV;
  constexpr int NN = NV * NV;
  constexpr int SYS = 3 * NN + NV;
  constexpr int FW = NV + 2 * NN;   // words per face: flux, d/dq_left, d/dq_right
  constexpr int FS = kTile + 1;     // faces per tile
  static_assert(FW * FS <= SYS * kTile, "face words must fit the output staging");
  __shared__ T sq[(kTile + 2) * NV];
  __shared__ T sw[SYS * kTile];     // face words, then the tile's rows of sys
  const Tile t = tiles[blockIdx.x];
  const int b = t.inst;
  if (active && !active[b]) return;
  const int64_t n = cell_off[b + 1] - cell_off[b];
  const int nt = (int)t.ncell;
  const int64_t base = dof_off[b];
  Mdl m(phys + (size_t)b * nphys);
  load_tile<Mdl>(sq, q + base, t.cell0, nt, n);
  __syncthreads();
  unsigned fl = 0;
  for (int k = threadIdx.x; k <= nt; k += blockDim.x) {   // face between cells k - 1 and k
    T H[NV], DL[NN], DR[NN];
    m.face_jac(&sq[k * NV], &sq[(k + 1) * NV], H, DL, DR, fl);
#pragma unroll
    for (int v = 0; v < NV; ++v) sw[v * FS + k] = H[v];
#pragma unroll
    for (int e = 0; e < NN; ++e) {
      sw[(NV + e) * FS + k] = DL[e];
      sw[(NV + NN + e) * FS + k] = DR[e];
    }
  }
  __syncthreads();
  const int i = threadIdx.x;
  T o[SYS];
  uint64_t nb = 0, yb = 0;
  if (i < nt) {
    const int64_t c = t.cell0 + i;
    const bool lw = !Mdl::periodic && c == 0;
    const bool rw = !Mdl::periodic && c == n - 1;
    T f[NV], Jm[NN], J0[NN], Jp[NN];
    const double x = ((double)c + 0.5) / (double)n;
    const FaceView<T> HL{sw + i, FS}, DLl{sw + NV * FS + i, FS}, DRl{sw + (NV + NN) * FS + i, FS};
    const FaceView<T> HR{sw + i + 1, FS}, DLr{sw + NV * FS + i + 1, FS},
        DRr{sw + (NV + NN) * FS + i + 1, FS};
    cell_combine(m, HL, DLl, DRl, HR, DLr, DRr, &sq[i * NV], &sq[(i + 1) * NV],
                 &sq[(i + 2) * NV], lw, rw, T(n), T(n) * T(n), x, f, Jm, J0, Jp, fl);
#pragma unroll
    for (int e = 0; e < NN; ++e) {
      o[e] = -dt * Jm[e];
      o[NN + e] = -dt * J0[e] + ((e % (NV + 1)) == 0 ? T(1) : T(0));
      o[2 * NN + e] = -dt * Jp[e];
    }
    const int64_t g = base + c * NV;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const T qv = sq[(i + 1) * NV + v];
      const T r = qv - qprev[g + v] - dt * f[v];
      o[3 * NN + v] = -r;
      if (!isfinite(r)) fl |= ROM_FLAG_NONFINITE;
      const uint64_t bits = isfinite(r) ? norm_bits(r) : ~0ull;
      nb = bits > nb ? bits : nb;
      const uint64_t yv = norm_bits(qv);
      yb = yv > yb ? yv : yb;
    }
  }
  __syncthreads();   // the face words are no longer read
  if (i < nt) {
#pragma unroll
    for (int e = 0; e < SYS; ++e) sw[i * SYS + e] = o[e];
  }
  __syncthreads();
  T* dst = sys + (cell_off[b] + t.cell0) * SYS;
  for (int e = threadIdx.x; e < nt * SYS; e += blockDim.x) dst[e] = sw[e];
  block_atomic_max2(norms ? &norms[b] : nullptr, nb, ynorms ? &ynorms[b] : nullptr, yb);
  flag_or<T>(flags, b, fl);
}

// The transposed system of k_assemble_adjoint for models of at most three
// variables, with each face's flux Jacobian evaluated once (nt + 3 faces of
// cells c0 - 2 .. c0 + nt + 1 into LDS); the blocks of cells i - 1, i and
// i + 1 are combined from them exactly as cell_jacobian does, and the rows
// are written from LDS with coalesced stores.
template <class Mdl, typename T>
__global__ __launch_bounds__(kTile) void k_assemble_adjoint_faces(
    const Tile* __restrict__ tiles, const int64_t* __restrict__ dof_off,
    const int64_t* __restrict__ cell_off, const double* __restrict__ phys, int nphys,
    const T* __restrict__ q, T dt, const T* __restrict__ rhs, T* __restrict__ sys,
    uint32_t* flags) {
  constexpr int NV = Mdl::NV;
  constexpr int NN = NV * NV;
  constexpr int SYS = 3 * NN + NV;
  constexpr int FW = NV + 2 * NN;
  constexpr int FS = kTile + 3;
  static_assert(FW * FS <= SYS * kTile, "face words must fit the output staging");
  __shared__ T sq[(kTile + 4) * NV];
  __shared__ T sw[SYS * kTile];
  const Tile t = tiles[blockIdx.x];
  const int b = t.inst;
  const int64_t n = cell_off[b + 1] - cell_off[b];
  const int nt = (int)t.ncell;
  const int64_t base = dof_off[b];
  Mdl m(phys + (size_t)b * nphys);
  // stage cells c0-2 .. c0+nt+1 (wrapped, or clamped at walls)
  for (int e = threadIdx.x; e < (nt + 4) * NV; e += blockDim.x) {
    const int lc = e / NV, v = e - (e / NV) * NV;
    int64_t c = t.cell0 - 2 + lc;
    if (Mdl::periodic) { c = ((c % n) + n) % n; }
    else { c = c < 0 ? 0 : (c >= n ? n - 1 : c); }
    sq[e] = q[base + c * NV + v];
  }
  __syncthreads();
  unsigned fl = 0;
  for (int k = threadIdx.x; k < nt + 3; k += blockDim.x) {   // face between staged k, k + 1
    T H[NV], DL[NN], DR[NN];
    m.face_jac(&sq[k * NV], &sq[(k + 1) * NV], H, DL, DR, fl);
#pragma unroll
    for (int v = 0; v < NV; ++v) sw[v * FS + k] = H[v];
#pragma unroll
    for (int e = 0; e < NN; ++e) {
      sw[(NV + e) * FS + k] = DL[e];
      sw[(NV + NN + e) * FS + k] = DR[e];
    }
  }
  __syncthreads();
  // blocks of the cell in staged slot sl (faces sl - 1 and sl)
  auto blocks = [&](int sl, int64_t cw, T* Jm, T* J0, T* Jp) {
    const bool lw = !Mdl::periodic && cw == 0, rw = !Mdl::periodic && cw == n - 1;
    T f[NV];
    const FaceView<T> HL{sw + sl - 1, FS}, DLl{sw + NV * FS + sl - 1, FS},
        DRl{sw + (NV + NN) * FS + sl - 1, FS};
    const FaceView<T> HR{sw + sl, FS}, DLr{sw + NV * FS + sl, FS}, DRr{sw + (NV + NN) * FS + sl, FS};
    cell_combine(m, HL, DLl, DRl, HR, DLr, DRr, &sq[(sl - 1) * NV], &sq[sl * NV],
                 &sq[(sl + 1) * NV], lw, rw, T(n), T(n) * T(n), ((double)cw + 0.5) / (double)n,
                 f, Jm, J0, Jp, fl);
  };
  const int i = threadIdx.x;
  T o[SYS];
  if (i < nt) {
    const int64_t c = t.cell0 + i;
    T Jm[NN], J0[NN], Jp[NN];
    blocks(i + 2, c, Jm, J0, Jp);                  // own diagonal block
#pragma unroll
    for (int r = 0; r < NV; ++r)
#pragma unroll
      for (int k = 0; k < NV; ++k)
        o[NN + r * NV + k] = -dt * J0[k * NV + r] + (r == k ? T(1) : T(0));
    {  // left neighbour's C block (row c-1, coupling to c), transposed -> our A
      const bool exists = Mdl::periodic || c - 1 >= 0;
      if (exists) blocks(i + 1, (c - 1 + n) % n, Jm, J0, Jp);
#pragma unroll
      for (int r = 0; r < NV; ++r)
#pragma unroll
        for (int k = 0; k < NV; ++k) o[r * NV + k] = exists ? -dt * Jp[k * NV + r] : T(0);
    }
    {  // right neighbour's A block (row c+1, coupling to c), transposed -> our C
      const bool exists = Mdl::periodic || c + 1 < n;
      if (exists) blocks(i + 3, (c + 1) % n, Jm, J0, Jp);
#pragma unroll
      for (int r = 0; r < NV; ++r)
#pragma unroll
        for (int k = 0; k < NV; ++k) o[2 * NN + r * NV + k] = exists ? -dt * Jm[k * NV + r] : T(0);
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) o[3 * NN + v] = rhs[base + c * NV + v];
  }
  __syncthreads();   // the face words are no longer read
  if (i < nt) {
#pragma unroll
    for (int e = 0; e < SYS; ++e) sw[i * SYS + e] = o[e];
  }
  __syncthreads();
  T* dst = sys + (cell_off[b] + t.cell0) * SYS;
  for (int e = threadIdx.x; e < nt * SYS; e += blockDim.x) dst[e] = sw[e];
  flag_or<T>(flags, b, fl);
}

// Transposed Newton system of the adjoint of a converged step:
// (I - dt J_f)^T x = rhs, written as a block-tridiagonal system per cell:
// A_i = (C_{i-1})^T, B_i = (B_i)^T, C_i = (A_{i+1})^T with the forward blocks
// A = -dt Jm, B = I - dt J0, C = -dt Jp.  Each thread recomputes the forward
// blocks of its two neighbours.
template <class Mdl, typename T>
__global__ __launch_bounds__(kTile) void k_assemble_adjoint(
    const Tile* __restrict__ tiles, const int64_t* __restrict__ dof_off,
    const int64_t* __restrict__ cell_off, const double* __restrict__ phys, int nphys,
    const T* __restrict__ q, T dt, const T* __restrict__ rhs, T* __restrict__ sys,
    uint32_t* flags) {
  constexpr int NV = Mdl::NV;
  constexpr int NN = NV * NV;
  constexpr int SYS = 3 * NN + NV;
  __shared__ T sq[(kTile + 4) * NV];
  const Tile t = tiles[blockIdx.x];
  const int b = t.inst;
  const int64_t n = cell_off[b + 1] - cell_off[b];
  const int nt = (int)t.ncell;
  const int64_t base = dof_off[b];
  Mdl m(phys + (size_t)b * nphys);
  // stage cells c0-2 .. c0+nt+1
  for (int e = threadIdx.x; e < (nt + 4) * NV; e += blockDim.x) {
    const int lc = e / NV, v = e - (e / NV) * NV;
    int64_t c = t.cell0 - 2 + lc;
    if (Mdl::periodic) { c = ((c % n) + n) % n; }
    else { c = c < 0 ? 0 : (c >= n ? n - 1 : c); }
    sq[e] = q[base + c * NV + v];
  }
  __syncthreads();
  const int i = threadIdx.x;
  unsigned fl = 0;
  if (i < nt) {
    const int64_t c = t.cell0 + i;
    T f[NV], Jm[NN], J0[NN], Jp[NN];
    T* o = sys + (cell_off[b] + c) * SYS;
    // own diagonal block
    {
      const bool lw = !Mdl::periodic && c == 0, rw = !Mdl::periodic && c == n - 1;
      cell_jacobian(m, &sq[(i + 1) * NV], &sq[(i + 2) * NV], &sq[(i + 3) * NV], lw, rw, T(n),
                    T(n) * T(n), ((double)c + 0.5) / (double)n, f, Jm, J0, Jp, fl);
#pragma unroll
      for (int r = 0; r < NV; ++r)
#pragma unroll
        for (int k = 0; k < NV; ++k)
          o[NN + r * NV + k] = -dt * J0[k * NV + r] + (r == k ? T(1) : T(0));
    }
    // left neighbour's C block (row c-1, coupling to c), transposed -> our A
    {
      const int64_t cl = c - 1;
      const bool exists = Mdl::periodic || cl >= 0;
      if (exists) {
        const int64_t cw = (cl + n) % n;
        const bool lw = !Mdl::periodic && cw == 0, rw = !Mdl::periodic && cw == n - 1;
        cell_jacobian(m, &sq[i * NV], &sq[(i + 1) * NV], &sq[(i + 2) * NV], lw, rw, T(n),
                      T(n) * T(n), ((double)cw + 0.5) / (double)n, f, Jm, J0, Jp, fl);
      }
#pragma unroll
      for (int r = 0; r < NV; ++r)
#pragma unroll
        for (int k = 0; k < NV; ++k) o[r * NV + k] = exists ? -dt * Jp[k * NV + r] : T(0);
    }
    // right neighbour's A block (row c+1, coupling to c), transposed -> our C
    {
      const int64_t cr = c + 1;
      const bool exists = Mdl::periodic || cr < n;
      if (exists) {
        const int64_t cw = cr % n;
        const bool lw = !Mdl::periodic && cw == 0, rw = !Mdl::periodic && cw == n - 1;
        cell_jacobian(m, &sq[(i + 2) * NV], &sq[(i + 3) * NV], &sq[(i + 4) * NV], lw, rw, T(n),
                      T(n) * T(n), ((double)cw + 0.5) / (double)n, f, Jm, J0, Jp, fl);
      }
#pragma unroll
      for (int r = 0; r < NV; ++r)
#pragma unroll
        for (int k = 0; k < NV; ++k) o[2 * NN + r * NV + k] = exists ? -dt * Jm[k * NV + r] : T(0);
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) o[3 * NN + v] = rhs[base + c * NV + v];
  }
  flag_or<T>(flags, b, fl);
}

// gq = J_f(q)^T w (be = 0) or gq = w - dt J_f^T w, gq_prev = -w (be = 1).
// Per cell c: contributions of face c (between c-1 and c) through dH/dq_R and of
// face c+1 through dH/dq_L, each with lambda = (w_right - w_left)/dx; the
// diffusion adjoint; the source adjoint.
template <class Mdl, typename T>
__global__ __launch_bounds__(kTile) void k_residual_vjp(
    const Tile* __restrict__ tiles, const int64_t* __restrict__ dof_off,
    const int64_t* __restrict__ cell_off, const double* __restrict__ phys, int nphys,
    const T* __restrict__ q, const T* __restrict__ w, T dt, int be, T* __restrict__ gq,
    T* __restrict__ gqp, uint32_t* flags) {
  constexpr int NV = Mdl::NV;
  constexpr int NN = NV * NV;
  __shared__ T sq[(kTile + 2) * NV];
  __shared__ T sw[(kTile + 2) * NV];
  const Tile t = tiles[blockIdx.x];
  const int b = t.inst;
  const int64_t n = cell_off[b + 1] - cell_off[b];
  const int nt = (int)t.ncell;
  const int64_t base = dof_off[b];
  Mdl m(phys + (size_t)b * nphys);
  load_tile<Mdl>(sq, q + base, t.cell0, nt, n);
  for (int e = threadIdx.x; e < (nt + 2) * NV; e += blockDim.x) {
    const int lc = e / NV, v = e - (e / NV) * NV;
    int64_t c = t.cell0 - 1 + lc;
    bool ghost = false;
    if (c < 0) { if (Mdl::periodic) c += n; else ghost = true; }
    else if (c >= n) { if (Mdl::periodic) c -= n; else ghost = true; }
    sw[e] = ghost ? T(0) : w[base + c * NV + v];   // no residual row outside walls
  }
  __syncthreads();
  const int i = threadIdx.x;
  unsigned fl = 0;
  if (i < nt) {
    const int64_t c = t.cell0 + i;
    const bool lw = !Mdl::periodic && c == 0, rw = !Mdl::periodic && c == n - 1;
    const T inv = T(n), inv2 = T(n) * T(n);
    T H[NV], DL[NN], DR[NN], g[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) g[v] = T(0);
    // face c (left): lambda = (w_c - w_{c-1}) / dx, acts through dH/dq_R (and dH/dq_L at a wall)
    m.face_jac(&sq[i * NV], &sq[(i + 1) * NV], H, DL, DR, fl);
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      T acc = T(0);
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        const T lam = (sw[(i + 1) * NV + v] - sw[i * NV + v]) * inv;
        acc += (DR[v * NV + k] + (lw ? DL[v * NV + k] : T(0))) * lam;
      }
      g[k] += acc;
    }
    // face c+1 (right): lambda = (w_{c+1} - w_c) / dx, acts through dH/dq_L (and dH/dq_R at a wall)
    m.face_jac(&sq[(i + 1) * NV], &sq[(i + 2) * NV], H, DL, DR, fl);
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      T acc = T(0);
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        const T lam = (sw[(i + 2) * NV + v] - sw[(i + 1) * NV + v]) * inv;
        acc += (DL[v * NV + k] + (rw ? DR[v * NV + k] : T(0))) * lam;
      }
      g[k] += acc;
    }
    // diffusion: row j contributes kappa w_j / dx^2 to its (ghost-mapped) neighbours
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const T kap = m.kappa(v);
      if (kap != T(0)) {
        const T wm = sw[i * NV + v], w0 = sw[(i + 1) * NV + v], wp = sw[(i + 2) * NV + v];
        T acc = wm + wp - T(2) * w0;
        if (lw) acc += w0;  // row 0's left ghost is cell 0 itself
        if (rw) acc += w0;
        g[v] += kap * inv2 * acc;
      }
    }
    if (Mdl::has_source) {
      T S[NV], DS[NN];
      m.source_jac(&sq[(i + 1) * NV], ((double)c + 0.5) / (double)n, S, DS, fl);
#pragma unroll
      for (int k = 0; k < NV; ++k) {
        T acc = T(0);
#pragma unroll
        for (int v = 0; v < NV; ++v) acc += DS[v * NV + k] * sw[(i + 1) * NV + v];
        g[k] += acc;
      }
    }
    const int64_t o = base + c * NV;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      if (be) {
        const T wv = sw[(i + 1) * NV + v];
        gq[o + v] = wv - dt * g[v];
        if (gqp) gqp[o + v] = -wv;
      } else {
        gq[o + v] = g[v];
      }
    }
  }
  flag_or<T>(flags, b, fl);
}

}  // namespace

template <class M>
struct Tag { using type = M; };

// Calls fn(Tag<Model>{}) for the model of the handle's problem.
template <typename T, class F>
rom_status with_model(const rom_batch* h, F&& fn) {
  switch (h->cfg.problem) {
    case ROM_BURGERS: return fn(Tag<BurgersModel<T>>{});
    case ROM_EULER_RUSANOV: return fn(Tag<EulerModel<T, false>>{});
    case ROM_EULER_HLLC: return fn(Tag<EulerModel<T, true>>{});
    case ROM_REACT: return fn(Tag<ReactModel<T>>{});
  }
  set_error("unknown problem");
  return ROM_E_INVAL;
}

template <typename T>
static rom_status residual_t(rom_batch* h, const void* q, const void* q_prev, double dt, void* out,
                             uint64_t* norms, const int32_t* active, hipStream_t s) {
  if (h->cfg.problem == ROM_EULER_RUSANOV || h->cfg.problem == ROM_EULER_HLLC) {
    // persistent grid of (blocks per CU) x CUs walking tiles of 256 CPT cells;
    // the shape comes from the autotuner (results do not depend on it)
    const ResidualShape sh = residual_shape(h, h->tune_residual);
    const Tile* tl = sh.cpt == 4 ? h->d_btiles : sh.cpt == 2 ? h->d_btiles2 : h->d_tiles;
    const int nt = sh.cpt == 4 ? h->n_btiles : sh.cpt == 2 ? h->n_btiles2 : h->n_tiles;
    const int grid = std::max(1, std::min(nt, h->n_cu * sh.blocks_per_cu));
    auto go = [&](auto kern) {
      hipLaunchKernelGGL(kern, dim3(grid), dim3(kEulerThreads), 0, s, tl, nt, h->d_phys,
                         h->cfg.n_phys, (const T*)q, (const T*)q_prev, (T)dt, (T*)out, h->flags,
                         norms, active);
    };
    auto pick = [&](auto hllc_tag) {
      constexpr bool HL = decltype(hllc_tag)::value;
      if (sh.nt) {
        if (sh.cpt == 4) go(k_residual_euler<T, HL, 4, true>);
        else if (sh.cpt == 2) go(k_residual_euler<T, HL, 2, true>);
        else go(k_residual_euler<T, HL, 1, true>);
      } else {
        if (sh.cpt == 4) go(k_residual_euler<T, HL, 4, false>);
        else if (sh.cpt == 2) go(k_residual_euler<T, HL, 2, false>);
        else go(k_residual_euler<T, HL, 1, false>);
      }
    };
    if (h->cfg.problem == ROM_EULER_HLLC) pick(std::true_type{});
    else pick(std::false_type{});
    return ROM_OK;
  }
  return with_model<T>(h, [&](auto tag) -> rom_status {
    using M = typename decltype(tag)::type;
    hipLaunchKernelGGL((k_residual<M, T>), dim3(h->n_tiles), dim3(kTile), 0, s, h->d_tiles,
                       h->d_dof_off, h->d_cell_off, h->d_phys, h->cfg.n_phys, (const T*)q,
                       (const T*)q_prev, (T)dt, (T*)out, h->flags, norms, active);
    return ROM_OK;
  });
}

rom_status launch_residual(rom_batch* h, const void* q, const void* q_prev, double dt, void* out,
                           hipStream_t s) {
  rom_status st = h->cfg.precision == ROM_F64
                      ? residual_t<double>(h, q, q_prev, dt, out, nullptr, nullptr, s)
                      : residual_t<float>(h, q, q_prev, dt, out, nullptr, nullptr, s);
  ROM_HIP_CHECK(hipGetLastError());
  return st;
}

rom_status launch_residual_norm(rom_batch* h, const void* q, const void* q_prev, double dt,
                                void* out, int it, hipStream_t s) {
  uint64_t* norms = h->norms + (size_t)it * h->cfg.n_inst;
  rom_status st = h->cfg.precision == ROM_F64
                      ? residual_t<double>(h, q, q_prev, dt, out, norms, h->active, s)
                      : residual_t<float>(h, q, q_prev, dt, out, norms, h->active, s);
  ROM_HIP_CHECK(hipGetLastError());
  return st;
}

// Launch shapes of the streaming Euler residual that the autotuner chooses
// from: (cells per thread, resident blocks per CU, non-temporal streaming),
// limited by LDS (FP32 tiles of 1024 / 512 / 256 cells use 45 / 23 / 11 KB;
// FP64 doubles that).
static const ResidualShape kShapesF32[] = {{4, 3, 0}, {4, 2, 0}, {2, 7, 0}, {2, 6, 0}, {2, 4, 0},
                                           {1, 8, 0}, {1, 12, 0}, {4, 3, 1}, {2, 7, 1}, {2, 6, 1},
                                           {1, 8, 1}, {1, 12, 1}};
static const ResidualShape kShapesF64[] = {{4, 1, 0}, {2, 3, 0}, {2, 2, 0}, {1, 6, 0},
                                           {2, 3, 1}, {1, 6, 1}};

int residual_shape_count(const rom_batch* h) {
  if (h->cfg.problem != ROM_EULER_RUSANOV && h->cfg.problem != ROM_EULER_HLLC) return 1;
  return h->cfg.precision == ROM_F32 ? (int)(sizeof(kShapesF32) / sizeof(kShapesF32[0]))
                                     : (int)(sizeof(kShapesF64) / sizeof(kShapesF64[0]));
}

ResidualShape residual_shape(const rom_batch* h, int i) {
  const int n = residual_shape_count(h);
  if (i < 0 || i >= n) i = 0;
  return h->cfg.precision == ROM_F32 ? kShapesF32[i] : kShapesF64[i];
}

template <typename T>
static rom_status assemble_t(rom_batch* h, const void* q, const void* q_prev, double dt, int it,
                             hipStream_t s) {
  return with_model<T>(h, [&](auto tag) -> rom_status {
    using M = typename decltype(tag)::type;
    auto go = [&](auto kern) {
      hipLaunchKernelGGL(kern, dim3(h->n_tiles), dim3(kTile), 0, s, h->d_tiles, h->d_dof_off,
                         h->d_cell_off, h->d_phys, h->cfg.n_phys, (const T*)q, (const T*)q_prev,
                         (T)dt, (T*)h->levels[0].sys, h->flags,
                         h->norms + (size_t)it * h->cfg.n_inst,
                         h->norms + (size_t)(h->cfg.newton_max + 1 + it) * h->cfg.n_inst,
                         h->active);
    };
    if constexpr (M::NV <= 3) go(k_assemble_faces<M, T>);
    else go(k_assemble<M, T>);
    return ROM_OK;
  });
}

rom_status launch_assemble(rom_batch* h, const void* q, const void* q_prev, double dt, int it,
                           hipStream_t s) {
  rom_status st = h->cfg.precision == ROM_F64 ? assemble_t<double>(h, q, q_prev, dt, it, s)
                                              : assemble_t<float>(h, q, q_prev, dt, it, s);
  ROM_HIP_CHECK(hipGetLastError());
  return st;
}

template <typename T>
static rom_status assemble_adj_t(rom_batch* h, const void* q, double dt, const void* rhs,
                                 hipStream_t s) {
  return with_model<T>(h, [&](auto tag) -> rom_status {
    using M = typename decltype(tag)::type;
    auto go = [&](auto kern) {
      hipLaunchKernelGGL(kern, dim3(h->n_tiles), dim3(kTile), 0, s, h->d_tiles, h->d_dof_off,
                         h->d_cell_off, h->d_phys, h->cfg.n_phys, (const T*)q, (T)dt,
                         (const T*)rhs, (T*)h->levels[0].sys, h->flags);
    };
    if constexpr (M::NV <= 3) go(k_assemble_adjoint_faces<M, T>);
    else go(k_assemble_adjoint<M, T>);
    return ROM_OK;
  });
}

rom_status launch_assemble_adjoint(rom_batch* h, const void* q, double dt, const void* rhs,
                                   hipStream_t s) {
  rom_status st = h->cfg.precision == ROM_F64 ? assemble_adj_t<double>(h, q, dt, rhs, s)
                                              : assemble_adj_t<float>(h, q, dt, rhs, s);
  ROM_HIP_CHECK(hipGetLastError());
  return st;
}

template <typename T>
static rom_status vjp_t(rom_batch* h, const void* q, const void* q_prev, double dt,
                        const void* gbar, void* gq, void* gq_prev, hipStream_t s) {
  return with_model<T>(h, [&](auto tag) -> rom_status {
    using M = typename decltype(tag)::type;
    hipLaunchKernelGGL((k_residual_vjp<M, T>), dim3(h->n_tiles), dim3(kTile), 0, s, h->d_tiles,
                       h->d_dof_off, h->d_cell_off, h->d_phys, h->cfg.n_phys, (const T*)q,
                       (const T*)gbar, (T)dt, q_prev ? 1 : 0, (T*)gq, (T*)gq_prev, h->flags);
    return ROM_OK;
  });
}

rom_status launch_residual_vjp(rom_batch* h, const void* q, const void* q_prev, double dt,
                               const void* gbar, void* gq, void* gq_prev, hipStream_t s) {
  rom_status st = h->cfg.precision == ROM_F64
                      ? vjp_t<double>(h, q, q_prev, dt, gbar, gq, gq_prev, s)
                      : vjp_t<float>(h, q, q_prev, dt, gbar, gq, gq_prev, s);
  ROM_HIP_CHECK(hipGetLastError());
  return st;
}

}  // namespace romhip
