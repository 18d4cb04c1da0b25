// Backward-Euler full-order step (eq. fom_discrete_solve, and the coarse step of
// eq. coarse_fom_backward_euler) for batches of small scalar instances, with
// the whole Newton loop of one instance inside one 1024-thread workgroup.
//
// Many small instances (the batched Burgers case: N <= 16384 cells each) leave
// a grid-wide Newton loop dominated by launch latency and by per-instance
// synchronisation.  Here thread k owns the part of m = ceil(N / 1024)
// consecutive cells [k m, k m + m) in registers; its last cell is a separator.
// Per Newton iteration:
//   1. the parts exchange their edge states through LDS (periodic halo);
//   2. each thread evaluates the backward-Euler residual r = y - y_prev - dt f(y)
//      and the Jacobian rows of its cells and eliminates its interior cells by
//      the Thomas recursion, x_j = g_j - V_j x_left_sep - C_j x_{j+1};
//   3. block reductions give ||r||_inf, ||y||_inf; the stopping test is the one
//      of the grid-wide path (||r||_inf <= tol; in FP32 also a last update at
//      round-off level, ||delta||_inf <= 8 eps_32 (1 + ||y||_inf));
//   4. the separators form a cyclic tridiagonal system of P <= 1024 unknowns in
//      LDS, solved by Sherman-Morrison on the corner entries and parallel
//      cyclic reduction with two right-hand sides;
//   5. back-substitution updates the owned cells in registers.
// The state is read once and written once; no atomics, no empty launches.
#include "internal.h"
#include "physics.h"

namespace romhip {

namespace {

constexpr int kFB = 1024;  // threads per workgroup = maximum number of parts

// Block-wide max of a non-negative double (NaN propagates as +inf by the
// callers); red has room for one value per wavefront.  All threads call it.
DEV double block_max(double v, double* red) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off));
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  double m = 0.0;
#pragma unroll
  for (int i = 0; i < kFB / 64; ++i) m = fmax(m, red[i]);
  return m;
}

DEV unsigned block_or(unsigned v, unsigned* red) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v |= __shfl_xor(v, off);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  unsigned m = 0;
#pragma unroll
  for (int i = 0; i < kFB / 64; ++i) m |= red[i];
  return m;
}

// Cyclic tridiagonal system of P >= 3 unknowns in LDS,
//   a_i x_{i-1} + b_i x_i + c_i x_{i+1} = d_i   (indices mod P),
// solved in place (x -> d).  The corner entries a_0 and c_{P-1} are removed by
// Sherman-Morrison with gamma = -b_0: T x = d and T z = u with T tridiagonal,
// then x -= (x_0 + a_0 x_{P-1}/gamma) / (1 + z_0 + a_0 z_{P-1}/gamma) z.  T is
// solved by parallel cyclic reduction with both right-hand sides (e holds u).
// Returns false on a zero pivot.  All threads of the block call it.
template <typename T>
DEV bool cyclic_solve(T* a, T* b, T* c, T* d, T* e, int P) {
  const int i = threadIdx.x;
  __syncthreads();  // the rows were just written by other threads
  const T alpha = a[0], beta = c[P - 1], gamma = -b[0];
  __syncthreads();
  if (i < P) {
    e[i] = i == 0 ? gamma : (i == P - 1 ? beta : T(0));
    if (i == 0) { b[0] -= gamma; a[0] = T(0); }
    if (i == P - 1) { b[P - 1] -= alpha * beta / gamma; c[P - 1] = T(0); }
  }
  __syncthreads();
  bool ok = gamma != T(0);
  for (int s = 1; s < P; s <<= 1) {
    T ai = 0, bi = 1, ci = 0, di = 0, ei = 0;
    T al = 0, bl = 1, cl = 0, dl = 0, el = 0;
    T ar = 0, br = 1, cr = 0, dr = 0, er = 0;
    if (i < P) {
      ai = a[i]; bi = b[i]; ci = c[i]; di = d[i]; ei = e[i];
      if (i - s >= 0) { al = a[i - s]; bl = b[i - s]; cl = c[i - s]; dl = d[i - s]; el = e[i - s]; }
      if (i + s < P) { ar = a[i + s]; br = b[i + s]; cr = c[i + s]; dr = d[i + s]; er = e[i + s]; }
    }
    __syncthreads();
    if (i < P) {
      if (bl == T(0) || br == T(0)) ok = false;
      const T k1 = bl != T(0) ? ai / bl : T(0);
      const T k2 = br != T(0) ? ci / br : T(0);
      a[i] = -al * k1;
      b[i] = bi - cl * k1 - ar * k2;
      c[i] = -cr * k2;
      d[i] = di - dl * k1 - dr * k2;
      e[i] = ei - el * k1 - er * k2;
    }
    __syncthreads();
  }
  if (i < P) {
    if (b[i] == T(0)) ok = false;
    const T bi = b[i] != T(0) ? b[i] : T(1);
    d[i] = d[i] / bi;
    e[i] = e[i] / bi;
  }
  __syncthreads();
  const T fact = (d[0] + alpha * d[P - 1] / gamma) / (T(1) + e[0] + alpha * e[P - 1] / gamma);
  __syncthreads();
  if (i < P) d[i] -= fact * e[i];
  __syncthreads();
  return ok;
}

// Row j of the Newton system of r(y) = y - y_prev - dt f(y) at a scalar cell:
// A y_{j-1} + B y_j + C y_{j+1} = d with A = -dt df_j/dy_{j-1}, B = 1 - dt
// df_j/dy_j, C = -dt df_j/dy_{j+1}, d = -r_j (the rows of the grid-wide path).
template <class Mdl, typename T>
DEV void newton_row(const Mdl& mdl, T qm, T qc, T qn, T qprev, T dt, T inv, T inv2, T& A, T& B,
                    T& C, T& d, unsigned& fl) {
  T f, Jm, J0, Jp;
  cell_jacobian(mdl, &qm, &qc, &qn, false, false, inv, inv2, 0.0, &f, &Jm, &J0, &Jp, fl);
  A = -dt * Jm;
  B = -dt * J0 + T(1);
  C = -dt * Jp;
  d = -(qc - qprev - dt * f);
}

// MM: the largest part length the register arrays hold (N <= 1024 MM).
// Each Newton iteration sweeps the owned cells twice, recomputing the
// Jacobian rows instead of storing them: (i) forward: residual norms, the
// separator row, the last interior cell's expression in the two separators
// and, accumulated along the elimination, the first interior cell's (x_0 =
// sum_j P_j (g_j - V_j x_left) + P x_right with P_j the product of -C_i over
// the cells before j); then the separator system is solved; (ii) forward
// with the left separator known, keeping (C_j, g_j), and back-substitution
// from the right separator.
template <class Mdl, typename T, int MM>
__global__ __launch_bounds__(kFB) void k_fom_newton_block(
    const int64_t* __restrict__ cell_off, const double* __restrict__ phys, int nphys,
    const T* q_prev, T* q_out, T dt, int newton_max, double tol, int32_t* __restrict__ iters,
    uint32_t* __restrict__ flags) {
  static_assert(Mdl::NV == 1 && Mdl::periodic && !Mdl::has_source, "scalar periodic models only");
  __shared__ T sL[kFB], sR[kFB];                  // edge states of every part
  __shared__ T sa[kFB], sb[kFB], sc[kFB], sd[kFB], se[kFB];  // separator system
  __shared__ double red[kFB / 64];
  __shared__ unsigned redu[kFB / 64];
  T* sV = sa;  // first-interior expressions share the system arrays (barrier between)
  T* sW = sb;
  T* sG = sc;
  const int b = blockIdx.x, tid = threadIdx.x;
  const int64_t n = cell_off[b + 1] - cell_off[b];
  const int m = (int)((n + kFB - 1) / kFB);
  const int P = (int)((n + m - 1) / m);
  const bool live = tid < P;
  const int64_t first = (int64_t)tid * m;
  const int len = live ? (int)(n - first < m ? n - first : m) : 0;
  auto part_len = [&](int k) { return (int)(n - (int64_t)k * m < m ? n - (int64_t)k * m : m); };
  const int kl = (tid + P - 1) % P, kr = (tid + 1) % P;
  const int len_r = live ? part_len(kr) : 0;
  const T* qp = q_prev + cell_off[b] + (live ? first : 0);   // this part's cells
  T* qo = q_out + cell_off[b] + (live ? first : 0);
  Mdl mdl(phys + (size_t)b * nphys);
  const T inv = T(n), inv2 = T(n) * T(n);

  T q[MM];
  // the part's state and previous state in registers, loaded unconditionally
  // (indices clamped to the part; a guarded load is waited for on its own)
  T qo_[MM];
  {
    const int lm = len > 0 ? len - 1 : 0;
#pragma unroll
    for (int j = 0; j < MM; ++j) qo_[j] = qp[j < lm ? j : lm];
  }
#pragma unroll
  for (int j = 0; j < MM; ++j) q[j] = j < len ? qo_[j] : T(0);
  unsigned fl = 0;
  int it = 0;
  bool conv = false, sing = false;
  double dprev = 0.0, ynorm = 0.0;
  // neighbours of cell j inside the part (halo values at the part's ends)
#define QM(j) ((j) == 0 ? hl : q[(j) == 0 ? 0 : (j) - 1])
#define QN(j) (((j) + 1 < MM && (j) + 1 < len) ? q[(j) + 1 < MM ? (j) + 1 : (j)] : hr)
  for (;; ++it) {
    // 1. halo exchange
    if (live) {
      T last = q[0];
#pragma unroll
      for (int j = 1; j < MM; ++j)
        if (j == len - 1) last = q[j];
      sL[tid] = q[0];
      sR[tid] = last;
    }
    __syncthreads();
    const T hl = live ? sR[kl] : T(0), hr = live ? sL[kr] : T(0);
    // (i) forward sweep
    T rmax = 0, ymax = 0;
    bool rfin = true;
    T As = 0, Bs = 1, Cs = 0, Ds = 0;      // separator row
    T Ch = 0, Vh = 0, gh = 0;              // x_j = gh - Vh x_left - Ch x_{j+1}
    // the first interior cell in the two separators, accumulated on the way:
    // x_0 = Ga - Va x_left + Pa x_right with Pa the running product of -Ch
    T Ga = 0, Va = 0, Pa = 1;
#pragma unroll
    for (int j = 0; j < MM; ++j) {
      if (j < len) {
        T A, B, C, d;
        newton_row(mdl, QM(j), q[j], QN(j), qo_[j], dt, inv, inv2, A, B, C, d, fl);
        if (!isfinite(d)) { fl |= ROM_FLAG_NONFINITE; rfin = false; }
        else rmax = fmax(rmax, fabs(d));
        ymax = fmax(ymax, fabs(q[j]));
        if (j == len - 1) {
          As = A; Bs = B; Cs = C; Ds = d;
        } else {
          const T Bt = j > 0 ? B - A * Ch : B;
          if (Bt == T(0)) sing = true;
          const T Bi = Bt != T(0) ? T(1) / Bt : T(0);
          if (j == 0) { gh = Bi * d; Vh = Bi * A; }
          else { gh = Bi * (d - A * gh); Vh = -(Bi * (A * Vh)); }
          Ch = Bi * C;
          Ga += Pa * gh;
          Va += Pa * Vh;
          Pa = -(Pa * Ch);
        }
      }
    }
    // 3. stopping test (identical on every thread)
    const double rn = block_max(rfin ? (double)rmax : INFINITY, red);
    const double yn = block_max((double)ymax, red);
    if (it < newton_max) ynorm = yn;
    conv = rn <= tol;
    if (!conv && sizeof(T) == 4 && it > 0)
      conv = dprev <= 8.0 * 1.1920928955078125e-07 * (1.0 + ynorm);
    if (conv || it == newton_max) break;
    // (ii) the first interior cell's expression x_0 = gr - Ar x_left - Wr x_right
    if (live && len >= 2) { sV[tid] = Va; sW[tid] = -Pa; sG[tid] = Ga; }
    __syncthreads();
    // 4. separator row A x_{s-1} + B x_s + C x_{s+1} = d in the separators:
    //    x_{s-1} = gh - Vh x_left - Ch x_s (forward sweep), and
    //    x_{s+1} = G' - V' x_s - W' x_{right of next} (next part's backward sweep)
    T al = As, be = Bs, ga = Cs, de = Ds;
    if (live) {
      if (len >= 2) { al = -As * Vh; be = Bs - As * Ch; de = Ds - As * gh; }
      if (len_r >= 2) { be = be - Cs * sV[kr]; ga = -Cs * sW[kr]; de = de - Cs * sG[kr]; }
    }
    __syncthreads();
    if (live) { sa[tid] = al; sb[tid] = be; sc[tid] = ga; sd[tid] = de; }
    if (!cyclic_solve(sa, sb, sc, sd, se, P)) sing = true;
    // (ii) forward sweep with x_left known, then back-substitution
    double dmax = 0.0;
    if (live) {
      const T xl = sd[kl], xr = sd[tid];
      T Cf[MM], gf[MM];
#pragma unroll
      for (int j = 0; j < MM; ++j) {
        Cf[j] = gf[j] = T(0);
        if (j < len - 1) {
          T A, B, C, d;
          newton_row(mdl, QM(j), q[j], QN(j), qo_[j], dt, inv, inv2, A, B, C, d, fl);
          const T Bt = j > 0 ? B - A * Cf[j > 0 ? j - 1 : 0] : B;
          const T Bi = Bt != T(0) ? T(1) / Bt : T(0);
          const T dd = j > 0 ? d - A * gf[j > 0 ? j - 1 : 0] : d - A * xl;
          Cf[j] = Bi * C;
          gf[j] = Bi * dd;
        }
      }
      T xn = xr;
#pragma unroll
      for (int j = MM - 1; j >= 0; --j) {
        if (j < len) {
          const T x = j == len - 1 ? xr : gf[j] - Cf[j] * xn;
          xn = x;
          q[j] += x;
          if (!isfinite(x)) dmax = INFINITY;
          else dmax = fmax(dmax, (double)fabs(x));
        }
      }
    }
    dprev = block_max(dmax, red);
  }
#undef QM
#undef QN
  if (sing) fl |= ROM_FLAG_SINGULAR;
  if (!conv) fl |= ROM_FLAG_NEWTON_NOCONV;
  fl = block_or(fl, redu);
#pragma unroll
  for (int j = 0; j < MM; ++j)
    if (j < len) qo[j] = q[j];
  if (tid == 0) {
    if (iters) iters[b] = it;
    if (fl) atomicOr(&flags[b], fl);
  }
}

}  // namespace

bool fom_block_ok(const rom_batch* h) {
  if (h->cfg.problem != ROM_BURGERS) return false;
  const int64_t cap = (int64_t)kFB * (h->cfg.precision == ROM_F32 ? 16 : 8);
  for (int64_t n : h->n_cells)
    if (n > cap) return false;
  return true;
}

rom_status launch_fom_block(rom_batch* h, const void* q_prev, double dt, void* q_out,
                            int32_t* iters, hipStream_t s) {
  const int B = h->cfg.n_inst;
  if (h->cfg.precision == ROM_F32)
    hipLaunchKernelGGL((k_fom_newton_block<BurgersModel<float>, float, 16>), dim3(B), dim3(kFB), 0,
                       s, h->d_cell_off, h->d_phys, h->cfg.n_phys, (const float*)q_prev,
                       (float*)q_out, (float)dt, h->cfg.newton_max, h->cfg.newton_tol, iters,
                       h->flags);
  else
    hipLaunchKernelGGL((k_fom_newton_block<BurgersModel<double>, double, 8>), dim3(B), dim3(kFB), 0,
                       s, h->d_cell_off, h->d_phys, h->cfg.n_phys, (const double*)q_prev,
                       (double*)q_out, dt, h->cfg.newton_max, h->cfg.newton_tol, iters, h->flags);
  ROM_HIP_CHECK(hipGetLastError());
  return ROM_OK;
}

}  // namespace romhip
