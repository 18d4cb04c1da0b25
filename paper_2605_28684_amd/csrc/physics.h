// Device-side physics of the full-order finite-volume models.
//
// Every model has the form (periodic or zero-gradient walls, dx = 1/N)
//   f_i = -(H(q_i, q_{i+1}) - H(q_{i-1}, q_i)) / dx
//         + kappa_v ((q_{i+1} - q_i) - (q_i - q_{i-1})) / dx^2 + S(q_i, x_i)
// with a two-point face flux H, a per-variable diffusion coefficient and a
// cell-local source.  The diffusion is evaluated difference-first, which keeps
// single-precision cancellation at the level of the differences.
//
//  Burgers   H = Godunov flux of u^2/2: max(g(max(a,0)), g(min(b,0))); kappa = nu
//            (paper Sec. 5.1, eq. burgers_pde_results; upwind read as Godunov)
//  Euler     H = Rusanov (App. B eqs. sod_rusanov_flux/speed) or HLLC (Toro,
//            Davis speeds); ideal gas; rho, p floored on recovery only
//  React     u: Godunov + nu_u; Y_l, T: face velocity (u_L+u_R)/2 times the
//            upwind value, kappa; Arrhenius source, inflow relaxation
//
// Branches (max/min/abs/upwind) are decided on values; ties take the first
// argument, and derivatives follow the branch taken.
#pragma once
#include <hip/hip_runtime.h>

#include <cmath>

#define DEV __device__ __forceinline__

namespace romhip {

constexpr double kRhoMin = 1e-10;
constexpr double kPMin = 1e-10;
constexpr double kTFloor = 1e-2;

// ---------------------------------------------------------------- forward-mode dual
template <typename T, int N>
struct Dual {
  T v;
  T d[N];
  DEV Dual() {}
  DEV Dual(T x) : v(x) {
#pragma unroll
    for (int i = 0; i < N; ++i) d[i] = T(0);
  }
};

template <typename T>
DEV T val(T x) { return x; }
template <typename T, int N>
DEV T val(const Dual<T, N>& x) { return x.v; }

template <typename T, int N>
DEV Dual<T, N> operator+(const Dual<T, N>& a, const Dual<T, N>& b) {
  Dual<T, N> r; r.v = a.v + b.v;
#pragma unroll
  for (int i = 0; i < N; ++i) r.d[i] = a.d[i] + b.d[i];
  return r;
}
template <typename T, int N>
DEV Dual<T, N> operator-(const Dual<T, N>& a, const Dual<T, N>& b) {
  Dual<T, N> r; r.v = a.v - b.v;
#pragma unroll
  for (int i = 0; i < N; ++i) r.d[i] = a.d[i] - b.d[i];
  return r;
}
template <typename T, int N>
DEV Dual<T, N> operator-(const Dual<T, N>& a) {
  Dual<T, N> r; r.v = -a.v;
#pragma unroll
  for (int i = 0; i < N; ++i) r.d[i] = -a.d[i];
  return r;
}
template <typename T, int N>
DEV Dual<T, N> operator*(const Dual<T, N>& a, const Dual<T, N>& b) {
  Dual<T, N> r; r.v = a.v * b.v;
#pragma unroll
  for (int i = 0; i < N; ++i) r.d[i] = a.d[i] * b.v + a.v * b.d[i];
  return r;
}
template <typename T, int N>
DEV Dual<T, N> operator/(const Dual<T, N>& a, const Dual<T, N>& b) {
  Dual<T, N> r; r.v = a.v / b.v;
  const T ib = T(1) / b.v;
#pragma unroll
  for (int i = 0; i < N; ++i) r.d[i] = (a.d[i] - r.v * b.d[i]) * ib;
  return r;
}
template <typename T, int N>
DEV Dual<T, N> operator+(const Dual<T, N>& a, T b) { Dual<T, N> r = a; r.v += b; return r; }
template <typename T, int N>
DEV Dual<T, N> operator+(T b, const Dual<T, N>& a) { Dual<T, N> r = a; r.v += b; return r; }
template <typename T, int N>
DEV Dual<T, N> operator-(const Dual<T, N>& a, T b) { Dual<T, N> r = a; r.v -= b; return r; }
template <typename T, int N>
DEV Dual<T, N> operator-(T b, const Dual<T, N>& a) { return Dual<T, N>(b) - a; }
template <typename T, int N>
DEV Dual<T, N> operator*(const Dual<T, N>& a, T b) {
  Dual<T, N> r; r.v = a.v * b;
#pragma unroll
  for (int i = 0; i < N; ++i) r.d[i] = a.d[i] * b;
  return r;
}
template <typename T, int N>
DEV Dual<T, N> operator*(T b, const Dual<T, N>& a) { return a * b; }
template <typename T, int N>
DEV Dual<T, N> operator/(const Dual<T, N>& a, T b) { return a * (T(1) / b); }
template <typename T, int N>
DEV Dual<T, N> operator/(T a, const Dual<T, N>& b) { return Dual<T, N>(a) / b; }

DEV float dsqrt(float x) { return sqrtf(x); }
DEV double dsqrt(double x) { return sqrt(x); }
template <typename T, int N>
DEV Dual<T, N> dsqrt(const Dual<T, N>& a) {
  Dual<T, N> r; r.v = dsqrt(a.v);
  const T k = T(0.5) / r.v;
#pragma unroll
  for (int i = 0; i < N; ++i) r.d[i] = a.d[i] * k;
  return r;
}
DEV float dexp(float x) { return expf(x); }
DEV double dexp(double x) { return exp(x); }

// max / min / abs deciding on values; ties take the first argument
template <typename S>
DEV S smax(const S& a, const S& b) { return val(a) >= val(b) ? a : b; }
template <typename S>
DEV S smin(const S& a, const S& b) { return val(a) <= val(b) ? a : b; }
template <typename S>
DEV S sabs(const S& a) { return val(a) >= decltype(val(a))(0) ? a : -a; }

// ---------------------------------------------------------------- Burgers face
// Godunov flux of g(u) = u^2/2 with derivatives (dF/da, dF/db).
template <typename T>
DEV T godunov(T a, T b, T& da, T& db) {
  const T a0 = a > T(0) ? a : T(0);
  const T b0 = b < T(0) ? b : T(0);
  const T g1 = T(0.5) * a0 * a0;
  const T g2 = T(0.5) * b0 * b0;
  if (g1 >= g2) { da = a0; db = T(0); return g1; }
  da = T(0); db = b0; return g2;
}

// ---------------------------------------------------------------- Euler faces
template <typename S, typename R>
DEV void euler_prim(const S U[3], R gamma, S& rf, S& u, S& p, S& c, unsigned& fl) {
  rf = smax(U[0], S(R(kRhoMin)));
  if (val(U[0]) < R(kRhoMin)) fl |= ROM_FLAG_FLOOR;
  u = U[1] / rf;
  const S pe = (gamma - R(1)) * (U[2] - R(0.5) * U[1] * u);
  if (val(pe) < R(kPMin)) fl |= ROM_FLAG_FLOOR;
  p = smax(pe, S(R(kPMin)));
  c = dsqrt(gamma * p / rf);
}

template <typename S, typename R>
DEV void rusanov_face(const S* UL, const S* UR, R gamma, S* F, unsigned& fl) {
  S rL, uL, pL, cL, rR, uR, pR, cR;
  euler_prim(UL, gamma, rL, uL, pL, cL, fl);
  euler_prim(UR, gamma, rR, uR, pR, cR, fl);
  const S s = smax(sabs(uL) + cL, sabs(uR) + cR);
  const S FL0 = UL[1], FL1 = UL[1] * uL + pL, FL2 = uL * (UL[2] + pL);
  const S FR0 = UR[1], FR1 = UR[1] * uR + pR, FR2 = uR * (UR[2] + pR);
  const R h = R(0.5);
  F[0] = h * (FL0 + FR0) - h * s * (UR[0] - UL[0]);
  F[1] = h * (FL1 + FR1) - h * s * (UR[1] - UL[1]);
  F[2] = h * (FL2 + FR2) - h * s * (UR[2] - UL[2]);
}

template <typename S, typename R>
DEV void hllc_face(const S* UL, const S* UR, R gamma, S* F, unsigned& fl) {
  S rL, uL, pL, cL, rR, uR, pR, cR;
  euler_prim(UL, gamma, rL, uL, pL, cL, fl);
  euler_prim(UR, gamma, rR, uR, pR, cR, fl);
  const S SL = smin(uL - cL, uR - cR);
  const S SR = smax(uL + cL, uR + cR);
  if (val(SL) >= R(0)) {
    F[0] = UL[1]; F[1] = UL[1] * uL + pL; F[2] = uL * (UL[2] + pL);
    return;
  }
  const S num = pR - pL + rL * uL * (SL - uL) - rR * uR * (SR - uR);
  const S den = rL * (SL - uL) - rR * (SR - uR);
  const S Ss = num / den;
  if (val(Ss) >= R(0)) {
    const S fac = rL * (SL - uL) / (SL - Ss);
    const S e = UL[2] / rL + (Ss - uL) * (Ss + pL / (rL * (SL - uL)));
    F[0] = UL[1] + SL * (fac - UL[0]);
    F[1] = UL[1] * uL + pL + SL * (fac * Ss - UL[1]);
    F[2] = uL * (UL[2] + pL) + SL * (fac * e - UL[2]);
    return;
  }
  if (val(SR) >= R(0)) {
    const S fac = rR * (SR - uR) / (SR - Ss);
    const S e = UR[2] / rR + (Ss - uR) * (Ss + pR / (rR * (SR - uR)));
    F[0] = UR[1] + SR * (fac - UR[0]);
    F[1] = UR[1] * uR + pR + SR * (fac * Ss - UR[1]);
    F[2] = uR * (UR[2] + pR) + SR * (fac * e - UR[2]);
    return;
  }
  F[0] = UR[1]; F[1] = UR[1] * uR + pR; F[2] = uR * (UR[2] + pR);
}

// ---------------------------------------------------------------- model structs
// Each model exposes: NV, periodic, kappa(v), face(L, R, H, fl) in the bulk
// type, face_jac(L, R, H, DL, DR, fl) with row-major NV x NV blocks
// dH/dq_L and dH/dq_R, and source / source_jac (cell-local terms).

template <typename T>
struct BurgersModel {
  static constexpr int NV = 1;
  static constexpr bool periodic = true;
  static constexpr bool has_source = false;
  T nu;
  DEV explicit BurgersModel(const double* ph) : nu(T(ph[0])) {}
  DEV T kappa(int) const { return nu; }
  DEV void face(const T* L, const T* R, T* H, unsigned&) const {
    T da, db; H[0] = godunov(L[0], R[0], da, db);
  }
  DEV void face_jac(const T* L, const T* R, T* H, T* DL, T* DR, unsigned&) const {
    H[0] = godunov(L[0], R[0], DL[0], DR[0]);
  }
  DEV void source(const T*, double, T*, unsigned&) const {}
  DEV void source_jac(const T*, double, T*, T*, unsigned&) const {}
};

template <typename T, bool HLLC>
struct EulerModel {
  static constexpr int NV = 3;
  static constexpr bool periodic = false;
  static constexpr bool has_source = false;
  T gamma;
  DEV explicit EulerModel(const double* ph) : gamma(T(ph[0])) {}
  DEV T kappa(int) const { return T(0); }
  DEV void face(const T* L, const T* R, T* H, unsigned& fl) const {
    if (HLLC) hllc_face<T, T>(L, R, gamma, H, fl);
    else rusanov_face<T, T>(L, R, gamma, H, fl);
  }
  DEV void face_jac(const T* L, const T* R, T* H, T* DL, T* DR, unsigned& fl) const {
    using D = Dual<T, 6>;
    D UL[3], UR[3], F[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      UL[k] = D(L[k]); UL[k].d[k] = T(1);
      UR[k] = D(R[k]); UR[k].d[3 + k] = T(1);
    }
    if (HLLC) hllc_face<D, T>(UL, UR, gamma, F, fl);
    else rusanov_face<D, T>(UL, UR, gamma, F, fl);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      H[i] = F[i].v;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        DL[i * 3 + k] = F[i].d[k];
        DR[i * 3 + k] = F[i].d[3 + k];
      }
    }
  }
  DEV void source(const T*, double, T*, unsigned&) const {}
  DEV void source_jac(const T*, double, T*, T*, unsigned&) const {}
};

// synthetic ten-species model: q = [Y_1..Y_10, T, u]
template <typename T>
struct ReactModel {
  static constexpr int NV = 12;
  static constexpr bool periodic = true;
  static constexpr bool has_source = true;
  const double* ph;  // nu_u, kappa, A, k_in, x_in, T_in, Y_in[10], a,b,c,d[12], E[12], Q[12]
  DEV explicit ReactModel(const double* p) : ph(p) {}
  DEV T kappa(int v) const { return v == 11 ? T(ph[0]) : T(ph[1]); }
  DEV void face(const T* L, const T* R, T* H, unsigned&) const {
    T da, db;
    H[11] = godunov(L[11], R[11], da, db);
    const T uf = T(0.5) * (L[11] + R[11]);
    const bool left = uf >= T(0);
#pragma unroll
    for (int v = 0; v < 11; ++v) H[v] = uf * (left ? L[v] : R[v]);
  }
  DEV void face_jac(const T* L, const T* R, T* H, T* DL, T* DR, unsigned&) const {
#pragma unroll
    for (int i = 0; i < 144; ++i) { DL[i] = T(0); DR[i] = T(0); }
    H[11] = godunov(L[11], R[11], DL[11 * 12 + 11], DR[11 * 12 + 11]);
    const T uf = T(0.5) * (L[11] + R[11]);
    const bool left = uf >= T(0);
#pragma unroll
    for (int v = 0; v < 11; ++v) {
      const T up = left ? L[v] : R[v];
      H[v] = uf * up;
      DL[v * 12 + 11] = T(0.5) * up;
      DR[v * 12 + 11] = T(0.5) * up;
      if (left) DL[v * 12 + v] = uf; else DR[v * 12 + v] = uf;
    }
  }
  DEV void source(const T* q, double x, T* S, unsigned& fl) const {
    const T A = T(ph[2]);
    const T Tc = q[10];
    if (Tc < T(kTFloor)) fl |= ROM_FLAG_FLOOR;
    const T Tf = Tc >= T(kTFloor) ? Tc : T(kTFloor);
#pragma unroll
    for (int v = 0; v < 12; ++v) S[v] = T(0);
    for (int j = 0; j < 12; ++j) {
      const int ia = int(ph[16 + j]), ib = int(ph[28 + j]), ic = int(ph[40 + j]), id = int(ph[52 + j]);
      const T w = A * dexp(-T(ph[64 + j]) / Tf) * q[ia] * q[ib];
      S[ia] -= w; S[ib] -= w; S[ic] += w; S[id] += w;
      S[10] += T(ph[76 + j]) * w;
    }
    if (x < ph[4]) {
      const T kin = T(ph[3]);
      for (int l = 0; l < 10; ++l) S[l] += kin * (T(ph[6 + l]) - q[l]);
      S[10] += kin * (T(ph[5]) - q[10]);
    }
  }
  // Row v of face_jac: H_v and row v of dH/dq_L, dH/dq_R, with the same
  // arithmetic as the full blocks.  Used where only sampled rows are needed.
  DEV void face_jac_row(const T* L, const T* R, int v, T& H, T* dl, T* dr) const {
#pragma unroll
    for (int w = 0; w < 12; ++w) { dl[w] = T(0); dr[w] = T(0); }
    const T uf = T(0.5) * (L[11] + R[11]);
    const bool left = uf >= T(0);
    if (v == 11) {
      H = godunov(L[11], R[11], dl[11], dr[11]);
    } else {
      const T up = left ? L[v] : R[v];
      H = uf * up;
      dl[11] = T(0.5) * up;
      dr[11] = T(0.5) * up;
#pragma unroll
      for (int w = 0; w < 11; ++w)
        if (w == v) { if (left) dl[w] = uf; else dr[w] = uf; }
    }
  }
  // Row v of source_jac: S_v and row v of dS/dq, accumulated in the same order
  // as the full block.
  DEV void source_jac_row(const T* q, double x, int v, T& Sv, T* ds, unsigned& fl) const {
    const T A = T(ph[2]);
    const T Tc = q[10];
    if (Tc < T(kTFloor)) fl |= ROM_FLAG_FLOOR;
    const bool live = Tc >= T(kTFloor);
    const T Tf = live ? Tc : T(kTFloor);
    Sv = T(0);
#pragma unroll
    for (int w = 0; w < 12; ++w) ds[w] = T(0);
    auto put = [&](int ia, int ib, T s, T dwa, T dwb, T dwT) {
#pragma unroll
      for (int w = 0; w < 12; ++w) {
        if (w == ia) ds[w] += s * dwa;
        if (w == ib) ds[w] += s * dwb;
        if (w == 10) ds[w] += s * dwT;
      }
    };
    for (int j = 0; j < 12; ++j) {
      const int ia = int(ph[16 + j]), ib = int(ph[28 + j]), ic = int(ph[40 + j]), id = int(ph[52 + j]);
      const T E = T(ph[64 + j]);
      const T k = A * dexp(-E / Tf);
      const T w = k * q[ia] * q[ib];
      const T dwa = k * q[ib], dwb = k * q[ia];
      const T dwT = live ? w * E / (Tf * Tf) : T(0);
      const int rows[4] = {ia, ib, ic, id};
      const T sg[4] = {T(-1), T(-1), T(1), T(1)};
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        if (rows[m] == v) {
          Sv += sg[m] * w;
          put(ia, ib, sg[m], dwa, dwb, dwT);
        }
      }
      if (v == 10) {
        const T Qj = T(ph[76 + j]);
        Sv += Qj * w;
        put(ia, ib, Qj, dwa, dwb, dwT);
      }
    }
    if (x < ph[4]) {
      const T kin = T(ph[3]);
      if (v < 10) Sv += kin * (T(ph[6 + v]) - q[v]);
      if (v == 10) Sv += kin * (T(ph[5]) - q[10]);
#pragma unroll
      for (int w = 0; w < 11; ++w)
        if (w == v) ds[w] -= kin;
    }
  }
  // S and dS/dq (row-major 12 x 12).  Reaction j adds g_j w_j to S and the outer
  // product g_j h_j to dS/dq, with g_j the stoichiometric column (-1 at the two
  // reactants, +1 at the two products, Q_j at the temperature) and h_j = dw_j/dq
  // (nonzero at the two reactants and the temperature); both are formed with
  // constant indices so that S and dS/dq stay in registers.
  DEV void source_jac(const T* q, double x, T* S, T* DS, unsigned& fl) const {
    const T A = T(ph[2]);
    const T Tc = q[10];
    if (Tc < T(kTFloor)) fl |= ROM_FLAG_FLOOR;
    const bool live = Tc >= T(kTFloor);
    const T Tf = live ? Tc : T(kTFloor);
#pragma unroll
    for (int v = 0; v < 12; ++v) S[v] = T(0);
#pragma unroll
    for (int i = 0; i < 144; ++i) DS[i] = T(0);
    for (int j = 0; j < 12; ++j) {
      const int ia = int(ph[16 + j]), ib = int(ph[28 + j]), ic = int(ph[40 + j]), id = int(ph[52 + j]);
      const T E = T(ph[64 + j]);
      const T k = A * dexp(-E / Tf);
      T qa = T(0), qb = T(0);
#pragma unroll
      for (int v = 0; v < 12; ++v) {
        if (v == ia) qa = q[v];
        if (v == ib) qb = q[v];
      }
      const T w = k * qa * qb;
      const T dwa = k * qb, dwb = k * qa;
      const T dwT = live ? w * E / (Tf * Tf) : T(0);
      const T Qj = T(ph[76 + j]);
      T g[12], hc[12];
#pragma unroll
      for (int v = 0; v < 12; ++v) {
        g[v] = (v == ia ? T(-1) : T(0)) + (v == ib ? T(-1) : T(0)) + (v == ic ? T(1) : T(0)) +
               (v == id ? T(1) : T(0)) + (v == 10 ? Qj : T(0));
        hc[v] = (v == ia ? dwa : T(0)) + (v == ib ? dwb : T(0)) + (v == 10 ? dwT : T(0));
      }
#pragma unroll
      for (int v = 0; v < 12; ++v) {
        S[v] += g[v] * w;
#pragma unroll
        for (int c = 0; c < 12; ++c) DS[v * 12 + c] += g[v] * hc[c];
      }
    }
    if (x < ph[4]) {
      const T kin = T(ph[3]);
#pragma unroll
      for (int l = 0; l < 10; ++l) {
        S[l] += kin * (T(ph[6 + l]) - q[l]);
        DS[l * 12 + l] -= kin;
      }
      S[10] += kin * (T(ph[5]) - q[10]);
      DS[10 * 12 + 10] -= kin;
    }
  }
};

// Jacobian blocks of f at cell i: Jm = df_i/dq_{i-1}, J0 = df_i/dq_i, Jp = df_i/dq_{i+1}
// and f_i itself.  sq holds cells i-1, i, i+1 at qm, q0, qp.  lw/rw mark a
// zero-gradient wall on the left / right (ghost = copy of the end cell).
// The cell's part given its two faces: face i-1/2 (flux HL, derivatives DLl /
// DRl with respect to q_{i-1} / q_i) and face i+1/2 (HR, DLr / DRr with respect
// to q_i / q_{i+1}).  Each face (FA) may be any indexable of NV or NV x NV
// values (registers or a view of LDS).
template <class Mdl, typename T, class FA>
DEV void cell_combine(const Mdl& m, const FA& HL, const FA& DLl, const FA& DRl, const FA& HR,
                      const FA& DLr, const FA& DRr, const T* qm, const T* q0, const T* qp,
                      bool lw, bool rw, T inv, T inv2, double x, T* f, T* Jm, T* J0, T* Jp,
                      unsigned& fl) {
  constexpr int NV = Mdl::NV;
  constexpr int NN = NV * NV;
  // f_i = -(HR - HL) inv
#pragma unroll
  for (int v = 0; v < NV; ++v) f[v] = -(HR[v] - HL[v]) * inv;
#pragma unroll
  for (int e = 0; e < NN; ++e) {
    Jm[e] = DLl[e] * inv;
    J0[e] = (DRl[e] - DLr[e]) * inv;
    Jp[e] = -DRr[e] * inv;
  }
  if (lw) {  // ghost q_{-1} = q_0: the left face depends on q_0 through both sides
#pragma unroll
    for (int e = 0; e < NN; ++e) { J0[e] += Jm[e]; Jm[e] = T(0); }
  }
  if (rw) {
#pragma unroll
    for (int e = 0; e < NN; ++e) { J0[e] += Jp[e]; Jp[e] = T(0); }
  }
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    const T kap = m.kappa(v);
    if (kap != T(0)) {
      f[v] += kap * ((qp[v] - q0[v]) - (q0[v] - qm[v])) * inv2;
      const T c = kap * inv2;
      // ghost neighbours fold onto the diagonal at walls
      Jm[v * NV + v] += lw ? T(0) : c;
      Jp[v * NV + v] += rw ? T(0) : c;
      J0[v * NV + v] += -T(2) * c + (lw ? c : T(0)) + (rw ? c : T(0));
    }
  }
  if (Mdl::has_source) {
    T S[NV], DS[NN];
    m.source_jac(q0, x, S, DS, fl);
#pragma unroll
    for (int v = 0; v < NV; ++v) f[v] += S[v];
#pragma unroll
    for (int e = 0; e < NN; ++e) J0[e] += DS[e];
  }
}

template <class Mdl, typename T>
DEV void cell_jacobian(const Mdl& m, const T* qm, const T* q0, const T* qp, bool lw, bool rw,
                       T inv, T inv2, double x, T* f, T* Jm, T* J0, T* Jp, unsigned& fl) {
  constexpr int NV = Mdl::NV;
  constexpr int NN = NV * NV;
  T HL[NV], HR[NV], DLl[NN], DRl[NN], DLr[NN], DRr[NN];
  m.face_jac(qm, q0, HL, DLl, DRl, fl);   // face i-1/2: (q_{i-1}, q_i)
  m.face_jac(q0, qp, HR, DLr, DRr, fl);   // face i+1/2: (q_i, q_{i+1})
  const T* hl = HL; const T* dll = DLl; const T* drl = DRl;
  const T* hr = HR; const T* dlr = DLr; const T* drr = DRr;
  cell_combine(m, hl, dll, drl, hr, dlr, drr, qm, q0, qp, lw, rw, inv, inv2, x, f, Jm, J0, Jp, fl);
}

}  // namespace romhip
