// Device functions of the vertex-centred residual: simplex geometry,
// limiters and the face fluxes, templated on the compute type (double for the
// FP64 path, float for the mixed path).
#pragma once
#include <hip/hip_runtime.h>

namespace vcx {

// local cell-edges (a, b), a < b
template <int ND> struct Edges;
template <> struct Edges<2> {
  static constexpr int NE = 3;
  __device__ static constexpr int a(int e) { return e == 2 ? 1 : 0; }
  __device__ static constexpr int b(int e) { return e == 0 ? 1 : 2; }
};
template <> struct Edges<3> {
  static constexpr int NE = 6;
  __device__ static constexpr int a(int e) { return e < 3 ? 0 : (e < 5 ? 1 : 2); }
  __device__ static constexpr int b(int e) { return e < 3 ? e + 1 : (e == 3 ? 2 : 3); }
};

// Node normals of a positively oriented simplex from the relative vertex
// coordinates e[k-1] = X_k - X_0: S_k = -n_d V grad(lambda_k), i.e. the
// outward area vector of the face opposite vertex k.  Returns the signed
// measure det(e) (= n_d! V).
template <int ND, typename T>
__device__ inline T simplex_normals(const T (&e)[ND][ND], T (&S)[ND + 1][ND]) {
  if constexpr (ND == 2) {
    S[1][0] = -e[1][1]; S[1][1] = e[1][0];
    S[2][0] = e[0][1];  S[2][1] = -e[0][0];
    S[0][0] = -(S[1][0] + S[2][0]);
    S[0][1] = -(S[1][1] + S[2][1]);
    return e[0][0] * e[1][1] - e[0][1] * e[1][0];
  } else {
    const T h = T(-0.5);
    S[1][0] = h * (e[1][1] * e[2][2] - e[1][2] * e[2][1]);
    S[1][1] = h * (e[1][2] * e[2][0] - e[1][0] * e[2][2]);
    S[1][2] = h * (e[1][0] * e[2][1] - e[1][1] * e[2][0]);
    S[2][0] = h * (e[2][1] * e[0][2] - e[2][2] * e[0][1]);
    S[2][1] = h * (e[2][2] * e[0][0] - e[2][0] * e[0][2]);
    S[2][2] = h * (e[2][0] * e[0][1] - e[2][1] * e[0][0]);
    S[3][0] = h * (e[0][1] * e[1][2] - e[0][2] * e[1][1]);
    S[3][1] = h * (e[0][2] * e[1][0] - e[0][0] * e[1][2]);
    S[3][2] = h * (e[0][0] * e[1][1] - e[0][1] * e[1][0]);
    for (int d = 0; d < 3; ++d) S[0][d] = -(S[1][d] + S[2][d] + S[3][d]);
    return e[0][0] * (e[1][1] * e[2][2] - e[1][2] * e[2][1]) -
           e[0][1] * (e[1][0] * e[2][2] - e[1][2] * e[2][0]) +
           e[0][2] * (e[1][0] * e[2][1] - e[1][1] * e[2][0]);
  }
}

// Sides of a 2D quadrilateral (vertices in counter-clockwise cyclic order):
// its cell-edges (its diagonals are not edges)
struct QuadEdges {
  static constexpr int NE = 4;
  __device__ static constexpr int a(int e) { return e; }
  __device__ static constexpr int b(int e) { return e == 3 ? 0 : e + 1; }
};

// Node normals of a counter-clockwise quadrilateral from its relative vertex
// coordinates e[k-1] = X_k - X_0 (eq. node_normal: in 2D each face is a side
// of two vertices, so S_k = -(S_f + S_g) over the two sides through k, which
// is the vector X_{k+1} - X_{k-1} turned a quarter counter-clockwise).
// Returns twice the area.
template <typename T>
__device__ inline T quad_normals(const T (&e)[3][2], T (&S)[4][2]) {
  // P_0 = 0, P_k = e[k-1]
  S[0][0] = -(e[0][1] - e[2][1]);
  S[0][1] = e[0][0] - e[2][0];
  S[1][0] = -e[1][1];
  S[1][1] = e[1][0];
  S[2][0] = -(e[2][1] - e[0][1]);
  S[2][1] = e[2][0] - e[0][0];
  S[3][0] = e[1][1];
  S[3][1] = -e[1][0];
  return (e[0][0] * e[1][1] - e[0][1] * e[1][0]) + (e[1][0] * e[2][1] - e[1][1] * e[2][0]);
}

// Cell shapes: the simplex of dimension ND (NV = ND + 1) and the 2D
// quadrilateral (NV = 4).  E: its cell-edges; normals(e, S): node normals,
// returning the measure that kvol turns into the volume; kdual: the dual-face
// vector of cell-edge (a, b) is (S_a - S_b) kdual (1/(n_d n_v) for simplices;
// for a quadrilateral 1/4, the segment from the side's midpoint to the mean
// of the vertices).
template <int ND, int NV>
struct Shape {
  static_assert(NV == ND + 1, "simplices");
  using E = Edges<ND>;
  static constexpr double kdual = 1.0 / double(ND * NV);
  static constexpr double kvol = ND == 2 ? 0.5 : 1.0 / 6.0;
  template <typename T>
  __device__ static T normals(const T (&e)[ND][ND], T (&S)[NV][ND]) {
    return simplex_normals<ND>(e, S);
  }
};
template <>
struct Shape<2, 4> {
  using E = QuadEdges;
  static constexpr double kdual = 0.25;
  static constexpr double kvol = 0.5;
  template <typename T>
  __device__ static T normals(const T (&e)[3][2], T (&S)[4][2]) {
    return quad_normals(e, S);
  }
};

// Slope limiter L(a, b) (kinds as vcx.h VCX_LIM_*).
template <typename T>
__device__ inline T slope_limit(int kind, T beta, T a, T b) {
  if (kind == 0) return T(0);
  if (kind == 4) return T(0.5) * (a + b);
  if (!(a * b > T(0))) return T(0);
  if (kind == 2) return T(2) * a * b / (a + b);
  T aa = fabs(a), bb = fabs(b);
  T r = kind == 1 ? fmin(aa, bb) : fmax(fmin(beta * aa, bb), fmin(aa, beta * bb));
  return a > T(0) ? r : -r;
}

// Flux limiter Psi of the limited Lax-Wendroff flux, R = a / b.
template <typename T>
__device__ inline T psi_limit(int kind, T beta, T a, T b) {
  if (kind == 0) return T(0);
  if (kind == 4) return T(1);
  if (!(a * b > T(0))) return T(0);
  T R = a / b;  // > 0
  if (kind == 2) return T(2) * R / (T(1) + R);
  T bt = kind == 1 ? T(1) : beta;
  return fmax(fmin(bt * R, T(1)), fmin(R, bt));
}

// Physical flux through the unit normal n of the reconstructed state
// W = (rho, rho u, rho E, rho Y, p).
template <int ND, int NSP, typename T>
__device__ inline void normal_flux(const T* W, const T* n, T* F, T& q) {
  constexpr int NV = 2 + ND + NSP;
  const T rho = W[0], p = W[NV];
  const T ir = T(1) / rho;
  q = T(0);
  for (int d = 0; d < ND; ++d) q += W[1 + d] * n[d];
  q *= ir;
  F[0] = rho * q;
  for (int d = 0; d < ND; ++d) F[1 + d] = W[1 + d] * q + p * n[d];
  F[1 + ND] = (W[1 + ND] + p) * q;
  for (int k = 0; k < NSP; ++k) F[2 + ND + k] = W[2 + ND + k] * q;
}

// Normal velocity q = (rho u . n) / rho of a reconstructed state, as
// normal_flux forms it.
template <int ND, typename T>
__device__ inline T normal_velocity(const T* W, const T* n) {
  T q = T(0);
  for (int d = 0; d < ND; ++d) q += W[1 + d] * n[d];
  return q * (T(1) / W[0]);
}

// HLLC flux through the area vector S (result scaled by |S|), Davis wave
// speeds, star states of the paper's multicomponent HLLC; gL, gR: ratio of
// specific heats of the left and right states.  Only the physical flux of
// the side a branch needs is formed.
template <int ND, int NSP, typename T>
__device__ inline void hllc_flux(const T* WL, const T* WR, const T* S, T gL, T gR, T* F) {
  constexpr int NV = 2 + ND + NSP;
  T A2 = T(0);
  for (int d = 0; d < ND; ++d) A2 += S[d] * S[d];
  const T A = sqrt(A2), iA = T(1) / A;
  T n[ND];
  for (int d = 0; d < ND; ++d) n[d] = S[d] * iA;
  const T qL = normal_velocity<ND>(WL, n), qR = normal_velocity<ND>(WR, n);
  const T rL = WL[0], rR = WR[0], pL = WL[NV], pR = WR[NV];
  const T aL = sqrt(gL * pL / rL), aR = sqrt(gR * pR / rR);
  const T SL = fmin(qL - aL, qR - aR), SR = fmax(qL + aL, qR + aR);
  const T mL = rL * (SL - qL), mR = rR * (SR - qR);
  const T Ss = (pR - pL + mL * qL - mR * qR) / (mL - mR);
  // the side whose flux the branch starts from
  const bool left = (T(0) <= SL) || (!(SR < T(0)) && T(0) <= Ss);
  T W[NV + 1];
  for (int v = 0; v <= NV; ++v) W[v] = left ? WL[v] : WR[v];
  T FK[NV], qK;
  normal_flux<ND, NSP>(W, n, FK, qK);
  if (T(0) <= SL || SR < T(0)) {
    for (int v = 0; v < NV; ++v) F[v] = A * FK[v];
  } else {
    const T SK = left ? SL : SR, rK = W[0], pK = W[NV];
    const T irK = T(1) / rK;
    const T fac = rK * (SK - qK) / (SK - Ss);
    const T dq = Ss - qK;
    // star state minus own state, times the wave speed
    F[0] = A * (FK[0] + SK * (fac - rK));
    for (int d = 0; d < ND; ++d)
      F[1 + d] = A * (FK[1 + d] + SK * (fac * (W[1 + d] * irK + dq * n[d]) - W[1 + d]));
    F[1 + ND] = A * (FK[1 + ND] + SK * (fac * (W[1 + ND] * irK + dq * (Ss + pK / (rK * (SK - qK)))) -
                                       W[1 + ND]));
    for (int k = 0; k < NSP; ++k)
      F[2 + ND + k] = A * (FK[2 + ND + k] + SK * (fac * irK - T(1)) * W[2 + ND + k]);
  }
}

// Roe flux (textbook; the paper names Riemann solvers but prints only HLLC),
// sqrt(rho) averages, Harten entropy fix on the acoustic waves.
template <int ND, int NSP, typename T>
__device__ inline void roe_flux(const T* WL, const T* WR, const T* S, T gamma, T fix, T* F) {
  constexpr int NV = 2 + ND + NSP;
  T A2 = T(0);
  for (int d = 0; d < ND; ++d) A2 += S[d] * S[d];
  const T A = sqrt(A2), iA = T(1) / A;
  T n[ND];
  for (int d = 0; d < ND; ++d) n[d] = S[d] * iA;
  T FL[NV], FR[NV], qL, qR;
  normal_flux<ND, NSP>(WL, n, FL, qL);
  normal_flux<ND, NSP>(WR, n, FR, qR);
  const T rL = WL[0], rR = WR[0], pL = WL[NV], pR = WR[NV];
  const T irL = T(1) / rL, irR = T(1) / rR;
  const T sL = sqrt(rL), sR = sqrt(rR), iw = T(1) / (sL + sR);
  const T wl = sL * iw, wr = sR * iw;
  T u[ND], uu = T(0), q = T(0);
  for (int d = 0; d < ND; ++d) {
    u[d] = wl * WL[1 + d] * irL + wr * WR[1 + d] * irR;
    uu += u[d] * u[d];
    q += u[d] * n[d];
  }
  const T H = wl * (WL[1 + ND] + pL) * irL + wr * (WR[1 + ND] + pR) * irR;
  const T a = sqrt((gamma - T(1)) * (H - T(0.5) * uu));
  const T rho = sL * sR;
  const T dp = pR - pL, dq = qR - qL;
  const T ia2 = T(1) / (a * a);
  const T a1 = T(0.5) * (dp - rho * a * dq) * ia2;
  const T a5 = T(0.5) * (dp + rho * a * dq) * ia2;
  const T a2 = (rR - rL) - dp * ia2;
  T l1 = fabs(q - a), l5 = fabs(q + a);
  const T l2 = fabs(q);
  const T del = fix * a;
  if (del > T(0)) {
    if (l1 < del) l1 = T(0.5) * (l1 * l1 + del * del) / del;
    if (l5 < del) l5 = T(0.5) * (l5 * l5 + del * del) / del;
  }
  const T w1 = l1 * a1, w2 = l2 * a2, w5 = l5 * a5;
  T Dv[NV];
  Dv[0] = w1 + w2 + w5;
  T udut = T(0);
  for (int d = 0; d < ND; ++d) {
    const T dut = (WR[1 + d] * irR - WL[1 + d] * irL) - dq * n[d];
    udut += u[d] * dut;
    Dv[1 + d] = w1 * (u[d] - a * n[d]) + w2 * u[d] + w5 * (u[d] + a * n[d]) + l2 * rho * dut;
  }
  Dv[1 + ND] = w1 * (H - q * a) + w2 * T(0.5) * uu + w5 * (H + q * a) + l2 * rho * udut;
  for (int k = 0; k < NSP; ++k) {
    const T YL = WL[2 + ND + k] * irL, YR = WR[2 + ND + k] * irR;
    Dv[2 + ND + k] = (w1 + w2 + w5) * (wl * YL + wr * YR) + l2 * rho * (YR - YL);
  }
  for (int v = 0; v < NV; ++v) F[v] = A * (T(0.5) * (FL[v] + FR[v]) - T(0.5) * Dv[v]);
}

// MUSCL-Hancock half step of one node's reconstructed gas variables
// w = (rho, m = rho u, rho E, rho Y, p), staged as rows of stride ld with
// gradient rows g[(v*ND + d)*ld]: writes h * dw/dt per row to out, where
// the rate comes from the quasi-linear Euler equations with the node's own
// state and gradients.  With du_k/dx_d = (dm_k/dx_d - u_k drho/dx_d)/rho,
//   rho: -div m            m_k: -(u.grad m_k + m_k div u) - dp/dx_k
//   rho E: -(u.grad(rho E + p) + (rho E + p) div u)
//   rho Y: -(u.grad(rho Y) + rho Y div u)     p: -(u.grad p + gamma p div u)
template <int ND, int NSP, typename T>
__device__ inline void hancock_half_step(const T* w, const T* g, int ld, int q, T gamma, T h, T* out) {
  constexpr int NVAR = 2 + ND + NSP, NR = NVAR + 1;
  const T rho = w[q], rinv = T(1) / rho;
  T u[ND], divu = T(0);
#pragma unroll
  for (int d = 0; d < ND; ++d) u[d] = w[(1 + d) * ld + q] * rinv;
#pragma unroll
  for (int d = 0; d < ND; ++d) divu += (g[((1 + d) * ND + d) * ld + q] - u[d] * g[d * ld + q]) * rinv;
  auto adv = [&](int v) {
    T a = T(0);
#pragma unroll
    for (int d = 0; d < ND; ++d) a += u[d] * g[(v * ND + d) * ld + q];
    return a;
  };
  const T p = w[(NR - 1) * ld + q], rhoE = w[(1 + ND) * ld + q], ap = adv(NR - 1);
  T dm = T(0);
#pragma unroll
  for (int d = 0; d < ND; ++d) dm += g[((1 + d) * ND + d) * ld + q];
  out[q] = -h * dm;
#pragma unroll
  for (int k = 0; k < ND; ++k)
    out[(1 + k) * ld + q] = -h * (adv(1 + k) + w[(1 + k) * ld + q] * divu + g[((NR - 1) * ND + k) * ld + q]);
  out[(1 + ND) * ld + q] = -h * (adv(1 + ND) + ap + (rhoE + p) * divu);
#pragma unroll
  for (int s = 0; s < NSP; ++s)
    out[(2 + ND + s) * ld + q] = -h * (adv(2 + ND + s) + w[(2 + ND + s) * ld + q] * divu);
  out[(NR - 1) * ld + q] = -h * (ap + gamma * p * divu);
}

// ---------------------------------------------------------------------------
// multi-species mixture (species data supplied by the caller)
// ---------------------------------------------------------------------------

struct MixParams {
  double W[16], a[16], b[16], c[16], Sc[16];
  double mu_ref, T_ref, Pr;
};

constexpr double kRgas = 8.314462618;
constexpr double kT0 = 298.15;
constexpr int kNewtonIters = 10;

// Sensible energy e_s(T) = sum_k Y_k (h_s,k(T) - R_k T) and c_v(T), with
// h_s,k = R_k (T - T0)(a + b (T + T0)/2000 + c (T^2 + T T0 + T0^2)/3e6),
// the integral of c_p,k = R_k (a + b T/1000 + c (T/1000)^2) from T0.
template <int NSP>
__device__ inline void mix_es_cv(const MixParams& mp, const double* Y, double T, double& es, double& cv) {
  const double dT = T - kT0, sT = T + kT0, qT = T * T + T * kT0 + kT0 * kT0, t = T * 1e-3;
  es = 0.0;
  cv = 0.0;
#pragma unroll
  for (int k = 0; k < NSP; ++k) {
    const double Rk = kRgas / mp.W[k];
    const double hs = Rk * dT * (mp.a[k] + mp.b[k] * sT * (1.0 / 2000.0) + mp.c[k] * qT * (1.0 / 3.0e6));
    es += Y[k] * (hs - Rk * T);
    cv += Y[k] * Rk * (mp.a[k] - 1.0 + t * (mp.b[k] + mp.c[k] * t));
  }
}

// Node state of the multi-species model from the conserved vector u[NVAR]:
// pressure, primitive fields prim = (velocity, T, Y) and aux = (gamma, mu,
// lambda, D_k, h_s,k).  The temperature solves e_s(T) = E - |u|^2/2 by a
// fixed number of Newton steps from 1000 K.  Returns false for a
// non-physical state.
template <int ND, int NSP>
__device__ inline bool ns_node_state(const MixParams& mp, const double* u, double& p, double* prim,
                                     double* aux) {
  const double rho = u[0], ir = 1.0 / rho;
  double ke = 0.0;
#pragma unroll
  for (int d = 0; d < ND; ++d) {
    prim[d] = u[1 + d] * ir;
    ke += prim[d] * prim[d];
  }
  double Y[NSP];
#pragma unroll
  for (int k = 0; k < NSP; ++k) Y[k] = u[2 + ND + k] * ir;
  const double es_target = u[1 + ND] * ir - 0.5 * ke;
  double T = 1000.0;
  for (int it = 0; it < kNewtonIters; ++it) {
    double es, cv;
    mix_es_cv<NSP>(mp, Y, T, es, cv);
    T -= (es - es_target) / cv;
  }
  double r = 0.0, cp = 0.0;
  const double t = T * 1e-3;
#pragma unroll
  for (int k = 0; k < NSP; ++k) {
    const double Rk = kRgas / mp.W[k];
    r += Y[k] * Rk;
    cp += Y[k] * Rk * (mp.a[k] + t * (mp.b[k] + mp.c[k] * t));
  }
  p = rho * r * T;
  prim[ND] = T;
#pragma unroll
  for (int k = 0; k < NSP; ++k) prim[ND + 1 + k] = Y[k];
  const double mu = mp.mu_ref * pow(T / mp.T_ref, 0.7);
  aux[0] = cp / (cp - r);
  aux[1] = mu;
  aux[2] = mu * cp / mp.Pr;
  const double dT = T - kT0, sT = T + kT0, qT = T * T + T * kT0 + kT0 * kT0;
#pragma unroll
  for (int k = 0; k < NSP; ++k) {
    aux[3 + k] = mu / (rho * mp.Sc[k]);
    aux[3 + NSP + k] = kRgas / mp.W[k] * dT *
                       (mp.a[k] + mp.b[k] * sT * (1.0 / 2000.0) + mp.c[k] * qT * (1.0 / 3.0e6));
  }
  return rho > 0.0 && T > 0.0 && isfinite(T) && isfinite(p);
}

// Face averages of the diffusive flux's node data: h (x_i + x_j) with h = 1/2.
template <int ND, int NSP, typename T>
struct ViscousFace {
  static constexpr int NP = ND + 1 + NSP;
  T rho, mu, lam;
  T p[NP];             // primitives (u, T, Y)
  T D[NSP], hs[NSP];   // species diffusivities and sensible enthalpies
  T g[NP * ND];        // gradients of the primitives, component q * ND + d
};

// Central diffusive flux through S of the multi-species Navier-Stokes
// equations from face averages of the two nodes: Newtonian stress with
// Stokes' hypothesis, Fourier heat flux plus species enthalpy transport, Fick
// species fluxes with the correction velocity V_c = sum_k D_k grad Y_k.
// Linear in S.  Writes Fv = (0, tau S, u.(tau S) - q.S, -J_k.S), to be
// subtracted from the convective flux.  hoop: on axisymmetric (x, r) meshes
// the face value of u_r / r, the cylindrical third term of div u.
template <int ND, int NSP, typename T>
__device__ inline void viscous_flux_face(const ViscousFace<ND, NSP, T>& a, const T* S, T* Fv, T hoop = T(0)) {
  T div = T(0);
#pragma unroll
  for (int d = 0; d < ND; ++d) div += a.g[d * ND + d];
  div += hoop;
  T utS = T(0);
#pragma unroll
  for (int i = 0; i < ND; ++i) {
    T ts = T(0);
#pragma unroll
    for (int j = 0; j < ND; ++j) ts += (a.g[i * ND + j] + a.g[j * ND + i]) * S[j];
    ts = a.mu * (ts - T(2.0 / 3.0) * div * S[i]);
    Fv[1 + i] = ts;
    utS += a.p[i] * ts;
  }
  T Vc[ND];
#pragma unroll
  for (int d = 0; d < ND; ++d) Vc[d] = T(0);
#pragma unroll
  for (int k = 0; k < NSP; ++k)
#pragma unroll
    for (int d = 0; d < ND; ++d) Vc[d] += a.D[k] * a.g[(ND + 1 + k) * ND + d];
  T VcS = T(0), gTS = T(0);
#pragma unroll
  for (int d = 0; d < ND; ++d) {
    VcS += Vc[d] * S[d];
    gTS += a.g[ND * ND + d] * S[d];
  }
  T qS = -a.lam * gTS;
#pragma unroll
  for (int k = 0; k < NSP; ++k) {
    T gYS = T(0);
#pragma unroll
    for (int d = 0; d < ND; ++d) gYS += a.g[(ND + 1 + k) * ND + d] * S[d];
    const T JS = -a.rho * (a.D[k] * gYS - a.p[ND + 1 + k] * VcS);
    qS += a.hs[k] * JS;
    Fv[2 + ND + k] = -JS;
  }
  Fv[0] = T(0);
  Fv[1 + ND] = utS - qS;
}

}  // namespace vcx
