// HIP kernels of the vertex-centred residual (gfx950, wave64).
//
// Data layout in HBM (internal space-filling-curve order, structure of arrays):
//   W   [nr][nn]       reconstructed variables (gas: conserved + pressure;
//                      drift-diffusion: densities)
//   G   [nr*nd][nn]    nodal gradients, component v*nd + d
//   PG  [nr*nd][P]     gradient partial sums, one per (tile, node) slot
//   PR  [nvar][P]      residual partial sums per slot
// Per step: dt -> K x (gradient tile pass, gradient gather, flux tile pass,
// gather + closure + RK stage update).  No floating-point atomics: every sum
// is taken in a fixed order (cells of a tile in curve order, then slots of a
// node in tile order), so results are bitwise reproducible.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "vcx_device.h"

namespace vcx {

constexpr int NXCD = 8;  // MI355X: 8 accelerator complex dies, round-robin dispatch

struct DevMesh {
  int nd, nv, nn, nc, ntiles, nslots, nb;
  int max_tile_cells, max_tile_nodes;
  double period[3];
  const double* x;          // [nd][nn]
  const int32_t* cell;      // [nv][nc]
  const uint32_t* shift;    // [nc]
  const uint16_t* lconn;    // [nv][nc]
  const int32_t* tile_cell; // [T+1]
  const int32_t* tile_slot; // [T+1]
  const int32_t* slot_node; // [P]
  const int32_t* slot_inc;  // [P+1]
  const uint16_t* inc;      // [nc*nv]
  const int32_t* node_slot; // [nn+1]
  const int32_t* slots_of;  // [P]
  const double* inv_vol;    // [nn]
  const double* vnode;      // [nn]
  const int32_t* bnd_index; // [nn] -1 or index into bnd_S
  const double* bnd_S;      // [nd][nb]
  const int32_t* perm;      // [nn] internal -> caller
};

// Per-solve device scalars of the time loop.
struct DevScalars {
  double t;             // committed time
  double dt;            // time step of the running step
  double t_end;         // <= 0: none
  double last_dt;
  double dt_query;
  unsigned long long dtmin;  // running minimum (bit pattern of a positive double)
  unsigned int counter;      // blocks of the dt kernel that finished
  int flag;                  // 1 unstable state, 2 invalid time step
  int bad;                   // some cell produced an invalid time step
  int active;                // the running step does work
  int pending;               // a started step awaits its commit
  long long steps;           // committed steps
};

struct Sched {
  double alpha;   // stage coefficient
  int final_stage;
  int residual_only;
};

// ---------------------------------------------------------------------------
// helpers
// ---------------------------------------------------------------------------

// Blocks are dispatched round-robin over the XCDs; give each XCD a contiguous
// range of tiles so neighbouring tiles share node data in the same L2.
__device__ inline int xcd_tile(int ntiles) {
  const int per = (ntiles + NXCD - 1) / NXCD;
  const int b = blockIdx.x;
  return (b % NXCD) * per + b / NXCD;
}

inline int xcd_grid(int ntiles) { return ((ntiles + NXCD - 1) / NXCD) * NXCD; }

__device__ inline bool step_inactive(const DevScalars* sc) {
  return sc != nullptr && sc->active == 0;
}

template <int ND>
__device__ inline void cell_rel_coords(const DevMesh& m, const double* sX, int maxn, const int (&l)[ND + 1],
                                       uint32_t code, double (&e)[ND][ND]) {
  for (int k = 1; k <= ND; ++k)
    for (int d = 0; d < ND; ++d) {
      const uint32_t b = (code >> (2 * ((k - 1) * ND + d))) & 3u;
      const double s = b == 1u ? m.period[d] : (b == 2u ? -m.period[d] : 0.0);
      e[k - 1][d] = sX[d * maxn + l[k]] + s - sX[d * maxn + l[0]];
    }
}

// ---------------------------------------------------------------------------
// gradient: per cell  g_tau = sum_k W_k S_k ; per node  G_i = -1/(nd nv V_i) sum g_tau
// ---------------------------------------------------------------------------

template <int ND, int NR>
__global__ void __launch_bounds__(256) k_grad_tile(DevMesh m, const double* __restrict__ W,
                                                   double* __restrict__ PG, const DevScalars* sc) {
  constexpr int NV = ND + 1, NC = NR * ND;
  if (step_inactive(sc)) return;
  const int t = xcd_tile(m.ntiles);
  if (t >= m.ntiles) return;
  extern __shared__ double lds[];
  const int maxn = m.max_tile_nodes, maxc = m.max_tile_cells;
  double* sW = lds;                 // [NR][maxn]
  double* sX = sW + NR * maxn;      // [ND][maxn]
  double* sC = sX + ND * maxn;      // [NC][maxc]
  const int c0 = m.tile_cell[t], nc = m.tile_cell[t + 1] - c0;
  const int s0 = m.tile_slot[t], ns = m.tile_slot[t + 1] - s0;
  for (int q = threadIdx.x; q < ns; q += blockDim.x) {
    const int g = m.slot_node[s0 + q];
#pragma unroll
    for (int v = 0; v < NR; ++v) sW[v * maxn + q] = W[(size_t)v * m.nn + g];
#pragma unroll
    for (int d = 0; d < ND; ++d) sX[d * maxn + q] = m.x[(size_t)d * m.nn + g];
  }
  __syncthreads();
  for (int lc = threadIdx.x; lc < nc; lc += blockDim.x) {
    const int c = c0 + lc;
    int l[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) l[k] = m.lconn[(size_t)k * m.nc + c];
    double e[ND][ND], S[NV][ND];
    cell_rel_coords<ND>(m, sX, maxn, l, m.shift[c], e);
    simplex_normals<ND>(e, S);
#pragma unroll
    for (int v = 0; v < NR; ++v) {
      double acc[ND];
#pragma unroll
      for (int d = 0; d < ND; ++d) acc[d] = 0.0;
#pragma unroll
      for (int k = 0; k < NV; ++k) {
        const double w = sW[v * maxn + l[k]];
#pragma unroll
        for (int d = 0; d < ND; ++d) acc[d] += w * S[k][d];
      }
#pragma unroll
      for (int d = 0; d < ND; ++d) sC[(v * ND + d) * maxc + lc] = acc[d];
    }
  }
  __syncthreads();
  for (int q = threadIdx.x; q < ns; q += blockDim.x) {
    double acc[NC];
#pragma unroll
    for (int j = 0; j < NC; ++j) acc[j] = 0.0;
    const int p0 = m.slot_inc[s0 + q], p1 = m.slot_inc[s0 + q + 1];
    for (int p = p0; p < p1; ++p) {
      const int lc = m.inc[p] >> 2;
#pragma unroll
      for (int j = 0; j < NC; ++j) acc[j] += sC[j * maxc + lc];
    }
#pragma unroll
    for (int j = 0; j < NC; ++j) PG[(size_t)j * m.nslots + s0 + q] = acc[j];
  }
}

template <int ND, int NR>
__global__ void __launch_bounds__(256) k_grad_gather(DevMesh m, const double* __restrict__ PG,
                                                     double* __restrict__ G, const DevScalars* sc) {
  constexpr int NC = NR * ND;
  if (step_inactive(sc)) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m.nn) return;
  const int a = m.node_slot[i], b = m.node_slot[i + 1];
  const double coef = -m.inv_vol[i] / double(ND * (ND + 1));
#pragma unroll
  for (int j = 0; j < NC; ++j) {
    double s = 0.0;
    for (int p = a; p < b; ++p) s += PG[(size_t)j * m.nslots + m.slots_of[p]];
    G[(size_t)j * m.nn + i] = coef * s;
  }
}

// ---------------------------------------------------------------------------
// gas flux pass
// ---------------------------------------------------------------------------

struct GasParams {
  double gamma, beta, entropy_fix;
  int limiter;
};

template <int ND, int NSP, int FLUX, typename CT>
__global__ void __launch_bounds__(256) k_flux_gas(DevMesh m, const double* __restrict__ W,
                                                  const double* __restrict__ G,
                                                  double* __restrict__ PR, GasParams gp,
                                                  const DevScalars* sc) {
  constexpr int NV = ND + 1, NVAR = 2 + ND + NSP, NR = NVAR + 1, NE = Edges<ND>::NE;
  if (step_inactive(sc)) return;
  const int t = xcd_tile(m.ntiles);
  if (t >= m.ntiles) return;
  extern __shared__ double lds[];
  const int maxn = m.max_tile_nodes, maxc = m.max_tile_cells;
  double* sX = lds;                       // [ND][maxn]
  double* sR = sX + ND * maxn;            // [NV*NVAR][maxc]
  CT* sW = reinterpret_cast<CT*>(sR + NV * NVAR * maxc);  // [NR][maxn]
  CT* sG = sW + NR * maxn;                // [NR*ND][maxn]
  const int c0 = m.tile_cell[t], nc = m.tile_cell[t + 1] - c0;
  const int s0 = m.tile_slot[t], ns = m.tile_slot[t + 1] - s0;
  for (int q = threadIdx.x; q < ns; q += blockDim.x) {
    const int g = m.slot_node[s0 + q];
#pragma unroll
    for (int v = 0; v < NR; ++v) sW[v * maxn + q] = CT(W[(size_t)v * m.nn + g]);
#pragma unroll
    for (int j = 0; j < NR * ND; ++j) sG[j * maxn + q] = CT(G[(size_t)j * m.nn + g]);
#pragma unroll
    for (int d = 0; d < ND; ++d) sX[d * maxn + q] = m.x[(size_t)d * m.nn + g];
  }
  __syncthreads();
  const CT gamma = CT(gp.gamma), beta = CT(gp.beta), fix = CT(gp.entropy_fix);
  for (int lc = threadIdx.x; lc < nc; lc += blockDim.x) {
    const int c = c0 + lc;
    int l[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) l[k] = m.lconn[(size_t)k * m.nc + c];
    double e[ND][ND], Sd[NV][ND];
    cell_rel_coords<ND>(m, sX, maxn, l, m.shift[c], e);
    simplex_normals<ND>(e, Sd);
    double acc[NV][NVAR];
#pragma unroll
    for (int k = 0; k < NV; ++k)
#pragma unroll
      for (int v = 0; v < NVAR; ++v) acc[k][v] = 0.0;
#pragma unroll
    for (int ed = 0; ed < NE; ++ed) {
      const int a = Edges<ND>::a(ed), b = Edges<ND>::b(ed);
      const int la = l[a], lb = l[b];
      CT S[ND], dx[ND];
#pragma unroll
      for (int d = 0; d < ND; ++d) {
        S[d] = CT((Sd[a][d] - Sd[b][d]) * (1.0 / double(ND * NV)));
        dx[d] = CT((a == 0 ? 0.0 : -e[a - 1][d]) + e[b - 1][d]);
      }
      CT WL[NR], WR[NR];
#pragma unroll
      for (int v = 0; v < NR; ++v) {
        const CT wi = sW[v * maxn + la], wj = sW[v * maxn + lb];
        CT gi = CT(0), gj = CT(0);
#pragma unroll
        for (int d = 0; d < ND; ++d) {
          gi += sG[(v * ND + d) * maxn + la] * dx[d];
          gj += sG[(v * ND + d) * maxn + lb] * dx[d];
        }
        const CT delta = wj - wi;
        // virtual upwind nodes l (behind i) and k (ahead of j)
        const CT dli = CT(2) * gi - delta, djk = CT(2) * gj - delta;
        WL[v] = wi + CT(0.5) * slope_limit<CT>(gp.limiter, beta, dli, delta);
        WR[v] = wj - CT(0.5) * slope_limit<CT>(gp.limiter, beta, delta, djk);
      }
      CT F[NVAR];
      if constexpr (FLUX == 0)
        hllc_flux<ND, NSP, CT>(WL, WR, S, gamma, F);
      else
        roe_flux<ND, NSP, CT>(WL, WR, S, gamma, fix, F);
#pragma unroll
      for (int v = 0; v < NVAR; ++v) {
        acc[a][v] += double(F[v]);
        acc[b][v] -= double(F[v]);
      }
    }
#pragma unroll
    for (int k = 0; k < NV; ++k)
#pragma unroll
      for (int v = 0; v < NVAR; ++v) sR[(k * NVAR + v) * maxc + lc] = acc[k][v];
  }
  __syncthreads();
  for (int q = threadIdx.x; q < ns; q += blockDim.x) {
    double acc[NVAR];
#pragma unroll
    for (int v = 0; v < NVAR; ++v) acc[v] = 0.0;
    const int p0 = m.slot_inc[s0 + q], p1 = m.slot_inc[s0 + q + 1];
    for (int p = p0; p < p1; ++p) {
      const int code = m.inc[p];
      const int lc = code >> 2, k = code & 3;
#pragma unroll
      for (int v = 0; v < NVAR; ++v) acc[v] += sR[(k * NVAR + v) * maxc + lc];
    }
#pragma unroll
    for (int v = 0; v < NVAR; ++v) PR[(size_t)v * m.nslots + s0 + q] = acc[v];
  }
}

// ---------------------------------------------------------------------------
// drift-diffusion flux pass (limited Lax-Wendroff + central diffusion)
// ---------------------------------------------------------------------------

struct DDParams {
  double zmu[4];   // z * mu per species
  double D[4];
  double beta;
  double dt_host;  // used when dt_dev is null
  const double* dt_dev;
  int limiter;
};

template <int ND, int NS, typename CT>
__global__ void __launch_bounds__(256) k_flux_dd(DevMesh m, const double* __restrict__ U,
                                                 const double* __restrict__ G,
                                                 const double* __restrict__ E,
                                                 double* __restrict__ PR, DDParams pp,
                                                 const DevScalars* sc) {
  constexpr int NV = ND + 1, NE = Edges<ND>::NE;
  if (step_inactive(sc)) return;
  const int t = xcd_tile(m.ntiles);
  if (t >= m.ntiles) return;
  extern __shared__ double lds[];
  const int maxn = m.max_tile_nodes, maxc = m.max_tile_cells;
  double* sX = lds;                      // [ND][maxn]
  double* sR = sX + ND * maxn;           // [NV*NS][maxc]
  CT* sU = reinterpret_cast<CT*>(sR + NV * NS * maxc);  // [NS][maxn]
  CT* sG = sU + NS * maxn;               // [NS*ND][maxn]
  CT* sE = sG + NS * ND * maxn;          // [ND][maxn]
  const int c0 = m.tile_cell[t], nc = m.tile_cell[t + 1] - c0;
  const int s0 = m.tile_slot[t], ns = m.tile_slot[t + 1] - s0;
  for (int q = threadIdx.x; q < ns; q += blockDim.x) {
    const int g = m.slot_node[s0 + q];
#pragma unroll
    for (int s = 0; s < NS; ++s) sU[s * maxn + q] = CT(U[(size_t)s * m.nn + g]);
#pragma unroll
    for (int j = 0; j < NS * ND; ++j) sG[j * maxn + q] = CT(G[(size_t)j * m.nn + g]);
#pragma unroll
    for (int d = 0; d < ND; ++d) {
      sX[d * maxn + q] = m.x[(size_t)d * m.nn + g];
      sE[d * maxn + q] = CT(E[(size_t)d * m.nn + g]);
    }
  }
  __syncthreads();
  const CT dt = CT(pp.dt_dev ? *pp.dt_dev : pp.dt_host);
  const CT beta = CT(pp.beta);
  for (int lc = threadIdx.x; lc < nc; lc += blockDim.x) {
    const int c = c0 + lc;
    int l[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) l[k] = m.lconn[(size_t)k * m.nc + c];
    double e[ND][ND], Sd[NV][ND];
    cell_rel_coords<ND>(m, sX, maxn, l, m.shift[c], e);
    simplex_normals<ND>(e, Sd);
    double acc[NV][NS];
#pragma unroll
    for (int k = 0; k < NV; ++k)
#pragma unroll
      for (int s = 0; s < NS; ++s) acc[k][s] = 0.0;
#pragma unroll
    for (int ed = 0; ed < NE; ++ed) {
      const int a = Edges<ND>::a(ed), b = Edges<ND>::b(ed);
      const int la = l[a], lb = l[b];
      CT S[ND], dx[ND], Ebar[ND];
#pragma unroll
      for (int d = 0; d < ND; ++d) {
        S[d] = CT((Sd[a][d] - Sd[b][d]) * (1.0 / double(ND * NV)));
        dx[d] = CT((a == 0 ? 0.0 : -e[a - 1][d]) + e[b - 1][d]);
        Ebar[d] = CT(0.5) * (sE[d * maxn + la] + sE[d * maxn + lb]);
      }
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        const CT zm = CT(pp.zmu[s]);
        CT v = CT(0), gV = CT(0), gS = CT(0), gA = CT(0), gB = CT(0);
#pragma unroll
        for (int d = 0; d < ND; ++d) {
          const CT Vd = zm * Ebar[d];
          const CT ga = sG[(s * ND + d) * maxn + la], gb = sG[(s * ND + d) * maxn + lb];
          const CT gbar = CT(0.5) * (ga + gb);
          v += Vd * S[d];
          gV += gbar * Vd;
          gS += gbar * S[d];
          gA += ga * dx[d];
          gB += gb * dx[d];
        }
        const CT ua = sU[s * maxn + la], ub = sU[s * maxn + lb];
        // upwind node w, downwind node m; the virtual node upwind of w
        const bool fwd = v >= CT(0);
        const CT uw = fwd ? ua : ub;
        const CT bb = fwd ? (ub - ua) : (ua - ub);
        const CT gw = fwd ? gA : -gB;
        const CT aa = CT(2) * gw - bb;
        const CT psi = psi_limit<CT>(pp.limiter, beta, aa, bb);
        const CT uf = uw + (CT(0.5) * bb - CT(0.5) * dt * gV) * psi;
        const CT F = uf * v - CT(pp.D[s]) * gS;
        acc[a][s] += double(F);
        acc[b][s] -= double(F);
      }
    }
#pragma unroll
    for (int k = 0; k < NV; ++k)
#pragma unroll
      for (int s = 0; s < NS; ++s) sR[(k * NS + s) * maxc + lc] = acc[k][s];
  }
  __syncthreads();
  for (int q = threadIdx.x; q < ns; q += blockDim.x) {
    double acc[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) acc[s] = 0.0;
    const int p0 = m.slot_inc[s0 + q], p1 = m.slot_inc[s0 + q + 1];
    for (int p = p0; p < p1; ++p) {
      const int code = m.inc[p];
      const int lc = code >> 2, k = code & 3;
#pragma unroll
      for (int s = 0; s < NS; ++s) acc[s] += sR[(k * NS + s) * maxc + lc];
    }
#pragma unroll
    for (int s = 0; s < NS; ++s) PR[(size_t)s * m.nslots + s0 + q] = acc[s];
  }
}

// ---------------------------------------------------------------------------
// node pass: gather partials + boundary closure + RK stage update
// ---------------------------------------------------------------------------

struct UpdateArgs {
  const double* PR;     // [nvar][P]
  const double* Win;    // stage input W (closure uses it)
  const double* Un;     // U^n rows
  double* Wout;         // stage output (may alias Win)
  double* rout;         // residual output (residual_only)
  const double* G;      // gradients (drift-diffusion closure)
  const double* E;      // field (drift-diffusion closure)
  double gamma;
  double zmu[4], D[4];
  int closure;
};

template <int ND, int NSP, int MODEL>
__global__ void __launch_bounds__(256) k_update(DevMesh m, UpdateArgs ua, Sched sd, DevScalars* sc) {
  constexpr int NVAR = MODEL == 0 ? 2 + ND + NSP : NSP;
  if (step_inactive(sc)) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m.nn) return;
  double r[NVAR];
  const int a = m.node_slot[i], b = m.node_slot[i + 1];
#pragma unroll
  for (int v = 0; v < NVAR; ++v) r[v] = 0.0;
  for (int p = a; p < b; ++p) {
    const int s = m.slots_of[p];
#pragma unroll
    for (int v = 0; v < NVAR; ++v) r[v] += ua.PR[(size_t)v * m.nslots + s];
  }
  if (ua.closure && m.nb > 0) {
    const int bi = m.bnd_index[i];
    if (bi >= 0) {
      double Sb[ND];
#pragma unroll
      for (int d = 0; d < ND; ++d) Sb[d] = m.bnd_S[(size_t)d * m.nb + bi];
      if constexpr (MODEL == 0) {
        // node flux F(W_i) . S_i^b
        double Wi[NVAR + 1];
#pragma unroll
        for (int v = 0; v <= NVAR; ++v) Wi[v] = ua.Win[(size_t)v * m.nn + i];
        double q = 0.0;
#pragma unroll
        for (int d = 0; d < ND; ++d) q += Wi[1 + d] * Sb[d];
        q /= Wi[0];
        const double p = Wi[NVAR];
        r[0] += Wi[0] * q;
#pragma unroll
        for (int d = 0; d < ND; ++d) r[1 + d] += Wi[1 + d] * q + p * Sb[d];
        r[1 + ND] += (Wi[1 + ND] + p) * q;
#pragma unroll
        for (int k = 0; k < NSP; ++k) r[2 + ND + k] += Wi[2 + ND + k] * q;
      } else {
        // convective plus diffusive node flux
#pragma unroll
        for (int s = 0; s < NVAR; ++s) {
          double vb = 0.0, gb = 0.0;
#pragma unroll
          for (int d = 0; d < ND; ++d) {
            vb += ua.zmu[s] * ua.E[(size_t)d * m.nn + i] * Sb[d];
            gb += ua.G[(size_t)(s * ND + d) * m.nn + i] * Sb[d];
          }
          r[s] += ua.Win[(size_t)s * m.nn + i] * vb - ua.D[s] * gb;
        }
      }
    }
  }
  if (sd.residual_only) {
#pragma unroll
    for (int v = 0; v < NVAR; ++v) ua.rout[(size_t)v * m.nn + i] = r[v];
    return;
  }
  const double f = sd.alpha * sc->dt * m.inv_vol[i];
  double u[NVAR];
#pragma unroll
  for (int v = 0; v < NVAR; ++v) {
    u[v] = ua.Un[(size_t)v * m.nn + i] - f * r[v];
    ua.Wout[(size_t)v * m.nn + i] = u[v];
  }
  bool ok = true;
  if constexpr (MODEL == 0) {
    double ke = 0.0;
#pragma unroll
    for (int d = 0; d < ND; ++d) ke += u[1 + d] * u[1 + d];
    const double p = (ua.gamma - 1.0) * (u[1 + ND] - 0.5 * ke / u[0]);
    ua.Wout[(size_t)NVAR * m.nn + i] = p;
    ok = u[0] > 0.0 && p > 0.0;
  }
#pragma unroll
  for (int v = 0; v < NVAR; ++v) ok = ok && isfinite(u[v]);
  if (sd.final_stage && !ok) atomicOr(&sc->flag, 1);
}

// ---------------------------------------------------------------------------
// time step: per cell, wave-level then block-level min, one atomic per block,
// the last block finalises (min is order independent: deterministic)
// ---------------------------------------------------------------------------

struct DtParams {
  int model;
  double cfl, fourier, gamma;
  double vmax_coef[4];  // |z mu| per species
  double D[4];
  int nspecies;
  int query;           // 1: only store the minimum in dt_query
};

__device__ inline void dt_commit(DevScalars* sc) {
  if (sc->pending) {
    if (sc->flag == 0) {
      sc->t += sc->dt;
      sc->last_dt = sc->dt;
      sc->steps += 1;
    }
    sc->pending = 0;
  }
}

template <int ND>
__global__ void __launch_bounds__(256) k_dt(DevMesh m, const double* __restrict__ W,
                                            const double* __restrict__ E, DtParams dp,
                                            DevScalars* sc) {
  constexpr int NV = ND + 1;
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  double dtc = INFINITY;
  if (c < m.nc) {
    int v[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] = m.cell[(size_t)k * m.nc + c];
    const uint32_t code = m.shift[c];
    double e[ND][ND], S[NV][ND];
#pragma unroll
    for (int k = 1; k <= ND; ++k)
#pragma unroll
      for (int d = 0; d < ND; ++d) {
        const uint32_t b = (code >> (2 * ((k - 1) * ND + d))) & 3u;
        const double s = b == 1u ? m.period[d] : (b == 2u ? -m.period[d] : 0.0);
        e[k - 1][d] = m.x[(size_t)d * m.nn + v[k]] + s - m.x[(size_t)d * m.nn + v[0]];
      }
    const double det = simplex_normals<ND>(e, S);
    double area = 0.0;
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      double s2 = 0.0;
#pragma unroll
      for (int d = 0; d < ND; ++d) s2 += S[k][d] * S[k][d];
      area += sqrt(s2);
    }
    // inscribed diameter 2 nd V / sum |S_k|, V = det / nd!
    const double dx = 2.0 * ND * (det / (ND == 2 ? 2.0 : 6.0)) / area;
    if (dp.model == 0) {
      double lam = 0.0;
      bool phys = true;
#pragma unroll
      for (int k = 0; k < NV; ++k) {
        const double rho = W[v[k]];
        double uu = 0.0;
#pragma unroll
        for (int d = 0; d < ND; ++d) {
          const double ud = W[(size_t)(1 + d) * m.nn + v[k]] / rho;
          uu += ud * ud;
        }
        const double p = W[(size_t)(m.nd + 2 + dp.nspecies) * m.nn + v[k]];
        phys = phys && rho > 0.0 && p > 0.0;
        lam = fmax(lam, sqrt(uu) + sqrt(dp.gamma * p / rho));
      }
      dtc = dp.cfl * dx / lam;
      if (!phys || !(dtc > 0.0)) dtc = -1.0;  // non-physical state: flagged below
    } else {
      double emax = 0.0;
#pragma unroll
      for (int k = 0; k < NV; ++k) {
        double e2 = 0.0;
#pragma unroll
        for (int d = 0; d < ND; ++d) {
          const double ed = E[(size_t)d * m.nn + v[k]];
          e2 += ed * ed;
        }
        emax = fmax(emax, sqrt(e2));
      }
      for (int s = 0; s < dp.nspecies; ++s) {
        const double vmax = dp.vmax_coef[s] * emax;
        if (vmax > 0.0) dtc = fmin(dtc, dp.cfl * dx / vmax);
        if (dp.D[s] > 0.0) dtc = fmin(dtc, dp.fourier * dx * dx / dp.D[s]);
      }
    }
  }
  // wave64 minimum, then across the block's waves
  for (int off = 32; off > 0; off >>= 1) dtc = fmin(dtc, __shfl_xor(dtc, off, 64));
  __shared__ double wmin[4];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) wmin[wv] = dtc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double b = wmin[0];
    for (int q = 1; q < (int)(blockDim.x >> 6); ++q) b = fmin(b, wmin[q]);
    if (b < 0.0) atomicOr(&sc->bad, 1);
    else atomicMin(&sc->dtmin, (unsigned long long)__double_as_longlong(b));
    __threadfence();
    const unsigned int done = atomicAdd(&sc->counter, 1u);
    if (done == gridDim.x - 1) {
      __threadfence();
      double d = __longlong_as_double((long long)atomicAdd(&sc->dtmin, 0ull));
      const bool bad = atomicAdd(&sc->bad, 0) != 0;
      if (dp.query) {
        sc->dt_query = bad ? -1.0 : d;
      } else {
        dt_commit(sc);
        sc->active = 0;
        const bool done_t = sc->t_end > 0.0 && sc->t >= sc->t_end;
        // a finished or failed solve ignores the (stale) state it was given
        if (sc->flag == 0 && !done_t) {
          if (sc->t_end > 0.0 && sc->t + d > sc->t_end) d = sc->t_end - sc->t;
          if (!bad && d > 0.0 && isfinite(d)) {
            sc->dt = d;
            sc->active = 1;
            sc->pending = 1;
          } else {
            sc->flag |= 2;
          }
        }
      }
      sc->dtmin = 0x7FF0000000000000ull;  // +inf
      sc->bad = 0;
      sc->counter = 0u;
    }
  }
}

__global__ void k_commit(DevScalars* sc) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    dt_commit(sc);
    sc->active = 0;
  }
}

// ---------------------------------------------------------------------------
// permutations between the caller's node order and the internal order
// ---------------------------------------------------------------------------

__global__ void k_gather_rows(const int32_t* __restrict__ perm, const double* __restrict__ src,
                              double* __restrict__ dst, int nn, int nrows) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nn) return;
  const int o = perm[i];
  for (int v = 0; v < nrows; ++v) dst[(size_t)v * nn + i] = src[(size_t)v * nn + o];
}

__global__ void k_scatter_rows(const int32_t* __restrict__ perm, const double* __restrict__ src,
                               double* __restrict__ dst, int nn, int nrows) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nn) return;
  const int o = perm[i];
  for (int v = 0; v < nrows; ++v) dst[(size_t)v * nn + o] = src[(size_t)v * nn + i];
}

// pressure row of the gas reconstructed variables from the conserved rows
__global__ void k_pressure(double* W, int nn, int nd, int nsp, double gamma) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nn) return;
  const double rho = W[i];
  double ke = 0.0;
  for (int d = 0; d < nd; ++d) {
    const double mv = W[(size_t)(1 + d) * nn + i];
    ke += mv * mv;
  }
  W[(size_t)(2 + nd + nsp) * nn + i] = (gamma - 1.0) * (W[(size_t)(1 + nd) * nn + i] - 0.5 * ke / rho);
}

// ---------------------------------------------------------------------------
// conservation sums: fixed assignment of nodes to blocks, fixed tree
// ---------------------------------------------------------------------------

__global__ void __launch_bounds__(256) k_sums_partial(const double* __restrict__ W,
                                                      const double* __restrict__ vnode, int nn,
                                                      int nrows, double* __restrict__ part) {
  __shared__ double red[256];
  for (int v = 0; v < nrows; ++v) {
    double s = 0.0;
    for (int i = blockIdx.x * 256 + threadIdx.x; i < nn; i += gridDim.x * 256)
      s += vnode[i] * W[(size_t)v * nn + i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
      __syncthreads();
    }
    if (threadIdx.x == 0) part[(size_t)v * gridDim.x + blockIdx.x] = red[0];
    __syncthreads();
  }
}

__global__ void __launch_bounds__(256) k_sums_final(const double* __restrict__ part, int nparts,
                                                    int nrows, double* __restrict__ out) {
  __shared__ double red[256];
  for (int v = 0; v < nrows; ++v) {
    double s = 0.0;
    for (int i = threadIdx.x; i < nparts; i += 256) s += part[(size_t)v * nparts + i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
      __syncthreads();
    }
    if (threadIdx.x == 0) out[v] = red[0];
    __syncthreads();
  }
}

}  // namespace vcx
