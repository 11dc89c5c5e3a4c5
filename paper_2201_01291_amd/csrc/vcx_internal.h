// Library-internal definitions shared by the C ABI (vcx_capi.hip), the
// per-model kernel tables (vcx_tab_*.hip) and the allocation-free residual
// (vcx_static.hip): the mesh and solver handles, the launch helpers, and the
// kernel table of one (model, dimension, species, flux, precision)
// instantiation.  Each table is instantiated in exactly one translation unit.
#pragma once
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "vcx.h"
#include "vcx_batch.h"
#include "vcx_kernels.h"
#include "vcx_mesh.h"

namespace vcx {
// sets the calling thread's error message (vcx_last_error) and returns s
vcx_status fail(vcx_status s, const std::string& msg);
}  // namespace vcx

using namespace vcx;

#define VCX_HIP(expr)                                                                     \
  do {                                                                                    \
    hipError_t e_ = (expr);                                                               \
    if (e_ != hipSuccess) return vcx::fail(VCX_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

#define VCX_TRY(expr)               \
  do {                              \
    vcx_status s_ = (expr);         \
    if (s_ != VCX_OK) return s_;    \
  } while (0)

constexpr int kNodeBlock = 256;

struct vcx_mesh_s {
  HostMesh h;
  DevMesh d{};
  std::vector<void*> allocs;
  hipStream_t stream = nullptr;
  int device = 0;
  int lds_max = 65536;  // dynamic LDS bytes one workgroup may allocate on this device
};

struct KernelTable;

struct vcx_solver_s {
  vcx_mesh mesh = nullptr;
  vcx_physics ph{};
  int nd = 0, nvar = 0, nr = 0;
  int nw = 0;   // rows of a state buffer (conserved, then pressure unless drift-diffusion)
  int ngf = 0;  // fields whose nodal gradients are computed
  double* W[2] = {nullptr, nullptr};
  // multi-species: node-major copies [nn][ldws] of the first nws rows of each
  // state buffer (staged by the gradient and flux passes), kept beside W by
  // every kernel that writes a state
  double* WS[2] = {nullptr, nullptr};
  int nws = 0, ldws = 0;
  // drift-diffusion on large simplex meshes: the node-gradient pass with a
  // node-major G (no partial sums, no completion)
  bool dd_ngrad = false;
  int cur = 0;
  double* G = nullptr;
  double* PG = nullptr;
  double* PR = nullptr;
  double* E = nullptr;
  double* io = nullptr;    // [max(nr*nd, nvar)][nn] staging in caller order
  double* rbuf = nullptr;  // [max(nr*nd, nvar)][nn] internal order
  DevLoop* lp = nullptr;          // time loop (two step states by parity)
  DevScalars* sc_host = nullptr;  // pinned mirror of the current state
  int spar = 0;                   // parity of the next step
  int node_blocks = 0, nsh_blocks = 1;
  double* part = nullptr;
  double* sums_dev = nullptr;
  double* sums_host = nullptr;     // pinned
  bool has_state = false;
  int host_flag = 0;
  long long steps_total = 0;
  int64_t steps_last = 0;
  const KernelTable* kt = nullptr;
  size_t lds_grad = 0, lds_flux = 0, lds_fused = 0;
  bool fused = false;      // time loop and residual run the fused gradient + flux pass
  double* gout = nullptr;  // fused passes: node gradients for the boundary closure, or null
  double* cbuf = nullptr;  // second closure option: [nb][nvar] closure fluxes of the stage input
  int tile_block = 256;
  int flux_block = 256;  // block of the flux tile pass (multi-species: covers the tile's edges)
  size_t bytes = 0;  // device bytes held by the solver (mesh excluded)
  // profiling
  bool prof = false;
  std::map<std::string, std::vector<std::pair<hipEvent_t, hipEvent_t>>> ev;
  std::map<std::string, std::pair<int64_t, double>> acc;
  std::vector<hipEvent_t> spare;
};

// ---------------------------------------------------------------------------
// launch helper with optional event timing
// ---------------------------------------------------------------------------

// node-major staged rows of the state buffer W (multi-species), or null
inline const double* ws_of(vcx_solver s, const double* W) {
  return W == s->W[0] ? s->WS[0] : (W == s->W[1] ? s->WS[1] : nullptr);
}

inline hipEvent_t take_event(vcx_solver s) {
  if (!s->spare.empty()) {
    hipEvent_t e = s->spare.back();
    s->spare.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

template <typename F>
inline vcx_status launch_on(vcx_solver s, hipStream_t st, bool prof, const char* name, F&& f) {
  // events are taken by the dispatch itself (start and end of the kernel)
  hipEvent_t a = nullptr, b = nullptr;
  if (prof) {
    a = take_event(s);
    b = take_event(s);
    if (!a || !b) a = b = nullptr;
  }
  (void)st;
  f(a, b);
  VCX_HIP(hipGetLastError());
  if (a && b) s->ev[name].push_back({a, b});
  return VCX_OK;
}

template <typename F>
inline vcx_status launch(vcx_solver s, const char* name, F&& f) {
  return launch_on(s, s->mesh->stream, s->prof, name, std::forward<F>(f));
}

// ---------------------------------------------------------------------------
// kernel table: one instantiation per (model, nd, species, flux, precision)
// ---------------------------------------------------------------------------

struct KernelTable {
  // fp64_out: G in FP64 whatever the flux pass stages (the gradient query)
  vcx_status (*grad)(vcx_solver, const double* Win, const GradCtl& gc, bool fp64_out);
  vcx_status (*grad_complete)(vcx_solver);
  vcx_status (*flux)(vcx_solver, const double* Win, const Finish& f, double dt_host);
  vcx_status (*update_shared)(vcx_solver, const Finish& f);
  vcx_status (*node_dt)(vcx_solver, const double* W);
  size_t (*lds_grad)(int maxn, int maxc);
  size_t (*lds_flux)(const DevMesh& d, int predictor);
  size_t (*lds_fused)(const DevMesh& d);  // 0: no fused pass for this model
  vcx_status (*fused)(vcx_solver, const double* Win, const Finish& f, const FusedCtl& fc, double dt_host);
  vcx_status (*allow_lds)(size_t grad_bytes, size_t flux_bytes, size_t fused_bytes);
  vcx_status (*aux)(vcx_solver, double* W);
  vcx_status (*batch_stage)(const struct BatchRun& br, hipStream_t stream, const BatchStage& st, bool prof);
  vcx_status (*closure2)(vcx_solver, const Finish& f);
  vcx_status (*prim_to_cons)(vcx_solver, double* W);
  int nw, ngf;
};

// A batch launch: device table of solves and block maps (see vcx_solve_batch).
struct BatchRun {
  vcx_solver lead;                 // physics of the batch
  BatchEntry* tab;
  int2* tile_map;
  int ntile_blocks;
  int2* grad_map;                  // blocks of the node-gradient pass: solve, slice
  int ngrad_blocks;
  bool dd_ngrad;                   // drift-diffusion solves on the node-gradient pass
  int2* sh_map;
  int nsh_blocks;
  size_t lds_grad, lds_flux;
  int tile_block, flux_block;
  bool fused;
};


inline MixParams mix_params(const vcx_physics& ph) {
  MixParams mp{};
  for (int k = 0; k < 16; ++k) {
    mp.W[k] = ph.Wk[k] > 0.0 ? ph.Wk[k] : 1.0;
    mp.a[k] = ph.cpa[k];
    mp.b[k] = ph.cpb[k];
    mp.c[k] = ph.cpc[k];
    mp.Sc[k] = ph.Sc[k] > 0.0 ? ph.Sc[k] : 1.0;
  }
  mp.mu_ref = ph.mu_ref;
  mp.T_ref = ph.T_ref > 0.0 ? ph.T_ref : 300.0;
  mp.Pr = ph.Pr > 0.0 ? ph.Pr : 1.0;
  return mp;
}

inline DtCoef dt_coef(const vcx_physics& ph) {
  DtCoef c{};
  c.cfl = ph.cfl;
  c.fourier = ph.fourier;
  c.gamma = ph.gamma;
  for (int k = 0; k < 4 && k < ph.nspecies; ++k) {
    c.zmu[k] = ph.z[k] * ph.mu[k];
    c.D[k] = ph.D[k];
    c.ez[k] = 1.602176634e-19 * ph.z[k];  // elementary charge [C] times the charge number
    c.mu[k] = ph.mu[k];
  }
  if (ph.model == VCX_MODEL_DRIFT_DIFFUSION && ph.diel > 0.0) c.adeps = ph.diel * 8.8541878128e-12;  // eps0 [F/m]
  return c;
}

// NV: vertices per cell, ND + 1 (simplices) or 4 (2D quadrilaterals; gas
// and drift-diffusion, separate gradient and flux passes, not batched)
template <int MODEL, int ND, int NSP, int FLUX, typename CT, int NV = ND + 1>
struct Impl {
  static constexpr int NVAR = MODEL == 1 ? NSP : 2 + ND + NSP;
  static constexpr int NR = MODEL == 1 ? NVAR : NVAR + 1;
  static constexpr bool SIMPLEX = NV == ND + 1;
  static constexpr int NP = MODEL == 2 ? ND + 1 + NSP : 0;   // primitives (u, T, Y)
  static constexpr int NGF = NR + NP;                        // fields with gradients
  static constexpr int NW = NR;  // rows of a state buffer: U, then p (the multi-species
                                 // primitives and aux live in the staged rows WS)

  static size_t lds_grad(int maxn, int maxc) {
    constexpr int FG = grad_group(NGF);  // fields staged per pass
    return sizeof(double) * ((size_t)(FG + ND) * maxn + (size_t)FG * ND * maxc) + inc_lds_bytes(NV, maxc);
  }
  static size_t lds_flux(const DevMesh& d, int predictor) {
    const int maxn = d.max_tile_nodes, maxc = d.max_tile_cells;
    // the gas predictor stages one more row set: the half-step increments
    const size_t pred = MODEL == 0 && predictor ? sizeof(CT) * (size_t)NR * maxn : 0;
    if constexpr (MODEL == 0 && cell_halves<ND, CT>() == 2)  // two planes of vertex parts
      return sizeof(double) * ((size_t)ND * maxn + (size_t)2 * NV * NVAR * maxc) +
             sizeof(CT) * (size_t)(NR + NR * ND) * maxn + pred + slot_lds_bytes(maxn) + inc_lds_bytes(NV, maxc);
    if constexpr (MODEL == 1 && cell_halves<ND, CT>() == 2)
      return sizeof(double) * ((size_t)ND * maxn + (size_t)2 * NV * NVAR * maxc) +
             sizeof(CT) * (size_t)(NSP + NSP * ND + ND) * maxn + slot_lds_bytes(maxn) + inc_lds_bytes(NV, maxc);
    if constexpr (MODEL == 2) return NsEdgeLds<ND, NSP, CT>::lds_bytes(maxn, maxc, d.max_tile_edges);
    size_t dbl = sizeof(double) * ((size_t)ND * maxn + (size_t)NV * NVAR * maxc);
    size_t ct = MODEL == 0   ? (size_t)(NR + NR * ND) * maxn
                : MODEL == 1 ? (size_t)(NSP + NSP * ND + ND) * maxn
                             : (size_t)(NW + NGF * ND) * maxn;
    return dbl + sizeof(CT) * ct + pred + slot_lds_bytes(maxn) + inc_lds_bytes(NV, maxc);
  }
  static constexpr bool FUSABLE = ND == 2 && MODEL != 2 && SIMPLEX;
  static size_t lds_fused(const DevMesh& d) {
    if constexpr (FUSABLE) {
      if (!d.has_halo) return 0;
      return fused_lds_bytes<ND, NSP, MODEL, CT>(d.max_tile_nodes, d.max_tile_cells, d.max_ext_nodes,
                                                 d.max_ext_cells, d.max_tile_ginc);
    } else {
      return 0;
    }
  }
  static DDParams dd_params(const vcx_physics& ph, double dt_host) {
    DDParams pp{};
    for (int k = 0; k < NSP && k < 4; ++k) {
      pp.zmu[k] = ph.z[k] * ph.mu[k];
      pp.D[k] = ph.D[k];
    }
    pp.beta = ph.beta;
    pp.dt_host = dt_host;
    pp.limiter = ph.limiter;
    return pp;
  }
  static vcx_status fused(vcx_solver s, const double* Win, const Finish& f, const FusedCtl& fc, double dt_host) {
    if constexpr (FUSABLE) {
      const DevMesh& m = s->mesh->d;
      GasParams gp{s->ph.gamma, s->ph.beta, s->ph.entropy_fix, s->ph.limiter};
      DDParams pp = dd_params(s->ph, dt_host);
      return launch(s, "flux", [&](hipEvent_t ea, hipEvent_t eb) {
        hipExtLaunchKernelGGL((k_fused<ND, NSP, MODEL, FLUX, CT>), dim3(xcd_grid(m.ntiles)), dim3(s->tile_block),
                              s->lds_fused, s->mesh->stream, ea, eb, 0, m, Win, s->PR, gp, pp, f, fc);
      });
    } else {
      return vcx::fail(VCX_E_ARG, "no fused pass for this model");
    }
  }
  static vcx_status grad(vcx_solver s, const double* Win, const GradCtl& gc, bool fp64_out) {
    const DevMesh& m = s->mesh->d;
    const int lead = gc.lp && gc.first_stage ? 1 : 0;
    if constexpr (node_gradient(MODEL, ND, NV)) {
      // the node-gradient pass (node-major G, complete); the multi-species
      // fields from the node-major staged rows, and G in the type the
      // multi-species flux pass stages
      const double* WS = ws_of(s, Win);
      if constexpr (MODEL == 2 && !std::is_same<CT, double>::value) {
        if (!fp64_out)
          return launch(s, "gradient", [&](hipEvent_t ea, hipEvent_t eb) {
            hipExtLaunchKernelGGL((k_grad_node<ND, NGF, true, CT>), dim3(xcd_grid(m.ng_nslices) + lead),
                                  dim3(64 * kGradNodeGroups), 0, s->mesh->stream, ea, eb, 0, m, Win, WS, s->ldws,
                                  reinterpret_cast<CT*>(s->G), gc);
          });
      }
      return launch(s, "gradient", [&](hipEvent_t ea, hipEvent_t eb) {
        hipExtLaunchKernelGGL((k_grad_node<ND, NGF, MODEL == 2>), dim3(xcd_grid(m.ng_nslices) + lead),
                              dim3(64 * kGradNodeGroups), 0, s->mesh->stream, ea, eb, 0, m, Win, WS, s->ldws, s->G,
                              gc);
      });
    } else {
      if constexpr (MODEL == 1 && SIMPLEX) {
        if (s->dd_ngrad)
          return launch(s, "gradient", [&](hipEvent_t ea, hipEvent_t eb) {
            hipExtLaunchKernelGGL((k_grad_node<ND, NGF>), dim3(xcd_grid(m.ng_nslices) + lead),
                                  dim3(64 * kGradNodeGroups), 0, s->mesh->stream, ea, eb, 0, m, Win,
                                  (const double*)nullptr, 0, s->G, gc);
          });
      }
      return launch(s, "gradient", [&](hipEvent_t ea, hipEvent_t eb) {
        hipExtLaunchKernelGGL((k_grad_tile<ND, NGF, NV>), dim3(xcd_grid(m.ntiles) + lead), dim3(s->tile_block),
                              s->lds_grad, s->mesh->stream, ea, eb, 0, m, Win, s->G, s->PG, gc);
      });
    }
  }
  static vcx_status grad_complete(vcx_solver s) {
    const DevMesh& m = s->mesh->d;
    if (m.nshared == 0 || node_gradient(MODEL, ND, NV) || s->dd_ngrad) return VCX_OK;
    return launch(s, "gradient_shared", [&](hipEvent_t ea, hipEvent_t eb) {
      hipExtLaunchKernelGGL((k_grad_shared<ND, NGF>), dim3((m.nshared + kGradSharedNodes - 1) / kGradSharedNodes),
                            dim3(256), 0, s->mesh->stream, ea, eb, 0, m, (const double*)s->PG, s->G);
    });
  }
  static vcx_status aux(vcx_solver s, double* W) {
    const DevMesh& m = s->mesh->d;
    if constexpr (MODEL == 0) {
      hipLaunchKernelGGL(k_pressure, dim3((m.nn + 255) / 256), dim3(256), 0, s->mesh->stream, W, m.nn,
                         m.nd, NSP, s->ph.gamma);
    } else if constexpr (MODEL == 2) {
      hipLaunchKernelGGL((k_ns_aux<ND, NSP>), dim3((m.nn + 255) / 256), dim3(256), 0, s->mesh->stream,
                         W, m.nn, mix_params(s->ph), const_cast<double*>(ws_of(s, W)), s->nws, s->ldws,
                         std::is_same<CT, double>::value ? 0 : 1);
    }
    VCX_HIP(hipGetLastError());
    return VCX_OK;
  }
  static vcx_status flux(vcx_solver s, const double* Win, const Finish& f, double dt_host) {
    const DevMesh& m = s->mesh->d;
    hipStream_t st = s->mesh->stream;
    if constexpr (MODEL == 0) {
      GasParams gp{s->ph.gamma, s->ph.beta, s->ph.entropy_fix, s->ph.limiter, dt_host};
      // a thread per cell and half: the cells rounded to wavefronts, per half
      const int fb = cell_halves<ND, CT>() == 2 ? std::min(256, 2 * ((m.max_tile_cells + 63) / 64) * 64)
                                                : s->tile_block;
      if (s->ph.predictor)
        return launch(s, "flux", [&](hipEvent_t ea, hipEvent_t eb) {
          hipExtLaunchKernelGGL((k_flux_gas<ND, NSP, FLUX, CT, false, true, NV>), dim3(xcd_grid(m.ntiles)),
                                dim3(fb), s->lds_flux, st, ea, eb, 0, m, Win, (const double*)s->G, s->PR, gp,
                                f);
        });
      if constexpr (ND == 2) {
        if (m.axi)
          return launch(s, "flux", [&](hipEvent_t ea, hipEvent_t eb) {
            hipExtLaunchKernelGGL((k_flux_gas<ND, NSP, FLUX, CT, true, false, NV>), dim3(xcd_grid(m.ntiles)),
                               dim3(s->tile_block), s->lds_flux, st, ea, eb, 0, m, Win, (const double*)s->G,
                               s->PR, gp, f);
          });
      }
      return launch(s, "flux", [&](hipEvent_t ea, hipEvent_t eb) {
        hipExtLaunchKernelGGL((k_flux_gas<ND, NSP, FLUX, CT, false, false, NV>), dim3(xcd_grid(m.ntiles)),
                           dim3(fb), s->lds_flux, st, ea, eb, 0, m, Win, (const double*)s->G,
                           s->PR, gp, f);
      });
    } else if constexpr (MODEL == 2) {
      GasParams gp{s->ph.gamma, s->ph.beta, s->ph.entropy_fix, s->ph.limiter};
      // (the node-gradient pass has left G complete and node-major; the
      // state rows are staged from their node-major copy)
      const double* WS = ws_of(s, Win);
      if constexpr (ND == 2) {
        if (m.axi)
          return launch(s, "flux", [&](hipEvent_t ea, hipEvent_t eb) {
            hipExtLaunchKernelGGL((k_flux_ns<ND, NSP, CT, true>), dim3(xcd_grid(m.ntiles)), dim3(s->flux_block),
                                  s->lds_flux, st, ea, eb, 0, m, WS, (const double*)s->G, s->PR, gp, f);
          });
      }
      return launch(s, "flux", [&](hipEvent_t ea, hipEvent_t eb) {
        hipExtLaunchKernelGGL((k_flux_ns<ND, NSP, CT>), dim3(xcd_grid(m.ntiles)), dim3(s->flux_block),
                           s->lds_flux, st, ea, eb, 0, m, WS, (const double*)s->G, s->PR, gp, f);
      });
    } else {
      DDParams pp{};
      for (int k = 0; k < NSP; ++k) {
        pp.zmu[k] = s->ph.z[k] * s->ph.mu[k];
        pp.D[k] = s->ph.D[k];
      }
      pp.beta = s->ph.beta;
      pp.dt_host = dt_host;
      pp.limiter = s->ph.limiter;
      const bool sg = s->ph.flux == VCX_FLUX_SG;
      VCX_TRY(grad_complete(s));
      Finish fg = f;
      fg.gfull = 1;
      if constexpr (ND == 2) {
        if (m.axi)
          return launch(s, "flux", [&](hipEvent_t ea, hipEvent_t eb) {
            if (sg)
              hipExtLaunchKernelGGL((k_flux_dd<ND, NSP, CT, true, true, NV>), dim3(xcd_grid(m.ntiles)),
                                    dim3(s->tile_block), s->lds_flux, st, ea, eb, 0, m, Win,
                                    (const double*)s->G, s->PR, pp, fg);
            else
              hipExtLaunchKernelGGL((k_flux_dd<ND, NSP, CT, true, false, NV>), dim3(xcd_grid(m.ntiles)),
                                    dim3(s->tile_block), s->lds_flux, st, ea, eb, 0, m, Win,
                                    (const double*)s->G, s->PR, pp, fg);
          });
      }
      const int fb = cell_halves<ND, CT>() == 2 ? std::min(256, 2 * ((m.max_tile_cells + 63) / 64) * 64)
                                                : s->tile_block;
      return launch(s, "flux", [&](hipEvent_t ea, hipEvent_t eb) {
        if (sg)
          hipExtLaunchKernelGGL((k_flux_dd<ND, NSP, CT, false, true, NV>), dim3(xcd_grid(m.ntiles)), dim3(fb),
                                s->lds_flux, st, ea, eb, 0, m, Win, (const double*)s->G, s->PR, pp, fg);
        else
          hipExtLaunchKernelGGL((k_flux_dd<ND, NSP, CT, false, false, NV>), dim3(xcd_grid(m.ntiles)), dim3(fb), s->lds_flux,
                                st, ea, eb, 0, m, Win, (const double*)s->G, s->PR, pp, fg);
      });
    }
  }
  static vcx_status update_shared(vcx_solver s, const Finish& f) {
    const DevMesh& m = s->mesh->d;
    Finish g = f;
    g.WSin = ws_of(s, f.Win);  // the stage input's staged rows (multi-species)
    if (MODEL == 2 && (!g.WSin || (!g.residual_only && !g.WSout)))
      return fail(VCX_E_STATE, "multi-species update without its staged rows");
    return launch(s, "update", [&](hipEvent_t ea, hipEvent_t eb) {
      hipExtLaunchKernelGGL((k_update_shared<ND, NSP, MODEL>), dim3(s->nsh_blocks), dim3(kNodeBlock), 0,
                         s->mesh->stream, ea, eb, 0, m, (const double*)s->PR, g);
    });
  }
  static vcx_status node_dt(vcx_solver s, const double* W) {
    const DevMesh& m = s->mesh->d;
    DtCoef dc = dt_coef(s->ph);
    MixParams mp = mix_params(s->ph);
    hipLaunchKernelGGL(k_node_slots_clear, dim3(1), dim3(kCandSlots), 0, s->mesh->stream, s->lp);
    VCX_HIP(hipGetLastError());
    return launch(s, "node_dt", [&](hipEvent_t ea, hipEvent_t eb) {
      hipExtLaunchKernelGGL((k_node_dt<ND, NSP, MODEL>), dim3(s->node_blocks), dim3(kNodeBlock), 0,
                         s->mesh->stream, ea, eb, 0, m, W, (const double*)s->E, dc, mp, s->lp);
    });
  }
  // Allow dynamic LDS above the 64 KiB default for the two tile kernels.
  static vcx_status allow_lds(size_t grad_bytes, size_t flux_bytes, size_t fused_bytes) {
    if constexpr (FUSABLE) {
      if (fused_bytes > 0) {
        VCX_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_fused<ND, NSP, MODEL, FLUX, CT>),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)fused_bytes));
        VCX_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_fused_batch<ND, NSP, MODEL, FLUX, CT>),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)fused_bytes));
      }
    }
    VCX_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_grad_tile<ND, NGF, NV>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)grad_bytes));
    if constexpr (MODEL == 0) {
      VCX_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_flux_gas<ND, NSP, FLUX, CT, false, false, NV>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)flux_bytes));
      VCX_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_flux_gas<ND, NSP, FLUX, CT, false, true, NV>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)flux_bytes));
      if constexpr (ND == 2)
        VCX_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_flux_gas<ND, NSP, FLUX, CT, true, false, NV>),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)flux_bytes));
    } else if constexpr (MODEL == 2) {
      VCX_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_flux_ns<ND, NSP, CT>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)flux_bytes));
      if constexpr (ND == 2)
        VCX_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_flux_ns<ND, NSP, CT, true>),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)flux_bytes));
    } else {
      VCX_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_flux_dd<ND, NSP, CT, false, false, NV>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)flux_bytes));
      VCX_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_flux_dd<ND, NSP, CT, false, true, NV>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)flux_bytes));
      if constexpr (ND == 2) {
        VCX_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_flux_dd<ND, NSP, CT, true, false, NV>),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)flux_bytes));
        VCX_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_flux_dd<ND, NSP, CT, true, true, NV>),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)flux_bytes));
      }
    }
    if constexpr (SIMPLEX) {  // (quadrilaterals have no batch kernels)
      VCX_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_grad_tile_batch<ND, NGF>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)grad_bytes));
      if constexpr (MODEL == 0)
        VCX_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_flux_gas_batch<ND, NSP, FLUX, CT>),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)flux_bytes));
      else if constexpr (MODEL == 2)
        VCX_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_flux_ns_batch<ND, NSP, CT>),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)flux_bytes));
      else
        VCX_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_flux_dd_batch<ND, NSP, CT>),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)flux_bytes));
    }
    return VCX_OK;
  }
  // one RK stage of every solve of a batch: gradient, flux, shared-node update
  static vcx_status batch_stage(const BatchRun& br, hipStream_t stream, const BatchStage& st, bool prof) {
    if constexpr (!SIMPLEX) {
      return vcx::fail(VCX_E_ARG, "solvers on quadrilateral meshes are not batched");
    } else {
      return batch_stage_simplex(br, stream, st, prof);
    }
  }
  static vcx_status batch_stage_simplex(const BatchRun& br, hipStream_t stream, const BatchStage& st, bool prof) {
    vcx_solver s = br.lead;
    // the node-gradient passes (multi-species; drift-diffusion on large
    // meshes) leave G complete, as in the single solve
    FinishShared fs{dt_coef(s->ph), mix_params(s->ph), s->ph.closure, br.fused ? 1 : 0,
                    MODEL == 2 || br.dd_ngrad ? 1 : 0, br.dd_ngrad ? 1 : 0};
    if constexpr (FUSABLE) {
      if (br.fused) {
        GasParams gp{s->ph.gamma, s->ph.beta, s->ph.entropy_fix, s->ph.limiter};
        DDParams pp = dd_params(s->ph, 0.0);
        VCX_TRY(launch_on(s, stream, prof, "flux", [&](hipEvent_t ea, hipEvent_t eb) {
          hipExtLaunchKernelGGL((k_fused_batch<ND, NSP, MODEL, FLUX, CT>), dim3(xcd_grid(br.ntile_blocks)),
                                dim3(br.tile_block), br.lds_flux, stream, ea, eb, 0, (const BatchEntry*)br.tab,
                                (const int2*)br.tile_map, br.ntile_blocks, st, gp, pp, fs);
        }));
        return launch_on(s, stream, prof, "update", [&](hipEvent_t ea, hipEvent_t eb) {
          hipExtLaunchKernelGGL((k_update_shared_batch<ND, NSP, MODEL>), dim3(br.nsh_blocks), dim3(kNodeBlock),
                                0, stream, ea, eb, 0, (const BatchEntry*)br.tab, (const int2*)br.sh_map, st, fs);
        });
      }
    }
    if constexpr (node_gradient(MODEL, ND, NV)) {
      VCX_TRY(launch_on(s, stream, prof, "gradient", [&](hipEvent_t ea, hipEvent_t eb) {
        hipExtLaunchKernelGGL((k_grad_node_batch<ND, NGF, MODEL == 2, typename std::conditional<MODEL == 2, CT, double>::type>),
                              dim3(xcd_grid(br.ngrad_blocks)),
                              dim3(64 * kGradNodeGroups), 0,
                              stream, ea, eb, 0, (const BatchEntry*)br.tab, (const int2*)br.grad_map,
                              br.ngrad_blocks, st);
      }));
    } else if (MODEL == 1 && br.dd_ngrad) {
      VCX_TRY(launch_on(s, stream, prof, "gradient", [&](hipEvent_t ea, hipEvent_t eb) {
        hipExtLaunchKernelGGL((k_grad_node_batch<ND, NGF>), dim3(xcd_grid(br.ngrad_blocks)),
                              dim3(64 * kGradNodeGroups), 0, stream, ea, eb, 0, (const BatchEntry*)br.tab,
                              (const int2*)br.grad_map, br.ngrad_blocks, st);
      }));
    } else {
      VCX_TRY(launch_on(s, stream, prof, "gradient", [&](hipEvent_t ea, hipEvent_t eb) {
        hipExtLaunchKernelGGL((k_grad_tile_batch<ND, NGF>), dim3(xcd_grid(br.ntile_blocks)),
                           dim3(br.tile_block), br.lds_grad, stream, ea, eb, 0, (const BatchEntry*)br.tab,
                           (const int2*)br.tile_map, br.ntile_blocks, st);
      }));
    }
    if constexpr (MODEL == 0) {
      GasParams gp{s->ph.gamma, s->ph.beta, s->ph.entropy_fix, s->ph.limiter};
      VCX_TRY(launch_on(s, stream, prof, "flux", [&](hipEvent_t ea, hipEvent_t eb) {
        hipExtLaunchKernelGGL((k_flux_gas_batch<ND, NSP, FLUX, CT>), dim3(xcd_grid(br.ntile_blocks)),
                           dim3(br.tile_block), br.lds_flux, stream, ea, eb, 0, (const BatchEntry*)br.tab,
                           (const int2*)br.tile_map, br.ntile_blocks, st, gp, fs);
      }));
    } else if constexpr (MODEL == 2) {
      GasParams gp{s->ph.gamma, s->ph.beta, s->ph.entropy_fix, s->ph.limiter};
      VCX_TRY(launch_on(s, stream, prof, "flux", [&](hipEvent_t ea, hipEvent_t eb) {
        hipExtLaunchKernelGGL((k_flux_ns_batch<ND, NSP, CT>), dim3(xcd_grid(br.ntile_blocks)),
                           dim3(br.flux_block), br.lds_flux, stream, ea, eb, 0, (const BatchEntry*)br.tab,
                           (const int2*)br.tile_map, br.ntile_blocks, st, gp, fs);
      }));
    } else {
      DDParams pp{};
      for (int k = 0; k < NSP; ++k) {
        pp.zmu[k] = s->ph.z[k] * s->ph.mu[k];
        pp.D[k] = s->ph.D[k];
      }
      pp.beta = s->ph.beta;
      pp.limiter = s->ph.limiter;
      VCX_TRY(launch_on(s, stream, prof, "flux", [&](hipEvent_t ea, hipEvent_t eb) {
        hipExtLaunchKernelGGL((k_flux_dd_batch<ND, NSP, CT>), dim3(xcd_grid(br.ntile_blocks)),
                           dim3(br.tile_block), br.lds_flux, stream, ea, eb, 0, (const BatchEntry*)br.tab,
                           (const int2*)br.tile_map, br.ntile_blocks, st, pp, fs);
      }));
    }
    return launch_on(s, stream, prof, "update", [&](hipEvent_t ea, hipEvent_t eb) {
      hipExtLaunchKernelGGL((k_update_shared_batch<ND, NSP, MODEL>), dim3(br.nsh_blocks), dim3(kNodeBlock), 0,
                         stream, ea, eb, 0, (const BatchEntry*)br.tab, (const int2*)br.sh_map, st, fs);
    });
  }
  // second closure option: boundary-node closure fluxes of the stage input
  static vcx_status closure2(vcx_solver s, const Finish& f) {
    const DevMesh& m = s->mesh->d;
    if constexpr (ND == 2 && MODEL != 2) {
      if (m.nb == 0) return VCX_OK;
      hipLaunchKernelGGL((k_closure2<ND, NSP, MODEL>), dim3((m.nb + 255) / 256), dim3(256), 0, s->mesh->stream,
                         m, f, s->cbuf);
      VCX_HIP(hipGetLastError());
      return VCX_OK;
    } else {
      return vcx::fail(VCX_E_ARG, "the interpolated closure is defined on plane 2D meshes");
    }
  }
  static vcx_status prim_to_cons(vcx_solver s, double* W) {
    const DevMesh& m = s->mesh->d;
    hipLaunchKernelGGL((k_prim_to_cons<ND, NSP, MODEL>), dim3((m.nn + 255) / 256), dim3(256), 0,
                       s->mesh->stream, W, m.nn, s->ph.gamma, mix_params(s->ph));
    VCX_HIP(hipGetLastError());
    return VCX_OK;
  }
  static const KernelTable* table() {
    static const KernelTable t{&grad,     &grad_complete, &flux,      &update_shared, &node_dt,
                               &lds_grad, &lds_flux,      &lds_fused, &fused,         &allow_lds,
                               &aux,      &batch_stage,   &closure2,  &prim_to_cons,  NW,
                               NGF};
    return &t;
  }
};

// Multi-species FP32 path: the gradient pass stores G in FP32, the values the
// flux pass stages.
inline bool g_fp32(vcx_solver s) {
  return s->ph.model == VCX_MODEL_NAVIER_STOKES && s->ph.precision == VCX_PREC_MIXED;
}

// Doubles of one staged-row buffer: nn FP64 rows of ldws, then on the FP32
// path the FP32 rows (nn rows of ns_row32 of the FP32 path's staged count).
inline size_t staged_doubles(size_t nn, int ldws, int nd, int nsp, bool fp32) {
  if (!ldws) return 0;
  return (size_t)ldws * nn + (fp32 ? ((size_t)ns_row32(ns_staged_rows(nd, nsp, false)) * nn + 1) / 2 : 0);
}

inline Finish make_finish(vcx_solver s) {
  Finish f{};
  f.cbuf = s->cbuf;
  f.G = s->G;
  f.PG = s->PG;
  f.E = s->E;
  f.dc = dt_coef(s->ph);
  f.mix = mix_params(s->ph);
  f.closure = s->ph.closure;
  f.nws = s->nws;
  f.ldws = s->ldws;
  // fused passes with a closure that reads gradients complete G on every
  // node; so do the node-gradient passes
  f.gfull = (s->fused && s->gout != nullptr) || s->ph.model == VCX_MODEL_NAVIER_STOKES || s->dd_ngrad;
  f.gnode = s->dd_ngrad ? 1 : 0;
  f.g32 = g_fp32(s) ? 1 : 0;
  return f;
}

// Kernel tables by model (one translation unit each); nullptr for an
// unsupported species count or flux.
namespace vcx {
const KernelTable* pick_table_gas2(const vcx_physics& ph);
const KernelTable* pick_table_gas3(const vcx_physics& ph);
const KernelTable* pick_table_dd(int nd, const vcx_physics& ph);
const KernelTable* pick_table_ns(int nd, const vcx_physics& ph);
// 2D quadrilateral meshes (gas and drift-diffusion)
const KernelTable* pick_table_quad(const vcx_physics& ph);
// validate physics against a mesh and pick its table (vcx_capi.hip)
vcx_status check_physics(vcx_mesh mesh, const vcx_physics& ph, const double* E, const KernelTable** kt);
// tile-edge tables of a mesh (host build and device upload, once)
// Build (host) and upload (device) the tables of the multi-species passes
// (tile edges, node gradient) of a mesh, once.
vcx_status ensure_tile_edges(vcx_mesh m);

// host-side configuration of a solver: sizes, LDS, fused pass, launch shapes
vcx_status configure_solver(vcx_solver s, vcx_mesh mesh, const vcx_physics& ph, const KernelTable* kt);
}  // namespace vcx

template <int MODEL, int ND, int NSP, int NV = ND + 1>
inline const KernelTable* pick_flux_prec(int flux, int prec) {
  if (MODEL != 0) return prec == VCX_PREC_MIXED ? Impl<MODEL, ND, NSP, 0, float, NV>::table()
                                                : Impl<MODEL, ND, NSP, 0, double, NV>::table();
  if (flux == VCX_FLUX_HLLC)
    return prec == VCX_PREC_MIXED ? Impl<MODEL, ND, NSP, 0, float, NV>::table()
                                  : Impl<MODEL, ND, NSP, 0, double, NV>::table();
  return prec == VCX_PREC_MIXED ? Impl<MODEL, ND, NSP, 1, float, NV>::table()
                                : Impl<MODEL, ND, NSP, 1, double, NV>::table();
}
