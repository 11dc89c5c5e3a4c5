// HIP kernels of the vertex-centred residual (gfx950, wave64).
//
// Data layout in HBM (internal space-filling-curve order, structure of arrays):
//   W   [nr][nn]       reconstructed variables (gas: conserved + pressure;
//                      drift-diffusion: densities)
//   G   [nr*nd][nn]    nodal gradients, component v*nd + d
//   PG  [P][nr*nd]     gradient partial sums, one per (tile, node) slot (slot-major,
//                      so gathering a node's partials touches one segment per slot)
//   PR  [P][nvar]      residual partial sums per slot
// Per step: dt -> K x (gradient tile pass, gradient gather, flux tile pass,
// gather + closure + RK stage update).  No floating-point atomics: every sum
// is taken in a fixed order (cells of a tile in curve order, then slots of a
// node in tile order), so results are bitwise reproducible.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "vcx_device.h"

namespace vcx {

constexpr int NXCD = 8;  // MI355X: 8 accelerator complex dies, round-robin dispatch

// Minimum waves per SIMD requested for the flux tile kernels (0: compiler
// default).  Higher occupancy hides more memory latency but may spill.
#ifndef VCX_FLUX_WAVES
#define VCX_FLUX_WAVES 0
#endif
#if VCX_FLUX_WAVES > 0
#define VCX_FLUX_BOUNDS __launch_bounds__(256, VCX_FLUX_WAVES)
#else
#define VCX_FLUX_BOUNDS __launch_bounds__(256)
#endif

// The fused drift-diffusion pass aims at four 256-thread blocks per CU (all
// tiles of a 200k-cell mesh resident at once); the gas passes need their
// registers more than the occupancy.
#define VCX_FUSED_BOUNDS __launch_bounds__(256, (MODEL == 1 ? 4 : 1))

struct DevMesh {
  int nd, nv, nn, nc, ntiles, nslots, nb, nshared;
  int max_tile_cells, max_tile_nodes;
  double period[3];
  const double* x;           // [nd][nn]
  const int32_t* cell;       // [nv][nc]
  const uint32_t* shift;     // [nc]
  const uint16_t* lconn;     // [nv][nc]
  const int32_t* tile_cell;  // [T+1]
  const int32_t* tile_slot;  // [T+1]
  const int32_t* slot_node;  // [P] node id, or ~node when the node has slots in other tiles
  const int32_t* slot_inc;   // [P+1]
  const uint16_t* inc;       // [nc*nv]
  const int32_t* tile_inc;   // [T+1] first incidence of each tile
  const int32_t* slot_pos;   // [P] position of the slot in its node's run of slots_of; the
                             // index of the slot's partial sums (a node's partials are contiguous)
  const int32_t* node_slot;  // [nn+1]
  const int32_t* slots_of;   // [P]
  const int2* slot_run;      // [P] [begin, end) of the slot's node run in slots_of
  const int32_t* shared;     // [nshared] nodes with more than one slot (ascending)
  const int2* shared_run;    // [nshared] [begin, end) of the shared node's run in slots_of
  // extended tiles (2D meshes): halo cells and nodes of each tile, and the
  // cells around each slot's node in ascending cell order (extended-local)
  int has_halo, nhalo, max_ext_cells, max_ext_nodes, max_tile_ginc;
  const int32_t* tile_hcell;  // [T+1]
  const uint16_t* hlconn;     // [nv][nhalo]
  const uint32_t* hshift;     // [nhalo]
  const int32_t* tile_hnode;  // [T+1]
  const int32_t* hnode;       // halo nodes (internal ids)
  const int32_t* slot_ginc;   // [P+1]
  const uint16_t* ginc;
  const int32_t* tile_ginc;   // [T+1]
  const double* inv_vol;     // [nn] 1 / V_i (gradients; the update on plane meshes)
  const double* vnode;       // [nn]
  // volumes of the update and of the conservation sums: V_i, or on
  // axisymmetric (x, r) meshes int r dA over the dual region (over 2 pi)
  const double* inv_vupd;    // [nn]
  const double* vupd;        // [nn]
  int axi;                   // axisymmetric (x, r) mesh
  const double* dxmin;       // [nn] smallest inscribed diameter of the cells around the node
  const int32_t* bnd_index;  // [nn] -1 or index into bnd_S
  const double* bnd_S;       // [nd][nb]
  // 2D boundary edge shares by boundary index (second closure option)
  const int32_t* bnd_node;   // [nb] internal ids of the boundary nodes
  const int32_t* bedge_ptr;  // [nb+1]
  const int32_t* bedge_nb;   // [nbe]
  const double* bedge_S;     // [nd][nbe]
  int nbe;
  const int32_t* perm;       // [nn] internal -> caller
  // tile edges (the multi-species flux pass): distinct edges of each tile's
  // cells, their cell-edges, and each slot's incident edges
  int has_edges, max_tile_edges;
  const int32_t* tile_edge;  // [T+1]
  const uint32_t* edge;      // [E] la | lb << 12 | image << 24
  const int32_t* edge_ce;    // [E+1] CSR into ce
  const uint16_t* ce;        // [nc*ne] (local cell << 4) | (cell-local edge << 1) | reversed
  const int32_t* slot_einc;  // [P+1] CSR into einc
  const uint16_t* einc;      // [2E] (tile edge << 1) | (slot's node is end b)
  // node gradient: per 64-node slice, the neighbours j != i of each node and
  // their coefficients C_ij, entry k of the slice's node l at
  // ng_off[slice] + 64 k + l (pad entries: j = i, C = 0)
  int has_ngrad, ng_nslices;
  long long ng_total;
  const long long* ng_off;   // [nslices+1]
  const int32_t* ng_nbr;     // [total]
  const double* ng_c;        // [nd][total]
};

// Per-solve device scalars of the time loop: the state of one step.
struct DevScalars {
  double t;        // committed time
  double dt;       // time step of the running step
  double t_end;    // <= 0: none
  double last_dt;
  double dt_query;
  int flag;        // 1 unstable state, 2 invalid time step
  int active;      // the running step does work
  int pending;     // a started step awaits its commit
  int dt_src;      // 0: candidates from the node pass, 1: from the last step
  int steps_left;  // steps this call may still start (< 0: unlimited)
  long long steps; // committed steps
};

// Time-step candidates are posted by atomic minimum into a few slots (block
// b into slot b mod kCandSlots), on an integer key that orders like the
// double, so that a reader takes the minimum of kCandSlots values.
constexpr int kCandSlots = 64;

// The time loop of a solve.  Steps alternate between two parities: a step
// of parity p decides from the state s[p ^ 1] (the previous step's, or the
// one set up by the host) into s[p], raises failures in found[p] and posts
// the time-step candidates of its new state in cand[p].  So no kernel of a
// step writes what another block of the same launch reads.
struct DevLoop {
  DevScalars s[2];
  int found[2];   // failures (1: unstable state) raised by a step's final stage
  int pad[2];
  long long cand[2][kCandSlots];  // candidates of each parity's new state
  long long cnode[kCandSlots];    // candidates of the node pass (after an upload or a query)
};

__host__ __device__ constexpr long long cand_empty() { return 0x7FF0000000000000ll; }  // +infinity

__device__ inline long long cand_key(double v) {
  const long long b = __double_as_longlong(v);
  return b >= 0 ? b : (b ^ 0x7FFFFFFFFFFFFFFFll);
}

__device__ inline double key_cand(long long k) {
  return __longlong_as_double(k >= 0 ? k : (k ^ 0x7FFFFFFFFFFFFFFFll));
}

__device__ inline void post_candidate(long long* slots, int b, double v) {
  __hip_atomic_fetch_min(&slots[b & (kCandSlots - 1)], cand_key(v), __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
}

// ---------------------------------------------------------------------------
// helpers
// ---------------------------------------------------------------------------

// Blocks are dispatched round-robin over the XCDs; give each XCD a contiguous
// range of tiles so neighbouring tiles share node data in the same L2.
__device__ inline int xcd_tile_of(int b, int ntiles) {
  const int per = (ntiles + NXCD - 1) / NXCD;
  return (b % NXCD) * per + b / NXCD;
}

__device__ inline int xcd_tile(int ntiles) { return xcd_tile_of(blockIdx.x, ntiles); }

inline int xcd_grid(int ntiles) { return ((ntiles + NXCD - 1) / NXCD) * NXCD; }

// Models whose gradient pass is the node pass (node-major G, complete on
// every node): the multi-species model, and the gas model on tetrahedra.
__host__ __device__ constexpr bool node_gradient(int model, int nd, int nv) {
  return nv == nd + 1 && (model == 2 || (model == 0 && nd == 3));
}
// Models whose flux pass leaves every node to the update pass (each slot
// writes its partial): the tetrahedral ones, where nearly every node of a
// tile is shared anyway, and finishing the few owned nodes inside the flux
// pass set its register peak.
__host__ __device__ constexpr bool update_all(int model, int nd) { return model == 2 || (model == 0 && nd == 3); }
// Stride of a node's row of node-major G: its components rounded up to an
// even count, so that every row starts 16-byte aligned.
__host__ __device__ constexpr int node_row(int nc) { return nc + (nc & 1); }
// Rows of the multi-species node-major staged copy of the state: conserved,
// p, primitives and gamma, mu, lambda, plus the species D and h_s rows where
// the flux pass stages them (FP32) instead of forming them (FP64).
__host__ __device__ constexpr int ns_staged_rows(int nd, int nsp, bool fp64) {
  return (2 + nd + nsp) + 1 + (nd + 1 + nsp) + (fp64 ? 3 : 3 + 2 * nsp);
}
// The FP64 rows of a staged-row buffer hold the FP64 path's staged values
// (ns_staged_rows(nd, nsp, true)); after its nn rows the FP32 path keeps its
// own staged values in FP32 ([nn][ns_row32(ns_staged_rows(nd, nsp, false))],
// rows 16-byte aligned) for its flux staging: the values that staging
// rounded FP64 rows to.
__host__ __device__ constexpr int ns_row32(int nws) { return (nws + 3) & ~3; }
// Stride of the FP64 staged rows: even (rows 16-byte aligned) and an odd
// number of 16-byte units, so that a field of many rows does not fall on a
// few memory channels as with a power-of-two stride.
__host__ __device__ constexpr int ns_row64(int nws) { return node_row(nws) % 4 == 0 ? node_row(nws) + 2 : node_row(nws); }

__device__ inline bool step_inactive(const DevScalars* sc) {
  return sc != nullptr && sc->active == 0;
}

// Minimum over the block (blockDim.x a multiple of 64, at most 256); valid in
// thread 0.  Every thread of the block must call it.
__device__ inline double block_min(double v) {
  __shared__ double wmin[4];
  for (int off = 32; off > 0; off >>= 1) v = fmin(v, __shfl_xor(v, off, 64));
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) wmin[wv] = v;
  __syncthreads();
  double b = wmin[0];
  for (int q = 1; q < (int)(blockDim.x >> 6); ++q) b = fmin(b, wmin[q]);
  return b;
}

template <int ND, int NV = ND + 1>
__device__ inline void cell_rel_coords(const DevMesh& m, const double* sX, int maxn, const int (&l)[NV],
                                       uint32_t code, double (&e)[NV - 1][ND]) {
  for (int k = 1; k < NV; ++k)
    for (int d = 0; d < ND; ++d) {
      const uint32_t b = (code >> (2 * ((k - 1) * ND + d))) & 3u;
      const double s = b == 1u ? m.period[d] : (b == 2u ? -m.period[d] : 0.0);
      e[k - 1][d] = sX[d * maxn + l[k]] + s - sX[d * maxn + l[0]];
    }
}

__device__ inline int slot_node_id(int v) { return v >= 0 ? v : ~v; }

// Element i (not a compile-time constant) of a small register array, by a
// chain of selects, so that the array stays in registers inside a loop that
// is not unrolled.
template <int N, typename T>
__device__ __attribute__((always_inline)) inline T pick(const T (&x)[N], int i) {
  T r = x[0];
#pragma unroll
  for (int k = 1; k < N; ++k) r = i == k ? x[k] : r;
  return r;
}

// Cell-edge ed (not unrolled) of a cell: its vertices a < b, their tile-local
// nodes, the dual-face vector S_ab = (S_a - S_b)/(n_d n_v) and the edge
// vector X_b - X_a from the relative coordinates e[k-1] = X_k - X_0, with the
// same arithmetic as the unrolled form; coef[k] = +1 (k = a), -1 (k = b) or 0
// carries the flux to the cell vertex sums as fma(F, coef[k], acc[k]), which
// rounds like acc[a] + F and acc[b] - F.
template <int ND, typename CT>
struct EdgeRolled {
  int a, b, la, lb;
  CT S[ND], dx[ND];
  double coef[ND + 1];
};

template <int ND, typename CT>
__device__ __attribute__((always_inline)) inline void edge_rolled(int ed, const int (&l)[ND + 1],
                                                                  const double (&e)[ND][ND],
                                                                  const double (&Sd)[ND + 1][ND],
                                                                  EdgeRolled<ND, CT>& g) {
  constexpr int NV = ND + 1;
  g.a = Edges<ND>::a(ed);
  g.b = Edges<ND>::b(ed);
  g.la = pick(l, g.a);
  g.lb = pick(l, g.b);
#pragma unroll
  for (int d = 0; d < ND; ++d) {
    double sc[NV], ec[ND];
#pragma unroll
    for (int k = 0; k < NV; ++k) sc[k] = Sd[k][d];
#pragma unroll
    for (int k = 0; k < ND; ++k) ec[k] = e[k][d];
    g.S[d] = CT((pick(sc, g.a) - pick(sc, g.b)) * (1.0 / double(ND * NV)));
    g.dx[d] = CT((g.a == 0 ? 0.0 : -pick(ec, g.a - 1)) + pick(ec, g.b - 1));
  }
#pragma unroll
  for (int k = 0; k < NV; ++k) g.coef[k] = k == g.a ? 1.0 : (k == g.b ? -1.0 : 0.0);
}

// The same for a compile-time edge.
template <int ED, int ND, typename CT>
__device__ __attribute__((always_inline)) inline void edge_static(const int (&l)[ND + 1], const double (&e)[ND][ND],
                                                                  const double (&Sd)[ND + 1][ND],
                                                                  EdgeRolled<ND, CT>& g) {
  constexpr int NV = ND + 1, a = Edges<ND>::a(ED), b = Edges<ND>::b(ED);
  g.a = a;
  g.b = b;
  g.la = l[a];
  g.lb = l[b];
#pragma unroll
  for (int d = 0; d < ND; ++d) {
    g.S[d] = CT((Sd[a][d] - Sd[b][d]) * (1.0 / double(ND * NV)));
    g.dx[d] = CT((a == 0 ? 0.0 : -e[a == 0 ? 0 : a - 1][d]) + e[b - 1][d]);
  }
#pragma unroll
  for (int k = 0; k < NV; ++k) g.coef[k] = k == a ? 1.0 : (k == b ? -1.0 : 0.0);
}

// Edge ed of a tetrahedron, ed the same in every lane: a scalar branch to the
// compile-time form (no run-time indexing of register arrays).
template <typename CT>
__device__ __attribute__((always_inline)) inline void edge_uniform3(int ed, const int (&l)[4], const double (&e)[3][3],
                                                                    const double (&Sd)[4][3], EdgeRolled<3, CT>& g) {
  switch (__builtin_amdgcn_readfirstlane(ed)) {
    case 0: edge_static<0, 3, CT>(l, e, Sd, g); break;
    case 1: edge_static<1, 3, CT>(l, e, Sd, g); break;
    case 2: edge_static<2, 3, CT>(l, e, Sd, g); break;
    case 3: edge_static<3, 3, CT>(l, e, Sd, g); break;
    case 4: edge_static<4, 3, CT>(l, e, Sd, g); break;
    default: edge_static<5, 3, CT>(l, e, Sd, g); break;
  }
}

// Tile topology read at the start of a tile pass, so that its loads are in
// flight together with the staging of the node data: this thread's cell and
// slot (the first iteration of the cell and slot loops) and up to NV of the
// tile's incidence codes, which are stored to LDS after the staging.
template <int NV>
struct TilePre {
  int c0, nc, s0, ns, pb, ninc;
  int l[NV];
  uint32_t shift;
  int sv, pos, p0, p1;  // slot threadIdx.x: node, partial index, incidence range in the tile
  int2 run;             // its node's run in slots_of
  int inc[NV];
};

template <int NV>
__device__ inline void tile_prefetch(const DevMesh& m, int t, TilePre<NV>& tp) {
  tp.c0 = m.tile_cell[t];
  tp.nc = m.tile_cell[t + 1] - tp.c0;
  tp.s0 = m.tile_slot[t];
  tp.ns = m.tile_slot[t + 1] - tp.s0;
  tp.pb = m.tile_inc[t];
  tp.ninc = m.tile_inc[t + 1] - tp.pb;
  const int i = threadIdx.x;
  if (i < tp.nc) {
#pragma unroll
    for (int k = 0; k < NV; ++k) tp.l[k] = m.lconn[(size_t)k * m.nc + tp.c0 + i];
    tp.shift = m.shift[tp.c0 + i];
  }
  if (i < tp.ns) {
    const int sl = tp.s0 + i;
    tp.sv = m.slot_node[sl];
    tp.pos = m.slot_pos[sl];
    tp.p0 = m.slot_inc[sl] - tp.pb;
    tp.p1 = m.slot_inc[sl + 1] - tp.pb;
    tp.run = m.slot_run[sl];
  }
#pragma unroll
  for (int j = 0; j < NV; ++j) {
    const int p = i + j * (int)blockDim.x;
    if (p < tp.ninc) tp.inc[j] = m.inc[tp.pb + p];
  }
}

template <int NV>
__device__ inline void tile_store_inc(const DevMesh& m, const TilePre<NV>& tp, uint16_t* sInc) {
#pragma unroll
  for (int j = 0; j < NV; ++j) {
    const int p = (int)threadIdx.x + j * (int)blockDim.x;
    if (p < tp.ninc) sInc[p] = (uint16_t)tp.inc[j];
  }
  for (int p = (int)threadIdx.x + NV * (int)blockDim.x; p < tp.ninc; p += blockDim.x)
    sInc[p] = m.inc[tp.pb + p];
}

struct SlotTopo {
  int sv, pos, p0, p1;
  int2 run;
};

// Slot table of a tile in LDS ([4][maxn] ints: node, partial index,
// incidence range), written while staging and read by the node pass, so
// that no registers hold it through the cell pass.
__device__ inline void slot_table_put(int* sSl, int maxn, int q, int sv, int pos, int p0, int p1) {
  sSl[q] = sv;
  sSl[maxn + q] = pos;
  sSl[2 * maxn + q] = p0;
  sSl[3 * maxn + q] = p1;
}

__device__ inline SlotTopo slot_table_get(const int* sSl, int maxn, int q) {
  return SlotTopo{sSl[q], sSl[maxn + q], sSl[2 * maxn + q], sSl[3 * maxn + q], make_int2(0, 0)};
}

template <int NV>
__device__ inline SlotTopo slot_topo(const DevMesh& m, const TilePre<NV>& tp, int q) {
  if (q == (int)threadIdx.x) return SlotTopo{tp.sv, tp.pos, tp.p0, tp.p1, tp.run};
  const int sl = tp.s0 + q;
  return SlotTopo{m.slot_node[sl], m.slot_pos[sl], m.slot_inc[sl] - tp.pb, m.slot_inc[sl + 1] - tp.pb,
                  m.slot_run[sl]};
}

template <int NV>
__device__ inline void cell_topo(const DevMesh& m, const TilePre<NV>& tp, int lc, int (&l)[NV],
                                 uint32_t& shift) {
  if (lc == (int)threadIdx.x) {
#pragma unroll
    for (int k = 0; k < NV; ++k) l[k] = tp.l[k];
    shift = tp.shift;
    return;
  }
#pragma unroll
  for (int k = 0; k < NV; ++k) l[k] = m.lconn[(size_t)k * m.nc + tp.c0 + lc];
  shift = m.shift[tp.c0 + lc];
}

// bytes of the incidence codes staged in LDS, rounded to doubles
__host__ __device__ inline size_t inc_lds_bytes(int nv, int maxc) {
  return ((size_t)nv * maxc * sizeof(uint16_t) + 7) / 8 * 8;
}

// bytes of a tile's slot table in LDS
__host__ __device__ inline size_t slot_lds_bytes(int maxn) { return (size_t)4 * maxn * sizeof(int); }

// LDS of the edge-based multi-species flux pass, in order: node coordinates
// (double), the tile edges' net fluxes (double [NVAR][maxe]), the cell-edge
// dual-face vectors (CT [ND][maxc * ne]), the node staging area of the two
// phases (CT rows: A = reconstructed rows, gamma and their gradients; B =
// rho, primitives, transport rows and the gradients of the primitives), the
// slot table and the slots' edge incidences.
template <int ND, int NSP, typename CT>
struct NsEdgeLds {
  static constexpr int NVAR = 2 + ND + NSP, NR = NVAR + 1, NP = ND + 1 + NSP, NA = 3 + 2 * NSP;
  static constexpr int NCE = ND == 2 ? 3 : 6;  // cell-edges per cell
  // FP64 forms D_k and h_s,k at the edge ends from mu, rho and T; FP32 stages them
  static constexpr bool RECOMPUTE = sizeof(CT) == 8;
  static constexpr int RA = NR + 1, CA = NR * ND;
  static constexpr int RB = 1 + NP + (RECOMPUTE ? 2 : NA - 1), CB = NP * ND;
  __host__ __device__ static size_t r8(size_t b) { return (b + 7) / 8 * 8; }
  __host__ __device__ static size_t x_bytes(int maxn) { return sizeof(double) * (size_t)ND * maxn; }
  __host__ __device__ static size_t f_bytes(int maxe) { return sizeof(double) * (size_t)NVAR * maxe; }
  __host__ __device__ static size_t s_bytes(int maxc) { return r8(sizeof(CT) * (size_t)ND * maxc * NCE); }
  __host__ __device__ static size_t area_bytes(int maxn) {
    return r8(sizeof(CT) * (size_t)(RA + CA > RB + CB ? RA + CA : RB + CB) * maxn);
  }
  __host__ __device__ static size_t lds_bytes(int maxn, int maxc, int maxe) {
    return x_bytes(maxn) + f_bytes(maxe) + s_bytes(maxc) + area_bytes(maxn) + slot_lds_bytes(maxn) +
           r8(sizeof(uint16_t) * 2 * (size_t)maxe);
  }
};

// Decision of a step from the state it starts from: commit the previous
// step unless it failed, then start this one (or stop at the end time, the
// step budget or on failure).  d is the smallest candidate of the state.
__device__ inline void step_decide(const DevScalars& prev, int found_prev, double d, DevScalars& n) {
  n = prev;
  const int fl = prev.flag | found_prev;
  if (n.pending) {
    if (fl == 0) {
      n.t += n.dt;
      n.last_dt = n.dt;
      n.steps += 1;
    }
    n.pending = 0;
  }
  n.flag = fl;
  n.active = 0;
  const bool done_t = (n.t_end > 0.0 && n.t >= n.t_end) || n.steps_left == 0;
  if (n.flag == 0 && !done_t) {
    if (!(d > 0.0) || !isfinite(d)) {
      n.flag |= 2;  // non-physical state or no limiting time scale
    } else {
      if (n.t_end > 0.0 && n.t + d > n.t_end) d = n.t_end - n.t;
      n.dt = d;
      n.active = 1;
      n.pending = 1;
      if (n.steps_left > 0) n.steps_left -= 1;
    }
  }
}

// Smallest candidate of the state a step of parity par starts from
// (block-wide, at least kCandSlots threads; valid in thread 0).
__device__ inline double step_candidate(const DevLoop* lp, int par) {
  const long long* slots = lp->s[par ^ 1].dt_src ? lp->cand[par ^ 1] : lp->cnode;
  const double v = threadIdx.x < kCandSlots ? key_cand(slots[threadIdx.x]) : INFINITY;
  return block_min(v);
}

// After the step of parity par has been decided (and before it posts): the
// candidates of the state it started from move on to parity par when the
// step does no work (the state stays the same), and the previous parity's
// slots and failures are emptied for the next step.  So after every step of
// parity q, cand[q] holds the current state's candidates and cand[q ^ 1] is
// empty.
__device__ inline void step_rollover(DevLoop* lp, int par, int active) {
  if (threadIdx.x < kCandSlots) {
    if (!active) lp->cand[par][threadIdx.x] = lp->cand[par ^ 1][threadIdx.x];
    lp->cand[par ^ 1][threadIdx.x] = cand_empty();
  }
  if (threadIdx.x == 0) lp->found[par ^ 1] = 0;
}

// One block decides the step of parity par and writes its state.
__device__ inline void step_start(DevLoop* lp, int par) {
  const double d = step_candidate(lp, par);
  __shared__ int act;
  if (threadIdx.x == 0) {
    DevScalars n;
    step_decide(lp->s[par ^ 1], lp->found[par ^ 1], d, n);
    lp->s[par] = n;
    act = n.active;
  }
  __syncthreads();
  step_rollover(lp, par, act);
}

// Commit the pending step of the state of parity par (end of a host call).
__device__ inline void step_finish(DevLoop* lp, int par) {
  DevScalars& sc = lp->s[par];
  const int fl = sc.flag | lp->found[par];
  if (sc.pending) {
    if (fl == 0) {
      sc.t += sc.dt;
      sc.last_dt = sc.dt;
      sc.steps += 1;
    }
    sc.pending = 0;
  }
  sc.flag = fl;
  lp->found[par] = 0;
  sc.active = 0;
}

// ---------------------------------------------------------------------------
// per-node time-step candidate: CFL dx_min / lambda and Fourier dx_min^2 / D
// with dx_min the smallest inscribed diameter of the cells around the node;
// the minimum over nodes equals the minimum over cells of the cell-based
// limits (the maximum speed of a cell is attained at one of its nodes).
// Returns -1 for a non-physical gas state.
// ---------------------------------------------------------------------------

struct DtCoef {
  double cfl, fourier, gamma;
  double zmu[4], D[4];
  // dielectric limit A_D eps0 / sum_s |q_s n_s mu_s| (0: off): A_D eps0,
  // e z_s and mu_s per species
  double adeps, ez[4], mu[4];
};

template <int ND, int NSP, int MODEL>
__device__ inline double node_dt(const DtCoef& c, double dx, const double* Ei, const double* u, double p) {
  if constexpr (MODEL == 0) {
    const double rho = u[0];
    double uu = 0.0;
#pragma unroll
    for (int d = 0; d < ND; ++d) {
      const double ud = u[1 + d] / rho;
      uu += ud * ud;
    }
    if (!(rho > 0.0) || !(p > 0.0)) return -1.0;
    const double lam = sqrt(uu) + sqrt(c.gamma * p / rho);
    return c.cfl * dx / lam;
  } else {
    double best = INFINITY;
#pragma unroll
    for (int s = 0; s < NSP; ++s) {
      double v2 = 0.0;
#pragma unroll
      for (int d = 0; d < ND; ++d) {
        const double vd = c.zmu[s] * Ei[d];
        v2 += vd * vd;
      }
      const double vmax = sqrt(v2);
      if (vmax > 0.0) best = fmin(best, c.cfl * dx / vmax);
      if (c.D[s] > 0.0) best = fmin(best, c.fourier * dx * dx / c.D[s]);
    }
    if (c.adeps > 0.0) {
      double sig = 0.0;
#pragma unroll
      for (int s = 0; s < NSP; ++s) sig += fabs(c.ez[s] * u[s] * c.mu[s]);
      if (sig > 0.0) best = fmin(best, c.adeps / sig);
    }
    return best;
  }
}

// Multi-species candidate: convective CFL dx/(|u| + a) with the mixture
// sound speed, diffusive F dx^2 / max(nu, lambda/(rho c_p), D_k) where
// lambda/(rho c_p) = mu/(rho Pr).
template <int ND, int NSP>
__device__ inline double ns_node_dt(double dx, const DtCoef& c, const MixParams& mp, double rho,
                                    const double* prim, double p, const double* aux, bool ok) {
  if (!ok) return -1.0;
  double uu = 0.0;
#pragma unroll
  for (int d = 0; d < ND; ++d) uu += prim[d] * prim[d];
  const double lam = sqrt(uu) + sqrt(aux[0] * p / rho);
  double dm = fmax(aux[1] / rho, aux[1] / (rho * mp.Pr));
#pragma unroll
  for (int k = 0; k < NSP; ++k) dm = fmax(dm, aux[3 + k]);
  double t = c.cfl * dx / lam;
  if (dm > 0.0) t = fmin(t, c.fourier * dx * dx / dm);
  return t;
}

// ---------------------------------------------------------------------------
// gradient: per cell  g_tau = sum_k W_k S_k ; per node  G_i = -1/(nd nv V_i) sum g_tau
// A node whose cells all lie in the tile gets G directly; a node shared with
// other tiles gets one partial sum per tile (PG), gathered by its readers.
// ---------------------------------------------------------------------------

struct GradCtl {
  DevLoop* lp;     // null outside the time loop
  int par;         // parity of the step
  int first_stage; // first stage: an extra block decides the step
};

// Fields per pass of the gradient kernel: at most 8 (at most 4 for states
// of more than 16 fields), in equal groups, so that the staged fields and
// cell parts of many-field states (multi-species Navier-Stokes) take a
// fraction of the LDS and more blocks fit on a CU.
__host__ __device__ constexpr int grad_group(int nr) {
  return nr > 16 ? (nr + (nr + 3) / 4 - 1) / ((nr + 3) / 4) : (nr + (nr + 7) / 8 - 1) / ((nr + 7) / 8);
}

template <int ND, int NR, int NV = ND + 1>
__device__ inline void grad_tile_body(const DevMesh& m, const double* __restrict__ W,
                                      double* __restrict__ G, double* __restrict__ PG,
                                      const GradCtl& ctl, int t, double* lds) {
  constexpr int NC = NR * ND, FG = grad_group(NR);
  // later stages of a step that does no work (set by an earlier launch)
  if (ctl.lp && !ctl.first_stage && ctl.lp->s[ctl.par].active == 0) return;
  TilePre<NV> tp;
  tile_prefetch<NV>(m, t, tp);
  const int maxn = m.max_tile_nodes, maxc = m.max_tile_cells;
  double* sW = lds;                 // [FG][maxn] fields of this group
  double* sX = sW + FG * maxn;      // [ND][maxn]
  double* sC = sX + ND * maxn;      // [FG*ND][maxc]
  uint16_t* sInc = reinterpret_cast<uint16_t*>(sC + FG * ND * maxc);
  const int nc = tp.nc, ns = tp.ns;
  double iv = 0.0;  // 1/V of this thread's slot node (tile-owned nodes)
  // the fields in groups of FG: stage, cell parts, node sums
  for (int v0 = 0; v0 < NR; v0 += FG) {
    if (v0 > 0) __syncthreads();  // the previous group's node sums have read sC
    for (int q = threadIdx.x; q < ns; q += blockDim.x) {
      const int sv = q == (int)threadIdx.x ? tp.sv : m.slot_node[tp.s0 + q];
      const int g = slot_node_id(sv);
      double w[FG];
#pragma unroll
      for (int vv = 0; vv < FG; ++vv)
        if (v0 + vv < NR) w[vv] = W[(size_t)(v0 + vv) * m.nn + g];
      if (v0 == 0) {
        if (q == (int)threadIdx.x && sv >= 0) iv = m.inv_vol[sv];
        double xx[ND];
#pragma unroll
        for (int d = 0; d < ND; ++d) xx[d] = m.x[(size_t)d * m.nn + g];
#pragma unroll
        for (int d = 0; d < ND; ++d) sX[d * maxn + q] = xx[d];
      }
#pragma unroll
      for (int vv = 0; vv < FG; ++vv)
        if (v0 + vv < NR) sW[vv * maxn + q] = w[vv];
    }
    if (v0 == 0) tile_store_inc<NV>(m, tp, sInc);
    __syncthreads();
    for (int lc = threadIdx.x; lc < nc; lc += blockDim.x) {
      int l[NV];
      uint32_t sh;
      cell_topo<NV>(m, tp, lc, l, sh);
      double e[NV - 1][ND], S[NV][ND];
      cell_rel_coords<ND, NV>(m, sX, maxn, l, sh, e);
      Shape<ND, NV>::normals(e, S);
#pragma unroll
      for (int vv = 0; vv < FG; ++vv) {
        if (v0 + vv >= NR) break;
        double acc[ND];
#pragma unroll
        for (int d = 0; d < ND; ++d) acc[d] = 0.0;
#pragma unroll
        for (int k = 0; k < NV; ++k) {
          const double w = sW[vv * maxn + l[k]];
#pragma unroll
          for (int d = 0; d < ND; ++d) acc[d] += w * S[k][d];
        }
#pragma unroll
        for (int d = 0; d < ND; ++d) sC[(vv * ND + d) * maxc + lc] = acc[d];
      }
    }
    __syncthreads();
    // this group's components, in chunks of JC to bound register use
    constexpr int NCG = FG * ND;
    constexpr int JC = NCG <= 24 ? NCG : 12;
    const int ncg = min(NR - v0, FG) * ND, j00 = v0 * ND;
    for (int q = threadIdx.x; q < ns; q += blockDim.x) {
      const SlotTopo st = slot_topo<NV>(m, tp, q);
      const int sv = st.sv;
      double coef = 0.0;
      if (sv >= 0) coef = -(q == (int)threadIdx.x ? iv : m.inv_vol[sv]) / double(ND * NV);
      for (int j0 = 0; j0 < ncg; j0 += JC) {
        double acc[JC];
#pragma unroll
        for (int jj = 0; jj < JC; ++jj) acc[jj] = 0.0;
        for (int p = st.p0; p < st.p1; ++p) {
          const int lc = sInc[p] >> 2;
#pragma unroll
          for (int jj = 0; jj < JC; ++jj)
            if (j0 + jj < ncg) acc[jj] += sC[(j0 + jj) * maxc + lc];
        }
        if (sv >= 0) {
#pragma unroll
          for (int jj = 0; jj < JC; ++jj)
            if (j0 + jj < ncg) G[(size_t)(j00 + j0 + jj) * m.nn + sv] = coef * acc[jj];
        } else {
#pragma unroll
          for (int jj = 0; jj < JC; ++jj)
            if (j0 + jj < ncg) PG[(size_t)st.pos * NC + j00 + j0 + jj] = acc[jj];
        }
      }
    }
  }
}

template <int ND, int NR, int NV = ND + 1>
__global__ void __launch_bounds__(256) k_grad_tile(DevMesh m, const double* __restrict__ W,
                                                   double* __restrict__ G, double* __restrict__ PG,
                                                   GradCtl ctl) {
  extern __shared__ double lds[];
  // in the first stage of a step, block 0 reduces the time-step candidates
  // and commits (the tiles take the other blocks, so that no tile waits on it)
  const int lead = ctl.lp && ctl.first_stage ? 1 : 0;
  if (lead && blockIdx.x == 0) {
    step_start(ctl.lp, ctl.par);
    return;
  }
  const int t = xcd_tile_of((int)blockIdx.x - lead, m.ntiles);
  if (t >= m.ntiles) return;
  grad_tile_body<ND, NR, NV>(m, W, G, PG, ctl, t, lds);
}

// gradient of a shared node g from its per-tile partial sums, taken over the
// node's slots in ascending tile order (the same order for every reader)
template <int NC, int ND>
__device__ inline void shared_gradient(const DevMesh& m, const double* __restrict__ PG, int g,
                                       int2 run, double (&out)[NC]) {
  const double coef = -m.inv_vol[g] / double(ND * m.nv);
#pragma unroll
  for (int j = 0; j < NC; ++j) out[j] = 0.0;
  for (int p = run.x; p < run.y; ++p) {
    const double* src = PG + (size_t)p * NC;
#pragma unroll
    for (int j = 0; j < NC; ++j) out[j] += src[j];
  }
#pragma unroll
  for (int j = 0; j < NC; ++j) out[j] *= coef;
}

// Components [C0, C0 + NCS) of node g from node-major rows (NC components
// per node, contiguous, of type ST) into LDS (sG [NCS][maxn]).
// The row is read in pairs from its first even component (NC is the row
// stride, even: every node's row starts pair-aligned).
template <int NC, int C0, int NCS, typename CT, typename ST = double>
__device__ inline void stage_gradient_row(const ST* __restrict__ G, int g, CT* sG, int maxn, int q) {
  static_assert(NC % 2 == 0, "node rows of an even stride");
  if constexpr (std::is_same<ST, float>::value && NC % 4 == 0) {
    // FP32 rows of a stride divisible by 4: 16-byte quads between leading
    // and trailing singles
    constexpr int HL = (4 - C0 % 4) % 4 < NCS ? (4 - C0 % 4) % 4 : NCS;
    constexpr int NQ = (NCS - HL) / 4, TL = NCS - HL - 4 * NQ;
    const float* src = G + (size_t)g * NC + C0;
#pragma unroll
    for (int k = 0; k < HL; ++k) sG[k * maxn + q] = CT(src[k]);
    const float4* p4 = reinterpret_cast<const float4*>(src + HL);
    float4 v[NQ == 0 ? 1 : NQ];
#pragma unroll
    for (int k = 0; k < NQ; ++k) v[k] = p4[k];
#pragma unroll
    for (int k = 0; k < NQ; ++k) {
      sG[(HL + 4 * k) * maxn + q] = CT(v[k].x);
      sG[(HL + 4 * k + 1) * maxn + q] = CT(v[k].y);
      sG[(HL + 4 * k + 2) * maxn + q] = CT(v[k].z);
      sG[(HL + 4 * k + 3) * maxn + q] = CT(v[k].w);
    }
#pragma unroll
    for (int k = 0; k < TL; ++k) sG[(HL + 4 * NQ + k) * maxn + q] = CT(src[HL + 4 * NQ + k]);
    return;
  }
  using P2 = typename std::conditional<std::is_same<ST, double>::value, double2, float2>::type;
  constexpr int H = C0 % 2;                // a leading odd component, read alone
  constexpr int NPAIR = (NCS - H) / 2;     // then pairs
  constexpr int T = NCS - H - 2 * NPAIR;   // and a trailing single
  const ST* src = G + (size_t)g * NC + C0;
  if constexpr (H) sG[q] = CT(src[0]);
  const P2* p2 = reinterpret_cast<const P2*>(src + H);
  constexpr int PC = NPAIR == 0 ? 1 : (NPAIR <= 16 ? NPAIR : 8);
  for (int k0 = 0; k0 < NPAIR; k0 += PC) {
    P2 v[PC];
#pragma unroll
    for (int kk = 0; kk < PC; ++kk)
      if (k0 + kk < NPAIR) v[kk] = p2[k0 + kk];
#pragma unroll
    for (int kk = 0; kk < PC; ++kk)
      if (k0 + kk < NPAIR) {
        sG[(H + 2 * (k0 + kk)) * maxn + q] = CT(v[kk].x);
        sG[(H + 2 * (k0 + kk) + 1) * maxn + q] = CT(v[kk].y);
      }
  }
  if constexpr (T) sG[(NCS - 1) * maxn + q] = CT(src[NCS - 1]);
}

// Stage the NC gradient components of the tile's q-th node into LDS: read G
// for a tile-owned node, gather the slot partials of a shared node (in
// ascending partial order, the same for every reader).  Loads of a chunk of
// components are all issued before the first store.
template <int NC, int ND, typename CT>
__device__ inline void stage_gradient(const DevMesh& m, const double* __restrict__ G,
                                      const double* __restrict__ PG, int sv, int2 run, CT* sG,
                                      int maxn, int q) {
  if (sv >= 0) {
    constexpr int JC = NC <= 32 ? NC : 16;
    for (int j0 = 0; j0 < NC; j0 += JC) {
      double v[JC];
#pragma unroll
      for (int jj = 0; jj < JC; ++jj)
        if (j0 + jj < NC) v[jj] = G[(size_t)(j0 + jj) * m.nn + sv];
#pragma unroll
      for (int jj = 0; jj < JC; ++jj)
        if (j0 + jj < NC) sG[(j0 + jj) * maxn + q] = CT(v[jj]);
    }
    return;
  }
  const int g = ~sv;
  const double coef = -m.inv_vol[g] / double(ND * m.nv);
  constexpr int JC = NC <= 24 ? NC : 12;
  for (int j0 = 0; j0 < NC; j0 += JC) {
    double acc[JC];
#pragma unroll
    for (int jj = 0; jj < JC; ++jj) acc[jj] = 0.0;
    int p = run.x;
    for (; p + 1 < run.y; p += 2) {
      const double* s0 = PG + (size_t)p * NC + j0;
      const double* s1 = s0 + NC;
      double a[JC], b[JC];
#pragma unroll
      for (int jj = 0; jj < JC; ++jj)
        if (j0 + jj < NC) {
          a[jj] = s0[jj];
          b[jj] = s1[jj];
        }
#pragma unroll
      for (int jj = 0; jj < JC; ++jj)
        if (j0 + jj < NC) acc[jj] = (acc[jj] + a[jj]) + b[jj];
    }
    if (p < run.y) {
      const double* s0 = PG + (size_t)p * NC + j0;
#pragma unroll
      for (int jj = 0; jj < JC; ++jj)
        if (j0 + jj < NC) acc[jj] += s0[jj];
    }
#pragma unroll
    for (int jj = 0; jj < JC; ++jj)
      if (j0 + jj < NC) sG[(j0 + jj) * maxn + q] = CT(coef * acc[jj]);
  }
}

// Complete G on the shared nodes of a tile-gradient pass (the
// drift-diffusion flux launcher runs it once per stage, so that its flux pass
// and closure read complete rows; also the gradient output).
// A block takes kGradSharedNodes shared nodes: its threads walk the (node,
// component) pairs component-fastest, so the reads of a partial row are
// contiguous, sum each component over the node's partials in run order
// (the order of shared_gradient), and the block then writes G node-fastest
// from LDS.
constexpr int kGradSharedNodes = 32;
template <int ND, int NR>
__device__ inline void grad_shared_body(const DevMesh& m, const double* __restrict__ PG,
                                        double* __restrict__ G, int k0) {
  constexpr int NC = NR * ND, NB = kGradSharedNodes;
  __shared__ double sg[NC * NB];
  __shared__ int snode[NB];
  const int nb = min(NB, m.nshared - k0);
  if (nb <= 0) return;
  if ((int)threadIdx.x < nb) snode[threadIdx.x] = m.shared[k0 + threadIdx.x];
  for (int idx = threadIdx.x; idx < nb * NC; idx += blockDim.x) {
    const int i = idx / NC, j = idx - i * NC;
    const int2 run = m.shared_run[k0 + i];
    double acc = 0.0;
    // four partials in flight at a time, added in run order
    int p = run.x;
    for (; p + 4 <= run.y; p += 4) {
      const double* src = PG + (size_t)p * NC + j;
      const double a = src[0], b = src[NC], c = src[2 * NC], d = src[3 * NC];
      acc += a;
      acc += b;
      acc += c;
      acc += d;
    }
    for (; p < run.y; ++p) acc += PG[(size_t)p * NC + j];
    sg[j * NB + i] = acc;
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < nb * NC; idx += blockDim.x) {
    const int j = idx / nb, i = idx - j * nb;
    const int g = snode[i];
    const double coef = -m.inv_vol[g] / double(ND * m.nv);
    G[(size_t)j * m.nn + g] = coef * sg[j * NB + i];
  }
}

template <int ND, int NR>
__global__ void __launch_bounds__(256) k_grad_shared(DevMesh m, const double* __restrict__ PG,
                                                     double* __restrict__ G) {
  grad_shared_body<ND, NR>(m, PG, G, (int)blockIdx.x * kGradSharedNodes);
}

// Node gradient: G_i = -1/(nd nv V_i) sum_{j != i} (W_j - W_i) C_ij over the
// node's neighbours j in ascending order (the cell sum regrouped by
// neighbour, the node's own term folded in through C_ii = -sum_{j != i} C_ij,
// which holds since a simplex's node normals sum to zero; no partial sums).  A block takes one 64-node slice: each of its
// kGradNodeGroups wavefronts takes an equal share of the fields for the
// slice's 64 nodes (lane = node), so the loads of a neighbour index, its coefficients and a field row
// are coalesced across the wavefront.  G is node-major (the NR * ND
// components of a node contiguous, component v * ND + d, rows of
// node_row(NR * ND)): the block gathers the slice's rows in LDS and writes
// them as one contiguous run.
#ifndef VCX_GRAD_NODE_GROUPS
#define VCX_GRAD_NODE_GROUPS 2
#endif
constexpr int kGradNodeGroups = VCX_GRAD_NODE_GROUPS;
// WSR: the fields come from the node-major staged rows WS ([nn][ldws]) of
// the multi-species model instead of the component-major W.  GT: the type
// G is stored in (sums in FP64 either way; FP32 for a flux pass that stages
// its gradients in FP32, which then reads the same values).
template <int ND, int NR, bool WSR = false, typename GT = double>
__device__ inline void grad_node_body(const DevMesh& m, const double* __restrict__ W,
                                      const double* __restrict__ WS, int ldws,
                                      GT* __restrict__ G, const GradCtl& ctl, int sl) {
  constexpr int FG = (NR + kGradNodeGroups - 1) / kGradNodeGroups, NC = NR * ND, NCP = node_row(NC);
  constexpr int LD = NCP + 1;
  __shared__ double sg[64 * LD];
  if (ctl.lp && !ctl.first_stage && ctl.lp->s[ctl.par].active == 0) return;
  const int lane = threadIdx.x & 63;
  const int v0 = (int)(threadIdx.x >> 6) * FG;
  const int i = sl * 64 + lane;
  const int nb = min(64, m.nn - sl * 64);  // nodes of this slice
  if (lane < nb && v0 < NR) {
    const long long o0 = m.ng_off[sl];
    const int w = (int)((m.ng_off[sl + 1] - o0) >> 6);
    double acc[FG][ND], wi[FG];
#pragma unroll
    for (int f = 0; f < FG; ++f) {
      wi[f] = 0.0;
      if (v0 + f < NR) wi[f] = WSR ? WS[(size_t)i * ldws + v0 + f] : W[(size_t)(v0 + f) * m.nn + i];
#pragma unroll
      for (int d = 0; d < ND; ++d) acc[f][d] = 0.0;
    }
#pragma unroll 2
    for (int k = 0; k < w; ++k) {
      const long long q = o0 + (long long)k * 64 + lane;
      const int j = m.ng_nbr[q];
      double c[ND];
#pragma unroll
      for (int d = 0; d < ND; ++d) c[d] = m.ng_c[(size_t)d * m.ng_total + q];
#pragma unroll
      for (int f = 0; f < FG; ++f) {
        if (v0 + f < NR) {
          const double dw = (WSR ? WS[(size_t)j * ldws + v0 + f] : W[(size_t)(v0 + f) * m.nn + j]) - wi[f];
#pragma unroll
          for (int d = 0; d < ND; ++d) acc[f][d] += dw * c[d];
        }
      }
    }
    const double coef = -m.inv_vol[i] / double(ND * m.nv);
#pragma unroll
    for (int f = 0; f < FG; ++f)
      if (v0 + f < NR)
#pragma unroll
        for (int d = 0; d < ND; ++d) sg[lane * LD + (v0 + f) * ND + d] = coef * acc[f][d];
  }
  __syncthreads();
  GT* out = G + (size_t)sl * 64 * NCP;
  for (int idx = threadIdx.x; idx < nb * NCP; idx += blockDim.x) {
    const int l = idx / NCP, c = idx - l * NCP;
    out[idx] = GT(c < NC ? sg[l * LD + c] : 0.0);  // (the padding component of an odd row: 0)
  }
}

template <int ND, int NR, bool WSR = false, typename GT = double>
__global__ void __launch_bounds__(64 * kGradNodeGroups) k_grad_node(DevMesh m, const double* __restrict__ W,
                                                   const double* __restrict__ WS, int ldws,
                                                   GT* __restrict__ G, GradCtl ctl) {
  // in the first stage of a step, block 0 reduces the time-step candidates
  // and commits (the slices take the other blocks)
  const int lead = ctl.lp && ctl.first_stage ? 1 : 0;
  if (lead && blockIdx.x == 0) {
    step_start(ctl.lp, ctl.par);
    return;
  }
  const int sl = xcd_tile_of((int)blockIdx.x - lead, m.ng_nslices);
  if (sl >= m.ng_nslices) return;
  grad_node_body<ND, NR, WSR, GT>(m, W, WS, ldws, G, ctl, sl);
}

// ---------------------------------------------------------------------------
// node finish: boundary closure + RK stage update (or residual output) + dt
// candidate of the new state
// ---------------------------------------------------------------------------

struct Finish {
  const double* Win;    // stage input W (closure)
  const double* Un;     // U^n rows
  double* Wout;         // stage output (may alias Win: each node is written by one thread)
  double* rout;         // residual output (residual_only)
  const double* G;      // gradients of complete nodes (drift-diffusion closure)
  const double* PG;     // gradient partials of shared nodes
  const double* E;      // field (drift-diffusion)
  DevScalars* sc;       // state of the running step; null: residual only
  int* found;           // failures raised by this step
  long long* cand;      // candidate slots of this step's new state
  DevLoop* roll;        // fused passes: the shared-node pass of the first stage rolls the
  int roll_par;         //   candidate slots over (step_rollover) for this parity
  int gfull;            // G holds the gradients of shared nodes too (fused passes with a
                        // closure, the node-gradient passes, the drift-diffusion flux
                        // pass after the shared-node completion)
  int gnode;            // drift-diffusion: G is node-major (rows of node_row(NSP * ND))
  int g32;              // multi-species FP32 path: G holds FP32 values
  DtCoef dc;
  MixParams mix;        // Navier-Stokes species data
  double alpha;
  int closure, final_stage, residual_only;
  const double* cbuf;   // second closure option: [nb][NVAR] closure fluxes of the stage input
  // multi-species: node-major rows ([nn][ldws], the first nws used) of the
  // stage input and output; the primitives and transport data of a node
  // are kept there only (the component-major buffers hold U and p)
  const double* WSin;
  double* WSout;
  int nws, ldws;
};

// Node inputs of the stage update, loaded ahead of the residual sums where
// registers allow: U^n, alpha dt / V_i, the node's dx_min and its field.
template <int NVAR, int ND>
struct NodeIn {
  double Un[NVAR];
  double fac;
  double dx;
  double E[ND];
};

template <int ND, int MODEL, int NVAR>
__device__ inline void node_in_load(const DevMesh& m, const Finish& f, double dt, int i,
                                    NodeIn<NVAR, ND>& ni) {
  if (f.residual_only) return;
#pragma unroll
  for (int v = 0; v < NVAR; ++v) ni.Un[v] = f.Un[(size_t)v * m.nn + i];
  ni.fac = f.alpha * dt * m.inv_vupd[i];
  ni.dx = m.dxmin[i];
  if constexpr (MODEL == 1) {
#pragma unroll
    for (int d = 0; d < ND; ++d) ni.E[d] = f.E[(size_t)d * m.nn + i];
  }
}

// Update inputs staged in LDS by a tile pass, by slot (null members: read
// from global memory).
struct NodeLds {
  const double* un;  // [NVAR][ldu] U^n rows
  int ldu;
  const double* iv;  // [maxn] 1/V
  const double* dx;  // [maxn] dx_min
  const double* e;   // [ND][lde] field (drift-diffusion)
  int lde;
};

template <int ND, int MODEL, int NVAR>
__device__ inline void node_in_lds(const DevMesh& m, const Finish& f, double dt, int i, int q,
                                   const NodeLds& nl, NodeIn<NVAR, ND>& ni) {
  if (f.residual_only) return;
#pragma unroll
  for (int v = 0; v < NVAR; ++v) ni.Un[v] = nl.un ? nl.un[v * nl.ldu + q] : f.Un[(size_t)v * m.nn + i];
  ni.fac = f.alpha * dt * (nl.iv ? nl.iv[q] : m.inv_vupd[i]);
  ni.dx = nl.dx ? nl.dx[q] : m.dxmin[i];
  if constexpr (MODEL == 1) {
#pragma unroll
    for (int d = 0; d < ND; ++d) ni.E[d] = nl.e ? nl.e[d * nl.lde + q] : f.E[(size_t)d * m.nn + i];
  }
}

// Node flux F(node k) . S of the boundary closure: the Euler flux of the
// stage state (inviscid part for Navier-Stokes), or the drift plus diffusive
// flux u_k V_k . S - D grad u_k . S for drift-diffusion.
template <int ND, int NSP, int MODEL, int NVAR>
__device__ inline void closure_flux(const DevMesh& m, const Finish& f, int k, bool shared, const double (&S)[ND],
                                    double (&F)[NVAR]) {
  if constexpr (MODEL != 1) {
    double Wk[NVAR + 1];
#pragma unroll
    for (int v = 0; v <= NVAR; ++v) Wk[v] = f.Win[(size_t)v * m.nn + k];
    double q = 0.0;
#pragma unroll
    for (int d = 0; d < ND; ++d) q += Wk[1 + d] * S[d];
    q /= Wk[0];
    const double p = Wk[NVAR];
    F[0] = Wk[0] * q;
#pragma unroll
    for (int d = 0; d < ND; ++d) F[1 + d] = Wk[1 + d] * q + p * S[d];
    F[1 + ND] = (Wk[1 + ND] + p) * q;
#pragma unroll
    for (int s = 0; s < NSP; ++s) F[2 + ND + s] = Wk[2 + ND + s] * q;
  } else {
    double gr[NSP * ND];
    if (f.gnode) {
#pragma unroll
      for (int j = 0; j < NSP * ND; ++j) gr[j] = f.G[(size_t)k * node_row(NSP * ND) + j];
    } else if (shared && !f.gfull) {
      shared_gradient<NSP * ND, ND>(m, f.PG, k, make_int2(m.node_slot[k], m.node_slot[k + 1]), gr);
    } else {
#pragma unroll
      for (int j = 0; j < NSP * ND; ++j) gr[j] = f.G[(size_t)j * m.nn + k];
    }
#pragma unroll
    for (int s = 0; s < NVAR; ++s) {
      double vb = 0.0, gb = 0.0;
#pragma unroll
      for (int d = 0; d < ND; ++d) {
        vb += f.dc.zmu[s] * f.E[(size_t)d * m.nn + k] * S[d];
        gb += gr[s * ND + d] * S[d];
      }
      F[s] = f.Win[(size_t)s * m.nn + k] * vb - f.dc.D[s] * gb;
    }
  }
}

// Axisymmetric multi-species: the hoop stress tau_theta_theta of node i,
// 2 eta u_r/r + lambda (u_r/r + du_r/dr + du_x/dx) with lambda = -2/3 eta
// (Stokes), u_r/r taking its limit du_r/dr on the axis.  The two velocity
// derivatives come from the node's (node-major) gradient row, u_r and eta
// from its staged row.
template <int ND, int NSP>
__device__ inline double ns_hoop_stress(const DevMesh& m, const Finish& f, int i) {
  constexpr int NVAR = 2 + ND + NSP, NR = NVAR + 1, NP = ND + 1 + NSP, NCP = node_row((NR + NP) * ND);
  constexpr int CR = (NR + 1) * ND + 1, CX = NR * ND;  // du_r/dr, du_x/dx
  const float* G32 = reinterpret_cast<const float*>(f.G);
  const double durdr = f.g32 ? double(G32[(size_t)i * NCP + CR]) : f.G[(size_t)i * NCP + CR];
  const double duxdx = f.g32 ? double(G32[(size_t)i * NCP + CX]) : f.G[(size_t)i * NCP + CX];
  const double* row = f.WSin + (size_t)i * f.ldws;
  const double eta = row[NR + NP + 1], ur = row[NR + 1];  // aux[1], prim[1]
  const double rr = m.x[(size_t)m.nn + i];
  const double hoop = rr > 0.0 ? ur / rr : durdr;
  return 2.0 * eta * hoop - 2.0 / 3.0 * eta * (hoop + durdr + duxdx);
}

// Node-major staged row of a multi-species node: its first nws state rows
// (conserved, p, primitives, then the transport/thermo rows) contiguous.
// The row starts 16-byte aligned (an even stride): it is written in pairs.
template <int ND, int NSP>
__device__ inline void ns_store_node_row32(float* row, const double (&u)[2 + ND + NSP], double p,
                                           const double (&prim)[ND + 1 + NSP], const double (&aux)[3 + 2 * NSP]) {
  constexpr int NVAR = 2 + ND + NSP, NP = ND + 1 + NSP, NA = 3 + 2 * NSP, NT = NVAR + 1 + NP + NA;
  constexpr int L = ns_row32(NT);
  float r[L];
#pragma unroll
  for (int v = 0; v < NVAR; ++v) r[v] = float(u[v]);
  r[NVAR] = float(p);
#pragma unroll
  for (int q = 0; q < NP; ++q) r[NVAR + 1 + q] = float(prim[q]);
#pragma unroll
  for (int q = 0; q < NA; ++q) r[NVAR + 1 + NP + q] = float(aux[q]);
#pragma unroll
  for (int c = NT; c < L; ++c) r[c] = 0.0f;
  float4* r4 = reinterpret_cast<float4*>(row);
#pragma unroll
  for (int c = 0; c < L; c += 4) r4[c / 4] = make_float4(r[c], r[c + 1], r[c + 2], r[c + 3]);
}

template <int ND, int NSP>
__device__ inline void ns_store_node_row(double* row, int nws, const double (&u)[2 + ND + NSP], double p,
                                         const double (&prim)[ND + 1 + NSP], const double (&aux)[3 + 2 * NSP]) {
  constexpr int NVAR = 2 + ND + NSP, NP = ND + 1 + NSP, NA = 3 + 2 * NSP, NT = NVAR + 1 + NP + NA;
  double r[NT + 1];
#pragma unroll
  for (int v = 0; v < NVAR; ++v) r[v] = u[v];
  r[NVAR] = p;
#pragma unroll
  for (int q = 0; q < NP; ++q) r[NVAR + 1 + q] = prim[q];
#pragma unroll
  for (int q = 0; q < NA; ++q) r[NVAR + 1 + NP + q] = aux[q];
  r[NT] = 0.0;
  double2* r2 = reinterpret_cast<double2*>(row);
#pragma unroll
  for (int c = 0; c < NT; c += 2)
    if (c < nws) r2[c / 2] = make_double2(r[c], r[c + 1]);  // (an odd nws also fills the row's padding)
}

template <int ND, int NSP, int MODEL, int NVAR>
__device__ inline double finish_node(const DevMesh& m, const Finish& f, int i, bool shared,
                                     double (&r)[NVAR], const NodeIn<NVAR, ND>& ni) {
  if (f.closure && m.nb > 0) {
    const int bi = m.bnd_index[i];
    if (bi >= 0) {
      if (ND == 2 && f.closure == 2) {
        // second option: computed from the stage input before the flux pass
        // (it reads neighbours, which the pass may overwrite in place)
#pragma unroll
        for (int v = 0; v < NVAR; ++v) r[v] += f.cbuf[(size_t)bi * NVAR + v];
      } else {
        // first option: the node flux through S_i^b
        double Sb[ND], F[NVAR];
#pragma unroll
        for (int d = 0; d < ND; ++d) Sb[d] = m.bnd_S[(size_t)d * m.nb + bi];
        closure_flux<ND, NSP, MODEL, NVAR>(m, f, i, shared, Sb, F);
#pragma unroll
        for (int v = 0; v < NVAR; ++v) r[v] += F[v];
      }
    }
  }
  bool on_axis = false;
  if constexpr ((MODEL == 0 || MODEL == 2) && ND == 2) {
    if (m.axi) {
      // axisymmetric gas: geometric source + p of the radial momentum over
      // the plane dual area (in the residual: - p_i A_i); the radial
      // velocity is set to zero on the axis after it
      r[2] -= f.Win[(size_t)NVAR * m.nn + i] * m.vnode[i];
      // multi-species: its diffusive part, minus the hoop stress
      if constexpr (MODEL == 2) r[2] += ns_hoop_stress<ND, NSP>(m, f, i) * m.vnode[i];
      on_axis = m.x[(size_t)m.nn + i] == 0.0;
    }
  }
  if (f.residual_only) {
#pragma unroll
    for (int v = 0; v < NVAR; ++v) f.rout[(size_t)v * m.nn + i] = r[v];
    return INFINITY;
  }
  double u[NVAR];
#pragma unroll
  for (int v = 0; v < NVAR; ++v) u[v] = ni.Un[v] - ni.fac * r[v];
  if constexpr ((MODEL == 0 || MODEL == 2) && ND == 2) {
    if (on_axis) u[2] = 0.0;
  }
#pragma unroll
  for (int v = 0; v < NVAR; ++v) f.Wout[(size_t)v * m.nn + i] = u[v];
  bool ok = true;
  double p = 0.0;
  if constexpr (MODEL == 0) {
    double ke = 0.0;
#pragma unroll
    for (int d = 0; d < ND; ++d) ke += u[1 + d] * u[1 + d];
    p = (f.dc.gamma - 1.0) * (u[1 + ND] - 0.5 * ke / u[0]);
    f.Wout[(size_t)NVAR * m.nn + i] = p;
    ok = u[0] > 0.0 && p > 0.0;
  }
  if constexpr (MODEL == 2) {
    // node aux of the new state: temperature, pressure, primitives, transport
    constexpr int NP = ND + 1 + NSP, NA = 3 + 2 * NSP;
    double prim[NP], aux[NA];
    ok = ns_node_state<ND, NSP>(f.mix, u, p, prim, aux);
    f.Wout[(size_t)NVAR * m.nn + i] = p;
    ns_store_node_row<ND, NSP>(f.WSout + (size_t)i * f.ldws, f.nws, u, p, prim, aux);
    if (f.g32)
      ns_store_node_row32<ND, NSP>(reinterpret_cast<float*>(f.WSout + (size_t)m.nn * f.ldws) +
                                       (size_t)i * ns_row32(ns_staged_rows(ND, NSP, false)),
                                   u, p, prim, aux);
#pragma unroll
    for (int v = 0; v < NVAR; ++v) ok = ok && isfinite(u[v]);
    if (!f.final_stage) return INFINITY;
    if (!ok) atomicOr(f.found, 1);
    return ns_node_dt<ND, NSP>(ni.dx, f.dc, f.mix, u[0], prim, p, aux, ok);
  }
#pragma unroll
  for (int v = 0; v < NVAR; ++v) ok = ok && isfinite(u[v]);
  if (!f.final_stage) return INFINITY;
  if (!ok) atomicOr(f.found, 1);
  return node_dt<ND, NSP, MODEL>(f.dc, ni.dx, ni.E, u, p);
}

// ---------------------------------------------------------------------------
// gas flux pass
// ---------------------------------------------------------------------------

struct GasParams {
  double gamma, beta, entropy_fix;
  int limiter;
  double dt_host;  // time step of the MUSCL-Hancock predictor outside the time loop
};

// ---------------------------------------------------------------------------
// drift-diffusion parameters (limited Lax-Wendroff + central diffusion)
// ---------------------------------------------------------------------------

struct DDParams {
  double zmu[4];   // z * mu per species
  double D[4];
  double beta;
  double dt_host;  // residual only
  int limiter;
};

// LDS strides of the arrays read by the cell flux loops: coordinates (ldx),
// reconstructed rows (ldw), gradients and field (ldg), cell accumulators (ldc)
struct CellLd {
  int ldx, ldw, ldg, ldc;
};

// Threads per cell of the gas and drift-diffusion flux passes: 2 for FP64
// tetrahedra (each takes three of the six edges), else 1.
template <int ND, typename CT>
__host__ __device__ constexpr int cell_halves() {
  return ND == 3 && sizeof(CT) == sizeof(double) ? 2 : 1;
}

// Gas fluxes of the tile's cells: MUSCL with virtual upwind nodes, slope
// limiter, HLLC or Roe; accumulated per cell vertex into sR.
// With HANCOCK, sH holds each slot's MUSCL-Hancock half-step increments
// (rows like sW), added to the face states of both ends.
template <int ND, int NSP, int FLUX, typename CT, int NV, bool AXI = false, bool HANCOCK = false>
__device__ inline void gas_cell_fluxes(const DevMesh& m, const TilePre<NV>& tp, const double* sX,
                                       const CT* sW, const CT* sG, double* sR, CellLd L,
                                       const GasParams& gp, const CT* sH = nullptr) {
  using SH = Shape<ND, NV>;
  constexpr int NVAR = 2 + ND + NSP, NR = NVAR + 1, NE = SH::E::NE;
  const CT gamma = CT(gp.gamma), beta = CT(gp.beta), fix = CT(gp.entropy_fix);
  // FP64 tetrahedra: two threads per cell, edges 0-2 and 3-5, each into its
  // own plane of vertex parts (sR and sR + NV*NVAR*ldc), which the node pass
  // adds: half the registers of a cell's six Riemann problems, so two
  // wavefronts per SIMD instead of one
  constexpr int NH = cell_halves<ND, CT>(), EH = NE / NH;
  const int ncp = NH == 1 ? tp.nc : (tp.nc + 63) / 64 * 64;
  for (int task = threadIdx.x; task < NH * ncp; task += blockDim.x) {
    int h = 0, lc = task;
    if constexpr (NH == 2) {
      h = __builtin_amdgcn_readfirstlane(task / ncp);
      lc = task - h * ncp;
      if (lc >= tp.nc) continue;
    }
    int l[NV];
    uint32_t sh;
    if constexpr (NH == 1) {
      cell_topo<NV>(m, tp, lc, l, sh);
    } else {
#pragma unroll
      for (int k = 0; k < NV; ++k) l[k] = m.lconn[(size_t)k * m.nc + tp.c0 + lc];
      sh = m.shift[tp.c0 + lc];
    }
    double e[NV - 1][ND], Sd[NV][ND];
    cell_rel_coords<ND, NV>(m, sX, L.ldx, l, sh, e);
    SH::normals(e, Sd);
    double acc[NV][NVAR];
#pragma unroll
    for (int k = 0; k < NV; ++k)
#pragma unroll
      for (int v = 0; v < NVAR; ++v) acc[k][v] = 0.0;
#pragma unroll
    for (int ed0 = 0; ed0 < NE; ++ed0) {
      if (NH == 2 && (ed0 / EH) != h) continue;
      const int ed = ed0;
      const int a = SH::E::a(ed), b = SH::E::b(ed);
      const int la = l[a], lb = l[b];
      CT S[ND], dx[ND];
#pragma unroll
      for (int d = 0; d < ND; ++d) {
        S[d] = CT((Sd[a][d] - Sd[b][d]) * SH::kdual);
        dx[d] = CT((a == 0 ? 0.0 : -e[a - 1][d]) + (b == 0 ? 0.0 : e[b - 1][d]));
      }
      CT WL[NR], WR[NR];
#pragma unroll
      for (int v = 0; v < NR; ++v) {
        const CT wi = sW[v * L.ldw + la], wj = sW[v * L.ldw + lb];
        CT gi = CT(0), gj = CT(0);
#pragma unroll
        for (int d = 0; d < ND; ++d) {
          gi += sG[(v * ND + d) * L.ldg + la] * dx[d];
          gj += sG[(v * ND + d) * L.ldg + lb] * dx[d];
        }
        const CT delta = wj - wi;
        // virtual upwind nodes l (behind i) and k (ahead of j)
        const CT dli = CT(2) * gi - delta, djk = CT(2) * gj - delta;
        WL[v] = wi + CT(0.5) * slope_limit<CT>(gp.limiter, beta, dli, delta);
        WR[v] = wj - CT(0.5) * slope_limit<CT>(gp.limiter, beta, delta, djk);
        if constexpr (HANCOCK) {
          WL[v] += sH[v * L.ldw + la];
          WR[v] += sH[v * L.ldw + lb];
        }
      }
      CT F[NVAR];
      if constexpr (FLUX == 0)
        hllc_flux<ND, NSP, CT>(WL, WR, S, gamma, gamma, F);
      else
        roe_flux<ND, NSP, CT>(WL, WR, S, gamma, fix, F);
      // axisymmetric (x, r): centroid radius of the edge's dual face piece
      double rw = 1.0;
      if constexpr (AXI) {
        static_assert(ND == 2, "axisymmetric meshes are (x, r) planes");
        double rr[NV], rc = 0.0;
#pragma unroll
        for (int k = 0; k < NV; ++k) rr[k] = sX[L.ldx + l[k]];
#pragma unroll
        for (int k = 0; k < NV; ++k) rc += rr[k];
        rc /= double(NV);
        rw = 0.5 * (0.5 * (rr[a] + rr[b]) + rc);
      }
#pragma unroll
      for (int v = 0; v < NVAR; ++v) {
        acc[a][v] += double(F[v]) * rw;
        acc[b][v] -= double(F[v]) * rw;
      }
    }
    double* sRh = sR + (size_t)h * NV * NVAR * L.ldc;
#pragma unroll
    for (int k = 0; k < NV; ++k)
#pragma unroll
      for (int v = 0; v < NVAR; ++v) sRh[(k * NVAR + v) * L.ldc + lc] = acc[k][v];
  }
}

// Second boundary-closure option (Sec. "Boundary conditions in AVIP", 2D):
// each half boundary edge carries the interpolated flux 0.75 F_i + 0.25 F_j;
// per boundary node, the sum over its half edges, in ascending order of the
// other end.  Runs after the gradient pass and before the flux pass of a
// stage.
template <int ND, int NSP, int MODEL>
__global__ void __launch_bounds__(256) k_closure2(DevMesh m, Finish f, double* __restrict__ cbuf) {
  constexpr int NVAR = MODEL == 1 ? NSP : 2 + ND + NSP;
  if (step_inactive(f.sc)) return;
  const int bi = blockIdx.x * blockDim.x + threadIdx.x;
  if (bi >= m.nb) return;
  const int i = m.bnd_node[bi];
  const bool shared_i = m.node_slot[i + 1] - m.node_slot[i] > 1;
  double c[NVAR];
#pragma unroll
  for (int v = 0; v < NVAR; ++v) c[v] = 0.0;
  for (int e = m.bedge_ptr[bi]; e < m.bedge_ptr[bi + 1]; ++e) {
    const int j = m.bedge_nb[e];
    double S[ND], Fi[NVAR], Fj[NVAR];
#pragma unroll
    for (int d = 0; d < ND; ++d) S[d] = m.bedge_S[(size_t)d * m.nbe + e];
    closure_flux<ND, NSP, MODEL, NVAR>(m, f, i, shared_i, S, Fi);
    closure_flux<ND, NSP, MODEL, NVAR>(m, f, j, m.node_slot[j + 1] - m.node_slot[j] > 1, S, Fj);
#pragma unroll
    for (int v = 0; v < NVAR; ++v) c[v] += 0.75 * Fi[v] + 0.25 * Fj[v];
  }
#pragma unroll
  for (int v = 0; v < NVAR; ++v) cbuf[(size_t)bi * NVAR + v] = c[v];
}

// Drift-diffusion fluxes of the tile's cells: limited Lax-Wendroff
// convective flux (upwind node w, downwind node m, virtual node upwind of w)
// plus central diffusion; accumulated per cell vertex into sR.
// Bernoulli function B(x) = x / (e^x - 1), B(0) = 1
template <typename T>
__device__ inline T bernoulli(T x) {
  if constexpr (sizeof(T) == sizeof(double))
    return x == T(0) ? T(1) : x / expm1(x);
  else
    return x == T(0) ? T(1) : x / expm1f(x);
}

// Scharfetter-Gummel flux of one species through the cell-edge vector S of
// the edge a -> b (dx = x_b - x_a): with S_par = c dx, c = S.dx / |dx|^2,
// exponential fitting along the edge, c D (B(-al) u_a - B(al) u_b) with
// al = V.dx / D (upwinding when D = 0), and the central flux
// (V u_bar - D g_bar) . (S - S_par) across it.  vS = V.S, gS = g_bar.S.
template <int ND, typename CT>
__device__ inline CT sg_edge_flux(CT ua, CT ub, const CT (&V)[ND], const CT (&S)[ND], const CT (&dx)[ND],
                                  CT D, const CT (&gbar)[ND], CT vS, CT gS) {
  CT h2 = CT(0), sdx = CT(0), vdx = CT(0), gdx = CT(0);
#pragma unroll
  for (int d = 0; d < ND; ++d) {
    h2 += dx[d] * dx[d];
    sdx += S[d] * dx[d];
    vdx += V[d] * dx[d];
    gdx += gbar[d] * dx[d];
  }
  const CT c = sdx / h2;
  CT fpar;
  if (D > CT(0)) {
    const CT al = vdx / D;
    fpar = c * D * (bernoulli<CT>(-al) * ua - bernoulli<CT>(al) * ub);
  } else {
    fpar = c * vdx * (vdx >= CT(0) ? ua : ub);
  }
  return fpar + CT(0.5) * (ua + ub) * (vS - c * vdx) - D * (gS - c * gdx);
}

// SG: the Scharfetter-Gummel flux instead of limited Lax-Wendroff with the
// central diffusive flux.
template <int ND, int NS, typename CT, int NV, bool AXI = false, bool SG = false>
__device__ inline void dd_cell_fluxes(const DevMesh& m, const TilePre<NV>& tp, const double* sX,
                                      const CT* sU, const CT* sG, const CT* sE, double* sR, CellLd L,
                                      CT dt, const DDParams& pp) {
  using SH = Shape<ND, NV>;
  constexpr int NE = SH::E::NE;
  static_assert(!AXI || ND == 2, "axisymmetric meshes are (x, r) planes");
  const CT beta = CT(pp.beta);
  // FP64 tetrahedra: two threads per cell, three edges each, into two
  // planes of vertex parts (as the gas pass)
  constexpr int NH = cell_halves<ND, CT>(), EH = NE / NH;
  const int ncp = NH == 1 ? tp.nc : (tp.nc + 63) / 64 * 64;
  for (int task = threadIdx.x; task < NH * ncp; task += blockDim.x) {
    int h = 0, lc = task;
    if constexpr (NH == 2) {
      h = __builtin_amdgcn_readfirstlane(task / ncp);
      lc = task - h * ncp;
      if (lc >= tp.nc) continue;
    }
    int l[NV];
    uint32_t sh;
    if constexpr (NH == 1) {
      cell_topo<NV>(m, tp, lc, l, sh);
    } else {
#pragma unroll
      for (int k = 0; k < NV; ++k) l[k] = m.lconn[(size_t)k * m.nc + tp.c0 + lc];
      sh = m.shift[tp.c0 + lc];
    }
    double e[NV - 1][ND], Sd[NV][ND];
    cell_rel_coords<ND, NV>(m, sX, L.ldx, l, sh, e);
    SH::normals(e, Sd);
    double acc[NV][NS];
#pragma unroll
    for (int k = 0; k < NV; ++k)
#pragma unroll
      for (int s = 0; s < NS; ++s) acc[k][s] = 0.0;
#pragma unroll
    for (int ed = 0; ed < NE; ++ed) {
      if (NH == 2 && ed / EH != h) continue;
      const int a = SH::E::a(ed), b = SH::E::b(ed);
      const int la = l[a], lb = l[b];
      CT S[ND], dx[ND], Ebar[ND];
#pragma unroll
      for (int d = 0; d < ND; ++d) {
        S[d] = CT((Sd[a][d] - Sd[b][d]) * SH::kdual);
        dx[d] = CT((a == 0 ? 0.0 : -e[a - 1][d]) + (b == 0 ? 0.0 : e[b - 1][d]));
        Ebar[d] = CT(0.5) * (sE[d * L.ldg + la] + sE[d * L.ldg + lb]);
      }
      // axisymmetric (x, r): the dual face piece of the edge, from its
      // midpoint to the centroid, revolves at the mean of their radii (first
      // Pappus-Guldinus theorem; the radius is never periodic)
      double rw = 1.0;
      if constexpr (AXI) {
        double r[NV], rc = 0.0;
#pragma unroll
        for (int k = 0; k < NV; ++k) r[k] = sX[L.ldx + l[k]];
#pragma unroll
        for (int k = 0; k < NV; ++k) rc += r[k];
        rc /= double(NV);
        rw = 0.5 * (0.5 * (r[a] + r[b]) + rc);
      }
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        const CT zm = CT(pp.zmu[s]);
        CT v = CT(0), gV = CT(0), gS = CT(0), gA = CT(0), gB = CT(0);
#pragma unroll
        for (int d = 0; d < ND; ++d) {
          const CT Vd = zm * Ebar[d];
          const CT ga = sG[(s * ND + d) * L.ldg + la], gb = sG[(s * ND + d) * L.ldg + lb];
          const CT gbar = CT(0.5) * (ga + gb);
          v += Vd * S[d];
          gV += gbar * Vd;
          gS += gbar * S[d];
          gA += ga * dx[d];
          gB += gb * dx[d];
        }
        const CT ua = sU[s * L.ldw + la], ub = sU[s * L.ldw + lb];
        if constexpr (SG) {
          CT V[ND], gbar[ND];
#pragma unroll
          for (int d = 0; d < ND; ++d) {
            V[d] = zm * Ebar[d];
            gbar[d] = CT(0.5) * (sG[(s * ND + d) * L.ldg + la] + sG[(s * ND + d) * L.ldg + lb]);
          }
          const CT F = sg_edge_flux<ND, CT>(ua, ub, V, S, dx, CT(pp.D[s]), gbar, v, gS);
          acc[a][s] += double(F) * rw;
          acc[b][s] -= double(F) * rw;
          continue;
        }
        // upwind node w, downwind node m; the virtual node upwind of w
        const bool fwd = v >= CT(0);
        const CT uw = fwd ? ua : ub;
        const CT bb = fwd ? (ub - ua) : (ua - ub);
        const CT gw = fwd ? gA : -gB;
        const CT aa = CT(2) * gw - bb;
        const CT psi = psi_limit<CT>(pp.limiter, beta, aa, bb);
        const CT uf = uw + (CT(0.5) * bb - CT(0.5) * dt * gV) * psi;
        const CT F = uf * v - CT(pp.D[s]) * gS;
        acc[a][s] += double(F) * rw;
        acc[b][s] -= double(F) * rw;
      }
    }
    double* sRh = sR + (size_t)h * NV * NS * L.ldc;
#pragma unroll
    for (int k = 0; k < NV; ++k)
#pragma unroll
      for (int s = 0; s < NS; ++s) sRh[(k * NS + s) * L.ldc + lc] = acc[k][s];
  }
}

// Node pass of a tile: residual sums of each slot over its incidences in a
// fixed order; a tile-owned node is finished (stage update, time-step
// candidate), a shared node's partial is stored at its partial index.
// Returns this thread's smallest candidate.
// ALLPR: every slot writes its partial (update_all models)
template <int ND, int NSP, int MODEL, int NVAR, bool HALVES = false, bool ALLPR = false>
__device__ inline double tile_node_pass(const DevMesh& m, const Finish& f, double dt, double* PR, int ns,
                                        const int* sSl, int ldsl, const uint16_t* sInc, const double* sR,
                                        int ldc, const NodeLds& nl = NodeLds{}) {
  double cand = INFINITY;
  for (int q = threadIdx.x; q < ns; q += blockDim.x) {
    const SlotTopo st = slot_table_get(sSl, ldsl, q);
    // update inputs first: their loads overlap the sums
    NodeIn<NVAR, ND> nq;
    if (!ALLPR && st.sv >= 0) node_in_lds<ND, MODEL, NVAR>(m, f, dt, st.sv, q, nl, nq);
    double r[NVAR];
#pragma unroll
    for (int v = 0; v < NVAR; ++v) r[v] = 0.0;
    for (int p = st.p0; p < st.p1; ++p) {
      const int code = sInc[p];
      const int lc = code >> 2, k = code & 3;
      if constexpr (HALVES) {
        const double* sR1 = sR + (size_t)(ND + 1) * NVAR * ldc;
#pragma unroll
        for (int v = 0; v < NVAR; ++v) r[v] += sR[(k * NVAR + v) * ldc + lc] + sR1[(k * NVAR + v) * ldc + lc];
      } else {
#pragma unroll
        for (int v = 0; v < NVAR; ++v) r[v] += sR[(k * NVAR + v) * ldc + lc];
      }
    }
    if (!ALLPR && st.sv >= 0) {
      cand = fmin(cand, finish_node<ND, NSP, MODEL, NVAR>(m, f, st.sv, false, r, nq));
    } else {
#pragma unroll
      for (int v = 0; v < NVAR; ++v) PR[(size_t)st.pos * NVAR + v] = r[v];
    }
  }
  return cand;
}

template <int ND, int NSP, int FLUX, typename CT, bool AXI = false, bool HANCOCK = false, int NV = ND + 1>
__device__ inline void flux_gas_body(DevMesh m, const double* __restrict__ W,
                                                  const double* __restrict__ G,
                                                  double* __restrict__ PR, GasParams gp, Finish f,
                                                  int t, double* lds) {
  constexpr int NVAR = 2 + ND + NSP, NR = NVAR + 1;
  if (step_inactive(f.sc)) return;
  TilePre<NV> tp;
  tile_prefetch<NV>(m, t, tp);
  const int maxn = m.max_tile_nodes, maxc = m.max_tile_cells;
  constexpr int NH = cell_halves<ND, CT>();
  double* sX = lds;                       // [ND][maxn]
  double* sR = sX + ND * maxn;            // [NH][NV*NVAR][maxc]
  CT* sW = reinterpret_cast<CT*>(sR + NH * NV * NVAR * maxc);  // [NR][maxn]
  CT* sG = sW + NR * maxn;                // [NR*ND][maxn]
  CT* sH = sG + NR * ND * maxn;           // predictor: [NR][maxn] half-step increments
  int* sSl = reinterpret_cast<int*>(sH + (HANCOCK ? NR * maxn : 0));
  uint16_t* sInc = reinterpret_cast<uint16_t*>(sSl + 4 * maxn);
  const int ns = tp.ns;
  for (int q = threadIdx.x; q < ns; q += blockDim.x) {
    const SlotTopo st = slot_topo<NV>(m, tp, q);
    slot_table_put(sSl, maxn, q, st.sv, st.pos, st.p0, st.p1);
    const int sv = st.sv;
    const int g = slot_node_id(sv);
    double w[NR], xx[ND];
#pragma unroll
    for (int v = 0; v < NR; ++v) w[v] = W[(size_t)v * m.nn + g];
#pragma unroll
    for (int d = 0; d < ND; ++d) xx[d] = m.x[(size_t)d * m.nn + g];
    if constexpr (node_gradient(0, ND, NV))
      stage_gradient_row<node_row(NR * ND), 0, NR * ND, CT>(G, g, sG, maxn, q);
    else
      stage_gradient<NR * ND, ND, CT>(m, G, f.PG, sv, st.run, sG, maxn, q);
#pragma unroll
    for (int v = 0; v < NR; ++v) sW[v * maxn + q] = CT(w[v]);
#pragma unroll
    for (int d = 0; d < ND; ++d) sX[d * maxn + q] = xx[d];
  }
  tile_store_inc<NV>(m, tp, sInc);
  __syncthreads();
  const double dt = f.sc ? f.sc->dt : gp.dt_host;
  if constexpr (HANCOCK) {
    // each slot's half-step increments from its staged state and gradients
    for (int q = threadIdx.x; q < ns; q += blockDim.x)
      hancock_half_step<ND, NSP, CT>(sW, sG, maxn, q, CT(gp.gamma), CT(0.5 * dt), sH);
    __syncthreads();
  }
  gas_cell_fluxes<ND, NSP, FLUX, CT, NV, AXI, HANCOCK>(m, tp, sX, sW, sG, sR, CellLd{maxn, maxn, maxn, maxc},
                                                       gp, sH);
  __syncthreads();
  constexpr bool ALLPR = update_all(0, ND) && NV == ND + 1;
  const double cand =
      tile_node_pass<ND, NSP, 0, NVAR, (NH == 2), ALLPR>(m, f, dt, PR, ns, sSl, maxn, sInc, sR, maxc);
  if (f.final_stage && f.sc) {
    const double b = block_min(cand);
    if (threadIdx.x == 0) post_candidate(f.cand, t, b);
  }
}

template <int ND, int NSP, int FLUX, typename CT, bool AXI = false, bool HANCOCK = false, int NV = ND + 1>
__global__ void VCX_FLUX_BOUNDS k_flux_gas(DevMesh m, const double* __restrict__ W,
                                                  const double* __restrict__ G,
                                                  double* __restrict__ PR, GasParams gp, Finish f) {
  extern __shared__ double lds[];
  const int t = xcd_tile(m.ntiles);
  if (t >= m.ntiles) return;
  flux_gas_body<ND, NSP, FLUX, CT, AXI, HANCOCK, NV>(m, W, G, PR, gp, f, t, lds);
}

// ---------------------------------------------------------------------------
// drift-diffusion flux pass
// ---------------------------------------------------------------------------

template <int ND, int NS, typename CT, bool AXI = false, bool SG = false, int NV = ND + 1>
__device__ inline void flux_dd_body(DevMesh m, const double* __restrict__ U,
                                                 const double* __restrict__ G,
                                                 double* __restrict__ PR, DDParams pp, Finish f,
                                                 int t, double* lds) {
  if (step_inactive(f.sc)) return;
  TilePre<NV> tp;
  tile_prefetch<NV>(m, t, tp);
  const int maxn = m.max_tile_nodes, maxc = m.max_tile_cells;
  constexpr int NH = cell_halves<ND, CT>();
  double* sX = lds;                      // [ND][maxn]
  double* sR = sX + ND * maxn;           // [NH][NV*NS][maxc]
  CT* sU = reinterpret_cast<CT*>(sR + NH * NV * NS * maxc);  // [NS][maxn]
  CT* sG = sU + NS * maxn;               // [NS*ND][maxn]
  CT* sE = sG + NS * ND * maxn;          // [ND][maxn]
  int* sSl = reinterpret_cast<int*>(sE + ND * maxn);
  uint16_t* sInc = reinterpret_cast<uint16_t*>(sSl + 4 * maxn);
  const double* E = f.E;
  const int ns = tp.ns;
  for (int q = threadIdx.x; q < ns; q += blockDim.x) {
    const SlotTopo st = slot_topo<NV>(m, tp, q);
    slot_table_put(sSl, maxn, q, st.sv, st.pos, st.p0, st.p1);
    const int sv = st.sv;
    const int g = slot_node_id(sv);
    double u[NS], xe[2 * ND];
#pragma unroll
    for (int s = 0; s < NS; ++s) u[s] = U[(size_t)s * m.nn + g];
#pragma unroll
    for (int d = 0; d < ND; ++d) {
      xe[d] = m.x[(size_t)d * m.nn + g];
      xe[ND + d] = E[(size_t)d * m.nn + g];
    }
    if (f.gnode)
      stage_gradient_row<node_row(NS * ND), 0, NS * ND, CT>(G, g, sG, maxn, q);
    else
      stage_gradient<NS * ND, ND, CT>(m, G, f.PG, f.gfull ? g : sv, st.run, sG, maxn, q);
#pragma unroll
    for (int s = 0; s < NS; ++s) sU[s * maxn + q] = CT(u[s]);
#pragma unroll
    for (int d = 0; d < ND; ++d) {
      sX[d * maxn + q] = xe[d];
      sE[d * maxn + q] = CT(xe[ND + d]);
    }
  }
  tile_store_inc<NV>(m, tp, sInc);
  __syncthreads();
  const double dt = f.sc ? f.sc->dt : pp.dt_host;
  dd_cell_fluxes<ND, NS, CT, NV, AXI, SG>(m, tp, sX, sU, sG, sE, sR, CellLd{maxn, maxn, maxn, maxc}, CT(dt), pp);
  __syncthreads();
  const double cand = tile_node_pass<ND, NS, 1, NS, (NH == 2)>(m, f, dt, PR, ns, sSl, maxn, sInc, sR, maxc);
  if (f.final_stage && f.sc) {
    const double b = block_min(cand);
    if (threadIdx.x == 0) post_candidate(f.cand, t, b);
  }
}

template <int ND, int NS, typename CT, bool AXI = false, bool SG = false, int NV = ND + 1>
__global__ void VCX_FLUX_BOUNDS k_flux_dd(DevMesh m, const double* __restrict__ U,
                                                 const double* __restrict__ G,
                                                 double* __restrict__ PR, DDParams pp, Finish f) {
  extern __shared__ double lds[];
  const int t = xcd_tile(m.ntiles);
  if (t >= m.ntiles) return;
  flux_dd_body<ND, NS, CT, AXI, SG, NV>(m, U, G, PR, pp, f, t, lds);
}

// ---------------------------------------------------------------------------
// fused gradient + flux pass over extended tiles (2D meshes): the tile's
// slots and halo nodes are staged, the gradient contributions of the tile's
// cells and halo cells are formed, every slot node's gradient is summed over
// all its cells in ascending cell order (so every tile forms the same sum for
// a shared node), and the flux and node passes follow in the same launch.
// In the first stage of a step every block decides the step itself from the
// previous parity's state; the block of tile 0 stores the decision.
// ---------------------------------------------------------------------------

struct FusedCtl {
  DevLoop* lp;     // null outside the time loop
  int par;         // parity of the step
  int first_stage;
  double* Gout;    // gradients of the slot nodes (drift-diffusion boundary closure) or null
};

template <int MODEL, int NSP, int ND>
struct FusedDims {
  static constexpr int NVAR = MODEL == 1 ? NSP : 2 + ND + NSP;
  static constexpr int NGF = MODEL == 1 ? NSP : NVAR + 1;  // rows with gradients
  static constexpr int NC = NGF * ND;
};

// LDS bytes of the fused pass
template <int ND, int NSP, int MODEL, typename CT>
__host__ __device__ inline size_t fused_lds_bytes(int maxn, int maxc, int maxne, int maxce, int maxgi) {
  using D = FusedDims<MODEL, NSP, ND>;
  constexpr int NV = ND + 1;
  const size_t cr = (size_t)D::NC * maxce > (size_t)NV * D::NVAR * maxc ? (size_t)D::NC * maxce
                                                                         : (size_t)NV * D::NVAR * maxc;
  size_t b = sizeof(double) * ((size_t)ND * maxne + (size_t)D::NGF * maxne + cr);
  b += sizeof(CT) * ((size_t)D::NC * maxn + (sizeof(CT) == sizeof(double) ? 0 : (size_t)D::NGF * maxn) +
                     (MODEL == 1 ? (size_t)ND * maxn : 0));
  b = (b + 7) / 8 * 8;
  b += slot_lds_bytes(maxn) + inc_lds_bytes(NV, maxc) + ((size_t)maxgi * sizeof(uint16_t) + 7) / 8 * 8;
  return b;
}

// Stage n 16-bit values to LDS: up to K per thread loaded before any store.
template <int K>
__device__ inline void stage_u16(const uint16_t* __restrict__ src, int n, uint16_t* dst) {
  uint16_t v[K];
#pragma unroll
  for (int j = 0; j < K; ++j) {
    const int p = (int)threadIdx.x + j * (int)blockDim.x;
    if (p < n) v[j] = src[p];
  }
#pragma unroll
  for (int j = 0; j < K; ++j) {
    const int p = (int)threadIdx.x + j * (int)blockDim.x;
    if (p < n) dst[p] = v[j];
  }
  for (int p = (int)threadIdx.x + K * (int)blockDim.x; p < n; p += blockDim.x) dst[p] = src[p];
}

template <int ND, int NSP, int MODEL, int FLUX, typename CT>
__device__ inline void fused_body(DevMesh m, const double* __restrict__ W, double* __restrict__ PR,
                                  GasParams gp, DDParams pp, Finish f, FusedCtl fc, int t, double* lds) {
  using D = FusedDims<MODEL, NSP, ND>;
  constexpr int NV = ND + 1, NVAR = D::NVAR, NGF = D::NGF, NC = D::NC;
  constexpr bool WCOPY = sizeof(CT) != sizeof(double);
  // the step: decided here in its first stage (after the staging, which
  // does not depend on it), read from its state in later stages
  __shared__ double s_dt;
  __shared__ int s_act;
  const bool loop = fc.lp != nullptr;
  const bool decide = loop && fc.first_stage;
  if (loop && !decide && fc.lp->s[fc.par].active == 0) return;
  double ck = INFINITY;  // this thread's candidate slot of the previous state
  if (decide && threadIdx.x < kCandSlots) {
    const long long* slots = fc.lp->s[fc.par ^ 1].dt_src ? fc.lp->cand[fc.par ^ 1] : fc.lp->cnode;
    ck = key_cand(slots[threadIdx.x]);
  }
  // (the step size is read from LDS where it is used, not held in registers)

  TilePre<NV> tp;
  tile_prefetch<NV>(m, t, tp);
  const int hc0 = m.tile_hcell[t], nhc = m.tile_hcell[t + 1] - hc0;
  const int hn0 = m.tile_hnode[t], nhn = m.tile_hnode[t + 1] - hn0;
  const int gb = m.tile_ginc[t], ngi = m.tile_ginc[t + 1] - gb;
  const int nc = tp.nc, ns = tp.ns, nce = nc + nhc;
  const int maxn = m.max_tile_nodes, maxc = m.max_tile_cells;
  const int maxne = m.max_ext_nodes, maxce = m.max_ext_cells;
  double* sX = lds;                                  // [ND][maxne]
  double* sWd = sX + ND * maxne;                     // [NGF][maxne]
  double* sCR = sWd + NGF * maxne;                   // gradient parts [NC][maxce], then residual parts
  const size_t ncr = (size_t)NC * maxce > (size_t)NV * NVAR * maxc ? (size_t)NC * maxce : (size_t)NV * NVAR * maxc;
  CT* sG = reinterpret_cast<CT*>(sCR + ncr);         // [NC][maxn]
  CT* sWc = sG + NC * maxn;                          // [NGF][maxn] when CT is not double
  CT* sE = sWc + (WCOPY ? NGF * maxn : 0);           // [ND][maxn] drift-diffusion field
  size_t off = (size_t)(sE + (MODEL == 1 ? ND * maxn : 0)) - (size_t)lds;
  off = (off + 7) / 8 * 8;
  int* sSl = reinterpret_cast<int*>(reinterpret_cast<char*>(lds) + off);
  uint16_t* sInc = reinterpret_cast<uint16_t*>(sSl + 4 * maxn);
  uint16_t* sGi = sInc + (inc_lds_bytes(NV, maxc) / sizeof(uint16_t));

  // halo cell topology of this thread's first two extended cells
  const int H = m.nhalo;
  int hl[2][NV];
  uint32_t hsh[2] = {0u, 0u};
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const int h = (int)threadIdx.x + j * (int)blockDim.x - nc;
    if (h >= 0 && h < nhc) {
#pragma unroll
      for (int k = 0; k < NV; ++k) hl[j][k] = m.hlconn[(size_t)k * H + hc0 + h];
      hsh[j] = m.hshift[hc0 + h];
    }
  }
  // ---- stage the slots and the halo nodes
  double iv = 0.0;     // 1/V of this thread's slot node
  double dxm = 0.0;    // its dx_min
  int g0 = 0, g1 = 0;  // its cells in sGi
  bool gw = false;     // this tile writes the node's gradient (closure output)
  for (int q = threadIdx.x; q < ns; q += blockDim.x) {
    const SlotTopo st = slot_topo<NV>(m, tp, q);
    slot_table_put(sSl, maxn, q, st.sv, st.pos, st.p0, st.p1);
    const int g = slot_node_id(st.sv);
    double w[NGF], xe[2 * ND];
#pragma unroll
    for (int v = 0; v < NGF; ++v) w[v] = W[(size_t)v * m.nn + g];
#pragma unroll
    for (int d = 0; d < ND; ++d) {
      xe[d] = m.x[(size_t)d * m.nn + g];
      if constexpr (MODEL == 1) xe[ND + d] = f.E[(size_t)d * m.nn + g];
    }
    if (q == (int)threadIdx.x) {
      iv = m.inv_vol[g];
      dxm = m.dxmin[g];
      g0 = m.slot_ginc[tp.s0 + q] - gb;
      g1 = m.slot_ginc[tp.s0 + q + 1] - gb;
      gw = st.pos == st.run.x;
    }
#pragma unroll
    for (int v = 0; v < NGF; ++v) {
      sWd[v * maxne + q] = w[v];
      if constexpr (WCOPY) sWc[v * maxn + q] = CT(w[v]);
    }
#pragma unroll
    for (int d = 0; d < ND; ++d) {
      sX[d * maxne + q] = xe[d];
      if constexpr (MODEL == 1) sE[d * maxn + q] = CT(xe[ND + d]);
    }
  }
  for (int h = threadIdx.x; h < nhn; h += blockDim.x) {
    const int g = m.hnode[hn0 + h];
    double w[NGF], xx[ND];
#pragma unroll
    for (int v = 0; v < NGF; ++v) w[v] = W[(size_t)v * m.nn + g];
#pragma unroll
    for (int d = 0; d < ND; ++d) xx[d] = m.x[(size_t)d * m.nn + g];
#pragma unroll
    for (int v = 0; v < NGF; ++v) sWd[v * maxne + ns + h] = w[v];
#pragma unroll
    for (int d = 0; d < ND; ++d) sX[d * maxne + ns + h] = xx[d];
  }
  tile_store_inc<NV>(m, tp, sInc);
  stage_u16<6>(m.ginc + gb, ngi, sGi);
  if (decide) {
    const double d = block_min(ck);
    if (threadIdx.x == 0) {
      DevScalars n;
      step_decide(fc.lp->s[fc.par ^ 1], fc.lp->found[fc.par ^ 1], d, n);
      if (t == 0) fc.lp->s[fc.par] = n;
      s_dt = n.dt;
      s_act = n.active;
    }
  } else if (threadIdx.x == 0) {
    s_dt = loop ? fc.lp->s[fc.par].dt : pp.dt_host;
    s_act = 1;
  }
  __syncthreads();
  if (!s_act) return;
  // ---- gradient parts of the tile's cells and halo cells: sum_k W_k S_k
  for (int ec = threadIdx.x; ec < nce; ec += blockDim.x) {
    int l[NV];
    uint32_t sh;
    if (ec < nc) {
      cell_topo<NV>(m, tp, ec, l, sh);
    } else {
      const int j = (ec - (int)threadIdx.x) / (int)blockDim.x;
      if (j < 2) {
#pragma unroll
        for (int k = 0; k < NV; ++k) l[k] = j == 0 ? hl[0][k] : hl[1][k];
        sh = j == 0 ? hsh[0] : hsh[1];
      } else {
        const int h = ec - nc;
#pragma unroll
        for (int k = 0; k < NV; ++k) l[k] = m.hlconn[(size_t)k * H + hc0 + h];
        sh = m.hshift[hc0 + h];
      }
    }
    double e[ND][ND], S[NV][ND];
    cell_rel_coords<ND>(m, sX, maxne, l, sh, e);
    simplex_normals<ND>(e, S);
#pragma unroll
    for (int v = 0; v < NGF; ++v) {
      double acc[ND];
#pragma unroll
      for (int d = 0; d < ND; ++d) acc[d] = 0.0;
#pragma unroll
      for (int k = 0; k < NV; ++k) {
        const double w = sWd[v * maxne + l[k]];
#pragma unroll
        for (int d = 0; d < ND; ++d) acc[d] += w * S[k][d];
      }
#pragma unroll
      for (int d = 0; d < ND; ++d) sCR[(v * ND + d) * maxce + ec] = acc[d];
    }
  }
  __syncthreads();
  // ---- node gradients of the slots over all their cells, ascending cell id
  constexpr int JC = NC <= 16 ? NC : 8;
  for (int q = threadIdx.x; q < ns; q += blockDim.x) {
    int a0 = g0, a1 = g1;
    double c = iv;
    bool wg = gw;
    if (q != (int)threadIdx.x) {
      const SlotTopo st = slot_topo<NV>(m, tp, q);
      c = m.inv_vol[slot_node_id(st.sv)];
      a0 = m.slot_ginc[tp.s0 + q] - gb;
      a1 = m.slot_ginc[tp.s0 + q + 1] - gb;
      wg = st.pos == st.run.x;
    }
    const double coef = -c / double(ND * NV);
    const int g = slot_node_id(sSl[q]);
    for (int j0 = 0; j0 < NC; j0 += JC) {
      double acc[JC];
#pragma unroll
      for (int jj = 0; jj < JC; ++jj) acc[jj] = 0.0;
      for (int p = a0; p < a1; ++p) {
        const int ec = sGi[p];
#pragma unroll
        for (int jj = 0; jj < JC; ++jj)
          if (j0 + jj < NC) acc[jj] += sCR[(j0 + jj) * maxce + ec];
      }
#pragma unroll
      for (int jj = 0; jj < JC; ++jj)
        if (j0 + jj < NC) {
          const double gv = coef * acc[jj];
          sG[(j0 + jj) * maxn + q] = CT(gv);
          if (fc.Gout && wg) fc.Gout[(size_t)(j0 + jj) * m.nn + g] = gv;
        }
    }
  }
  __syncthreads();
  // ---- fluxes of the tile's cells (the residual parts take the gradient parts' place);
  // the slots' 1/V and dx_min go to the part of the gradient area that the
  // residual parts leave free, for the node pass
  double* sR = sCR;
  const size_t tail = (size_t)NV * NVAR * maxc;
  const bool tail_ok = ncr >= tail + 2 * (size_t)maxn;
  if (tail_ok) {
    for (int q = threadIdx.x; q < ns; q += blockDim.x) {
      double a = iv, b = dxm;
      if (q != (int)threadIdx.x) {
        const int g = slot_node_id(sSl[q]);
        a = m.inv_vol[g];
        b = m.dxmin[g];
      }
      sCR[tail + q] = a;
      sCR[tail + maxn + q] = b;
    }
  }
  const CT* sW = WCOPY ? sWc : reinterpret_cast<const CT*>(sWd);
  const int ldw = WCOPY ? maxn : maxne;
  if constexpr (MODEL == 1)
    dd_cell_fluxes<ND, NSP, CT, NV>(m, tp, sX, sW, sG, sE, sR, CellLd{maxne, ldw, maxn, maxc}, CT(s_dt), pp);
  else
    gas_cell_fluxes<ND, NSP, FLUX, CT, NV>(m, tp, sX, sW, sG, sR, CellLd{maxne, ldw, maxn, maxc}, gp);
  __syncthreads();
  NodeLds nl{};
  if (f.Un == f.Win) {  // U^n is the staged state (first stage)
    nl.un = sWd;
    nl.ldu = maxne;
  }
  if (tail_ok) {
    nl.iv = sCR + tail;
    nl.dx = sCR + tail + maxn;
  }
  if constexpr (MODEL == 1 && !WCOPY) {
    nl.e = reinterpret_cast<const double*>(sE);
    nl.lde = maxn;
  }
  const double cand = tile_node_pass<ND, NSP, MODEL, NVAR>(m, f, s_dt, PR, ns, sSl, maxn, sInc, sR, maxc, nl);
  if (f.final_stage && loop) {
    const double b = block_min(cand);
    if (threadIdx.x == 0) post_candidate(f.cand, t, b);
  }
}

template <int ND, int NSP, int MODEL, int FLUX, typename CT>
__global__ void VCX_FUSED_BOUNDS k_fused(DevMesh m, const double* __restrict__ W, double* __restrict__ PR,
                                        GasParams gp, DDParams pp, Finish f, FusedCtl fc) {
  extern __shared__ double lds[];
  const int t = xcd_tile(m.ntiles);
  if (t >= m.ntiles) return;
  fused_body<ND, NSP, MODEL, FLUX, CT>(m, W, PR, gp, pp, f, fc, t, lds);
}

// ---------------------------------------------------------------------------
// multi-species Navier-Stokes flux pass: MUSCL on (U, p), HLLC with each
// side's own gamma, minus the central diffusive flux
// W rows: U [NVAR], p, prim (velocity, T, Y) [NP], aux [NA]; gradients of the
// first NR + NP rows.
// ---------------------------------------------------------------------------

// Multi-species flux tile pass over the tile's distinct edges.  For an edge
// (a, b) the MUSCL face states (virtual-node reconstruction with the nodal
// gradients) depend on its two nodes only, so they are formed once per edge;
// the HLLC flux is taken for each of the edge's cell-edges with that cell's
// dual-face vector (the flux is not linear in it); the central diffusive
// flux is linear in the dual-face vector, so it is taken once with their
// sum.  The edge's net flux F goes to node a as +F and to node b as -F; each
// slot sums its edges in a fixed order into its partial (node pass), and the
// update pass finishes every node.  The node data come from the node-major
// staged rows WS and the node-major G.
// AXI: axisymmetric (x, r) meshes; every cell-edge's dual-face vector is
// weighted by the centroid radius of its face piece (revolved face over
// 2 pi) and the diffusive flux takes the cylindrical div u.
template <int ND, int NSP, typename CT, bool AXI = false>
__device__ inline void flux_ns_body(DevMesh m, const double* __restrict__ WS,
                                    const double* __restrict__ G,
                                    double* __restrict__ PR, GasParams gp, Finish f, int t, double* lds) {
  static_assert(!AXI || ND == 2, "axisymmetric meshes are (x, r) planes");
  using L = NsEdgeLds<ND, NSP, CT>;
  constexpr int NV = ND + 1, NVAR = 2 + ND + NSP, NR = NVAR + 1, NCE = L::NCE;
  // the node-major staged rows: all but the species D and h_s rows where
  // FP64 forms them (ns_staged_rows)
  constexpr int NWS = ns_staged_rows(ND, NSP, L::RECOMPUTE), LWS = ns_row64(NWS);
  constexpr int NP = ND + 1 + NSP, NC = (NR + NP) * ND;
  constexpr int RA = L::RA, CA = L::CA, RB = L::RB, CB = L::CB;
  static_assert(RB == 1 + NP + (NWS - NR - NP - 1), "phase B stages rho, the primitives and the staged tail");
  const CT* GC = reinterpret_cast<const CT*>(G);  // G is stored in the staging type
  // the staged rows in the staging type: FP64, or the FP32 rows after the
  // FP64 ones (of the FP64 path's stride)
  constexpr bool R32 = std::is_same<CT, float>::value;
  constexpr int LWR = R32 ? ns_row32(NWS) : LWS;
  constexpr int LW64 = ns_row64(ns_staged_rows(ND, NSP, true));
  const CT* WR = R32 ? reinterpret_cast<const CT*>(WS + (size_t)m.nn * LW64) : reinterpret_cast<const CT*>(WS);
  if (step_inactive(f.sc)) return;
  const int c0 = m.tile_cell[t], nc = m.tile_cell[t + 1] - c0;
  const int s0 = m.tile_slot[t], ns = m.tile_slot[t + 1] - s0;
  const int e0 = m.tile_edge[t], ne = m.tile_edge[t + 1] - e0;
  const int pb = m.slot_einc[s0], ninc = m.slot_einc[s0 + ns] - pb;
  const int maxn = m.max_tile_nodes, maxc = m.max_tile_cells, maxe = m.max_tile_edges;
  const int mce = maxc * NCE;
  char* base = reinterpret_cast<char*>(lds);
  double* sX = reinterpret_cast<double*>(base);                      // [ND][maxn]
  double* sF = reinterpret_cast<double*>(base + L::x_bytes(maxn));   // [NVAR][maxe]
  CT* sS = reinterpret_cast<CT*>(base + L::x_bytes(maxn) + L::f_bytes(maxe));  // [ND][maxc*NCE]
  CT* sW = reinterpret_cast<CT*>(base + L::x_bytes(maxn) + L::f_bytes(maxe) + L::s_bytes(maxc));
  int* sSl = reinterpret_cast<int*>(reinterpret_cast<char*>(sW) + L::area_bytes(maxn));
  uint16_t* sEi = reinterpret_cast<uint16_t*>(sSl + 4 * maxn);
  const CT beta = CT(gp.beta);

  uint32_t pdesc = 0;
  int pq0 = 0, pq1 = 0;
  if ((int)threadIdx.x < ne) {
    pdesc = m.edge[e0 + threadIdx.x];
    pq0 = m.edge_ce[e0 + threadIdx.x];
    pq1 = m.edge_ce[e0 + threadIdx.x + 1];
  }
  // the topology of this thread's first cell, loaded with the edge
  // descriptors (both overlap the staging)
  int pl[NV];
  uint32_t pshift = 0;
  if ((int)threadIdx.x < nc) {
#pragma unroll
    for (int k = 0; k < NV; ++k) pl[k] = m.lconn[(size_t)k * m.nc + c0 + threadIdx.x];
    pshift = m.shift[c0 + threadIdx.x];
  }
  // The node pass, and the FP32 path's staging, take two threads per slot
  // where the block has them (half h of slot q at thread h * ns + q, so that
  // a wavefront's lanes mostly take the same half).  Staging halves: the
  // first the state rows, coordinates and slot table with the first part of
  // the gradient row, the second the rest of the gradient row.  (Split
  // staging was slower for the FP64 pass: 4.43 -> 4.58 ms on C4.)
  const int tpn = (int)blockDim.x >= 2 * ns ? 2 : 1;
  const int tps = sizeof(CT) == 4 ? tpn : 1;
  constexpr int CA0 = CA / 3, CB0 = CB / 3;  // gradient components the first half stages
  // ---- phase A staging: coordinates, reconstructed rows, gamma, gradients
  {
    CT* sG = sW + RA * maxn;
    for (int t = threadIdx.x; t < tps * ns; t += blockDim.x) {
      const int h = t >= ns ? 1 : 0, q = t - h * ns;
      const int sl = s0 + q;
      const int sv = m.slot_node[sl];
      const int g = slot_node_id(sv);
      if (h == 0) {
        slot_table_put(sSl, maxn, q, sv, m.slot_pos[sl], m.slot_einc[sl] - pb, m.slot_einc[sl + 1] - pb);
        double xx[ND];
#pragma unroll
        for (int d = 0; d < ND; ++d) xx[d] = m.x[(size_t)d * m.nn + g];
        stage_gradient_row<LWR, 0, NR, CT, CT>(WR, g, sW, maxn, q);
        sW[NR * maxn + q] = WR[(size_t)g * LWR + NR + NP];
        if (tps == 2)
          stage_gradient_row<node_row(NC), 0, CA0, CT, CT>(GC, g, sG, maxn, q);
        else
          stage_gradient_row<node_row(NC), 0, CA, CT, CT>(GC, g, sG, maxn, q);
#pragma unroll
        for (int d = 0; d < ND; ++d) sX[d * maxn + q] = xx[d];
      } else {
        stage_gradient_row<node_row(NC), CA0, CA - CA0, CT, CT>(GC, g, sG + CA0 * maxn, maxn, q);
      }
    }
    for (int p = threadIdx.x; p < ninc; p += blockDim.x) sEi[p] = m.einc[pb + p];
  }
  __syncthreads();
  // ---- dual-face vectors of every cell-edge: S_ab = (S_a - S_b) / (n_d n_v)
  for (int lc = threadIdx.x; lc < nc; lc += blockDim.x) {
    const bool first = lc == (int)threadIdx.x;
    int l[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) l[k] = first ? pl[k] : (int)m.lconn[(size_t)k * m.nc + c0 + lc];
    double e[ND][ND], Sd[NV][ND];
    cell_rel_coords<ND>(m, sX, maxn, l, first ? pshift : m.shift[c0 + lc], e);
    simplex_normals<ND>(e, Sd);
    double rr[NV], rc = 0.0;
    if constexpr (AXI) {
#pragma unroll
      for (int k = 0; k < NV; ++k) rr[k] = sX[maxn + l[k]];
      rc = (rr[0] + rr[1] + rr[2]) / 3.0;
    }
#pragma unroll
    for (int ed = 0; ed < NCE; ++ed) {
      const int a = Edges<ND>::a(ed), b = Edges<ND>::b(ed);
      // axisymmetric: the face piece from the edge midpoint to the centroid,
      // revolved, carries its mean radius
      const double rw = AXI ? 0.5 * (0.5 * (rr[a] + rr[b]) + rc) : 1.0;
#pragma unroll
      for (int d = 0; d < ND; ++d)
        sS[d * mce + lc * NCE + ed] = CT((Sd[a][d] - Sd[b][d]) * (1.0 / double(ND * NV)) * rw);
    }
  }
  __syncthreads();
  // ---- convective flux of each edge: face states once, HLLC per cell-edge
  for (int le = threadIdx.x; le < ne; le += blockDim.x) {
    const CT* sG = sW + RA * maxn;
    const bool first = le == (int)threadIdx.x;
    const uint32_t desc = first ? pdesc : m.edge[e0 + le];
    const int la = desc & 4095u, lb = (desc >> 12) & 4095u;
    CT dx[ND];
#pragma unroll
    for (int d = 0; d < ND; ++d) {
      const uint32_t im = (desc >> (24 + 2 * d)) & 3u;
      const double sh = im == 1u ? m.period[d] : (im == 2u ? -m.period[d] : 0.0);
      dx[d] = CT(sX[d * maxn + lb] + sh - sX[d * maxn + la]);
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
      const CT dli = CT(2) * gi - delta, djk = CT(2) * gj - delta;
      WL[v] = wi + CT(0.5) * slope_limit<CT>(gp.limiter, beta, dli, delta);
      WR[v] = wj - CT(0.5) * slope_limit<CT>(gp.limiter, beta, delta, djk);
    }
    const CT gL = sW[NR * maxn + la], gR = sW[NR * maxn + lb];
    double Fs[NVAR];
#pragma unroll
    for (int v = 0; v < NVAR; ++v) Fs[v] = 0.0;
    const int q0 = first ? pq0 : m.edge_ce[e0 + le], q1 = first ? pq1 : m.edge_ce[e0 + le + 1];
    for (int q = q0; q < q1; ++q) {
      const int code = m.ce[q];
      const int k = (code >> 4) * NCE + ((code >> 1) & 7);
      const CT sg = (code & 1) ? CT(-1) : CT(1);
      CT S[ND], F[NVAR];
#pragma unroll
      for (int d = 0; d < ND; ++d) S[d] = sg * sS[d * mce + k];
      hllc_flux<ND, NSP, CT>(WL, WR, S, gL, gR, F);
#pragma unroll
      for (int v = 0; v < NVAR; ++v) Fs[v] += double(F[v]);
    }
#pragma unroll
    for (int v = 0; v < NVAR; ++v) sF[v * maxe + le] = Fs[v];
  }
  __syncthreads();  // every convective flux has read phase A

  // ---- phase B staging: rho, primitives, transport rows, primitive gradients
  {
    CT* sG = sW + RB * maxn;
    for (int t = threadIdx.x; t < tps * ns; t += blockDim.x) {
      const int h = t >= ns ? 1 : 0, q = t - h * ns;
      const int g = slot_node_id(sSl[q]);
      if (h == 0) {
        sW[q] = WR[(size_t)g * LWR];
        stage_gradient_row<LWR, NR, NP, CT, CT>(WR, g, sW + maxn, maxn, q);
        stage_gradient_row<LWR, NR + NP + 1, NWS - NR - NP - 1, CT, CT>(WR, g, sW + (1 + NP) * maxn, maxn, q);
        if (tps == 2)
          stage_gradient_row<node_row(NC), CA, CB0, CT, CT>(GC, g, sG, maxn, q);
        else
          stage_gradient_row<node_row(NC), CA, CB, CT, CT>(GC, g, sG, maxn, q);
      } else {
        stage_gradient_row<node_row(NC), CA + CB0, CB - CB0, CT, CT>(GC, g, sG + CB0 * maxn, maxn, q);
      }
    }
  }
  __syncthreads();
  // ---- diffusive flux of each edge, with the sum of its dual-face vectors
  for (int le = threadIdx.x; le < ne; le += blockDim.x) {
    const CT* sG = sW + RB * maxn;
    const bool first = le == (int)threadIdx.x;
    const uint32_t desc = first ? pdesc : m.edge[e0 + le];
    const int la = desc & 4095u, lb = (desc >> 12) & 4095u;
    CT S[ND];
#pragma unroll
    for (int d = 0; d < ND; ++d) S[d] = CT(0);
    const int q0 = first ? pq0 : m.edge_ce[e0 + le], q1 = first ? pq1 : m.edge_ce[e0 + le + 1];
    for (int q = q0; q < q1; ++q) {
      const int code = m.ce[q];
      const int k = (code >> 4) * NCE + ((code >> 1) & 7);
#pragma unroll
      for (int d = 0; d < ND; ++d) S[d] = (code & 1) ? S[d] - sS[d * mce + k] : S[d] + sS[d * mce + k];
    }
    // face averages h (x_a + x_b) of the diffusive flux's node data
    const CT h = CT(0.5);
    ViscousFace<ND, NSP, CT> fa;
    fa.rho = h * (sW[la] + sW[lb]);
#pragma unroll
    for (int q = 0; q < NP; ++q) fa.p[q] = h * (sW[(1 + q) * maxn + la] + sW[(1 + q) * maxn + lb]);
    if constexpr (L::RECOMPUTE) {
      const CT mui = sW[(1 + NP) * maxn + la], muj = sW[(1 + NP) * maxn + lb];
      const CT rhoi = sW[la], rhoj = sW[lb];
      fa.mu = h * (mui + muj);
      fa.lam = h * (sW[(2 + NP) * maxn + la] + sW[(2 + NP) * maxn + lb]);
      // D_k = mu / (rho Sc_k) and h_s,k(T) of each end, as the node state forms them
      const double Ti = sW[(1 + ND) * maxn + la], Tj = sW[(1 + ND) * maxn + lb];
      const double dTi = Ti - kT0, sTi = Ti + kT0, qTi = Ti * Ti + Ti * kT0 + kT0 * kT0;
      const double dTj = Tj - kT0, sTj = Tj + kT0, qTj = Tj * Tj + Tj * kT0 + kT0 * kT0;
#pragma unroll
      for (int k = 0; k < NSP; ++k) {
        fa.D[k] = h * (mui / (rhoi * f.mix.Sc[k]) + muj / (rhoj * f.mix.Sc[k]));
        const double hi = kRgas / f.mix.W[k] * dTi *
                          (f.mix.a[k] + f.mix.b[k] * sTi * (1.0 / 2000.0) + f.mix.c[k] * qTi * (1.0 / 3.0e6));
        const double hj = kRgas / f.mix.W[k] * dTj *
                          (f.mix.a[k] + f.mix.b[k] * sTj * (1.0 / 2000.0) + f.mix.c[k] * qTj * (1.0 / 3.0e6));
        fa.hs[k] = h * (hi + hj);
      }
    } else {
      fa.mu = h * (sW[(1 + NP) * maxn + la] + sW[(1 + NP) * maxn + lb]);
      fa.lam = h * (sW[(2 + NP) * maxn + la] + sW[(2 + NP) * maxn + lb]);
#pragma unroll
      for (int k = 0; k < NSP; ++k) {
        fa.D[k] = h * (sW[(3 + NP + k) * maxn + la] + sW[(3 + NP + k) * maxn + lb]);
        fa.hs[k] = h * (sW[(3 + NP + NSP + k) * maxn + la] + sW[(3 + NP + NSP + k) * maxn + lb]);
      }
    }
#pragma unroll
    for (int q = 0; q < NP * ND; ++q) fa.g[q] = h * (sG[q * maxn + la] + sG[q * maxn + lb]);
    CT Fv[NVAR], hoop = CT(0);
    if constexpr (AXI) {
      // u_r / r at the edge midpoint; on an edge along the axis its limit,
      // the mean of the ends' d u_r / d r
      const CT rbar = h * CT(sX[maxn + la] + sX[maxn + lb]);
      hoop = rbar > CT(0) ? fa.p[1] / rbar : fa.g[1 * ND + 1];
    }
    viscous_flux_face<ND, NSP, CT>(fa, S, Fv, hoop);
#pragma unroll
    for (int v = 0; v < NVAR; ++v) sF[v * maxe + le] -= double(Fv[v]);
  }
  __syncthreads();

  // ---- node pass: each slot sums its edges' fluxes in ascending edge order
  // into its partial; the update pass finishes every node.  (Most nodes of
  // a tetrahedral tile are shared anyway, and finishing the few owned ones
  // here set the pass's register peak.)
  // (two threads per slot: each sums half of the variables)
  constexpr int NH = (NVAR + 1) / 2;
  for (int t = threadIdx.x; t < tpn * ns; t += blockDim.x) {
    const int h = t >= ns ? 1 : 0, q = t - h * ns;
    const SlotTopo st = slot_table_get(sSl, maxn, q);
    const int v0 = tpn == 2 && h == 1 ? NH : 0, nv = tpn == 2 ? (h == 0 ? NH : NVAR - NH) : NVAR;
    double r[NVAR];
#pragma unroll
    for (int v = 0; v < NVAR; ++v) r[v] = 0.0;
    for (int p = st.p0; p < st.p1; ++p) {
      const int code = sEi[p];
      const int le = code >> 1;
      const double sgn = (code & 1) ? -1.0 : 1.0;
#pragma unroll
      for (int v = 0; v < NVAR; ++v)
        if (v < nv) r[v] += sgn * sF[(v0 + v) * maxe + le];
    }
#pragma unroll
    for (int v = 0; v < NVAR; ++v)
      if (v < nv) PR[(size_t)st.pos * NVAR + v0 + v] = r[v];
  }
}

template <int ND, int NSP, typename CT, bool AXI = false>
__global__ void VCX_FLUX_BOUNDS k_flux_ns(DevMesh m, const double* __restrict__ WS,
                                          const double* __restrict__ G,
                                          double* __restrict__ PR, GasParams gp, Finish f) {
  extern __shared__ double lds[];
  const int t = xcd_tile(m.ntiles);
  if (t >= m.ntiles) return;
  flux_ns_body<ND, NSP, CT, AXI>(m, WS, G, PR, gp, f, t, lds);
}

// Primitive rows -> conserved rows, in place on the first nvar rows of W:
// gas (rho, u, p, Y) with the constant-gamma ideal gas; multi-species
// (rho, u, T, Y) with the mixture's sensible energy e_s(T); drift-diffusion
// densities are left as they are.
template <int ND, int NSP, int MODEL>
__global__ void __launch_bounds__(256) k_prim_to_cons(double* __restrict__ W, int nn, double gamma,
                                                      MixParams mp) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (MODEL == 1 || i >= nn) return;
  const double rho = W[i];
  double ke = 0.0;
#pragma unroll
  for (int d = 0; d < ND; ++d) {
    const double u = W[(size_t)(1 + d) * nn + i];
    ke += u * u;
    W[(size_t)(1 + d) * nn + i] = rho * u;
  }
  double Y[NSP > 0 ? NSP : 1];
#pragma unroll
  for (int k = 0; k < NSP; ++k) {
    Y[k] = W[(size_t)(2 + ND + k) * nn + i];
    W[(size_t)(2 + ND + k) * nn + i] = rho * Y[k];
  }
  const double q = W[(size_t)(1 + ND) * nn + i];  // p (gas) or T (multi-species)
  double e;
  if constexpr (MODEL == 2) {
    double es, cv;
    mix_es_cv<NSP>(mp, Y, q, es, cv);
    e = rho * (es + 0.5 * ke);
  } else {
    e = q / (gamma - 1.0) + 0.5 * rho * ke;
  }
  W[(size_t)(1 + ND) * nn + i] = e;
}

// multi-species node data of an uploaded state: p (component-major, beside U)
// and the node-major staged row
template <int ND, int NSP>
__global__ void __launch_bounds__(256) k_ns_aux(double* __restrict__ W, int nn, MixParams mp,
                                                double* __restrict__ WS, int nws, int ldws, int ws32) {
  constexpr int NVAR = 2 + ND + NSP, NP = ND + 1 + NSP, NA = 3 + 2 * NSP;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nn) return;
  double u[NVAR], prim[NP], aux[NA], p;
#pragma unroll
  for (int v = 0; v < NVAR; ++v) u[v] = W[(size_t)v * nn + i];
  ns_node_state<ND, NSP>(mp, u, p, prim, aux);
  W[(size_t)NVAR * nn + i] = p;
  ns_store_node_row<ND, NSP>(WS + (size_t)i * ldws, nws, u, p, prim, aux);
  if (ws32)
    ns_store_node_row32<ND, NSP>(reinterpret_cast<float*>(WS + (size_t)nn * ldws) +
                                     (size_t)i * ns_row32(ns_staged_rows(ND, NSP, false)),
                                 u, p, prim, aux);
}

// ---------------------------------------------------------------------------
// shared nodes: gather the per-tile residual partials, then finish
// ---------------------------------------------------------------------------

template <int ND, int NSP, int MODEL>
__device__ inline void update_shared_body(const DevMesh& m, const double* __restrict__ PR,
                                          const Finish& f, int b) {
  constexpr int NVAR = MODEL == 1 ? NSP : 2 + ND + NSP;
  if (f.roll && b == 0) step_rollover(f.roll, f.roll_par, f.roll->s[f.roll_par].active);
  if (step_inactive(f.sc)) return;
  // the next step reduces the candidates written by this stage
  if (f.final_stage && f.sc && b == 0 && threadIdx.x == 0) f.sc->dt_src = 1;  // cand[par] from now on
  const int k = b * blockDim.x + threadIdx.x;
  double cand = INFINITY;
  // update_all models leave every node to this pass (each node's run of
  // partials, one for an owned node); the others the shared ones
  constexpr bool ALL = update_all(MODEL, ND);
  if (k < (ALL ? m.nn : m.nshared)) {
    const int i = ALL ? k : m.shared[k];
    const int2 run = ALL ? make_int2(m.node_slot[k], m.node_slot[k + 1]) : m.shared_run[k];
    NodeIn<NVAR, ND> ni;
    node_in_load<ND, MODEL, NVAR>(m, f, f.sc ? f.sc->dt : 0.0, i, ni);
    double r[NVAR];
#pragma unroll
    for (int v = 0; v < NVAR; ++v) r[v] = 0.0;
    for (int p = run.x; p < run.y; ++p) {
      const double* src = PR + (size_t)p * NVAR;
#pragma unroll
      for (int v = 0; v < NVAR; ++v) r[v] += src[v];
    }
    cand = finish_node<ND, NSP, MODEL, NVAR>(m, f, i, true, r, ni);
  }
  if (f.final_stage && f.sc) {
    const double bm = block_min(cand);
    if (threadIdx.x == 0) post_candidate(f.cand, m.ntiles + b, bm);
  }
}

template <int ND, int NSP, int MODEL>
__global__ void __launch_bounds__(256) k_update_shared(DevMesh m, const double* __restrict__ PR,
                                                       Finish f) {
  update_shared_body<ND, NSP, MODEL>(m, PR, f, blockIdx.x);
}

// dt candidates of the current state, one per 256 nodes (after an upload or
// for a time-step query)
template <int ND, int NSP, int MODEL>
__global__ void __launch_bounds__(256) k_node_dt(DevMesh m, const double* __restrict__ W,
                                                 const double* __restrict__ E, DtCoef dc,
                                                 MixParams mp, DevLoop* lp) {
  constexpr int NVAR = MODEL == 1 ? NSP : 2 + ND + NSP;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  double cand = INFINITY;
  if (i < m.nn) {
    double u[NVAR];
#pragma unroll
    for (int v = 0; v < NVAR; ++v) u[v] = W[(size_t)v * m.nn + i];
    double p = MODEL != 1 ? W[(size_t)NVAR * m.nn + i] : 0.0;
    if constexpr (MODEL == 2) {
      // primitives and transport data formed again from U, as the update
      // and the upload form them (the same function of U, so the same values)
      constexpr int NP = ND + 1 + NSP, NA = 3 + 2 * NSP;
      double prim[NP], aux[NA];
      ns_node_state<ND, NSP>(mp, u, p, prim, aux);
      const bool ok = u[0] > 0.0 && prim[ND] > 0.0 && isfinite(prim[ND]);
      cand = ns_node_dt<ND, NSP>(m.dxmin[i], dc, mp, u[0], prim, p, aux, ok);
    } else {
      double Ei[ND] = {};
      if constexpr (MODEL == 1) {
#pragma unroll
        for (int d = 0; d < ND; ++d) Ei[d] = E[(size_t)d * m.nn + i];
      }
      cand = node_dt<ND, NSP, MODEL>(dc, m.dxmin[i], Ei, u, p);
    }
  }
  const double b = block_min(cand);
  if (threadIdx.x == 0) {
    post_candidate(lp->cnode, blockIdx.x, b);
    // the next step (either parity) takes its candidates from this pass
    if (blockIdx.x == 0) lp->s[0].dt_src = lp->s[1].dt_src = 0;
  }
}

// empty the node-pass slots (before a node pass)
static __global__ void k_node_slots_clear(DevLoop* lp) {
  if (threadIdx.x < kCandSlots) lp->cnode[threadIdx.x] = cand_empty();
}

static __global__ void __launch_bounds__(256) k_dt_query(DevLoop* lp) {
  const double v = threadIdx.x < kCandSlots ? key_cand(lp->cnode[threadIdx.x]) : INFINITY;
  const double d = block_min(v);
  if (threadIdx.x == 0) lp->s[0].dt_query = lp->s[1].dt_query = (d > 0.0 && isfinite(d)) ? d : -1.0;
}

// end of a host call: commit the last step (of parity par)
static __global__ void k_commit(DevLoop* lp, int par) {
  if (threadIdx.x == 0 && blockIdx.x == 0) step_finish(lp, par);
}

// smallest inscribed diameter 2 nd V / sum_k |S_k| over the cells of each node
template <int ND, int NV = ND + 1>
__global__ void __launch_bounds__(256) k_cell_dx(DevMesh m, unsigned long long* __restrict__ dxbits) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= m.nc) return;
  int v[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) v[k] = m.cell[(size_t)k * m.nc + c];
  const uint32_t code = m.shift[c];
  double e[NV - 1][ND], S[NV][ND];
#pragma unroll
  for (int k = 1; k < NV; ++k)
#pragma unroll
    for (int d = 0; d < ND; ++d) {
      const uint32_t b = (code >> (2 * ((k - 1) * ND + d))) & 3u;
      const double s = b == 1u ? m.period[d] : (b == 2u ? -m.period[d] : 0.0);
      e[k - 1][d] = m.x[(size_t)d * m.nn + v[k]] + s - m.x[(size_t)d * m.nn + v[0]];
    }
  const double det = Shape<ND, NV>::normals(e, S);
  double area = 0.0;
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    double s2 = 0.0;
#pragma unroll
    for (int d = 0; d < ND; ++d) s2 += S[k][d] * S[k][d];
    area += sqrt(s2);
  }
  const double dx = 2.0 * ND * (NV == ND + 1 ? det / (ND == 2 ? 2.0 : 6.0) : det * Shape<ND, NV>::kvol) / area;
  const unsigned long long bits = (unsigned long long)__double_as_longlong(dx);
#pragma unroll
  for (int k = 0; k < NV; ++k) atomicMin(&dxbits[v[k]], bits);
}

// ---------------------------------------------------------------------------
// batched launches: one launch covers the tiles (or shared-node blocks) of
// several independent solves, each with its own mesh, buffers and time loop.
// A device table holds one entry per solve; a block map gives each block its
// solve and its local tile / block.  Every solve of a batch shares the model
// and scheme parameters.
// ---------------------------------------------------------------------------

struct BatchEntry {
  DevMesh m;
  double* W[2];     // state buffers; the current one is W[(step + phase) & 1]
  double* WS[2];    // multi-species: their node-major staged rows, or null
  int nws, ldws;
  double* G;
  int g32;          // multi-species FP32 path: G holds FP32 values
  double* PG;
  double* PR;
  const double* E;
  DevLoop* lp;
  double* gout;     // fused passes: node gradients for the boundary closure, or null
  int phase;        // buffer parity of the solve at batch step 0
  int spar;         // step parity of the solve at batch step 0
};

struct BatchStage {
  int step;         // batch step counter
  int stage;        // 1..K
  int final_stage;
  double alpha;
};

struct FinishShared {
  DtCoef dc;
  MixParams mix;
  int closure;
  int fused;        // the stage runs the fused gradient + flux pass
  int gcomplete;    // G is complete on shared nodes before the flux pass (node-gradient passes)
  int gnode;        // drift-diffusion node-gradient pass: G node-major
};

__device__ inline Finish batch_finish(const BatchEntry& e, const BatchStage& st,
                                      const FinishShared& fs, const double** Win) {
  const int cur = (st.step + e.phase) & 1;
  Finish f{};
  f.Un = e.W[cur];
  f.Wout = e.W[cur ^ 1];
  f.WSin = st.stage == 1 ? e.WS[cur] : e.WS[cur ^ 1];
  f.WSout = e.WS[cur ^ 1];
  f.nws = e.nws;
  f.ldws = e.ldws;
  f.Win = st.stage == 1 ? e.W[cur] : e.W[cur ^ 1];
  f.G = e.G;
  f.g32 = e.g32;
  f.PG = e.PG;
  f.E = e.E;
  const int par = (st.step + e.spar) & 1;
  f.sc = &e.lp->s[par];
  f.found = &e.lp->found[par];
  f.cand = e.lp->cand[par];
  if (fs.fused && st.stage == 1) {
    f.roll = e.lp;
    f.roll_par = par;
  }
  f.gfull = (fs.fused && e.gout != nullptr) || fs.gcomplete;
  f.gnode = fs.gnode;
  f.dc = fs.dc;
  f.mix = fs.mix;
  f.alpha = st.alpha;
  f.closure = fs.closure;
  f.final_stage = st.final_stage;
  f.residual_only = 0;
  *Win = f.Win;
  return f;
}

template <int ND, int NR>
__global__ void __launch_bounds__(256) k_grad_tile_batch(const BatchEntry* __restrict__ tab,
                                                         const int2* __restrict__ map, int nblocks,
                                                         BatchStage st) {
  extern __shared__ double lds[];
  const int g = xcd_tile(nblocks);
  if (g >= nblocks) return;
  const int2 ml = map[g];
  const BatchEntry& e = tab[ml.x];
  const int par = (st.step + e.spar) & 1;
  if (ml.y < 0) {
    // the solve's decision entry: the step that starts now
    if (st.stage == 1) step_start(e.lp, par);
    return;
  }
  const int cur = (st.step + e.phase) & 1;
  const double* Win = st.stage == 1 ? e.W[cur] : e.W[cur ^ 1];
  GradCtl ctl{e.lp, par, st.stage == 1 ? 1 : 0};
  grad_tile_body<ND, NR>(e.m, Win, e.G, e.PG, ctl, ml.y, lds);
}

// node gradient of every solve of a batch (block map: solve, node slice;
// slice -1 is the solve's decision entry)
template <int ND, int NR, bool WSR = false, typename GT = double>
__global__ void __launch_bounds__(64 * kGradNodeGroups) k_grad_node_batch(const BatchEntry* __restrict__ tab,
                                                         const int2* __restrict__ map, int nblocks,
                                                         BatchStage st) {
  const int g = xcd_tile(nblocks);
  if (g >= nblocks) return;
  const int2 ml = map[g];
  const BatchEntry& e = tab[ml.x];
  const int par = (st.step + e.spar) & 1;
  if (ml.y < 0) {
    if (st.stage == 1) step_start(e.lp, par);
    return;
  }
  const int cur = (st.step + e.phase) & 1;
  const double* Win = st.stage == 1 ? e.W[cur] : e.W[cur ^ 1];
  GradCtl ctl{e.lp, par, st.stage == 1 ? 1 : 0};
  const double* WSin = st.stage == 1 ? e.WS[cur] : e.WS[cur ^ 1];
  grad_node_body<ND, NR, WSR, GT>(e.m, Win, WSin, e.ldws, reinterpret_cast<GT*>(e.G), ctl, ml.y);
}

template <int ND, int NSP, int FLUX, typename CT>
__global__ void VCX_FLUX_BOUNDS k_flux_gas_batch(const BatchEntry* __restrict__ tab,
                                                 const int2* __restrict__ map, int nblocks,
                                                 BatchStage st, GasParams gp, FinishShared fs) {
  extern __shared__ double lds[];
  const int g = xcd_tile(nblocks);
  if (g >= nblocks) return;
  const int2 ml = map[g];
  if (ml.y < 0) return;  // a solve's reducer entry of the gradient pass
  const BatchEntry& e = tab[ml.x];
  const double* Win;
  const Finish f = batch_finish(e, st, fs, &Win);
  flux_gas_body<ND, NSP, FLUX, CT>(e.m, Win, e.G, e.PR, gp, f, ml.y, lds);
}

template <int ND, int NS, typename CT>
__global__ void VCX_FLUX_BOUNDS k_flux_dd_batch(const BatchEntry* __restrict__ tab,
                                                const int2* __restrict__ map, int nblocks,
                                                BatchStage st, DDParams pp, FinishShared fs) {
  extern __shared__ double lds[];
  const int g = xcd_tile(nblocks);
  if (g >= nblocks) return;
  const int2 ml = map[g];
  if (ml.y < 0) return;  // a solve's reducer entry of the gradient pass
  const BatchEntry& e = tab[ml.x];
  const double* Win;
  const Finish f = batch_finish(e, st, fs, &Win);
  flux_dd_body<ND, NS, CT>(e.m, Win, e.G, e.PR, pp, f, ml.y, lds);
}

template <int ND, int NSP, typename CT>
__global__ void VCX_FLUX_BOUNDS k_flux_ns_batch(const BatchEntry* __restrict__ tab,
                                                const int2* __restrict__ map, int nblocks,
                                                BatchStage st, GasParams gp, FinishShared fs) {
  extern __shared__ double lds[];
  const int g = xcd_tile(nblocks);
  if (g >= nblocks) return;
  const int2 ml = map[g];
  if (ml.y < 0) return;  // a solve's reducer entry of the gradient pass
  const BatchEntry& e = tab[ml.x];
  const double* Win;
  const Finish f = batch_finish(e, st, fs, &Win);
  const int cur = (st.step + e.phase) & 1;
  flux_ns_body<ND, NSP, CT>(e.m, st.stage == 1 ? e.WS[cur] : e.WS[cur ^ 1], e.G, e.PR, gp, f, ml.y, lds);
}

template <int ND, int NSP, int MODEL, int FLUX, typename CT>
__global__ void VCX_FUSED_BOUNDS k_fused_batch(const BatchEntry* __restrict__ tab,
                                              const int2* __restrict__ map, int nblocks, BatchStage st,
                                              GasParams gp, DDParams pp, FinishShared fs) {
  extern __shared__ double lds[];
  const int g = xcd_tile(nblocks);
  if (g >= nblocks) return;
  const int2 ml = map[g];
  if (ml.y < 0) return;
  const BatchEntry& e = tab[ml.x];
  const double* Win;
  const Finish f = batch_finish(e, st, fs, &Win);
  const int par = (st.step + e.spar) & 1;
  FusedCtl fc{e.lp, par, st.stage == 1 ? 1 : 0, e.gout};
  fused_body<ND, NSP, MODEL, FLUX, CT>(e.m, Win, e.PR, gp, pp, f, fc, ml.y, lds);
}

template <int ND, int NSP, int MODEL>
__global__ void __launch_bounds__(256) k_update_shared_batch(const BatchEntry* __restrict__ tab,
                                                             const int2* __restrict__ map,
                                                             BatchStage st, FinishShared fs) {
  const int2 ml = map[blockIdx.x];
  const BatchEntry& e = tab[ml.x];
  const double* Win;
  const Finish f = batch_finish(e, st, fs, &Win);
  update_shared_body<ND, NSP, MODEL>(e.m, e.PR, f, ml.y);
}

// per-solve control of a batch call: end time and step budget
static __global__ void k_batch_control(const BatchEntry* __restrict__ tab, int n,
                                const double* __restrict__ t_end, const int* __restrict__ steps) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  // the state the first batch step starts from
  DevScalars& sc = tab[i].lp->s[tab[i].spar ^ 1];
  sc.t_end = t_end[i];
  sc.steps_left = steps[i];
}

// after nq batch steps: commit every solve's last step and copy the
// scalars to one array
static __global__ void k_batch_commit(const BatchEntry* __restrict__ tab, int n, int nq,
                               DevScalars* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int par = (tab[i].spar + nq + 1) & 1;  // parity of batch step nq - 1
  step_finish(tab[i].lp, par);
  out[i] = tab[i].lp->s[par];
}

// ---------------------------------------------------------------------------
// permutations between the caller's node order and the internal order
// ---------------------------------------------------------------------------

static __global__ void k_gather_rows(const int32_t* __restrict__ perm, const double* __restrict__ src,
                              double* __restrict__ dst, int nn, int nrows) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nn) return;
  const int o = perm[i];
  for (int v = 0; v < nrows; ++v) dst[(size_t)v * nn + i] = src[(size_t)v * nn + o];
}

// the first nrows components of node-major rows (stride per node) into
// caller-order rows
static __global__ void k_scatter_node_rows(const int32_t* __restrict__ perm, const double* __restrict__ src,
                                           double* __restrict__ dst, int nn, int nrows, int stride) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nn) return;
  const int o = perm[i];
  for (int v = 0; v < nrows; ++v) dst[(size_t)v * nn + o] = src[(size_t)i * stride + v];
}

static __global__ void k_scatter_rows(const int32_t* __restrict__ perm, const double* __restrict__ src,
                               double* __restrict__ dst, int nn, int nrows) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nn) return;
  const int o = perm[i];
  for (int v = 0; v < nrows; ++v) dst[(size_t)v * nn + o] = src[(size_t)v * nn + i];
}

// pressure row of the gas reconstructed variables from the conserved rows
// Space charge rho / eps0 = (e / eps0) sum_s z_s n_s of a drift-diffusion
// state (internal order) into q (caller order).
static __global__ void __launch_bounds__(256) k_space_charge(const double* __restrict__ W, int nn, int nsp,
                                                             double z0, double z1, double z2, double z3,
                                                             double e_eps0, const int32_t* __restrict__ perm,
                                                             double* __restrict__ q) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nn) return;
  const double z[4] = {z0, z1, z2, z3};
  double c = 0.0;
  for (int k = 0; k < nsp && k < 4; ++k) c += z[k] * W[(size_t)k * nn + i];
  q[perm[i]] = e_eps0 * c;
}

static __global__ void k_pressure(double* W, int nn, int nd, int nsp, double gamma) {
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

static __global__ void __launch_bounds__(256) k_sums_partial(const double* __restrict__ W,
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

static __global__ void __launch_bounds__(256) k_sums_final(const double* __restrict__ part, int nparts,
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
