// C ABI of the vertex-centred residual library (declarations in include/vcx.h).
#include "vcx_internal.h"

using namespace vcx;

namespace {
thread_local std::string g_err;
}  // namespace

vcx_status vcx::fail(vcx_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

static vcx_status harvest(vcx_solver s) {
  if (s->ev.empty()) return VCX_OK;
  VCX_HIP(hipStreamSynchronize(s->mesh->stream));
  for (auto& kv : s->ev) {
    auto& a = s->acc[kv.first];
    for (auto& pr : kv.second) {
      float ms = 0.f;
      VCX_HIP(hipEventElapsedTime(&ms, pr.first, pr.second));
      a.first += 1;
      a.second += ms;
      s->spare.push_back(pr.first);
      s->spare.push_back(pr.second);
    }
    kv.second.clear();
  }
  return VCX_OK;
}

static const KernelTable* pick_table(int nd, int nv, const vcx_physics& ph) {
  if (nv != nd + 1) return pick_table_quad(ph);
  if (ph.model == VCX_MODEL_GAS) return nd == 2 ? pick_table_gas2(ph) : pick_table_gas3(ph);
  if (ph.model == VCX_MODEL_NAVIER_STOKES) return pick_table_ns(nd, ph);
  return pick_table_dd(nd, ph);
}

// ---------------------------------------------------------------------------
// mesh
// ---------------------------------------------------------------------------

template <typename T>
static vcx_status upload(vcx_mesh m, const std::vector<T>& v, const T** out) {
  if (v.empty()) {
    *out = nullptr;
    return VCX_OK;
  }
  void* p = nullptr;
  if (hipMalloc(&p, sizeof(T) * v.size()) != hipSuccess)
    return fail(VCX_E_OOM, "hipMalloc failed for mesh arrays");
  m->allocs.push_back(p);
  VCX_HIP(hipMemcpyAsync(p, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice, m->stream));
  *out = static_cast<const T*>(p);
  return VCX_OK;
}

static void free_mesh(vcx_mesh m) {
  if (!m) return;
  for (void* p : m->allocs) (void)hipFree(p);
  delete m;
}

extern "C" vcx_status vcx_mesh_preprocess(int ndim, int64_t nnodes, const double* xyz,
                                          int64_t ncells, int nv, const int64_t* cells,
                                          const double* period, int64_t stats[10]) {
  if (!stats) return fail(VCX_E_ARG, "stats is NULL");
  HostMesh h;
  int code = 0;
  std::string err = preprocess_mesh(ndim, nnodes, xyz, ncells, nv, cells, period,
                                    default_tile_limits(ndim), h, &code);
  if (!err.empty()) return fail(code == -2 ? VCX_E_MESH : VCX_E_ARG, err);
  stats[0] = h.nn;
  stats[1] = h.nc;
  stats[2] = h.nc * h.ne;
  stats[3] = h.ntiles();
  stats[4] = h.nslots();
  stats[5] = (int64_t)h.bnd_node.size();
  stats[6] = h.max_tile_cells;
  stats[7] = h.max_tile_nodes;
  std::memcpy(&stats[8], &h.vol_cells, 8);
  std::memcpy(&stats[9], &h.vol_nodes, 8);
  return VCX_OK;
}

extern "C" vcx_status vcx_mesh_create(int ndim, int64_t nnodes, const double* xyz,
                                      int64_t ncells, int nv, const int64_t* cells,
                                      const double* period, void* stream, vcx_mesh* out) {
  return vcx_mesh_create_tiled(ndim, nnodes, xyz, ncells, nv, cells, period, 0, 0, stream, out);
}

static vcx_status create_mesh(int ndim, int64_t nnodes, const double* xyz, int64_t ncells, int nv,
                              const int64_t* cells, const double* period, int max_tile_cells,
                              int max_tile_nodes, void* stream, bool axi, vcx_mesh* out);

extern "C" vcx_status vcx_mesh_create_tiled(int ndim, int64_t nnodes, const double* xyz,
                                            int64_t ncells, int nv, const int64_t* cells,
                                            const double* period, int max_tile_cells,
                                            int max_tile_nodes, void* stream, vcx_mesh* out) {
  return create_mesh(ndim, nnodes, xyz, ncells, nv, cells, period, max_tile_cells, max_tile_nodes, stream,
                     false, out);
}

extern "C" vcx_status vcx_mesh_create_axisymmetric(int64_t nnodes, const double* xr, int64_t ncells,
                                                   const int64_t* cells, double period_x, int max_tile_cells,
                                                   int max_tile_nodes, void* stream, vcx_mesh* out) {
  const double period[2] = {period_x, 0.0};
  return create_mesh(2, nnodes, xr, ncells, 3, cells, period, max_tile_cells, max_tile_nodes, stream, true,
                     out);
}

extern "C" vcx_status vcx_mesh_create_axisymmetric_nv(int64_t nnodes, const double* xr, int64_t ncells, int nv,
                                                      const int64_t* cells, double period_x, int max_tile_cells,
                                                      int max_tile_nodes, void* stream, vcx_mesh* out) {
  if (nv != 3 && nv != 4) return fail(VCX_E_ARG, "axisymmetric cells are triangles (nv 3) or quadrilaterals (nv 4)");
  const double period[2] = {period_x, 0.0};
  return create_mesh(2, nnodes, xr, ncells, nv, cells, period, max_tile_cells, max_tile_nodes, stream, true,
                     out);
}

// Drift-diffusion meshes above this many cells take the separate passes
// (1.8M cells: 120 against 158 us per step with the tile gradient; 200k
// cells: the fused pass 26 against 33 us).
constexpr int64_t kFusedMaxCells = int64_t(1) << 20;

// Build (host) and upload (device) the node-gradient tables of a simplex
// mesh, once (the host copies are released after the upload).
static vcx_status ensure_node_gradient(vcx_mesh m) {
  if (m->d.has_ngrad) return VCX_OK;
  HostMesh& h = m->h;
  std::string err = build_node_gradient(h);
  if (!err.empty()) return fail(VCX_E_MESH, err);
  DevMesh& d = m->d;
  const int64_t* off = nullptr;
  const int32_t* nbr = nullptr;
  const double* c = nullptr;
  VCX_TRY(upload(m, h.ng_off, &off));
  VCX_TRY(upload(m, h.ng_nbr, &nbr));
  VCX_TRY(upload(m, h.ng_c, &c));
  VCX_HIP(hipStreamSynchronize(m->stream));
  d.ng_off = reinterpret_cast<const long long*>(off);
  d.ng_nbr = nbr;
  d.ng_c = c;
  d.ng_nslices = (int)(h.ng_off.size() - 1);
  d.ng_total = (long long)h.ng_off.back();
  d.has_ngrad = 1;
  std::vector<int64_t>().swap(h.ng_off);
  std::vector<int32_t>().swap(h.ng_nbr);
  std::vector<double>().swap(h.ng_c);
  return VCX_OK;
}

// Build (host) and upload (device) the tables of the multi-species passes
// of a simplex mesh, once: tile edges (flux pass) and node gradient.
vcx_status vcx::ensure_tile_edges(vcx_mesh m) {
  if (m->d.has_edges) return VCX_OK;
  if (m->h.nv != m->h.nd + 1) return fail(VCX_E_ARG, "the multi-species model runs on simplex meshes");
  VCX_TRY(ensure_node_gradient(m));
  std::string err = build_tile_edges(m->h);
  if (!err.empty()) return fail(VCX_E_MESH, err);
  const HostMesh& h = m->h;
  DevMesh& d = m->d;
  const int32_t *te = nullptr, *ece = nullptr, *sei = nullptr;
  const uint32_t* ed = nullptr;
  const uint16_t *ce = nullptr, *ei = nullptr;
  VCX_TRY(upload(m, h.tile_edge, &te));
  VCX_TRY(upload(m, h.edge, &ed));
  VCX_TRY(upload(m, h.edge_ce, &ece));
  VCX_TRY(upload(m, h.ce, &ce));
  VCX_TRY(upload(m, h.slot_einc, &sei));
  VCX_TRY(upload(m, h.einc, &ei));
  d.tile_edge = te;
  d.edge = ed;
  d.edge_ce = ece;
  d.ce = ce;
  d.slot_einc = sei;
  d.einc = ei;
  d.max_tile_edges = h.max_tile_edges;
  d.has_edges = 1;
  return VCX_OK;
}

static vcx_status create_mesh(int ndim, int64_t nnodes, const double* xyz, int64_t ncells, int nv,
                              const int64_t* cells, const double* period, int max_tile_cells,
                              int max_tile_nodes, void* stream, bool axi, vcx_mesh* out) {
  if (!out) return fail(VCX_E_ARG, "out is NULL");
  *out = nullptr;
  if (ndim != 2 && ndim != 3) return fail(VCX_E_ARG, "ndim must be 2 or 3");
  TileLimits lim = default_tile_limits(ndim);
  if (max_tile_cells > 0) lim.max_cells = max_tile_cells;
  if (max_tile_nodes > 0) lim.max_nodes = max_tile_nodes;
  if (lim.max_cells > 1024) return fail(VCX_E_ARG, "max_tile_cells must be <= 1024");
  vcx_mesh m = new (std::nothrow) vcx_mesh_s();
  if (!m) return fail(VCX_E_OOM, "host allocation failed");
  int code = 0;
  std::string err = preprocess_mesh(ndim, nnodes, xyz, ncells, nv, cells, period, lim, m->h, &code, axi);
  if (!err.empty()) {
    delete m;
    return fail(code == -2 ? VCX_E_MESH : VCX_E_ARG, err);
  }
  m->stream = static_cast<hipStream_t>(stream);
  // (the device count first: it initialises the runtime in a process whose
  // first HIP call this is)
  int ndev = 0;
  hipError_t he = hipGetDeviceCount(&ndev);
  if (he == hipSuccess && ndev <= 0) he = hipErrorNoDevice;
  if (he == hipSuccess) he = hipGetDevice(&m->device);
  if (he == hipSuccess)
    he = hipDeviceGetAttribute(&m->lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, m->device);
  if (he != hipSuccess) {
    delete m;
    return fail(VCX_E_HIP, std::string("no usable HIP device: ") + hipGetErrorString(he));
  }
  const HostMesh& h = m->h;
  DevMesh& d = m->d;
  d.nd = h.nd;
  d.nv = h.nv;
  d.nn = (int)h.nn;
  d.nc = (int)h.nc;
  d.ntiles = (int)h.ntiles();
  d.nslots = (int)h.nslots();
  d.nb = (int)h.bnd_node.size();
  d.max_tile_cells = h.max_tile_cells;
  d.max_tile_nodes = h.max_tile_nodes;
  for (int k = 0; k < 3; ++k) d.period[k] = h.period[k];
  std::vector<double> inv(h.nn);
  for (int64_t i = 0; i < h.nn; ++i) inv[i] = 1.0 / h.vnode[i];
  std::vector<int32_t> bidx(h.nn, -1);
  for (size_t q = 0; q < h.bnd_node.size(); ++q) bidx[h.bnd_node[q]] = (int32_t)q;
  // derived tables: each tile's first incidence, each slot's position in its
  // node's run (the index of its partial sums), each shared node's run
  std::vector<int32_t> tile_inc(h.tile_slot.size()), slot_pos(h.slot_node.size());
  for (size_t t = 0; t < h.tile_slot.size(); ++t) tile_inc[t] = h.slot_inc[h.tile_slot[t]];
  for (size_t p = 0; p < h.slots_of.size(); ++p) slot_pos[h.slots_of[p]] = (int32_t)p;
  std::vector<int32_t> tile_ginc;
  if (h.has_halo) {
    tile_ginc.resize(h.tile_slot.size());
    for (size_t t = 0; t < h.tile_slot.size(); ++t) tile_ginc[t] = h.slot_ginc[h.tile_slot[t]];
  }
  std::vector<int32_t> srun(2 * h.shared.size());
  for (size_t k = 0; k < h.shared.size(); ++k) {
    srun[2 * k] = h.node_slot[h.shared[k]];
    srun[2 * k + 1] = h.node_slot[h.shared[k] + 1];
  }
  vcx_status st = VCX_OK;
  auto chk = [&](vcx_status s) {
    if (st == VCX_OK) st = s;
  };
  chk(upload(m, h.x, &d.x));
  chk(upload(m, h.cell, &d.cell));
  chk(upload(m, h.shift, &d.shift));
  chk(upload(m, h.lconn, &d.lconn));
  chk(upload(m, h.tile_cell, &d.tile_cell));
  chk(upload(m, h.tile_slot, &d.tile_slot));
  chk(upload(m, h.slot_node, &d.slot_node));
  chk(upload(m, h.slot_inc, &d.slot_inc));
  chk(upload(m, h.inc, &d.inc));
  {
    chk(upload(m, tile_inc, &d.tile_inc));
    chk(upload(m, slot_pos, &d.slot_pos));
    const int32_t* sr = nullptr;
    chk(upload(m, srun, &sr));
    d.shared_run = reinterpret_cast<const int2*>(sr);
  }
  chk(upload(m, h.node_slot, &d.node_slot));
  chk(upload(m, h.slots_of, &d.slots_of));
  chk(upload(m, h.shared, &d.shared));
  {
    const int32_t* run = nullptr;
    chk(upload(m, h.slot_run, &run));
    d.slot_run = reinterpret_cast<const int2*>(run);
  }
  d.nshared = (int)h.shared.size();
  if (h.has_halo) {
    d.has_halo = 1;
    d.nhalo = (int)h.hshift.size();
    d.max_ext_cells = h.max_ext_cells;
    d.max_ext_nodes = h.max_ext_nodes;
    d.max_tile_ginc = h.max_tile_ginc;
    chk(upload(m, h.tile_hcell, &d.tile_hcell));
    chk(upload(m, h.hlconn, &d.hlconn));
    chk(upload(m, h.hshift, &d.hshift));
    chk(upload(m, h.tile_hnode, &d.tile_hnode));
    chk(upload(m, h.hnode, &d.hnode));
    chk(upload(m, h.slot_ginc, &d.slot_ginc));
    chk(upload(m, h.ginc, &d.ginc));
    chk(upload(m, tile_ginc, &d.tile_ginc));
  }
  chk(upload(m, inv, &d.inv_vol));
  chk(upload(m, h.vnode, &d.vnode));
  d.axi = h.axi ? 1 : 0;
  if (h.axi) {
    // the update and the conservation sums use the revolved volumes
    std::vector<double> invu(h.nn);
    for (int64_t i = 0; i < h.nn; ++i) invu[i] = 1.0 / h.vupd[i];
    chk(upload(m, invu, &d.inv_vupd));
    chk(upload(m, h.vupd, &d.vupd));
  } else {
    d.inv_vupd = d.inv_vol;
    d.vupd = d.vnode;
  }
  chk(upload(m, bidx, &d.bnd_index));
  chk(upload(m, h.bnd_S, &d.bnd_S));
  chk(upload(m, h.bnd_node, &d.bnd_node));
  d.nbe = (int)h.bedge_nb.size();
  if (h.nd == 2) {
    chk(upload(m, h.bedge_ptr, &d.bedge_ptr));
    chk(upload(m, h.bedge_nb, &d.bedge_nb));
    chk(upload(m, h.bedge_S, &d.bedge_S));
  }
  chk(upload(m, h.perm, &d.perm));
  // tile-edge tables of the multi-species flux pass: 3D meshes at creation,
  // 2D meshes when their first Navier-Stokes solver is created
  if (st == VCX_OK && h.nd == 3) st = ensure_tile_edges(m);
  // node-gradient tables of large 2D simplex meshes (the separate
  // drift-diffusion passes) at creation too, not in a solver's first call
  if (st == VCX_OK && h.nd == 2 && h.nv == 3 && h.nc > kFusedMaxCells) st = ensure_node_gradient(m);
  if (st == VCX_OK) {
    // smallest inscribed diameter of the cells around each node (time step)
    void* p = nullptr;
    if (hipMalloc(&p, sizeof(double) * h.nn) != hipSuccess) {
      st = fail(VCX_E_OOM, "hipMalloc failed for mesh arrays");
    } else {
      m->allocs.push_back(p);
      d.dxmin = static_cast<const double*>(p);
      auto* bits = static_cast<unsigned long long*>(p);
      if (hipMemsetAsync(p, 0xFF, sizeof(double) * h.nn, m->stream) != hipSuccess)
        st = fail(VCX_E_HIP, "hipMemsetAsync failed");
      else if (d.nd == 2 && h.nv == 4)
        hipLaunchKernelGGL((k_cell_dx<2, 4>), dim3((d.nc + 255) / 256), dim3(256), 0, m->stream, d, bits);
      else if (d.nd == 2)
        hipLaunchKernelGGL(k_cell_dx<2>, dim3((d.nc + 255) / 256), dim3(256), 0, m->stream, d, bits);
      else
        hipLaunchKernelGGL(k_cell_dx<3>, dim3((d.nc + 255) / 256), dim3(256), 0, m->stream, d, bits);
      if (st == VCX_OK && hipGetLastError() != hipSuccess) st = fail(VCX_E_HIP, "k_cell_dx launch failed");
    }
  }
  if (st == VCX_OK && hipStreamSynchronize(m->stream) != hipSuccess)
    st = fail(VCX_E_HIP, "mesh upload failed");
  if (st != VCX_OK) {
    free_mesh(m);
    return st;
  }
  *out = m;
  return VCX_OK;
}

extern "C" vcx_status vcx_mesh_destroy(vcx_mesh m) {
  if (!m) return fail(VCX_E_ARG, "mesh is NULL");
  (void)hipStreamSynchronize(m->stream);
  free_mesh(m);
  return VCX_OK;
}

extern "C" vcx_status vcx_mesh_info(vcx_mesh m, int64_t out[8]) {
  if (!m || !out) return fail(VCX_E_ARG, "NULL argument");
  out[0] = m->h.nn;
  out[1] = m->h.nc;
  out[2] = m->h.nc * m->h.ne;
  out[3] = m->h.ntiles();
  out[4] = m->h.nslots();
  out[5] = (int64_t)m->h.bnd_node.size();
  out[6] = m->h.max_tile_cells;
  out[7] = m->h.max_tile_nodes;
  return VCX_OK;
}

extern "C" vcx_status vcx_mesh_geometry(vcx_mesh m, double* Vn, double* Sb) {
  if (!m) return fail(VCX_E_ARG, "mesh is NULL");
  const HostMesh& h = m->h;
  if (Vn)
    for (int64_t i = 0; i < h.nn; ++i) Vn[h.perm[i]] = h.vnode[i];
  if (Sb) {
    std::memset(Sb, 0, sizeof(double) * h.nd * h.nn);
    size_t nb = h.bnd_node.size();
    for (size_t q = 0; q < nb; ++q)
      for (int d = 0; d < h.nd; ++d) Sb[(size_t)d * h.nn + h.perm[h.bnd_node[q]]] = h.bnd_S[d * nb + q];
  }
  return VCX_OK;
}

// ---------------------------------------------------------------------------
// solver
// ---------------------------------------------------------------------------

static void free_solver(vcx_solver s) {
  if (!s) return;
  for (double* p : {s->W[0], s->W[1], s->WS[0], s->WS[1], s->G, s->PG, s->PR, s->E, s->io, s->rbuf, s->part,
                    s->sums_dev, s->cbuf})
    if (p) (void)hipFree(p);
  if (s->lp) (void)hipFree(s->lp);
  if (s->sc_host) (void)hipHostFree(s->sc_host);
  if (s->sums_host) (void)hipHostFree(s->sums_host);
  for (auto& kv : s->ev)
    for (auto& pr : kv.second) {
      (void)hipEventDestroy(pr.first);
      (void)hipEventDestroy(pr.second);
    }
  for (hipEvent_t e : s->spare) (void)hipEventDestroy(e);
  delete s;
}

static bool same_scheme(const vcx_physics& a, const vcx_physics& b) {
  return std::memcmp(&a, &b, sizeof(vcx_physics)) == 0;
}

// Device buffers of a solver, in doubles (one definition for creation and
// for the footprint query used by admission control).
struct SolverSizes {
  size_t W = 0, WS = 0, G = 0, PG = 0, PR = 0, io = 0, part = 0, sums = 0, E = 0;
  int node_blocks = 0, nsh_blocks = 1;
  size_t bytes() const {
    auto r = [](size_t n) { return sizeof(double) * std::max<size_t>(n, 1); };
    return 2 * r(W) + (WS ? 2 * r(WS) : 0) + r(G) + r(PG) + r(PR) + 2 * r(io) + r(part) + r(sums) +
           (E ? r(E) : 0) + sizeof(DevLoop);
  }
};

// Row stride of the multi-species node-major staged rows (0: other models).
// FP64 staged rows: conserved, p, primitives, gamma, mu, lambda (the FP32
// path stages the species D and h_s rows from its FP32 copy)
static int staged_row_stride(int nd, const vcx_physics& ph) {
  if (ph.model != VCX_MODEL_NAVIER_STOKES) return 0;
  return ns_row64(ns_staged_rows(nd, ph.nspecies, true));
}

static SolverSizes solver_sizes(const DevMesh& d, int nd, int nvar, int nr, int nw, int ngf, int model,
                                size_t ws_doubles) {
  SolverSizes z;
  const size_t nn = (size_t)d.nn, P = (size_t)d.nslots;
  z.W = (size_t)nw * nn;
  z.WS = ws_doubles;
  z.G = (size_t)node_row(ngf * nd) * nn;  // (node-major rows are padded to an even stride)
  z.PG = (size_t)ngf * nd * P;
  z.PR = (size_t)nvar * P;
  z.io = std::max<size_t>((size_t)ngf * nd, (size_t)nw) * nn;
  z.part = (size_t)nr * 256;
  z.sums = (size_t)nr;
  z.E = model == VCX_MODEL_DRIFT_DIFFUSION ? (size_t)nd * nn : 0;
  z.node_blocks = (int)((nn + kNodeBlock - 1) / kNodeBlock);
  // (update_all models finish every node in the update pass)
  const int nupd = update_all(model, nd) ? d.nn : d.nshared;
  z.nsh_blocks = std::max(1, (nupd + kNodeBlock - 1) / kNodeBlock);
  return z;
}

static vcx_status dmalloc(double** p, size_t n) {
  if (hipMalloc(reinterpret_cast<void**>(p), sizeof(double) * std::max<size_t>(n, 1)) != hipSuccess)
    return fail(VCX_E_OOM, "hipMalloc failed for solver buffers");
  return VCX_OK;
}

// Reset the time loop to t0 and compute the time-step candidates of the
// current state (consumed by the first step).
static vcx_status reset_scalars(vcx_solver s, double t0, bool prime) {
  DevScalars z{};
  z.t = t0;
  z.steps_left = -1;
  DevLoop l{};
  l.s[0] = l.s[1] = z;
  for (int q = 0; q < kCandSlots; ++q) l.cand[0][q] = l.cand[1][q] = l.cnode[q] = cand_empty();
  *s->sc_host = z;
  VCX_HIP(hipMemcpyAsync(s->lp, &l, sizeof(DevLoop), hipMemcpyHostToDevice, s->mesh->stream));
  if (prime) VCX_TRY(s->kt->node_dt(s, s->W[s->cur]));
  VCX_HIP(hipStreamSynchronize(s->mesh->stream));
  s->spar = 0;
  s->host_flag = 0;
  s->steps_total = 0;
  return VCX_OK;
}

// electric field (host or device, caller order) -> s->E (internal order), synchronised
static vcx_status upload_field(vcx_solver s, const double* E, int is_device = 0) {
  const DevMesh& d = s->mesh->d;
  const size_t nn = (size_t)d.nn;
  VCX_HIP(hipMemcpyAsync(s->io, E, sizeof(double) * s->nd * nn,
                         is_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s->mesh->stream));
  hipLaunchKernelGGL(k_gather_rows, dim3((nn + 255) / 256), dim3(256), 0, s->mesh->stream, d.perm,
                     (const double*)s->io, s->E, (int)nn, s->nd);
  VCX_HIP(hipGetLastError());
  VCX_HIP(hipStreamSynchronize(s->mesh->stream));
  return VCX_OK;
}

vcx_status vcx::solver_set_field(vcx_solver s, const double* E) {
  if (!s || !E || !s->E) return fail(VCX_E_ARG, "no field to set");
  return upload_field(s, E);
}

extern "C" vcx_status vcx_solver_set_field(vcx_solver s, const double* E, int is_device) {
  if (!s || !E) return fail(VCX_E_ARG, "NULL argument");
  if (!s->E) return fail(VCX_E_ARG, "the solver's model has no electric field");
  VCX_TRY(upload_field(s, E, is_device));
  if (s->has_state) {
    // the time-step candidates of the current state follow the new field
    VCX_TRY(s->kt->node_dt(s, s->W[s->cur]));
    VCX_HIP(hipStreamSynchronize(s->mesh->stream));
  }
  return VCX_OK;
}

extern "C" vcx_status vcx_solver_charge(vcx_solver s, double* q, int is_device) {
  if (!s || !q) return fail(VCX_E_ARG, "NULL argument");
  if (s->ph.model != VCX_MODEL_DRIFT_DIFFUSION) return fail(VCX_E_ARG, "space charge needs a drift-diffusion solver");
  if (!s->has_state) return fail(VCX_E_STATE, "no state uploaded");
  const DevMesh& d = s->mesh->d;
  double* dst = is_device ? q : s->io;
  const double e_eps0 = 1.602176634e-19 / 8.8541878128e-12;  // elementary charge / vacuum permittivity
  hipLaunchKernelGGL(k_space_charge, dim3((d.nn + 255) / 256), dim3(256), 0, s->mesh->stream,
                     (const double*)s->W[s->cur], d.nn, s->nvar, s->ph.z[0], s->ph.z[1], s->ph.z[2],
                     s->ph.z[3], e_eps0, d.perm, dst);
  VCX_HIP(hipGetLastError());
  if (!is_device)
    VCX_HIP(hipMemcpyAsync(q, s->io, sizeof(double) * d.nn, hipMemcpyDeviceToHost, s->mesh->stream));
  VCX_HIP(hipStreamSynchronize(s->mesh->stream));
  return VCX_OK;
}

bool vcx::solver_matches(vcx_solver s, vcx_mesh mesh, const vcx_physics* ph) {
  return s && s->mesh == mesh && same_scheme(s->ph, *ph);
}

// Check a physics struct against a mesh and pick its kernel table.
vcx_status vcx::check_physics(vcx_mesh mesh, const vcx_physics& ph, const double* E,
                              const KernelTable** kt_out) {
  const int nd = mesh->h.nd;
  if (ph.model != VCX_MODEL_GAS && ph.model != VCX_MODEL_DRIFT_DIFFUSION &&
      ph.model != VCX_MODEL_NAVIER_STOKES)
    return fail(VCX_E_ARG, "unknown model");
  if (ph.model == VCX_MODEL_NAVIER_STOKES) {
    for (int k = 0; k < ph.nspecies && k < VCX_MAX_SPECIES; ++k)
      if (!(ph.Wk[k] > 0.0) || !(ph.Sc[k] > 0.0))
        return fail(VCX_E_ARG, "Navier-Stokes species need positive molar masses and Schmidt numbers");
    if (!(ph.mu_ref >= 0.0) || !(ph.T_ref > 0.0) || !(ph.Pr > 0.0))
      return fail(VCX_E_ARG, "Navier-Stokes needs mu_ref >= 0, T_ref > 0, Pr > 0");
  }
  if (mesh->h.nv != nd + 1 && ph.model == VCX_MODEL_NAVIER_STOKES)
    return fail(VCX_E_ARG, "quadrilateral meshes support the gas and drift-diffusion models");
  if (ph.closure < 0 || ph.closure > 2) return fail(VCX_E_ARG, "closure must be 0, 1 or 2");
  if (ph.closure == 2 && (nd != 2 || mesh->h.axi || ph.model == VCX_MODEL_NAVIER_STOKES))
    return fail(VCX_E_ARG, "the interpolated boundary closure is defined on plane 2D meshes (gas and "
                           "drift-diffusion)");
  if (ph.rk_stages < 1 || ph.rk_stages > 4) return fail(VCX_E_ARG, "rk_stages must be 1..4");
  if (ph.predictor != 0 && ph.predictor != 1) return fail(VCX_E_ARG, "predictor must be 0 or 1");
  if (ph.predictor && (ph.model != VCX_MODEL_GAS || mesh->h.axi || ph.rk_stages != 1))
    return fail(VCX_E_ARG, "the MUSCL-Hancock predictor is defined for the gas model on plane meshes with "
                           "rk_stages = 1");
  if (ph.limiter < 0 || ph.limiter > 4) return fail(VCX_E_ARG, "unknown limiter");
  if (ph.precision != VCX_PREC_FP64 && ph.precision != VCX_PREC_MIXED)
    return fail(VCX_E_ARG, "unknown precision");
  if (ph.model == VCX_MODEL_GAS && ph.flux != VCX_FLUX_HLLC && ph.flux != VCX_FLUX_ROE)
    return fail(VCX_E_ARG, "unknown flux");
  if (ph.model == VCX_MODEL_DRIFT_DIFFUSION && ph.flux != VCX_FLUX_LLW && ph.flux != VCX_FLUX_SG)
    return fail(VCX_E_ARG, "drift-diffusion flux must be VCX_FLUX_LLW or VCX_FLUX_SG");
  if (!(ph.cfl > 0.0)) return fail(VCX_E_ARG, "cfl must be > 0");
  if (ph.model == VCX_MODEL_GAS && !(ph.gamma > 1.0)) return fail(VCX_E_ARG, "gamma must be > 1");
  if (ph.model == VCX_MODEL_DRIFT_DIFFUSION) {
    if (!E) return fail(VCX_E_ARG, "drift-diffusion needs the electric field E");
    for (int k = 0; k < ph.nspecies && k < VCX_MAX_SPECIES; ++k)
      if (ph.D[k] < 0.0) return fail(VCX_E_ARG, "negative diffusion coefficient");
  }
  const KernelTable* kt = pick_table(nd, mesh->h.nv, ph);
  if (!kt) return fail(VCX_E_ARG, "unsupported species count for this model");
  *kt_out = kt;
  return VCX_OK;
}

// Sizes, LDS footprints, fused-pass choice and launch shapes of a solver
// (host fields only; no device memory is touched).
vcx_status vcx::configure_solver(vcx_solver s, vcx_mesh mesh, const vcx_physics& ph, const KernelTable* kt) {
  const int nd = mesh->h.nd;
  s->mesh = mesh;
  s->ph = ph;
  s->nd = nd;
  s->nvar = ph.model == VCX_MODEL_DRIFT_DIFFUSION ? ph.nspecies : 2 + nd + ph.nspecies;
  s->nr = ph.model == VCX_MODEL_DRIFT_DIFFUSION ? s->nvar : s->nvar + 1;
  s->nw = kt->nw;
  s->ngf = kt->ngf;
  s->ldws = staged_row_stride(nd, ph);
  s->nws = s->ldws ? ns_staged_rows(nd, ph.nspecies, true) : 0;
  s->kt = kt;
  const DevMesh& d = mesh->d;
  // (the node-gradient pass takes no dynamic LDS)
  const bool nodeg = node_gradient(ph.model, nd, mesh->h.nv);
  if (nodeg && !d.has_ngrad) return fail(VCX_E_ARG, "the mesh has no node-gradient tables");
  s->lds_grad = nodeg ? 0 : kt->lds_grad(d.max_tile_nodes, d.max_tile_cells);
  if (ph.model == VCX_MODEL_NAVIER_STOKES && !(d.has_edges && d.has_ngrad))
    return fail(VCX_E_ARG, "the mesh has no tile-edge and node-gradient tables (created by the first "
                           "Navier-Stokes solver)");
  s->lds_flux = kt->lds_flux(d, ph.predictor);
  if (s->lds_grad > (size_t)mesh->lds_max || s->lds_flux > (size_t)mesh->lds_max) {
    const size_t need = std::max(s->lds_grad, s->lds_flux);
    return fail(VCX_E_ARG, "tile LDS footprint " + std::to_string(need) + " B exceeds the device limit " +
                               std::to_string(mesh->lds_max) +
                               " B for this model; create the mesh with smaller tiles");
  }
  // the fused gradient + flux pass where the mesh has extended tiles and
  // they fit the device's LDS
  s->lds_fused = kt->lds_fused(d);
  // the fused pass is for plane meshes; axisymmetric ones take the
  // gradient + flux passes, whose flux carries the face radii
  // (and the interpolated closure reads neighbours' gradients, complete only
  // after a separate gradient pass)
  // (the predictor and the Scharfetter-Gummel flux take the separate passes too)
  const bool sg = ph.model == VCX_MODEL_DRIFT_DIFFUSION && ph.flux == VCX_FLUX_SG;
  // Drift-diffusion meshes above kFusedMaxCells take the separate passes
  // (on simplices the node gradient with a node-major G, else the tile
  // gradient and the shared-node completion), which outrun the fused
  // pass once the launches are long, while the fused pass's two launches win
  // on small meshes.
  const bool big_dd = ph.model == VCX_MODEL_DRIFT_DIFFUSION && d.nc > kFusedMaxCells;
  s->fused = !d.axi && ph.closure != 2 && !ph.predictor && !sg && !big_dd && s->lds_fused > 0 &&
             s->lds_fused <= (size_t)mesh->lds_max;
  if (!s->fused) s->lds_fused = 0;
  s->dd_ngrad = ph.model == VCX_MODEL_DRIFT_DIFFUSION && !s->fused && d.has_ngrad;
  if (s->dd_ngrad) s->lds_grad = 0;
  if (std::max({s->lds_grad, s->lds_flux, s->lds_fused}) > 65536)
    VCX_TRY(kt->allow_lds(s->lds_grad, s->lds_flux, s->lds_fused));
  s->tile_block = std::min(256, ((d.max_tile_cells + 63) / 64) * 64);
  s->flux_block = ph.model == VCX_MODEL_NAVIER_STOKES
                      ? std::min(256, ((std::max(d.max_tile_cells, d.max_tile_edges) + 63) / 64) * 64)
                      : s->tile_block;
  s->node_blocks = (int)((d.nn + kNodeBlock - 1) / kNodeBlock);
  const int nupd = update_all(ph.model, nd) ? d.nn : d.nshared;
  s->nsh_blocks = std::max(1, (nupd + kNodeBlock - 1) / kNodeBlock);
  return VCX_OK;
}

extern "C" vcx_status vcx_solver_create(vcx_mesh mesh, const vcx_physics* phys, const double* E,
                                        vcx_solver* out) {
  if (!mesh || !phys || !out) return fail(VCX_E_ARG, "NULL argument");
  *out = nullptr;
  const vcx_physics& ph = *phys;
  const int nd = mesh->h.nd;
  const KernelTable* kt = nullptr;
  VCX_TRY(check_physics(mesh, ph, E, &kt));
  if (ph.model == VCX_MODEL_NAVIER_STOKES) VCX_TRY(ensure_tile_edges(mesh));
  if (ph.model == VCX_MODEL_DRIFT_DIFFUSION && mesh->h.nc > kFusedMaxCells && mesh->h.nv == nd + 1)
    VCX_TRY(ensure_node_gradient(mesh));
  vcx_solver s = new (std::nothrow) vcx_solver_s();
  if (!s) return fail(VCX_E_OOM, "host allocation failed");
  {
    vcx_status cs = configure_solver(s, mesh, ph, kt);
    if (cs != VCX_OK) {
      delete s;
      return cs;
    }
  }
  const DevMesh& d = mesh->d;
  const SolverSizes z = solver_sizes(d, nd, s->nvar, s->nr, s->nw, s->ngf, ph.model,
                                     staged_doubles((size_t)d.nn, s->ldws, nd, ph.nspecies, g_fp32(s)));
  s->bytes = z.bytes();
  vcx_status st = VCX_OK;
  auto chk = [&](vcx_status x) {
    if (st == VCX_OK) st = x;
  };
  chk(dmalloc(&s->W[0], z.W));
  chk(dmalloc(&s->W[1], z.W));
  if (z.WS) {
    chk(dmalloc(&s->WS[0], z.WS));
    chk(dmalloc(&s->WS[1], z.WS));
  }
  chk(dmalloc(&s->G, z.G));
  if (s->fused && ph.model == VCX_MODEL_DRIFT_DIFFUSION && ph.closure && d.nb > 0) s->gout = s->G;
  chk(dmalloc(&s->PG, z.PG));
  chk(dmalloc(&s->PR, z.PR));
  chk(dmalloc(&s->io, z.io));
  chk(dmalloc(&s->rbuf, z.io));
  chk(dmalloc(&s->part, z.part));
  chk(dmalloc(&s->sums_dev, z.sums));
  if (ph.closure == 2 && d.nb > 0) {
    chk(dmalloc(&s->cbuf, (size_t)d.nb * s->nvar));
    s->bytes += sizeof(double) * (size_t)d.nb * s->nvar;
  }
  s->node_blocks = z.node_blocks;
  s->nsh_blocks = z.nsh_blocks;
  if (st == VCX_OK && hipMalloc(reinterpret_cast<void**>(&s->lp), sizeof(DevLoop)) != hipSuccess)
    st = fail(VCX_E_OOM, "hipMalloc failed");
  if (st == VCX_OK &&
      hipHostMalloc(reinterpret_cast<void**>(&s->sc_host), sizeof(DevScalars), 0) != hipSuccess)
    st = fail(VCX_E_OOM, "hipHostMalloc failed");
  if (st == VCX_OK &&
      hipHostMalloc(reinterpret_cast<void**>(&s->sums_host), sizeof(double) * s->nr, 0) != hipSuccess)
    st = fail(VCX_E_OOM, "hipHostMalloc failed");
  if (st == VCX_OK && ph.model == VCX_MODEL_DRIFT_DIFFUSION) {
    chk(dmalloc(&s->E, z.E));
    if (st == VCX_OK) st = upload_field(s, E);
  }
  if (st == VCX_OK) st = reset_scalars(s, 0.0, false);
  if (st != VCX_OK) {
    free_solver(s);
    return st;
  }
  *out = s;
  return VCX_OK;
}

extern "C" vcx_status vcx_solver_destroy(vcx_solver s) {
  if (!s) return fail(VCX_E_ARG, "solver is NULL");
  (void)hipStreamSynchronize(s->mesh->stream);
  free_solver(s);
  return VCX_OK;
}

extern "C" int vcx_solver_nvar(vcx_solver s) { return s ? s->nvar : -1; }

static vcx_status copy_in(vcx_solver s, const double* src, size_t rows, int is_device) {
  const size_t bytes = sizeof(double) * rows * s->mesh->d.nn;
  VCX_HIP(hipMemcpyAsync(s->io, src, bytes, is_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                         s->mesh->stream));
  return VCX_OK;
}

// internal-order rows -> caller pointer (host or device), synchronised
static vcx_status copy_out(vcx_solver s, const double* src_internal, size_t rows, double* dst,
                           int is_device) {
  const int nn = s->mesh->d.nn;
  double* target = is_device ? dst : s->io;
  hipLaunchKernelGGL(k_scatter_rows, dim3((nn + 255) / 256), dim3(256), 0, s->mesh->stream,
                     s->mesh->d.perm, src_internal, target, nn, (int)rows);
  VCX_HIP(hipGetLastError());
  if (!is_device)
    VCX_HIP(hipMemcpyAsync(dst, s->io, sizeof(double) * rows * nn, hipMemcpyDeviceToHost,
                           s->mesh->stream));
  VCX_HIP(hipStreamSynchronize(s->mesh->stream));
  return VCX_OK;
}

extern "C" vcx_status vcx_state_upload(vcx_solver s, const double* U, int is_device) {
  if (!s || !U) return fail(VCX_E_ARG, "NULL argument");
  const DevMesh& d = s->mesh->d;
  VCX_TRY(copy_in(s, U, s->nvar, is_device));
  hipLaunchKernelGGL(k_gather_rows, dim3((d.nn + 255) / 256), dim3(256), 0, s->mesh->stream,
                     d.perm, (const double*)s->io, s->W[s->cur], d.nn, s->nvar);
  VCX_HIP(hipGetLastError());
  VCX_TRY(s->kt->aux(s, s->W[s->cur]));
  s->has_state = true;
  return reset_scalars(s, 0.0, true);
}

extern "C" vcx_status vcx_state_upload_primitive(vcx_solver s, const double* P, int is_device) {
  if (!s || !P) return fail(VCX_E_ARG, "NULL argument");
  const DevMesh& d = s->mesh->d;
  VCX_TRY(copy_in(s, P, s->nvar, is_device));
  hipLaunchKernelGGL(k_gather_rows, dim3((d.nn + 255) / 256), dim3(256), 0, s->mesh->stream,
                     d.perm, (const double*)s->io, s->W[s->cur], d.nn, s->nvar);
  VCX_HIP(hipGetLastError());
  VCX_TRY(s->kt->prim_to_cons(s, s->W[s->cur]));
  VCX_TRY(s->kt->aux(s, s->W[s->cur]));
  s->has_state = true;
  return reset_scalars(s, 0.0, true);
}

extern "C" vcx_status vcx_state_set_time(vcx_solver s, double t) {
  if (!s) return fail(VCX_E_ARG, "NULL solver");
  if (!s->has_state) return fail(VCX_E_STATE, "no state uploaded");
  return reset_scalars(s, t, true);
}

extern "C" vcx_status vcx_state_download(vcx_solver s, double* U, int is_device) {
  if (!s || !U) return fail(VCX_E_ARG, "NULL argument");
  if (!s->has_state) return fail(VCX_E_STATE, "no state uploaded");
  return copy_out(s, s->W[s->cur], s->nvar, U, is_device);
}

extern "C" vcx_status vcx_gradient(vcx_solver s, double* G, int is_device) {
  if (!s || !G) return fail(VCX_E_ARG, "NULL argument");
  if (!s->has_state) return fail(VCX_E_STATE, "no state uploaded");
  GradCtl gc{nullptr, 0, 0};
  VCX_TRY(s->kt->grad(s, s->W[s->cur], gc, true));
  VCX_TRY(s->kt->grad_complete(s));
  if (node_gradient(s->ph.model, s->nd, s->mesh->h.nv) || s->dd_ngrad) {
    // node-major gradient rows: their first nr * nd components
    const int nn = s->mesh->d.nn;
    double* target = is_device ? G : s->io;
    hipLaunchKernelGGL(k_scatter_node_rows, dim3((nn + 255) / 256), dim3(256), 0, s->mesh->stream,
                       s->mesh->d.perm, (const double*)s->G, target, nn, s->nr * s->nd, node_row(s->ngf * s->nd));
    VCX_HIP(hipGetLastError());
    if (!is_device)
      VCX_HIP(hipMemcpyAsync(G, s->io, sizeof(double) * (size_t)s->nr * s->nd * nn, hipMemcpyDeviceToHost,
                             s->mesh->stream));
    VCX_HIP(hipStreamSynchronize(s->mesh->stream));
    return VCX_OK;
  }
  return copy_out(s, s->G, (size_t)s->nr * s->nd, G, is_device);
}

extern "C" vcx_status vcx_residual(vcx_solver s, double dt, double* r, int is_device) {
  if (!s || !r) return fail(VCX_E_ARG, "NULL argument");
  if (!s->has_state) return fail(VCX_E_STATE, "no state uploaded");
  const double* Win = s->W[s->cur];
  Finish f = make_finish(s);
  f.Win = Win;
  f.rout = s->rbuf;
  f.residual_only = 1;
  if (s->fused) {
    FusedCtl fc{nullptr, 0, 0, s->gout};
    VCX_TRY(s->kt->fused(s, Win, f, fc, dt));
  } else {
    GradCtl gc{nullptr, 0, 0};
    VCX_TRY(s->kt->grad(s, Win, gc, false));
    if (s->ph.closure == 2) VCX_TRY(s->kt->closure2(s, f));
    VCX_TRY(s->kt->flux(s, Win, f, dt));
  }
  VCX_TRY(s->kt->update_shared(s, f));
  return copy_out(s, s->rbuf, s->nvar, r, is_device);
}

static vcx_status read_scalars(vcx_solver s) {
  // the state of the last launched step (parity spar ^ 1)
  VCX_HIP(hipMemcpyAsync(s->sc_host, &s->lp->s[s->spar ^ 1], sizeof(DevScalars), hipMemcpyDeviceToHost,
                         s->mesh->stream));
  VCX_HIP(hipStreamSynchronize(s->mesh->stream));
  return VCX_OK;
}

extern "C" vcx_status vcx_timestep(vcx_solver s, double* dt) {
  if (!s || !dt) return fail(VCX_E_ARG, "NULL argument");
  if (!s->has_state) return fail(VCX_E_STATE, "no state uploaded");
  VCX_TRY(s->kt->node_dt(s, s->W[s->cur]));
  hipLaunchKernelGGL(k_dt_query, dim3(1), dim3(256), 0, s->mesh->stream, s->lp);
  VCX_HIP(hipGetLastError());
  VCX_TRY(read_scalars(s));
  *dt = s->sc_host->dt_query;
  if (!(*dt > 0.0)) return fail(VCX_E_UNSTABLE, "non-physical state: no valid time step");
  return VCX_OK;
}

// end time of a host call, set in the state the next step starts from
__global__ void k_set_tend(DevLoop* lp, int par_prev, double t_end) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    lp->s[par_prev].t_end = t_end;
    lp->s[par_prev].steps_left = -1;
  }
}

static const double RK_ALPHA[5][5] = {
    {0, 0, 0, 0, 0},
    {0, 0, 0, 0, 0},
    {0, 0, 1.0 / 2.0, 0, 0},
    {0, 0, 1.0 / 3.0, 1.0 / 2.0, 0},
    {0, 0, 1.0 / 4.0, 1.0 / 3.0, 1.0 / 2.0},
};

// Enqueue one time step on the solver's stream: K stages of (gradient tile
// pass, flux tile pass, shared-node update).  The first gradient pass also
// reduces the previous pass's time-step candidates and commits the previous
// step; the last stage produces the candidates of the next step.
static vcx_status enqueue_step(vcx_solver s) {
  const int K = s->ph.rk_stages;
  double* Wn = s->W[s->cur];
  double* Wk = s->W[1 - s->cur];
  const int par = s->spar;
  Finish f = make_finish(s);
  f.sc = &s->lp->s[par];
  f.found = &s->lp->found[par];
  f.cand = s->lp->cand[par];
  f.Un = Wn;
  f.Wout = Wk;
  f.WSout = s->WS[1 - s->cur];
  for (int k = 1; k <= K; ++k) {
    const double* Win = k == 1 ? Wn : Wk;
    // stage k of K uses alpha_{k+1}; the last one is the full update
    f.Win = Win;
    f.alpha = k < K ? RK_ALPHA[K][k + 1] : 1.0;
    f.final_stage = k == K ? 1 : 0;
    if (s->fused) {
      // the first stage decides the step in every block; its shared-node
      // pass rolls the candidate slots over
      FusedCtl fc{s->lp, par, k == 1 ? 1 : 0, s->gout};
      f.roll = k == 1 ? s->lp : nullptr;
      f.roll_par = par;
      VCX_TRY(s->kt->fused(s, Win, f, fc, 0.0));
    } else {
      GradCtl gc{s->lp, par, k == 1 ? 1 : 0};
      VCX_TRY(s->kt->grad(s, Win, gc, false));
      if (s->ph.closure == 2) VCX_TRY(s->kt->closure2(s, f));
      VCX_TRY(s->kt->flux(s, Win, f, 0.0));
    }
    VCX_TRY(s->kt->update_shared(s, f));
  }
  s->cur = 1 - s->cur;
  s->spar ^= 1;
  return VCX_OK;
}

extern "C" vcx_status vcx_step(vcx_solver s, int nsteps, double t_end, double* t, double* dt_last) {
  if (!s) return fail(VCX_E_ARG, "NULL solver");
  if (nsteps < 0) return fail(VCX_E_ARG, "nsteps must be >= 0");
  if (!s->has_state) return fail(VCX_E_STATE, "no state uploaded");
  if (s->host_flag) return fail(VCX_E_UNSTABLE, "solver is in a failed state; upload a new state");
  const int cur0 = s->cur;
  const long long steps0 = s->steps_total;
  hipLaunchKernelGGL(k_set_tend, dim3(1), dim3(1), 0, s->mesh->stream, s->lp, s->spar ^ 1, t_end);
  VCX_HIP(hipGetLastError());
  const int chunk = t_end > 0.0 ? 16 : 256;
  int launched = 0;
  while (launched < nsteps) {
    const int n = std::min(chunk, nsteps - launched);
    for (int q = 0; q < n; ++q) VCX_TRY(enqueue_step(s));
    launched += n;
    hipLaunchKernelGGL(k_commit, dim3(1), dim3(1), 0, s->mesh->stream, s->lp, s->spar ^ 1);
    VCX_HIP(hipGetLastError());
    VCX_TRY(read_scalars(s));
    if (s->sc_host->flag) break;
    if (t_end > 0.0 && s->sc_host->t >= t_end) break;
  }
  if (launched == 0) VCX_TRY(read_scalars(s));
  const DevScalars& h = *s->sc_host;
  s->steps_total = h.steps;
  s->steps_last = h.steps - steps0;
  s->cur = (int)((cur0 + s->steps_last) % 2);
  if (t) *t = h.t;
  if (dt_last) *dt_last = h.last_dt;
  VCX_TRY(harvest(s));
  if (h.flag) {
    s->host_flag = h.flag;
    return fail(VCX_E_UNSTABLE, h.flag & 1 ? "state became non-finite or non-physical"
                                           : "no valid time step (non-physical state)");
  }
  return VCX_OK;
}

extern "C" int64_t vcx_steps_done(vcx_solver s) { return s ? s->steps_last : -1; }

extern "C" vcx_status vcx_state_time(vcx_solver s, double* t, double* dt_last) {
  if (!s) return fail(VCX_E_ARG, "NULL solver");
  if (t) *t = s->sc_host->t;
  if (dt_last) *dt_last = s->sc_host->last_dt;
  return VCX_OK;
}

// ---------------------------------------------------------------------------
// batch groups: the solves advanced together by one launch per kernel
// ---------------------------------------------------------------------------

template <typename T>
static vcx_status dev_array(T** p, int* cap, int need) {
  if (*cap >= need && *p) return VCX_OK;
  if (*p) (void)hipFree(*p);
  *p = nullptr;
  const int c = std::max(need, 2 * *cap);
  if (hipMalloc(reinterpret_cast<void**>(p), sizeof(T) * (size_t)std::max(c, 1)) != hipSuccess) {
    *cap = 0;
    return fail(VCX_E_OOM, "hipMalloc failed for batch tables");
  }
  *cap = c;
  return VCX_OK;
}

struct vcx::BatchGroup {
  hipStream_t stream = nullptr;   // where the group's work is enqueued
  hipStream_t cap = nullptr;      // private stream used only to capture graphs
  bool graphs = false;
  std::vector<vcx_solver> mem;
  std::vector<long long> steps0;  // member step counters when the table was built
  std::vector<int> phase0;        // member buffer parity when the table was built
  std::vector<int> spar0;         // member step parity when the table was built
  int q = 0;                      // batch steps enqueued since the table was built
  BatchRun br{};
  // device tables
  BatchEntry* tab = nullptr;
  int2* tile_map = nullptr;
  int2* grad_map = nullptr;
  int2* sh_map = nullptr;
  double* tend = nullptr;
  int* steps = nullptr;
  DevScalars* out = nullptr;
  DevScalars* out_host = nullptr;  // pinned
  int cap_tab = 0, cap_tiles = 0, cap_grad = 0, cap_sh = 0, cap_tend = 0, cap_steps = 0, cap_out = 0, cap_host = 0;
  hipGraphExec_t pair = nullptr;   // two batch steps (parities 0 and 1), captured once per table
  ~BatchGroup() {
    if (pair) (void)hipGraphExecDestroy(pair);
    for (void* p : {(void*)tab, (void*)tile_map, (void*)grad_map, (void*)sh_map, (void*)tend, (void*)steps,
                    (void*)out})
      if (p) (void)hipFree(p);
    if (out_host) (void)hipHostFree(out_host);
    if (cap) (void)hipStreamDestroy(cap);
  }
};

static BatchEntry entry_of(vcx_solver s) {
  BatchEntry e{};
  e.m = s->mesh->d;
  e.W[0] = s->W[0];
  e.W[1] = s->W[1];
  e.WS[0] = s->WS[0];
  e.WS[1] = s->WS[1];
  e.nws = s->nws;
  e.ldws = s->ldws;
  e.g32 = g_fp32(s) ? 1 : 0;
  e.G = s->G;
  e.PG = s->PG;
  e.PR = s->PR;
  e.E = s->E;
  e.lp = s->lp;
  e.gout = s->gout;
  e.spar = s->spar;
  e.phase = s->cur;
  return e;
}

// Enqueue batch step q (all K stages) on stream st.
static vcx_status batch_step(const BatchRun& br, hipStream_t st, int q, bool prof) {
  const int K = br.lead->ph.rk_stages;
  for (int k = 1; k <= K; ++k) {
    BatchStage bs{q, k, k == K ? 1 : 0, k < K ? RK_ALPHA[K][k + 1] : 1.0};
    VCX_TRY(br.lead->kt->batch_stage(br, st, bs, prof));
  }
  return VCX_OK;
}

vcx_status vcx::batch_create(hipStream_t stream, bool graphs, BatchGroup** out) {
  auto* g = new (std::nothrow) BatchGroup();
  if (!g) return fail(VCX_E_OOM, "host allocation failed");
  g->stream = stream;
  g->graphs = graphs;
  if (graphs && hipStreamCreateWithFlags(&g->cap, hipStreamNonBlocking) != hipSuccess) {
    delete g;
    return fail(VCX_E_HIP, "stream creation failed");
  }
  *out = g;
  return VCX_OK;
}

void vcx::batch_destroy(BatchGroup* g) {
  if (!g) return;
  (void)hipStreamSynchronize(g->stream);
  delete g;
}

size_t vcx::batch_size(const BatchGroup* g) { return g ? g->mem.size() : 0; }

vcx_status vcx::batch_set(BatchGroup* g, vcx_solver* ss, int n, const int* steps_left,
                          const double* t_end) {
  if (!g || n < 0 || (n > 0 && (!ss || !steps_left || !t_end))) return fail(VCX_E_ARG, "bad batch");
  if (g->pair) {
    (void)hipGraphExecDestroy(g->pair);
    g->pair = nullptr;
  }
  for (int i = 0; i < n; ++i)
    if (ss[i] && (ss[i]->mesh->h.axi || ss[i]->mesh->h.nv != ss[i]->mesh->h.nd + 1 ||
                  ss[i]->ph.closure == 2 || ss[i]->ph.predictor ||
                  (ss[i]->ph.model == VCX_MODEL_DRIFT_DIFFUSION && ss[i]->ph.flux == VCX_FLUX_SG)))
      return fail(VCX_E_ARG, "solvers on axisymmetric meshes, with the interpolated closure, the "
                             "predictor or the Scharfetter-Gummel flux are not batched");
  g->mem.assign(ss, ss + n);
  g->q = 0;
  if (n == 0) return VCX_OK;
  vcx_solver lead = ss[0];
  std::vector<BatchEntry> tab(n);
  std::vector<int2> tmap, gmap, smap;
  size_t lg = 0, lf = 0, lfu = 0;
  int block = 64, fblock = 64;
  g->steps0.resize(n);
  g->phase0.resize(n);
  g->spar0.resize(n);
  // each solve's reducer entry first (dispatched early), then the tiles
  for (int i = 0; i < n; ++i) tmap.push_back(make_int2(i, -1));
  gmap = tmap;
  for (int i = 0; i < n; ++i) {
    vcx_solver s = ss[i];
    tab[i] = entry_of(s);
    g->steps0[i] = s->steps_total;
    g->phase0[i] = s->cur;
    g->spar0[i] = s->spar;
    for (int t = 0; t < s->mesh->d.ntiles; ++t) tmap.push_back(make_int2(i, t));
    if (node_gradient(s->ph.model, s->nd, s->mesh->h.nv) || s->dd_ngrad)
      for (int b = 0; b < s->mesh->d.ng_nslices; ++b) gmap.push_back(make_int2(i, b));
    for (int b = 0; b < s->nsh_blocks; ++b) smap.push_back(make_int2(i, b));
    lg = std::max(lg, s->lds_grad);
    lf = std::max(lf, s->lds_flux);
    lfu = std::max(lfu, s->lds_fused);
    block = std::max(block, s->tile_block);
    fblock = std::max(fblock, s->flux_block);
  }
  const bool fused = lead->fused;
  const int lds_max = lead->mesh->lds_max;
  if (lg > (size_t)lds_max || lf > (size_t)lds_max || lfu > (size_t)lds_max)
    return fail(VCX_E_ARG, "batch LDS footprint too large");
  if (std::max({lg, lf, lfu}) > 65536) VCX_TRY(lead->kt->allow_lds(lg, lf, lfu));
  VCX_TRY(dev_array(&g->tab, &g->cap_tab, n));
  VCX_TRY(dev_array(&g->tend, &g->cap_tend, n));
  VCX_TRY(dev_array(&g->steps, &g->cap_steps, n));
  VCX_TRY(dev_array(&g->out, &g->cap_out, n));
  VCX_TRY(dev_array(&g->tile_map, &g->cap_tiles, (int)tmap.size()));
  VCX_TRY(dev_array(&g->grad_map, &g->cap_grad, (int)gmap.size()));
  VCX_TRY(dev_array(&g->sh_map, &g->cap_sh, (int)smap.size()));
  if (g->cap_host < n) {
    if (g->out_host) (void)hipHostFree(g->out_host);
    g->out_host = nullptr;
    g->cap_host = 0;
    if (hipHostMalloc(reinterpret_cast<void**>(&g->out_host), sizeof(DevScalars) * g->cap_out, 0) != hipSuccess)
      return fail(VCX_E_OOM, "hipHostMalloc failed for batch scalars");
    g->cap_host = g->cap_out;
  }
  // the members' own streams must be idle: the group's stream takes over
  for (vcx_solver s : g->mem) VCX_HIP(hipStreamSynchronize(s->mesh->stream));
  hipStream_t st = g->stream;
  VCX_HIP(hipMemcpyAsync(g->tab, tab.data(), sizeof(BatchEntry) * n, hipMemcpyHostToDevice, st));
  VCX_HIP(hipMemcpyAsync(g->tile_map, tmap.data(), sizeof(int2) * tmap.size(), hipMemcpyHostToDevice, st));
  VCX_HIP(hipMemcpyAsync(g->grad_map, gmap.data(), sizeof(int2) * gmap.size(), hipMemcpyHostToDevice, st));
  VCX_HIP(hipMemcpyAsync(g->sh_map, smap.data(), sizeof(int2) * smap.size(), hipMemcpyHostToDevice, st));
  VCX_HIP(hipMemcpyAsync(g->tend, t_end, sizeof(double) * n, hipMemcpyHostToDevice, st));
  VCX_HIP(hipMemcpyAsync(g->steps, steps_left, sizeof(int) * n, hipMemcpyHostToDevice, st));
  hipLaunchKernelGGL(k_batch_control, dim3((n + 63) / 64), dim3(64), 0, st, (const BatchEntry*)g->tab, n,
                     (const double*)g->tend, (const int*)g->steps);
  VCX_HIP(hipGetLastError());
  // host arrays above are the caller's: wait for the copies before returning
  VCX_HIP(hipStreamSynchronize(st));
  BatchRun& br = g->br;
  br.lead = lead;
  br.tab = g->tab;
  br.tile_map = g->tile_map;
  br.ntile_blocks = (int)tmap.size();
  br.grad_map = g->grad_map;
  br.ngrad_blocks = (int)gmap.size();
  br.dd_ngrad = lead->dd_ngrad;
  br.sh_map = g->sh_map;
  br.nsh_blocks = (int)smap.size();
  br.lds_grad = lg;
  br.fused = fused;
  br.lds_flux = fused ? lfu : lf;
  br.tile_block = std::min(256, block);
  br.flux_block = std::min(256, fblock);
  if (g->graphs && !lead->prof) {
    hipGraph_t graph = nullptr;
    VCX_HIP(hipStreamBeginCapture(g->cap, hipStreamCaptureModeThreadLocal));
    vcx_status s0 = batch_step(br, g->cap, 0, false);
    if (s0 == VCX_OK) s0 = batch_step(br, g->cap, 1, false);
    hipError_t e = hipStreamEndCapture(g->cap, &graph);
    if (s0 != VCX_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return s0;
    }
    if (e != hipSuccess) return fail(VCX_E_HIP, std::string("graph capture failed: ") + hipGetErrorString(e));
    e = hipGraphInstantiate(&g->pair, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) {
      g->pair = nullptr;
      return fail(VCX_E_HIP, std::string("graph instantiation failed: ") + hipGetErrorString(e));
    }
  }
  return VCX_OK;
}

vcx_status vcx::batch_run(BatchGroup* g, int nsteps) {
  if (!g || g->mem.empty() || nsteps <= 0) return VCX_OK;
  const bool prof = g->br.lead->prof;
  int left = nsteps;
  // graph replays need an even step counter (the graph holds parities 0, 1)
  if (g->pair && (g->q & 1) && left > 0) {
    VCX_TRY(batch_step(g->br, g->stream, g->q, prof));
    g->q += 1;
    left -= 1;
  }
  if (g->pair) {
    for (; left >= 2; left -= 2, g->q += 2) VCX_HIP(hipGraphLaunch(g->pair, g->stream));
  }
  for (; left > 0; --left, ++g->q) VCX_TRY(batch_step(g->br, g->stream, g->q, prof));
  return VCX_OK;
}

vcx_status vcx::batch_sync(BatchGroup* g, std::vector<int>* ended) {
  if (ended) ended->clear();
  if (!g || g->mem.empty()) return VCX_OK;
  const int n = (int)g->mem.size();
  hipLaunchKernelGGL(k_batch_commit, dim3((n + 63) / 64), dim3(64), 0, g->stream, (const BatchEntry*)g->tab,
                     n, g->q, g->out);
  VCX_HIP(hipGetLastError());
  VCX_HIP(hipMemcpyAsync(g->out_host, g->out, sizeof(DevScalars) * n, hipMemcpyDeviceToHost, g->stream));
  VCX_HIP(hipStreamSynchronize(g->stream));
  for (int i = 0; i < n; ++i) {
    vcx_solver s = g->mem[i];
    const DevScalars& h = g->out_host[i];
    *s->sc_host = h;
    s->spar = (g->spar0[i] + g->q) & 1;
    s->steps_last = h.steps - s->steps_total;
    s->steps_total = h.steps;
    s->cur = (int)((g->phase0[i] + (h.steps - g->steps0[i])) % 2);
    if (h.flag) s->host_flag = h.flag;
    if (ended) ended->push_back(h.flag != 0 || h.steps_left == 0 || (h.t_end > 0.0 && h.t >= h.t_end));
  }
  VCX_TRY(harvest(g->br.lead));
  return VCX_OK;
}

vcx_status vcx::solver_footprint(vcx_mesh mesh, const vcx_physics* ph, size_t* bytes) {
  if (!mesh || !ph || !bytes) return fail(VCX_E_ARG, "NULL argument");
  const KernelTable* kt = pick_table(mesh->h.nd, mesh->h.nv, *ph);
  if (!kt) return fail(VCX_E_ARG, "unsupported model / species count");
  const int nd = mesh->h.nd;
  const int nvar = ph->model == VCX_MODEL_DRIFT_DIFFUSION ? ph->nspecies : 2 + nd + ph->nspecies;
  const int nr = ph->model == VCX_MODEL_DRIFT_DIFFUSION ? nvar : nvar + 1;
  const bool ws32 = ph->model == VCX_MODEL_NAVIER_STOKES && ph->precision == VCX_PREC_MIXED;
  *bytes = solver_sizes(mesh->d, nd, nvar, nr, kt->nw, kt->ngf, ph->model,
                        staged_doubles((size_t)mesh->d.nn, staged_row_stride(nd, *ph), nd, ph->nspecies, ws32))
               .bytes();
  return VCX_OK;
}

bool vcx::batch_compatible(vcx_solver a, vcx_solver b) {
  return a->kt == b->kt && a->fused == b->fused && a->dd_ngrad == b->dd_ngrad && same_scheme(a->ph, b->ph);
}

vcx_status vcx::set_error(vcx_status s, const char* msg) { return fail(s, msg ? msg : ""); }
int vcx::mesh_ndim(vcx_mesh m) { return m ? m->h.nd : 0; }
int64_t vcx::mesh_nnodes(vcx_mesh m) { return m ? m->d.nn : 0; }
const vcx::HostMesh* vcx::mesh_host(vcx_mesh m) { return m ? &m->h : nullptr; }
bool vcx::mesh_axisymmetric(vcx_mesh m) { return m && m->h.axi; }
bool vcx::mesh_simplex(vcx_mesh m) { return m && m->h.nv == m->h.nd + 1; }
hipStream_t vcx::mesh_stream(vcx_mesh m) { return m ? m->stream : nullptr; }
const int32_t* vcx::mesh_perm_device(vcx_mesh m) { return m ? m->d.perm : nullptr; }
int vcx::solver_failed(vcx_solver s) { return s ? s->host_flag : 0; }

extern "C" vcx_status vcx_solver_footprint(vcx_mesh mesh, const vcx_physics* phys, size_t* bytes) {
  return vcx::solver_footprint(mesh, phys, bytes);
}

static vcx_status solve_batch(vcx_solver* ss, int n, const int* nsteps, const double* t_end, bool graphs) {
  if (!ss || n <= 0 || !nsteps || !t_end) return fail(VCX_E_ARG, "NULL argument or empty batch");
  for (int i = 0; i < n; ++i) {
    if (!ss[i]) return fail(VCX_E_ARG, "NULL solver in batch");
    if (!ss[i]->has_state) return fail(VCX_E_STATE, "batch member without a state");
    if (ss[i]->host_flag) return fail(VCX_E_UNSTABLE, "batch member in a failed state");
    if (nsteps[i] < 0) return fail(VCX_E_ARG, "nsteps must be >= 0");
    if (ss[i]->mesh->h.axi) return fail(VCX_E_ARG, "solvers on axisymmetric meshes are not batched");
    if (ss[i]->mesh->h.nv != ss[i]->mesh->h.nd + 1)
      return fail(VCX_E_ARG, "solvers on quadrilateral meshes are not batched");
    if (ss[i]->ph.closure == 2) return fail(VCX_E_ARG, "solvers with the interpolated closure are not batched");
    if (ss[i]->ph.predictor) return fail(VCX_E_ARG, "solvers with the MUSCL-Hancock predictor are not batched");
    if (ss[i]->ph.model == VCX_MODEL_DRIFT_DIFFUSION && ss[i]->ph.flux == VCX_FLUX_SG)
      return fail(VCX_E_ARG, "solvers with the Scharfetter-Gummel flux are not batched");
    if (!batch_compatible(ss[i], ss[0]))
      return fail(VCX_E_ARG, "batch members must share the model and scheme parameters");
    for (int j = 0; j < i; ++j)
      if (ss[j] == ss[i]) return fail(VCX_E_ARG, "a solver appears twice in the batch");
  }
  BatchGroup* g = nullptr;
  VCX_TRY(batch_create(ss[0]->mesh->stream, graphs, &g));
  std::unique_ptr<BatchGroup, void (*)(BatchGroup*)> hold(g, batch_destroy);
  std::vector<long long> steps0(n);
  for (int i = 0; i < n; ++i) steps0[i] = ss[i]->steps_total;
  VCX_TRY(batch_set(g, ss, n, nsteps, t_end));
  int maxsteps = 0;
  for (int i = 0; i < n; ++i) maxsteps = std::max(maxsteps, nsteps[i]);
  std::vector<int> ended(n, 0);
  int q = 0;
  do {
    // a chunk ends where the first live member's budget does (host checks in
    // between); members with an end time are checked every 16 steps
    int c = 256;
    for (int i = 0; i < n; ++i) {
      const long long left = nsteps[i] - (ss[i]->steps_total - steps0[i]);
      if (ended[i] || left <= 0) continue;
      c = (int)std::min<long long>(c, left);
      if (t_end[i] > 0.0) c = std::min(c, 16);
    }
    c = std::max(1, std::min(c, maxsteps - q));
    VCX_TRY(batch_run(g, c));
    q += c;
    VCX_TRY(batch_sync(g, &ended));
  } while (q < maxsteps && std::count(ended.begin(), ended.end(), 0) > 0);
  bool any_fail = false;
  for (int i = 0; i < n; ++i) {
    ss[i]->steps_last = ss[i]->steps_total - steps0[i];
    any_fail = any_fail || ss[i]->host_flag != 0;
  }
  if (any_fail) return fail(VCX_E_UNSTABLE, "at least one batch member became unstable");
  return VCX_OK;
}

extern "C" vcx_status vcx_solve_batch(vcx_solver* ss, int n, const int* nsteps, const double* t_end) {
  return solve_batch(ss, n, nsteps, t_end, true);
}

extern "C" vcx_status vcx_solve_batch_eager(vcx_solver* ss, int n, const int* nsteps, const double* t_end) {
  return solve_batch(ss, n, nsteps, t_end, false);
}

extern "C" vcx_status vcx_conservation_sums(vcx_solver s, double* sums) {
  if (!s || !sums) return fail(VCX_E_ARG, "NULL argument");
  if (!s->has_state) return fail(VCX_E_STATE, "no state uploaded");
  const DevMesh& d = s->mesh->d;
  hipLaunchKernelGGL(k_sums_partial, dim3(256), dim3(256), 0, s->mesh->stream,
                     (const double*)s->W[s->cur], d.vupd, d.nn, s->nvar, s->part);
  hipLaunchKernelGGL(k_sums_final, dim3(1), dim3(256), 0, s->mesh->stream, (const double*)s->part,
                     256, s->nvar, s->sums_dev);
  VCX_HIP(hipGetLastError());
  VCX_HIP(hipMemcpyAsync(s->sums_host, s->sums_dev, sizeof(double) * s->nvar, hipMemcpyDeviceToHost,
                         s->mesh->stream));
  VCX_HIP(hipStreamSynchronize(s->mesh->stream));
  std::memcpy(sums, s->sums_host, sizeof(double) * s->nvar);
  return VCX_OK;
}

extern "C" vcx_status vcx_profile_enable(vcx_solver s, int enable) {
  if (!s) return fail(VCX_E_ARG, "NULL solver");
  VCX_TRY(harvest(s));
  s->prof = enable != 0;
  s->acc.clear();
  return VCX_OK;
}

extern "C" vcx_status vcx_profile_query(vcx_solver s, const char* kernel, int64_t* count,
                                        double* total_ms) {
  if (!s || !kernel || !count || !total_ms) return fail(VCX_E_ARG, "NULL argument");
  VCX_TRY(harvest(s));
  auto it = s->acc.find(kernel);
  *count = it == s->acc.end() ? 0 : it->second.first;
  *total_ms = it == s->acc.end() ? 0.0 : it->second.second;
  return VCX_OK;
}

extern "C" const char* vcx_last_error(void) { return g_err.c_str(); }
