// Host-side mesh preprocessing: validation, orientation, median-dual nodal
// volumes, boundary node normals, space-filling-curve renumbering and the
// fixed cell tiles with their deterministic gather tables.
//
// Geometry follows Sec. "Nomenclature and notations" of the paper: the node
// normal S_k of a simplex is the outward area vector of the face opposite k,
// which equals -n_d V grad(lambda_k) with lambda_k the barycentric coordinate
// of vertex k; the boundary node normal S_i^b gives every boundary face's
// area vector in equal shares to its n_d nodes.
#include "vcx_mesh.h"

#include <algorithm>
#include <array>
#include <cmath>
#include <numeric>

namespace vcx {

TileLimits default_tile_limits(int nd) {
  if (nd == 2) return {256, 192};
  return {128, 96};
}


namespace {

uint64_t spread_bits(uint64_t v, int nd) {
  // interleave the low 21 bits of v with (nd - 1) zero bits between them
  uint64_t r = 0;
  for (int b = 0; b < 21; ++b) r |= ((v >> b) & 1ull) << (b * nd);
  return r;
}

uint64_t morton(const double* p, const double* lo, const double* span, int nd) {
  uint64_t code = 0;
  for (int d = 0; d < nd; ++d) {
    double t = span[d] > 0 ? (p[d] - lo[d]) / span[d] : 0.0;
    t = std::min(std::max(t, 0.0), 1.0);
    uint64_t q = (uint64_t)(t * ((1u << 21) - 1));
    code |= spread_bits(q, nd) << d;
  }
  return code;
}

// relative vertex coordinates e_k = X_k - X_0 of a cell, k = 1..nv-1
void relative_coords(const HostMesh& m, const double* x, const int64_t* v, uint32_t code,
                     double e[3][3]) {
  for (int k = 1; k < m.nv; ++k)
    for (int d = 0; d < m.nd; ++d) {
      double s = shift_of(code, k, d, m.nd);
      e[k - 1][d] = x[(int64_t)d * m.nn + v[k]] + s * m.period[d] - x[(int64_t)d * m.nn + v[0]];
    }
}

double signed_measure(int nd, const double e[3][3]) {
  if (nd == 2) return e[0][0] * e[1][1] - e[0][1] * e[1][0];
  return e[0][0] * (e[1][1] * e[2][2] - e[1][2] * e[2][1]) -
         e[0][1] * (e[1][0] * e[2][2] - e[1][2] * e[2][0]) +
         e[0][2] * (e[1][0] * e[2][1] - e[1][1] * e[2][0]);
}

// node normals of a positively oriented simplex from its relative coordinates
void node_normals(int nd, const double e[3][3], double S[4][3]) {
  if (nd == 2) {
    S[1][0] = -e[1][1]; S[1][1] = e[1][0];
    S[2][0] = e[0][1];  S[2][1] = -e[0][0];
    S[0][0] = -S[1][0] - S[2][0];
    S[0][1] = -S[1][1] - S[2][1];
    return;
  }
  auto cross = [](const double* a, const double* b, double* c) {
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
  };
  double c[3];
  cross(e[1], e[2], c);
  for (int d = 0; d < 3; ++d) S[1][d] = -0.5 * c[d];
  cross(e[2], e[0], c);
  for (int d = 0; d < 3; ++d) S[2][d] = -0.5 * c[d];
  cross(e[0], e[1], c);
  for (int d = 0; d < 3; ++d) S[3][d] = -0.5 * c[d];
  for (int d = 0; d < 3; ++d) S[0][d] = -(S[1][d] + S[2][d] + S[3][d]);
}

}  // namespace

// Tiles of consecutive cells, each closed at lim.max_cells cells or
// lim.max_nodes distinct nodes, with their slot, incidence and run tables.
std::string build_tiling(const HostMesh& m, TileLimits lim, Tiling& out) {
  const int nv = m.nv;
  const int64_t nn = m.nn, nc = m.nc;
  out = Tiling();
  std::vector<int64_t> stamp(nn, -1);
  out.tile_cell.push_back(0);
  int64_t tcount = 0, ncount = 0;
  for (int64_t c = 0; c < nc; ++c) {
    int fresh = 0;
    for (int k = 0; k < nv; ++k)
      if (stamp[m.cell[(size_t)k * nc + c]] != (int64_t)out.tile_cell.size() - 1) ++fresh;
    if (tcount > 0 && (tcount + 1 > lim.max_cells || ncount + fresh > lim.max_nodes)) {
      out.tile_cell.push_back((int32_t)c);
      tcount = 0;
      ncount = 0;
      fresh = nv;
    }
    int64_t t = (int64_t)out.tile_cell.size() - 1;
    for (int k = 0; k < nv; ++k) {
      int32_t i = m.cell[(size_t)k * nc + c];
      if (stamp[i] != t) { stamp[i] = t; ++ncount; }
    }
    ++tcount;
  }
  out.tile_cell.push_back((int32_t)nc);
  int64_t T = out.ntiles();

  out.lconn.resize((size_t)nv * nc);
  out.tile_slot.assign(1, 0);
  std::vector<int32_t> local(nn, -1);
  std::vector<int32_t> tnodes;
  std::vector<std::vector<uint16_t>> tinc;
  out.slot_inc.assign(1, 0);
  for (int64_t t = 0; t < T; ++t) {
    int32_t c0 = out.tile_cell[t], c1 = out.tile_cell[t + 1];
    tnodes.clear();
    for (int32_t c = c0; c < c1; ++c)
      for (int k = 0; k < nv; ++k) tnodes.push_back(m.cell[(size_t)k * nc + c]);
    std::sort(tnodes.begin(), tnodes.end());
    tnodes.erase(std::unique(tnodes.begin(), tnodes.end()), tnodes.end());
    for (size_t q = 0; q < tnodes.size(); ++q) local[tnodes[q]] = (int32_t)q;
    tinc.assign(tnodes.size(), {});
    for (int32_t c = c0; c < c1; ++c)
      for (int k = 0; k < nv; ++k) {
        int32_t l = local[m.cell[(size_t)k * nc + c]];
        out.lconn[(size_t)k * nc + c] = (uint16_t)l;
        tinc[l].push_back((uint16_t)(((c - c0) << 2) | k));
      }
    for (size_t q = 0; q < tnodes.size(); ++q) {
      out.slot_node.push_back(tnodes[q]);
      for (uint16_t code : tinc[q]) out.inc.push_back(code);
      out.slot_inc.push_back((int32_t)out.inc.size());
    }
    out.tile_slot.push_back((int32_t)out.slot_node.size());
    out.max_tile_cells = std::max(out.max_tile_cells, (int)(c1 - c0));
    out.max_tile_nodes = std::max(out.max_tile_nodes, (int)tnodes.size());
  }

  // ---- node -> slots (ascending tile order)
  int64_t P = out.nslots();
  out.node_slot.assign(nn + 1, 0);
  for (int64_t s = 0; s < P; ++s) out.node_slot[out.slot_node[s] + 1]++;
  for (int64_t i = 0; i < nn; ++i) out.node_slot[i + 1] += out.node_slot[i];
  out.slots_of.resize(P);
  std::vector<int32_t> fill(out.node_slot.begin(), out.node_slot.end() - 1);
  for (int64_t s = 0; s < P; ++s) out.slots_of[fill[out.slot_node[s]]++] = (int32_t)s;
  for (int64_t i = 0; i < nn; ++i)
    if (out.node_slot[i + 1] == out.node_slot[i]) return "node not referenced by any cell";
  // nodes split over several tiles: gathered through partial sums
  for (int64_t i = 0; i < nn; ++i)
    if (out.node_slot[i + 1] - out.node_slot[i] > 1) out.shared.push_back((int32_t)i);
  out.slot_run.resize(2 * P);
  for (int64_t s = 0; s < P; ++s) {
    int32_t g = out.slot_node[s];
    out.slot_run[2 * s] = out.node_slot[g];
    out.slot_run[2 * s + 1] = out.node_slot[g + 1];
    if (out.node_slot[g + 1] - out.node_slot[g] > 1) out.slot_node[s] = ~g;
  }

  return "";
}

// Node-gradient tables: neighbours j != i of each node in ascending order
// and C_ij = sum over the cells c holding i and j of S_j^c, accumulated in
// ascending cell order; then the 64-node slices.
std::string build_node_gradient(HostMesh& m) {
  const int nd = m.nd, nv = m.nv;
  const int64_t nn = m.nn, nc = m.nc;
  if (nv != nd + 1) return "node-gradient tables are built for simplices";
  // cells around each node, ascending
  std::vector<int64_t> cs(nn + 1, 0);
  for (int64_t c = 0; c < nc; ++c)
    for (int k = 0; k < nv; ++k) cs[m.cell[(size_t)k * nc + c] + 1]++;
  for (int64_t i = 0; i < nn; ++i) cs[i + 1] += cs[i];
  std::vector<int32_t> cells_of((size_t)cs[nn]);
  {
    std::vector<int64_t> fill(cs.begin(), cs.end() - 1);
    for (int64_t c = 0; c < nc; ++c)
      for (int k = 0; k < nv; ++k) cells_of[fill[m.cell[(size_t)k * nc + c]]++] = (int32_t)c;
  }
  // neighbour lists (CSR) and their coefficients
  std::vector<int64_t> np(nn + 1, 0);
  std::vector<int32_t> nb;
  std::vector<int32_t> tmp;
  for (int64_t i = 0; i < nn; ++i) {
    tmp.clear();
    for (int64_t q = cs[i]; q < cs[i + 1]; ++q)
      for (int k = 0; k < nv; ++k) tmp.push_back(m.cell[(size_t)k * nc + cells_of[q]]);
    std::sort(tmp.begin(), tmp.end());
    tmp.erase(std::unique(tmp.begin(), tmp.end()), tmp.end());
    // the node itself is left out: a simplex's node normals sum to zero, so
    // its coefficient is minus the sum of the others and the gradient takes
    // the differences W_j - W_i instead
    tmp.erase(std::lower_bound(tmp.begin(), tmp.end(), (int32_t)i));
    nb.insert(nb.end(), tmp.begin(), tmp.end());
    np[i + 1] = (int64_t)nb.size();
  }
  std::vector<double> cv((size_t)nd * nb.size(), 0.0);  // [entry][nd]
  for (int64_t i = 0; i < nn; ++i) {
    const int32_t* row = nb.data() + np[i];
    const int64_t deg = np[i + 1] - np[i];
    for (int64_t q = cs[i]; q < cs[i + 1]; ++q) {
      const int32_t c = cells_of[q];
      int64_t v[4];
      for (int k = 0; k < nv; ++k) v[k] = m.cell[(size_t)k * nc + c];
      double e[3][3], S[4][3];
      relative_coords(m, m.x.data(), v, m.shift[c], e);
      node_normals(nd, e, S);
      for (int k = 0; k < nv; ++k) {
        if (v[k] == i) continue;
        const int64_t at = std::lower_bound(row, row + deg, (int32_t)v[k]) - row;
        for (int d = 0; d < nd; ++d) cv[(size_t)(np[i] + at) * nd + d] += S[k][d];
      }
    }
  }
  // slices of kNgSlice nodes, padded to the slice's largest count
  const int W = HostMesh::kNgSlice;
  const int64_t ns = (nn + W - 1) / W;
  m.ng_off.assign(ns + 1, 0);
  for (int64_t sl = 0; sl < ns; ++sl) {
    int64_t w = 0;
    for (int64_t i = sl * W; i < std::min(nn, (sl + 1) * W); ++i) w = std::max(w, np[i + 1] - np[i]);
    m.ng_off[sl + 1] = m.ng_off[sl] + w * W;
  }
  const int64_t tot = m.ng_off[ns];
  m.ng_nbr.assign(tot, 0);
  m.ng_c.assign((size_t)nd * tot, 0.0);
  for (int64_t sl = 0; sl < ns; ++sl) {
    const int64_t w = (m.ng_off[sl + 1] - m.ng_off[sl]) / W;
    for (int l = 0; l < W; ++l) {
      const int64_t i = sl * W + l;
      for (int64_t k = 0; k < w; ++k) {
        const int64_t at = m.ng_off[sl] + k * W + l;
        if (i < nn && k < np[i + 1] - np[i]) {
          m.ng_nbr[at] = nb[np[i] + k];
          for (int d = 0; d < nd; ++d) m.ng_c[(size_t)d * tot + at] = cv[(size_t)(np[i] + k) * nd + d];
        } else {
          m.ng_nbr[at] = (int32_t)std::min(i, nn - 1);  // C = 0
        }
      }
    }
  }
  m.has_ngrad = true;
  return "";
}

std::string preprocess_mesh(int nd, int64_t nn, const double* xyz, int64_t nc, int nv,
                            const int64_t* cells, const double* period, TileLimits lim,
                            HostMesh& m, int* code, bool axisymmetric) {
  *code = -1;
  if (nd != 2 && nd != 3) return "ndim must be 2 or 3";
  if (nv != nd + 1 && !(nd == 2 && nv == 4))
    return "cells must be simplices (nv = ndim + 1) or, in 2D, quadrilaterals (nv = 4)";
  if (nn <= 0 || nc <= 0 || !xyz || !cells) return "empty mesh or NULL array";
  if (nn >= (int64_t)INT32_MAX || nc * nv >= (int64_t)INT32_MAX) return "mesh too large for 32-bit indices";
  if (lim.max_cells < 1 || lim.max_cells > 1024 || lim.max_nodes < nv || lim.max_nodes > 4096)
    return "tile limits out of range";
  m = HostMesh();
  const bool quad = nv == 4 && nd == 2;
  m.nd = nd; m.nv = nv; m.ne = quad ? 4 : (nd == 2 ? 3 : 6); m.nn = nn; m.nc = nc; m.lim = lim;
  for (int d = 0; d < nd; ++d) {
    double L = period ? period[d] : 0.0;
    if (!(L >= 0.0) || !std::isfinite(L)) return "period entries must be finite and >= 0";
    m.period[d] = L;
    if (L > 0.0) m.has_period = true;
  }
  for (int64_t q = 0; q < (int64_t)nd * nn; ++q)
    if (!std::isfinite(xyz[q])) return "non-finite coordinate";
  if (axisymmetric) {
    if (nd != 2) return "axisymmetric meshes are two-dimensional (x, r)";
    if (m.period[1] > 0.0) return "the radius of an axisymmetric mesh cannot be periodic";
    for (int64_t i = 0; i < nn; ++i)
      if (xyz[nn + i] < 0.0) return "axisymmetric meshes need r >= 0";
    m.axi = true;
  }

  // ---- connectivity, periodic images, orientation, volumes (caller order)
  *code = -2;
  std::vector<int64_t> cv((size_t)nc * nv);
  std::vector<uint32_t> sh(nc, 0u);
  std::vector<double> vol(nc);
  double vmax = 0.0;
  for (int64_t c = 0; c < nc; ++c) {
    int64_t* v = &cv[(size_t)c * nv];
    for (int k = 0; k < nv; ++k) {
      v[k] = cells[(int64_t)k * nc + c];
      if (v[k] < 0 || v[k] >= nn) return "cell index out of range";
      for (int q = 0; q < k; ++q)
        if (v[q] == v[k]) return "cell repeats a node";
    }
    uint32_t s = 0;
    for (int k = 1; k < nv; ++k)
      for (int d = 0; d < nd; ++d) {
        if (m.period[d] <= 0.0) continue;
        double dx = xyz[(int64_t)d * nn + v[k]] - xyz[(int64_t)d * nn + v[0]];
        double img = -std::nearbyint(dx / m.period[d]);
        if (std::fabs(img) > 1.0) return "periodic cell spans more than one box length";
        if (img == 1.0) s |= 1u << (2 * ((k - 1) * nd + d));
        if (img == -1.0) s |= 2u << (2 * ((k - 1) * nd + d));
      }
    double e[3][3];
    relative_coords(m, xyz, v, s, e);
    if (quad) {
      // twice the signed area (shoelace from vertex 0); a clockwise cell is
      // reversed (vertices 1 and 3 swap, with their periodic images)
      auto area2 = [](const double (&q)[3][3]) {
        return (q[0][0] * q[1][1] - q[0][1] * q[1][0]) + (q[1][0] * q[2][1] - q[1][1] * q[2][0]);
      };
      double a2 = area2(e);
      if (a2 < 0.0) {
        std::swap(v[1], v[3]);
        const uint32_t f1 = s & 0xFu, f3 = (s >> 8) & 0xFu;
        s = (s & ~0xF0Fu) | f3 | (f1 << 8);
        relative_coords(m, xyz, v, s, e);
        a2 = area2(e);
      }
      // convex: every corner turns counter-clockwise
      const double P[4][2] = {{0.0, 0.0}, {e[0][0], e[0][1]}, {e[1][0], e[1][1]}, {e[2][0], e[2][1]}};
      for (int k = 0; k < 4; ++k) {
        const double* p0 = P[k];
        const double* p1 = P[(k + 1) % 4];
        const double* p2 = P[(k + 2) % 4];
        const double cr = (p1[0] - p0[0]) * (p2[1] - p1[1]) - (p1[1] - p0[1]) * (p2[0] - p1[0]);
        if (!(cr > 0.0)) return "non-convex or degenerate quadrilateral";
      }
      sh[c] = s;
      vol[c] = 0.5 * a2;
      vmax = std::max(vmax, vol[c]);
      continue;
    }
    double det = signed_measure(nd, e);
    if (det < 0.0) {
      // reorient: swap vertices 1 and 2 together with their periodic images
      std::swap(v[1], v[2]);
      uint32_t s1 = (s >> 0) & ((1u << (2 * nd)) - 1u);
      uint32_t s2 = (s >> (2 * nd)) & ((1u << (2 * nd)) - 1u);
      s = (s & ~((1u << (4 * nd)) - 1u)) | s2 | (s1 << (2 * nd));
      relative_coords(m, xyz, v, s, e);
      det = signed_measure(nd, e);
    }
    sh[c] = s;
    vol[c] = det / (nd == 2 ? 2.0 : 6.0);
    vmax = std::max(vmax, vol[c]);
  }
  for (int64_t c = 0; c < nc; ++c)
    if (!(vol[c] > 1e-12 * vmax)) return "degenerate (zero-volume) cell";

  // ---- space-filling-curve order of nodes
  double lo[3], hi[3], span[3];
  for (int d = 0; d < nd; ++d) {
    lo[d] = INFINITY; hi[d] = -INFINITY;
    for (int64_t i = 0; i < nn; ++i) {
      lo[d] = std::min(lo[d], xyz[(int64_t)d * nn + i]);
      hi[d] = std::max(hi[d], xyz[(int64_t)d * nn + i]);
    }
    span[d] = hi[d] - lo[d];
  }
  std::vector<uint64_t> key(nn);
  for (int64_t i = 0; i < nn; ++i) {
    double p[3];
    for (int d = 0; d < nd; ++d) p[d] = xyz[(int64_t)d * nn + i];
    key[i] = morton(p, lo, span, nd);
  }
  std::vector<int32_t> order(nn);
  std::iota(order.begin(), order.end(), 0);
  std::sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
    return key[a] != key[b] ? key[a] < key[b] : a < b;
  });
  std::vector<int32_t> inv(nn);
  for (int64_t i = 0; i < nn; ++i) inv[order[i]] = (int32_t)i;
  m.perm = order;
  m.x.resize((size_t)nd * nn);
  for (int d = 0; d < nd; ++d)
    for (int64_t i = 0; i < nn; ++i) m.x[(size_t)d * nn + i] = xyz[(int64_t)d * nn + order[i]];

  // ---- cell order: curve key of the (wrapped) centroid
  std::vector<uint64_t> ckey(nc);
  for (int64_t c = 0; c < nc; ++c) {
    const int64_t* v = &cv[(size_t)c * nv];
    double e[3][3];
    relative_coords(m, xyz, v, sh[c], e);
    double p[3];
    for (int d = 0; d < nd; ++d) {
      double s = 0.0;
      for (int k = 1; k < nv; ++k) s += e[k - 1][d];
      p[d] = xyz[(int64_t)d * nn + v[0]] + s / nv;
      if (m.period[d] > 0.0) p[d] = lo[d] + std::fmod(std::fmod(p[d] - lo[d], m.period[d]) + m.period[d], m.period[d]);
    }
    ckey[c] = morton(p, lo, span, nd);
  }
  std::vector<int64_t> corder(nc);
  std::iota(corder.begin(), corder.end(), 0);
  std::sort(corder.begin(), corder.end(), [&](int64_t a, int64_t b) {
    return ckey[a] != ckey[b] ? ckey[a] < ckey[b] : a < b;
  });
  m.cell.resize((size_t)nv * nc);
  m.shift.resize(nc);
  std::vector<double> cvol(nc);
  for (int64_t c = 0; c < nc; ++c) {
    int64_t src = corder[c];
    for (int k = 0; k < nv; ++k) m.cell[(size_t)k * nc + c] = inv[cv[(size_t)src * nv + k]];
    m.shift[c] = sh[src];
    cvol[c] = vol[src];
  }

  // ---- median-dual nodal volumes (cell order, deterministic)
  m.vnode.assign(nn, 0.0);
  m.vol_cells = 0.0;
  for (int64_t c = 0; c < nc; ++c) {
    m.vol_cells += cvol[c];
    for (int k = 0; k < nv; ++k) m.vnode[m.cell[(size_t)k * nc + c]] += cvol[c] / nv;
  }
  m.vol_nodes = 0.0;
  for (int64_t i = 0; i < nn; ++i) m.vol_nodes += m.vnode[i];
  m.vupd = m.vnode;
  if (m.axi && quad) {
    // int r dA over node k's dual region in each quadrilateral: (X_k, midpoint
    // of side k, centre C = mean of the vertices, midpoint of side k-1), as the
    // triangles (X_k, M_k, C) and (X_k, C, M_p), each of first moment area
    // times mean vertex radius; r is not periodic, x differences come from the
    // unwrapped relative coordinates
    std::fill(m.vupd.begin(), m.vupd.end(), 0.0);
    for (int64_t c = 0; c < nc; ++c) {
      int64_t v[4];
      for (int k = 0; k < 4; ++k) v[k] = m.cell[(size_t)k * nc + c];
      double e[3][3];
      for (int k = 1; k < 4; ++k)
        for (int d = 0; d < 2; ++d)
          e[k - 1][d] = m.x[(size_t)d * nn + v[k]] + shift_of(m.shift[c], k, d, nd) * m.period[d] -
                        m.x[(size_t)d * nn + v[0]];
      const double P[4][2] = {{0.0, m.x[(size_t)nn + v[0]]},
                              {e[0][0], m.x[(size_t)nn + v[1]]},
                              {e[1][0], m.x[(size_t)nn + v[2]]},
                              {e[2][0], m.x[(size_t)nn + v[3]]}};
      const double C[2] = {0.25 * (P[0][0] + P[1][0] + P[2][0] + P[3][0]),
                           0.25 * (P[0][1] + P[1][1] + P[2][1] + P[3][1])};
      auto tri = [](const double* a, const double* b, const double* q) {
        const double ar = 0.5 * std::fabs((b[0] - a[0]) * (q[1] - a[1]) - (b[1] - a[1]) * (q[0] - a[0]));
        return ar * (a[1] + b[1] + q[1]) / 3.0;
      };
      for (int k = 0; k < 4; ++k) {
        const double* X = P[k];
        const double* Xn = P[(k + 1) % 4];
        const double* Xp = P[(k + 3) % 4];
        const double Mk[2] = {0.5 * (X[0] + Xn[0]), 0.5 * (X[1] + Xn[1])};
        const double Mp[2] = {0.5 * (X[0] + Xp[0]), 0.5 * (X[1] + Xp[1])};
        m.vupd[v[k]] += tri(X, Mk, C) + tri(X, C, Mp);
      }
    }
    for (int64_t i = 0; i < nn; ++i)
      if (!(m.vupd[i] > 0.0)) return "axisymmetric node with a zero revolved volume";
  } else if (m.axi) {
    // int r dA over node k's dual region in each triangle: the quadrilateral
    // (X_k, midpoint k-l, centroid, midpoint k-m), two triangles of area A/6
    // whose first moments are area times the mean vertex radius (second
    // Pappus-Guldinus theorem over 2 pi); r is not periodic
    std::fill(m.vupd.begin(), m.vupd.end(), 0.0);
    for (int64_t c = 0; c < nc; ++c) {
      double r[3];
      for (int k = 0; k < 3; ++k) r[k] = m.x[(size_t)nn + m.cell[(size_t)k * nc + c]];
      const double rc = (r[0] + r[1] + r[2]) / 3.0;
      for (int k = 0; k < 3; ++k) {
        const double ml = 0.5 * (r[k] + r[(k + 1) % 3]), mq = 0.5 * (r[k] + r[(k + 2) % 3]);
        m.vupd[m.cell[(size_t)k * nc + c]] += cvol[c] / 6.0 * ((r[k] + ml + rc) / 3.0 + (r[k] + rc + mq) / 3.0);
      }
    }
    for (int64_t i = 0; i < nn; ++i)
      if (!(m.vupd[i] > 0.0)) return "axisymmetric node with a zero revolved volume";
  }

  // ---- boundary faces (owned by exactly one cell) and boundary node normals
  struct Face { std::array<int32_t, 3> n; int32_t c; int8_t k; };
  std::vector<Face> faces((size_t)nc * nv);
  for (int64_t c = 0; c < nc; ++c)
    for (int k = 0; k < nv; ++k) {
      Face& f = faces[(size_t)c * nv + k];
      f.n = {-1, -1, -1};
      if (quad) {
        // face k of a quadrilateral: its side k -> k+1
        f.n[0] = m.cell[(size_t)k * nc + c];
        f.n[1] = m.cell[(size_t)((k + 1) % 4) * nc + c];
      } else {
        // face k of a simplex: the one opposite vertex k
        int q = 0;
        for (int v = 0; v < nv; ++v)
          if (v != k) f.n[q++] = m.cell[(size_t)v * nc + c];
      }
      std::sort(f.n.begin(), f.n.begin() + nd);
      f.c = (int32_t)c;
      f.k = (int8_t)k;
    }
  std::sort(faces.begin(), faces.end(), [](const Face& a, const Face& b) {
    return a.n != b.n ? a.n < b.n : a.c < b.c;
  });
  std::vector<double> Sb((size_t)nd * nn, 0.0);
  std::vector<char> isb(nn, 0);
  struct EdgeShare { int32_t i, j; double S[2]; };
  std::vector<EdgeShare> shares;
  for (size_t a = 0; a < faces.size();) {
    size_t b = a + 1;
    while (b < faces.size() && faces[b].n == faces[a].n) ++b;
    if (b - a > 2) return "non-manifold face shared by more than two cells";
    if (b - a == 1) {
      int64_t c = faces[a].c;
      int64_t v[4];
      for (int k = 0; k < nv; ++k) v[k] = m.cell[(size_t)k * nc + c];
      double e[3][3], S[4][3];
      for (int k = 1; k < nv; ++k)
        for (int d = 0; d < nd; ++d)
          e[k - 1][d] = m.x[(size_t)d * nn + v[k]] + shift_of(m.shift[c], k, d, nd) * m.period[d] -
                        m.x[(size_t)d * nn + v[0]];
      if (quad) {
        // outward normal of side k -> k+1 (counter-clockwise cell), in the
        // slot the simplex path reads
        const int k = faces[a].k, l = (k + 1) % 4;
        const double xk = k == 0 ? 0.0 : e[k - 1][0], yk = k == 0 ? 0.0 : e[k - 1][1];
        const double xl = l == 0 ? 0.0 : e[l - 1][0], yl = l == 0 ? 0.0 : e[l - 1][1];
        S[k][0] = yl - yk;
        S[k][1] = -(xl - xk);
      } else {
        node_normals(nd, e, S);
      }
      for (int q = 0; q < nd; ++q) {
        int32_t i = faces[a].n[q];
        isb[i] = 1;
        // axisymmetric: node i's half of the edge revolves at radius (3 r_i + r_j)/4
        const double w = m.axi ? 0.75 * m.x[(size_t)nn + i] + 0.25 * m.x[(size_t)nn + faces[a].n[1 - q]] : 1.0;
        for (int d = 0; d < nd; ++d) Sb[(size_t)d * nn + i] += S[faces[a].k][d] / nd * w;
        if (nd == 2) shares.push_back({i, faces[a].n[1 - q], {S[faces[a].k][0] / 2, S[faces[a].k][1] / 2}});
      }
    }
    a = b;
  }
  for (int64_t i = 0; i < nn; ++i)
    if (isb[i]) m.bnd_node.push_back((int32_t)i);
  size_t nb = m.bnd_node.size();
  m.bnd_S.resize((size_t)nd * nb);
  for (size_t q = 0; q < nb; ++q)
    for (int d = 0; d < nd; ++d) m.bnd_S[(size_t)d * nb + q] = Sb[(size_t)d * nn + m.bnd_node[q]];
  if (nd == 2) {
    // bnd_node is ascending, so the boundary index orders like the node id
    std::sort(shares.begin(), shares.end(), [](const EdgeShare& a, const EdgeShare& b) {
      return a.i != b.i ? a.i < b.i : a.j < b.j;
    });
    m.bedge_ptr.assign(nb + 1, 0);
    m.bedge_nb.resize(shares.size());
    m.bedge_S.resize(2 * shares.size());
    size_t q = 0;
    for (size_t e = 0; e < shares.size(); ++e) {
      while (m.bnd_node[q] != shares[e].i) m.bedge_ptr[++q] = (int32_t)e;
      m.bedge_nb[e] = shares[e].j;
      m.bedge_S[e] = shares[e].S[0];
      m.bedge_S[shares.size() + e] = shares[e].S[1];
    }
    while (q < nb) m.bedge_ptr[++q] = (int32_t)shares.size();
  }

  // ---- tiles
  {
    Tiling t;
    std::string e = build_tiling(m, lim, t);
    if (!e.empty()) return e;
    m.tile_cell = std::move(t.tile_cell);
    m.tile_slot = std::move(t.tile_slot);
    m.slot_node = std::move(t.slot_node);
    m.lconn = std::move(t.lconn);
    m.slot_inc = std::move(t.slot_inc);
    m.inc = std::move(t.inc);
    m.node_slot = std::move(t.node_slot);
    m.slots_of = std::move(t.slots_of);
    m.shared = std::move(t.shared);
    m.slot_run = std::move(t.slot_run);
    m.max_tile_cells = t.max_tile_cells;
    m.max_tile_nodes = t.max_tile_nodes;
  }

  if (nd == 2 && !quad) build_halos(m);
  *code = 0;
  return "";
}

void build_halos(HostMesh& m) {
  const int nv = m.nv;
  const int64_t nn = m.nn, nc = m.nc, T = m.ntiles();
  // cells around each node, ascending cell id
  std::vector<int32_t> cstart(nn + 1, 0), cells_of((size_t)nc * nv);
  for (int64_t c = 0; c < nc; ++c)
    for (int k = 0; k < nv; ++k) cstart[m.cell[(size_t)k * nc + c] + 1]++;
  for (int64_t i = 0; i < nn; ++i) cstart[i + 1] += cstart[i];
  {
    std::vector<int32_t> fill(cstart.begin(), cstart.end() - 1);
    for (int64_t c = 0; c < nc; ++c)
      for (int k = 0; k < nv; ++k) cells_of[fill[m.cell[(size_t)k * nc + c]]++] = (int32_t)c;
  }
  std::vector<int32_t> loc(nn, -1), hc, hn;
  std::vector<std::vector<uint16_t>> hl(nv);
  m.tile_hcell.assign(1, 0);
  m.tile_hnode.assign(1, 0);
  m.slot_ginc.assign(1, 0);
  m.ginc.clear();
  m.hnode.clear();
  m.hshift.clear();
  m.max_ext_cells = m.max_ext_nodes = m.max_tile_ginc = 0;
  for (int64_t t = 0; t < T; ++t) {
    const int32_t c0 = m.tile_cell[t], c1 = m.tile_cell[t + 1];
    const int32_t s0 = m.tile_slot[t], s1 = m.tile_slot[t + 1];
    const int32_t ncl = c1 - c0, ns = s1 - s0;
    for (int32_t s = s0; s < s1; ++s) {
      const int32_t v = m.slot_node[s];
      loc[v >= 0 ? v : ~v] = s - s0;
    }
    // halo cells: cells of the tile's shared nodes outside the tile
    hc.clear();
    for (int32_t s = s0; s < s1; ++s) {
      const int32_t v = m.slot_node[s];
      if (v >= 0) continue;
      const int32_t g = ~v;
      for (int32_t p = cstart[g]; p < cstart[g + 1]; ++p)
        if (cells_of[p] < c0 || cells_of[p] >= c1) hc.push_back(cells_of[p]);
    }
    std::sort(hc.begin(), hc.end());
    hc.erase(std::unique(hc.begin(), hc.end()), hc.end());
    // halo nodes: vertices of halo cells that are not slots of the tile
    hn.clear();
    for (int32_t c : hc)
      for (int k = 0; k < nv; ++k) {
        const int32_t i = m.cell[(size_t)k * nc + c];
        if (loc[i] < 0) hn.push_back(i);
      }
    std::sort(hn.begin(), hn.end());
    hn.erase(std::unique(hn.begin(), hn.end()), hn.end());
    for (size_t q = 0; q < hn.size(); ++q) loc[hn[q]] = ns + (int32_t)q;
    for (int32_t c : hc) {
      for (int k = 0; k < nv; ++k) hl[k].push_back((uint16_t)loc[m.cell[(size_t)k * nc + c]]);
      m.hshift.push_back(m.shift[c]);
    }
    for (int32_t i : hn) m.hnode.push_back(i);
    // cells around each slot node in ascending cell id, extended-local
    const size_t g0 = m.ginc.size();
    for (int32_t s = s0; s < s1; ++s) {
      const int32_t v = m.slot_node[s], g = v >= 0 ? v : ~v;
      for (int32_t p = cstart[g]; p < cstart[g + 1]; ++p) {
        const int32_t c = cells_of[p];
        int32_t e;
        if (c >= c0 && c < c1) {
          e = c - c0;
        } else {
          e = ncl + (int32_t)(std::lower_bound(hc.begin(), hc.end(), c) - hc.begin());
        }
        m.ginc.push_back((uint16_t)e);
      }
      m.slot_ginc.push_back((int32_t)m.ginc.size());
    }
    m.tile_hcell.push_back(m.tile_hcell.back() + (int32_t)hc.size());
    m.tile_hnode.push_back(m.tile_hnode.back() + (int32_t)hn.size());
    m.max_ext_cells = std::max(m.max_ext_cells, ncl + (int)hc.size());
    m.max_ext_nodes = std::max(m.max_ext_nodes, ns + (int)hn.size());
    m.max_tile_ginc = std::max(m.max_tile_ginc, (int)(m.ginc.size() - g0));
    for (int32_t s = s0; s < s1; ++s) {
      const int32_t v = m.slot_node[s];
      loc[v >= 0 ? v : ~v] = -1;
    }
    for (int32_t i : hn) loc[i] = -1;
  }
  const size_t H = m.hshift.size();
  m.hlconn.resize((size_t)nv * H);
  for (int k = 0; k < nv; ++k) std::copy(hl[k].begin(), hl[k].end(), m.hlconn.begin() + (size_t)k * H);
  m.has_halo = m.max_ext_cells < 65536 && m.max_ext_nodes < 65536;
}


std::string build_tile_edges(HostMesh& m) {
  if (m.has_edges) return "";
  const int nd = m.nd, NE = m.ne;
  const int64_t nc = m.nc, T = m.ntiles();
  // local cell-edges (a, b), a < b, in the kernels' order
  static const int E2[3][2] = {{0, 1}, {0, 2}, {1, 2}};
  static const int E3[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};
  const int(*EE)[2] = nd == 2 ? E2 : E3;
  m.tile_edge.assign(1, 0);
  m.edge.clear();
  m.edge_ce.assign(1, 0);
  m.ce.clear();
  m.ce.reserve((size_t)nc * NE);
  m.slot_einc.assign(1, 0);
  m.einc.clear();
  m.max_tile_edges = 0;
  // one record per cell-edge of a tile: its unordered end pair, its position
  // in cell order, and its code
  struct CE {
    uint32_t key;  // min end << 16 | max end
    int pos;
    uint16_t code;
    int la, lb;    // ends in the cell-edge's own orientation
    uint32_t image;
  };
  struct Grp {
    int begin, end, first;
  };
  std::vector<CE> rec;
  std::vector<Grp> grp;
  std::vector<int> cnt, fill;
  std::vector<uint16_t> sinc;
  for (int64_t t = 0; t < T; ++t) {
    const int32_t c0 = m.tile_cell[t], c1 = m.tile_cell[t + 1];
    const int ns = m.tile_slot[t + 1] - m.tile_slot[t];
    if (ns > 4095 || (c1 - c0) > 2047) return "tile too large for the tile-edge tables";
    rec.clear();
    for (int32_t c = c0; c < c1; ++c) {
      const int lc = c - c0;
      for (int e = 0; e < NE; ++e) {
        const int a = EE[e][0], b = EE[e][1];
        const int la = m.lconn[(size_t)a * nc + c], lb = m.lconn[(size_t)b * nc + c];
        uint32_t image = 0;
        for (int d = 0; d < nd; ++d) {
          const int sa = a == 0 ? 0 : shift_of(m.shift[c], a, d, nd);
          const int sb = shift_of(m.shift[c], b, d, nd);
          const int ds = sb - sa;
          if (ds < -1 || ds > 1) return "cell edge spans more than one periodic image";
          image |= (uint32_t)(ds == 1 ? 1u : (ds == -1 ? 2u : 0u)) << (2 * d);
        }
        const uint32_t key = la < lb ? ((uint32_t)la << 16 | (uint32_t)lb) : ((uint32_t)lb << 16 | (uint32_t)la);
        rec.push_back(CE{key, (int)rec.size(), (uint16_t)((lc << 4) | (e << 1)), la, lb, image});
      }
    }
    std::stable_sort(rec.begin(), rec.end(), [](const CE& x, const CE& y) { return x.key < y.key; });
    grp.clear();
    for (int i = 0; i < (int)rec.size();) {
      int j = i;
      while (j < (int)rec.size() && rec[j].key == rec[i].key) ++j;
      grp.push_back(Grp{i, j, rec[i].pos});  // stable: rec[i] is the first appearance
      i = j;
    }
    // descending cell-edge count, then first appearance
    std::sort(grp.begin(), grp.end(), [](const Grp& x, const Grp& y) {
      return (x.end - x.begin) != (y.end - y.begin) ? (x.end - x.begin) > (y.end - y.begin) : x.first < y.first;
    });
    if (grp.size() > 32767) return "tile too large for the tile-edge tables";
    cnt.assign(ns + 1, 0);
    for (const Grp& g : grp) {
      ++cnt[rec[g.begin].la + 1];
      ++cnt[rec[g.begin].lb + 1];
    }
    for (int q = 0; q < ns; ++q) cnt[q + 1] += cnt[q];
    fill.assign(cnt.begin(), cnt.end() - 1);
    sinc.assign(2 * grp.size(), 0);
    for (size_t k = 0; k < grp.size(); ++k) {
      const CE& f = rec[grp[k].begin];  // orientation and image of the first appearance
      m.edge.push_back((uint32_t)f.la | ((uint32_t)f.lb << 12) | (f.image << 24));
      for (int i = grp[k].begin; i < grp[k].end; ++i)
        m.ce.push_back((uint16_t)(rec[i].code | (rec[i].la == f.la ? 0 : 1)));
      m.edge_ce.push_back((int32_t)m.ce.size());
      // each slot's incident edges, in ascending tile-edge order
      sinc[fill[f.la]++] = (uint16_t)(k << 1);
      sinc[fill[f.lb]++] = (uint16_t)((k << 1) | 1);
    }
    for (int q = 0; q < ns; ++q) {
      for (int p = cnt[q]; p < cnt[q + 1]; ++p) m.einc.push_back(sinc[p]);
      m.slot_einc.push_back((int32_t)m.einc.size());
    }
    m.tile_edge.push_back((int32_t)m.edge.size());
    m.max_tile_edges = std::max(m.max_tile_edges, (int)grp.size());
  }
  if ((int64_t)m.ce.size() != nc * NE) return "tile-edge tables do not cover every cell-edge";
  m.has_edges = true;
  return "";
}

}  // namespace vcx
