// Host-side mesh preprocessing for the vertex-centred residual library.
#pragma once
#include <cstdint>
#include <string>
#include <vector>

namespace vcx {

// Tile limits: cells per tile (= threads of the tile kernels) and distinct
// nodes per tile (rows of the LDS node cache).
struct TileLimits {
  int max_cells;
  int max_nodes;
};

TileLimits default_tile_limits(int nd);

// A tiling of the cells (consecutive cells in the internal order, each tile
// closed at max_cells cells or max_nodes distinct nodes) with its slot tables:
// a tile's nodes are its slots; a node with slots in several tiles is shared
// and gathered through per-slot partial sums in ascending tile order.
struct Tiling {
  std::vector<int32_t> tile_cell;  // [T+1] first cell of each tile
  std::vector<int32_t> tile_slot;  // [T+1] first slot of each tile
  std::vector<int32_t> slot_node;  // [P] node of each slot (ascending inside a tile); ~node
                                   // when the node also has slots in other tiles
  std::vector<uint16_t> lconn;     // [nv][nc] tile-local node of each cell vertex
  std::vector<int32_t> slot_inc;   // [P+1] CSR into inc
  std::vector<uint16_t> inc;       // [nc*nv] (local cell << 2) | vertex, ascending cell
  std::vector<int32_t> node_slot;  // [nn+1] CSR into slots_of
  std::vector<int32_t> slots_of;   // [P] slots of each node, ascending tile
  std::vector<int32_t> shared;     // nodes with more than one slot, ascending
  std::vector<int32_t> slot_run;   // [2P] per slot: [begin, end) of its node's run in slots_of
  int max_tile_cells = 0, max_tile_nodes = 0;
  int64_t ntiles() const { return (int64_t)tile_cell.size() - 1; }
  int64_t nslots() const { return (int64_t)slot_node.size(); }
};

// Mesh after preprocessing, in the internal (space-filling-curve) order.
struct HostMesh {
  int nd = 0, nv = 0, ne = 0;
  int64_t nn = 0, nc = 0;
  double period[3] = {0, 0, 0};
  bool has_period = false;

  std::vector<int32_t> perm;      // [nn] internal node -> caller node
  std::vector<double> x;          // [nd][nn] coordinates (internal order)
  std::vector<int32_t> cell;      // [nv][nc] internal node ids, positively oriented
  std::vector<uint32_t> shift;    // [nc] periodic image code of vertices 1..nv-1
  std::vector<double> vnode;      // [nn] median-dual volume V_i
  double vol_cells = 0.0, vol_nodes = 0.0;
  // axisymmetric (x, r) meshes: the update divides by int r dA over each
  // node's dual region (vupd; equal to vnode otherwise), fluxes carry the
  // centroid radius of their dual face piece, and bnd_S is weighted by the
  // centroid radius of each node's share of its boundary edges
  bool axi = false;
  std::vector<double> vupd;       // [nn]

  // boundary closure
  std::vector<int32_t> bnd_node;  // [nb] internal ids (ascending)
  std::vector<double> bnd_S;      // [nd][nb] boundary node normals S_i^b
  // 2D: each boundary node's shares of its boundary edges (the other end
  // and the outward normal share S_f / 2), by boundary index, ascending
  // other end (second boundary-closure option)
  std::vector<int32_t> bedge_ptr;  // [nb+1]
  std::vector<int32_t> bedge_nb;   // [nbe]
  std::vector<double> bedge_S;     // [nd][nbe]

  // tiles
  TileLimits lim{};
  std::vector<int32_t> tile_cell;  // [T+1] first cell of each tile
  std::vector<int32_t> tile_slot;  // [T+1] first slot of each tile
  std::vector<int32_t> slot_node;  // [P] node of each slot (ascending inside a tile); ~node
                                   // when the node also has slots in other tiles
  std::vector<uint16_t> lconn;     // [nv][nc] tile-local node of each cell vertex
  std::vector<int32_t> slot_inc;   // [P+1] CSR into inc
  std::vector<uint16_t> inc;       // [nc*nv] (local cell << 2) | vertex, ascending cell
  std::vector<int32_t> node_slot;  // [nn+1] CSR into slots_of
  std::vector<int32_t> slots_of;   // [P] slots of each node, ascending tile
  std::vector<int32_t> shared;     // nodes with more than one slot, ascending
  std::vector<int32_t> slot_run;   // [2P] per slot: [begin, end) of its node's run in slots_of
  int max_tile_cells = 0, max_tile_nodes = 0;

  // extended tiles (2D): each tile plus the halo cells around its shared
  // nodes, so that a tile pass can form complete nodal gradients itself.
  // Extended-local nodes: the tile's slots first, then its halo nodes;
  // extended-local cells: the tile's cells first, then its halo cells.
  bool has_halo = false;
  std::vector<int32_t> tile_hcell;  // [T+1] offsets of each tile's halo cells
  std::vector<uint16_t> hlconn;     // [nv][H] extended-local node of each halo cell vertex
  std::vector<uint32_t> hshift;     // [H] periodic image code of each halo cell
  std::vector<int32_t> tile_hnode;  // [T+1] offsets of each tile's halo nodes
  std::vector<int32_t> hnode;       // halo nodes (internal ids), ascending inside a tile
  std::vector<int32_t> slot_ginc;   // [P+1] CSR into ginc
  std::vector<uint16_t> ginc;       // extended-local cells around each slot's node, ascending cell id
  int max_ext_cells = 0, max_ext_nodes = 0, max_tile_ginc = 0;

  // tile edges: the distinct edges of each tile's cells (built on demand by
  // build_tile_edges for the edge-based flux pass).  Within a tile, edges are
  // ordered by descending number of cell-edges (ties: first appearance), so
  // that the threads of a wavefront take edges with similar work.
  bool has_edges = false;
  std::vector<int32_t> tile_edge;  // [T+1] first tile edge of each tile
  std::vector<uint32_t> edge;      // [E] la | lb << 12 | image << 24: tile-local ends a -> b and the
                                   // periodic image of b relative to a (2 bits per axis: 1 -> +1, 2 -> -1)
  std::vector<int32_t> edge_ce;    // [E+1] CSR into ce
  std::vector<uint16_t> ce;        // [nc * ne] (local cell << 4) | (cell-local edge << 1) | reversed
  std::vector<int32_t> slot_einc;  // [P+1] CSR into einc
  std::vector<uint16_t> einc;      // [2E] per slot: (tile edge << 1) | (1 if the slot's node is end b)
  int max_tile_edges = 0;

  // node gradient (built by build_node_gradient): for each node i its
  // neighbours j, the other nodes of its cells, ascending, and C_ij, the sum
  // of the node normals S_j of the cells holding both i and j.  A simplex's
  // node normals sum to zero, so C_ii = -sum_{j != i} C_ij and the cell-sum
  // gradient is G_i = -1/(nd nv V_i) sum_{j != i} (W_j - W_i) C_ij.  Nodes in
  // slices of 64 (one per wavefront), each slice padded to its largest
  // neighbour count (pad entries: j = i, C = 0); entry k of the slice's node
  // l at off + 64 k + l.
  static constexpr int kNgSlice = 64;
  bool has_ngrad = false;
  std::vector<int64_t> ng_off;  // [nslices + 1]
  std::vector<int32_t> ng_nbr;  // [total]
  std::vector<double> ng_c;     // [nd][total]

  int64_t ntiles() const { return (int64_t)tile_cell.size() - 1; }
  int64_t nslots() const { return (int64_t)slot_node.size(); }
};

// Tile the cells of a preprocessed mesh; returns "" or an error message.
std::string build_tiling(const HostMesh& m, TileLimits lim, Tiling& t);

// Node-gradient tables of a preprocessed simplex mesh (HostMesh::ng_*).
std::string build_node_gradient(HostMesh& m);

// Returns "" on success, else an error message; *code receives the status
// (-1 argument, -2 mesh).
std::string preprocess_mesh(int nd, int64_t nn, const double* xyz, int64_t nc, int nv,
                            const int64_t* cells, const double* period, TileLimits lim,
                            HostMesh& out, int* code, bool axisymmetric = false);

// Build the extended-tile tables of a preprocessed mesh (any dimension).
void build_halos(HostMesh& m);

// Build the tile-edge tables of a preprocessed mesh (any dimension);
// returns "" or an error message.
std::string build_tile_edges(HostMesh& m);

// Decode the periodic image of vertex k (1..nv-1) along axis d: -1, 0, +1.
inline int shift_of(uint32_t code, int k, int d, int nd) {
  uint32_t b = (code >> (2 * ((k - 1) * nd + d))) & 3u;
  return b == 1u ? 1 : (b == 2u ? -1 : 0);
}

}  // namespace vcx
