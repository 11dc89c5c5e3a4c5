/*
 * vcx.h -- C ABI of the MI355X (gfx950) vertex-centred explicit residual.
 *
 * The library evaluates, on one GPU, the explicit finite-volume residual of
 * "AVIP: a low temperature plasma code" (arXiv 2201.01291) on unstructured
 * triangle and tetrahedron meshes, and advances it with the paper's
 * low-storage Runge-Kutta schemes:
 *
 *   residual   r_i = sum over the cells tau around node i, over the cell-edges
 *              (i,j) of tau, of the flux through the dual-surface piece S_ij
 *              (eq. vertex_centered_flux), plus the node-flux closure on
 *              boundary nodes (Sec. "Boundary conditions in AVIP");
 *   gas        MUSCL reconstruction with virtual upwind nodes
 *              (eq. virtual_node_reconstruction) of the conserved variables and
 *              pressure, slope limiters, HLLC (Sec. "The HLLC solver") or Roe
 *              flux, passive species carried in the mass fractions;
 *   drift-diff limited Lax-Wendroff convective flux plus central diffusive flux
 *              (Secs. "Limited Lax-Wendroff scheme", "Central difference
 *              diffusive flux integration"), prescribed electric field;
 *   time step  cell-based convective / diffusive limits, minimum over cells
 *              and species (Sec. "Time step computation");
 *   update     U(k) = U^n - alpha_k dt r(U(k-1)) / V_i, U^{n+1} = U^n -
 *              dt r(U(K)) / V_i with the alphas of table rk_coeffs.
 *
 * Conventions
 *   - Every function returns a vcx_status and never throws.  On error the
 *     message of the last failing call of the calling thread is returned by
 *     vcx_last_error().
 *   - Host arrays are owned by the caller and copied during the call.  Device
 *     arrays passed with is_device = 1 must be device memory of the device the
 *     handle lives on; they are read or written on the handle's stream.
 *   - Node order at the boundary is always the caller's order; the internal
 *     space-filling-curve renumbering is hidden.
 *   - Layout: structure of arrays, [variable][node] (row-major, node fastest).
 *   - Residual sign: r_i is the integrated net outflow, dU_i/dt = -r_i / V_i,
 *     so on a periodic mesh sum_i r_i = 0.
 *   - Streams: all device work of a handle is ordered on the hipStream_t
 *     given at creation (NULL = default stream).  Calls that return host
 *     values synchronise that stream.
 *   - A handle may be used by one thread at a time.
 */
#ifndef VCX_H
#define VCX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  VCX_OK = 0,
  VCX_E_ARG = -1,      /* invalid argument or unsupported combination */
  VCX_E_MESH = -2,     /* invalid mesh: index out of range, degenerate cell,
                          non-manifold face, periodic cell wider than half the box */
  VCX_E_OOM = -3,      /* device or host allocation failed */
  VCX_E_HIP = -4,      /* HIP runtime error (no device, launch failure, ...) */
  VCX_E_UNSTABLE = -5, /* state became non-finite or non-physical (rho<=0 or
                          p<=0); the state is left at the last good step */
  VCX_E_BUSY = -6,     /* resource budget exhausted (server) */
  VCX_E_STATE = -7     /* call out of order (e.g. step before state_upload) */
} vcx_status;

enum {
  VCX_MODEL_GAS = 0,              /* Euler + passive species, ideal gas, constant gamma */
  VCX_MODEL_DRIFT_DIFFUSION = 1,  /* charged species in a prescribed field */
  VCX_MODEL_NAVIER_STOKES = 2     /* multi-species Navier-Stokes transport (eq. ns_reactive
                                     without sources): HLLC + viscous, heat and species
                                     diffusion; temperature from the sensible energy */
};
enum {
  VCX_FLUX_HLLC = 0, /* gas */
  VCX_FLUX_ROE = 1,  /* gas */
  VCX_FLUX_LLW = 0,  /* drift-diffusion: limited Lax-Wendroff + central diffusion */
  VCX_FLUX_SG = 2    /* drift-diffusion: Scharfetter-Gummel (Sec. "Scharfetter Gummel
                        scheme"): along each edge the flux of the 1D steady
                        advection-diffusion solution through its two nodal values,
                        c D (B(-a) u_i - B(a) u_j) with S_par = c (x_j - x_i),
                        a = V . (x_j - x_i) / D, B(x) = x / (e^x - 1) (upwinding
                        when D = 0); across the edge the central flux
                        (V u_bar - D grad u_bar) . (S - S_par); V the mean drift of
                        the two nodes.  Separate gradient and flux passes (not
                        fused); not batched or served (VCX_E_ARG). */
};
enum {
  VCX_LIM_FIRST_ORDER = 0, /* zero slope / Psi = 0 (first-order upwind) */
  VCX_LIM_MINMOD = 1,
  VCX_LIM_VANLEER = 2,
  VCX_LIM_SWEBY = 3,       /* Sweby beta limiter, 1 <= beta <= 2 */
  VCX_LIM_NONE = 4         /* unlimited: centred slope / Psi = 1 (plain Lax-Wendroff) */
};
enum {
  VCX_PREC_FP64 = 0,  /* everything in FP64 */
  VCX_PREC_MIXED = 1  /* reconstruction, limiters and fluxes in FP32; gradients,
                         residual accumulation, update, time step and sums in FP64 */
};

#define VCX_MAX_SPECIES 16

/* Physical model and scheme parameters. */
typedef struct {
  int32_t model;      /* VCX_MODEL_* */
  int32_t flux;       /* gas: VCX_FLUX_HLLC or VCX_FLUX_ROE; drift-diffusion:
                         VCX_FLUX_LLW or VCX_FLUX_SG (else VCX_E_ARG);
                         multi-species: ignored (HLLC) */
  int32_t limiter;    /* VCX_LIM_* */
  int32_t rk_stages;  /* 1..4 (table rk_coeffs) */
  int32_t nspecies;   /* gas: passive species (0, 2 or 9 supported);
                         drift-diffusion: charged species (1 or 2);
                         Navier-Stokes: species (2 or 9), HLLC only */
  int32_t closure;    /* boundary closure (Sec. "Boundary conditions in AVIP"):
                         0 none, 1 node flux F(U_i) . S_i^b, 2 (plane 2D meshes,
                         gas and drift-diffusion) interpolated fluxes
                         0.75 F_i + 0.25 F_j on each half boundary edge */
  int32_t precision;  /* VCX_PREC_* */
  int32_t predictor;  /* gas model on plane meshes with rk_stages = 1: 1 adds the
                         MUSCL-Hancock half-step evolution (after Toro, Chap. 14,
                         which Sec. "The HLLC solver" names) to the face states:
                         each end's reconstructed (rho, rho u, rho E, rho Y, p)
                         gains dt/2 times its time derivative from the
                         quasi-linear Euler equations with the nodal state and
                         gradients; 0 none.  Other combinations: VCX_E_ARG.
                         Not batched (vcx_solve_batch, the server). */
  double beta;        /* Sweby beta */
  double cfl;         /* convective CFL number */
  double fourier;     /* diffusive Fourier number */
  double gamma;       /* ratio of specific heats (gas) */
  double entropy_fix; /* Roe: Harten delta as a fraction of the Roe sound speed */
  double z[VCX_MAX_SPECIES];   /* drift-diffusion charge sign per species */
  double mu[VCX_MAX_SPECIES];  /* mobility [m^2/(V s)] */
  double D[VCX_MAX_SPECIES];   /* diffusion coefficient [m^2/s] */
  /* Navier-Stokes mixture: per species molar mass W [kg/mol], heat capacity
   * c_p(T) = (R/W)(cpa + cpb t + cpc t^2) with t = T/1000, Schmidt number;
   * mu = mu_ref (T/T_ref)^0.7, lambda = mu c_p / Pr, D_k = mu / (rho Sc_k).
   * Sensible enthalpies are taken from 298.15 K; the total non-chemical energy
   * is rho (e_s + |u|^2/2) with e_s = sum Y_k (h_s,k - R T / W_k). */
  double Wk[VCX_MAX_SPECIES];
  double cpa[VCX_MAX_SPECIES], cpb[VCX_MAX_SPECIES], cpc[VCX_MAX_SPECIES];
  double Sc[VCX_MAX_SPECIES];
  double mu_ref, T_ref, Pr;
  /* drift-diffusion: constant A_D of the dielectric time step A_D eps0 /
   * sum_s |q_s n_s mu_s| (Sec. "Time step computation"), taken per node;
   * 0 leaves the limit out (the paper gives no value) */
  double diel;
} vcx_physics;

typedef struct vcx_mesh_s *vcx_mesh;
typedef struct vcx_solver_s *vcx_solver;
typedef struct vcx_server_s *vcx_server;

/* Build a device mesh (Sec. "Nomenclature and notations").
 *   ndim      2 or 3
 *   nv        vertices per cell: ndim + 1 (triangles, tetrahedra) or, in 2D,
 *             4 (convex quadrilaterals, vertices in cyclic order: node
 *             normals from eq. node_normal, S_k = -(sum of the outward
 *             normals of the two sides through k), the four sides as the
 *             cell-edges, dual faces from the side midpoints to the mean of
 *             the vertices).  Quadrilateral meshes run the gas and
 *             drift-diffusion models, with separate gradient and flux passes;
 *             they are not batched, served or taken by the Poisson solver
 *             (VCX_E_ARG)
 *   xyz       host [ndim][nnodes] coordinates
 *   cells     host [nv][ncells] node indices (any vertex orientation)
 *   period    host [ndim] box length of each periodic axis, 0 for an open
 *             axis, or NULL (no periodicity)
 *   stream    hipStream_t for the uploads and for every later use
 * Computes node normals, median-dual volumes V_i = sum V_tau / n_v, boundary
 * node normals, a space-filling-curve node/cell order and the fixed cell
 * tiles used by the deterministic scatter.  Tetrahedral meshes, and triangle
 * meshes above 2^20 cells, also get the node-gradient tables (each node's
 * neighbours and their coefficients, about 15 entries of 28 B per node in
 * 3D) and, in 3D, the tile-edge tables of the multi-species flux pass; a 2D
 * mesh gets the latter two when its first multi-species solver is created.
 * Errors: VCX_E_ARG, VCX_E_MESH, VCX_E_OOM, VCX_E_HIP. */
vcx_status vcx_mesh_create(int ndim, int64_t nnodes, const double *xyz, int64_t ncells, int nv,
                           const int64_t *cells, const double *period, void *stream,
                           vcx_mesh *out);
/* As vcx_mesh_create with explicit tile limits: at most max_tile_cells cells
 * (<= 1024) and max_tile_nodes distinct nodes per tile; 0 selects the
 * defaults (2D 256 / 192, 3D 128 / 96).  Smaller tiles lower the LDS
 * footprint of the tile kernels (needed by models with many variables),
 * larger tiles lower the partial-sum traffic. */
vcx_status vcx_mesh_create_tiled(int ndim, int64_t nnodes, const double *xyz, int64_t ncells,
                                 int nv, const int64_t *cells, const double *period,
                                 int max_tile_cells, int max_tile_nodes, void *stream,
                                 vcx_mesh *out);
/* Axisymmetric domain (Sec. "Cylindrical frames", eq. vertex_centered_flux_axi):
 * a triangle mesh of the (x, r) half-plane, xr host [2][nnodes] with r >= 0,
 * cells host [3][ncells]; period_x > 0 makes x periodic (r never is).  Fluxes
 * through the revolved dual faces carry the centroid radius of each dual
 * face piece (first Pappus-Guldinus theorem), node volumes of the update and
 * of vcx_conservation_sums are int r dA over each node's dual region (second
 * theorem; exact, and non-zero on the axis), and boundary closures use the
 * radius-weighted boundary normals; all over 2 pi.  Nodal gradients stay
 * planar.  Gas and multi-species solvers add the geometric source p A_i
 * (plane dual area) to the radial momentum (Sec. "Geometric source terms")
 * and set the radial velocity to zero on the axis after each stage.  The
 * multi-species model also takes the diffusive source of eq.
 * ns_cyl_source_terms, -(2 eta u_r/r + lambda (u_r/r + du_r/dr + du_x/dx)) A_i
 * with lambda = -2/3 eta and u_r/r -> du_r/dr on the axis, and the
 * cylindrical div u (with u_r/r at the edge midpoint) in its diffusive
 * fluxes.  All three models; such solvers are not batched or served
 * (VCX_E_ARG).  vcx_mesh_geometry returns the planar V_i and the
 * radius-weighted S_i^b.  Errors as vcx_mesh_create_tiled, and VCX_E_ARG
 * for r < 0. */
vcx_status vcx_mesh_create_axisymmetric(int64_t nnodes, const double *xr, int64_t ncells,
                                        const int64_t *cells, double period_x, int max_tile_cells,
                                        int max_tile_nodes, void *stream, vcx_mesh *out);
/* As vcx_mesh_create_axisymmetric with nv vertices per cell: 3 (triangles)
 * or 4 (convex quadrilaterals in cyclic order, see vcx_mesh_create_tiled);
 * cells host [nv][ncells].  A quadrilateral's dual piece of a side runs from
 * the side's midpoint to the mean of the vertices and carries its mean
 * radius; node volumes are int r dA over the exact dual regions. */
vcx_status vcx_mesh_create_axisymmetric_nv(int64_t nnodes, const double *xr, int64_t ncells, int nv,
                                           const int64_t *cells, double period_x, int max_tile_cells,
                                           int max_tile_nodes, void *stream, vcx_mesh *out);
vcx_status vcx_mesh_destroy(vcx_mesh mesh);

/* Mesh counters: out[0] nnodes, [1] ncells, [2] cell-edges (faces),
 * [3] tiles, [4] partial slots, [5] boundary nodes, [6] max cells per tile,
 * [7] max nodes per tile. */
vcx_status vcx_mesh_info(vcx_mesh mesh, int64_t out[8]);

/* Median-dual nodal volumes [nnodes] and boundary node normals
 * [ndim][nnodes] (zero on interior nodes), caller's node order, host. */
vcx_status vcx_mesh_geometry(vcx_mesh mesh, double *Vn, double *Sb);

/* Host-only dry run of the preprocessing of vcx_mesh_create (no device
 * needed): same validation, same tiles.  stats as in vcx_mesh_info, plus
 * stats[8] = total volume of the cells, stats[9] = sum of nodal volumes
 * (bit patterns of doubles, via memcpy). */
vcx_status vcx_mesh_preprocess(int ndim, int64_t nnodes, const double *xyz, int64_t ncells,
                               int nv, const int64_t *cells, const double *period,
                               int64_t stats[10]);

/* Create a solver (state buffers, scheme parameters) on a mesh.
 *   E   drift-diffusion only: host [ndim][nnodes] electric field at the
 *       nodes (caller order), copied; NULL for gas.
 * Unsupported species counts, or tiles whose LDS footprint exceeds the
 * device's per-workgroup limit, give VCX_E_ARG. */
vcx_status vcx_solver_create(vcx_mesh mesh, const vcx_physics *phys, const double *E,
                             vcx_solver *out);
vcx_status vcx_solver_destroy(vcx_solver s);

/* Replace the prescribed electric field of a drift-diffusion solver
 * (E [ndim][nnodes], caller order, host or device per is_device), e.g. with
 * the field of vcx_poisson_field for a step coupled to the Poisson
 * equation.  The time-step candidates of the current state are recomputed
 * with the new field (Sec. "Time step computation"), so the next step's
 * time step uses it; time and step count are kept.  Synchronises the
 * mesh's stream.  Errors: VCX_E_ARG (NULL argument, or a model without a
 * field), VCX_E_HIP. */
vcx_status vcx_solver_set_field(vcx_solver s, const double *E, int is_device);

/* Space charge of a drift-diffusion solver's current state, the right-hand
 * side of the Poisson equation (Sec. "Integrating the Poisson equation"):
 * q_i = (e / eps0) sum_s z_s n_s,i at the nodes, with z_s the species'
 * charge numbers of its physics (at most 4 species), e = 1.602176634e-19 C
 * and eps0 = 8.8541878128e-12 F/m.  q: [nnodes] in caller order, host or
 * device (is_device), written on the mesh's stream; synchronises it.
 * Errors: VCX_E_ARG (NULL, not drift-diffusion), VCX_E_STATE (no state),
 * VCX_E_HIP. */
vcx_status vcx_solver_charge(vcx_solver s, double *q, int is_device);

/* Number of conserved variables (gas 2 + ndim + nspecies; DD nspecies). */
int vcx_solver_nvar(vcx_solver s);

/* State [nvar][nnodes] in the caller's node order; is_device selects a host
 * or device pointer.  Upload resets the time to 0 (or to t0 with
 * vcx_state_set_time). */
vcx_status vcx_state_upload(vcx_solver s, const double *U, int is_device);
vcx_status vcx_state_download(vcx_solver s, double *U, int is_device);
vcx_status vcx_state_set_time(vcx_solver s, double t);
/* Upload a state given in primitive variables P [nvar][nnodes] (caller
 * order, host or device per is_device), converted on the device with the
 * solver's own equation of state: gas rows (rho, u_1..u_nd, p, Y_1..Y_N) ->
 * rho E = p / (gamma - 1) + rho |u|^2 / 2; Navier-Stokes rows (rho, u, T,
 * Y) -> rho E = rho (e_s(T) + |u|^2 / 2) with the mixture's sensible energy
 * (the total non-chemical energy of eq. ns_reactive); drift-diffusion rows
 * are the densities themselves.  Otherwise as vcx_state_upload. */
vcx_status vcx_state_upload_primitive(vcx_solver s, const double *P, int is_device);

/* Nodal gradients of the reconstructed variables of the current state,
 * [nr][ndim][nnodes] (gas nr = nvar + 1 with pressure last; DD nr = nvar),
 * caller order (Sec. "Integrating the Poisson equation", cell gradient, then
 * the volume-weighted average over the cells around the node). */
vcx_status vcx_gradient(vcx_solver s, double *G, int is_device);

/* Residual of the current state, FP64 [nvar][nnodes], caller order.  dt is
 * used by the limited Lax-Wendroff flux and the gas predictor's half step
 * (vcx_physics.predictor); other physics ignore it. */
vcx_status vcx_residual(vcx_solver s, double dt, double *r, int is_device);

/* Allocation-free variant of vcx_residual, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc): the residual of the state U on this mesh with this
 * physics, without a solver.
 *   U    device [nvar][nnodes], caller's node order (read)
 *   E    drift-diffusion: device [ndim][nnodes] field, caller order; else NULL
 *   dt   used by the limited Lax-Wendroff flux and the gas predictor only
 *   r    device [nvar][nnodes], caller order (written)
 * Result: bit for bit that of vcx_residual on a solver of the same mesh and
 * physics holding U.  The call allocates nothing: every intermediate array
 * (reconstructed rows, nodal gradients, tile partials, the field in internal
 * order) lives in one static device array of vcx_noalloc_scratch_bytes()
 * (64 MiB) per device, which the library holds until the process ends.
 * Meshes and physics that need more return VCX_E_ARG (e.g. 2D
 * drift-diffusion up to about 300k nodes), as does the multi-species model
 * on a 2D mesh that has no multi-species solver yet (its tables are built
 * by the first one).  All calls on one device share
 * that array and the work runs on the mesh's stream; the call returns once
 * it is complete, so calls must not overlap on one GPU (several threads or
 * streams at once race).  Errors: VCX_E_ARG (NULL argument, unsupported
 * physics, too large), VCX_E_HIP. */
vcx_status vcx_residual_noalloc(vcx_mesh mesh, const vcx_physics *phys, const double *U,
                                const double *E, double dt, double *r);
/* Bytes of the per-device scratch array of vcx_residual_noalloc. */
size_t vcx_noalloc_scratch_bytes(void);

/* CFL / Fourier time step of the current state (minimum over cells and
 * species). */
vcx_status vcx_timestep(vcx_solver s, double *dt);

/* Advance nsteps steps (time step recomputed every step; the last step is
 * clipped to t_end when t_end > 0, and no step starts once t >= t_end).
 * Returns the time reached and the last time step.  VCX_E_UNSTABLE leaves
 * the state at the last good step. */
vcx_status vcx_step(vcx_solver s, int nsteps, double t_end, double *t, double *dt_last);

/* Steps completed by the last vcx_step / vcx_solve_batch call on s. */
int64_t vcx_steps_done(vcx_solver s);

/* Time t and last completed step size of s after its last vcx_step /
 * vcx_solve_batch call (t0 and 0 right after an upload).  NULL outputs are
 * skipped. */
vcx_status vcx_state_time(vcx_solver s, double *t, double *dt_last);

/* Advance n independent solvers (each on its own mesh, or several on one
 * mesh) together, the batched execution of the explicit scheme (Sec. "Time
 * integration" applied per solve).  Per RK stage one launch per kernel covers
 * the tiles and the shared nodes of every member: a device table holds one
 * descriptor per solve (mesh arrays, state buffers, time-step scalars) and a
 * block map gives each workgroup its solve and local tile.  Each member
 * keeps its own time loop: its own dt (CFL/Fourier minimum over its own
 * cells), step budget nsteps[i] (>= 0) and end time t_end[i] (<= 0: none;
 * the last step is clipped to it).  Results are bitwise identical to those
 * of vcx_step on each solver alone.
 * Requirements: every member has a state (vcx_state_upload), is not in a
 * failed state, appears once, and all members have byte-identical
 * physics structs: same model, scheme, precision and constants.  The call runs on the
 * first member's stream after synchronising the others' and returns when
 * every member has finished.
 * Errors: VCX_E_ARG (NULL, empty, duplicate or mixed-physics batch),
 * VCX_E_STATE (member without state), VCX_E_UNSTABLE (one or more members
 * blew up: each of those keeps its last good state and its flag; the others
 * completed normally), VCX_E_OOM / VCX_E_HIP. */
vcx_status vcx_solve_batch(vcx_solver *s, int n, const int *nsteps, const double *t_end);

/* vcx_solve_batch with every kernel launched directly (vcx_solve_batch
 * replays two batch steps captured once into a HIP graph).  Same results,
 * bit for bit; for comparison and for callers that avoid graphs. */
vcx_status vcx_solve_batch_eager(vcx_solver *s, int n, const int *nsteps, const double *t_end);

/* Device bytes a solver with this physics on this mesh would allocate
 * (state buffers and, for the multi-species model, their node-major staged
 * copies, gradients, tile partials, staging, time-step scalars; the mesh's
 * own arrays are not included).  Used for admission by device-memory
 * footprint. */
vcx_status vcx_solver_footprint(vcx_mesh mesh, const vcx_physics *phys, size_t *bytes);

/* ---------------------------------------------------------------------------
 * Serving: continuous batching of independent solves
 *
 * A server owns a scheduler thread and a stream on the current device.
 * Requests (a mesh, a physics struct, an initial state, a step budget and
 * an end time) are queued by vcx_server_submit and admitted in arrival
 * order while fewer than max_slots requests run and the sum of the running
 * requests' vcx_solver_footprint stays within hbm_budget bytes.  Admitted
 * states stay resident in device memory; all running requests with the same
 * physics are advanced together by batched launches (as vcx_solve_batch, in
 * chunks of at most chunk_steps steps), and a request that arrives while
 * others run joins at the next chunk boundary.  Finished requests release
 * their slot and memory at once.  Each result is bitwise identical to the
 * same solve run alone with vcx_step.
 * Meshes passed to submit must outlive their requests.  Server calls are
 * thread-safe.
 * --------------------------------------------------------------------------- */

/* use_graphs = 1 replays captured HIP graphs (see vcx_solve_batch). */
vcx_status vcx_server_create(size_t hbm_budget, int max_slots, int chunk_steps, int use_graphs,
                             vcx_server *out);

/* Queue a request.  U0: host [nvar][nnodes] in caller order; E: host
 * [ndim][nnodes] electric field for drift-diffusion (else ignored, may be
 * NULL); both copied.  nsteps >= 0; t_end <= 0: none.  *id identifies the
 * request.  A request whose footprint exceeds the budget completes with
 * VCX_E_OOM. */
vcx_status vcx_server_submit(vcx_server sv, vcx_mesh mesh, const vcx_physics *phys, const double *U0,
                             const double *E, int nsteps, double t_end, int64_t *id);

/* *done = 1 once the request has finished; then *result holds its status
 * (VCX_OK, VCX_E_UNSTABLE with the last good state, VCX_E_OOM, VCX_E_BUSY
 * when the server shut down first, ...) and *t_out its time.  With a
 * non-NULL U_out (host, [nvar][nnodes]) the final state is copied and the
 * request is forgotten: later calls with its id return VCX_E_ARG.  result,
 * U_out and t_out may be NULL. */
vcx_status vcx_server_poll(vcx_server sv, int64_t id, int *done, vcx_status *result, double *U_out,
                           double *t_out);

/* Block until the request finished or timeout_s seconds passed (< 0: no
 * limit); *done as in vcx_server_poll. */
vcx_status vcx_server_wait(vcx_server sv, int64_t id, double timeout_s, int *done);

/* out[17]: submitted, completed, failed, queued, running, member steps done,
 * chunks run, mean running requests per chunk, request latency p50 / p99
 * (submit to finish, ms), step latency p50 / p99 (wall time of a scheduler
 * iteration / its steps, ms), bytes of running requests, peak bytes held
 * (running plus idle), peak running requests, status of the last device
 * error (0 = none), bytes of idle solvers.  Finished requests leave their
 * solver idle for reuse by a later request with the same mesh and physics
 * (idle solvers count against the budget and are freed, least recently
 * used first, when a new request needs the room). */
vcx_status vcx_server_stats(vcx_server sv, double *out);

/* Cancel queued requests (VCX_E_BUSY), finish running ones, stop the
 * scheduler and free the server. */
vcx_status vcx_server_destroy(vcx_server sv);

/* ---- Poisson solve for the electric field (Sec. "Integrating the Poisson
 * equation", Sec. "Boundary conditions") ------------------------------- */
typedef struct vcx_poisson_s *vcx_poisson;

/* Operator of a mesh: the matrix of -lap phi integrated over the nodal
 * volumes (eq. poisson_discretization_cartesian with the sign of the remark
 * on the implementation), L_ik = sum over the cells holding nodes i and k of
 * S_i . S_k / (V_tau n_d^2), assembled in FP64 on the host and kept on the
 * device, with the nodal-gradient operator of E = -grad phi.
 * dirichlet: [nnodes] (caller order), nonzero marks a Dirichlet node, or
 *   NULL for none.  Every other node is free; a free boundary node takes
 *   Neumann data (zero normal field unless E_n is given to the solve).
 * Without Dirichlet nodes (periodic or all-Neumann meshes) the system is
 * singular: a uniform background charge makes it compatible (the solve
 * removes the volume mean of q) and phi is returned with zero volume mean.
 * On an axisymmetric mesh (vcx_mesh_create_axisymmetric) the operator is
 * that of Sec. "Axisymmetric configuration": the planar cell gradient
 * dotted with int r n dl over each node's dual boundary, with revolved
 * volumes and boundary surfaces (all over 2 pi); it is not symmetric.
 * The operator lives on the mesh's stream; the mesh must outlive it.
 * Errors: VCX_E_ARG (NULL mesh or out, too large for 32-bit indices),
 * VCX_E_OOM, VCX_E_HIP. */
vcx_status vcx_poisson_create(vcx_mesh mesh, const int32_t *dirichlet, vcx_poisson *out);
vcx_status vcx_poisson_destroy(vcx_poisson p);

/* Solve sum_k L_ik phi_k = q_i V_i - En_i |S_i^b| on free nodes with
 * phi_i = phiD_i on Dirichlet nodes in FP64 on the device: conjugate
 * gradients with a two-level preconditioner (Jacobi plus an aggregation
 * coarse space), or on axisymmetric meshes BiCGStab with Jacobi; dot
 * products are reduced in a fixed order, so results are bitwise
 * reproducible.  Arrays are [nnodes] in caller order, all host or
 * all device (is_device):
 *   q    rho / eps0 at the nodes (required);
 *   phiD imposed potential, read on Dirichlet nodes only (NULL: zero);
 *   En   imposed normal field, read on free boundary nodes (NULL: zero);
 *   phi  in: initial guess on free nodes; out: the potential.
 * Stops when |r| <= tol |b - L_fD phi_D| (or tol |r_0| when that is zero),
 * or after max_iter iterations.  iters and relres (may be NULL) receive
 * the iteration count and |r| over that reference.  Returns VCX_E_STATE,
 * with phi holding the last iterate, when max_iter is reached first or
 * when BiCGStab breaks down (r^.r = 0, r^.v = 0 or omega = 0) above the
 * tolerance; VCX_E_UNSTABLE when the residual becomes non-finite (a NaN or
 * infinity in q, phiD, En or the initial phi); VCX_E_ARG for NULL q or phi,
 * tol <= 0 or max_iter < 0; VCX_E_HIP.  VCX_OK means |r| <= tol times the
 * reference. */
vcx_status vcx_poisson_solve(vcx_poisson p, const double *q, const double *phiD, const double *En,
                             double *phi, int is_device, double tol, int max_iter, int *iters,
                             double *relres);

/* E = -grad phi at the nodes with the nodal gradient of the scheme (the
 * volume-weighted mean of the cell gradients): phi [nnodes] in, E
 * [ndim][nnodes] out, caller order, host or device (is_device).  A
 * drift-diffusion solver takes the result through vcx_solver_create or, for
 * a coupled step, vcx_solver_set_field. */
vcx_status vcx_poisson_field(vcx_poisson p, const double *phi, double *E, int is_device);
/* As vcx_poisson_field plus a background field: E = E_bg - grad phi, with
 * Ebg [ndim][nnodes] in caller order on the same side (host or device) as
 * phi and E; Ebg may be the same array as E.  The field of a step coupled to
 * the Poisson equation under an applied field (Sec. "Bagheri benchmark").
 * Errors: VCX_E_ARG (NULL argument), VCX_E_HIP. */
vcx_status vcx_poisson_field_add(vcx_poisson p, const double *phi, const double *Ebg, double *E,
                                 int is_device);
/* Operator and preconditioner sizes: out[0] rows, [1] nonzeros, [2] coarse
 * unknowns of the aggregation level (0 for BiCGStab), [3] 0 conjugate
 * gradients, 1 BiCGStab. */
vcx_status vcx_poisson_info(vcx_poisson p, int64_t out[4]);


/* sum_i V_i U_i per variable [nvar] (FP64, fixed-order tree). */
vcx_status vcx_conservation_sums(vcx_solver s, double *sums);

/* Per-kernel timing with HIP events on the solver's stream.  enable = 1 turns
 * it on and clears the counters.  Kernel names: "gradient" (gradient tile
 * pass; its first launch of a step also reduces the time step), "flux" (flux
 * tile pass with the update of nodes owned by one tile), "update" (update of
 * nodes shared by several tiles), "node_dt", "gradient_shared".  count =
 * launches timed, total_ms = sum of their durations. */
vcx_status vcx_profile_enable(vcx_solver s, int enable);
vcx_status vcx_profile_query(vcx_solver s, const char *kernel, int64_t *count, double *total_ms);

const char *vcx_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
