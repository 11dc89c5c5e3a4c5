/*
 * oracle.h -- plain FP64 CPU oracle for the vertex-centred explicit residual
 * of "AVIP: a low temperature plasma code" (arXiv 2201.01291).
 *
 * TEST INFRASTRUCTURE.  Only the test-suite, the smoke check and the CPU
 * baseline of the benchmark may load this library.  It shares no code,
 * header, table or helper with the HIP library; it is a slow, literal,
 * sequential transcription of the scheme used to check the GPU results.
 *
 * Array conventions (all caller-owned, host memory):
 *   xyz    [nd][nn]      node coordinates
 *   cells  [nv][nc]      simplex connectivity (int64), nv = nd + 1
 *   period [nd] or NULL  box length of each periodic axis, 0 for an open axis
 *   U      [nvar][nn]    nodal conserved state
 *   E      [nd][nn]      prescribed electric field (drift-diffusion)
 *   G      [nvar][nd][nn] nodal gradients
 *   r      [nvar][nn]    residual = integrated net outflow, dU_i/dt = -r_i/V_i
 *
 * Status codes: 0 ok, -1 bad argument, -2 bad mesh, -3 out of memory,
 * -5 unstable (non-finite state, rho<=0 or p<=0).
 */
#ifndef VCX_ORACLE_H
#define VCX_ORACLE_H
#include <stdint.h>

#define OM_MAXSP 16

typedef struct {
  int32_t model;      /* 0 gas (Euler + passive species), 1 drift-diffusion,
                         2 multi-species Navier-Stokes transport */
  int32_t flux;       /* gas: 0 HLLC, 1 Roe; drift-diffusion: 0 limited Lax-Wendroff,
                         2 Scharfetter-Gummel */
  int32_t limiter;    /* 0 first order, 1 minmod, 2 van Leer, 3 Sweby(beta), 4 unlimited */
  int32_t rk;         /* 1..4, low-storage table */
  int32_t nspecies;   /* gas: passive species; drift-diffusion: charged species */
  int32_t closure;    /* 1: node-flux boundary closure on boundary nodes; 2: interpolated
                         fluxes 0.75 F_i + 0.25 F_j on each half boundary edge (2D) */
  int32_t predictor;  /* gas, plane meshes, rk = 1: 1 adds the MUSCL-Hancock half-step
                         evolution to the reconstructed face states, 0 none */
  double beta;        /* Sweby parameter */
  double cfl, fourier;
  double gamma;
  double entropy_fix; /* Roe: Harten delta as a fraction of the Roe sound speed */
  double z[OM_MAXSP], mu[OM_MAXSP], D[OM_MAXSP];  /* drift-diffusion species */
  /* multi-species Navier-Stokes: synthetic species data */
  double Wk[OM_MAXSP];                 /* molar mass [kg/mol] */
  double cpa[OM_MAXSP], cpb[OM_MAXSP], cpc[OM_MAXSP]; /* c_p = R/W (a + b t + c t^2), t = T/1000 */
  double Sc[OM_MAXSP];                 /* Schmidt numbers */
  double mu_ref, T_ref, Pr;            /* mu = mu_ref (T/T_ref)^0.7, lambda = mu c_p / Pr */
  double diel;                         /* drift-diffusion: dielectric time-step constant A_D (0: off) */
} om_phys;

typedef struct om_mesh om_mesh;

om_mesh *om_mesh_create(int nd, int64_t nn, const double *xyz, int64_t nc, int nv,
                        const int64_t *cells, const double *period, int *status);
/* axi = 1: (x, r) plane of an axisymmetric domain (2D, r >= 0, r not
 * periodic): radius-weighted fluxes and node volumes over 2 pi */
om_mesh *om_mesh_create_axi(int nd, int64_t nn, const double *xyz, int64_t nc, int nv,
                            const int64_t *cells, const double *period, int axi, int *status);
void om_axi_geometry(const om_mesh *m, double *Vp, double *Sbr);
void om_mesh_destroy(om_mesh *m);
void om_mesh_counts(const om_mesh *m, int64_t *out /* nn, nc, nbnd_faces, nbnd_nodes */);

/* geometry export: S [nc][nv][nd], Vc [nc], Vn [nn], Sb [nd][nn] */
void om_geometry(const om_mesh *m, double *S, double *Vc, double *Vn, double *Sb);
/* per cell-edge dual normals S_ij [nc][ne][nd] and endpoints [nc][ne][2] */
void om_edge_normals(const om_mesh *m, double *Sij, int64_t *ends);

void om_gradient(const om_mesh *m, int nvar, const double *W, double *G);

/* point-wise building blocks */
double om_slope_limiter(int kind, double beta, double a, double b);
double om_psi_limiter(int kind, double beta, double a, double b);
void om_euler_flux(int nd, int nsp, const double *W, const double *S, double *F);
void om_hllc(int nd, int nsp, double gL, double gR, const double *WL, const double *WR,
             const double *S, double *F);
void om_roe(int nd, int nsp, double gamma, double fix, const double *WL, const double *WR,
            const double *S, double *F);
/* MUSCL-Hancock half-step rate at one node: the time derivative of the
 * reconstructed gas variables w = (rho, rho u, rho E, rho Y, p) [nr] from the
 * Euler equations in quasi-linear form, with the node's state and nodal
 * gradients g [nr][nd] (row-major); out [nr] */
void om_hancock_rate(int nd, int nsp, double gamma, const double *w, const double *g, double *out);
/* Scharfetter-Gummel flux of one species through the cell-edge vector S of
 * edge i -> j (dx = x_j - x_i), face drift V [nd], diffusion D and face
 * gradient gbar [nd] */
double om_sg_flux(int nd, double ui, double uj, const double *V, const double *S, const double *dx,
                  double D, const double *gbar);
/* branch counters of om_hllc / om_roe since the last reset (test
 * instrumentation): [0] HLLC 0 <= S_L, [1] HLLC S_R < 0, [2] HLLC left star,
 * [3] HLLC right star, [4] Roe calls, [5] Roe calls with the entropy fix
 * active; out may be NULL, reset != 0 clears them */
void om_flux_branches(int64_t *out, int reset);

/* multi-species node state from conserved U_i [nvar]: out = T, p, gamma, mu,
 * lambda, D_1..D_N, hs_1..hs_N */
void om_ns_node(int nd, const om_phys *ph, const double *Ui, double *out);
/* conserved multi-species state U [nvar] from prim = (rho, u_1..u_nd, T,
 * Y_1..Y_N) */
void om_ns_conserved(int nd, const om_phys *ph, const double *prim, double *U);
/* central viscous + heat + species-diffusion flux through S (sign: to be
 * subtracted from the convective flux) from face-end primitive data */
void om_viscous_flux(int nd, int nsp, const double *prim_i, const double *prim_j,
                     double rho_i, double rho_j, const double *aux_i, const double *aux_j,
                     const double *gprim_i, const double *gprim_j, const double *S, double *Fv);

int om_residual(const om_mesh *m, const om_phys *ph, const double *U, const double *E,
                double dt, double *r);
int om_flux_scale(const om_mesh *m, const om_phys *ph, const double *U, const double *E,
                  double dt, double *out);
int om_timestep(const om_mesh *m, const om_phys *ph, const double *U, const double *E,
                double *dt);
int om_step(const om_mesh *m, const om_phys *ph, double *U, const double *E, int nsteps,
            double t_end, double *t, double *dt_last, int *steps_done);
void om_sums(const om_mesh *m, int nvar, const double *U, double *sums, double *abssums);

/* Poisson operator: coordinate triplets (nv*nv per cell) of the matrix of
 * -lap phi integrated over the nodal volumes, and |S_i^b| per node */
void om_poisson_coo(const om_mesh *m, int64_t *I, int64_t *K, double *val);
void om_boundary_measure(const om_mesh *m, double *out);
int om_nvar(int nd, const om_phys *ph);

#endif
