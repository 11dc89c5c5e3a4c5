/*
 * oracle.c -- plain FP64 CPU oracle of the vertex-centred explicit residual
 * described in "AVIP: a low temperature plasma code" (arXiv 2201.01291).
 *
 * TEST INFRASTRUCTURE ONLY.  The test-suite, the smoke check and the CPU
 * baseline of the benchmark are the only users.  Nothing here is shared with
 * the HIP library: geometry, gradients, limiters, fluxes and the time loop
 * are written out again, sequentially, in the order the paper states them.
 *
 * Paper passages followed (section / equation names of the paper):
 *   geometry      Sec. "Nomenclature and notations", eq. (node_normal); the
 *                 dual normal identity sum_j S_ij = S_i/n_d and the 2D value
 *                 n_ij = (n_i - n_j)/6 (Sec. "Integrating the Poisson
 *                 equation", cartesian and axisymmetric parts)
 *   cell gradient Sec. "Integrating the Poisson equation":
 *                 grad phi_tau = -1/(V_tau n_d) sum_k phi_k S_k
 *   residual      eq. (vertex_centered_flux): a sum over the cells around a
 *                 node of the flux through each cell-edge piece of the dual
 *                 surface
 *   drift-diff.   Sec. "Limited Lax-Wendroff scheme" and "Central difference
 *                 diffusive flux integration"; Sec. "Scharfetter Gummel
 *                 scheme" (exponential fitting along the edge, central
 *                 across it)
 *   Euler         Sec. "The HLLC solver", eq. (hllc_formulation_mutlicomponent);
 *                 Sec. "The MUSCL procedure implementation in AVIP",
 *                 eq. (virtual_node_reconstruction) and the co-reconstruction
 *                 of pressure
 *   closure       Sec. "Boundary conditions in AVIP", first option (node flux)
 *                 and, in 2D, the second (interpolated 0.75 / 0.25 fluxes)
 *   axisymmetry   Sec. "Cylindrical frames" (Pappus-Guldinus theorems),
 *                 eq. (vertex_centered_flux_axi), Sec. "Geometric source
 *                 terms", eq. (ns_cyl_source_terms): the convective p and,
 *                 for the multi-species model, the diffusive hoop-stress
 *                 source, with the cylindrical velocity divergence in the
 *                 diffusive fluxes; drift-diffusion, gas and multi-species
 *   time step     Sec. "Time step computation", eqs. (dt_conv), (dt_diff) and
 *                 the dielectric time step
 *   RK            Sec. "Time integration of the HLLC MUSCL-Hancock solver",
 *                 table (rk_coeffs)
 *   predictor     the MUSCL-Hancock half-step evolution the paper names (Sec.
 *                 "The HLLC solver" and "Effect of multicomponent mixture",
 *                 after Toro, Chap. 14) without writing it out: here the face
 *                 states gain dt/2 times the node's time derivative of the
 *                 reconstructed variables from the quasi-linear Euler
 *                 equations and the nodal gradients (gas, plane meshes, RK1)
 *   multi-species eq. (ns_reactive) without sources (transport only), total
 *                 non-chemical energy; temperature from the sensible energy by
 *                 iteration and pressure co-reconstructed (Sec. "Effect of
 *                 multicomponent mixture"); central diffusive fluxes as in
 *                 Sec. "Central difference diffusive flux integration"
 *
 * Readings where the paper is silent or garbled (listed in the design notes):
 *   nodal volume V_i = sum_tau V_tau / n_v (median dual);
 *   nodal gradient = volume-weighted average of the cell gradients;
 *   limiters in slope form from van Leer (1974) and Sweby (1984);
 *   LLW ratio r = (u_w - u_k)/(u_m - u_w) (upwind node w, downwind m);
 *   HLLC wave speeds: Davis estimates; species star entry = factor * rho*Y;
 *   Roe flux (not in the paper): textbook, Harten fix on acoustic waves;
 *   RK stage formula carries the time step: U(k) = U^n - a_k dt r/V;
 *   cell size dx = 2 n_d V_tau / sum_k |S_k| (inscribed diameter);
 *   multi-species: synthetic species data (c_p polynomials, molar masses,
 *   Schmidt numbers), mu = mu_ref (T/T_ref)^0.7, lambda = mu c_p / Pr,
 *   D_k = mu / (rho Sc_k), Hirschfelder-Curtiss correction velocity,
 *   Newtonian stress with Stokes' hypothesis, face values as means of the two
 *   cell-edge nodes, temperature by 10 Newton iterations from 1000 K, the
 *   HLLC sound speed of each side from its own node's gamma, inviscid node
 *   flux closure on boundaries.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

struct om_mesh {
  int nd, nv, ne;
  int64_t nn, nc;
  int64_t *cell; /* [nc][nv] */
  double *X;     /* [nc][nv][nd] unwrapped vertex coordinates */
  double *S;     /* [nc][nv][nd] node normals S_k (simplex: outward normal of the opposite
                    face; quadrilateral: minus the sum of its two sides' outward normals) */
  double *orient; /* [nc] quadrilaterals: +1 counter-clockwise vertex order, -1 clockwise */
  double *Vc;    /* [nc] */
  double *Vn;    /* [nn] */
  double *Sb;    /* [nn][nd] boundary node normals */
  char *bnd;     /* [nn] node lies on the domain boundary */
  int64_t nbfaces;
  /* axisymmetric (x, r) meshes (Sec. "Cylindrical frames"): the second
   * coordinate is the radius; fluxes through revolved dual faces carry the
   * centroid radius of the face (first Pappus-Guldinus theorem), node volumes
   * are int r dA over the dual region (second theorem), both over 2 pi */
  int axi;
  double *Rf;    /* [nc][ne] centroid radius of each cell-edge piece of the dual surface */
  double *Vp;    /* [nn] int_{A_i} r dA */
  double *Sbr;   /* [nn][nd] boundary node normals weighted by the centroid radius */
  double *Rn;    /* [nn] node radius */
  /* 2D boundary edges (a, b) with their outward normal share S_f / 2 of
   * each end (boundary-closure option 2) */
  int64_t nbe;
  int64_t *be;   /* [nbe][2] */
  double *beS;   /* [nbe][2] */
};

/* local cell-edges: of a simplex every vertex pair, oriented from the lower
 * to the higher local vertex; of a quadrilateral its four sides in cyclic
 * order (its diagonals are not edges) */
static const int TRI_EDGES[3][2] = {{0, 1}, {0, 2}, {1, 2}};
static const int TET_EDGES[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};
static const int QUAD_EDGES[4][2] = {{0, 1}, {1, 2}, {2, 3}, {3, 0}};

static int is_quad(const om_mesh *m) { return m->nd == 2 && m->nv == 4; }

static const int *edge_of(const om_mesh *m, int e) {
  if (m->nv == 3) return TRI_EDGES[e];
  return is_quad(m) ? QUAD_EDGES[e] : TET_EDGES[e];
}

int om_nvar(int nd, const om_phys *ph) {
  if (ph->model == 1) return ph->nspecies;
  return 2 + nd + ph->nspecies;
}

/* ------------------------------------------------------------------ */
/* multi-species mixture (synthetic species data)                       */
/* ------------------------------------------------------------------ */

#define OM_RGAS 8.314462618
#define OM_T0 298.15
#define OM_NEWTON 10
#define OM_ECHARGE 1.602176634e-19  /* elementary charge [C] */
#define OM_EPS0 8.8541878128e-12    /* vacuum permittivity [F/m] */

/* species sensible enthalpy hs_k(T) = int_{T0}^{T} c_p,k */
static double species_hs(const om_phys *ph, int k, double T) {
  double Rk = OM_RGAS / ph->Wk[k];
  return Rk * (ph->cpa[k] * (T - OM_T0) + ph->cpb[k] * (T * T - OM_T0 * OM_T0) / 2000.0 +
               ph->cpc[k] * (T * T * T - OM_T0 * OM_T0 * OM_T0) / 3.0e6);
}

static double species_cp(const om_phys *ph, int k, double T) {
  double t = T / 1000.0;
  return OM_RGAS / ph->Wk[k] * (ph->cpa[k] + ph->cpb[k] * t + ph->cpc[k] * t * t);
}

/* mixture sensible energy e_s(T) = sum Y_k (hs_k(T) - R_k T) and c_v(T) */
static void mixture_es_cv(const om_phys *ph, const double *Y, double T, double *es, double *cv) {
  double e = 0.0, c = 0.0;
  for (int k = 0; k < ph->nspecies; k++) {
    double Rk = OM_RGAS / ph->Wk[k];
    e += Y[k] * (species_hs(ph, k, T) - Rk * T);
    c += Y[k] * (species_cp(ph, k, T) - Rk);
  }
  *es = e;
  *cv = c;
}

/* Conserved multi-species state from primitives prim = (rho, u_1..u_nd, T,
 * Y_1..Y_N): U = (rho, rho u, rho (e_s(T) + |u|^2/2), rho Y) with the total
 * non-chemical energy of eq. (ns_reactive). */
void om_ns_conserved(int nd, const om_phys *ph, const double *prim, double *U) {
  int ns = ph->nspecies;
  double rho = prim[0], T = prim[1 + nd], uu = 0.0, es, cv;
  for (int d = 0; d < nd; d++) uu += prim[1 + d] * prim[1 + d];
  mixture_es_cv(ph, prim + 2 + nd, T, &es, &cv);
  U[0] = rho;
  for (int d = 0; d < nd; d++) U[1 + d] = rho * prim[1 + d];
  U[1 + nd] = rho * (es + 0.5 * uu);
  for (int k = 0; k < ns; k++) U[2 + nd + k] = rho * prim[2 + nd + k];
}

/* Node state of the multi-species model: out = T, p, gamma, mu, lambda,
 * D_1..D_N, hs_1..hs_N (the temperature solves e_s(T) = E - |u|^2/2). */
void om_ns_node(int nd, const om_phys *ph, const double *Ui, double *out) {
  int ns = ph->nspecies;
  double rho = Ui[0], uu = 0.0, Y[OM_MAXSP];
  for (int d = 0; d < nd; d++) uu += (Ui[1 + d] / rho) * (Ui[1 + d] / rho);
  double es_target = Ui[1 + nd] / rho - 0.5 * uu;
  for (int k = 0; k < ns; k++) Y[k] = Ui[2 + nd + k] / rho;
  double T = 1000.0, es, cv;
  for (int it = 0; it < OM_NEWTON; it++) {
    mixture_es_cv(ph, Y, T, &es, &cv);
    T -= (es - es_target) / cv;
  }
  double r = 0.0, cp = 0.0;
  for (int k = 0; k < ns; k++) {
    r += Y[k] * OM_RGAS / ph->Wk[k];
    cp += Y[k] * species_cp(ph, k, T);
  }
  double mu = ph->mu_ref * pow(T / ph->T_ref, 0.7);
  out[0] = T;
  out[1] = rho * r * T;
  out[2] = cp / (cp - r);
  out[3] = mu;
  out[4] = mu * cp / ph->Pr;
  for (int k = 0; k < ns; k++) {
    out[5 + k] = mu / (rho * ph->Sc[k]);
    out[5 + ns + k] = species_hs(ph, k, T);
  }
}

/* Central diffusive fluxes through S (Sec. "Central difference diffusive flux
 * integration" applied to every diffusive term of eq. ns_reactive): face
 * values are means of the two nodes, gradients the means of the nodal
 * gradients.  prim = (u_1..u_nd, T, Y_1..Y_N), aux = (gamma, mu, lambda,
 * D_k, hs_k), gprim [np][nd].  Returns Fv = (0, tau.S, u.(tau.S) - q.S,
 * -J_k.S), to be subtracted from the convective flux. */
/* hoop: on axisymmetric (x, r) meshes the face value of u_r / r, the third
 * term of the velocity divergence in cylindrical coordinates (0 otherwise) */
static void viscous_flux_div(int nd, int nsp, const double *prim_i, const double *prim_j,
                             double rho_i, double rho_j, const double *aux_i, const double *aux_j,
                             const double *gprim_i, const double *gprim_j, const double *S,
                             double hoop, double *Fv) {
  double rho = 0.5 * (rho_i + rho_j);
  double mu = 0.5 * (aux_i[1] + aux_j[1]), lam = 0.5 * (aux_i[2] + aux_j[2]);
  double u[3], Gu[3][3], div = 0.0;
  for (int a = 0; a < nd; a++) {
    u[a] = 0.5 * (prim_i[a] + prim_j[a]);
    for (int b = 0; b < nd; b++) Gu[a][b] = 0.5 * (gprim_i[a * nd + b] + gprim_j[a * nd + b]);
    div += Gu[a][a];
  }
  div += hoop;
  double tauS[3];
  for (int a = 0; a < nd; a++) {
    tauS[a] = 0.0;
    for (int b = 0; b < nd; b++) {
      double tau = mu * (Gu[a][b] + Gu[b][a] - (a == b ? 2.0 / 3.0 * div : 0.0));
      tauS[a] += tau * S[b];
    }
  }
  /* species diffusion with the correction velocity Vc = sum_k D_k grad Y_k */
  double Vc[3] = {0, 0, 0}, gY[OM_MAXSP][3], D[OM_MAXSP], Yf[OM_MAXSP];
  for (int k = 0; k < nsp; k++) {
    D[k] = 0.5 * (aux_i[3 + k] + aux_j[3 + k]);
    Yf[k] = 0.5 * (prim_i[nd + 1 + k] + prim_j[nd + 1 + k]);
    for (int d = 0; d < nd; d++) {
      gY[k][d] = 0.5 * (gprim_i[(nd + 1 + k) * nd + d] + gprim_j[(nd + 1 + k) * nd + d]);
      Vc[d] += D[k] * gY[k][d];
    }
  }
  double qS = 0.0;
  for (int d = 0; d < nd; d++) qS += -lam * 0.5 * (gprim_i[nd * nd + d] + gprim_j[nd * nd + d]) * S[d];
  Fv[0] = 0.0;
  double utauS = 0.0;
  for (int a = 0; a < nd; a++) {
    Fv[1 + a] = tauS[a];
    utauS += u[a] * tauS[a];
  }
  for (int k = 0; k < nsp; k++) {
    double JS = 0.0;
    for (int d = 0; d < nd; d++) JS += -rho * (D[k] * gY[k][d] - Yf[k] * Vc[d]) * S[d];
    double hs = 0.5 * (aux_i[3 + nsp + k] + aux_j[3 + nsp + k]);
    qS += hs * JS;
    Fv[2 + nd + k] = -JS;
  }
  Fv[1 + nd] = utauS - qS;
}

void om_viscous_flux(int nd, int nsp, const double *prim_i, const double *prim_j,
                     double rho_i, double rho_j, const double *aux_i, const double *aux_j,
                     const double *gprim_i, const double *gprim_j, const double *S, double *Fv) {
  viscous_flux_div(nd, nsp, prim_i, prim_j, rho_i, rho_j, aux_i, aux_j, gprim_i, gprim_j, S, 0.0, Fv);
}

/* ------------------------------------------------------------------ */
/* geometry                                                             */
/* ------------------------------------------------------------------ */

/* Node normal S_k of a simplex: for a simplex every face holds n_d nodes, so
 * eq. (node_normal) gives S_k = (minus the sum of the faces through k), which
 * equals the outward area vector of the face opposite k.  Computed directly
 * as that face's area vector, oriented away from vertex k. */
static void simplex_normals(int nd, const double *X, double *S, double *V) {
  if (nd == 2) {
    double e1x = X[2] - X[0], e1y = X[3] - X[1];
    double e2x = X[4] - X[0], e2y = X[5] - X[1];
    *V = 0.5 * fabs(e1x * e2y - e1y * e2x);
    for (int k = 0; k < 3; k++) {
      int a = (k + 1) % 3, b = (k + 2) % 3;
      double tx = X[2 * b] - X[2 * a], ty = X[2 * b + 1] - X[2 * a + 1];
      double nx = ty, ny = -tx;
      double ox = X[2 * a] - X[2 * k], oy = X[2 * a + 1] - X[2 * k + 1];
      if (nx * ox + ny * oy < 0.0) { nx = -nx; ny = -ny; }
      S[2 * k] = nx;
      S[2 * k + 1] = ny;
    }
  } else {
    double e[3][3];
    for (int q = 0; q < 3; q++)
      for (int d = 0; d < 3; d++) e[q][d] = X[3 * (q + 1) + d] - X[d];
    double det = e[0][0] * (e[1][1] * e[2][2] - e[1][2] * e[2][1]) -
                 e[0][1] * (e[1][0] * e[2][2] - e[1][2] * e[2][0]) +
                 e[0][2] * (e[1][0] * e[2][1] - e[1][1] * e[2][0]);
    *V = fabs(det) / 6.0;
    for (int k = 0; k < 4; k++) {
      int f[3], q = 0;
      for (int v = 0; v < 4; v++)
        if (v != k) f[q++] = v;
      double a[3], b[3], n[3], o[3];
      for (int d = 0; d < 3; d++) {
        a[d] = X[3 * f[1] + d] - X[3 * f[0] + d];
        b[d] = X[3 * f[2] + d] - X[3 * f[0] + d];
        o[d] = X[3 * f[0] + d] - X[3 * k + d];
      }
      n[0] = 0.5 * (a[1] * b[2] - a[2] * b[1]);
      n[1] = 0.5 * (a[2] * b[0] - a[0] * b[2]);
      n[2] = 0.5 * (a[0] * b[1] - a[1] * b[0]);
      if (n[0] * o[0] + n[1] * o[1] + n[2] * o[2] < 0.0) {
        n[0] = -n[0]; n[1] = -n[1]; n[2] = -n[2];
      }
      for (int d = 0; d < 3; d++) S[3 * k + d] = n[d];
    }
  }
}

/* Node normals of a convex quadrilateral (2D, vertices in cyclic order)
 * from eq. (node_normal): in 2D every face is a side with two vertices, so
 * S_k = -(S_f + S_g) over the two sides f, g through k, S_f the outward side
 * normals of side length; V the area.  Returns 0 for a non-convex or
 * degenerate cell.  *orient: +1 counter-clockwise, -1 clockwise. */
static int quad_normals(const double *X, double *S, double *V, double *orient) {
  double A2 = 0.0; /* twice the signed area (shoelace) */
  for (int k = 0; k < 4; k++) {
    const int l = (k + 1) % 4;
    A2 += X[2 * k] * X[2 * l + 1] - X[2 * l] * X[2 * k + 1];
  }
  const double o = A2 > 0.0 ? 1.0 : -1.0;
  for (int k = 0; k < 4; k++) {
    const int l = (k + 1) % 4, q = (k + 2) % 4;
    const double ax = X[2 * l] - X[2 * k], ay = X[2 * l + 1] - X[2 * k + 1];
    const double bx = X[2 * q] - X[2 * l], by = X[2 * q + 1] - X[2 * l + 1];
    if ((ax * by - ay * bx) * o <= 0.0) return 0; /* every corner turns the same way */
  }
  double N[4][2];
  for (int k = 0; k < 4; k++) {
    const int l = (k + 1) % 4;
    const double tx = X[2 * l] - X[2 * k], ty = X[2 * l + 1] - X[2 * k + 1];
    N[k][0] = o * ty;
    N[k][1] = -o * tx;
  }
  for (int k = 0; k < 4; k++) {
    const int p = (k + 3) % 4;
    S[2 * k] = -(N[k][0] + N[p][0]);
    S[2 * k + 1] = -(N[k][1] + N[p][1]);
  }
  *V = 0.5 * fabs(A2);
  *orient = o;
  return 1;
}

/* Outward normal (of side length) of side k -> k+1 of a quadrilateral */
static void quad_side_normal(const double *X, int k, double orient, double *n) {
  const int l = (k + 1) % 4;
  n[0] = orient * (X[2 * l + 1] - X[2 * k + 1]);
  n[1] = -orient * (X[2 * l] - X[2 * k]);
}

typedef struct {
  int64_t key[3];
  int64_t cell;
  int k;
} face_rec;

static int face_cmp(const void *pa, const void *pb) {
  const face_rec *a = pa, *b = pb;
  for (int q = 0; q < 3; q++) {
    if (a->key[q] < b->key[q]) return -1;
    if (a->key[q] > b->key[q]) return 1;
  }
  if (a->cell < b->cell) return -1;
  if (a->cell > b->cell) return 1;
  return 0;
}

static void sort_small(int64_t *v, int n) {
  for (int i = 1; i < n; i++)
    for (int j = i; j > 0 && v[j - 1] > v[j]; j--) {
      int64_t t = v[j]; v[j] = v[j - 1]; v[j - 1] = t;
    }
}

void om_mesh_destroy(om_mesh *m) {
  if (!m) return;
  free(m->cell); free(m->X); free(m->S); free(m->Vc); free(m->Vn); free(m->Sb); free(m->bnd);
  free(m->Rf); free(m->Vp); free(m->Sbr); free(m->Rn); free(m->be); free(m->beS); free(m->orient);
  free(m);
}

om_mesh *om_mesh_create(int nd, int64_t nn, const double *xyz, int64_t nc, int nv,
                        const int64_t *cells, const double *period, int *status) {
  return om_mesh_create_axi(nd, nn, xyz, nc, nv, cells, period, 0, status);
}

om_mesh *om_mesh_create_axi(int nd, int64_t nn, const double *xyz, int64_t nc, int nv,
                            const int64_t *cells, const double *period, int axi, int *status) {
  *status = -1;
  if (!(nd == 2 || nd == 3) || !(nv == nd + 1 || (nd == 2 && nv == 4)) || nn <= 0 || nc <= 0 || !xyz ||
      !cells)
    return NULL;
  if (axi && (nd != 2 || (period && period[1] > 0.0))) return NULL;  /* (x, r) plane, r not periodic */
  if (axi)
    for (int64_t i = 0; i < nn; i++)
      if (xyz[nn + i] < 0.0) return NULL;
  om_mesh *m = calloc(1, sizeof(*m));
  if (!m) { *status = -3; return NULL; }
  m->nd = nd; m->nv = nv; m->ne = nv == 3 ? 3 : (nd == 2 ? 4 : 6); m->nn = nn; m->nc = nc;
  m->orient = calloc(nc, sizeof(double));
  if (!m->orient) { om_mesh_destroy(m); *status = -3; return NULL; }
  m->cell = malloc(sizeof(int64_t) * nc * nv);
  m->X = malloc(sizeof(double) * nc * nv * nd);
  m->S = malloc(sizeof(double) * nc * nv * nd);
  m->Vc = malloc(sizeof(double) * nc);
  m->Vn = calloc(nn, sizeof(double));
  m->Sb = calloc(nn * nd, sizeof(double));
  m->bnd = calloc(nn, 1);
  if (!m->cell || !m->X || !m->S || !m->Vc || !m->Vn || !m->Sb || !m->bnd) {
    om_mesh_destroy(m); *status = -3; return NULL;
  }
  double vmax = 0.0;
  for (int64_t c = 0; c < nc; c++) {
    for (int k = 0; k < nv; k++) {
      int64_t i = cells[(int64_t)k * nc + c];
      if (i < 0 || i >= nn) { om_mesh_destroy(m); *status = -2; return NULL; }
      m->cell[c * nv + k] = i;
    }
    /* unwrap to the minimum image of the first vertex */
    double *X = m->X + c * nv * nd;
    for (int k = 0; k < nv; k++)
      for (int d = 0; d < nd; d++) {
        double x = xyz[(int64_t)d * nn + m->cell[c * nv + k]];
        if (period && period[d] > 0.0 && k > 0) {
          double x0 = X[d];
          x -= period[d] * nearbyint((x - x0) / period[d]);
        }
        X[k * nd + d] = x;
      }
    if (is_quad(m)) {
      if (!quad_normals(X, m->S + c * nv * nd, &m->Vc[c], &m->orient[c])) {
        om_mesh_destroy(m); *status = -2; return NULL;
      }
    } else {
      simplex_normals(nd, X, m->S + c * nv * nd, &m->Vc[c]);
    }
    if (m->Vc[c] > vmax) vmax = m->Vc[c];
  }
  for (int64_t c = 0; c < nc; c++)
    if (!(m->Vc[c] > 1e-12 * vmax)) { om_mesh_destroy(m); *status = -2; return NULL; }
  for (int64_t c = 0; c < nc; c++)
    for (int k = 0; k < nv; k++) m->Vn[m->cell[c * nv + k]] += m->Vc[c] / nv;
  if (axi) {
    m->axi = 1;
    m->Rf = malloc(sizeof(double) * nc * m->ne);
    m->Vp = calloc(nn, sizeof(double));
    m->Sbr = calloc(nn * nd, sizeof(double));
    m->Rn = malloc(sizeof(double) * nn);
    if (!m->Rf || !m->Vp || !m->Sbr || !m->Rn) { om_mesh_destroy(m); *status = -3; return NULL; }
    for (int64_t i = 0; i < nn; i++) m->Rn[i] = xyz[nn + i];
    for (int64_t c = 0; c < nc; c++) {
      if (is_quad(m)) {
        /* quadrilateral: the dual piece of side (a, b) runs from its
         * midpoint to the centre C (mean of the vertices); node k's dual
         * region is the quadrilateral (X_k, M_k, C, M_p) with M_k, M_p the
         * midpoints of its two sides, split into triangles (X_k, M_k, C) and
         * (X_k, C, M_p) whose first moments are area times mean radius */
        const double *X = m->X + c * 8;
        double C[2] = {0.0, 0.0};
        for (int k = 0; k < 4; k++) {
          C[0] += 0.25 * X[2 * k];
          C[1] += 0.25 * X[2 * k + 1];
        }
        for (int e = 0; e < 4; e++) {
          const int *ab = edge_of(m, e);
          m->Rf[c * m->ne + e] = 0.5 * (0.5 * (X[2 * ab[0] + 1] + X[2 * ab[1] + 1]) + C[1]);
        }
        for (int k = 0; k < 4; k++) {
          const int l = (k + 1) % 4, p = (k + 3) % 4;
          const double Mk[2] = {0.5 * (X[2 * k] + X[2 * l]), 0.5 * (X[2 * k + 1] + X[2 * l + 1])};
          const double Mp[2] = {0.5 * (X[2 * k] + X[2 * p]), 0.5 * (X[2 * k + 1] + X[2 * p + 1])};
          const double *P0 = X + 2 * k;
          const double a1 = 0.5 * fabs((Mk[0] - P0[0]) * (C[1] - P0[1]) - (Mk[1] - P0[1]) * (C[0] - P0[0]));
          const double a2 = 0.5 * fabs((C[0] - P0[0]) * (Mp[1] - P0[1]) - (C[1] - P0[1]) * (Mp[0] - P0[0]));
          m->Vp[m->cell[c * 4 + k]] += a1 * (P0[1] + Mk[1] + C[1]) / 3.0 + a2 * (P0[1] + C[1] + Mp[1]) / 3.0;
        }
        continue;
      }
      const double *X = m->X + c * 3 * 2;
      const double r[3] = {X[1], X[3], X[5]};
      const double rc = (r[0] + r[1] + r[2]) / 3.0;
      /* dual piece of edge (a, b): from the edge midpoint to the centroid */
      for (int e = 0; e < 3; e++) {
        const int *ab = edge_of(m, e);
        const double rm = 0.5 * (r[ab[0]] + r[ab[1]]);
        m->Rf[c * m->ne + e] = 0.5 * (rm + rc);
      }
      /* node k's dual region in the triangle: the quadrilateral (X_k,
       * midpoint k-l, centroid, midpoint k-m), two triangles of area A/6 */
      for (int k = 0; k < 3; k++) {
        const int l = (k + 1) % 3, q = (k + 2) % 3;
        const double ml = 0.5 * (r[k] + r[l]), mq = 0.5 * (r[k] + r[q]);
        const double mom = m->Vc[c] / 6.0 * ((r[k] + ml + rc) / 3.0 + (r[k] + rc + mq) / 3.0);
        m->Vp[m->cell[c * 3 + k]] += mom;
      }
    }
  }

  /* boundary faces: faces owned by exactly one cell */
  int64_t nf = nc * nv;
  face_rec *f = malloc(sizeof(face_rec) * nf);
  if (!f) { om_mesh_destroy(m); *status = -3; return NULL; }
  for (int64_t c = 0; c < nc; c++)
    for (int k = 0; k < nv; k++) {
      face_rec *r = &f[c * nv + k];
      int q = 0;
      r->key[0] = r->key[1] = r->key[2] = -1;
      if (is_quad(m)) {
        /* face k of a quadrilateral: its side k -> k+1 */
        r->key[0] = m->cell[c * nv + k];
        r->key[1] = m->cell[c * nv + (k + 1) % 4];
      } else {
        /* face k of a simplex: the one opposite vertex k */
        for (int v = 0; v < nv; v++)
          if (v != k) r->key[q++] = m->cell[c * nv + v];
      }
      sort_small(r->key, nd);
      r->cell = c;
      r->k = k;
    }
  qsort(f, nf, sizeof(face_rec), face_cmp);
  if (nd == 2) {
    m->be = malloc(sizeof(int64_t) * 2 * nf);
    m->beS = malloc(sizeof(double) * 2 * nf);
    if (!m->be || !m->beS) { free(f); om_mesh_destroy(m); *status = -3; return NULL; }
  }
  for (int64_t a = 0; a < nf;) {
    int64_t b = a + 1;
    while (b < nf && memcmp(f[b].key, f[a].key, sizeof(f[a].key)) == 0) b++;
    if (b - a > 2) { free(f); om_mesh_destroy(m); *status = -2; return NULL; }
    if (b - a == 1) {
      /* its outward area vector: of the face opposite vertex k of a simplex,
       * S_k; of side k of a quadrilateral, that side's outward normal.  Each
       * of its n_d nodes receives an equal share (boundary node normal S_i^b) */
      double Sq[2];
      const double *Sk = m->S + (f[a].cell * nv + f[a].k) * nd;
      if (is_quad(m)) {
        quad_side_normal(m->X + f[a].cell * 8, f[a].k, m->orient[f[a].cell], Sq);
        Sk = Sq;
      }
      for (int q = 0; q < nd; q++) {
        int64_t i = f[a].key[q];
        m->bnd[i] = 1;
        for (int d = 0; d < nd; d++) m->Sb[i * nd + d] += Sk[d] / nd;
        if (m->axi) {
          /* node i's half of the boundary edge: centroid radius (3 r_i + r_j)/4 */
          const int64_t j = f[a].key[1 - q];
          const double rf = 0.75 * xyz[nn + i] + 0.25 * xyz[nn + j];
          for (int d = 0; d < nd; d++) m->Sbr[i * nd + d] += Sk[d] / nd * rf;
        }
      }
      if (nd == 2) {
        m->be[m->nbe * 2] = f[a].key[0];
        m->be[m->nbe * 2 + 1] = f[a].key[1];
        m->beS[m->nbe * 2] = Sk[0] / 2;
        m->beS[m->nbe * 2 + 1] = Sk[1] / 2;
        m->nbe++;
      }
      m->nbfaces++;
    }
    a = b;
  }
  free(f);
  *status = 0;
  return m;
}

void om_mesh_counts(const om_mesh *m, int64_t *out) {
  int64_t nb = 0;
  for (int64_t i = 0; i < m->nn; i++) nb += m->bnd[i];
  out[0] = m->nn; out[1] = m->nc; out[2] = m->nbfaces; out[3] = nb;
}

/* axisymmetric meshes: int_{A_i} r dA per node (else copies V_i), and the
 * radius-weighted boundary normals [nd][nn] */
void om_axi_geometry(const om_mesh *m, double *Vp, double *Sbr) {
  for (int64_t i = 0; i < m->nn; i++) {
    if (Vp) Vp[i] = m->axi ? m->Vp[i] : m->Vn[i];
    if (Sbr)
      for (int d = 0; d < m->nd; d++) Sbr[d * m->nn + i] = m->axi ? m->Sbr[i * m->nd + d] : m->Sb[i * m->nd + d];
  }
}

void om_geometry(const om_mesh *m, double *S, double *Vc, double *Vn, double *Sb) {
  if (S) memcpy(S, m->S, sizeof(double) * m->nc * m->nv * m->nd);
  if (Vc) memcpy(Vc, m->Vc, sizeof(double) * m->nc);
  if (Vn) memcpy(Vn, m->Vn, sizeof(double) * m->nn);
  if (Sb)
    for (int d = 0; d < m->nd; d++)
      for (int64_t i = 0; i < m->nn; i++) Sb[d * m->nn + i] = m->Sb[i * m->nd + d];
}

/* dual-surface normal of cell-edge (a,b): S_ab = (S_a - S_b) / (n_d n_v) */
static void edge_normal(const om_mesh *m, int64_t c, int a, int b, double *Sab) {
  if (is_quad(m)) {
    /* the dual face in a quadrilateral: the segment from the side's midpoint
     * to the cell centre (mean of the vertices), oriented from a to b */
    const double *X = m->X + c * 8;
    double cx = 0.0, cy = 0.0;
    for (int k = 0; k < 4; k++) {
      cx += 0.25 * X[2 * k];
      cy += 0.25 * X[2 * k + 1];
    }
    const double tx = cx - 0.5 * (X[2 * a] + X[2 * b]), ty = cy - 0.5 * (X[2 * a + 1] + X[2 * b + 1]);
    double nx = ty, ny = -tx;
    if (nx * (X[2 * b] - X[2 * a]) + ny * (X[2 * b + 1] - X[2 * a + 1]) < 0.0) {
      nx = -nx;
      ny = -ny;
    }
    Sab[0] = nx;
    Sab[1] = ny;
    return;
  }
  const double *S = m->S + c * m->nv * m->nd;
  for (int d = 0; d < m->nd; d++)
    Sab[d] = (S[a * m->nd + d] - S[b * m->nd + d]) / (double)(m->nd * m->nv);
}

void om_edge_normals(const om_mesh *m, double *Sij, int64_t *ends) {
  for (int64_t c = 0; c < m->nc; c++)
    for (int e = 0; e < m->ne; e++) {
      const int *ab = edge_of(m, e);
      edge_normal(m, c, ab[0], ab[1], Sij + (c * m->ne + e) * m->nd);
      ends[(c * m->ne + e) * 2] = m->cell[c * m->nv + ab[0]];
      ends[(c * m->ne + e) * 2 + 1] = m->cell[c * m->nv + ab[1]];
    }
}

/* ------------------------------------------------------------------ */
/* gradients                                                            */
/* ------------------------------------------------------------------ */

/* cell gradient grad W_tau = -1/(n_d V_tau) sum_k W_k S_k, then the nodal
 * gradient as the volume-weighted mean over the cells around the node:
 * grad W_i = (1/V_i) sum_tau (V_tau/n_v) grad W_tau */
void om_gradient(const om_mesh *m, int nvar, const double *W, double *G) {
  int nd = m->nd, nv = m->nv;
  int64_t nn = m->nn;
  memset(G, 0, sizeof(double) * nvar * nd * nn);
  for (int64_t c = 0; c < m->nc; c++) {
    const double *S = m->S + c * nv * nd;
    for (int v = 0; v < nvar; v++) {
      double g[3] = {0, 0, 0};
      for (int k = 0; k < nv; k++) {
        double w = W[(int64_t)v * nn + m->cell[c * nv + k]];
        for (int d = 0; d < nd; d++) g[d] += w * S[k * nd + d];
      }
      for (int d = 0; d < nd; d++) g[d] *= -1.0 / (nd * m->Vc[c]);
      for (int k = 0; k < nv; k++) {
        int64_t i = m->cell[c * nv + k];
        for (int d = 0; d < nd; d++) G[((int64_t)v * nd + d) * nn + i] += m->Vc[c] / nv * g[d];
      }
    }
  }
  for (int v = 0; v < nvar; v++)
    for (int d = 0; d < nd; d++)
      for (int64_t i = 0; i < nn; i++) G[((int64_t)v * nd + d) * nn + i] /= m->Vn[i];
}

/* ------------------------------------------------------------------ */
/* limiters                                                             */
/* ------------------------------------------------------------------ */

static double sgn(double x) { return x > 0 ? 1.0 : (x < 0 ? -1.0 : 0.0); }

/* Slope form L(a, b) of the limited slope (van Leer 1974, Sweby 1984):
 * 0 first order, 1 minmod, 2 van Leer harmonic mean, 3 Sweby-beta,
 * 4 unlimited centred slope (a + b)/2. */
double om_slope_limiter(int kind, double beta, double a, double b) {
  if (kind == 0) return 0.0;
  if (kind == 4) return 0.5 * (a + b);
  if (a * b <= 0.0) return 0.0;
  double aa = fabs(a), bb = fabs(b);
  if (kind == 1) return sgn(a) * (aa < bb ? aa : bb);
  if (kind == 2) return 2.0 * a * b / (a + b);
  double m1 = beta * aa < bb ? beta * aa : bb;
  double m2 = aa < beta * bb ? aa : beta * bb;
  return sgn(a) * (m1 > m2 ? m1 : m2);
}

/* Flux-limiter form Psi(R) with R = a/b for the limited Lax-Wendroff flux:
 * 0 upwind (Psi = 0), 1 minmod, 2 van Leer (R+|R|)/(1+|R|), 3 Sweby-beta
 * max(0, min(beta R, 1), min(R, beta)), 4 plain Lax-Wendroff (Psi = 1).
 * Psi = 0 when a*b <= 0 (which includes b = 0). */
double om_psi_limiter(int kind, double beta, double a, double b) {
  if (kind == 0) return 0.0;
  if (kind == 4) return 1.0;
  if (a * b <= 0.0) return 0.0;
  double R = a / b;
  if (kind == 2) return (R + fabs(R)) / (1.0 + fabs(R));
  double bt = kind == 1 ? 1.0 : beta;
  double m1 = bt * R < 1.0 ? bt * R : 1.0;
  double m2 = R < bt ? R : bt;
  double p = m1 > m2 ? m1 : m2;
  return p > 0.0 ? p : 0.0;
}

/* ------------------------------------------------------------------ */
/* gas fluxes; W = (rho, rho u_1..rho u_nd, rho E, rho Y_1..rho Y_ns, p)   */
/* ------------------------------------------------------------------ */

/* physical Euler flux F(W) . S (tensor form of Sec. "The HLLC solver") */
void om_euler_flux(int nd, int nsp, const double *W, const double *S, double *F) {
  double rho = W[0], rhoE = W[1 + nd], p = W[2 + nd + nsp];
  double q = 0.0;
  for (int d = 0; d < nd; d++) q += W[1 + d] / rho * S[d];
  F[0] = rho * q;
  for (int d = 0; d < nd; d++) F[1 + d] = W[1 + d] * q + p * S[d];
  F[1 + nd] = (rhoE + p) * q;
  for (int k = 0; k < nsp; k++) F[2 + nd + k] = W[2 + nd + k] * q;
}

/* Branch counters of the two Riemann fluxes, for tests that must show an
 * input reaches a given branch: [0] HLLC 0 <= S_L, [1] HLLC S_R < 0, [2] HLLC
 * left star state, [3] HLLC right star state, [4] Roe calls, [5] Roe calls
 * with Harten's fix active on an acoustic wave. */
static int64_t om_branch_count[6];

/* MUSCL-Hancock half-step rate at one node.  The reconstructed variables
 * are w = (rho, m = rho u, rho E, rho Y_s, p) with gradients g.  The velocity
 * gradient follows from the momentum and density gradients,
 * du_k/dx_d = (dm_k/dx_d - u_k drho/dx_d) / rho, and the Euler equations give
 *   d rho/dt    = -div m
 *   d m_k/dt    = -(u . grad m_k + m_k div u) - dp/dx_k
 *   d rho E/dt  = -(u . grad (rho E) + u . grad p + (rho E + p) div u)
 *   d rho Y/dt  = -(u . grad (rho Y) + rho Y div u)
 *   d p/dt      = -(u . grad p + gamma p div u)   (constant-gamma ideal gas) */
void om_hancock_rate(int nd, int nsp, double gamma, const double *w, const double *g, double *out) {
  const int nvar = 2 + nd + nsp, nr = nvar + 1;
  const double rho = w[0], rhoE = w[1 + nd], p = w[nr - 1];
  double u[3], du[3][3], divu = 0.0;
  for (int k = 0; k < nd; k++) u[k] = w[1 + k] / rho;
  for (int k = 0; k < nd; k++)
    for (int d = 0; d < nd; d++) du[k][d] = (g[(1 + k) * nd + d] - u[k] * g[d]) / rho;
  for (int d = 0; d < nd; d++) divu += du[d][d];
  /* u . grad of row v */
  double adv[2 + 3 + OM_MAXSP + 1];
  for (int v = 0; v < nr; v++) {
    adv[v] = 0.0;
    for (int d = 0; d < nd; d++) adv[v] += u[d] * g[v * nd + d];
  }
  out[0] = 0.0;
  for (int d = 0; d < nd; d++) out[0] -= g[(1 + d) * nd + d];
  for (int k = 0; k < nd; k++) out[1 + k] = -(adv[1 + k] + w[1 + k] * divu) - g[(nr - 1) * nd + k];
  out[1 + nd] = -(adv[1 + nd] + adv[nr - 1] + (rhoE + p) * divu);
  for (int s = 0; s < nsp; s++) out[2 + nd + s] = -(adv[2 + nd + s] + w[2 + nd + s] * divu);
  out[nr - 1] = -(adv[nr - 1] + gamma * p * divu);
}

void om_flux_branches(int64_t *out, int reset) {
  for (int k = 0; k < 6; k++) {
    if (out) out[k] = om_branch_count[k];
    if (reset) om_branch_count[k] = 0;
  }
}

/* HLLC flux through the area vector S (|S| times the unit-normal flux).
 * The rotation to the edge frame of the paper is written without forming the
 * rotation matrix: normal velocity q = u.n, tangential velocity kept as is.
 * Star state: eq. (hllc_formulation_mutlicomponent).  gL, gR: ratio of
 * specific heats of the two sides. */
void om_hllc(int nd, int nsp, double gL, double gR, const double *WL, const double *WR,
             const double *S, double *F) {
  int nvar = 2 + nd + nsp;
  double A = 0.0;
  for (int d = 0; d < nd; d++) A += S[d] * S[d];
  A = sqrt(A);
  double n[3] = {0, 0, 0};
  for (int d = 0; d < nd; d++) n[d] = S[d] / A;
  double rL = WL[0], rR = WR[0], pL = WL[nvar], pR = WR[nvar];
  double qL = 0, qR = 0;
  for (int d = 0; d < nd; d++) { qL += WL[1 + d] / rL * n[d]; qR += WR[1 + d] / rR * n[d]; }
  double aL = sqrt(gL * pL / rL), aR = sqrt(gR * pR / rR);
  double SL = fmin(qL - aL, qR - aR), SR = fmax(qL + aL, qR + aR);
  double Ss = (pR - pL + rL * qL * (SL - qL) - rR * qR * (SR - qR)) /
              (rL * (SL - qL) - rR * (SR - qR));
  double FK[2 + 3 + OM_MAXSP];
  if (0.0 <= SL) {
    om_branch_count[0]++;
    om_euler_flux(nd, nsp, WL, n, FK);
  } else if (SR < 0.0) {
    om_branch_count[1]++;
    om_euler_flux(nd, nsp, WR, n, FK);
  } else {
    om_branch_count[(0.0 <= Ss) ? 2 : 3]++;
    const double *WK = (0.0 <= Ss) ? WL : WR;
    double SK = (0.0 <= Ss) ? SL : SR;
    double rK = WK[0], pK = WK[nvar];
    double qK = (0.0 <= Ss) ? qL : qR;
    om_euler_flux(nd, nsp, WK, n, FK);
    double fac = rK * (SK - qK) / (SK - Ss);
    double Us[2 + 3 + OM_MAXSP];
    Us[0] = fac;
    for (int d = 0; d < nd; d++) Us[1 + d] = fac * (WK[1 + d] / rK + (Ss - qK) * n[d]);
    Us[1 + nd] = fac * (WK[1 + nd] / rK + (Ss - qK) * (Ss + pK / (rK * (SK - qK))));
    for (int k = 0; k < nsp; k++) Us[2 + nd + k] = fac * WK[2 + nd + k] / rK;
    for (int v = 0; v < nvar; v++) FK[v] += SK * (Us[v] - WK[v]);
  }
  for (int v = 0; v < nvar; v++) F[v] = A * FK[v];
}

/* Roe flux (textbook, not given in the paper): F = (F_L + F_R)/2 - 1/2 sum
 * |lambda_k| alpha_k K_k with sqrt(rho)-weighted averages; passive species
 * travel with the contact.  Harten's fix |l| -> (l^2 + d^2)/(2d) for |l| < d
 * on the two acoustic waves, d = fix * (Roe sound speed). */
void om_roe(int nd, int nsp, double gamma, double fix, const double *WL, const double *WR,
            const double *S, double *F) {
  int nvar = 2 + nd + nsp;
  double A = 0.0;
  for (int d = 0; d < nd; d++) A += S[d] * S[d];
  A = sqrt(A);
  double n[3] = {0, 0, 0};
  for (int d = 0; d < nd; d++) n[d] = S[d] / A;
  double rL = WL[0], rR = WR[0], pL = WL[nvar], pR = WR[nvar];
  double uL[3] = {0, 0, 0}, uR[3] = {0, 0, 0};
  for (int d = 0; d < nd; d++) { uL[d] = WL[1 + d] / rL; uR[d] = WR[1 + d] / rR; }
  double HL = (WL[1 + nd] + pL) / rL, HR = (WR[1 + nd] + pR) / rR;
  double sL = sqrt(rL), sR = sqrt(rR), w = sL + sR;
  double u[3] = {0, 0, 0}, uu = 0.0, q = 0.0, qL = 0.0, qR = 0.0;
  for (int d = 0; d < nd; d++) {
    u[d] = (sL * uL[d] + sR * uR[d]) / w;
    uu += u[d] * u[d];
    q += u[d] * n[d];
    qL += uL[d] * n[d];
    qR += uR[d] * n[d];
  }
  double H = (sL * HL + sR * HR) / w;
  double a = sqrt((gamma - 1.0) * (H - 0.5 * uu));
  double rho = sL * sR;
  double dr = rR - rL, dp = pR - pL, dq = qR - qL;
  double a1 = (dp - rho * a * dq) / (2.0 * a * a);
  double a5 = (dp + rho * a * dq) / (2.0 * a * a);
  double a2 = dr - dp / (a * a);
  double l1 = fabs(q - a), l2 = fabs(q), l5 = fabs(q + a);
  double delta = fix * a;
  om_branch_count[4]++;
  if (delta > 0.0) {
    if (l1 < delta || l5 < delta) om_branch_count[5]++;
    if (l1 < delta) l1 = (l1 * l1 + delta * delta) / (2.0 * delta);
    if (l5 < delta) l5 = (l5 * l5 + delta * delta) / (2.0 * delta);
  }
  double Dis[2 + 3 + OM_MAXSP];
  /* acoustic waves */
  Dis[0] = l1 * a1 + l2 * a2 + l5 * a5;
  for (int d = 0; d < nd; d++)
    Dis[1 + d] = l1 * a1 * (u[d] - a * n[d]) + l2 * a2 * u[d] + l5 * a5 * (u[d] + a * n[d]);
  Dis[1 + nd] = l1 * a1 * (H - q * a) + l2 * a2 * 0.5 * uu + l5 * a5 * (H + q * a);
  /* shear waves: jump of the tangential velocity */
  double dut[3] = {0, 0, 0}, udut = 0.0;
  for (int d = 0; d < nd; d++) {
    dut[d] = (uR[d] - uL[d]) - dq * n[d];
    udut += u[d] * dut[d];
  }
  for (int d = 0; d < nd; d++) Dis[1 + d] += l2 * rho * dut[d];
  Dis[1 + nd] += l2 * rho * udut;
  /* species: carried by the acoustic and entropy waves plus their own contact */
  for (int k = 0; k < nsp; k++) {
    double YL = WL[2 + nd + k] / rL, YR = WR[2 + nd + k] / rR;
    double Y = (sL * YL + sR * YR) / w;
    Dis[2 + nd + k] = (l1 * a1 + l2 * a2 + l5 * a5) * Y + l2 * rho * (YR - YL);
  }
  double FL[2 + 3 + OM_MAXSP], FR[2 + 3 + OM_MAXSP];
  om_euler_flux(nd, nsp, WL, n, FL);
  om_euler_flux(nd, nsp, WR, n, FR);
  for (int v = 0; v < nvar; v++) F[v] = A * (0.5 * (FL[v] + FR[v]) - 0.5 * Dis[v]);
}

/* ------------------------------------------------------------------ */
/* residuals                                                            */
/* ------------------------------------------------------------------ */

static double pressure_of(int nd, const double *U, int64_t nn, int64_t i, double gamma) {
  double rho = U[i], ke = 0.0;
  for (int d = 0; d < nd; d++) {
    double m = U[(int64_t)(1 + d) * nn + i];
    ke += m * m;
  }
  return (gamma - 1.0) * (U[(int64_t)(1 + nd) * nn + i] - 0.5 * ke / rho);
}

static int residual_gas(const om_mesh *m, const om_phys *ph, const double *U, double dt, double *r,
                        int absmode) {
  int nd = m->nd, nv = m->nv, nsp = ph->nspecies;
  int nvar = 2 + nd + nsp, nr = nvar + 1;
  int ns_model = ph->model == 2;
  int np = nd + 1 + nsp, na = 3 + 2 * nsp;
  int64_t nn = m->nn;
  /* reconstructed variables: conserved state plus pressure */
  double *W = malloc(sizeof(double) * nr * nn);
  double *G = malloc(sizeof(double) * nr * nd * nn);
  /* multi-species: primitive fields (u, T, Y), their gradients, node aux */
  double *P = ns_model ? malloc(sizeof(double) * np * nn) : NULL;
  double *GP = ns_model ? malloc(sizeof(double) * np * nd * nn) : NULL;
  double *A = ns_model ? malloc(sizeof(double) * na * nn) : NULL;
  if (!W || !G || (ns_model && (!P || !GP || !A))) {
    free(W); free(G); free(P); free(GP); free(A);
    return -3;
  }
  memcpy(W, U, sizeof(double) * nvar * nn);
  if (!ns_model) {
    for (int64_t i = 0; i < nn; i++) W[(int64_t)nvar * nn + i] = pressure_of(nd, U, nn, i, ph->gamma);
  } else {
    double Ui[2 + 3 + OM_MAXSP], out[5 + 2 * OM_MAXSP];
    for (int64_t i = 0; i < nn; i++) {
      for (int v = 0; v < nvar; v++) Ui[v] = U[(int64_t)v * nn + i];
      om_ns_node(nd, ph, Ui, out);
      W[(int64_t)nvar * nn + i] = out[1];
      for (int d = 0; d < nd; d++) P[(int64_t)d * nn + i] = Ui[1 + d] / Ui[0];
      P[(int64_t)nd * nn + i] = out[0];
      for (int k = 0; k < nsp; k++) P[(int64_t)(nd + 1 + k) * nn + i] = Ui[2 + nd + k] / Ui[0];
      A[i] = out[2];
      for (int q = 1; q < na; q++) A[(int64_t)q * nn + i] = out[2 + q];
    }
    om_gradient(m, np, P, GP);
  }
  om_gradient(m, nr, W, G);
  /* MUSCL-Hancock predictor: dt/2 times each node's half-step rate */
  double *H = NULL;
  if (ph->predictor) {
    H = malloc(sizeof(double) * nr * nn);
    if (!H) {
      free(W); free(G); free(P); free(GP); free(A);
      return -3;
    }
    double wi[2 + 3 + OM_MAXSP + 1], gi[(2 + 3 + OM_MAXSP + 1) * 3], hi[2 + 3 + OM_MAXSP + 1];
    for (int64_t i = 0; i < nn; i++) {
      for (int v = 0; v < nr; v++) {
        wi[v] = W[(int64_t)v * nn + i];
        for (int d = 0; d < nd; d++) gi[v * nd + d] = G[((int64_t)v * nd + d) * nn + i];
      }
      om_hancock_rate(nd, nsp, ph->gamma, wi, gi, hi);
      for (int v = 0; v < nr; v++) H[(int64_t)v * nn + i] = 0.5 * dt * hi[v];
    }
  }
  memset(r, 0, sizeof(double) * nvar * nn);
  for (int64_t c = 0; c < m->nc; c++) {
    const double *X = m->X + c * nv * nd;
    for (int e = 0; e < m->ne; e++) {
      const int *ab = edge_of(m, e);
      int64_t i = m->cell[c * nv + ab[0]], j = m->cell[c * nv + ab[1]];
      double Sij[3], dx[3];
      edge_normal(m, c, ab[0], ab[1], Sij);
      for (int d = 0; d < nd; d++) dx[d] = X[ab[1] * nd + d] - X[ab[0] * nd + d];
      double WL[2 + 3 + OM_MAXSP + 1], WR[2 + 3 + OM_MAXSP + 1];
      for (int v = 0; v < nr; v++) {
        double wi = W[(int64_t)v * nn + i], wj = W[(int64_t)v * nn + j];
        double gi = 0.0, gj = 0.0;
        for (int d = 0; d < nd; d++) {
          gi += G[((int64_t)v * nd + d) * nn + i] * dx[d];
          gj += G[((int64_t)v * nd + d) * nn + j] * dx[d];
        }
        double delta = wj - wi;
        /* virtual upwind nodes: U_i - U_l = 2 grad U_i . ij - (U_j - U_i),
         * U_k - U_j = 2 grad U_j . ij - (U_j - U_i) */
        double d_li = 2.0 * gi - delta, d_jk = 2.0 * gj - delta;
        double bar_i = om_slope_limiter(ph->limiter, ph->beta, d_li, delta);
        double bar_j = om_slope_limiter(ph->limiter, ph->beta, delta, d_jk);
        WL[v] = wi + 0.5 * bar_i;
        WR[v] = wj - 0.5 * bar_j;
        if (H) {
          WL[v] += H[(int64_t)v * nn + i];
          WR[v] += H[(int64_t)v * nn + j];
        }
      }
      double F[2 + 3 + OM_MAXSP];
      if (ns_model) {
        /* HLLC with each side's own node gamma, minus the diffusive flux */
        om_hllc(nd, nsp, A[i], A[j], WL, WR, Sij, F);
        double pi[3 + 1 + OM_MAXSP], pj[3 + 1 + OM_MAXSP], ai[3 + 2 * OM_MAXSP], aj[3 + 2 * OM_MAXSP];
        double gi[(3 + 1 + OM_MAXSP) * 3], gj[(3 + 1 + OM_MAXSP) * 3], Fv[2 + 3 + OM_MAXSP];
        for (int q = 0; q < np; q++) {
          pi[q] = P[(int64_t)q * nn + i];
          pj[q] = P[(int64_t)q * nn + j];
          for (int d = 0; d < nd; d++) {
            gi[q * nd + d] = GP[((int64_t)q * nd + d) * nn + i];
            gj[q * nd + d] = GP[((int64_t)q * nd + d) * nn + j];
          }
        }
        for (int q = 0; q < na; q++) {
          ai[q] = A[(int64_t)q * nn + i];
          aj[q] = A[(int64_t)q * nn + j];
        }
        double hoop = 0.0;
        if (m->axi) {
          /* u_r / r at the edge midpoint; on an edge along the axis (u_r = 0
           * at both ends) its limit, the mean of the ends' d u_r / d r */
          const double rbar = 0.5 * (X[ab[0] * nd + 1] + X[ab[1] * nd + 1]);
          hoop = rbar > 0.0 ? 0.5 * (pi[1] + pj[1]) / rbar : 0.5 * (gi[1 * nd + 1] + gj[1 * nd + 1]);
        }
        viscous_flux_div(nd, nsp, pi, pj, U[i], U[j], ai, aj, gi, gj, Sij, hoop, Fv);
        for (int v = 0; v < nvar; v++) F[v] -= Fv[v];
      } else if (ph->flux == 0) {
        om_hllc(nd, nsp, ph->gamma, ph->gamma, WL, WR, Sij, F);
      } else {
        om_roe(nd, nsp, ph->gamma, ph->entropy_fix, WL, WR, Sij, F);
      }
      if (m->axi)
        for (int v = 0; v < nvar; v++) F[v] *= m->Rf[c * m->ne + e]; /* revolved face, over 2 pi */
      for (int v = 0; v < nvar; v++) {
        r[(int64_t)v * nn + i] += absmode ? fabs(F[v]) : F[v];
        r[(int64_t)v * nn + j] -= absmode ? -fabs(F[v]) : F[v];
      }
    }
  }
  if (ph->closure == 2) {
    /* boundary closure, second option (2D): the flux through each half of a
     * boundary edge is interpolated, 0.75 F(U_i) + 0.25 F(U_j) */
    double Wa[2 + 3 + OM_MAXSP + 1], Wb[2 + 3 + OM_MAXSP + 1];
    double Fa[2 + 3 + OM_MAXSP], Fb[2 + 3 + OM_MAXSP];
    for (int64_t e = 0; e < m->nbe; e++) {
      const int64_t a = m->be[2 * e], b = m->be[2 * e + 1];
      for (int v = 0; v < nr; v++) {
        Wa[v] = W[(int64_t)v * nn + a];
        Wb[v] = W[(int64_t)v * nn + b];
      }
      om_euler_flux(nd, nsp, Wa, m->beS + 2 * e, Fa);
      om_euler_flux(nd, nsp, Wb, m->beS + 2 * e, Fb);
      for (int v = 0; v < nvar; v++) {
        const double fa = 0.75 * Fa[v] + 0.25 * Fb[v], fb = 0.75 * Fb[v] + 0.25 * Fa[v];
        r[(int64_t)v * nn + a] += absmode ? fabs(fa) : fa;
        r[(int64_t)v * nn + b] += absmode ? fabs(fb) : fb;
      }
    }
  } else if (ph->closure) {
    /* boundary closure, first option: the flux through the boundary part of
     * the dual surface is the node flux F(U_i) . S_i^b */
    double Wi[2 + 3 + OM_MAXSP + 1], F[2 + 3 + OM_MAXSP];
    for (int64_t i = 0; i < nn; i++) {
      if (!m->bnd[i]) continue;
      for (int v = 0; v < nr; v++) Wi[v] = W[(int64_t)v * nn + i];
      om_euler_flux(nd, nsp, Wi, m->axi ? m->Sbr + i * nd : m->Sb + i * nd, F);
      for (int v = 0; v < nvar; v++) r[(int64_t)v * nn + i] += absmode ? fabs(F[v]) : F[v];
    }
  }
  if (m->axi) {
    /* geometric source of the radial momentum (Sec. "Geometric source
     * terms"): + p over the plane dual area, i.e. - p_i A_i in the residual */
    for (int64_t i = 0; i < nn; i++) {
      const double src = W[(int64_t)nvar * nn + i] * m->Vn[i];
      r[(int64_t)2 * nn + i] += absmode ? fabs(src) : -src;
    }
    if (ns_model) {
      /* its diffusive part, eq. (ns_cyl_source_terms): - 2 eta u_r/r
       * - lambda (u_r/r + d u_r/d r + d u_x/d x) with the second viscosity
       * lambda = -2/3 eta (Stokes), i.e. minus the hoop stress tau_theta_theta;
       * at a node on the axis u_r/r takes its limit d u_r/d r */
      for (int64_t i = 0; i < nn; i++) {
        const double eta = A[(int64_t)1 * nn + i], ur = P[(int64_t)1 * nn + i], rr = m->Rn[i];
        const double durdr = GP[((int64_t)1 * nd + 1) * nn + i], duxdx = GP[((int64_t)0 * nd + 0) * nn + i];
        const double hoop = rr > 0.0 ? ur / rr : durdr;
        const double tth = 2.0 * eta * hoop - 2.0 / 3.0 * eta * (hoop + durdr + duxdx);
        const double src = -tth * m->Vn[i];
        r[(int64_t)2 * nn + i] += absmode ? fabs(src) : -src;
      }
    }
  }
  free(W);
  free(G);
  free(P);
  free(GP);
  free(A);
  free(H);
  return 0;
}

/* Limited Lax-Wendroff convective flux plus central diffusive flux for every
 * charged species, per cell-edge (Sec. "Limited Lax-Wendroff scheme"). */
/* Bernoulli function B(x) = x / (e^x - 1), B(0) = 1 */
static double bernoulli(double x) { return x == 0.0 ? 1.0 : x / expm1(x); }

/* face gradient (grad u_i + grad u_j) / 2 of one species, into a static
 * buffer of nd values */
static const double *gbar_of(int nd, const double *g, int64_t nn, int64_t i, int64_t j) {
  static double gb[3];
  for (int d = 0; d < nd; d++) gb[d] = 0.5 * (g[(int64_t)d * nn + i] + g[(int64_t)d * nn + j]);
  return gb;
}

/* Scharfetter-Gummel flux through the cell-edge vector S of edge i -> j
 * (dx = x_j - x_i, h = |dx|), face drift V, diffusion D, face gradient gbar.
 * S is split into S_par = (S . dx / h^2) dx along the edge and
 * S_perp = S - S_par.  Along the edge the flux of the 1D steady
 * advection-diffusion solution between u_i and u_j:
 *   F . S_par = V . S_par (u_j - e^a u_i) / (1 - e^a),  a = h V . dx/h / D,
 * written with the Bernoulli function as (S . dx / h^2) D (B(-a) u_i - B(a) u_j)
 * (the same function, without the cancellation at a -> 0); D = 0 gives its
 * limit, upwinding.  Across the edge the central flux
 *   F . S_perp = V (u_i + u_j)/2 . S_perp - D gbar . S_perp. */
double om_sg_flux(int nd, double ui, double uj, const double *V, const double *S, const double *dx,
                  double D, const double *gbar) {
  double h2 = 0.0, sdx = 0.0, vdx = 0.0, vS = 0.0, gS = 0.0, gdx = 0.0;
  for (int d = 0; d < nd; d++) {
    h2 += dx[d] * dx[d];
    sdx += S[d] * dx[d];
    vdx += V[d] * dx[d];
    vS += V[d] * S[d];
    gS += gbar[d] * S[d];
    gdx += gbar[d] * dx[d];
  }
  const double c = sdx / h2;  /* S_par = c dx */
  double Fpar;
  if (D > 0.0) {
    const double a = vdx / D;
    Fpar = c * D * (bernoulli(-a) * ui - bernoulli(a) * uj);
  } else {
    Fpar = c * vdx * (vdx >= 0.0 ? ui : uj);
  }
  const double vperp = vS - c * vdx, gperp = gS - c * gdx;
  return Fpar + 0.5 * (ui + uj) * vperp - D * gperp;
}

static double sg_flux(int nd, double ui, double uj, const double *V, const double *S, const double *dx,
                      double D, const double *gbar) {
  return om_sg_flux(nd, ui, uj, V, S, dx, D, gbar);
}

static int residual_dd(const om_mesh *m, const om_phys *ph, const double *U, const double *E,
                       double dt, double *r, int absmode) {
  int nd = m->nd, nv = m->nv, ns = ph->nspecies;
  int64_t nn = m->nn;
  double *G = malloc(sizeof(double) * ns * nd * nn);
  if (!G) return -3;
  om_gradient(m, ns, U, G);
  memset(r, 0, sizeof(double) * ns * nn);
  for (int64_t c = 0; c < m->nc; c++) {
    const double *X = m->X + c * nv * nd;
    for (int e = 0; e < m->ne; e++) {
      const int *ab = edge_of(m, e);
      int64_t i = m->cell[c * nv + ab[0]], j = m->cell[c * nv + ab[1]];
      double Sij[3], dx[3];
      edge_normal(m, c, ab[0], ab[1], Sij);
      for (int d = 0; d < nd; d++) dx[d] = X[ab[1] * nd + d] - X[ab[0] * nd + d];
      for (int s = 0; s < ns; s++) {
        const double *u = U + (int64_t)s * nn;
        const double *g = G + (int64_t)s * nd * nn;
        double zm = ph->z[s] * ph->mu[s];
        double Vij[3], v = 0.0, gV = 0.0, gS = 0.0;
        for (int d = 0; d < nd; d++) {
          Vij[d] = 0.5 * (zm * E[(int64_t)d * nn + i] + zm * E[(int64_t)d * nn + j]);
          v += Vij[d] * Sij[d];
        }
        for (int d = 0; d < nd; d++) {
          double gbar = 0.5 * (g[(int64_t)d * nn + i] + g[(int64_t)d * nn + j]);
          gV += gbar * Vij[d];
          gS += gbar * Sij[d];
        }
        if (ph->flux == 2) {
          /* Scharfetter-Gummel (Sec. "Scharfetter Gummel scheme"): S_ij =
           * S_par + S_perp along / across the edge; exponential fitting
           * along it, central across it */
          double F = sg_flux(nd, u[i], u[j], Vij, Sij, dx, ph->D[s], gbar_of(nd, g, nn, i, j));
          if (m->axi) F *= m->Rf[c * m->ne + e];
          r[(int64_t)s * nn + i] += absmode ? fabs(F) : F;
          r[(int64_t)s * nn + j] -= absmode ? -fabs(F) : F;
          continue;
        }
        /* upwind node w and downwind node m of the edge, virtual node k
         * upwind of w: u_w - u_k = grad u_w . (2 w->m) - (u_m - u_w) */
        int64_t w = v >= 0.0 ? i : j, mm = v >= 0.0 ? j : i;
        double sdir = v >= 0.0 ? 1.0 : -1.0;
        double b = u[mm] - u[w];
        double gw = 0.0;
        for (int d = 0; d < nd; d++) gw += g[(int64_t)d * nn + w] * sdir * dx[d];
        double a = 2.0 * gw - b;
        double psi = om_psi_limiter(ph->limiter, ph->beta, a, b);
        double uf = u[w] + (0.5 * b - 0.5 * dt * gV) * psi;
        double F = uf * v - ph->D[s] * gS;
        if (m->axi) F *= m->Rf[c * m->ne + e]; /* flux through the revolved face, over 2 pi */
        r[(int64_t)s * nn + i] += absmode ? fabs(F) : F;
        r[(int64_t)s * nn + j] -= absmode ? -fabs(F) : F;
      }
    }
  }
  if (ph->closure == 2) {
    /* second option (2D): 0.75 F_i + 0.25 F_j on each half boundary edge,
     * F_k = u_k V_k . S - D grad u_k . S */
    for (int64_t e = 0; e < m->nbe; e++) {
      const int64_t ab[2] = {m->be[2 * e], m->be[2 * e + 1]};
      const double *S = m->beS + 2 * e;
      for (int s = 0; s < ns; s++) {
        double F[2];
        for (int q = 0; q < 2; q++) {
          const int64_t i = ab[q];
          double zm = ph->z[s] * ph->mu[s], vb = 0.0, gb = 0.0;
          for (int d = 0; d < nd; d++) {
            vb += zm * E[(int64_t)d * nn + i] * S[d];
            gb += G[((int64_t)s * nd + d) * nn + i] * S[d];
          }
          F[q] = U[(int64_t)s * nn + i] * vb - ph->D[s] * gb;
        }
        const double fa = 0.75 * F[0] + 0.25 * F[1], fb = 0.75 * F[1] + 0.25 * F[0];
        r[(int64_t)s * nn + ab[0]] += absmode ? fabs(fa) : fa;
        r[(int64_t)s * nn + ab[1]] += absmode ? fabs(fb) : fb;
      }
    }
  } else if (ph->closure) {
    /* supersonic-type boundary: F = F_C + F_D with node values */
    for (int64_t i = 0; i < nn; i++) {
      if (!m->bnd[i]) continue;
      const double *Sb = m->axi ? m->Sbr + i * nd : m->Sb + i * nd;
      for (int s = 0; s < ns; s++) {
        double zm = ph->z[s] * ph->mu[s], vb = 0.0, gb = 0.0;
        for (int d = 0; d < nd; d++) {
          vb += zm * E[(int64_t)d * nn + i] * Sb[d];
          gb += G[((int64_t)s * nd + d) * nn + i] * Sb[d];
        }
        double F = U[(int64_t)s * nn + i] * vb - ph->D[s] * gb;
        r[(int64_t)s * nn + i] += absmode ? fabs(F) : F;
      }
    }
  }
  free(G);
  return 0;
}

static int residual_any(const om_mesh *m, const om_phys *ph, const double *U, const double *E,
                        double dt, double *r, int absmode) {
  if (!m || !ph || !U || !r) return -1;
  /* the interpolated closure is given for planar 2D meshes */
  if (ph->closure == 2 && (m->nd != 2 || m->axi || ph->model == 2)) return -1;
  if (ph->nspecies < 0 || ph->nspecies > OM_MAXSP) return -1;
  /* the predictor: constant-gamma gas on plane meshes, one-stage time step */
  if (ph->predictor && (ph->model != 0 || m->axi || ph->rk != 1)) return -1;
  if (ph->model == 0 || ph->model == 2) {
    return residual_gas(m, ph, U, dt, r, absmode);
  }
  if (ph->model == 1) {
    if (!E || ph->nspecies < 1) return -1;
    if (ph->flux != 0 && ph->flux != 2) return -1; /* 0 limited Lax-Wendroff, 2 Scharfetter-Gummel */
    return residual_dd(m, ph, U, E, dt, r, absmode);
  }
  return -1;
}

int om_residual(const om_mesh *m, const om_phys *ph, const double *U, const double *E,
                double dt, double *r) {
  return residual_any(m, ph, U, E, dt, r, 0);
}

/* Flux magnitude per node: sum over the node's cell-edges (and closure) of
 * |F . S|, per variable -- the scale against which residual differences are
 * measured (a residual is a difference of such fluxes). */
int om_flux_scale(const om_mesh *m, const om_phys *ph, const double *U, const double *E,
                  double dt, double *out) {
  return residual_any(m, ph, U, E, dt, out, 1);
}

/* ------------------------------------------------------------------ */
/* time step                                                            */
/* ------------------------------------------------------------------ */

/* cell size: inscribed-sphere diameter 2 n_d V_tau / sum_k |S_k| */
static double cell_size(const om_mesh *m, int64_t c) {
  double sum = 0.0;
  for (int k = 0; k < m->nv; k++) {
    double s2 = 0.0;
    for (int d = 0; d < m->nd; d++) {
      double s = m->S[(c * m->nv + k) * m->nd + d];
      s2 += s * s;
    }
    sum += sqrt(s2);
  }
  return 2.0 * m->nd * m->Vc[c] / sum;
}

int om_timestep(const om_mesh *m, const om_phys *ph, const double *U, const double *E,
                double *dt_out) {
  int nd = m->nd, nv = m->nv;
  int64_t nn = m->nn;
  double dt = INFINITY;
  for (int64_t c = 0; c < m->nc; c++) {
    double dx = cell_size(m, c);
    if (ph->model == 2) {
      /* convective limit with the mixture sound speed, viscous limit with the
       * largest of nu, thermal diffusivity and species diffusivities */
      double lam = 0.0, dmax = 0.0, Ui[2 + 3 + OM_MAXSP], out[5 + 2 * OM_MAXSP];
      int nvar = 2 + nd + ph->nspecies;
      for (int k = 0; k < nv; k++) {
        int64_t i = m->cell[c * nv + k];
        for (int v = 0; v < nvar; v++) Ui[v] = U[(int64_t)v * nn + i];
        double rho = Ui[0], uu = 0.0;
        if (!(rho > 0.0)) return -5;
        for (int d = 0; d < nd; d++) uu += (Ui[1 + d] / rho) * (Ui[1 + d] / rho);
        om_ns_node(nd, ph, Ui, out);
        if (!(out[0] > 0.0)) return -5;
        double l = sqrt(uu) + sqrt(out[2] * out[1] / rho);
        if (l > lam) lam = l;
        /* thermal diffusivity lambda / (rho c_p) = mu / (rho Pr) */
        double nu = out[3] / rho, kap = out[3] / (rho * ph->Pr);
        double dm = nu > kap ? nu : kap;
        for (int s = 0; s < ph->nspecies; s++)
          if (out[5 + s] > dm) dm = out[5 + s];
        if (dm > dmax) dmax = dm;
      }
      double t = ph->cfl * dx / lam;
      if (t < dt) dt = t;
      if (dmax > 0.0) {
        t = ph->fourier * dx * dx / dmax;
        if (t < dt) dt = t;
      }
    } else if (ph->model == 0) {
      double lam = 0.0;
      for (int k = 0; k < nv; k++) {
        int64_t i = m->cell[c * nv + k];
        double rho = U[i], uu = 0.0;
        for (int d = 0; d < nd; d++) {
          double ud = U[(int64_t)(1 + d) * nn + i] / rho;
          uu += ud * ud;
        }
        double p = pressure_of(nd, U, nn, i, ph->gamma);
        if (!(rho > 0.0) || !(p > 0.0)) return -5; /* non-physical state: no time step */
        double l = sqrt(uu) + sqrt(ph->gamma * p / rho);
        if (l > lam) lam = l;
      }
      double t = ph->cfl * dx / lam;
      if (t < dt) dt = t;
    } else {
      for (int s = 0; s < ph->nspecies; s++) {
        double vmax = 0.0;
        for (int k = 0; k < nv; k++) {
          int64_t i = m->cell[c * nv + k];
          double v2 = 0.0;
          for (int d = 0; d < nd; d++) {
            double vd = ph->z[s] * ph->mu[s] * E[(int64_t)d * nn + i];
            v2 += vd * vd;
          }
          if (sqrt(v2) > vmax) vmax = sqrt(v2);
        }
        if (vmax > 0.0) {
          double t = ph->cfl * dx / vmax;
          if (t < dt) dt = t;
        }
        if (ph->D[s] > 0.0) {
          double t = ph->fourier * dx * dx / ph->D[s];
          if (t < dt) dt = t;
        }
      }
      /* dielectric limit A_D eps0 / sum_s |q_s n_s mu_s|, with the
       * conductivity of the cell taken at its most conductive node */
      if (ph->diel > 0.0) {
        double smax = 0.0;
        for (int k = 0; k < nv; k++) {
          int64_t i = m->cell[c * nv + k];
          double sig = 0.0;
          for (int s = 0; s < ph->nspecies; s++)
            sig += fabs(OM_ECHARGE * ph->z[s] * U[(int64_t)s * nn + i] * ph->mu[s]);
          if (sig > smax) smax = sig;
        }
        if (smax > 0.0) {
          double t = ph->diel * OM_EPS0 / smax;
          if (t < dt) dt = t;
        }
      }
    }
  }
  *dt_out = dt;
  if (!(dt > 0.0) || !isfinite(dt)) return -5;
  return 0;
}

/* ------------------------------------------------------------------ */
/* Runge-Kutta                                                          */
/* ------------------------------------------------------------------ */

/* alpha_2..alpha_4 of the low-storage table, beta_K = 1 */
static const double RK_ALPHA[5][5] = {
    {0, 0, 0, 0, 0},
    {0, 0, 0, 0, 0},
    {0, 0, 1.0 / 2.0, 0, 0},
    {0, 0, 1.0 / 3.0, 1.0 / 2.0, 0},
    {0, 0, 1.0 / 4.0, 1.0 / 3.0, 1.0 / 2.0},
};

static int state_ok(const om_mesh *m, const om_phys *ph, const double *U) {
  int nvar = om_nvar(m->nd, ph);
  int64_t nn = m->nn;
  for (int64_t q = 0; q < (int64_t)nvar * nn; q++)
    if (!isfinite(U[q])) return 0;
  if (ph->model == 0)
    for (int64_t i = 0; i < nn; i++) {
      if (!(U[i] > 0.0)) return 0;
      if (!(pressure_of(m->nd, U, nn, i, ph->gamma) > 0.0)) return 0;
    }
  if (ph->model == 2) {
    double Ui[2 + 3 + OM_MAXSP], out[5 + 2 * OM_MAXSP];
    for (int64_t i = 0; i < nn; i++) {
      for (int v = 0; v < nvar; v++) Ui[v] = U[(int64_t)v * nn + i];
      if (!(Ui[0] > 0.0)) return 0;
      om_ns_node(m->nd, ph, Ui, out);
      if (!(out[0] > 0.0) || !isfinite(out[0])) return 0;
    }
  }
  return 1;
}

int om_step(const om_mesh *m, const om_phys *ph, double *U, const double *E, int nsteps,
            double t_end, double *t, double *dt_last, int *steps_done) {
  if (ph->rk < 1 || ph->rk > 4) return -1;
  int nvar = om_nvar(m->nd, ph);
  int64_t nn = m->nn, tot = (int64_t)nvar * nn;
  const double *vol = m->axi ? m->Vp : m->Vn; /* the node volume the update divides by */
  double *U0 = malloc(sizeof(double) * tot), *Uk = malloc(sizeof(double) * tot);
  double *r = malloc(sizeof(double) * tot);
  if (!U0 || !Uk || !r) { free(U0); free(Uk); free(r); return -3; }
  int st = 0, done = 0;
  for (int n = 0; n < nsteps; n++) {
    if (t_end > 0.0 && *t >= t_end) break;
    double dt;
    st = om_timestep(m, ph, U, E, &dt);
    if (st) break;
    if (t_end > 0.0 && *t + dt > t_end) dt = t_end - *t;
    memcpy(U0, U, sizeof(double) * tot);
    memcpy(Uk, U, sizeof(double) * tot);
    for (int k = 2; k <= ph->rk + 1; k++) {
      /* k <= K: intermediate stage U(k) = U^n - alpha_k dt r(U(k-1))/V;
       * k == K+1: final update U^{n+1} = U^n - dt r(U(K))/V */
      double a = k <= ph->rk ? RK_ALPHA[ph->rk][k] : 1.0;
      st = om_residual(m, ph, Uk, E, dt, r);
      if (st) break;
      for (int v = 0; v < nvar; v++)
        for (int64_t i = 0; i < nn; i++)
          Uk[(int64_t)v * nn + i] = U0[(int64_t)v * nn + i] - a * dt * r[(int64_t)v * nn + i] / vol[i];
      /* axisymmetric gas: the radial velocity is set to zero on the axis
       * after the geometric source terms */
      if (m->axi && (ph->model == 0 || ph->model == 2))
        for (int64_t i = 0; i < nn; i++)
          if (m->Rn[i] == 0.0) Uk[(int64_t)2 * nn + i] = 0.0;
    }
    if (st) break;
    if (!state_ok(m, ph, Uk)) { st = -5; break; }
    memcpy(U, Uk, sizeof(double) * tot);
    *t += dt;
    *dt_last = dt;
    done++;
  }
  if (steps_done) *steps_done = done;
  free(U0); free(Uk); free(r);
  return st;
}

/* ------------------------------------------------------------------ */
/* conservation diagnostic                                              */
/* ------------------------------------------------------------------ */

/* sum_i V_i U_i per variable with Neumaier-compensated summation, and the
 * normalisation sum_i V_i |U_i| */
void om_sums(const om_mesh *m, int nvar, const double *U, double *sums, double *abssums) {
  for (int v = 0; v < nvar; v++) {
    double s = 0.0, comp = 0.0, a = 0.0, acomp = 0.0;
    for (int64_t i = 0; i < m->nn; i++) {
      double x = (m->axi ? m->Vp[i] : m->Vn[i]) * U[(int64_t)v * m->nn + i];
      double t = s + x;
      if (fabs(s) >= fabs(x)) comp += (s - t) + x; else comp += (x - t) + s;
      s = t;
      double ax = fabs(x), ta = a + ax;
      if (a >= ax) acomp += (a - ta) + ax; else acomp += (ax - ta) + a;
      a = ta;
    }
    sums[v] = s + comp;
    if (abssums) abssums[v] = a + acomp;
  }
}

/* ------------------------------------------------------------------ */
/* Poisson operator (Sec. "Integrating the Poisson equation")           */
/* ------------------------------------------------------------------ */

/* Matrix of -lap phi integrated over the nodal volumes, eq.
 * (poisson_discretization_cartesian) with its sign turned as in the
 * remark on the implementation: row i, column k receives
 * S_i . S_k / (V_tau n_d^2) from every cell tau holding both nodes (the
 * paper's coefficient a_ik with the opposite sign).  Written as coordinate
 * triplets, nv * nv per cell in cell order; equal (i, k) pairs are to be
 * summed by the caller. */
void om_poisson_coo(const om_mesh *m, int64_t *I, int64_t *K, double *val) {
  const int nd = m->nd, nv = m->nv;
  int64_t q = 0;
  if (m->axi) {
    /* axisymmetric (Sec. "Axisymmetric configuration"): the planar cell
     * gradient -1/(A n_d) sum_k phi_k n_k dotted with int r n dl over node
     * i's dual boundary inside the triangle, (1/24)[(4 r_c + 2 r_i + r_j +
     * r_k) n_i - (2 r_c + r_i + r_j) n_j - (2 r_c + r_i + r_k) n_k] with r_c
     * the centroid radius (the 2 pi cancels against the revolved volumes);
     * the matrix is not symmetric */
    for (int64_t c = 0; c < m->nc; c++) {
      const double *S = m->S + c * 6, *X = m->X + c * 6;
      const double r[3] = {X[1], X[3], X[5]};
      const double rc = (r[0] + r[1] + r[2]) / 3.0;
      for (int a = 0; a < 3; a++) {
        const int j = (a + 1) % 3, k = (a + 2) % 3;
        double wv[2];
        for (int d = 0; d < 2; d++)
          wv[d] = ((4 * rc + 2 * r[a] + r[j] + r[k]) * S[a * 2 + d] - (2 * rc + r[a] + r[j]) * S[j * 2 + d] -
                   (2 * rc + r[a] + r[k]) * S[k * 2 + d]) / 24.0;
        for (int b = 0; b < 3; b++) {
          I[q] = m->cell[c * 3 + a];
          K[q] = m->cell[c * 3 + b];
          val[q] = (S[b * 2] * wv[0] + S[b * 2 + 1] * wv[1]) / (2.0 * m->Vc[c]);
          q++;
        }
      }
    }
    return;
  }
  for (int64_t c = 0; c < m->nc; c++) {
    const double *S = m->S + c * nv * nd;
    const double w = 1.0 / (m->Vc[c] * nd * nd);
    for (int a = 0; a < nv; a++)
      for (int b = 0; b < nv; b++) {
        double dot = 0.0;
        for (int d = 0; d < nd; d++) dot += S[a * nd + d] * S[b * nd + d];
        I[q] = m->cell[c * nv + a];
        K[q] = m->cell[c * nv + b];
        val[q] = dot * w;
        q++;
      }
  }
}

/* |S_i^b| per node: length (2D) or area (3D) of the boundary normal of a
 * node, 0 away from the boundary; weights the Neumann data E_n (Sec.
 * "Neumann boundary conditions"). */
void om_boundary_measure(const om_mesh *m, double *out) {
  const double *Sb = m->axi ? m->Sbr : m->Sb; /* revolved boundary surface over 2 pi */
  for (int64_t i = 0; i < m->nn; i++) {
    double s = 0.0;
    for (int d = 0; d < m->nd; d++) s += Sb[i * m->nd + d] * Sb[i * m->nd + d];
    out[i] = m->bnd[i] ? sqrt(s) : 0.0;
  }
}
