// Poisson solve for the electric potential (declarations in include/vcx.h).
//
// Sec. "Integrating the Poisson equation": integrating -lap phi = rho/eps0
// over the nodal volume V_i, with the cell gradient constant in each cell,
// gives row i of a sparse symmetric system whose coefficient for node k is
// the sum over the cells holding i and k of S_i . S_k / (V_tau n_d^2).  Since
// S_k = -n_d V_tau grad(lambda_k) (lambda: barycentric coordinates), this is
// V_tau grad(lambda_i) . grad(lambda_k), the form assembled here.
// Sec. "Boundary conditions": Dirichlet rows carry the imposed value,
// Neumann data enter the right-hand side as -E_n |S_i^b|, and a boundary
// node with nothing imposed has a zero normal field.
//
// Device layout: CSR rows in the internal node order (space-filling curve),
// FP64 values.  The solve is preconditioned conjugate gradients with a
// two-level additive preconditioner: Jacobi plus a coarse space of
// aggregates (runs of consecutive curve-ordered nodes, piecewise-constant
// prolongation), whose small dense operator is inverted on the host; three
// kernels per iteration (coarse correction, search direction and product,
// update).  The operator of an axisymmetric mesh (Sec. "Axisymmetric
// configuration") is not symmetric: it is solved by BiCGStab with Jacobi
// preconditioning, three kernels per iteration, with the same fixed-order
// reductions.  Every dot product is reduced in a fixed order:
// each block writes one partial, and every block of the next kernel sums all
// partials in the same order, so all blocks take the same scalars and the
// iterates are bitwise reproducible.  Convergence is decided on the device;
// the host launches iterations in chunks and reads one small record per
// chunk.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "vcx.h"
#include "vcx_batch.h"

namespace {

using vcx::HostMesh;

constexpr int kThreads = 256;

vcx_status err(vcx_status s, const std::string& m) { return vcx::set_error(s, m.c_str()); }

#define PS_HIP(expr)                                                                    \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess) return err(VCX_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

struct PoissonDev {
  int n, nd, nnz, singular;
  int agg;              // nodes per aggregate: 64, 128 or a multiple of kThreads
  int nc;               // aggregates
  int rpb;              // rows per block, max(agg, kThreads): whole aggregates
  int nb;               // blocks of the solver kernels (one partial sum each)
  const int* rp;        // [n+1]
  const int* col;       // [nnz]
  const double* val;    // [nnz] matrix of -lap phi over the nodal volumes
  const double* gval;   // [nd][nnz] E = -grad phi: E_d,i = sum_k gval_d,ik phi_k
  const double* dinv;   // [n] 1 / L_ii on free nodes, 0 on Dirichlet nodes
  const double* vn;     // [n] nodal volumes
  const double* sbm;    // [n] |S_i^b| on boundary nodes, 0 elsewhere
  const double* ainv;   // [nc][nc] inverse of the coarse operator R L R^T
  const int32_t* perm;  // [n] internal -> caller
};

// Partial-sum rows (one double per block each); rows ending in 0/1 are
// double-buffered by iteration parity.
enum {
  P_DRR0 = 0, P_DRR1,  // sum D^-1 r^2 (fine part of r.z)
  P_RR0, P_RR1,        // r.r
  P_PQ,                // p.q
  P_GC,                // g_b c_b (coarse part of r.z)
  P_B, P_V, P_BB, P_VX, P_RRI,
  P_RHO0, P_RHO1,      // BiCGStab: r^.r
  P_RV, P_TS, P_TT,    // BiCGStab: r^.v, t.s, t.t
  P_NROWS
};

struct CgCtl {
  int done;       // iterations stop (converged, or a fault below)
  int iters;      // iterations taken when done
  int last;       // last iteration started
  int fault;      // 0 none, 1 non-finite residual, 2 BiCGStab breakdown above the tolerance
  double rr;      // squared residual norm of the last iterate
  double ref2;    // squared norm the tolerance is relative to
  double rz[2];   // r.z of the iterates, by parity (BiCGStab: r^.r)
  double alpha, omega;  // BiCGStab step lengths of the last iteration
};

struct CgVec {
  double *x, *r, *p0, *p1, *q, *b;
  double *rh, *v0, *v1, *t;  // BiCGStab: shadow residual, A p^ (by parity), A s^
  double* g;     // [nc] restriction R r (sum of r over each aggregate's free nodes)
  double* c;     // [nc] coarse correction A_c^-1 g
  double* part;  // [P_NROWS][nc]
  CgCtl* ctl;
};

// Sum over a wavefront: a fixed butterfly of shuffles (every lane ends with
// the same value).
__device__ inline double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Sum over the block: wavefront sums, then the wavefronts in order.  The
// same arithmetic in every block and every thread.
__device__ double block_sum(double v) {
  __shared__ double wsum[kThreads / 64];
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = v;
  __syncthreads();
  double out = wsum[0];
  for (int w = 1; w < kThreads / 64; ++w) out += wsum[w];
  __syncthreads();
  return out;
}

// Sums of N rows of block partials at once (the loads of all rows in
// flight together), each in the order of sum_partials.
template <int N>
__device__ void sum_partials_n(const double* const (&rows)[N], int nb, double (&out)[N]) {
  __shared__ double wsum[N][kThreads / 64];
  double v[N];
#pragma unroll
  for (int q = 0; q < N; ++q) v[q] = 0.0;
  for (int k = threadIdx.x; k < nb; k += kThreads)
#pragma unroll
    for (int q = 0; q < N; ++q) v[q] += rows[q][k];
#pragma unroll
  for (int q = 0; q < N; ++q) {
    v[q] = wave_sum(v[q]);
    if ((threadIdx.x & 63) == 0) wsum[q][threadIdx.x >> 6] = v[q];
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < N; ++q) {
    out[q] = wsum[q][0];
    for (int w = 1; w < kThreads / 64; ++w) out[q] += wsum[q][w];
  }
  __syncthreads();
}

// Sum of one row of block partials in a fixed order (same in every block).
__device__ double sum_partials(const double* row, int nb) {
  double s = 0.0;
  for (int k = threadIdx.x; k < nb; k += kThreads) s += row[k];
  return block_sum(s);
}

// The stop flag as one value for the whole block (it may be written by
// block 0 of the same launch while other blocks read it).
__device__ bool block_done(const CgCtl* ctl) {
  __shared__ int flag;
  if (threadIdx.x == 0) flag = __hip_atomic_load(&ctl->done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __syncthreads();
  const bool d = flag != 0;
  __syncthreads();
  return d;
}

__device__ void put_partial(double* row, double v) {
  const double s = block_sum(v);
  if (threadIdx.x == 0) row[blockIdx.x] = s;
}

// Rows of this block: [i0, i1), whole aggregates
__device__ inline void agg_rows(const PoissonDev& P, int& i0, int& i1) {
  i0 = blockIdx.x * P.rpb;
  i1 = min(P.n, i0 + P.rpb);
}

// Restriction g = R r of this block's aggregates from each thread's sum v
// of r over its rows: one block sum (an aggregate of kThreads rows or more),
// or the sum over the agg consecutive threads of each aggregate (each
// thread then holds one row), from the wavefront sums in order.
__device__ void put_restriction(const PoissonDev& P, double* g, double v) {
  __shared__ double wsum[kThreads / 64];
  constexpr int NW = kThreads / 64;
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = v;
  __syncthreads();
  // wavefronts per aggregate: 1 (64 nodes), 2 (128) or all of the block
  const int wpa = min(P.agg, kThreads) / 64;
  const int t = threadIdx.x;
  if (t < NW / wpa) {
    double s = wsum[t * wpa];
    for (int w = 1; w < wpa; ++w) s += wsum[t * wpa + w];
    const int a = P.agg >= kThreads ? (int)blockIdx.x : (int)(blockIdx.x * (kThreads / P.agg) + t);
    if (a < P.nc) g[a] = s;
  }
  __syncthreads();
}

// Preconditioned residual of node j: z = D^-1 r + c_(aggregate of j) on free
// nodes (two-level additive: Jacobi plus the aggregation coarse space), 0 on
// Dirichlet nodes.
__device__ inline double precond(const PoissonDev& P, const CgVec& X, int j) {
  const double dj = P.dinv[j];
  return dj != 0.0 ? dj * X.r[j] + X.c[j / P.agg] : 0.0;
}

// Right-hand side q V - E_n |S^b| on free nodes, the initial iterate (guess
// on free nodes, imposed values on Dirichlet nodes); partial sums of b and V.
__global__ void __launch_bounds__(kThreads) k_cg_init1(PoissonDev P, CgVec X, const double* __restrict__ q,
                                                        const double* __restrict__ phiD,
                                                        const double* __restrict__ En,
                                                        const double* __restrict__ phi0) {
  int i0, i1;
  agg_rows(P, i0, i1);
  double sb = 0.0, sv = 0.0;
  for (int i = i0 + threadIdx.x; i < i1; i += kThreads) {
    const int o = P.perm[i];
    double b = 0.0;
    if (P.dinv[i] != 0.0) {
      b = q[o] * P.vn[i];
      if (En) b -= En[o] * P.sbm[i];
      X.x[i] = phi0 ? phi0[o] : 0.0;
    } else {
      X.x[i] = phiD ? phiD[o] : 0.0;
    }
    X.b[i] = b;
    sb += b;
    sv += P.vn[i];
  }
  put_partial(X.part + P_B * P.nb, sb);
  put_partial(X.part + P_V * P.nb, sv);
}

// Singular systems: the uniform background that makes b sum to zero.
// Initial residual r = b - L x on free rows, p = 0; partial sums of D^-1 r^2,
// r.r and |b - L_fD x_D|^2 (the norm the tolerance refers to), and g = R r.
__global__ void __launch_bounds__(kThreads) k_cg_init2(PoissonDev P, CgVec X) {
  double bmean = 0.0;
  if (P.singular) bmean = sum_partials(X.part + P_B * P.nb, P.nb) / sum_partials(X.part + P_V * P.nb, P.nb);
  int i0, i1;
  agg_rows(P, i0, i1);
  double drr = 0.0, rr = 0.0, bb = 0.0, gs = 0.0;
  for (int i = i0 + threadIdx.x; i < i1; i += kThreads) {
    const double di = P.dinv[i];
    double r = 0.0;
    if (di != 0.0) {
      double b = X.b[i];
      if (P.singular) {
        b -= P.vn[i] * bmean;
        X.b[i] = b;
      }
      double ax = 0.0, ad = 0.0;
      for (int e = P.rp[i]; e < P.rp[i + 1]; ++e) {
        const int k = P.col[e];
        const double t = P.val[e] * X.x[k];
        ax += t;
        if (P.dinv[k] == 0.0) ad += t;
      }
      r = b - ax;
      const double bt = b - ad;
      bb += bt * bt;
    }
    X.r[i] = r;
    X.p0[i] = 0.0;
    X.p1[i] = 0.0;
    drr += di * r * r;
    rr += r * r;
    gs += r;
  }
  put_partial(X.part + P_DRR0 * P.nb, drr);
  put_partial(X.part + P_RR0 * P.nb, rr);
  put_partial(X.part + P_RRI * P.nb, rr);
  put_partial(X.part + P_BB * P.nb, bb);
  put_restriction(P, X.g, gs);
}

// Coarse correction of iterate k: c_a = (A_c^-1 g)_a for this block's
// aggregates, and their coarse part sum g_a c_a of r.z.
__global__ void __launch_bounds__(kThreads) k_cg_c(PoissonDev P, CgVec X) {
  if (block_done(X.ctl)) return;
  const int per = P.rpb / P.agg, a0 = blockIdx.x * per, a1 = min(P.nc, a0 + per);
  if (per == 1) {
    const double* row = P.ainv + (size_t)a0 * P.nc;
    double s = 0.0;
    for (int j = threadIdx.x; j < P.nc; j += kThreads) s += row[j] * X.g[j];
    const double ca = block_sum(s);
    if (threadIdx.x == 0) {
      X.c[a0] = ca;
      X.part[P_GC * P.nb + blockIdx.x] = X.g[a0] * ca;
    }
    return;
  }
  // several aggregates per block (at most one per wavefront): one wavefront
  // each, lanes over the row, a fixed butterfly of shuffles
  __shared__ double cw[kThreads / 64];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, a = a0 + w;
  if (a < a1) {
    const double* row = P.ainv + (size_t)a * P.nc;
    double v = 0.0;
    for (int j = lane; j < P.nc; j += 64) v += row[j] * X.g[j];
    v = wave_sum(v);
    if (lane == 0) {
      X.c[a] = v;
      cw[w] = v;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double gc = 0.0;
    for (int b = a0; b < a1; ++b) gc += X.g[b] * cw[b - a0];
    X.part[P_GC * P.nb + blockIdx.x] = gc;
  }
}

// Iteration k, first half: stop test on the residual of iterate k; else
// r.z, beta = (r.z)_k / (r.z)_(k-1), p_k = z + beta p_(k-1) and q = L p_k
// (rows form z and p_k of their neighbours themselves, in the same
// arithmetic as the neighbour's own row), partial sums of p.q.
__global__ void __launch_bounds__(kThreads) k_cg_a(PoissonDev P, CgVec X, int k, double tol2) {
  if (block_done(X.ctl)) return;
  const int cur = k & 1;
  const double* const rows[5] = {X.part + (P_RR0 + cur) * P.nb, X.part + P_BB * P.nb, X.part + P_RRI * P.nb,
                                  X.part + (P_DRR0 + cur) * P.nb, X.part + P_GC * P.nb};
  double sums[5];
  sum_partials_n<5>(rows, P.nb, sums);
  const double rr = sums[0];
  // relative to |b - L_fD x_D| (the free system's right-hand side), or to
  // the initial residual when that is zero
  const double bb = sums[1];
  const double ref2 = bb > 0.0 ? bb : sums[2];
  const double rz = sums[3] + sums[4];
  // a non-finite residual (e.g. a NaN in q) stops the iteration as a fault
  const bool bad = !isfinite(rr) || !isfinite(ref2) || !isfinite(rz);
  const bool conv = bad || !(rr > tol2 * ref2);  // also stops on rr = 0
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    X.ctl->last = k;
    X.ctl->rr = rr;
    X.ctl->ref2 = ref2;
    X.ctl->rz[cur] = rz;
    if (conv) {
      X.ctl->iters = k;
      if (bad) X.ctl->fault = 1;
      __hip_atomic_store(&X.ctl->done, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
  if (conv) return;
  const double beta = k == 0 ? 0.0 : rz / X.ctl->rz[cur ^ 1];
  const double* po = cur ? X.p1 : X.p0;  // p_(k-1) (zero at k = 0)
  double* pn = cur ? X.p0 : X.p1;        // p_k
  int i0, i1;
  agg_rows(P, i0, i1);
  double pq = 0.0;
  for (int i = i0 + threadIdx.x; i < i1; i += kThreads) {
    double p = 0.0, qv = 0.0;
    if (P.dinv[i] != 0.0) {
      p = precond(P, X, i) + beta * po[i];
      for (int e = P.rp[i]; e < P.rp[i + 1]; ++e) {
        const int j = P.col[e];
        qv += P.val[e] * (precond(P, X, j) + beta * po[j]);
      }
    }
    pn[i] = p;
    X.q[i] = qv;
    pq += p * qv;
  }
  put_partial(X.part + P_PQ * P.nb, pq);
}

// Iteration k, second half: alpha = (r.z)_k / (p.q); x += alpha p,
// r -= alpha q; partial sums of D^-1 r^2 and r.r of iterate k+1 and its
// restriction g = R r.
__global__ void __launch_bounds__(kThreads) k_cg_b(PoissonDev P, CgVec X, int k) {
  if (block_done(X.ctl)) return;
  const int cur = k & 1, nxt = cur ^ 1;
  const double alpha = X.ctl->rz[cur] / sum_partials(X.part + P_PQ * P.nb, P.nb);
  const double* pn = cur ? X.p0 : X.p1;
  int i0, i1;
  agg_rows(P, i0, i1);
  double drr = 0.0, rr = 0.0, gs = 0.0;
  for (int i = i0 + threadIdx.x; i < i1; i += kThreads) {
    const double di = P.dinv[i];
    if (di == 0.0) continue;
    X.x[i] += alpha * pn[i];
    const double r = X.r[i] - alpha * X.q[i];
    X.r[i] = r;
    drr += di * r * r;
    rr += r * r;
    gs += r;
  }
  put_partial(X.part + (P_DRR0 + nxt) * P.nb, drr);
  put_partial(X.part + (P_RR0 + nxt) * P.nb, rr);
  put_restriction(P, X.g, gs);
}

// ---- BiCGStab (non-symmetric operators of axisymmetric meshes), Jacobi
// preconditioned on the right: p^ = D^-1 p, s^ = D^-1 s.

// Initial residual r = b - L x on free rows, shadow residual r^ = r, p = v =
// 0; partial sums of r^.r, r.r and |b - L_fD x_D|^2.
__global__ void __launch_bounds__(kThreads) k_bi_init2(PoissonDev P, CgVec X) {
  double bmean = 0.0;
  if (P.singular) bmean = sum_partials(X.part + P_B * P.nb, P.nb) / sum_partials(X.part + P_V * P.nb, P.nb);
  int i0, i1;
  agg_rows(P, i0, i1);
  double rr = 0.0, bb = 0.0;
  for (int i = i0 + threadIdx.x; i < i1; i += kThreads) {
    double r = 0.0;
    if (P.dinv[i] != 0.0) {
      double b = X.b[i];
      if (P.singular) {
        b -= P.vn[i] * bmean;
        X.b[i] = b;
      }
      double ax = 0.0, ad = 0.0;
      for (int e = P.rp[i]; e < P.rp[i + 1]; ++e) {
        const int k = P.col[e];
        const double t = P.val[e] * X.x[k];
        ax += t;
        if (P.dinv[k] == 0.0) ad += t;
      }
      r = b - ax;
      const double bt = b - ad;
      bb += bt * bt;
    }
    X.r[i] = r;
    X.rh[i] = r;
    X.p0[i] = X.p1[i] = 0.0;
    X.v0[i] = X.v1[i] = 0.0;
    rr += r * r;
  }
  put_partial(X.part + P_RHO0 * P.nb, rr);
  put_partial(X.part + P_RR0 * P.nb, rr);
  put_partial(X.part + P_RRI * P.nb, rr);
  put_partial(X.part + P_BB * P.nb, bb);
}

// Iteration k, part 1: stop test on r_k; beta = (rho_k/rho_(k-1))
// (alpha/omega); p_k = r + beta (p_(k-1) - omega v_(k-1)); v_k = L p^_k
// (neighbours' p^ formed in the same arithmetic as their own rows);
// partial sums of r^.v_k.
__global__ void __launch_bounds__(kThreads) k_bi_a(PoissonDev P, CgVec X, int k, double tol2) {
  if (block_done(X.ctl)) return;
  const int cur = k & 1;
  const double rr = sum_partials(X.part + (P_RR0 + cur) * P.nb, P.nb);
  const double bb = sum_partials(X.part + P_BB * P.nb, P.nb);
  const double ref2 = bb > 0.0 ? bb : sum_partials(X.part + P_RRI * P.nb, P.nb);
  const double rho = sum_partials(X.part + (P_RHO0 + cur) * P.nb, P.nb);
  // converged; or a fault: a non-finite residual, or a breakdown (r^.r = 0,
  // or omega = 0 with r != 0) above the tolerance
  const bool bad = !isfinite(rr) || !isfinite(ref2) || !isfinite(rho);
  const bool ok = !bad && !(rr > tol2 * ref2);
  const bool brk = !bad && !ok && (rho == 0.0 || (k > 0 && X.ctl->omega == 0.0));
  const bool conv = ok || bad || brk;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    X.ctl->last = k;
    X.ctl->rr = rr;
    X.ctl->ref2 = ref2;
    X.ctl->rz[cur] = rho;
    if (conv) {
      X.ctl->iters = k;
      if (bad) X.ctl->fault = 1;
      if (brk) X.ctl->fault = 2;
      __hip_atomic_store(&X.ctl->done, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
  if (conv) return;
  double beta = 0.0, om = 0.0;
  if (k > 0) {
    om = X.ctl->omega;
    beta = (rho / X.ctl->rz[cur ^ 1]) * (X.ctl->alpha / om);
  }
  const double* po = cur ? X.p1 : X.p0;  // p_(k-1)
  const double* vo = cur ? X.v1 : X.v0;  // v_(k-1)
  double* pn = cur ? X.p0 : X.p1;
  double* vn = cur ? X.v0 : X.v1;
  int i0, i1;
  agg_rows(P, i0, i1);
  double rv = 0.0;
  for (int i = i0 + threadIdx.x; i < i1; i += kThreads) {
    double p = 0.0, v = 0.0;
    if (P.dinv[i] != 0.0) {
      p = X.r[i] + beta * (po[i] - om * vo[i]);
      for (int e = P.rp[i]; e < P.rp[i + 1]; ++e) {
        const int j = P.col[e];
        const double pj = X.r[j] + beta * (po[j] - om * vo[j]);
        v += P.val[e] * (P.dinv[j] * pj);
      }
    }
    pn[i] = p;
    vn[i] = v;
    rv += X.rh[i] * v;
  }
  put_partial(X.part + P_RV * P.nb, rv);
}

// Iteration k, part 2: alpha = rho_k / r^.v_k; s = r - alpha v_k;
// t = L s^ (neighbours' s^ formed the same way); partial sums of t.s, t.t.
__global__ void __launch_bounds__(kThreads) k_bi_b(PoissonDev P, CgVec X, int k) {
  if (block_done(X.ctl)) return;
  const int cur = k & 1;
  const double rv = sum_partials(X.part + P_RV * P.nb, P.nb);
  if (!(rv != 0.0) || !isfinite(rv)) {  // breakdown: stop at the current iterate
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      X.ctl->iters = k;
      X.ctl->fault = isfinite(rv) ? 2 : 1;
      __hip_atomic_store(&X.ctl->done, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    return;
  }
  const double alpha = X.ctl->rz[cur] / rv;
  if (blockIdx.x == 0 && threadIdx.x == 0) X.ctl->alpha = alpha;
  const double* vn = cur ? X.v0 : X.v1;
  int i0, i1;
  agg_rows(P, i0, i1);
  double ts = 0.0, tt = 0.0;
  for (int i = i0 + threadIdx.x; i < i1; i += kThreads) {
    double t = 0.0, sv = 0.0;
    if (P.dinv[i] != 0.0) {
      sv = X.r[i] - alpha * vn[i];
      for (int e = P.rp[i]; e < P.rp[i + 1]; ++e) {
        const int j = P.col[e];
        t += P.val[e] * (P.dinv[j] * (X.r[j] - alpha * vn[j]));
      }
    }
    X.t[i] = t;
    ts += t * sv;
    tt += t * t;
  }
  put_partial(X.part + P_TS * P.nb, ts);
  put_partial(X.part + P_TT * P.nb, tt);
}

// Iteration k, part 3: omega = t.s / t.t; x += alpha p^ + omega s^;
// r = s - omega t; partial sums of r^.r and r.r of iterate k+1.
__global__ void __launch_bounds__(kThreads) k_bi_c(PoissonDev P, CgVec X, int k) {
  if (block_done(X.ctl)) return;
  const int cur = k & 1, nxt = cur ^ 1;
  const double tt = sum_partials(X.part + P_TT * P.nb, P.nb);
  const double om = tt > 0.0 ? sum_partials(X.part + P_TS * P.nb, P.nb) / tt : 0.0;
  if (blockIdx.x == 0 && threadIdx.x == 0) X.ctl->omega = om;
  const double alpha = X.ctl->alpha;
  const double* pn = cur ? X.p0 : X.p1;
  const double* vn = cur ? X.v0 : X.v1;
  int i0, i1;
  agg_rows(P, i0, i1);
  double rho = 0.0, rr = 0.0;
  for (int i = i0 + threadIdx.x; i < i1; i += kThreads) {
    const double di = P.dinv[i];
    if (di == 0.0) continue;
    const double sv = X.r[i] - alpha * vn[i];
    X.x[i] += alpha * (di * pn[i]) + om * (di * sv);
    const double r = sv - om * X.t[i];
    X.r[i] = r;
    rho += X.rh[i] * r;
    rr += r * r;
  }
  put_partial(X.part + (P_RHO0 + nxt) * P.nb, rho);
  put_partial(X.part + (P_RR0 + nxt) * P.nb, rr);
}

// Singular systems: phi with zero volume mean.
__global__ void __launch_bounds__(kThreads) k_cg_mean1(PoissonDev P, CgVec X) {
  int i0, i1;
  agg_rows(P, i0, i1);
  double s = 0.0;
  for (int i = i0 + threadIdx.x; i < i1; i += kThreads) s += P.vn[i] * X.x[i];
  put_partial(X.part + P_VX * P.nb, s);
}

__global__ void __launch_bounds__(kThreads) k_cg_mean2(PoissonDev P, CgVec X) {
  const double m = sum_partials(X.part + P_VX * P.nb, P.nb) / sum_partials(X.part + P_V * P.nb, P.nb);
  int i0, i1;
  agg_rows(P, i0, i1);
  for (int i = i0 + threadIdx.x; i < i1; i += kThreads) X.x[i] -= m;
}

__global__ void __launch_bounds__(kThreads) k_cg_scatter(PoissonDev P, const double* __restrict__ x,
                                                          double* __restrict__ out) {
  const int i = blockIdx.x * kThreads + threadIdx.x;
  if (i < P.n) out[P.perm[i]] = x[i];
}

__global__ void __launch_bounds__(kThreads) k_gather(PoissonDev P, const double* __restrict__ in,
                                                      double* __restrict__ x) {
  const int i = blockIdx.x * kThreads + threadIdx.x;
  if (i < P.n) x[i] = in[P.perm[i]];
}

// E = -grad phi at the nodes (phi in internal order), out in caller order.
__global__ void __launch_bounds__(kThreads) k_field(PoissonDev P, const double* __restrict__ phi,
                                                     const double* bg, double* E) {
  const int i = blockIdx.x * kThreads + threadIdx.x;
  if (i >= P.n) return;
  double e[3] = {0.0, 0.0, 0.0};
  for (int q = P.rp[i]; q < P.rp[i + 1]; ++q) {
    const double f = phi[P.col[q]];
    for (int d = 0; d < P.nd; ++d) e[d] += P.gval[(size_t)d * P.nnz + q] * f;
  }
  // caller order; a background field (caller order, may alias E) is added
  const int o = P.perm[i];
  for (int d = 0; d < P.nd; ++d) {
    const size_t k = (size_t)d * P.n + o;
    E[k] = bg ? bg[k] + e[d] : e[d];
  }
}

// Host assembly: per node, the (column, value, gradient weights) entries of
// its cells, sorted by column with equal columns summed in cell order.
struct Entry {
  int col;
  int cell;
  double v, g[3];
};

void simplex_grads(int nd, const double (&X)[4][3], double (&grad)[4][3], double& vol) {
  if (nd == 2) {
    const double ax = X[1][0] - X[0][0], ay = X[1][1] - X[0][1];
    const double bx = X[2][0] - X[0][0], by = X[2][1] - X[0][1];
    const double det = ax * by - ay * bx;
    vol = 0.5 * std::fabs(det);
    // rows of the inverse of [e1 e2]^T: grad lambda_1, grad lambda_2
    grad[1][0] = by / det;
    grad[1][1] = -bx / det;
    grad[2][0] = -ay / det;
    grad[2][1] = ax / det;
    grad[0][0] = -(grad[1][0] + grad[2][0]);
    grad[0][1] = -(grad[1][1] + grad[2][1]);
    return;
  }
  double e[3][3];
  for (int k = 0; k < 3; ++k)
    for (int d = 0; d < 3; ++d) e[k][d] = X[k + 1][d] - X[0][d];
  // grad lambda_k (k = 1..3) are the rows of the inverse transpose of the
  // matrix with rows e_k: cross products of the other two edge vectors / det
  const double c0[3] = {e[1][1] * e[2][2] - e[1][2] * e[2][1], e[1][2] * e[2][0] - e[1][0] * e[2][2],
                        e[1][0] * e[2][1] - e[1][1] * e[2][0]};
  const double c1[3] = {e[2][1] * e[0][2] - e[2][2] * e[0][1], e[2][2] * e[0][0] - e[2][0] * e[0][2],
                        e[2][0] * e[0][1] - e[2][1] * e[0][0]};
  const double c2[3] = {e[0][1] * e[1][2] - e[0][2] * e[1][1], e[0][2] * e[1][0] - e[0][0] * e[1][2],
                        e[0][0] * e[1][1] - e[0][1] * e[1][0]};
  const double det = e[0][0] * c0[0] + e[0][1] * c0[1] + e[0][2] * c0[2];
  vol = std::fabs(det) / 6.0;
  for (int d = 0; d < 3; ++d) {
    grad[1][d] = c0[d] / det;
    grad[2][d] = c1[d] / det;
    grad[3][d] = c2[d] / det;
    grad[0][d] = -(grad[1][d] + grad[2][d] + grad[3][d]);
  }
}

// Inverse of a dense SPD matrix (row-major, n x n) by Cholesky: A = L L^T,
// A^-1 = L^-T L^-1.  Returns false if A is not numerically positive definite.
bool spd_inverse(std::vector<double>& A, int n) {
  std::vector<double> L((size_t)n * n, 0.0);
  for (int j = 0; j < n; ++j) {
    double d = A[(size_t)j * n + j];
    for (int k = 0; k < j; ++k) d -= L[(size_t)j * n + k] * L[(size_t)j * n + k];
    if (!(d > 0.0)) return false;
    const double ljj = std::sqrt(d);
    L[(size_t)j * n + j] = ljj;
    for (int i = j + 1; i < n; ++i) {
      double v = A[(size_t)i * n + j];
      for (int k = 0; k < j; ++k) v -= L[(size_t)i * n + k] * L[(size_t)j * n + k];
      L[(size_t)i * n + j] = v / ljj;
    }
  }
  // M = L^-1 (lower triangular), column by column; stored transposed,
  // Mt[c][i] = M[i][c], so that every inner loop runs over contiguous memory
  std::vector<double> Mt((size_t)n * n, 0.0);
  for (int c = 0; c < n; ++c) {
    double* mc = &Mt[(size_t)c * n];
    mc[c] = 1.0 / L[(size_t)c * n + c];
    for (int i = c + 1; i < n; ++i) {
      const double* li = &L[(size_t)i * n];
      double v = 0.0;
      for (int k = c; k < i; ++k) v -= li[k] * mc[k];
      mc[i] = v / li[i];
    }
  }
  // A^-1 = M^T M: (i, j) is the product of columns i and j of M
  for (int i = 0; i < n; ++i)
    for (int j = 0; j <= i; ++j) {
      const double* mi = &Mt[(size_t)i * n];
      const double* mj = &Mt[(size_t)j * n];
      double v = 0.0;
      for (int k = i; k < n; ++k) v += mi[k] * mj[k];
      A[(size_t)i * n + j] = v;
      A[(size_t)j * n + i] = v;
    }
  return true;
}

constexpr int kMaxCoarse = 2048;

}  // namespace

struct vcx_poisson_s {
  vcx_mesh mesh = nullptr;
  hipStream_t stream = nullptr;
  PoissonDev P{};
  CgVec X{};
  std::vector<void*> allocs;
  double* stage = nullptr;  // [4][n] caller-order inputs
  double* fbuf = nullptr;   // [nd][n] field rows for host outputs
  CgCtl* ctl_host = nullptr;
  int n = 0, nd = 0;
  bool bicg = false;  // non-symmetric operator (axisymmetric mesh): BiCGStab
};

static vcx_status dev_alloc(vcx_poisson p, size_t bytes, void** out) {
  PS_HIP(hipMalloc(out, std::max<size_t>(bytes, 8)));
  p->allocs.push_back(*out);
  return VCX_OK;
}

template <typename T>
static vcx_status upload(vcx_poisson p, const std::vector<T>& h, const T** out) {
  void* d = nullptr;
  vcx_status st = dev_alloc(p, sizeof(T) * h.size(), &d);
  if (st != VCX_OK) return st;
  if (!h.empty()) PS_HIP(hipMemcpy(d, h.data(), sizeof(T) * h.size(), hipMemcpyHostToDevice));
  *out = static_cast<const T*>(d);
  return VCX_OK;
}

static void release(vcx_poisson p) {
  if (p->stream) (void)hipStreamSynchronize(p->stream);
  for (void* a : p->allocs) (void)hipFree(a);
  if (p->ctl_host) (void)hipHostFree(p->ctl_host);
  delete p;
}

extern "C" vcx_status vcx_poisson_create(vcx_mesh mesh, const int32_t* dirichlet, vcx_poisson* out) {
  if (!mesh || !out) return err(VCX_E_ARG, "NULL argument");
  *out = nullptr;
  const HostMesh& h = *vcx::mesh_host(mesh);
  const int nd = h.nd, nv = h.nv;
  const int64_t n = h.nn, nc = h.nc;
  if (nv != nd + 1) return err(VCX_E_ARG, "the Poisson operator is assembled on simplex meshes");
  if (n >= (int64_t)1 << 31) return err(VCX_E_ARG, "mesh too large for 32-bit rows");
  // Dirichlet flags in the internal order
  std::vector<char> dir((size_t)n, 0);
  bool any_dir = false;
  if (dirichlet)
    for (int64_t i = 0; i < n; ++i)
      if (dirichlet[h.perm[i]]) dir[(size_t)i] = 1, any_dir = true;
  // node -> cells incidence, cells ascending
  std::vector<int64_t> nc_ptr((size_t)n + 1, 0);
  for (int64_t c = 0; c < nc; ++c)
    for (int k = 0; k < nv; ++k) nc_ptr[(size_t)h.cell[(size_t)k * nc + c] + 1]++;
  for (int64_t i = 0; i < n; ++i) nc_ptr[(size_t)i + 1] += nc_ptr[(size_t)i];
  std::vector<int64_t> fill(nc_ptr.begin(), nc_ptr.end() - 1);
  std::vector<int32_t> nc_cell((size_t)nc_ptr[(size_t)n]);
  std::vector<int8_t> nc_vert((size_t)nc_ptr[(size_t)n]);
  for (int64_t c = 0; c < nc; ++c)
    for (int k = 0; k < nv; ++k) {
      const int64_t i = h.cell[(size_t)k * nc + c];
      nc_cell[(size_t)fill[(size_t)i]] = (int32_t)c;
      nc_vert[(size_t)fill[(size_t)i]++] = (int8_t)k;
    }
  // rows
  std::vector<int32_t> rp((size_t)n + 1, 0), col;
  std::vector<double> val, gv[3], dinv((size_t)n, 0.0), sbm((size_t)n, 0.0);
  col.reserve((size_t)n * (nd == 2 ? 7 : 15));
  val.reserve(col.capacity());
  std::vector<Entry> ent;
  for (int64_t i = 0; i < n; ++i) {
    ent.clear();
    for (int64_t t = nc_ptr[(size_t)i]; t < nc_ptr[(size_t)i + 1]; ++t) {
      const int64_t c = nc_cell[(size_t)t];
      const int a = nc_vert[(size_t)t];
      double X[4][3] = {}, grad[4][3] = {}, vol = 0.0;
      for (int k = 0; k < nv; ++k) {
        const int64_t g = h.cell[(size_t)k * nc + c];
        for (int d = 0; d < nd; ++d) {
          double x = h.x[(size_t)d * n + g];
          if (k > 0 && h.has_period) x += vcx::shift_of(h.shift[(size_t)c], k, d, nd) * h.period[d];
          X[k][d] = x;
        }
      }
      simplex_grads(nd, X, grad, vol);
      // axisymmetric: int r n dl over node a's dual boundary in the cell is
      // sum over its other vertices j of the segment normal (S_a - S_j)/6
      // (S_k = -2 A grad lambda_k) times the segment's centroid radius
      // (r_a + r_j + 2 r_c)/4; the row then takes -grad lambda_k . that
      double wa[3] = {0, 0, 0};
      if (h.axi) {
        const double rc = (X[0][1] + X[1][1] + X[2][1]) / 3.0;
        for (int j = 0; j < 3; ++j) {
          if (j == a) continue;
          const double rr = X[a][1] + X[j][1] + 2.0 * rc;
          for (int d = 0; d < 2; ++d) wa[d] += -(vol / 12.0) * (grad[a][d] - grad[j][d]) * rr;
        }
      }
      for (int k = 0; k < nv; ++k) {
        Entry e{};
        e.col = h.cell[(size_t)k * nc + c];
        e.cell = (int)c;
        double dot = 0.0;
        if (h.axi) {
          for (int d = 0; d < nd; ++d) dot -= grad[k][d] * wa[d];
          e.v = dot;
        } else {
          for (int d = 0; d < nd; ++d) dot += grad[a][d] * grad[k][d];
          e.v = vol * dot;
        }
        // E_i = -(1/V_i) sum_tau (V_tau/n_v) grad phi_tau, grad phi_tau = sum_k phi_k grad lambda_k
        for (int d = 0; d < nd; ++d) e.g[d] = -(vol / nv) * grad[k][d];
        ent.push_back(e);
      }
    }
    std::stable_sort(ent.begin(), ent.end(), [](const Entry& x, const Entry& y) { return x.col < y.col; });
    const double inv_v = 1.0 / h.vnode[(size_t)i];
    size_t q = 0;
    while (q < ent.size()) {
      const int c = ent[q].col;
      double v = 0.0, g[3] = {0, 0, 0};
      for (; q < ent.size() && ent[q].col == c; ++q) {
        v += ent[q].v;
        for (int d = 0; d < nd; ++d) g[d] += ent[q].g[d];
      }
      if (dir[(size_t)i] && c != i) v = 0.0;  // Dirichlet row: identity (kept out of the CG)
      col.push_back(c);
      val.push_back(v);
      for (int d = 0; d < nd; ++d) gv[d].push_back(g[d] * inv_v);
      if (c == i && !dir[(size_t)i]) dinv[(size_t)i] = 1.0 / v;
    }
    rp[(size_t)i + 1] = (int32_t)col.size();
  }
  if (col.size() >= ((size_t)1 << 31)) return err(VCX_E_ARG, "operator too large for 32-bit indices");
  for (size_t b = 0; b < h.bnd_node.size(); ++b) {
    double s = 0.0;
    for (int d = 0; d < nd; ++d) s += h.bnd_S[(size_t)d * h.bnd_node.size() + b] * h.bnd_S[(size_t)d * h.bnd_node.size() + b];
    sbm[(size_t)h.bnd_node[b]] = std::sqrt(s);
  }
  std::vector<double> gall;
  gall.reserve(col.size() * nd);
  for (int d = 0; d < nd; ++d) gall.insert(gall.end(), gv[d].begin(), gv[d].end());

  auto* p = new (std::nothrow) vcx_poisson_s();
  if (!p) return err(VCX_E_OOM, "host allocation failed");
  p->mesh = mesh;
  p->stream = vcx::mesh_stream(mesh);
  p->n = (int)n;
  p->nd = nd;
  PoissonDev& P = p->P;
  P.n = (int)n;
  P.nd = nd;
  P.nnz = (int)col.size();
  P.singular = any_dir ? 0 : 1;
  P.perm = vcx::mesh_perm_device(mesh);
  vcx_status st = VCX_OK;
  auto chk = [&](vcx_status s) {
    if (st == VCX_OK) st = s;
  };
  chk(upload(p, rp, &P.rp));
  chk(upload(p, col, &P.col));
  chk(upload(p, val, &P.val));
  chk(upload(p, gall, &P.gval));
  chk(upload(p, dinv, &P.dinv));
  chk(upload(p, h.vupd, &P.vn));  // revolved volumes on axisymmetric meshes
  chk(upload(p, sbm, &P.sbm));
  // aggregates: runs of 64, 128 or a multiple of kThreads consecutive nodes
  // of the space-filling curve, at most kMaxCoarse of them (a block holds
  // whole aggregates); coarse operator A_c = R L R^T over free nodes,
  // inverted densely on the host
  const int64_t per = (n + kMaxCoarse - 1) / kMaxCoarse;
  P.agg = per <= 64 ? 64 : per <= 128 ? 128 : (int)(((per + kThreads - 1) / kThreads) * kThreads);
  P.nc = (int)((n + P.agg - 1) / P.agg);
  P.rpb = std::max(P.agg, kThreads);
  P.nb = (int)((n + P.rpb - 1) / P.rpb);
  const int ncg = P.nc;
  p->bicg = h.axi;
  // the coarse space serves the symmetric operator (conjugate gradients);
  // axisymmetric operators go to BiCGStab with Jacobi alone
  std::vector<double> Ac(h.axi ? 1 : (size_t)ncg * ncg, 0.0);
  for (int64_t i = 0; i < n && !h.axi; ++i) {
    if (dir[(size_t)i]) continue;
    const int a = (int)(i / P.agg);
    for (int32_t e = rp[(size_t)i]; e < rp[(size_t)i + 1]; ++e) {
      const int j = col[(size_t)e];
      if (!dir[(size_t)j]) Ac[(size_t)a * ncg + j / P.agg] += val[(size_t)e];
    }
  }
  if (!h.axi) {
    double tr = 0.0;
    for (int a = 0; a < ncg; ++a) tr += Ac[(size_t)a * ncg + a];
    for (int a = 0; a < ncg; ++a)
      if (Ac[(size_t)a * ncg + a] == 0.0) Ac[(size_t)a * ncg + a] = tr > 0.0 ? tr / ncg : 1.0;  // no free node
    if (!any_dir) {
      // constants are the null space: (A_c + mu 1 1^T)^-1 acts as the
      // pseudo-inverse on restrictions of residuals, which sum to zero
      const double mu = tr / ((double)ncg * ncg);
      for (double& v : Ac) v += mu;
    }
    if (!spd_inverse(Ac, ncg)) st = err(VCX_E_MESH, "coarse Poisson operator is not positive definite");
  }
  chk(upload(p, Ac, &P.ainv));
  CgVec& X = p->X;
  double** vecs[10] = {&X.x, &X.r, &X.p0, &X.p1, &X.q, &X.b, &X.rh, &X.v0, &X.v1, &X.t};
  for (double** v : vecs) {
    void* d = nullptr;
    chk(dev_alloc(p, sizeof(double) * (size_t)n, &d));
    *v = static_cast<double*>(d);
  }
  void* d = nullptr;
  chk(dev_alloc(p, sizeof(double) * ncg, &d));
  X.g = static_cast<double*>(d);
  chk(dev_alloc(p, sizeof(double) * ncg, &d));
  X.c = static_cast<double*>(d);
  chk(dev_alloc(p, sizeof(double) * P_NROWS * (size_t)P.nb, &d));
  X.part = static_cast<double*>(d);
  chk(dev_alloc(p, sizeof(CgCtl), &d));
  X.ctl = static_cast<CgCtl*>(d);
  chk(dev_alloc(p, sizeof(double) * 4 * (size_t)n, &d));
  p->stage = static_cast<double*>(d);
  chk(dev_alloc(p, sizeof(double) * nd * (size_t)n, &d));
  p->fbuf = static_cast<double*>(d);
  if (st == VCX_OK && hipHostMalloc(reinterpret_cast<void**>(&p->ctl_host), sizeof(CgCtl)) != hipSuccess)
    st = err(VCX_E_OOM, "pinned host allocation failed");
  if (st != VCX_OK) {
    release(p);
    return st;
  }
  *out = p;
  return VCX_OK;
}

extern "C" vcx_status vcx_poisson_destroy(vcx_poisson p) {
  if (!p) return err(VCX_E_ARG, "NULL handle");
  release(p);
  return VCX_OK;
}

// caller-order input: device pointer as is, host array staged on the device
static vcx_status stage_in(vcx_poisson p, const double* src, int slot, int is_device, const double** out) {
  if (!src) {
    *out = nullptr;
    return VCX_OK;
  }
  if (is_device) {
    *out = src;
    return VCX_OK;
  }
  double* dst = p->stage + (size_t)slot * p->n;
  PS_HIP(hipMemcpyAsync(dst, src, sizeof(double) * p->n, hipMemcpyHostToDevice, p->stream));
  *out = dst;
  return VCX_OK;
}

extern "C" vcx_status vcx_poisson_solve(vcx_poisson p, const double* q, const double* phiD, const double* En,
                                        double* phi, int is_device, double tol, int max_iter, int* iters,
                                        double* relres) {
  if (!p || !q || !phi) return err(VCX_E_ARG, "NULL argument");
  if (!(tol > 0.0) || max_iter < 0) return err(VCX_E_ARG, "need tol > 0 and max_iter >= 0");
  const double *dq, *dD, *dE, *d0;
  vcx_status st = stage_in(p, q, 0, is_device, &dq);
  if (st == VCX_OK) st = stage_in(p, phiD, 1, is_device, &dD);
  if (st == VCX_OK) st = stage_in(p, En, 2, is_device, &dE);
  if (st == VCX_OK) st = stage_in(p, phi, 3, is_device, &d0);
  if (st != VCX_OK) return st;
  const dim3 grid(p->P.nb), block(kThreads);
  PS_HIP(hipMemsetAsync(p->X.ctl, 0, sizeof(CgCtl), p->stream));
  hipLaunchKernelGGL(k_cg_init1, grid, block, 0, p->stream, p->P, p->X, dq, dD, dE, d0);
  if (p->bicg)
    hipLaunchKernelGGL(k_bi_init2, grid, block, 0, p->stream, p->P, p->X);
  else
    hipLaunchKernelGGL(k_cg_init2, grid, block, 0, p->stream, p->P, p->X);
  PS_HIP(hipGetLastError());
  const double tol2 = tol * tol;
  // one iteration: conjugate gradients (coarse correction, direction and
  // product, update) or BiCGStab (three parts); the first kernel of each
  // holds the stop test
  auto head = [&](int it) {
    if (p->bicg) {
      hipLaunchKernelGGL(k_bi_a, grid, block, 0, p->stream, p->P, p->X, it, tol2);
    } else {
      hipLaunchKernelGGL(k_cg_c, grid, block, 0, p->stream, p->P, p->X);
      hipLaunchKernelGGL(k_cg_a, grid, block, 0, p->stream, p->P, p->X, it, tol2);
    }
  };
  auto tail = [&](int it) {
    if (p->bicg) {
      hipLaunchKernelGGL(k_bi_b, grid, block, 0, p->stream, p->P, p->X, it);
      hipLaunchKernelGGL(k_bi_c, grid, block, 0, p->stream, p->P, p->X, it);
    } else {
      hipLaunchKernelGGL(k_cg_b, grid, block, 0, p->stream, p->P, p->X, it);
    }
  };
  int k = 0, chunk = 8;
  bool done = false;
  while (!done) {
    // iterations k .. k+c-1, then the stop test of iterate k+c (which also
    // does the first part of iteration k+c when it does not stop)
    const int c = std::min(chunk, max_iter - k);
    for (int j = 0; j < c; ++j) {
      head(k + j);
      tail(k + j);
    }
    k += c;
    head(k);
    PS_HIP(hipGetLastError());
    PS_HIP(hipMemcpyAsync(p->ctl_host, p->X.ctl, sizeof(CgCtl), hipMemcpyDeviceToHost, p->stream));
    PS_HIP(hipStreamSynchronize(p->stream));
    done = p->ctl_host->done || k >= max_iter;
    chunk = std::min(chunk * 2, 256);
    if (!done) {
      // the test launch above did iteration k's first part: finish it
      tail(k);
      k += 1;
    }
  }
  if (p->P.singular) {
    hipLaunchKernelGGL(k_cg_mean1, grid, block, 0, p->stream, p->P, p->X);
    hipLaunchKernelGGL(k_cg_mean2, grid, block, 0, p->stream, p->P, p->X);
  }
  double* dst = is_device ? phi : p->stage;
  hipLaunchKernelGGL(k_cg_scatter, dim3((p->n + kThreads - 1) / kThreads), block, 0, p->stream, p->P,
                     (const double*)p->X.x, dst);
  PS_HIP(hipGetLastError());
  if (!is_device) PS_HIP(hipMemcpyAsync(phi, p->stage, sizeof(double) * p->n, hipMemcpyDeviceToHost, p->stream));
  PS_HIP(hipStreamSynchronize(p->stream));
  const CgCtl& c = *p->ctl_host;
  const int it = c.done ? c.iters : c.last;
  const double rel = c.ref2 > 0.0 ? std::sqrt(c.rr / c.ref2) : std::sqrt(c.rr);
  if (iters) *iters = it;
  if (relres) *relres = rel;
  if (c.fault == 1 || !std::isfinite(rel))
    return err(VCX_E_UNSTABLE, "non-finite residual in the Poisson solve (non-finite q, phiD or En)");
  if (c.fault == 2)
    return err(VCX_E_STATE, "BiCGStab breakdown before the tolerance was reached");
  if (!c.done) return err(VCX_E_STATE, "conjugate gradients did not reach the tolerance within max_iter");
  if (!(rel <= tol)) return err(VCX_E_STATE, "the Poisson solve stopped above the tolerance");
  return VCX_OK;
}

static vcx_status field(vcx_poisson p, const double* phi, const double* Ebg, double* E, int is_device) {
  if (!p || !phi || !E) return err(VCX_E_ARG, "NULL argument");
  const double* dphi;
  vcx_status st = stage_in(p, phi, 0, is_device, &dphi);
  if (st != VCX_OK) return st;
  const dim3 g1((p->n + kThreads - 1) / kThreads), block(kThreads);
  double* tmp = p->stage + (size_t)p->n;  // phi in the internal order
  hipLaunchKernelGGL(k_gather, g1, block, 0, p->stream, p->P, dphi, tmp);
  double* rows = is_device ? E : p->fbuf;
  const double* bg = Ebg;
  if (Ebg && !is_device) {  // host background: staged in the output rows
    PS_HIP(hipMemcpyAsync(p->fbuf, Ebg, sizeof(double) * (size_t)p->nd * p->n, hipMemcpyHostToDevice,
                          p->stream));
    bg = p->fbuf;
  }
  hipLaunchKernelGGL(k_field, g1, block, 0, p->stream, p->P, (const double*)tmp, bg, rows);
  PS_HIP(hipGetLastError());
  if (!is_device)
    PS_HIP(hipMemcpyAsync(E, p->fbuf, sizeof(double) * (size_t)p->nd * p->n, hipMemcpyDeviceToHost, p->stream));
  PS_HIP(hipStreamSynchronize(p->stream));
  return VCX_OK;
}

extern "C" vcx_status vcx_poisson_field(vcx_poisson p, const double* phi, double* E, int is_device) {
  return field(p, phi, nullptr, E, is_device);
}

extern "C" vcx_status vcx_poisson_field_add(vcx_poisson p, const double* phi, const double* Ebg, double* E,
                                            int is_device) {
  if (!Ebg) return err(VCX_E_ARG, "NULL background field");
  return field(p, phi, Ebg, E, is_device);
}

extern "C" vcx_status vcx_poisson_info(vcx_poisson p, int64_t out[4]) {
  if (!p || !out) return err(VCX_E_ARG, "NULL argument");
  out[0] = p->n;
  out[1] = p->P.nnz;
  out[2] = p->bicg ? 0 : p->P.nc;
  out[3] = p->bicg ? 1 : 0;
  return VCX_OK;
}
