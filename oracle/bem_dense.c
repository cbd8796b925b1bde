/*
 * FP64 dense boundary-element oracle for mixed-dielectric Poisson
 * electrostatics (Yokota, Bardhan, Knepley, Barba, Hamada, arXiv:1007.4591).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * statement of what the GPU library computes.  Only the tests, the smoke
 * check and the CPU-baseline leg of the benchmark may load it.  It shares no
 * code, header, table or helper with the GPU library.
 *
 * Discretisation (Section 2.1, the matrix statement A x = B q, phi = C x):
 *   flat triangular panels with one piecewise-constant unknown each, one
 *   quadrature point at the centroid; panel i has centroid c_i, outward unit
 *   normal n_i and area a_i.  G(r, r') = 1 / (4 pi |r - r'|).
 *
 *   E_i   = sum_q q_q  n_i . grad_r G(r, r_q) |_{r = c_i}           (field B q)
 *   K'_ij = a_j n_i . grad_r G(r, c_j) |_{r = c_i},  K'_ii = 0         (flat panel)
 *   A     = (1 - f/2) I - f K',    f = 1 - eps_in / eps_out
 *   solve A x = f E                 (interior-limit reading of eq. ASC)
 *   (C x)_q = sum_j a_j x_j G(r_q, c_j)                               (eq. reac)
 *   dG    = (2 pi K / eps_in) q^T C x   [kcal/mol], K = 332.06 kcal A/(mol e^2)
 *   BIBEE/CFA (eq. CFA): x = f E;  BIBEE/P: x = f E / (1 - f/2);
 *   BIBEE with K' replaced by +1/2: x = f E / (1 - f)  (numpy front end).
 *   Adjoint: A^T y = C^T q,  d dG/dq = kappa (C x + f B^T y),
 *            d dG/dr_q = kappa q_q [grad SL(a x) + f grad DL(y)](r_q),
 *   kappa = 2 pi K / eps_in, DL(y)(r) = sum_i y_i n_i.(r - c_i)/(4 pi |r - c_i|^3).
 *
 * Every row sum runs over sources in index order, so results do not depend
 * on the OpenMP thread count.  Build without -ffast-math and with
 * -ffp-contract=off.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_PI 3.14159265358979323846
#define OR_INV4PI (1.0 / (4.0 * OR_PI))

/* ------------------------------------------------------------ geometry */

/* Centroid, outward unit normal (right-hand rule on v0, v1, v2) and area.
 * Returns 0, or 1 if a triangle index is out of range, 2 if an area is zero
 * or not finite. */
int or_geometry(const double *verts, int64_t nv, const int32_t *tris, int64_t nt,
                double *c, double *n, double *a) {
  int bad = 0;
  for (int64_t i = 0; i < nt; ++i) {
    int32_t i0 = tris[3 * i], i1 = tris[3 * i + 1], i2 = tris[3 * i + 2];
    if (i0 < 0 || i1 < 0 || i2 < 0 || i0 >= nv || i1 >= nv || i2 >= nv) { bad = 1; continue; }
    const double *v0 = verts + 3 * (int64_t)i0, *v1 = verts + 3 * (int64_t)i1, *v2 = verts + 3 * (int64_t)i2;
    double e1[3], e2[3], m[3];
    for (int d = 0; d < 3; ++d) {
      c[3 * i + d] = (v0[d] + v1[d] + v2[d]) / 3.0;
      e1[d] = v1[d] - v0[d];
      e2[d] = v2[d] - v0[d];
    }
    m[0] = e1[1] * e2[2] - e1[2] * e2[1];
    m[1] = e1[2] * e2[0] - e1[0] * e2[2];
    m[2] = e1[0] * e2[1] - e1[1] * e2[0];
    double len = sqrt(m[0] * m[0] + m[1] * m[1] + m[2] * m[2]);
    if (!(len > 0.0) || !isfinite(len)) { if (!bad) bad = 2; a[i] = 0.0; continue; }
    a[i] = 0.5 * len;
    for (int d = 0; d < 3; ++d) n[3 * i + d] = m[d] / len;
  }
  return bad;
}

/* ------------------------------------------------ primitive pair kernels */

/* n_t . grad_r G(r, s) at r = t */
static inline double ngrad_G(const double *t, const double *nt, const double *s) {
  double dx = t[0] - s[0], dy = t[1] - s[1], dz = t[2] - s[2];
  double r2 = dx * dx + dy * dy + dz * dz;
  double r = sqrt(r2);
  return -(dx * nt[0] + dy * nt[1] + dz * nt[2]) * OR_INV4PI / (r2 * r);
}

static inline double G(const double *t, const double *s) {
  double dx = t[0] - s[0], dy = t[1] - s[1], dz = t[2] - s[2];
  return OR_INV4PI / sqrt(dx * dx + dy * dy + dz * dz);
}

/* potential at t of a unit dipole with direction m at s: m.(t - s)/(4 pi |t-s|^3) */
static inline double dipole_pot(const double *t, const double *s, const double *m) {
  double dx = t[0] - s[0], dy = t[1] - s[1], dz = t[2] - s[2];
  double r2 = dx * dx + dy * dy + dz * dz;
  double r = sqrt(r2);
  return (dx * m[0] + dy * m[1] + dz * m[2]) * OR_INV4PI / (r2 * r);
}

/* ------------------------------------------------------- dense operators */

/* E = B q: E_i = sum_q q_q n_i . grad G(c_i, r_q) */
void or_field_B(const double *c, const double *n, int64_t N, const double *rq, const double *q,
                int64_t Q, double *E) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < N; ++i) {
    double s = 0.0;
    for (int64_t k = 0; k < Q; ++k) s += q[k] * ngrad_G(c + 3 * i, n + 3 * i, rq + 3 * k);
    E[i] = s;
  }
}

/* (K' x)_i for the rows listed in rows[0..nrows) (rows == NULL: all rows) */
void or_apply_Kp_rows(const double *c, const double *n, const double *a, int64_t N, const double *x,
                      const int64_t *rows, int64_t nrows, double *out) {
  int64_t R = rows ? nrows : N;
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t r = 0; r < R; ++r) {
    int64_t i = rows ? rows[r] : r;
    double s = 0.0;
    for (int64_t j = 0; j < N; ++j) {
      if (j == i) continue;
      s += a[j] * x[j] * ngrad_G(c + 3 * i, n + 3 * i, c + 3 * j);
    }
    out[r] = s;
  }
}

/* y = A x = (1 - f/2) x - f K' x on the listed rows */
void or_apply_A_rows(const double *c, const double *n, const double *a, int64_t N, double f,
                     const double *x, const int64_t *rows, int64_t nrows, double *out) {
  or_apply_Kp_rows(c, n, a, N, x, rows, nrows, out);
  int64_t R = rows ? nrows : N;
  for (int64_t r = 0; r < R; ++r) {
    int64_t i = rows ? rows[r] : r;
    out[r] = (1.0 - 0.5 * f) * x[i] - f * out[r];
  }
}

/* (K'^T y)_i = a_i sum_{j != i} y_j n_j.(c_i - c_j)/(4 pi |c_i - c_j|^3) */
void or_apply_KpT_rows(const double *c, const double *n, const double *a, int64_t N,
                       const double *y, const int64_t *rows, int64_t nrows, double *out) {
  int64_t R = rows ? nrows : N;
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t r = 0; r < R; ++r) {
    int64_t i = rows ? rows[r] : r;
    double s = 0.0;
    for (int64_t j = 0; j < N; ++j) {
      if (j == i) continue;
      s += y[j] * dipole_pot(c + 3 * i, c + 3 * j, n + 3 * j);
    }
    out[r] = a[i] * s;
  }
}

void or_apply_AT_rows(const double *c, const double *n, const double *a, int64_t N, double f,
                      const double *y, const int64_t *rows, int64_t nrows, double *out) {
  or_apply_KpT_rows(c, n, a, N, y, rows, nrows, out);
  int64_t R = rows ? nrows : N;
  for (int64_t r = 0; r < R; ++r) {
    int64_t i = rows ? rows[r] : r;
    out[r] = (1.0 - 0.5 * f) * y[i] - f * out[r];
  }
}

/* (C x)_q = sum_j a_j x_j G(r_q, c_j) */
void or_apply_C(const double *c, const double *a, int64_t N, const double *rq, int64_t Q,
                const double *x, double *phi) {
#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < Q; ++k) {
    double s = 0.0;
    for (int64_t j = 0; j < N; ++j) s += a[j] * x[j] * G(rq + 3 * k, c + 3 * j);
    phi[k] = s;
  }
}

/* (C^T q)_j = a_j sum_q q_q G(c_j, r_q) */
void or_apply_CT(const double *c, const double *a, int64_t N, const double *rq, const double *q,
                 int64_t Q, double *out) {
#pragma omp parallel for schedule(static)
  for (int64_t j = 0; j < N; ++j) {
    double s = 0.0;
    for (int64_t k = 0; k < Q; ++k) s += q[k] * G(c + 3 * j, rq + 3 * k);
    out[j] = a[j] * s;
  }
}

/* (B^T y)_q = sum_i y_i n_i.(r_q - c_i)/(4 pi |r_q - c_i|^3) = DL(y)(r_q) */
void or_apply_BT(const double *c, const double *n, int64_t N, const double *rq, int64_t Q,
                 const double *y, double *out) {
#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < Q; ++k) {
    double s = 0.0;
    for (int64_t i = 0; i < N; ++i) s += y[i] * dipole_pot(rq + 3 * k, c + 3 * i, n + 3 * i);
    out[k] = s;
  }
}

/* grad_r [ sum_j w_j G(r, c_j) + sum_j d_j n_j.(r - c_j)/(4 pi |r - c_j|^3) ] at r = r_q.
 * w (monopole weights) or d (dipole strengths) may be NULL. */
void or_grad_at_points(const double *c, const double *n, int64_t N, const double *w,
                       const double *d, const double *rq, int64_t Q, double *out) {
#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < Q; ++k) {
    double gx = 0.0, gy = 0.0, gz = 0.0;
    for (int64_t j = 0; j < N; ++j) {
      double dx = rq[3 * k] - c[3 * j], dy = rq[3 * k + 1] - c[3 * j + 1], dz = rq[3 * k + 2] - c[3 * j + 2];
      double r2 = dx * dx + dy * dy + dz * dz;
      double r = sqrt(r2);
      double ir3 = 1.0 / (r2 * r);
      if (w) {
        double s = -w[j] * ir3;
        gx += s * dx; gy += s * dy; gz += s * dz;
      }
      if (d) {
        const double *m = n + 3 * j;
        double md = m[0] * dx + m[1] * dy + m[2] * dz;
        double ir5 = ir3 / r2;
        gx += d[j] * (m[0] * ir3 - 3.0 * md * dx * ir5);
        gy += d[j] * (m[1] * ir3 - 3.0 * md * dy * ir5);
        gz += d[j] * (m[2] * ir3 - 3.0 * md * dz * ir5);
      }
    }
    out[3 * k] = gx * OR_INV4PI;
    out[3 * k + 1] = gy * OR_INV4PI;
    out[3 * k + 2] = gz * OR_INV4PI;
  }
}

/* Explicit A (row-major N x N), for small N only. */
void or_assemble_A(const double *c, const double *n, const double *a, int64_t N, double f, double *Am) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < N; ++i) {
    for (int64_t j = 0; j < N; ++j) {
      double kij = (i == j) ? 0.0 : a[j] * ngrad_G(c + 3 * i, n + 3 * i, c + 3 * j);
      Am[i * N + j] = (i == j ? (1.0 - 0.5 * f) : 0.0) - f * kij;
    }
  }
}

/* ----------------------------------------------------------------- GMRES */

typedef struct {
  const double *c, *n, *a;
  int64_t N;
  double f;
  int transpose;
} or_op;

static void op_apply(const or_op *op, const double *x, double *y) {
  if (op->transpose)
    or_apply_AT_rows(op->c, op->n, op->a, op->N, op->f, x, NULL, 0, y);
  else
    or_apply_A_rows(op->c, op->n, op->a, op->N, op->f, x, NULL, 0, y);
}

static double dot(const double *u, const double *v, int64_t N) {
  double s = 0.0;
  for (int64_t i = 0; i < N; ++i) s += u[i] * v[i];
  return s;
}

/* Restarted GMRES(m) of Saad and Schultz: x0 = 0, Arnoldi with modified
 * Gram-Schmidt, Givens rotations on the Hessenberg matrix, stop when the
 * Givens residual estimate |g_{k+1}| / |b| <= tol, then the explicit
 * residual |b - A x| / |b| is returned in *relres.  restart <= 0 means no
 * restart (m = maxit).  Returns 0 if converged (explicit residual <= tol),
 * 1 otherwise. */
int or_gmres(const double *c, const double *n, const double *a, int64_t N, double f, int transpose,
             const double *b, double *x, double tol, int maxit, int restart, int *iters_out,
             double *relres) {
  or_op op = {c, n, a, N, f, transpose};
  int m = (restart <= 0 || restart > maxit) ? maxit : restart;
  double *V = (double *)calloc((size_t)(m + 1) * (size_t)N, sizeof(double));
  double *H = (double *)calloc((size_t)(m + 1) * (size_t)m, sizeof(double));
  double *cs = (double *)calloc((size_t)m, sizeof(double));
  double *sn = (double *)calloc((size_t)m, sizeof(double));
  double *g = (double *)calloc((size_t)(m + 1), sizeof(double));
  double *yv = (double *)calloc((size_t)m, sizeof(double));
  double *r = (double *)calloc((size_t)N, sizeof(double));
  double *w = (double *)calloc((size_t)N, sizeof(double));
  for (int64_t i = 0; i < N; ++i) x[i] = 0.0;
  double bnorm = sqrt(dot(b, b, N));
  int iters = 0, converged = 0;
  double res = 0.0;
  if (bnorm == 0.0) {
    converged = 1;
    goto done;
  }
  for (int64_t i = 0; i < N; ++i) r[i] = b[i];
  while (1) {
    double beta = sqrt(dot(r, r, N));
    if (beta / bnorm <= tol) { converged = 1; break; }
    if (iters >= maxit) break;
    for (int64_t i = 0; i < N; ++i) V[i] = r[i] / beta;
    for (int k = 0; k <= m; ++k) g[k] = 0.0;
    g[0] = beta;
    int k = 0;
    for (; k < m && iters < maxit; ++k) {
      double *vk = V + (size_t)k * N, *vn = V + (size_t)(k + 1) * N;
      op_apply(&op, vk, w);
      for (int i = 0; i <= k; ++i) {
        double h = dot(w, V + (size_t)i * N, N);
        H[i * m + k] = h;
        const double *vi = V + (size_t)i * N;
        for (int64_t t = 0; t < N; ++t) w[t] -= h * vi[t];
      }
      double hn = sqrt(dot(w, w, N));
      H[(k + 1) * m + k] = hn;
      if (hn > 0.0)
        for (int64_t t = 0; t < N; ++t) vn[t] = w[t] / hn;
      for (int i = 0; i < k; ++i) {
        double h0 = H[i * m + k], h1 = H[(i + 1) * m + k];
        H[i * m + k] = cs[i] * h0 + sn[i] * h1;
        H[(i + 1) * m + k] = -sn[i] * h0 + cs[i] * h1;
      }
      double h0 = H[k * m + k], h1 = H[(k + 1) * m + k];
      double den = sqrt(h0 * h0 + h1 * h1);
      cs[k] = den > 0.0 ? h0 / den : 1.0;
      sn[k] = den > 0.0 ? h1 / den : 0.0;
      H[k * m + k] = den;
      H[(k + 1) * m + k] = 0.0;
      g[k + 1] = -sn[k] * g[k];
      g[k] = cs[k] * g[k];
      ++iters;
      if (fabs(g[k + 1]) / bnorm <= tol || hn == 0.0) { ++k; break; }
    }
    /* back substitution on the k x k upper-triangular system */
    for (int i = k - 1; i >= 0; --i) {
      double s = g[i];
      for (int j = i + 1; j < k; ++j) s -= H[i * m + j] * yv[j];
      yv[i] = s / H[i * m + i];
    }
    for (int i = 0; i < k; ++i) {
      const double *vi = V + (size_t)i * N;
      for (int64_t t = 0; t < N; ++t) x[t] += yv[i] * vi[t];
    }
    op_apply(&op, x, w);
    for (int64_t t = 0; t < N; ++t) r[t] = b[t] - w[t];
  }
done:
  if (bnorm > 0.0) {
    op_apply(&op, x, w);
    for (int64_t t = 0; t < N; ++t) r[t] = b[t] - w[t];
    res = sqrt(dot(r, r, N)) / bnorm;
    converged = res <= tol;
  }
  if (iters_out) *iters_out = iters;
  if (relres) *relres = res;
  free(V); free(H); free(cs); free(sn); free(g); free(yv); free(r); free(w);
  return converged ? 0 : 1;
}

/* ------------------------------------------------------------- energies */

/* kappa q^T phi */
double or_energy_from_phi(const double *q, const double *phi, int64_t Q, double kappa) {
  double s = 0.0;
  for (int64_t k = 0; k < Q; ++k) s += q[k] * phi[k];
  return kappa * s;
}
