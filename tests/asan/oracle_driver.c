/*
 * Host-only driver of the dense oracle (oracle/bem_dense.c) for a build
 * with AddressSanitizer and UndefinedBehaviorSanitizer: every entry point
 * runs once on a small closed mesh (an octahedron refined once, 32 flat
 * triangles) with a few charges inside, restarted and full GMRES, and the
 * ragged row subsets.  Exit status 0 if every output is finite; the
 * sanitizers abort on any out-of-bounds access or undefined operation.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int or_geometry(const double *verts, int64_t nv, const int32_t *tris, int64_t nt, double *c, double *n, double *a);
void or_field_B(const double *c, const double *n, int64_t N, const double *rq, const double *q, int64_t Q,
                double *E);
void or_apply_Kp_rows(const double *c, const double *n, const double *a, int64_t N, const double *x,
                      const int64_t *rows, int64_t nrows, double *out);
void or_apply_A_rows(const double *c, const double *n, const double *a, int64_t N, double f, const double *x,
                     const int64_t *rows, int64_t nrows, double *out);
void or_apply_KpT_rows(const double *c, const double *n, const double *a, int64_t N, const double *y,
                       const int64_t *rows, int64_t nrows, double *out);
void or_apply_AT_rows(const double *c, const double *n, const double *a, int64_t N, double f, const double *y,
                      const int64_t *rows, int64_t nrows, double *out);
void or_apply_C(const double *c, const double *a, int64_t N, const double *rq, int64_t Q, const double *x,
                double *phi);
void or_apply_CT(const double *c, const double *a, int64_t N, const double *rq, const double *q, int64_t Q,
                 double *out);
void or_apply_BT(const double *c, const double *n, int64_t N, const double *rq, int64_t Q, const double *y,
                 double *out);
void or_grad_at_points(const double *c, const double *n, int64_t N, const double *w, const double *d,
                       const double *rq, int64_t Q, double *out);
void or_assemble_A(const double *c, const double *n, const double *a, int64_t N, double f, double *Am);
int or_gmres(const double *c, const double *n, const double *a, int64_t N, double f, int transpose, const double *b,
             double *x, double tol, int maxit, int restart, int *iters_out, double *relres_out);
double or_energy_from_phi(const double *q, const double *phi, int64_t Q, double kappa);

static int finite_all(const double *v, int64_t n) {
  for (int64_t i = 0; i < n; ++i)
    if (!isfinite(v[i])) return 0;
  return 1;
}

/* midpoint of edge (i, j), projected to the unit sphere; appended to V */
static int32_t midpoint(double *V, int32_t *nv, int32_t i, int32_t j) {
  double m[3], r = 0.0;
  for (int d = 0; d < 3; ++d) {
    m[d] = 0.5 * (V[3 * i + d] + V[3 * j + d]);
    r += m[d] * m[d];
  }
  r = sqrt(r);
  for (int d = 0; d < 3; ++d) V[3 * *nv + d] = m[d] / r;
  return (*nv)++;
}

int main(void) {
  /* octahedron, faces counter-clockwise seen from outside */
  double V[3 * 64] = {1, 0, 0, -1, 0, 0, 0, 1, 0, 0, -1, 0, 0, 0, 1, 0, 0, -1};
  int32_t nv = 6;
  const int32_t oct[8][3] = {{0, 2, 4}, {2, 1, 4}, {1, 3, 4}, {3, 0, 4},
                             {2, 0, 5}, {1, 2, 5}, {3, 1, 5}, {0, 3, 5}};
  enum { NT = 32, Q = 3 };
  int32_t tri[3 * NT];
  for (int f = 0; f < 8; ++f) {
    const int32_t a = oct[f][0], b = oct[f][1], c = oct[f][2];
    const int32_t ab = midpoint(V, &nv, a, b), bc = midpoint(V, &nv, b, c), ca = midpoint(V, &nv, c, a);
    const int32_t t[4][3] = {{a, ab, ca}, {ab, b, bc}, {ca, bc, c}, {ab, bc, ca}};
    for (int k = 0; k < 4; ++k)
      for (int d = 0; d < 3; ++d) tri[3 * (4 * f + k) + d] = t[k][d];
  }
  double *c = malloc(sizeof(double) * 3 * NT), *n = malloc(sizeof(double) * 3 * NT), *a = malloc(sizeof(double) * NT);
  if (or_geometry(V, nv, tri, NT, c, n, a) != 0) return 2;
  const double rq[3 * Q] = {0.1, 0.0, 0.0, -0.2, 0.3, 0.1, 0.0, -0.1, 0.4};
  const double q[Q] = {1.0, -0.5, 0.25};
  const double f = 0.95;
  double E[NT], x[NT], y[NT], out[NT], phi[Q], grad[3 * Q], Am[NT * NT], w[NT];
  const int64_t rows[5] = {0, 3, 17, 30, 31};
  or_field_B(c, n, NT, rq, q, Q, E);
  for (int i = 0; i < NT; ++i) {
    E[i] *= f;
    w[i] = a[i] * E[i];
  }
  int iters = 0;
  double rr = 0.0;
  int ok = finite_all(E, NT);
  ok &= or_gmres(c, n, a, NT, f, 0, E, x, 1e-12, 200, 0, &iters, &rr) == 0;
  ok &= or_gmres(c, n, a, NT, f, 1, E, y, 1e-12, 200, 4, &iters, &rr) == 0;
  or_apply_Kp_rows(c, n, a, NT, x, NULL, 0, out);
  ok &= finite_all(out, NT);
  or_apply_A_rows(c, n, a, NT, f, x, rows, 5, out);
  ok &= finite_all(out, 5);
  or_apply_KpT_rows(c, n, a, NT, y, rows, 5, out);
  ok &= finite_all(out, 5);
  or_apply_AT_rows(c, n, a, NT, f, y, NULL, 0, out);
  ok &= finite_all(out, NT);
  or_apply_C(c, a, NT, rq, Q, x, phi);
  ok &= finite_all(phi, Q);
  or_apply_CT(c, a, NT, rq, q, Q, out);
  ok &= finite_all(out, NT);
  or_apply_BT(c, n, NT, rq, Q, y, phi);
  ok &= finite_all(phi, Q);
  or_grad_at_points(c, n, NT, w, y, rq, Q, grad);
  ok &= finite_all(grad, 3 * Q);
  or_assemble_A(c, n, a, NT, f, Am);
  ok &= finite_all(Am, NT * NT);
  ok &= isfinite(or_energy_from_phi(q, phi, Q, 1.0));
  free(c);
  free(n);
  free(a);
  printf("%s iters=%d relres=%.3e\n", ok ? "ok" : "FAIL", iters, rr);
  return ok ? 0 : 1;
}
