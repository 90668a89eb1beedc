/*
 * p1e_oracle.c -- plain FP64 reference ("oracle") for P1 finite-element energies.
 *
 * TEST INFRASTRUCTURE ONLY. Only the test suite, the package smoke check and the CPU-baseline
 * leg of the benchmark load this code. The product path never links, imports or calls it,
 * and it shares no code with the product (its own geometry, densities, patches, sums).
 *
 * It follows Moskovka & Valdman, "Fast MATLAB evaluation of nonlinear energies using FEM in
 * 2D and 3D: Nodal elements" (arXiv 2109.01158), written as slow, obvious element loops:
 *
 *   geometry     Section 4.1: element sizes |T| and P1 basis gradients from the vertex
 *                coordinates (B = [x_1-x_0, ..., x_dim-x_0], grad phi_l = row l of B^-1 for
 *                l >= 1, grad phi_0 = -sum of the others).
 *   F_T          eq. (Dv): F_T[j][m] = sum_l v[I(T,l)][j] * d phi_{T,l} / d x_m.
 *   densities    eq. (neoHook): W = C1 (|F|^2 - dim - 2 log det F) + D1 (det F - 1)^2;
 *                eq. (pLaplacian): W = |grad v|^p / p; and the same with the component-wise
 *                norm, W = sum_m |d v / d x_m|^p / p, whose minima are the energies printed
 *                for Benchmark 6 (Table 6);
 *                St. Venant-Kirchhoff, the extension Section 2 names after eq. (neoHook)
 *                (the paper gives no formula; the textbook one): W = C1 |E|^2 + D1 (tr E)^2
 *                with the Green-Lagrange strain E = (F^T F - I) / 2, C1 = mu, D1 = lambda / 2;
 *                Ginzburg-Landau, the scalar example Section 7 names for adding first-gradient
 *                problems (the textbook energy eps/2 |grad u|^2 + (u^2 - 1)^2 / 4, with C1 and
 *                D1 as its two coefficients): |T| C1 |grad u|^2 + D1 int_T (u^2 - 1)^2 dx, the
 *                integral of the P1 field's quartic taken exactly by expanding the power of
 *                u = sum_l u_l lambda_l over vertex tuples and integrating each barycentric
 *                monomial by int_T lambda^a = |T| dim! a! / (|a| + dim)!.
 *   J_grad       eq. (Denergy): sum over elements of |T| W(F_T), element order,
 *                Neumaier-compensated.
 *   b = M f      Section 3.2, eqs. (mass2D), (linearTerm2): consistent P1 mass matrix with
 *                element entries |T| (1 + delta_ab) / ((dim+1)(dim+2)).
 *   exact grad   Section 6.2, eq. (dWFv): dW/dF from the chain rule with d det F / dF_jm the
 *                signed 2x2 minor (cofactor) and d I1 / dF_jm = 2 F_jm, scattered per element.
 *   patch FD     Section 6.1, eqs. (CD), (CDS), (jgradpm), (sumpatch): for every free DOF n of
 *                node i, perturb v_n by +eps and -eps, recompute F_T (eq. Dv) on every element
 *                of the nodal patch T^i and difference the two patch sums of |T| W; and the
 *                fourth-order scheme on +-eps, +-2 eps (orc_grad_patch_fd4).
 *
 * Conventions (readings of the paper): J = J_grad - b.v (the linear part enters with a minus
 * sign); (Neo-Hookean) det F <= 0 or a non-finite density makes the element "bad": the energy
 * is +Inf and the bad elements are counted (St. Venant-Kirchhoff is finite for every F). For the p-Laplacian the gradient of |g|^p/p at g = 0 is 0.
 *
 * Build: gcc -O2 -ffp-contract=off -fPIC -shared (no OpenMP: single-threaded on purpose).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { ORC_PLAPLACE = 1, ORC_NEOHOOKE = 2, ORC_SVK = 3, ORC_GL = 4, ORC_PLAPLACE_ORTHO = 5 };

typedef struct {
  int32_t dim;    /* 2 or 3 */
  int32_t ncomp;  /* d: 1 (scalar) or dim (vector) */
  int32_t kind;   /* ORC_PLAPLACE, ORC_NEOHOOKE or ORC_SVK */
  int32_t pad_;
  int64_t nn, ne;
  const int32_t *conn;   /* [ne][dim+1] */
  const double *coords;  /* [nn][dim] */
  double p, C1, D1;
} orc_problem;

/* ---------------------------------------------------------------- Neumaier sum */
typedef struct { double s, c; } orc_acc;

static void acc_add(orc_acc *a, double x) {
  double t = a->s + x;
  if (fabs(a->s) >= fabs(x)) a->c += (a->s - t) + x;
  else a->c += (x - t) + a->s;
  a->s = t;
}
static double acc_result(const orc_acc *a) { return a->s + a->c; }

/* ---------------------------------------------------------------- small matrices */
static double det2(double a, double b, double c, double d) { return a * d - b * c; }

static double det_mat(int dim, double A[3][3]) {
  if (dim == 2) return det2(A[0][0], A[0][1], A[1][0], A[1][1]);
  return A[0][0] * A[1][1] * A[2][2] + A[0][2] * A[1][0] * A[2][1] + A[0][1] * A[1][2] * A[2][0]
       - A[0][2] * A[1][1] * A[2][0] - A[0][1] * A[1][0] * A[2][2] - A[0][0] * A[1][2] * A[2][1];
}

/* cof[j][m] = (-1)^(j+m) * det(A with row j and column m removed) */
static void cofactor(int dim, double A[3][3], double cof[3][3]) {
  if (dim == 2) {
    cof[0][0] = A[1][1];
    cof[0][1] = -A[1][0];
    cof[1][0] = -A[0][1];
    cof[1][1] = A[0][0];
    return;
  }
  for (int j = 0; j < 3; ++j) {
    for (int m = 0; m < 3; ++m) {
      double sub[2][2];
      int r = 0;
      for (int jj = 0; jj < 3; ++jj) {
        if (jj == j) continue;
        int c = 0;
        for (int mm = 0; mm < 3; ++mm) {
          if (mm == m) continue;
          sub[r][c++] = A[jj][mm];
        }
        ++r;
      }
      double minor = det2(sub[0][0], sub[0][1], sub[1][0], sub[1][1]);
      cof[j][m] = ((j + m) % 2 == 0) ? minor : -minor;
    }
  }
}

/* ---------------------------------------------------------------- geometry */
/* vol[e] = |det B|/dim!, dphi[e][l][m] = d phi_l / d x_m for element e. Returns the number of
 * elements with det B == 0 (degenerate). */
int64_t orc_geometry(const orc_problem *P, double *vol, double *dphi) {
  const int dim = P->dim, k = dim + 1;
  int64_t ndegen = 0;
  for (int64_t e = 0; e < P->ne; ++e) {
    const int32_t *T = P->conn + e * k;
    double B[3][3] = {{0}};
    for (int l = 1; l <= dim; ++l)
      for (int m = 0; m < dim; ++m)
        B[m][l - 1] = P->coords[(int64_t)T[l] * dim + m] - P->coords[(int64_t)T[0] * dim + m];
    double det = det_mat(dim, B);
    double fact = (dim == 2) ? 2.0 : 6.0;
    vol[e] = fabs(det) / fact;
    if (det == 0.0) ++ndegen;
    /* B^-1 = cof(B)^T / det B; row (l-1) of B^-1 is grad phi_l */
    double cof[3][3];
    cofactor(dim, B, cof);
    double *g = dphi + e * k * dim;
    for (int m = 0; m < dim; ++m) g[m] = 0.0;
    for (int l = 1; l <= dim; ++l) {
      for (int m = 0; m < dim; ++m) {
        double binv_lm = cof[m][l - 1] / det; /* (B^-1)[l-1][m] = cof(B)[m][l-1] / det */
        g[l * dim + m] = binv_lm;
        g[m] -= binv_lm;
      }
    }
  }
  return ndegen;
}

/* ---------------------------------------------------------------- P1 polynomial integrals */
static double factorial(int n) {
  double f = 1.0;
  for (int i = 2; i <= n; ++i) f *= i;
  return f;
}

/* int_T lambda_0^a[0] ... lambda_dim^a[dim] dx = |T| dim! a[0]! ... a[dim]! / (|a| + dim)! */
static double bary_moment(int dim, double vol, const int *a) {
  double num = factorial(dim);
  int tot = 0;
  for (int l = 0; l <= dim; ++l) {
    num *= factorial(a[l]);
    tot += a[l];
  }
  return vol * num / factorial(tot + dim);
}

/* int_T u^k lambda_m dx (m < 0: without the factor lambda_m) for u = sum_l u_l lambda_l, k <= 4:
 * the power expanded over all ordered k-tuples of vertices, each product of barycentric
 * coordinates integrated by bary_moment */
static double int_power(int dim, double vol, const double *u, int k, int m) {
  const int nv = dim + 1;
  int ntup = 1;
  for (int i = 0; i < k; ++i) ntup *= nv;
  double sum = 0.0;
  for (int t = 0; t < ntup; ++t) {
    int a[4] = {0, 0, 0, 0};
    double prod = 1.0;
    int r = t;
    for (int i = 0; i < k; ++i) {
      const int l = r % nv;
      r /= nv;
      a[l] += 1;
      prod *= u[l];
    }
    if (m >= 0) a[m] += 1;
    sum += prod * bary_moment(dim, vol, a);
  }
  return sum;
}

/* (Ginzburg-Landau) nodal values of element T */
static void element_values(const orc_problem *P, const double *v, const int32_t *T, double *u) {
  for (int l = 0; l <= P->dim; ++l) u[l] = v[T[l]];
}

/* int_T (u^2 - 1)^2 dx = int u^4 - 2 int u^2 + |T| */
static double gl_potential(int dim, double vol, const double *u) {
  return int_power(dim, vol, u, 4, -1) - 2.0 * int_power(dim, vol, u, 2, -1) + vol;
}

/* d/du_m int_T (u^2 - 1)^2 dx = int_T 4 u (u^2 - 1) lambda_m dx */
static double gl_potential_du(int dim, double vol, const double *u, int m) {
  return 4.0 * int_power(dim, vol, u, 3, m) - 4.0 * int_power(dim, vol, u, 1, m);
}

/* |T| W of element e with nodal field v: |T| W(F_T) for the gradient densities, plus
 * D1 int_T (u^2 - 1)^2 for Ginzburg-Landau (where W(F_T) = C1 |grad u|^2) */
static double density(const orc_problem *P, double F[3][3], int *bad);
static double element_energy(const orc_problem *P, const double *v, int64_t e, double vol,
                             double F[3][3], int *bad) {
  double E = vol * density(P, F, bad);
  if (P->kind == ORC_GL && !*bad) {
    double u[4];
    element_values(P, v, P->conn + e * (P->dim + 1), u);
    E += P->D1 * gl_potential(P->dim, vol, u);
    if (!isfinite(E)) { *bad = 1; return INFINITY; }
  }
  return E;
}

/* ---------------------------------------------------------------- F_T and densities */
/* F[j][m] = sum_l v[I(T,l)][j] * dphi_l[m]  (eq. Dv) */
static void element_F(const orc_problem *P, const double *v, const int32_t *T,
                      const double *dphi_e, double F[3][3]) {
  const int dim = P->dim, d = P->ncomp;
  for (int j = 0; j < 3; ++j)
    for (int m = 0; m < 3; ++m) F[j][m] = 0.0;
  for (int l = 0; l <= dim; ++l)
    for (int j = 0; j < d; ++j)
      for (int m = 0; m < dim; ++m)
        F[j][m] += v[(int64_t)T[l] * d + j] * dphi_e[l * dim + m];
}

/* Green-Lagrange strain E = (F^T F - I) / 2 */
static void green_strain(int dim, double F[3][3], double E[3][3]) {
  for (int j = 0; j < dim; ++j)
    for (int m = 0; m < dim; ++m) {
      double c = 0.0;
      for (int q = 0; q < dim; ++q) c += F[q][j] * F[q][m];
      E[j][m] = 0.5 * (c - (j == m ? 1.0 : 0.0));
    }
}

/* W(F); sets *bad when (Neo-Hookean) det F <= 0 or the value is not finite */
static double density(const orc_problem *P, double F[3][3], int *bad) {
  const int dim = P->dim;
  double W;
  if (P->kind == ORC_SVK) {
    double E[3][3], tr = 0.0, ee = 0.0;
    green_strain(dim, F, E);
    for (int j = 0; j < dim; ++j) {
      tr += E[j][j];
      for (int m = 0; m < dim; ++m) ee += E[j][m] * E[j][m];
    }
    W = P->C1 * ee + P->D1 * tr * tr;
  } else if (P->kind == ORC_NEOHOOKE) {
    double I1 = 0.0;
    for (int j = 0; j < dim; ++j)
      for (int m = 0; m < dim; ++m) I1 += F[j][m] * F[j][m];
    double det = det_mat(dim, F);
    if (!(det > 0.0)) { *bad = 1; return INFINITY; }
    W = P->C1 * (I1 - dim - 2.0 * log(det)) + P->D1 * (det - 1.0) * (det - 1.0);
  } else if (P->kind == ORC_GL) {
    double s = 0.0;
    for (int m = 0; m < dim; ++m) s += F[0][m] * F[0][m];
    W = P->C1 * s; /* the gradient part; the potential is added per element */
  } else if (P->kind == ORC_PLAPLACE_ORTHO) {
    W = 0.0;
    for (int m = 0; m < dim; ++m) W += pow(fabs(F[0][m]), P->p);
    W /= P->p;
  } else {
    double s = 0.0;
    for (int m = 0; m < dim; ++m) s += F[0][m] * F[0][m];
    W = pow(sqrt(s), P->p) / P->p;
  }
  if (!isfinite(W)) { *bad = 1; return INFINITY; }
  return W;
}

/* dW/dF (d x dim), Section 6.2 */
static void density_dF(const orc_problem *P, double F[3][3], double D[3][3], int *bad) {
  const int dim = P->dim;
  for (int j = 0; j < 3; ++j)
    for (int m = 0; m < 3; ++m) D[j][m] = 0.0;
  if (P->kind == ORC_SVK) {
    /* dW/dF = F S with S = dW/dE = 2 C1 E + 2 D1 (tr E) I (second Piola-Kirchhoff stress) */
    double E[3][3], S2[3][3], tr = 0.0;
    green_strain(dim, F, E);
    for (int j = 0; j < dim; ++j) tr += E[j][j];
    for (int j = 0; j < dim; ++j)
      for (int m = 0; m < dim; ++m)
        S2[j][m] = 2.0 * P->C1 * E[j][m] + (j == m ? 2.0 * P->D1 * tr : 0.0);
    for (int j = 0; j < dim; ++j)
      for (int m = 0; m < dim; ++m)
        for (int q = 0; q < dim; ++q) D[j][m] += F[j][q] * S2[q][m];
  } else if (P->kind == ORC_NEOHOOKE) {
    double det = det_mat(dim, F);
    if (!(det > 0.0)) { *bad = 1; return; }
    double cof[3][3];
    cofactor(dim, F, cof);
    for (int j = 0; j < dim; ++j)
      for (int m = 0; m < dim; ++m)
        D[j][m] = P->C1 * (2.0 * F[j][m] - (2.0 / det) * cof[j][m])
                + 2.0 * P->D1 * (det - 1.0) * cof[j][m];
  } else if (P->kind == ORC_GL) {
    for (int m = 0; m < dim; ++m) D[0][m] = 2.0 * P->C1 * F[0][m];
  } else if (P->kind == ORC_PLAPLACE_ORTHO) {
    /* d/dg_m |g_m|^p / p = |g_m|^(p-2) g_m, 0 at g_m = 0 (p > 1) */
    for (int m = 0; m < dim; ++m)
      D[0][m] = F[0][m] != 0.0 ? pow(fabs(F[0][m]), P->p - 2.0) * F[0][m] : 0.0;
  } else {
    double s = 0.0;
    for (int m = 0; m < dim; ++m) s += F[0][m] * F[0][m];
    double norm = sqrt(s);
    double scale = (norm > 0.0) ? pow(norm, P->p - 2.0) : 0.0;
    for (int m = 0; m < dim; ++m) D[0][m] = scale * F[0][m];
  }
  for (int j = 0; j < 3; ++j)
    for (int m = 0; m < 3; ++m)
      if (!isfinite(D[j][m])) *bad = 1;
}

/* ---------------------------------------------------------------- energy */
/* J_grad = sum_T |T| W(F_T) (eq. Denergy). v is the full nodal field [nn][d]. Returns the
 * number of bad elements (then *jgrad = +Inf). */
int64_t orc_energy(const orc_problem *P, const double *v, const double *vol, const double *dphi,
                   double *jgrad) {
  const int dim = P->dim, k = dim + 1;
  orc_acc acc = {0.0, 0.0};
  int64_t nbad = 0;
  for (int64_t e = 0; e < P->ne; ++e) {
    double F[3][3];
    element_F(P, v, P->conn + e * k, dphi + e * k * dim, F);
    int bad = 0;
    double E = element_energy(P, v, e, vol[e], F, &bad);
    if (bad) { ++nbad; continue; }
    acc_add(&acc, E);
  }
  *jgrad = nbad ? INFINITY : acc_result(&acc);
  return nbad;
}

/* Per-element densities W(F_T) (bad elements get +Inf; Ginzburg-Landau: the gradient part). */
void orc_densities(const orc_problem *P, const double *v, const double *dphi, double *W_out) {
  const int dim = P->dim, k = dim + 1;
  for (int64_t e = 0; e < P->ne; ++e) {
    double F[3][3];
    element_F(P, v, P->conn + e * k, dphi + e * k * dim, F);
    int bad = 0;
    W_out[e] = density(P, F, &bad);
  }
}

/* ---------------------------------------------------------------- b = M f */
void orc_load_vector(const orc_problem *P, const double *vol, const double *f, double *b) {
  const int dim = P->dim, k = dim + 1, d = P->ncomp;
  memset(b, 0, sizeof(double) * (size_t)P->nn * d);
  const double denom = (double)((dim + 1) * (dim + 2));
  for (int64_t e = 0; e < P->ne; ++e) {
    const int32_t *T = P->conn + e * k;
    for (int a = 0; a < k; ++a)
      for (int c = 0; c < k; ++c) {
        double Mac = vol[e] * (a == c ? 2.0 : 1.0) / denom;
        for (int j = 0; j < d; ++j)
          b[(int64_t)T[a] * d + j] += Mac * f[(int64_t)T[c] * d + j];
      }
  }
}

/* compensated dot product sum_n x_n y_n */
double orc_dot(int64_t n, const double *x, const double *y) {
  orc_acc acc = {0.0, 0.0};
  for (int64_t i = 0; i < n; ++i) acc_add(&acc, x[i] * y[i]);
  return acc_result(&acc);
}

/* ---------------------------------------------------------------- exact gradient */
/* g[i][j] = sum_{T containing i} |T| sum_m dW/dF_jm(F_T) dphi_{T,l(i)}[m], all nodes, no load
 * term. Element-loop scatter. Returns the number of bad elements. */
int64_t orc_grad_exact(const orc_problem *P, const double *v, const double *vol,
                       const double *dphi, double *g) {
  const int dim = P->dim, k = dim + 1, d = P->ncomp;
  memset(g, 0, sizeof(double) * (size_t)P->nn * d);
  int64_t nbad = 0;
  for (int64_t e = 0; e < P->ne; ++e) {
    const int32_t *T = P->conn + e * k;
    const double *dp = dphi + e * k * dim;
    double F[3][3], D[3][3];
    element_F(P, v, T, dp, F);
    int bad = 0;
    density_dF(P, F, D, &bad);
    if (bad) { ++nbad; continue; }
    for (int l = 0; l < k; ++l)
      for (int j = 0; j < d; ++j) {
        double s = 0.0;
        for (int m = 0; m < dim; ++m) s += D[j][m] * dp[l * dim + m];
        g[(int64_t)T[l] * d + j] += vol[e] * s;
      }
    if (P->kind == ORC_GL) {
      double u[4];
      element_values(P, v, T, u);
      for (int l = 0; l < k; ++l) g[T[l]] += P->D1 * gl_potential_du(dim, vol[e], u, l);
    }
  }
  return nbad;
}

/* ---------------------------------------------------------------- nodal patches */
/* patch_ptr[nn+1], patch_elem[(dim+1) ne]: elements containing node i in ascending order. */
void orc_patches(const orc_problem *P, int64_t *patch_ptr, int64_t *patch_elem) {
  const int k = P->dim + 1;
  memset(patch_ptr, 0, sizeof(int64_t) * (size_t)(P->nn + 1));
  for (int64_t e = 0; e < P->ne; ++e)
    for (int l = 0; l < k; ++l) patch_ptr[P->conn[e * k + l] + 1] += 1;
  for (int64_t i = 0; i < P->nn; ++i) patch_ptr[i + 1] += patch_ptr[i];
  int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)(P->nn > 0 ? P->nn : 1));
  for (int64_t i = 0; i < P->nn; ++i) fill[i] = patch_ptr[i];
  for (int64_t e = 0; e < P->ne; ++e)
    for (int l = 0; l < k; ++l) {
      int32_t i = P->conn[e * k + l];
      patch_elem[fill[i]++] = e;
    }
  free(fill);
}

/* ---------------------------------------------------------------- patch central differences */
/* |W|_abs: the sum of the magnitudes of the density's terms (rounding scale of W) */
static double density_abs(const orc_problem *P, double F[3][3], double W) {
  if (P->kind == ORC_SVK) {
    /* E_jm = ((F^T F)_jm - delta_jm) / 2 carries a rounding of about dim u ((|F|^T |F|)_jm
     * + delta_jm) / 2; W moves by |dW/dE_jm| = |S_jm| times that */
    const int dim = P->dim;
    double E[3][3], tr = 0.0, sc = 0.0;
    green_strain(dim, F, E);
    for (int j = 0; j < dim; ++j) tr += E[j][j];
    for (int j = 0; j < dim; ++j)
      for (int m = 0; m < dim; ++m) {
        double c = 0.0;
        for (int q = 0; q < dim; ++q) c += fabs(F[q][j]) * fabs(F[q][m]);
        const double S = fabs(2.0 * P->C1 * E[j][m] + (j == m ? 2.0 * P->D1 * tr : 0.0));
        sc += S * 0.5 * dim * (c + (j == m ? 1.0 : 0.0));
      }
    return fabs(W) + sc;
  }
  if (P->kind == ORC_GL) return fabs(W); /* the potential's scale is added by the caller */
  if (P->kind != ORC_NEOHOOKE) return fabs(W);
  const int dim = P->dim;
  double I1 = 0.0;
  for (int j = 0; j < dim; ++j)
    for (int m = 0; m < dim; ++m) I1 += F[j][m] * F[j][m];
  double det = det_mat(dim, F);
  return P->C1 * (I1 + dim + 2.0 * fabs(log(det))) + P->D1 * (det - 1.0) * (det - 1.0);
}

/* |T| |W|_abs of element e, plus (Ginzburg-Landau) the potential's scale
 * D1 (int u^4 + 2 int u^2 + |T|) */
static double element_energy_abs(const orc_problem *P, const double *v, int64_t e, double vol,
                                 double F[3][3]) {
  int bad = 0;
  const double W = density(P, F, &bad);
  double A = vol * density_abs(P, F, W);
  if (P->kind == ORC_GL) {
    double u[4];
    element_values(P, v, P->conn + e * (P->dim + 1), u);
    A += P->D1 * (int_power(P->dim, vol, u, 4, -1) + 2.0 * int_power(P->dim, vol, u, 2, -1) + vol);
  }
  return A;
}

/* For every DOF listed in dofs[0..ndofs) (global DOF index n = d*i + j), with e_n the n-th unit
 * vector:  g = [ sum_{T in T^i} |T| W(F_T(v + eps e_n)) - sum_{T in T^i} |T| W(F_T(v - eps e_n)) ]
 *              / (2 eps).
 * F_T(v +- eps e_n) is recomputed from the perturbed nodal values by eq. (Dv); the two patch
 * sums are accumulated separately (Neumaier, ascending element order) and then differenced.
 * Optional rounding scales per DOF: cond[q] = sum_T |T| (|W+|_abs + |W-|_abs) and
 * gabs[q] = sum_T |T| |W+ - W-| / (2 eps).
 * v is modified during the call and restored. Returns the number of bad evaluations. */
int64_t orc_grad_patch_fd(const orc_problem *P, double *v, const double *vol,
                          const double *dphi, const int64_t *patch_ptr,
                          const int64_t *patch_elem, double eps, int64_t ndofs,
                          const int64_t *dofs, double *g, double *cond, double *gabs) {
  const int dim = P->dim, k = dim + 1;
  const int d = P->ncomp;
  int64_t nbad = 0;
  for (int64_t q = 0; q < ndofs; ++q) {
    const int64_t n = dofs[q];
    const int64_t i = n / d;
    const double v0 = v[n];
    orc_acc Sp = {0.0, 0.0}, Sm = {0.0, 0.0};
    double C = 0.0, A = 0.0;
    for (int64_t t = patch_ptr[i]; t < patch_ptr[i + 1]; ++t) {
      const int64_t e = patch_elem[t];
      double Fp[3][3], Fm[3][3];
      int bad = 0;
      v[n] = v0 + eps;
      element_F(P, v, P->conn + e * k, dphi + e * k * dim, Fp);
      const double Ep = element_energy(P, v, e, vol[e], Fp, &bad);
      const double Cp = bad ? 0.0 : element_energy_abs(P, v, e, vol[e], Fp);
      v[n] = v0 - eps;
      element_F(P, v, P->conn + e * k, dphi + e * k * dim, Fm);
      const double Em = element_energy(P, v, e, vol[e], Fm, &bad);
      const double Cm = bad ? 0.0 : element_energy_abs(P, v, e, vol[e], Fm);
      v[n] = v0;
      if (bad) { ++nbad; continue; }
      acc_add(&Sp, Ep);
      acc_add(&Sm, Em);
      C += Cp + Cm;
      A += fabs(Ep - Em) / (2.0 * eps);
    }
    g[q] = (acc_result(&Sp) - acc_result(&Sm)) / (2.0 * eps);
    if (cond) cond[q] = C;
    if (gabs) gabs[q] = A;
  }
  return nbad;
}

/* Fourth-order patch central differences, the higher-accuracy scheme Section 6.1 says the
 * central-difference code generalises to: with S(h) = sum_{T in T^i} |T| W(F_T(v + h e_n)),
 *   g = [8 (S(eps) - S(-eps)) - (S(2 eps) - S(-2 eps))] / (12 eps),
 * each S a separate Neumaier sum in ascending element order, F_T recomputed by eq. (Dv) from
 * the perturbed nodal value. Rounding scales per DOF (optional):
 *   cond[q] = sum_T |T| (8 (|W(eps)|_abs + |W(-eps)|_abs) + |W(2eps)|_abs + |W(-2eps)|_abs) / 6,
 *   gabs[q] = sum_T |T| (8 |W(eps) - W(-eps)| + 2 |W(2eps) - W(-2eps)|) / (12 eps).
 * v is modified during the call and restored. Returns the number of bad evaluations. */
int64_t orc_grad_patch_fd4(const orc_problem *P, double *v, const double *vol,
                           const double *dphi, const int64_t *patch_ptr,
                           const int64_t *patch_elem, double eps, int64_t ndofs,
                           const int64_t *dofs, double *g, double *cond, double *gabs) {
  const int dim = P->dim, k = dim + 1;
  const int d = P->ncomp;
  const double steps[4] = {eps, -eps, 2.0 * eps, -2.0 * eps};
  int64_t nbad = 0;
  for (int64_t q = 0; q < ndofs; ++q) {
    const int64_t n = dofs[q];
    const int64_t i = n / d;
    const double v0 = v[n];
    orc_acc S[4] = {{0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}};
    double C = 0.0, A = 0.0;
    for (int64_t t = patch_ptr[i]; t < patch_ptr[i + 1]; ++t) {
      const int64_t e = patch_elem[t];
      double W[4], Wabs[4]; /* element energies |T| W and their scales at the four steps */
      int bad = 0;
      for (int h = 0; h < 4; ++h) {
        double F[3][3];
        v[n] = v0 + steps[h];
        element_F(P, v, P->conn + e * k, dphi + e * k * dim, F);
        W[h] = element_energy(P, v, e, vol[e], F, &bad);
        Wabs[h] = bad ? 0.0 : element_energy_abs(P, v, e, vol[e], F);
      }
      v[n] = v0;
      if (bad) { ++nbad; continue; }
      for (int h = 0; h < 4; ++h) acc_add(&S[h], W[h]);
      C += (8.0 * (Wabs[0] + Wabs[1]) + Wabs[2] + Wabs[3]) / 6.0;
      A += (8.0 * fabs(W[0] - W[1]) + 2.0 * fabs(W[2] - W[3])) / (12.0 * eps);
    }
    const double d1 = acc_result(&S[0]) - acc_result(&S[1]);
    const double d2 = acc_result(&S[2]) - acc_result(&S[3]);
    g[q] = (8.0 * d1 - d2) / (12.0 * eps);
    if (cond) cond[q] = C;
    if (gabs) gabs[q] = A;
  }
  return nbad;
}
