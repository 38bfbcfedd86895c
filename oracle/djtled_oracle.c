/*
 * DJ-TLED oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, double-precision CPU implementation of the direct Jacobian
 * total Lagrangian explicit dynamics (DJ-TLED) method of Zhang, "A direct
 * Jacobian total Lagrangian explicit dynamics finite element algorithm for
 * real-time simulation of hyperelastic materials" (arXiv 2106.14189).
 *
 * Only the tests, the smoke check and the CPU-baseline leg of the benchmark
 * may load this library.  The GPU library shares no code, header, table or
 * helper with it.  Every function follows the paper in its own order and
 * notation: the element force is Table 3 evaluated literally, with the
 * constants of Algorithm 1 (pre-computation steps 1-4) built from the G
 * matrices of Appendix B and the vectors of Appendix C.  An independent
 * classical TLED force (Eq. 4 with the stress of Eq. 54 and its transversely
 * isotropic analogue derived from Eq. 7) is provided as a cross-check.
 *
 * Readings of passages the paper leaves open (each is also listed in the
 * design notes of the repository):
 *  - Eq. 11 is read as  tJ = 0J + Hxi * Ue  with Ue the n_e x 3 matrix of
 *    nodal displacements, so that row i of J is d x / d xi_i as in Eq. 3.
 *  - T4 uses volume coordinates h = (1-xi-eta-zeta, xi, eta, zeta) (Sec. 7)
 *    and 0V = det(0J)/6; H8 is evaluated at the centre (one-point Gauss,
 *    Sec. 1) with 0V = 8 det(0J).
 *  - H8 hourglass control, which the paper cites but does not state, is the
 *    Flanagan-Belytschko stiffness form written in the reference
 *    configuration: gamma_a = Gamma_a - sum_i (Gamma_a . X_i) dh/dX_i,
 *    f = k sum_a gamma_a (gamma_a^T U), k = kappa_hg (kappa + 4 mu / 3)
 *    0V sum |dh/dX|^2 / 8.  PARITY UNPINNED against the paper (no numbers
 *    are printed); pinned internally by the energy gradient and by its null
 *    space containing every affine field.
 *  - Lumped mass m_i = sum_e rho 0V_e / n_e; central differences with
 *    lumped mass-proportional damping D = alpha M (Eq. 13), textbook form.
 *  - Eq. 14: L_e = 3V / A_max (T4, the smallest altitude) or, for the
 *    one-point H8, L_e = 1 / sqrt(2 sum |dh/dX|^2) (the Flanagan-Belytschko
 *    eigenvalue bound; h / sqrt(3) for a cube); c = sqrt((kappa + 4 mu_0 / 3 +
 *    4 (eta_a + eta_b)) / rho), with mu_0 the initial shear modulus (mu, or
 *    2 (C10 + C01) for Mooney-Rivlin) and the fibre moduli of the model (0
 *    for the isotropic models).
 *  - Mooney-Rivlin: C10 = mu / 2 from E and nu (as Sec. 5.1 does), C01 given
 *    per element; kappa from E and nu.  Orthotropic: eta_b = ratio_b * mu.
 *  - Average nodal pressure (named in Sec. 7 against volumetric locking, not
 *    defined there): the volumetric energy sum_n V_n kappa_n (J_n - 1)^2 / 2
 *    on 1/n_e-weighted nodal volume averages; ora_forces_anp is its gradient.
 *  - Displacement boundary conditions overwrite the constrained components
 *    after each update with s(t) * target; s is 1, linear or the quintic
 *    smoothstep tau^3 (10 - 15 tau + 6 tau^2).
 *  - Dynamic relaxation residual r = |(F - R)_free|_2 / |F_constrained|_2,
 *    checked every check_every steps once the load ramp has completed.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORA_NH 0
#define ORA_TI 1
#define ORA_OT 2
#define ORA_MR 3

/* ------------------------------------------------------------------ */
/* 3x3 matrix helpers (row-major)                                       */
/* ------------------------------------------------------------------ */
static double det3(const double a[9]) {
    return a[0] * (a[4] * a[8] - a[5] * a[7]) - a[1] * (a[3] * a[8] - a[5] * a[6]) +
           a[2] * (a[3] * a[7] - a[4] * a[6]);
}

static int inv3(const double a[9], double r[9]) {
    double d = det3(a);
    if (d == 0.0) return -1;
    r[0] = (a[4] * a[8] - a[5] * a[7]) / d;
    r[1] = (a[2] * a[7] - a[1] * a[8]) / d;
    r[2] = (a[1] * a[5] - a[2] * a[4]) / d;
    r[3] = (a[5] * a[6] - a[3] * a[8]) / d;
    r[4] = (a[0] * a[8] - a[2] * a[6]) / d;
    r[5] = (a[2] * a[3] - a[0] * a[5]) / d;
    r[6] = (a[3] * a[7] - a[4] * a[6]) / d;
    r[7] = (a[1] * a[6] - a[0] * a[7]) / d;
    r[8] = (a[0] * a[4] - a[1] * a[3]) / d;
    return 0;
}

static void mul3(const double a[9], const double b[9], double c[9]) {
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            double s = 0.0;
            for (int k = 0; k < 3; k++) s += a[3 * i + k] * b[3 * k + j];
            c[3 * i + j] = s;
        }
}

static void tr3(const double a[9], double t[9]) {
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) t[3 * j + i] = a[3 * i + j];
}

static double trace3(const double a[9]) { return a[0] + a[4] + a[8]; }

/* ------------------------------------------------------------------ */
/* Shape-function natural derivatives H_xi (3 x n_e), Sec. 2.2 / Eq. 6   */
/* ------------------------------------------------------------------ */
/* H8 node order: (-,-,-) (+,-,-) (+,+,-) (-,+,-) (-,-,+) (+,-,+) (+,+,+) (-,+,+) */
static const int H8_NAT[8][3] = {{-1, -1, -1}, {1, -1, -1}, {1, 1, -1}, {-1, 1, -1},
                                  {-1, -1, 1},  {1, -1, 1},  {1, 1, 1},  {-1, 1, 1}};

static void shape_derivs(int ne, double H[3][8]) {
    memset(H, 0, sizeof(double) * 24);
    if (ne == 4) {
        /* h = (1 - xi - eta - zeta, xi, eta, zeta) */
        for (int i = 0; i < 3; i++) {
            H[i][0] = -1.0;
            H[i][i + 1] = 1.0;
        }
    } else {
        /* h_a = (1 + xi_a xi)(1 + eta_a eta)(1 + zeta_a zeta) / 8 at xi = 0 */
        for (int a = 0; a < 8; a++)
            for (int i = 0; i < 3; i++) H[i][a] = H8_NAT[a][i] / 8.0;
    }
}

/* Flanagan-Belytschko hourglass base vectors Gamma_alpha (xi-eta, eta-zeta,
   zeta-xi, xi-eta-zeta products of the nodal natural coordinates). */
static void hourglass_base(double G[4][8]) {
    for (int a = 0; a < 8; a++) {
        double x = H8_NAT[a][0], y = H8_NAT[a][1], z = H8_NAT[a][2];
        G[0][a] = x * y;
        G[1][a] = y * z;
        G[2][a] = z * x;
        G[3][a] = x * y * z;
    }
}

/* ------------------------------------------------------------------ */
/* Context                                                               */
/* ------------------------------------------------------------------ */
typedef struct {
    int ne, n_nodes, n_elems, model;
    double rho, hg_kappa;
    double H[3][8];
    double *X;                /* n_nodes x 3 */
    int *conn;                /* n_elems x ne */
    double *mu, *kappa, *eta; /* per element */
    double *fibre;            /* per element unit fibre direction a (TI, OT) */
    double *eta_b, *fibre_b;  /* OT: second fibre modulus and unit direction b */
    double *c01;              /* MR: C01 (C10 = mu / 2) */
    /* Algorithm 1, pre-computation, per element */
    double *J0, *detJ0, *V;   /* step 1 */
    double *G;                /* step 2: six 3x3 matrices, Appendix B */
    double *m1, *m4, *m6;     /* step 3: Appendix C, Eqs. C.1, C.2, C.3 */
    double *M2;               /* step 3: Eq. C.5 (6 x 6) */
    double *I1m, *I4m, *I6m;  /* step 4: Eqs. 37, 45, 46 */
    double *I2m;              /* step 4: Eqs. 40-41, six 3x3 matrices */
    double *dhdX;             /* Eq. 6 (TLED route, hourglass) : 3 x ne */
    double *gam, *khg;        /* hourglass shape vectors (4 x 8) and stiffness */
    double *mass;             /* lumped nodal mass */
    double dt_crit;
    /* all-cores timing build only: node -> (element, local node) incidences in
       ascending element order, and a per-incidence force array */
    int *inc_off, *inc;
    double *fe;
} ora_ctx;

void ora_destroy(ora_ctx *c) {
    if (!c) return;
    free(c->X); free(c->conn); free(c->mu); free(c->kappa); free(c->eta); free(c->fibre);
    free(c->eta_b); free(c->fibre_b); free(c->c01); free(c->m6); free(c->M2); free(c->I6m); free(c->I2m);
    free(c->J0); free(c->detJ0); free(c->V); free(c->G); free(c->m1); free(c->m4);
    free(c->I1m); free(c->I4m); free(c->dhdX); free(c->gam); free(c->khg); free(c->mass);
    free(c->inc_off); free(c->inc); free(c->fe);
    free(c);
}

/* Material constants from Young's modulus and Poisson's ratio:
   mu = E / (2 (1 + nu)), kappa = E / (3 (1 - 2 nu)) (worked values in Sec. 5.1 and Sec. 6). */
void ora_lame(double E, double nu, double *mu, double *kappa) {
    *mu = E / (2.0 * (1.0 + nu));
    *kappa = E / (3.0 * (1.0 - 2.0 * nu));
}

/* Appendix B: G_k = 0J^{-1} E_k 0J^{-T}, with E_k the symmetric unit patterns
   of Eq. 16 in the order 11, 22, 33, 12, 13, 23. */
static void g_matrices(const double J0inv[9], double G[6][9]) {
    static const int P[6][2] = {{0, 0}, {1, 1}, {2, 2}, {0, 1}, {0, 2}, {1, 2}};
    double JinvT[9];
    tr3(J0inv, JinvT);
    for (int k = 0; k < 6; k++) {
        double E[9] = {0}, t[9];
        E[3 * P[k][0] + P[k][1]] = 1.0;
        E[3 * P[k][1] + P[k][0]] = 1.0;
        mul3(J0inv, E, t);
        mul3(t, JinvT, G[k]);
    }
}

/* Eq. 18: ghat = [g11 g22 g33 g12 g13 g23] of tJ tJ^T (Eq. 17). */
static void ghat_of(const double tJ[9], double g[6]) {
    double tJT[9], gg[9];
    tr3(tJ, tJT);
    mul3(tJ, tJT, gg);
    g[0] = gg[0]; g[1] = gg[4]; g[2] = gg[8];
    g[3] = gg[1]; g[4] = gg[2]; g[5] = gg[5];
}

static double face_area_tri(const double *p, const double *q, const double *r) {
    double u[3], v[3], w[3];
    for (int i = 0; i < 3; i++) { u[i] = q[i] - p[i]; v[i] = r[i] - p[i]; }
    w[0] = u[1] * v[2] - u[2] * v[1];
    w[1] = u[2] * v[0] - u[0] * v[2];
    w[2] = u[0] * v[1] - u[1] * v[0];
    return 0.5 * sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
}

/* Characteristic length of Eq. 14 for one element (reading stated in the header). */
static double char_length(const ora_ctx *c, int e) {
    const int *cn = c->conn + (size_t)e * c->ne;
    double amax = 0.0;
    if (c->ne == 4) {
        static const int F[4][3] = {{1, 2, 3}, {0, 2, 3}, {0, 1, 3}, {0, 1, 2}};
        for (int f = 0; f < 4; f++) {
            double a = face_area_tri(c->X + 3 * cn[F[f][0]], c->X + 3 * cn[F[f][1]], c->X + 3 * cn[F[f][2]]);
            if (a > amax) amax = a;
        }
        return 3.0 * c->V[e] / amax;
    } else {
        /* one-point hexahedron: the Flanagan-Belytschko maximum-eigenvalue
           bound gives L_e = 1 / sqrt(2 sum_{a,i} (dh_a/dX_i)^2)  (h / sqrt(3) for a cube) */
        const double *B = c->dhdX + (size_t)24 * e;
        double sb = 0.0;
        for (int i = 0; i < 24; i++) sb += B[i] * B[i];
        return 1.0 / sqrt(2.0 * sb);
    }
}

/*
 * Build the oracle context: copies the mesh and runs Algorithm 1's
 * pre-computation literally for every element.
 *   ne      4 (T4) or 8 (H8)
 *   X       n_nodes x 3 reference coordinates
 *   conn    n_elems x ne node indices
 *   model   ORA_NH, ORA_TI, ORA_OT or ORA_MR (Table 3 rows)
 *   E, nu   per-element Young's modulus and Poisson's ratio
 *   eta_ratio, fibre   TI, OT: eta_a = eta_ratio * mu, fibre a (n_elems x 3)
 *   eta_b_ratio, fibre_b   OT: eta_b = eta_b_ratio * mu, fibre b (n_elems x 3)
 *   c01     MR: C01 per element (C10 = mu / 2)
 * On failure returns NULL and sets *err: -1 argument, -2 bad mesh (index out
 * of range or det(0J) <= 0).
 */
ora_ctx *ora_create(int ne, int n_nodes, int n_elems, const double *X, const int *conn, int model,
                    const double *E, const double *nu, const double *eta_ratio, const double *fibre,
                    const double *eta_b_ratio, const double *fibre_b, const double *c01,
                    double rho, double hg_kappa, int *err) {
    *err = 0;
    const int fib_a = (model == ORA_TI || model == ORA_OT), fib_b = (model == ORA_OT);
    if ((ne != 4 && ne != 8) || n_nodes <= 0 || n_elems <= 0 || model < ORA_NH || model > ORA_MR ||
        (fib_a && (!eta_ratio || !fibre)) || (fib_b && (!eta_b_ratio || !fibre_b)) ||
        (model == ORA_MR && !c01) || rho <= 0.0) {
        *err = -1;
        return NULL;
    }
    ora_ctx *c = (ora_ctx *)calloc(1, sizeof(ora_ctx));
    c->ne = ne; c->n_nodes = n_nodes; c->n_elems = n_elems; c->model = model;
    c->rho = rho; c->hg_kappa = hg_kappa;
    shape_derivs(ne, c->H);
    size_t E_ = (size_t)n_elems;
    c->X = (double *)malloc(sizeof(double) * 3 * (size_t)n_nodes);
    memcpy(c->X, X, sizeof(double) * 3 * (size_t)n_nodes);
    c->conn = (int *)malloc(sizeof(int) * ne * E_);
    memcpy(c->conn, conn, sizeof(int) * ne * E_);
    c->mu = (double *)malloc(sizeof(double) * E_);
    c->kappa = (double *)malloc(sizeof(double) * E_);
    c->eta = (double *)calloc(E_, sizeof(double));
    c->fibre = (double *)calloc(3 * E_, sizeof(double));
    c->eta_b = (double *)calloc(E_, sizeof(double));
    c->fibre_b = (double *)calloc(3 * E_, sizeof(double));
    c->c01 = (double *)calloc(E_, sizeof(double));
    c->m6 = (double *)calloc(6 * E_, sizeof(double));
    c->M2 = (double *)calloc(36 * E_, sizeof(double));
    c->I6m = (double *)calloc(9 * E_, sizeof(double));
    c->I2m = (double *)calloc(54 * E_, sizeof(double));
    c->J0 = (double *)malloc(sizeof(double) * 9 * E_);
    c->detJ0 = (double *)malloc(sizeof(double) * E_);
    c->V = (double *)malloc(sizeof(double) * E_);
    c->G = (double *)malloc(sizeof(double) * 54 * E_);
    c->m1 = (double *)malloc(sizeof(double) * 6 * E_);
    c->m4 = (double *)calloc(6 * E_, sizeof(double));
    c->I1m = (double *)malloc(sizeof(double) * 9 * E_);
    c->I4m = (double *)calloc(9 * E_, sizeof(double));
    c->dhdX = (double *)malloc(sizeof(double) * 3 * ne * E_);
    c->gam = (double *)calloc(32 * E_, sizeof(double));
    c->khg = (double *)calloc(E_, sizeof(double));
    c->mass = (double *)calloc((size_t)n_nodes, sizeof(double));

    for (size_t i = 0; i < (size_t)ne * E_; i++)
        if (conn[i] < 0 || conn[i] >= n_nodes) { *err = -2; ora_destroy(c); return NULL; }

    double Gam[4][8];
    hourglass_base(Gam);
    double dtc = INFINITY;
    for (size_t e = 0; e < E_; e++) {
        const int *cn = conn + e * ne;
        ora_lame(E[e], nu[e], &c->mu[e], &c->kappa[e]);
        if (fib_a) {
            c->eta[e] = eta_ratio[e] * c->mu[e];
            double n = sqrt(fibre[3 * e] * fibre[3 * e] + fibre[3 * e + 1] * fibre[3 * e + 1] +
                            fibre[3 * e + 2] * fibre[3 * e + 2]);
            if (!(n > 0.0)) { *err = -1; ora_destroy(c); return NULL; }
            for (int k = 0; k < 3; k++) c->fibre[3 * e + k] = fibre[3 * e + k] / n;
        }
        if (fib_b) {
            c->eta_b[e] = eta_b_ratio[e] * c->mu[e];
            double n = sqrt(fibre_b[3 * e] * fibre_b[3 * e] + fibre_b[3 * e + 1] * fibre_b[3 * e + 1] +
                            fibre_b[3 * e + 2] * fibre_b[3 * e + 2]);
            if (!(n > 0.0)) { *err = -1; ora_destroy(c); return NULL; }
            for (int k = 0; k < 3; k++) c->fibre_b[3 * e + k] = fibre_b[3 * e + k] / n;
        }
        if (model == ORA_MR) c->c01[e] = c01[e];
        /* Step 1: 0J = H_xi X_e (Eq. 3), det(0J), 0V, A = a a^T */
        double *J0 = c->J0 + 9 * e;
        for (int i = 0; i < 3; i++)
            for (int k = 0; k < 3; k++) {
                double s = 0.0;
                for (int a = 0; a < ne; a++) s += c->H[i][a] * X[3 * cn[a] + k];
                J0[3 * i + k] = s;
            }
        double d = det3(J0);
        if (!(d > 0.0)) { *err = -2; ora_destroy(c); return NULL; }
        c->detJ0[e] = d;
        c->V[e] = (ne == 4) ? d / 6.0 : 8.0 * d;
        double J0inv[9], J0invT[9];
        inv3(J0, J0inv);
        tr3(J0inv, J0invT);
        double A[9], Bm[9];
        const double *av = c->fibre + 3 * e, *bv = c->fibre_b + 3 * e;
        for (int i = 0; i < 3; i++)
            for (int j = 0; j < 3; j++) {
                A[3 * i + j] = av[i] * av[j];
                Bm[3 * i + j] = bv[i] * bv[j];
            }
        /* Step 2: G matrices (Appendix B) */
        double (*G)[9] = (double (*)[9])(c->G + 54 * e);
        g_matrices(J0inv, G);
        /* Step 3: m1 = [tr G_k] (C.1), m4 = [tr(A G_k)] (C.2), m6 = [tr(B G_k)] (C.3),
           W = [tr(G_k^T G_l)] (C.4) and M2 = (m1 m1^T - W) / 2 (C.5) */
        for (int k = 0; k < 6; k++) {
            c->m1[6 * e + k] = trace3(G[k]);
            if (fib_a) {
                double AG[9];
                mul3(A, G[k], AG);
                c->m4[6 * e + k] = trace3(AG);
            }
            if (fib_b) {
                double BG[9];
                mul3(Bm, G[k], BG);
                c->m6[6 * e + k] = trace3(BG);
            }
        }
        if (model == ORA_MR)
            for (int k = 0; k < 6; k++)
                for (int l = 0; l < 6; l++) {
                    double GT[9], P[9];
                    tr3(G[k], GT);
                    mul3(GT, G[l], P);
                    c->M2[36 * e + 6 * k + l] = 0.5 * (c->m1[6 * e + k] * c->m1[6 * e + l] - trace3(P));
                }
        /* Step 4: I1m = 2 0V 0J^{-T} 0J^{-1} (Eq. 37), I4m = 2 0V 0J^{-T} A 0J^{-1} (Eq. 45),
           I6m = 2 0V 0J^{-T} B 0J^{-1} (Eq. 46), I2,k = 2 0V 0J^{-T} (tr(G_k) I - G_k) 0J^{-1} (Eq. 41) */
        double t[9], t2[9];
        mul3(J0invT, J0inv, t);
        for (int i = 0; i < 9; i++) c->I1m[9 * e + i] = 2.0 * c->V[e] * t[i];
        if (fib_a) {
            mul3(J0invT, A, t);
            mul3(t, J0inv, t2);
            for (int i = 0; i < 9; i++) c->I4m[9 * e + i] = 2.0 * c->V[e] * t2[i];
        }
        if (fib_b) {
            mul3(J0invT, Bm, t);
            mul3(t, J0inv, t2);
            for (int i = 0; i < 9; i++) c->I6m[9 * e + i] = 2.0 * c->V[e] * t2[i];
        }
        if (model == ORA_MR)
            for (int k = 0; k < 6; k++) {
                double Q[9];
                const double tg = trace3(G[k]);
                for (int i = 0; i < 9; i++) Q[i] = -G[k][i];
                Q[0] += tg; Q[4] += tg; Q[8] += tg;
                mul3(J0invT, Q, t);
                mul3(t, J0inv, t2);
                for (int i = 0; i < 9; i++) c->I2m[54 * e + 9 * k + i] = 2.0 * c->V[e] * t2[i];
            }
        /* Eq. 6: 0B = dh/dX = 0J^{-1} H_xi */
        double *B = c->dhdX + (size_t)3 * ne * e;
        for (int i = 0; i < 3; i++)
            for (int a = 0; a < ne; a++) {
                double s = 0.0;
                for (int k = 0; k < 3; k++) s += J0inv[3 * i + k] * c->H[k][a];
                B[ne * i + a] = s;
            }
        /* Hourglass shape vectors and stiffness (H8 only; reading stated above) */
        if (ne == 8) {
            double sb = 0.0;
            for (int i = 0; i < 3 * ne; i++) sb += B[i] * B[i];
            c->khg[e] = hg_kappa * (c->kappa[e] + 4.0 * (c->mu[e] + 2.0 * c->c01[e]) / 3.0) * c->V[e] * sb / 8.0;
            for (int al = 0; al < 4; al++) {
                double gx[3] = {0, 0, 0};
                for (int b = 0; b < 8; b++)
                    for (int k = 0; k < 3; k++) gx[k] += Gam[al][b] * (X[3 * cn[b] + k] - X[3 * cn[0] + k]);
                for (int a = 0; a < 8; a++) {
                    double s = Gam[al][a];
                    for (int k = 0; k < 3; k++) s -= gx[k] * B[ne * k + a];
                    c->gam[32 * e + 8 * al + a] = s;
                }
            }
        }
        /* lumped mass (each node gets rho 0V / n_e) */
        for (int a = 0; a < ne; a++) c->mass[cn[a]] += c->rho * c->V[e] / ne;
    }
    /* Eq. 14: critical time step */
    for (size_t e = 0; e < E_; e++) {
        double cw = sqrt((c->kappa[e] + 4.0 * (c->mu[e] + 2.0 * c->c01[e]) / 3.0 + 4.0 * (c->eta[e] + c->eta_b[e])) /
                         c->rho);
        double L = char_length(c, (int)e);
        if (L / cw < dtc) dtc = L / cw;
    }
    c->dt_crit = dtc;
#ifdef _OPENMP
    /* incidence lists for the all-cores assembly (see ora_forces) */
    c->inc_off = (int *)calloc((size_t)c->n_nodes + 1, sizeof(int));
    c->inc = (int *)malloc(sizeof(int) * E_ * ne);
    c->fe = (double *)malloc(sizeof(double) * 3 * E_ * ne);
    for (size_t q = 0; q < E_ * (size_t)ne; q++) c->inc_off[c->conn[q] + 1]++;
    for (int n = 0; n < c->n_nodes; n++) c->inc_off[n + 1] += c->inc_off[n];
    {
        int *fill = (int *)malloc(sizeof(int) * ((size_t)c->n_nodes + 1));
        memcpy(fill, c->inc_off, sizeof(int) * ((size_t)c->n_nodes + 1));
        for (size_t q = 0; q < E_ * (size_t)ne; q++) c->inc[fill[c->conn[q]]++] = (int)q;
        free(fill);
    }
#endif
    return c;
}

/* Threads the element loop uses (1 unless built with OpenMP). */
int ora_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

double ora_dt_crit(const ora_ctx *c) { return c->dt_crit; }
void ora_mass(const ora_ctx *c, double *m) { memcpy(m, c->mass, sizeof(double) * c->n_nodes); }

/*
 * Per-element constants for inspection by tests.  out receives, in order:
 * J0 (9), detJ0 (1), V (1), I1m (9), m1 (6), I4m (9), m4 (6), dhdX (3 x ne),
 * mu, kappa, eta (3), hourglass k (1), gamma (32).
 */
int ora_element_constants(const ora_ctx *c, int e, double *out) {
    if (e < 0 || e >= c->n_elems) return -1;
    double *o = out;
    memcpy(o, c->J0 + 9 * e, 9 * sizeof(double)); o += 9;
    *o++ = c->detJ0[e];
    *o++ = c->V[e];
    memcpy(o, c->I1m + 9 * e, 9 * sizeof(double)); o += 9;
    memcpy(o, c->m1 + 6 * e, 6 * sizeof(double)); o += 6;
    memcpy(o, c->I4m + 9 * e, 9 * sizeof(double)); o += 9;
    memcpy(o, c->m4 + 6 * e, 6 * sizeof(double)); o += 6;
    memcpy(o, c->dhdX + (size_t)3 * c->ne * e, 3 * c->ne * sizeof(double)); o += 3 * c->ne;
    *o++ = c->mu[e]; *o++ = c->kappa[e]; *o++ = c->eta[e];
    *o++ = c->khg[e];
    memcpy(o, c->gam + 32 * e, 32 * sizeof(double));
    return 0;
}

/* Element displacement matrix Ue (n_e x 3) */
static void gather_u(const ora_ctx *c, int e, const double *u, double Ue[8][3]) {
    const int *cn = c->conn + (size_t)e * c->ne;
    for (int a = 0; a < c->ne; a++)
        for (int k = 0; k < 3; k++) Ue[a][k] = u[3 * cn[a] + k];
}

/* Hourglass force f_a = k sum_alpha gamma_alpha[a] q_alpha, q_alpha = gamma_alpha^T Ue. */
static void hourglass_force(const ora_ctx *c, int e, const double Ue[8][3], double Fe[8][3]) {
    const double *g = c->gam + 32 * e;
    for (int al = 0; al < 4; al++) {
        double q[3] = {0, 0, 0};
        for (int b = 0; b < 8; b++)
            for (int k = 0; k < 3; k++) q[k] += g[8 * al + b] * Ue[b][k];
        for (int a = 0; a < 8; a++)
            for (int k = 0; k < 3; k++) Fe[a][k] += c->khg[e] * g[8 * al + a] * q[k];
    }
}

/*
 * DJ-TLED element force, Algorithm 1 run-time steps 1-4, Table 3 (NH, TI, OT and MR rows).
 * Fe[a][k] is component k of the force at local node a (column a of the 3 x n_e F).
 * Returns J (the volume ratio of Eq. 12).
 */
/* pvol: NULL, or per element the pressure dPsi_vol/dJ to use instead of the
   element's own kappa (J - 1) (average nodal pressure, ora_forces_anp). */
static double force_djtled_p(const ora_ctx *c, int e, const double Ue[8][3], double Fe[8][3], const double *pvol) {
    const int ne = c->ne;
    const double *J0 = c->J0 + 9 * e;
    /* step 1: tJ = 0J + H_xi Ue (Eq. 11), tJ^{-1}, J = det(tJ) det(0J)^{-1} (Eq. 12) */
    double tJ[9], tJinv[9], tJT[9];
    for (int i = 0; i < 3; i++)
        for (int k = 0; k < 3; k++) {
            double s = J0[3 * i + k];
            for (int a = 0; a < ne; a++) s += c->H[i][a] * Ue[a][k];
            tJ[3 * i + k] = s;
        }
    double J = det3(tJ) / c->detJ0[e];
    inv3(tJ, tJinv);
    tr3(tJ, tJT);
    /* step 2: ghat (Eq. 18) */
    double g[6];
    ghat_of(tJ, g);
    /* step 3: I1 = ghat^T m1 (Eq. 27), I2 = ghat^T M2 ghat (Eq. 28), I4 = ghat^T m4 (Eq. 31),
       I6 = ghat^T m6 (Eq. 32) */
    double I1 = 0.0, I2 = 0.0, I4 = 0.0, I6 = 0.0;
    for (int k = 0; k < 6; k++) {
        I1 += g[k] * c->m1[6 * e + k];
        I4 += g[k] * c->m4[6 * e + k];
        I6 += g[k] * c->m6[6 * e + k];
        for (int l = 0; l < 6; l++) I2 += g[k] * c->M2[36 * e + 6 * k + l] * g[l];
    }
    double Jm23 = pow(J, -2.0 / 3.0);
    double I1b = Jm23 * I1, I2b = Jm23 * Jm23 * I2, I4b = Jm23 * I4, I6b = Jm23 * I6;
    /* step 4: Table 3.  dPsi/dI1b = mu/2 (C10 for MR), dPsi/dI2b = C01 (MR), dPsi/dI4b = eta_a (I4b - 1),
       dPsi/dI6b = eta_b (I6b - 1), J dPsi/dJ = kappa J (J - 1) */
    double mu = c->mu[e], kap = c->kappa[e];
    double d1 = 0.5 * mu, d2 = (c->model == ORA_MR) ? c->c01[e] : 0.0;
    double d4 = c->eta[e] * (I4b - 1.0), d6 = c->eta_b[e] * (I6b - 1.0);
    double Imix[9];
    for (int i = 0; i < 9; i++) {
        double gI2 = 0.0;  /* ghat^T . I2m (Eq. 42) */
        for (int k = 0; k < 6; k++) gI2 += g[k] * c->I2m[54 * e + 9 * k + i];
        Imix[i] = d1 * c->I1m[9 * e + i] + Jm23 * d2 * gI2 + d4 * c->I4m[9 * e + i] + d6 * c->I6m[9 * e + i];
    }
    double vol = -2.0 / 3.0 * (d1 * I1b + 2.0 * d2 * I2b + d4 * I4b + d6 * I6b) +
                 (pvol ? J * pvol[e] : kap * J * (J - 1.0));
    double M[9], t[9];
    mul3(tJT, Imix, t);
    for (int i = 0; i < 9; i++) M[i] = Jm23 * t[i] + vol * c->V[e] * tJinv[i];
    /* F = M H_xi : column a = sum_i M[:, i] H_xi[i][a] */
    for (int a = 0; a < ne; a++)
        for (int k = 0; k < 3; k++) {
            double s = 0.0;
            for (int i = 0; i < 3; i++) s += M[3 * k + i] * c->H[i][a];
            Fe[a][k] = s;
        }
    if (ne == 8) hourglass_force(c, e, Ue, Fe);
    return J;
}

/*
 * Classical TLED element force (Eq. 4): F = X S 0B 0V with X = I + u 0B^T
 * (Table 8, TLED column), C = X^T X, and S = 2 dPsi/dC of Eq. 7 for the
 * Table 3 energies, with the invariants taken from C directly:
 *   S = J^{-2/3} (2 d1 I + 2 d4 A + 2 d6 B) + 2 d2 J^{-4/3} (I1 I - C)
 *       + (-(2/3) (d1 I1b + 2 d2 I2b + d4 I4b + d6 I6b) + kappa J (J - 1)) C^{-1},
 * d1 = mu/2 (C10), d2 = C01, d4 = eta_a (I4b - 1), d6 = eta_b (I6b - 1).
 */
static double force_tled(const ora_ctx *c, int e, const double Ue[8][3], double Fe[8][3]) {
    const int ne = c->ne;
    const double *B = c->dhdX + (size_t)3 * ne * e;
    double X[9];
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            double s = (i == j) ? 1.0 : 0.0;
            for (int a = 0; a < ne; a++) s += Ue[a][i] * B[ne * j + a];
            X[3 * i + j] = s;
        }
    double J = det3(X);
    double XT[9], C[9], Cinv[9];
    tr3(X, XT);
    mul3(XT, X, C);
    inv3(C, Cinv);
    const double *a = c->fibre + 3 * e, *bb = c->fibre_b + 3 * e;
    double C2[9];
    mul3(C, C, C2);
    double I1 = trace3(C), I2 = 0.5 * (I1 * I1 - trace3(C2)), I4 = 0.0, I6 = 0.0;
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            I4 += a[i] * C[3 * i + j] * a[j];
            I6 += bb[i] * C[3 * i + j] * bb[j];
        }
    double Jm23 = pow(J, -2.0 / 3.0);
    double I1b = Jm23 * I1, I2b = Jm23 * Jm23 * I2, I4b = Jm23 * I4, I6b = Jm23 * I6;
    double mu = c->mu[e], kap = c->kappa[e];
    double d1 = 0.5 * mu, d2 = (c->model == ORA_MR) ? c->c01[e] : 0.0;
    double d4 = c->eta[e] * (I4b - 1.0), d6 = c->eta_b[e] * (I6b - 1.0);
    double p = -2.0 / 3.0 * (d1 * I1b + 2.0 * d2 * I2b + d4 * I4b + d6 * I6b) + kap * J * (J - 1.0);
    double S[9];
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            const double dij = (i == j ? 1.0 : 0.0);
            S[3 * i + j] = Jm23 * (2.0 * d1 * dij + 2.0 * d4 * a[i] * a[j] + 2.0 * d6 * bb[i] * bb[j]) +
                           2.0 * d2 * Jm23 * Jm23 * (I1 * dij - C[3 * i + j]) + p * Cinv[3 * i + j];
        }
    double XS[9];
    mul3(X, S, XS);
    for (int b = 0; b < ne; b++)
        for (int k = 0; k < 3; k++) {
            double s = 0.0;
            for (int j = 0; j < 3; j++) s += XS[3 * k + j] * B[ne * j + b];
            Fe[b][k] = s * c->V[e];
        }
    if (ne == 8) hourglass_force(c, e, Ue, Fe);
    return J;
}

static double force_djtled(const ora_ctx *c, int e, const double Ue[8][3], double Fe[8][3]) {
    return force_djtled_p(c, e, Ue, Fe, NULL);
}

/*
 * Global internal force sum_e F^(e) (Eq. 13), assembled in element order.
 * route 0: DJ-TLED (Table 3); route 1: classical TLED (Eq. 4).
 * Returns 0, or -3 if some element has J <= 0 (its index in *bad_elem).
 */
int ora_forces(const ora_ctx *c, const double *u, double *f, int route, int *bad_elem) {
#ifdef _OPENMP
    /* All-cores timing build (never used for parity): the element forces are
       formed in parallel, then every node adds its incidences in ascending
       element order -- the order of the loop below -- from zero, so the sums
       are the serial ones bit for bit. */
    {
        const int ne = c->ne;
        int first_bad = c->n_elems;
#pragma omp parallel for schedule(static) reduction(min : first_bad)
        for (int e = 0; e < c->n_elems; e++) {
            double Ue[8][3], Fe[8][3];
            gather_u(c, e, u, Ue);
            double J = (route == 0) ? force_djtled(c, e, Ue, Fe) : force_tled(c, e, Ue, Fe);
            if (!(J > 0.0) && e < first_bad) first_bad = e;
            for (int a = 0; a < ne; a++)
                for (int k = 0; k < 3; k++) c->fe[3 * ((size_t)e * ne + a) + k] = Fe[a][k];
        }
#pragma omp parallel for schedule(static)
        for (int n = 0; n < c->n_nodes; n++) {
            double s0 = 0.0, s1 = 0.0, s2 = 0.0;
            for (int q = c->inc_off[n]; q < c->inc_off[n + 1]; q++) {
                const double *g = c->fe + 3 * (size_t)c->inc[q];
                s0 += g[0];
                s1 += g[1];
                s2 += g[2];
            }
            f[3 * n] = s0;
            f[3 * n + 1] = s1;
            f[3 * n + 2] = s2;
        }
        if (bad_elem) *bad_elem = first_bad < c->n_elems ? first_bad : -1;
        return first_bad < c->n_elems ? -3 : 0;
    }
#endif
    memset(f, 0, sizeof(double) * 3 * (size_t)c->n_nodes);
    int rc = 0;
    if (bad_elem) *bad_elem = -1;
    for (int e = 0; e < c->n_elems; e++) {
        double Ue[8][3], Fe[8][3];
        gather_u(c, e, u, Ue);
        double J = (route == 0) ? force_djtled(c, e, Ue, Fe) : force_tled(c, e, Ue, Fe);
        if (!(J > 0.0) && rc == 0) {
            rc = -3;
            if (bad_elem) *bad_elem = e;
        }
        const int *cn = c->conn + (size_t)e * c->ne;
        for (int a = 0; a < c->ne; a++)
            for (int k = 0; k < 3; k++) f[3 * cn[a] + k] += Fe[a][k];
    }
    return rc;
}

/* Forces of a single element (for tests); Fe is ne x 3. */
int ora_element_force(const ora_ctx *c, int e, const double *Ue_in, double *Fe_out, int route) {
    if (e < 0 || e >= c->n_elems) return -1;
    double Ue[8][3], Fe[8][3];
    for (int a = 0; a < c->ne; a++)
        for (int k = 0; k < 3; k++) Ue[a][k] = Ue_in[3 * a + k];
    if (route == 0) force_djtled(c, e, Ue, Fe); else force_tled(c, e, Ue, Fe);
    for (int a = 0; a < c->ne; a++)
        for (int k = 0; k < 3; k++) Fe_out[3 * a + k] = Fe[a][k];
    return 0;
}

/*
 * Average nodal pressure (the locking remedy Sec. 7 mentions for nearly
 * incompressible tissue), in its variational reading: the volumetric energy
 * is carried by the nodes, sum_n V_n kappa_n (J_n - 1)^2 / 2, with nodal
 * volume V_n = sum_e 0V_e / n_e, volume ratio J_n = sum_e (0V_e / n_e) J_e / V_n
 * and modulus kappa_n = sum_e (0V_e / n_e) kappa_e / V_n over the elements
 * around n.  Its gradient is the Table 3 force with each element's pressure
 * kappa_e (J_e - 1) replaced by the mean of kappa_n (J_n - 1) over the
 * element's nodes.  Returns 0, or -3 with *bad_elem if some J_e <= 0.
 */
int ora_forces_anp(const ora_ctx *c, const double *u, double *f, int *bad_elem) {
    const int ne = c->ne, E_ = c->n_elems, N_ = c->n_nodes;
    double *Je = (double *)calloc((size_t)E_, sizeof(double));
    double *Vn = (double *)calloc((size_t)N_, sizeof(double));
    double *Jn = (double *)calloc((size_t)N_, sizeof(double));
    double *Kn = (double *)calloc((size_t)N_, sizeof(double));
    double *pb = (double *)calloc((size_t)E_, sizeof(double));
    int rc = 0;
    if (bad_elem) *bad_elem = -1;
    for (int e = 0; e < E_; e++) {
        double Ue[8][3], tJ[9];
        gather_u(c, e, u, Ue);
        const double *J0 = c->J0 + 9 * e;
        for (int i = 0; i < 3; i++)
            for (int k = 0; k < 3; k++) {
                double s = J0[3 * i + k];
                for (int a = 0; a < ne; a++) s += c->H[i][a] * Ue[a][k];
                tJ[3 * i + k] = s;
            }
        Je[e] = det3(tJ) / c->detJ0[e];  /* Eq. 12 */
        if (!(Je[e] > 0.0) && rc == 0) {
            rc = -3;
            if (bad_elem) *bad_elem = e;
        }
        const int *cn = c->conn + (size_t)e * ne;
        for (int a = 0; a < ne; a++) {
            const double w = c->V[e] / ne;
            Vn[cn[a]] += w;
            Jn[cn[a]] += w * Je[e];
            Kn[cn[a]] += w * c->kappa[e];
        }
    }
    for (int n = 0; n < N_; n++)
        if (Vn[n] > 0.0) {
            Jn[n] /= Vn[n];
            Kn[n] /= Vn[n];
        }
    for (int e = 0; e < E_; e++) {
        const int *cn = c->conn + (size_t)e * ne;
        double s = 0.0;
        for (int a = 0; a < ne; a++) s += Kn[cn[a]] * (Jn[cn[a]] - 1.0);
        pb[e] = s / ne;
    }
    memset(f, 0, sizeof(double) * 3 * (size_t)N_);
    for (int e = 0; e < E_; e++) {
        double Ue[8][3], Fe[8][3];
        gather_u(c, e, u, Ue);
        force_djtled_p(c, e, Ue, Fe, pb);
        const int *cn = c->conn + (size_t)e * ne;
        for (int a = 0; a < ne; a++)
            for (int k = 0; k < 3; k++) f[3 * cn[a] + k] += Fe[a][k];
    }
    free(Je); free(Vn); free(Jn); free(Kn); free(pb);
    return rc;
}

/*
 * Strain energy E(u) = sum_e 0V_e Psi_e (Table 3 strain energy densities,
 * computed from X = I + u 0B^T, C = X^T X) plus the hourglass energy
 * k/2 sum_alpha |q_alpha|^2 for H8.
 */
double ora_energy(const ora_ctx *c, const double *u) {
    double Etot = 0.0;
    for (int e = 0; e < c->n_elems; e++) {
        double Ue[8][3];
        gather_u(c, e, u, Ue);
        const int ne = c->ne;
        const double *B = c->dhdX + (size_t)3 * ne * e;
        double X[9];
        for (int i = 0; i < 3; i++)
            for (int j = 0; j < 3; j++) {
                double s = (i == j) ? 1.0 : 0.0;
                for (int a = 0; a < ne; a++) s += Ue[a][i] * B[ne * j + a];
                X[3 * i + j] = s;
            }
        double J = det3(X);
        double XT[9], C[9];
        tr3(X, XT);
        mul3(XT, X, C);
        const double *av = c->fibre + 3 * e, *bv = c->fibre_b + 3 * e;
        double C2[9];
        mul3(C, C, C2);
        double I1 = trace3(C), I2 = 0.5 * (I1 * I1 - trace3(C2)), I4 = 0.0, I6 = 0.0;
        for (int i = 0; i < 3; i++)
            for (int j = 0; j < 3; j++) {
                I4 += av[i] * C[3 * i + j] * av[j];
                I6 += bv[i] * C[3 * i + j] * bv[j];
            }
        double Jm23 = pow(J, -2.0 / 3.0);
        /* Table 3 energies: mu/2 (I1b - 3) is C10 (I1b - 3) with C10 = mu / 2 */
        double psi = 0.5 * c->mu[e] * (Jm23 * I1 - 3.0) + 0.5 * c->kappa[e] * (J - 1.0) * (J - 1.0);
        psi += 0.5 * c->eta[e] * (Jm23 * I4 - 1.0) * (Jm23 * I4 - 1.0);
        psi += 0.5 * c->eta_b[e] * (Jm23 * I6 - 1.0) * (Jm23 * I6 - 1.0);
        if (c->model == ORA_MR) psi += c->c01[e] * (Jm23 * Jm23 * I2 - 3.0);
        Etot += c->V[e] * psi;
        if (ne == 8) {
            const double *g = c->gam + 32 * e;
            for (int al = 0; al < 4; al++) {
                double q[3] = {0, 0, 0};
                for (int b = 0; b < 8; b++)
                    for (int k = 0; k < 3; k++) q[k] += g[8 * al + b] * Ue[b][k];
                Etot += 0.5 * c->khg[e] * (q[0] * q[0] + q[1] * q[1] + q[2] * q[2]);
            }
        }
    }
    return Etot;
}

/*
 * Strain invariants by the Jacobian formulations of Table 1, from 0J, tJ and a
 * fibre direction a:  out = [I1 (Eq. 27), I2 (Eq. 28), I3 (Eq. 29), I4 (Eq. 31)],
 * using G (Appendix B), m1 (C.1), W (C.4), M2 (C.5) and m4 (C.2).
 */
void ora_jacobian_invariants(const double *J0, const double *tJ, const double *a, double *out) {
    double J0inv[9], G[6][9], g[6];
    inv3(J0, J0inv);
    g_matrices(J0inv, G);
    ghat_of(tJ, g);
    double m1[6], m4[6], W[36];
    double A[9];
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) A[3 * i + j] = a[i] * a[j];
    for (int k = 0; k < 6; k++) {
        double AG[9];
        m1[k] = trace3(G[k]);
        mul3(A, G[k], AG);
        m4[k] = trace3(AG);
    }
    for (int k = 0; k < 6; k++)
        for (int l = 0; l < 6; l++) {
            double GT[9], P[9];
            tr3(G[k], GT);
            mul3(GT, G[l], P);
            W[6 * k + l] = trace3(P);
        }
    double I1 = 0.0, I4 = 0.0, I2 = 0.0;
    for (int k = 0; k < 6; k++) { I1 += g[k] * m1[k]; I4 += g[k] * m4[k]; }
    for (int k = 0; k < 6; k++)
        for (int l = 0; l < 6; l++) I2 += g[k] * 0.5 * (m1[k] * m1[l] - W[6 * k + l]) * g[l];
    double r = det3(tJ) / det3(J0);
    out[0] = I1; out[1] = I2; out[2] = r * r; out[3] = I4;
}

/* Load-ramp shape s(t / t_ramp): 0 none (always 1), 1 linear, 2 quintic smoothstep. */
static double ramp_value(int ramp, double t, double t_ramp) {
    if (ramp == 0 || t_ramp <= 0.0) return 1.0;
    double tau = t / t_ramp;
    if (tau >= 1.0) return 1.0;
    if (tau <= 0.0) return 0.0;
    if (ramp == 1) return tau;
    return tau * tau * tau * (10.0 - 15.0 * tau + 6.0 * tau * tau);
}

/* Dynamic relaxation residual |(F - R)_free|_2 / |F_constrained|_2.  It is
   relative to the reaction at the constrained components; with no reaction
   (for instance at a start from rest before any prescribed value is applied)
   it is undefined and taken as infinite, so a relaxation never stops there. */
static double residual_of(const ora_ctx *c, const double *f, const double *R, const unsigned char *cmask) {
    double num = 0.0, den = 0.0;
    for (int i = 0; i < 3 * c->n_nodes; i++) {
        double r = f[i] - (R ? R[i] : 0.0);
        if (cmask[i]) den += f[i] * f[i]; else num += r * r;
    }
    if (den > 0.0) return sqrt(num) / sqrt(den);
    return INFINITY;
}

/*
 * Explicit time stepping (Eq. 13 with central differences), n_steps steps from
 * global step index step0.  (u_cur, u_prev) = (u^n, u^{n-1}) are updated in place.
 *   u^{n+1}_i = A_i (R_i - F_i(u^n)) + B u^n_i + C u^{n-1}_i
 *   A_i = 2 dt^2 / ((2 + alpha dt) m_i),  B = 4 / (2 + alpha dt),  C = (alpha dt - 2) / (alpha dt + 2)
 * followed by u^{n+1}[node, k] = s(t_{n+1}) target[k] for every component k in
 * bc_mask[j] (bit k) of constrained node bc_node[j].
 * relax != 0: every check_every steps once the ramp is complete, the residual of
 * u^n is evaluated first and the run stops, without advancing, if it is <= tol.
 * anp != 0: F is the average-nodal-pressure internal force (ora_forces_anp).
 * Returns 0 (all steps done), 1 (converged), -3 (element inverted), -4 (non-finite).
 */
int ora_run(const ora_ctx *c, double *u_cur, double *u_prev, const double *R, int n_bc, const int *bc_node,
            const int *bc_mask, const double *bc_target, int ramp, double t_ramp, double dt, double alpha,
            long step0, int n_steps, int relax, double tol, int check_every, double *residual_out,
            int *steps_done, int anp) {
    const int N3 = 3 * c->n_nodes;
    double *f = (double *)malloc(sizeof(double) * N3);
    double *un = (double *)malloc(sizeof(double) * N3);
    unsigned char *cmask = (unsigned char *)calloc(N3, 1);
    for (int j = 0; j < n_bc; j++)
        for (int k = 0; k < 3; k++)
            if (bc_mask[j] & (1 << k)) cmask[3 * bc_node[j] + k] = 1;
    const double Bc = 4.0 / (2.0 + alpha * dt);
    const double Cc = (alpha * dt - 2.0) / (alpha * dt + 2.0);
    int rc = 0, s = 0;
    if (residual_out) *residual_out = NAN;
    if (check_every <= 0) check_every = 1;
    for (s = 0; s < n_steps; s++) {
        long n = step0 + s;
        int bad;
        if ((anp ? ora_forces_anp(c, u_cur, f, &bad) : ora_forces(c, u_cur, f, 0, &bad)) != 0) { rc = -3; break; }
        if (relax && (s % check_every) == 0 && ramp_value(ramp, (double)n * dt, t_ramp) >= 1.0) {
            double r = residual_of(c, f, R, cmask);
            if (residual_out) *residual_out = r;
            if (r <= tol) { rc = 1; break; }
        }
        for (int i = 0; i < c->n_nodes; i++) {
            double A = 2.0 * dt * dt / ((2.0 + alpha * dt) * c->mass[i]);
            for (int k = 0; k < 3; k++) {
                int q = 3 * i + k;
                un[q] = A * ((R ? R[q] : 0.0) - f[q]) + Bc * u_cur[q] + Cc * u_prev[q];
            }
        }
        double sv = ramp_value(ramp, (double)(n + 1) * dt, t_ramp);
        for (int j = 0; j < n_bc; j++)
            for (int k = 0; k < 3; k++)
                if (bc_mask[j] & (1 << k)) un[3 * bc_node[j] + k] = sv * bc_target[3 * j + k];
        int finite = 1;
        for (int q = 0; q < N3; q++)
            if (!isfinite(un[q])) { finite = 0; break; }
        memcpy(u_prev, u_cur, sizeof(double) * N3);
        memcpy(u_cur, un, sizeof(double) * N3);
        if (!finite) { rc = -4; s++; break; }
    }
    if (steps_done) *steps_done = s;
    free(f); free(un); free(cmask);
    return rc;
}

/* Residual of a state (same definition as used by ora_run). */
double ora_residual(const ora_ctx *c, const double *u, const double *R, int n_bc, const int *bc_node,
                    const int *bc_mask) {
    const int N3 = 3 * c->n_nodes;
    double *f = (double *)malloc(sizeof(double) * N3);
    unsigned char *cmask = (unsigned char *)calloc(N3, 1);
    for (int j = 0; j < n_bc; j++)
        for (int k = 0; k < 3; k++)
            if (bc_mask[j] & (1 << k)) cmask[3 * bc_node[j] + k] = 1;
    ora_forces(c, u, f, 0, NULL);
    double r = residual_of(c, f, R, cmask);
    free(f); free(cmask);
    return r;
}
