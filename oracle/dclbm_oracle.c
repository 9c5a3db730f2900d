/*
 * dclbm_oracle.c -- TEST INFRASTRUCTURE, not part of the product.
 *
 * A plain, slow, FP64 CPU implementation of the lattice Boltzmann step on a
 * nested-box refined mesh with the cell-vertex direct coupling (DC) of
 * Astoul, Wissocq, Boussuge, Sengissen & Sagaut, "Lattice Boltzmann method for
 * computational aeroacoustics on non-uniform meshes: a direct grid coupling
 * approach" (arXiv:2004.14887).  It exists only to check the HIP library: only
 * the test suite, the smoke check and the benchmark's CPU-baseline leg may
 * load it.  It shares no code, header, table or generator with the HIP path.
 *
 * Everything is node by node, in the order the paper gives the algorithm
 * (Sec. 3.5, "Steps of the algorithm"), generalised recursively to more than
 * two levels.  No fusion, no blocking, no reordering.  Storage is AoS per
 * level: f[node][Q] (post-collision) and pre[node][Q] (post-streaming,
 * completed pre-collision), so that nothing about its layout resembles the
 * device code.
 *
 * Readings of points the paper leaves open (binding for this file):
 *  - Eq.(TempInt): the weights -1/8, 3/4, 3/8 are taken at coarse times
 *    t-dt^c, t, t+dt^c (the only times for which those are the quadratic
 *    Lagrange weights of the fine mid-step); at a level's first step, where no
 *    t-dt^c value exists, the linear mean of t and t+dt^c is used.
 *  - Sec. 3.5 steps 2e/3c: every direction with Gamma_i = R is rebuilt with
 *    Eq.(rescff) (under DC2 that is P u M^f), so the completed moments equal X.
 *  - Sec. 3.2 spatial interpolation: 4-point Lagrange along the interface
 *    line, centred (-1,9,9,-1)/16, one-sided (5,15,-5,1)/16 at line ends,
 *    tensor product at 3-D face centres; stencil nodes are co-located nodes.
 *  - Newton: start from the raw moments of h, stop when the infinity norm of
 *    the update is below the tolerance (1e-12 in Sec. 3.2).
 *  - Collision of co-located nodes uses the shared equilibrium f^(0)(X)
 *    (Sec. 6 and Sec. 3.4, Eq.(rescfc)).
 *  - Collision model: BGK, f* = f^(0) + (1 - 1/tau)(f - f^(0)), i.e. the
 *    regularised scheme of Eq.(LBMscheme_reg) with f^(1) = f - f^(0), psi = 0.
 */
#include "dclbm_oracle.h"

#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#define MAXQ 19
#define MAXL 4

enum { C_HOLE = 0, C_BULK = 1, C_TFC = 2, C_TFF = 3, C_IE = 4 };

typedef struct {
    int D, Q;
    int xi[MAXQ][3];
    double w[MAXQ];
    double cs2;
} lattice_t;

/* Sec. 2, Eq.(xi_i), Eq.(w_i) for D3Q19; D2Q9 numbered as in Fig. 1
 * (1=E 2=NE 3=N 4=NW 5=W 6=SW 7=S 8=SE), textbook weights 4/9, 1/9, 1/36. */
static int make_lattice(int which, lattice_t* L)
{
    memset(L, 0, sizeof(*L));
    L->cs2 = 1.0 / 3.0;
    if (which == ORC_D2Q9) {
        static const int v[9][2] = {{0, 0}, {1, 0}, {1, 1}, {0, 1}, {-1, 1},
                                    {-1, 0}, {-1, -1}, {0, -1}, {1, -1}};
        L->D = 2;
        L->Q = 9;
        for (int i = 0; i < 9; ++i) {
            L->xi[i][0] = v[i][0];
            L->xi[i][1] = v[i][1];
            L->xi[i][2] = 0;
            int n2 = v[i][0] * v[i][0] + v[i][1] * v[i][1];
            L->w[i] = n2 == 0 ? 4.0 / 9.0 : (n2 == 1 ? 1.0 / 9.0 : 1.0 / 36.0);
        }
        return 0;
    }
    if (which == ORC_D3Q19) {
        static const int v[19][3] = {
            {0, 0, 0},  {1, 0, 0},   {-1, 0, 0}, {0, 1, 0},  {0, -1, 0},
            {0, 0, 1},  {0, 0, -1},  {1, 1, 0},  {-1, -1, 0}, {1, -1, 0},
            {-1, 1, 0}, {1, 0, 1},   {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
            {0, 1, 1},  {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};
        L->D = 3;
        L->Q = 19;
        for (int i = 0; i < 19; ++i) {
            int n2 = 0;
            for (int a = 0; a < 3; ++a) {
                L->xi[i][a] = v[i][a];
                n2 += v[i][a] * v[i][a];
            }
            L->w[i] = n2 == 0 ? 1.0 / 3.0 : (n2 == 1 ? 1.0 / 18.0 : 1.0 / 36.0);
        }
        return 0;
    }
    return -1;
}

/* ------------------------------------------------------------------------- */
/* Equilibrium, Sec. 2 Eq.(fEqH)/(fEq_herm):                                  */
/*   f0_i = w_i rho [1 + xi.u/c^2 + H2_i:uu/(2c^4)                            */
/*                   + (eq_order 3) sum_{a!=g} H3_{i,aag} u_a^2 u_g/(2c^6)]   */
/* with H2_i:uu = (xi.u)^2 - c^2|u|^2 and H3_{i,aag} = xi_a^2 xi_g - c^2 xi_g. */
/* ------------------------------------------------------------------------- */
static double third_order_sum(const lattice_t* L, int i, const double u[3])
{
    double s = 0.0;
    for (int a = 0; a < L->D; ++a)
        for (int g = 0; g < L->D; ++g) {
            if (a == g) continue;
            double H3 = (double)(L->xi[i][a] * L->xi[i][a] * L->xi[i][g]) - L->cs2 * L->xi[i][g];
            s += H3 * u[a] * u[a] * u[g];
        }
    return s;
}

static double feq_i(const lattice_t* L, int eq_order, int i, double rho, const double u[3])
{
    double c2 = L->cs2;
    double cu = 0.0, uu = 0.0;
    for (int a = 0; a < L->D; ++a) {
        cu += L->xi[i][a] * u[a];
        uu += u[a] * u[a];
    }
    double b = 1.0 + cu / c2 + (cu * cu - c2 * uu) / (2.0 * c2 * c2);
    if (eq_order == 3) b += third_order_sum(L, i, u) / (2.0 * c2 * c2 * c2);
    return L->w[i] * rho * b;
}

/* d f0_i / d X, X = (rho, u_1..u_D): analytic derivative of the expression above. */
static void dfeq_i(const lattice_t* L, int eq_order, int i, double rho, const double u[3], double d[4])
{
    double c2 = L->cs2;
    double cu = 0.0;
    for (int a = 0; a < L->D; ++a) cu += L->xi[i][a] * u[a];
    d[0] = feq_i(L, eq_order, i, rho, u) / rho;
    for (int b = 0; b < L->D; ++b) {
        double v = L->xi[i][b] / c2 + (cu * L->xi[i][b] - c2 * u[b]) / (c2 * c2);
        if (eq_order == 3) {
            double s = 0.0;
            for (int a = 0; a < L->D; ++a)
                for (int g = 0; g < L->D; ++g) {
                    if (a == g) continue;
                    double H3 = (double)(L->xi[i][a] * L->xi[i][a] * L->xi[i][g]) - c2 * L->xi[i][g];
                    double dd = 0.0;
                    if (a == b) dd += 2.0 * u[a] * u[g];
                    if (g == b) dd += u[a] * u[a];
                    s += H3 * dd;
                }
            v += s / (2.0 * c2 * c2 * c2);
        }
        d[1 + b] = L->w[i] * rho * v;
    }
}

/* ------------------------------------------------------------------------- */
/* Newton-Raphson for F(X) = sum_i Gamma_i Phi_i (h_i - f0_i(X)) = 0,          */
/* Sec. 3.2 Eq.(system_fi) and Eq.(updated_macro).                            */
/* ------------------------------------------------------------------------- */
static int solve_gepp(int n, double A[4][4], double b[4], double x[4])
{
    /* Gaussian elimination with partial pivoting. */
    double M[4][5];
    for (int r = 0; r < n; ++r) {
        for (int c = 0; c < n; ++c) M[r][c] = A[r][c];
        M[r][n] = b[r];
    }
    for (int k = 0; k < n; ++k) {
        int p = k;
        for (int r = k + 1; r < n; ++r)
            if (fabs(M[r][k]) > fabs(M[p][k])) p = r;
        if (M[p][k] == 0.0) return -1;
        if (p != k)
            for (int c = 0; c <= n; ++c) {
                double t = M[k][c];
                M[k][c] = M[p][c];
                M[p][c] = t;
            }
        for (int r = k + 1; r < n; ++r) {
            double m = M[r][k] / M[k][k];
            for (int c = k; c <= n; ++c) M[r][c] -= m * M[k][c];
        }
    }
    for (int r = n - 1; r >= 0; --r) {
        double s = M[r][n];
        for (int c = r + 1; c < n; ++c) s -= M[r][c] * x[c];
        x[r] = s / M[r][r];
    }
    return 0;
}

static void residual(const lattice_t* L, int eq_order, const double* h, const double* G,
                     const double X[4], double F[4])
{
    int n = L->D + 1;
    double u[3] = {0, 0, 0};
    for (int a = 0; a < L->D; ++a) u[a] = X[1 + a];
    for (int r = 0; r < n; ++r) F[r] = 0.0;
    for (int i = 0; i < L->Q; ++i) {
        double d = G[i] * (h[i] - feq_i(L, eq_order, i, X[0], u));
        F[0] += d;
        for (int a = 0; a < L->D; ++a) F[1 + a] += L->xi[i][a] * d;
    }
}

static int newton(const lattice_t* L, int eq_order, const double* h, const double* G,
                  double tol, int maxit, double X[4], int* iters)
{
    int n = L->D + 1;
    /* initial guess: raw moments of h */
    double rho = 0.0, j[3] = {0, 0, 0};
    for (int i = 0; i < L->Q; ++i) {
        rho += h[i];
        for (int a = 0; a < L->D; ++a) j[a] += L->xi[i][a] * h[i];
    }
    X[0] = rho;
    for (int a = 0; a < L->D; ++a) X[1 + a] = j[a] / rho;
    for (int a = L->D; a < 3; ++a) X[1 + a] = 0.0;
    for (int it = 1; it <= maxit; ++it) {
        double F[4], J[4][4], rhs[4], dX[4];
        residual(L, eq_order, h, G, X, F);
        for (int r = 0; r < n; ++r)
            for (int c = 0; c < n; ++c) J[r][c] = 0.0;
        double u[3] = {0, 0, 0};
        for (int a = 0; a < L->D; ++a) u[a] = X[1 + a];
        for (int i = 0; i < L->Q; ++i) {
            double d[4];
            dfeq_i(L, eq_order, i, X[0], u, d);
            double phi[4] = {1.0, (double)L->xi[i][0], (double)L->xi[i][1], (double)L->xi[i][2]};
            for (int r = 0; r < n; ++r)
                for (int c = 0; c < n; ++c) J[r][c] -= G[i] * phi[r] * d[c];
        }
        for (int r = 0; r < n; ++r) rhs[r] = -F[r];
        if (solve_gepp(n, J, rhs, dX) != 0) return -2;
        double nrm = 0.0;
        for (int r = 0; r < n; ++r) {
            X[r] += dX[r];
            if (fabs(dX[r]) > nrm) nrm = fabs(dX[r]);
        }
        if (!(nrm == nrm)) return -3;
        if (nrm < tol) {
            *iters = it;
            return 0;
        }
    }
    *iters = maxit;
    return -1;
}

/* ------------------------------------------------------------------------- */
/* Index sets (Sec. 3.2, Sec. 3.4 Table "choice_Gamma_fine", App. B)          */
/* K^f: directions streamed on the fine copy; K^c: on the coarse copy.        */
/* ------------------------------------------------------------------------- */
static int sets_from_known(const lattice_t* L, unsigned Kf, unsigned Kc, int coupling,
                           unsigned* P, unsigned* Qf, unsigned* Qc, unsigned* Mf,
                           unsigned* Mc, unsigned* gammaR)
{
    unsigned all = (1u << L->Q) - 1u;
    *P = Kf & Kc;
    *Qf = Kf & ~Kc;
    *Qc = Kc & ~Kf;
    *Mf = all & ~Kf;
    *Mc = all & ~Kc;
    /* DC1: (1,f) on P and Q^f, (R,c) on M^f.  DC2: (R,c) on P and M^f. */
    if (coupling == 1)
        *gammaR = *Mf;
    else if (coupling == 2)
        *gammaR = *P | *Mf;
    else
        return -1;
    /* every coarse-sourced direction must be known on the coarse copy and
     * every fine-sourced one on the fine copy */
    if ((*gammaR & ~Kc) != 0) return -2;
    if (((all & ~*gammaR) & ~Kf) != 0) return -2;
    return 0;
}

/* 4-point Lagrange weights for a hanging node at odd position k on a line of
 * co-located nodes at even positions 0..N (Sec. 3.2, fourth-order 1-D). */
static void line_stencil(int k, int N, int pos[4], double w[4])
{
    if (k == 1) {
        pos[0] = 0; pos[1] = 2; pos[2] = 4; pos[3] = 6;
        w[0] = 5.0 / 16; w[1] = 15.0 / 16; w[2] = -5.0 / 16; w[3] = 1.0 / 16;
    } else if (k == N - 1) {
        pos[0] = N; pos[1] = N - 2; pos[2] = N - 4; pos[3] = N - 6;
        w[0] = 5.0 / 16; w[1] = 15.0 / 16; w[2] = -5.0 / 16; w[3] = 1.0 / 16;
    } else {
        pos[0] = k - 3; pos[1] = k - 1; pos[2] = k + 1; pos[3] = k + 3;
        w[0] = -1.0 / 16; w[1] = 9.0 / 16; w[2] = 9.0 / 16; w[3] = -1.0 / 16;
    }
}

/* ------------------------------------------------------------------------- */
/* Mesh                                                                       */
/* ------------------------------------------------------------------------- */
typedef struct {
    int n[3];          /* nodes per axis (n[2] = 1 in 2-D) */
    long long N;       /* total nodes (dense) */
    int periodic;      /* level 0 only */
    int has_child;
    int clo[3], chi[3];/* child box in this level's node coords, [clo,chi] closed */
    int plo[3];        /* own box lower corner in the parent's node coords */
    double off[3];     /* level-0 coordinate of node 0 */
    double tau;
    unsigned char* cls;
    double* f;         /* post-collision [N][Q] */
    double* pre;       /* post-streaming / completed pre-collision [N][Q] */
    double* X;         /* shared macros at TF^f / TF^c nodes [N][4] */
    long long* tfc_id; /* TF^c node -> history slot, -1 otherwise */
    long long n_tfc;
    double* H;         /* history ring [n_tfc][3][Q]: slot 0 = t-dt, 1 = t, 2 = t+dt */
    long long captures;/* number of history captures made on this level */
    /* H-RR only */
    double* M;         /* (rho, u) of every active node at the level's current time [N][4] */
    double* Mring;     /* post-streaming (rho, u) at the coarse times t-dt, t, t+dt [3][N][4] (levels with a child) */
    double* G;         /* gradients: d_b u_a, then sum_g d_g Psi_abg [N][2][3][3] */
} level_t;

struct orc_sim {
    lattice_t L;
    int eq_order, coupling, nlev;
    level_t lv[MAXL];
    double newton_tol;
    int newton_maxit;
    double R_override; /* planted-mistake hook for tests; 0 = off */
    int collision;     /* 0: BGK; 1: H-RR */
    double hrr_sigma;  /* weight of the projected part of a_1^(2), Eq.(a12_HRR) */
    int hrr_psi;       /* cubic Mach correction psi_i of App. A on (1) or off (0) */
    unsigned char* region; /* refined region of level 1 as a mask of level-0 cells over its box (NULL: the box) */
    int sponge_w;      /* absorbing layer on level 0: width in cells (0 = none) */
    double sponge_sigma;
    double sponge_u[3];/* target velocity of the layer (target density 1) */
    long long newton_calls;
    int newton_max_iters;
    long long newton_iter_hist[8];
    int error;
    long long coarse_steps;
    int n_probes;
    int* probes;       /* level-0 node coords [n_probes][3] */
    long long probe_cap, probe_len;
    double* probe_series;
};

static long long nid(const level_t* v, int x, int y, int z)
{
    return ((long long)z * v->n[1] + y) * v->n[0] + x;
}

static void classify_level(const lattice_t* L, level_t* v, int l)
{
    for (int z = 0; z < v->n[2]; ++z)
        for (int y = 0; y < v->n[1]; ++y)
            for (int x = 0; x < v->n[0]; ++x) {
                int k[3] = {x, y, z};
                int c = C_BULK;
                if (v->has_child) {
                    int inside_strict = 1, inside_closed = 1;
                    for (int a = 0; a < L->D; ++a) {
                        if (!(k[a] > v->clo[a] && k[a] < v->chi[a])) inside_strict = 0;
                        if (!(k[a] >= v->clo[a] && k[a] <= v->chi[a])) inside_closed = 0;
                    }
                    if (inside_strict)
                        c = C_HOLE;
                    else if (inside_closed)
                        c = C_TFC;
                }
                if (c == C_BULK && l > 0) {
                    int boundary = 0, all_even = 1;
                    for (int a = 0; a < L->D; ++a) {
                        if (k[a] == 0 || k[a] == v->n[a] - 1) boundary = 1;
                        if (k[a] % 2) all_even = 0;
                    }
                    if (boundary) c = all_even ? C_TFF : C_IE;
                }
                v->cls[nid(v, x, y, z)] = (unsigned char)c;
            }
}

/* Co-located interface node at fine position (x, y) of level v? */
static int is_tff(const level_t* v, int x, int y)
{
    return x >= 0 && y >= 0 && x < v->n[0] && y < v->n[1] && v->cls[nid(v, x, y, 0)] == C_TFF;
}

/* 4-point stencil of hanging node k on a refined region's boundary (2-D,
 * one odd coordinate): along its odd axis, the centred points k-3..k+3 when
 * all four are co-located interface nodes, else the one-sided points
 * k-1..k+5 or k+1..k-5, else the linear pair k-1, k+1 (a boundary run of one
 * parent cell between two steps).  The weights are those of R6; on a box
 * boundary the rule gives the box line's stencils.  Returns the number of
 * points used, -1 if none fits. */
static int region_stencil(const level_t* v, const int k[3], int pos[4], double w[4])
{
    const int a = (k[0] & 1) ? 0 : 1;
    int p[3] = {k[0], k[1], 0};
#define TFF_AT(o) (p[a] = k[a] + (o), is_tff(v, p[0], p[1]))
    if (TFF_AT(-3) && TFF_AT(-1) && TFF_AT(1) && TFF_AT(3)) {
        const int o[4] = {-3, -1, 1, 3};
        const double ww[4] = {-1.0 / 16, 9.0 / 16, 9.0 / 16, -1.0 / 16};
        for (int j = 0; j < 4; ++j) pos[j] = k[a] + o[j], w[j] = ww[j];
        return 4;
    }
    for (int sg = 1; sg >= -1; sg -= 2) {
        if (TFF_AT(-sg) && TFF_AT(sg) && TFF_AT(3 * sg) && TFF_AT(5 * sg)) {
            const int o[4] = {-sg, sg, 3 * sg, 5 * sg};
            const double ww[4] = {5.0 / 16, 15.0 / 16, -5.0 / 16, 1.0 / 16};
            for (int j = 0; j < 4; ++j) pos[j] = k[a] + o[j], w[j] = ww[j];
            return 4;
        }
    }
    if (TFF_AT(-1) && TFF_AT(1)) {
        pos[0] = k[a] - 1, pos[1] = k[a] + 1, pos[2] = pos[3] = k[a] - 1;
        w[0] = w[1] = 0.5, w[2] = w[3] = 0.0;
        return 2;
    }
#undef TFF_AT
    return -1;
}

/* Node k of level v, displaced by d; returns its id, or -1 if it is not an
 * active node of that level. */
static long long active_at(const lattice_t* L, const level_t* v, const int k[3], const int d[3])
{
    int q[3] = {k[0] + d[0], k[1] + d[1], k[2] + d[2]};
    for (int a = 0; a < 3; ++a) {
        if (a >= L->D) {
            q[a] = 0;
            continue;
        }
        if (v->periodic) {
            q[a] %= v->n[a];
            if (q[a] < 0) q[a] += v->n[a];
        } else if (q[a] < 0 || q[a] >= v->n[a]) {
            return -1;
        }
    }
    long long id = nid(v, q[0], q[1], q[2]);
    return v->cls[id] == C_HOLE ? -1 : id;
}

/* Known-direction masks of a co-located node: fine node k on level l and its
 * coarse copy on level l-1. */
static void known_masks(const orc_sim* s, int l, const int k[3], unsigned* Kf, unsigned* Kc)
{
    const lattice_t* L = &s->L;
    const level_t* fv = &s->lv[l];
    const level_t* cv = &s->lv[l - 1];
    int p[3] = {0, 0, 0};
    for (int a = 0; a < L->D; ++a) p[a] = fv->plo[a] + k[a] / 2;
    *Kf = 0;
    *Kc = 0;
    for (int i = 0; i < L->Q; ++i) {
        int d[3] = {-L->xi[i][0], -L->xi[i][1], -L->xi[i][2]};
        if (active_at(L, fv, k, d) >= 0) *Kf |= 1u << i;
        if (active_at(L, cv, p, d) >= 0) *Kc |= 1u << i;
    }
}

static void free_sim(orc_sim* s)
{
    if (!s) return;
    free(s->region);
    for (int l = 0; l < MAXL; ++l) {
        level_t* v = &s->lv[l];
        free(v->cls);
        free(v->f);
        free(v->pre);
        free(v->X);
        free(v->tfc_id);
        free(v->H);
        free(v->M);
        free(v->Mring);
        free(v->G);
    }
    free(s->probes);
    free(s->probe_series);
    free(s);
}

orc_sim* orc_create(int lattice, int eq_order, int coupling, const int n0[3], int n_levels,
                    const int* boxes, double tau0, int n_probes, const int* probes,
                    long long probe_capacity, char* err, int errlen)
{
    orc_sim* s = (orc_sim*)calloc(1, sizeof(orc_sim));
#define FAIL(...)                                          \
    do {                                                   \
        if (err && errlen > 0) snprintf(err, errlen, __VA_ARGS__); \
        free_sim(s);                                       \
        return NULL;                                       \
    } while (0)
    if (!s) return NULL;
    if (make_lattice(lattice, &s->L) != 0) FAIL("bad lattice");
    if (eq_order != 2 && eq_order != 3) FAIL("eq_order must be 2 or 3");
    if (coupling != 1 && coupling != 2) FAIL("coupling must be 1 (DC1) or 2 (DC2)");
    if (n_levels < 1 || n_levels > MAXL) FAIL("n_levels out of range");
    if (!(tau0 > 0.5)) FAIL("tau0 must exceed 1/2");
    const lattice_t* L = &s->L;
    s->eq_order = eq_order;
    s->coupling = coupling;
    s->nlev = n_levels;
    s->newton_tol = 1e-12;
    s->newton_maxit = 20;
    double tau = tau0;
    for (int l = 0; l < n_levels; ++l) {
        level_t* v = &s->lv[l];
        if (l == 0) {
            for (int a = 0; a < 3; ++a) v->n[a] = a < L->D ? n0[a] : 1;
            v->periodic = 1;
            for (int a = 0; a < 3; ++a) v->off[a] = 0.0;
            for (int a = 0; a < L->D; ++a)
                if (v->n[a] < 8) FAIL("level-0 extent must be at least 8");
        } else {
            const int* b = boxes + 6 * (l - 1);
            level_t* pv = &s->lv[l - 1];
            for (int a = 0; a < 3; ++a) {
                if (a >= L->D) {
                    v->n[a] = 1;
                    v->plo[a] = 0;
                    v->off[a] = 0.0;
                    continue;
                }
                int lo = b[a], hi = b[3 + a];
                if (hi - lo < 3) FAIL("level %d box side below 3 parent cells", l);
                if (lo < 2 || hi > pv->n[a] - 1 - 2)
                    FAIL("level %d box needs a margin of 2 parent cells", l);
                v->n[a] = 2 * (hi - lo) + 1;
                v->plo[a] = lo;
                v->off[a] = pv->off[a] + lo / (double)(1 << (l - 1));
                pv->clo[a] = lo;
                pv->chi[a] = hi;
            }
            pv->has_child = 1;
        }
        v->tau = tau;
        tau = 2.0 * tau - 0.5; /* Eq.(rescTau) */
        v->N = (long long)v->n[0] * v->n[1] * v->n[2];
    }
    for (int l = 0; l < n_levels; ++l) {
        level_t* v = &s->lv[l];
        v->cls = (unsigned char*)malloc(v->N);
        v->f = (double*)malloc(sizeof(double) * v->N * L->Q);
        v->pre = (double*)malloc(sizeof(double) * v->N * L->Q);
        v->X = (double*)malloc(sizeof(double) * v->N * 4);
        if (!v->cls || !v->f || !v->pre || !v->X) FAIL("out of host memory");
        classify_level(L, v, l);
        for (long long q = 0; q < v->N * L->Q; ++q) v->f[q] = v->pre[q] = NAN;
        for (long long q = 0; q < v->N * 4; ++q) v->X[q] = NAN;
        if (v->has_child) {
            v->tfc_id = (long long*)malloc(sizeof(long long) * v->N);
            if (!v->tfc_id) FAIL("out of host memory");
            v->n_tfc = 0;
            for (long long q = 0; q < v->N; ++q) v->tfc_id[q] = v->cls[q] == C_TFC ? v->n_tfc++ : -1;
            v->H = (double*)malloc(sizeof(double) * v->n_tfc * 3 * L->Q);
            if (!v->H) FAIL("out of host memory");
            for (long long q = 0; q < v->n_tfc * 3 * L->Q; ++q) v->H[q] = NAN;
        }
    }
    /* every co-located pair must admit a valid choice of couples */
    for (int l = 1; l < n_levels; ++l) {
        level_t* v = &s->lv[l];
        for (int z = 0; z < v->n[2]; ++z)
            for (int y = 0; y < v->n[1]; ++y)
                for (int x = 0; x < v->n[0]; ++x) {
                    if (v->cls[nid(v, x, y, z)] != C_TFF) continue;
                    int k[3] = {x, y, z};
                    unsigned Kf, Kc, P, Qf, Qc, Mf, Mc, gR;
                    known_masks(s, l, k, &Kf, &Kc);
                    if (sets_from_known(L, Kf, Kc, coupling, &P, &Qf, &Qc, &Mf, &Mc, &gR) != 0)
                        FAIL("level %d node (%d,%d,%d): invalid interface sets", l, x, y, z);
                }
    }
    s->n_probes = n_probes;
    s->probe_cap = probe_capacity;
    if (n_probes > 0) {
        s->probes = (int*)malloc(sizeof(int) * 3 * n_probes);
        s->probe_series = (double*)calloc((size_t)(probe_capacity > 0 ? probe_capacity : 1) * n_probes,
                                          sizeof(double));
        if (!s->probes || !s->probe_series) FAIL("out of host memory");
        for (int p = 0; p < n_probes; ++p)
            for (int a = 0; a < 3; ++a) {
                int c = a < L->D ? probes[3 * p + a] : 0;
                if (a < L->D && (c < 0 || c >= s->lv[0].n[a])) FAIL("probe %d outside the domain", p);
                s->probes[3 * p + a] = c;
            }
    }
    return s;
#undef FAIL
}

void orc_destroy(orc_sim* s) { free_sim(s); }

/* A refined level-1 region made of level-0 cells (Sec. 3.4 closing paragraph
 * and App. B: the interface is the boundary of the region, whatever its
 * shape, and the node sets follow from which neighbours exist).  mask covers
 * the cells of level 1's box, x fastest; 1 = refined.  Reading of the node
 * classes: a level-0 node is a hole when all its incident cells are refined,
 * a co-located (TF^c) node when some are; a level-1 node is active when any
 * of its incident parent cells is refined and on the interface when not all
 * are (cells outside the box count as not refined); interface nodes with all
 * coordinates even are co-located (TF^f), the others hanging (IE).  Inactive
 * level-1 nodes are holes of that level.  Only for two levels in 2-D, before
 * any initialisation; 0 on success, -1 on a bad argument, -2 if a
 * co-located node admits no valid couples or a hanging node has no
 * co-located neighbours on its line. */
static int region_refined(const orc_sim* s, int cx, int cy)
{
    const level_t* v0 = &s->lv[0];
    const int nx = v0->chi[0] - v0->clo[0], ny = v0->chi[1] - v0->clo[1];
    if (cx < 0 || cy < 0 || cx >= nx || cy >= ny) return 0;
    return s->region[(long long)cy * nx + cx] != 0;
}

int orc_set_region(orc_sim* s, const unsigned char* mask)
{
    if (!s || !mask || s->nlev != 2 || s->L.D != 2 || s->lv[0].captures != 0) return -1;
    const lattice_t* L = &s->L;
    level_t* v0 = &s->lv[0];
    level_t* v1 = &s->lv[1];
    const int nx = v0->chi[0] - v0->clo[0], ny = v0->chi[1] - v0->clo[1];
    free(s->region);
    s->region = (unsigned char*)malloc((size_t)nx * ny);
    if (!s->region) return -1;
    memcpy(s->region, mask, (size_t)nx * ny);
    /* level 0: count the refined cells incident to each node of the closed box */
    for (int y = 0; y < v0->n[1]; ++y)
        for (int x = 0; x < v0->n[0]; ++x) {
            int c = C_BULK;
            if (x >= v0->clo[0] && x <= v0->chi[0] && y >= v0->clo[1] && y <= v0->chi[1]) {
                int r = 0;
                for (int dy = -1; dy <= 0; ++dy)
                    for (int dx = -1; dx <= 0; ++dx) r += region_refined(s, x - v0->clo[0] + dx, y - v0->clo[1] + dy);
                c = r == 4 ? C_HOLE : (r > 0 ? C_TFC : C_BULK);
            }
            v0->cls[nid(v0, x, y, 0)] = (unsigned char)c;
        }
    /* level 1: incident parent cells of fine node k: both neighbours of an
     * even coordinate, the one cell of an odd coordinate */
    for (int y = 0; y < v1->n[1]; ++y)
        for (int x = 0; x < v1->n[0]; ++x) {
            int tot = 0, r = 0;
            for (int cy = (y - 1) >> 1; cy <= y >> 1; ++cy)
                for (int cx = (x - 1) >> 1; cx <= x >> 1; ++cx) {
                    ++tot;
                    r += region_refined(s, cx, cy);
                }
            int c = C_HOLE;
            if (r > 0) c = r < tot ? ((x % 2 == 0 && y % 2 == 0) ? C_TFF : C_IE) : C_BULK;
            v1->cls[nid(v1, x, y, 0)] = (unsigned char)c;
        }
    /* the coarse co-located list and its history ring */
    v0->n_tfc = 0;
    for (long long q = 0; q < v0->N; ++q) v0->tfc_id[q] = v0->cls[q] == C_TFC ? v0->n_tfc++ : -1;
    free(v0->H);
    v0->H = (double*)malloc(sizeof(double) * (v0->n_tfc > 0 ? v0->n_tfc : 1) * 3 * L->Q);
    if (!v0->H) return -1;
    for (long long q = 0; q < v0->n_tfc * 3 * L->Q; ++q) v0->H[q] = NAN;
    for (int y = 0; y < v1->n[1]; ++y)
        for (int x = 0; x < v1->n[0]; ++x) {
            const unsigned char c = v1->cls[nid(v1, x, y, 0)];
            int k[3] = {x, y, 0};
            if (c == C_TFF) {
                unsigned Kf, Kc, P, Qf, Qc, Mf, Mc, gR;
                known_masks(s, 1, k, &Kf, &Kc);
                if (sets_from_known(L, Kf, Kc, s->coupling, &P, &Qf, &Qc, &Mf, &Mc, &gR) != 0) return -2;
            } else if (c == C_IE) {
                int pos[4];
                double w[4];
                if (region_stencil(v1, k, pos, w) < 0) return -2;
            }
        }
    return 0;
}

int orc_level_dims(const orc_sim* s, int l, int dims[3])
{
    if (l < 0 || l >= s->nlev) return -1;
    for (int a = 0; a < 3; ++a) dims[a] = s->lv[l].n[a];
    return 0;
}

int orc_level_tau(const orc_sim* s, int l, double* tau)
{
    if (l < 0 || l >= s->nlev) return -1;
    *tau = s->lv[l].tau;
    return 0;
}

int orc_classes(const orc_sim* s, int l, unsigned char* out)
{
    if (l < 0 || l >= s->nlev) return -1;
    memcpy(out, s->lv[l].cls, s->lv[l].N);
    return 0;
}

void orc_set_newton(orc_sim* s, double tol, int maxit)
{
    s->newton_tol = tol;
    s->newton_maxit = maxit;
}

void orc_plant_R(orc_sim* s, double R) { s->R_override = R; }

/* Collision model: 0 BGK, 1 H-RR with weight sigma of the projected part and
 * the cubic Mach correction on or off (Sec. 2; on refined meshes with the
 * interface gradients of Sec. 3.3).  Call before orc_init. */
int orc_set_collision(orc_sim* s, int kind, double sigma, int psi_on)
{
    if (kind != 0 && kind != 1) return -1;
    if (!(sigma >= 0.0 && sigma <= 1.0)) return -1;
    s->collision = kind;
    s->hrr_sigma = sigma;
    s->hrr_psi = psi_on ? 1 : 0;
    if (kind == 1)
        for (int l = 0; l < s->nlev; ++l) {
            level_t* v = &s->lv[l];
            if (!v->M) v->M = (double*)malloc(sizeof(double) * v->N * 4);
            if (!v->G) v->G = (double*)malloc(sizeof(double) * v->N * 18);
            if (v->has_child && !v->Mring) v->Mring = (double*)malloc(sizeof(double) * 3 * v->N * 4);
            if (!v->M || !v->G || (v->has_child && !v->Mring)) return -1;
            for (long long q = 0; q < v->N * 4; ++q) v->M[q] = NAN;
            for (long long q = 0; q < v->N * 18; ++q) v->G[q] = NAN;
            if (v->Mring)
                for (long long q = 0; q < 3 * v->N * 4; ++q) v->Mring[q] = NAN;
        }
    return 0;
}

/* rescaling factor between level l (fine) and l-1 (coarse), Eq.(fneqResc) */
static double R_of(const orc_sim* s, int l)
{
    if (s->R_override != 0.0) return s->R_override;
    return s->lv[l].tau / (2.0 * s->lv[l - 1].tau);
}

/* Initial state: populations at equilibrium with the given fields, Sec. 4.1. */
int orc_init(orc_sim* s, int l, const double* rho, const double* u)
{
    if (l < 0 || l >= s->nlev) return -1;
    const lattice_t* L = &s->L;
    level_t* v = &s->lv[l];
    for (long long q = 0; q < v->N; ++q) {
        if (v->cls[q] == C_HOLE) continue;
        double uu[3] = {0, 0, 0};
        for (int a = 0; a < L->D; ++a) uu[a] = u[a * v->N + q];
        for (int i = 0; i < L->Q; ++i) {
            double fe = feq_i(L, s->eq_order, i, rho[q], uu);
            v->f[q * L->Q + i] = fe;
            v->pre[q * L->Q + i] = fe;
        }
        v->X[q * 4 + 0] = rho[q];
        for (int a = 0; a < 3; ++a) v->X[q * 4 + 1 + a] = uu[a];
        if (v->M)
            for (int a = 0; a < 4; ++a) v->M[q * 4 + a] = v->X[q * 4 + a];
        if (v->Mring)
            for (int r = 0; r < 3; ++r)
                for (int a = 0; a < 4; ++a) v->Mring[(r * v->N + q) * 4 + a] = v->X[q * 4 + a];
        if (v->has_child && v->tfc_id[q] >= 0)
            for (int r = 0; r < 3; ++r)
                for (int i = 0; i < L->Q; ++i)
                    v->H[(v->tfc_id[q] * 3 + r) * L->Q + i] = v->f[q * L->Q + i];
    }
    v->captures = 0;
    return 0;
}

/* Streaming, Eq.(LBMequation): pre_i(x) = f_i(x - xi_i) where that node exists. */
static void stream_level(orc_sim* s, int l)
{
    const lattice_t* L = &s->L;
    level_t* v = &s->lv[l];
#pragma omp parallel for collapse(2) schedule(static)
    for (int z = 0; z < v->n[2]; ++z)
        for (int y = 0; y < v->n[1]; ++y)
            for (int x = 0; x < v->n[0]; ++x) {
                long long q = nid(v, x, y, z);
                if (v->cls[q] == C_HOLE) continue;
                int k[3] = {x, y, z};
                for (int i = 0; i < L->Q; ++i) {
                    int d[3] = {-L->xi[i][0], -L->xi[i][1], -L->xi[i][2]};
                    long long src = active_at(L, v, k, d);
                    v->pre[q * L->Q + i] = src >= 0 ? v->f[src * L->Q + i] : NAN;
                }
            }
}

/* History of the coarse populations streamed onto co-located nodes
 * (needed by Eq.(TempInt)): shift the ring and store the new values. */
static void capture_history(orc_sim* s, int l)
{
    const lattice_t* L = &s->L;
    level_t* v = &s->lv[l];
#pragma omp parallel for schedule(static)
    for (long long q = 0; q < v->N; ++q) {
        long long t = v->tfc_id[q];
        if (t < 0) continue;
        double* H = v->H + t * 3 * L->Q;
        for (int i = 0; i < L->Q; ++i) {
            H[0 * L->Q + i] = H[1 * L->Q + i];
            H[1 * L->Q + i] = H[2 * L->Q + i];
            H[2 * L->Q + i] = v->pre[q * L->Q + i];
        }
    }
    if (v->Mring) {
        /* H-RR: the post-streaming macroscopic fields of the whole level at
         * the same coarse times, for the coarse-stencil gradients of the
         * child's co-located nodes (Sec. 3.3); only nodes outside the child
         * box are read, and their populations are complete */
#pragma omp parallel for schedule(static)
        for (long long q = 0; q < v->N; ++q) {
            double* R0 = v->Mring + q * 4;
            double* R1 = v->Mring + (v->N + q) * 4;
            double* R2 = v->Mring + (2 * v->N + q) * 4;
            for (int a = 0; a < 4; ++a) {
                R0[a] = R1[a];
                R1[a] = R2[a];
            }
            const double* pre = v->pre + q * L->Q;
            double r = 0.0, j[3] = {0, 0, 0};
            for (int i = 0; i < L->Q; ++i) {
                r += pre[i];
                for (int a = 0; a < L->D; ++a) j[a] += L->xi[i][a] * pre[i];
            }
            R2[0] = r;
            for (int a = 0; a < 3; ++a) R2[1 + a] = a < L->D ? j[a] / r : 0.0;
        }
    }
    v->captures += 1;
}

/* Eq.(TempInt): coarse value seen by a fine substep.  substep 1 (asynchronous)
 * sits half-way between coarse times t and t+dt^c: quadratic Lagrange
 * interpolation through t-dt^c, t, t+dt^c; when the coarse level has made a
 * single step there is no t-dt^c value and the linear mean is used.
 * substep 2 (synchronous) coincides with t+dt^c. */
static double time_interp(long long captures, int substep, double Hm, double H0, double Hp)
{
    if (substep == 2) return Hp;
    if (captures <= 1) return 0.5 * H0 + 0.5 * Hp;
    return -0.125 * Hm + 0.75 * H0 + 0.375 * Hp;
}

static void coarse_input(const orc_sim* s, int lc, long long tfc, int substep, double* g)
{
    const lattice_t* L = &s->L;
    const level_t* cv = &s->lv[lc];
    const double* H = cv->H + tfc * 3 * L->Q;
    for (int i = 0; i < L->Q; ++i)
        g[i] = time_interp(cv->captures, substep, H[i], H[L->Q + i], H[2 * L->Q + i]);
}

/* Steps 2d-2e / 3c: Newton for X at each TF^f node of level l, then rebuild
 * every direction coupled to the coarse grid with Eq.(rescff). */
static int reconstruct_tf(orc_sim* s, int l, int substep)
{
    const lattice_t* L = &s->L;
    level_t* v = &s->lv[l];
    level_t* cv = &s->lv[l - 1];
    double R = R_of(s, l);
    int failed = 0;
    long long calls = 0;
    int max_iters = s->newton_max_iters;
#pragma omp parallel for collapse(2) schedule(dynamic, 4) reduction(+ : calls) reduction(max : max_iters)
    for (int z = 0; z < v->n[2]; ++z)
        for (int y = 0; y < v->n[1]; ++y)
            for (int x = 0; x < v->n[0]; ++x) {
                long long q = nid(v, x, y, z);
                if (v->cls[q] != C_TFF) continue;
                int k[3] = {x, y, z};
                unsigned Kf, Kc, P, Qf, Qc, Mf, Mc, gR = 0;
                known_masks(s, l, k, &Kf, &Kc);
                sets_from_known(L, Kf, Kc, s->coupling, &P, &Qf, &Qc, &Mf, &Mc, &gR);
                int p[3] = {0, 0, 0};
                for (int a = 0; a < L->D; ++a) p[a] = v->plo[a] + k[a] / 2;
                long long pq = nid(cv, p[0], p[1], p[2]);
                double g[MAXQ], h[MAXQ], G[MAXQ], X[4];
                coarse_input(s, l - 1, cv->tfc_id[pq], substep, g);
                double* pre = v->pre + q * L->Q;
                for (int i = 0; i < L->Q; ++i) {
                    int coarse = (gR >> i) & 1u;
                    G[i] = coarse ? R : 1.0;
                    h[i] = coarse ? g[i] : pre[i];
                }
                int iters = 0;
                int rc = newton(L, s->eq_order, h, G, s->newton_tol, s->newton_maxit, X, &iters);
                calls++;
                if (iters > max_iters) max_iters = iters;
#pragma omp atomic
                s->newton_iter_hist[iters < 7 ? iters : 7]++;
                if (rc != 0) {
#pragma omp atomic write
                    failed = 1;
                    continue;
                }
                double u[3] = {X[1], X[2], X[3]};
                for (int i = 0; i < L->Q; ++i) {
                    if (!((gR >> i) & 1u)) continue;
                    double fe = feq_i(L, s->eq_order, i, X[0], u);
                    pre[i] = fe + R * (g[i] - fe);
                }
                for (int a = 0; a < 4; ++a) v->X[q * 4 + a] = X[a];
            }
    s->newton_calls += calls;
    s->newton_max_iters = max_iters;
    if (failed) {
        s->error = 1;
        return -1;
    }
    return 0;
}

/* Steps 2g / 3e: complete the hanging (IE) nodes by 1-D interpolation of the
 * completed co-located values along the interface line(s). */
static void interpolate_ie(orc_sim* s, int l)
{
    const lattice_t* L = &s->L;
    level_t* v = &s->lv[l];
#pragma omp parallel for collapse(2) schedule(static)
    for (int z = 0; z < v->n[2]; ++z)
        for (int y = 0; y < v->n[1]; ++y)
            for (int x = 0; x < v->n[0]; ++x) {
                long long q = nid(v, x, y, z);
                if (v->cls[q] != C_IE) continue;
                int k[3] = {x, y, z};
                /* odd axes carry a 1-D stencil, even axes a single point */
                int npts[3], pos[3][4];
                double w[3][4];
                for (int a = 0; a < 3; ++a) {
                    if (a < L->D && (k[a] % 2)) {
                        npts[a] = 4;
                        if (s->region)
                            region_stencil(v, k, pos[a], w[a]);
                        else
                            line_stencil(k[a], v->n[a] - 1, pos[a], w[a]);
                    } else {
                        npts[a] = 1;
                        pos[a][0] = k[a];
                        w[a][0] = 1.0;
                    }
                }
                for (int i = 0; i < L->Q; ++i) {
                    int d[3] = {-L->xi[i][0], -L->xi[i][1], -L->xi[i][2]};
                    if (active_at(L, v, k, d) >= 0) continue; /* streamed: known */
                    double acc = 0.0;
                    for (int c = 0; c < npts[2]; ++c)
                        for (int b = 0; b < npts[1]; ++b)
                            for (int a = 0; a < npts[0]; ++a) {
                                long long sq = nid(v, pos[0][a], pos[1][b], pos[2][c]);
                                acc += w[0][a] * w[1][b] * w[2][c] * v->pre[sq * L->Q + i];
                            }
                    v->pre[q * L->Q + i] = acc;
                }
            }
}

/* Step 3f: coarse co-located populations rebuilt from the completed fine
 * ones, Eq.(rescfc), for all directions; the coarse copy takes X. */
static void restrict_tfc(orc_sim* s, int l)
{
    const lattice_t* L = &s->L;
    level_t* v = &s->lv[l];
    level_t* fv = &s->lv[l + 1];
    double R = R_of(s, l + 1);
#pragma omp parallel for collapse(2) schedule(static)
    for (int z = 0; z < v->n[2]; ++z)
        for (int y = 0; y < v->n[1]; ++y)
            for (int x = 0; x < v->n[0]; ++x) {
                long long q = nid(v, x, y, z);
                if (v->cls[q] != C_TFC) continue;
                int k[3] = {0, 0, 0}, xyz[3] = {x, y, z};
                for (int a = 0; a < L->D; ++a) k[a] = 2 * (xyz[a] - v->clo[a]);
                long long fq = nid(fv, k[0], k[1], k[2]);
                const double* X = fv->X + fq * 4;
                double u[3] = {X[1], X[2], X[3]};
                for (int i = 0; i < L->Q; ++i) {
                    double fe = feq_i(L, s->eq_order, i, X[0], u);
                    v->pre[q * L->Q + i] = fe + (fv->pre[fq * L->Q + i] - fe) / R;
                }
                for (int a = 0; a < 4; ++a) v->X[q * 4 + a] = X[a];
            }
}

/* ------------------------------------------------------------------------- */
/* H-RR collision, Sec. 2 (one periodic level).  For every node, from the     */
/* post-streaming populations of the level and its macroscopic fields:       */
/*   psi_i = -w_i/(2c^4) H2_i:(div Psi)           (App. A, Eq.(psi); the     */
/*           sign that cancels the lattice's missing third-order moments)    */
/*   a1PR  = sum_i H2_i (f_i - f0_i + psi_i/2)    (Eq.(a1Proj))               */
/*   a1FD  = -tau rho c^2 (d_b u_a + d_a u_b)     (Eq.(a1FD_scheme))          */
/*   a1    = sigma a1PR + (1 - sigma) a1FD        (Eq.(a12_HRR))              */
/*   a1^(3)_aab = 2 u_a a1_ab + u_b a1_aa         (Eq.(a13RR))                */
/*   f1reg_i = w_i [H2_i:a1/(2c^4) + sum_{a!=b} H3_{i,aab} a1^(3)_aab/(2c^6)] */
/*   f*_i  = f0_i + (1 - 1/tau) f1reg_i + psi_i/2 (Eq.(LBMscheme_reg))        */
/* with centred differences over the periodic neighbours (Eq.(PSI_FD)) and   */
/* Psi the third-order moments of the Maxwell-Boltzmann distribution minus   */
/* those of the lattice equilibrium: rho u_a^3 on aaa, and in D3Q19          */
/* rho u_b u_g^2 / 2 on aab (g the third axis) and rho u_x u_y u_z on xyz.   */
/* ------------------------------------------------------------------------- */
static double H2(const lattice_t* L, int i, int a, int b)
{
    return (double)(L->xi[i][a] * L->xi[i][b]) - (a == b ? L->cs2 : 0.0);
}

/* Psi_abg at one node from its macroscopic state (symmetric in a, b, g). */
static double Psi(const lattice_t* L, double rho, const double u[3], int a, int b, int g)
{
    int n[3] = {0, 0, 0};
    n[a]++;
    n[b]++;
    n[g]++;
    if (n[0] == 3 || n[1] == 3 || n[2] == 3) return rho * u[a] * u[a] * u[a];
    if (L->D == 2) return 0.0;
    if (n[0] == 1 && n[1] == 1 && n[2] == 1) return rho * u[0] * u[1] * u[2];
    /* two equal indices: Psi_aab = rho u_b u_g^2 / 2, g the axis not in {a, b} */
    int dbl = n[0] == 2 ? 0 : (n[1] == 2 ? 1 : 2);
    int sgl = n[0] == 1 ? 0 : (n[1] == 1 ? 1 : 2);
    int third = 3 - dbl - sgl;
    return 0.5 * rho * u[sgl] * u[third] * u[third];
}

/* Macroscopic fields of every active node of level l at the current time:
 * co-located nodes (TF^f, TF^c) carry X, the others the moments of their
 * post-streaming (completed) populations. */
static void hrr_macros(orc_sim* s, int l)
{
    const lattice_t* L = &s->L;
    level_t* v = &s->lv[l];
#pragma omp parallel for schedule(static)
    for (long long q = 0; q < v->N; ++q) {
        const unsigned char c = v->cls[q];
        double* M = v->M + q * 4;
        if (c == C_HOLE) {
            for (int a = 0; a < 4; ++a) M[a] = NAN;
            continue;
        }
        if (c == C_TFF || c == C_TFC) {
            for (int a = 0; a < 4; ++a) M[a] = v->X[q * 4 + a];
            continue;
        }
        const double* pre = v->pre + q * L->Q;
        double r = 0.0, j[3] = {0, 0, 0};
        for (int i = 0; i < L->Q; ++i) {
            r += pre[i];
            for (int a = 0; a < L->D; ++a) j[a] += L->xi[i][a] * pre[i];
        }
        M[0] = r;
        for (int a = 0; a < 3; ++a) M[1 + a] = a < L->D ? j[a] / r : 0.0;
    }
}

/* (rho, u) of the parent node P of level l's co-located node stencil at the
 * time of level l's substep: the parent's post-streaming fields interpolated
 * with the weights of Eq.(TempInt) (the reading of the ring as for the
 * populations), Sec. 3.3. */
static void parent_macros(const orc_sim* s, int l, int substep, const int P[3], double out[4])
{
    const level_t* pv = &s->lv[l - 1];
    const long long q = nid(pv, P[0], P[1], P[2]);
    for (int a = 0; a < 4; ++a)
        out[a] = time_interp(pv->captures, substep, pv->Mring[q * 4 + a], pv->Mring[(pv->N + q) * 4 + a],
                             pv->Mring[(2 * pv->N + q) * 4 + a]);
}

/* Gradient tensors of one node from the macroscopic fields at its stencil
 * points, at distance h (level-l units) on either side along each axis:
 *   G[0][a][b] = d_b u_a,   G[1][a][b] = sum_g d_g Psi_abg,
 * centred differences (v(+) - v(-)) / (2 h), Eq.(a1FD_scheme), Eq.(PSI_FD).
 * Mm[b], Mp[b] are the (rho, u) at the points -h e_b and +h e_b. */
static void stencil_gradients(const lattice_t* L, double h, const double Mm[3][4], const double Mp[3][4],
                              double G[2][3][3])
{
    for (int t = 0; t < 2; ++t)
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) G[t][a][b] = 0.0;
    for (int b = 0; b < L->D; ++b)
        for (int a = 0; a < L->D; ++a) G[0][a][b] = (Mp[b][1 + a] - Mm[b][1 + a]) / (2.0 * h);
    for (int a = 0; a < L->D; ++a)
        for (int b = 0; b < L->D; ++b)
            for (int g = 0; g < L->D; ++g)
                G[1][a][b] += (Psi(L, Mp[g][0], Mp[g] + 1, a, b, g) - Psi(L, Mm[g][0], Mm[g] + 1, a, b, g)) / (2.0 * h);
}

/* Gradients of every active node of level l (H-RR), from the fields of
 * hrr_macros and of the neighbouring levels:
 *  - bulk nodes and coarse co-located (TF^c) nodes: the level's own stencil,
 *    h = 1 (periodic on level 0); a neighbour in the hole takes the child's
 *    node co-located with it at the same time (Sec. 3.5 step 3d: the coarse
 *    strain tensor on TF^c);
 *  - fine co-located (TF^f) nodes: the coarse stencil, h = 2 (Sec. 3.3,
 *    Fig. gradC): points inside the level are its own nodes, points outside
 *    are parent nodes at the substep's time (interpolated in time at the
 *    asynchronous substep, Sec. 3.5 step 2f); differences over 2h = 4 fine
 *    cells give the fine-scale values S^c / 2 and psi^c / 2 of
 *    Eq.(PijResc) and Eq.(PSIResc) directly;
 *  - hanging (IE) nodes: interpolated from the TF^f nodes of their line
 *    stencil with the weights of their populations (Sec. 3.5 steps 2g/3e). */
static void hrr_gradients(orc_sim* s, int l, int substep)
{
    const lattice_t* L = &s->L;
    level_t* v = &s->lv[l];
#pragma omp parallel for collapse(2) schedule(static)
    for (int z = 0; z < v->n[2]; ++z)
        for (int y = 0; y < v->n[1]; ++y)
            for (int x = 0; x < v->n[0]; ++x) {
                const long long q = nid(v, x, y, z);
                const unsigned char c = v->cls[q];
                if (c == C_HOLE || c == C_IE) continue;
                const int k[3] = {x, y, z};
                double Mm[3][4], Mp[3][4];
                const int h = c == C_TFF ? 2 : 1;
                for (int b = 0; b < L->D; ++b)
                    for (int sgn = -1; sgn <= 1; sgn += 2) {
                        double* out = sgn < 0 ? Mm[b] : Mp[b];
                        int d[3] = {0, 0, 0};
                        d[b] = sgn * h;
                        int kk[3] = {k[0] + d[0], k[1] + d[1], k[2] + d[2]};
                        /* a point of a fine co-located node's stencil outside the level,
                         * or (refined regions) on a missing node of it, is a parent node:
                         * its fine partner would exist if it were co-located or a hole,
                         * so it is a bulk node of the parent */
                        if (c == C_TFF && (kk[b] < 0 || kk[b] > v->n[b] - 1 || active_at(L, v, k, d) < 0)) {
                            int P[3] = {0, 0, 0};
                            for (int a = 0; a < L->D; ++a) P[a] = v->plo[a] + k[a] / 2;
                            P[b] += sgn;
                            parent_macros(s, l, substep, P, out);
                            continue;
                        }
                        const long long nq = active_at(L, v, k, d);
                        if (nq >= 0) {
                            for (int a = 0; a < 4; ++a) out[a] = v->M[nq * 4 + a];
                            continue;
                        }
                        /* a hole: the child's co-located node */
                        const level_t* cv = &s->lv[l + 1];
                        int kc[3] = {0, 0, 0};
                        for (int a = 0; a < L->D; ++a) kc[a] = 2 * (kk[a] - v->clo[a]);
                        const long long cq = nid(cv, kc[0], kc[1], kc[2]);
                        for (int a = 0; a < 4; ++a) out[a] = cv->M[cq * 4 + a];
                    }
                double G[2][3][3];
                stencil_gradients(L, (double)h, Mm, Mp, G);
                memcpy(v->G + q * 18, G, sizeof(G));
            }
    if (l == 0) return;
#pragma omp parallel for collapse(2) schedule(static)
    for (int z = 0; z < v->n[2]; ++z)
        for (int y = 0; y < v->n[1]; ++y)
            for (int x = 0; x < v->n[0]; ++x) {
                const long long q = nid(v, x, y, z);
                if (v->cls[q] != C_IE) continue;
                const int k[3] = {x, y, z};
                int npts[3], pos[3][4];
                double w[3][4];
                for (int a = 0; a < 3; ++a) {
                    if (a < L->D && (k[a] % 2)) {
                        npts[a] = 4;
                        if (s->region)
                            region_stencil(v, k, pos[a], w[a]);
                        else
                            line_stencil(k[a], v->n[a] - 1, pos[a], w[a]);
                    } else {
                        npts[a] = 1;
                        pos[a][0] = k[a];
                        w[a][0] = 1.0;
                    }
                }
                double* G = v->G + q * 18;
                for (int e = 0; e < 18; ++e) G[e] = 0.0;
                for (int cc = 0; cc < npts[2]; ++cc)
                    for (int bb = 0; bb < npts[1]; ++bb)
                        for (int aa = 0; aa < npts[0]; ++aa) {
                            const long long sq = nid(v, pos[0][aa], pos[1][bb], pos[2][cc]);
                            const double wt = w[0][aa] * w[1][bb] * w[2][cc];
                            for (int e = 0; e < 18; ++e) G[e] += wt * v->G[sq * 18 + e];
                        }
            }
}

/* The H-RR collision of every active node of level l from its completed
 * pre-collision populations, its macroscopic fields (X at co-located nodes)
 * and its gradients. */
static void collide_level_hrr(orc_sim* s, int l, int substep)
{
    const lattice_t* L = &s->L;
    level_t* v = &s->lv[l];
    const int D = L->D, Q = L->Q;
    const double c2 = L->cs2, tau = v->tau;
    hrr_macros(s, l);
    hrr_gradients(s, l, substep);
#pragma omp parallel for schedule(static)
    for (long long q = 0; q < v->N; ++q) {
        if (v->cls[q] == C_HOLE) continue;
        const double* pre = v->pre + q * Q;
        const double rho = v->M[q * 4];
        const double uq[3] = {v->M[q * 4 + 1], v->M[q * 4 + 2], v->M[q * 4 + 3]};
        double G[2][3][3];
        memcpy(G, v->G + q * 18, sizeof(G));
        double f0[MAXQ], psi[MAXQ], a1[3][3] = {{0}};
        for (int i = 0; i < Q; ++i) {
            f0[i] = feq_i(L, s->eq_order, i, rho, uq);
            double t = 0.0;
            if (s->hrr_psi)
                for (int a = 0; a < D; ++a)
                    for (int b = 0; b < D; ++b) t += H2(L, i, a, b) * G[1][a][b];
            psi[i] = -L->w[i] / (2.0 * c2 * c2) * t;
        }
        for (int a = 0; a < D; ++a)
            for (int b = 0; b < D; ++b) {
                double pr = 0.0;
                for (int i = 0; i < Q; ++i) pr += H2(L, i, a, b) * (pre[i] - f0[i] + 0.5 * psi[i]);
                const double fd = -tau * rho * c2 * (G[0][a][b] + G[0][b][a]);
                a1[a][b] = s->hrr_sigma * pr + (1.0 - s->hrr_sigma) * fd;
            }
        for (int i = 0; i < Q; ++i) {
            double t2 = 0.0, t3 = 0.0;
            for (int a = 0; a < D; ++a)
                for (int b = 0; b < D; ++b) t2 += H2(L, i, a, b) * a1[a][b];
            for (int a = 0; a < D; ++a)
                for (int b = 0; b < D; ++b) {
                    if (a == b) continue;
                    const double H3 = (double)(L->xi[i][a] * L->xi[i][a] * L->xi[i][b]) - c2 * L->xi[i][b];
                    const double a13 = 2.0 * uq[a] * a1[a][b] + uq[b] * a1[a][a];
                    t3 += H3 * a13;
                }
            const double f1 = L->w[i] * (t2 / (2.0 * c2 * c2) + t3 / (2.0 * c2 * c2 * c2));
            v->f[q * Q + i] = f0[i] + (1.0 - 1.0 / tau) * f1 + 0.5 * psi[i];
        }
    }
}

/* Gradient tensors of level l from the current state (test access). */
int orc_hrr_gradients(orc_sim* s, int l, int substep, double* out)
{
    if (s->collision != 1 || l < 0 || l >= s->nlev) return -1;
    level_t* v = &s->lv[l];
    /* the finer levels first: a coarse co-located node reads its child's fields */
    for (int k = s->nlev - 1; k >= l; --k) hrr_macros(s, k);
    hrr_gradients(s, l, substep);
    memcpy(out, v->G, sizeof(double) * v->N * 18);
    return 0;
}

/* BGK collision of every active node of level l; co-located nodes use X. */
static void collide_level(orc_sim* s, int l, int substep)
{
    if (s->collision == 1) {
        collide_level_hrr(s, l, substep);
        return;
    }
    const lattice_t* L = &s->L;
    level_t* v = &s->lv[l];
    double omega = 1.0 / v->tau;
#pragma omp parallel for schedule(static)
    for (long long q = 0; q < v->N; ++q) {
        unsigned char c = v->cls[q];
        if (c == C_HOLE) continue;
        const double* pre = v->pre + q * L->Q;
        double rho, u[3] = {0, 0, 0};
        if (c == C_TFF || c == C_TFC) {
            rho = v->X[q * 4];
            for (int a = 0; a < 3; ++a) u[a] = v->X[q * 4 + 1 + a];
        } else {
            double j[3] = {0, 0, 0};
            rho = 0.0;
            for (int i = 0; i < L->Q; ++i) {
                rho += pre[i];
                for (int a = 0; a < L->D; ++a) j[a] += L->xi[i][a] * pre[i];
            }
            for (int a = 0; a < L->D; ++a) u[a] = j[a] / rho;
        }
        for (int i = 0; i < L->Q; ++i) {
            double fe = feq_i(L, s->eq_order, i, rho, u);
            v->f[q * L->Q + i] = fe + (1.0 - omega) * (pre[i] - fe);
        }
    }
}

/* Absorbing layer (the paper only cites one, for its convected-vortex runs,
 * Sec. 4.2.1; reading): on level 0, at nodes within W cells of the periodic
 * seam, after the collision
 *   f_i <- f_i - sigma(x) (f0_i(rho, u) - f0_i(1, u_t)),
 * (rho, u) the node's moments, u_t the target velocity, with the strength
 * sigma(x) = sigma_max ((W - e) / W)^2, e = min over the axes of the node's
 * distance in cells to the nearest outermost node of the domain (0 there).
 * The moments are driven towards (1, u_t) and the deviation from the target
 * equilibrium shrinks by 1 - sigma each step; outside the layer nothing
 * changes. */
static double sponge_strength(const orc_sim* s, const int k[3])
{
    const level_t* v = &s->lv[0];
    int e = v->n[0];
    for (int a = 0; a < s->L.D; ++a) {
        const int ea = k[a] < v->n[a] - 1 - k[a] ? k[a] : v->n[a] - 1 - k[a];
        if (ea < e) e = ea;
    }
    if (e >= s->sponge_w) return 0.0;
    const double r = (double)(s->sponge_w - e) / (double)s->sponge_w;
    return s->sponge_sigma * r * r;
}

static void sponge_level0(orc_sim* s)
{
    const lattice_t* L = &s->L;
    level_t* v = &s->lv[0];
    double fet[MAXQ];
    for (int i = 0; i < L->Q; ++i) fet[i] = feq_i(L, s->eq_order, i, 1.0, s->sponge_u);
#pragma omp parallel for collapse(2) schedule(static)
    for (int z = 0; z < v->n[2]; ++z)
        for (int y = 0; y < v->n[1]; ++y)
            for (int x = 0; x < v->n[0]; ++x) {
                const int k[3] = {x, y, z};
                const long long q = nid(v, x, y, z);
                if (v->cls[q] == C_HOLE) continue;
                const double sig = sponge_strength(s, k);
                if (sig == 0.0) continue;
                double* f = v->f + q * L->Q;
                double rho = 0.0, j[3] = {0, 0, 0}, u[3] = {0, 0, 0};
                for (int i = 0; i < L->Q; ++i) {
                    rho += f[i];
                    for (int a = 0; a < L->D; ++a) j[a] += L->xi[i][a] * f[i];
                }
                for (int a = 0; a < L->D; ++a) u[a] = j[a] / rho;
                for (int i = 0; i < L->Q; ++i) f[i] -= sig * (feq_i(L, s->eq_order, i, rho, u) - fet[i]);
            }
}

int orc_set_sponge(orc_sim* s, int width, double sigma_max, const double* u_target)
{
    if (!s || width < 0 || !(sigma_max >= 0.0 && sigma_max <= 1.0)) return -1;
    const level_t* v = &s->lv[0];
    for (int a = 0; a < s->L.D; ++a)
        if (2 * width >= v->n[a]) return -1;
    if (s->nlev > 1) {
        /* the child's closed box must lie outside the layer */
        for (int a = 0; a < s->L.D; ++a)
            if (v->clo[a] < width || v->chi[a] > v->n[a] - 1 - width) return -1;
    }
    s->sponge_w = width;
    s->sponge_sigma = sigma_max;
    for (int a = 0; a < 3; ++a) s->sponge_u[a] = (u_target && a < s->L.D) ? u_target[a] : 0.0;
    return 0;
}

/* One step of level l; substep = 1 (asynchronous) or 2 (synchronous) with
 * respect to the parent, 0 on level 0.  Each level advances twice per step of
 * its parent (acoustic scaling, Sec. 3.1), recursively. */
static int advance(orc_sim* s, int l, int substep)
{
    level_t* v = &s->lv[l];
    stream_level(s, l);                       /* 2a-2c / 3a-3b */
    if (v->has_child) capture_history(s, l);
    if (l > 0) {
        if (reconstruct_tf(s, l, substep) != 0) return -1; /* 2d-2e / 3c */
        interpolate_ie(s, l);                 /* 2g / 3e */
    }
    if (v->has_child) {
        if (advance(s, l + 1, 1) != 0) return -1;
        if (advance(s, l + 1, 2) != 0) return -1;
        restrict_tfc(s, l);                   /* 3f */
    }
    collide_level(s, l, substep);             /* 2h / 3g */
    if (l == 0 && s->sponge_w > 0) sponge_level0(s);
    return 0;
}

/* Probe p' = c_s^2 (rho - 1) with rho the post-collision density, taken on
 * the finest level whose closed box contains the point. */
static void probe_sample(orc_sim* s)
{
    const lattice_t* L = &s->L;
    if (s->n_probes == 0 || s->probe_len >= s->probe_cap) return;
    for (int p = 0; p < s->n_probes; ++p) {
        int* c = s->probes + 3 * p;
        double val = NAN;
        for (int l = s->nlev - 1; l >= 0; --l) {
            const level_t* v = &s->lv[l];
            int k[3] = {0, 0, 0}, inside = 1;
            for (int a = 0; a < L->D; ++a) {
                double kk = (c[a] - v->off[a]) * (double)(1 << l);
                if (kk < -1e-9 || kk > v->n[a] - 1 + 1e-9) inside = 0;
                k[a] = (int)floor(kk + 0.5);
            }
            if (!inside) continue;
            long long q = nid(v, k[0], k[1], k[2]);
            if (v->cls[q] == C_HOLE) continue;
            double rho = 0.0;
            for (int i = 0; i < L->Q; ++i) rho += v->f[q * L->Q + i];
            val = L->cs2 * (rho - 1.0);
            break;
        }
        s->probe_series[s->probe_len * s->n_probes + p] = val;
    }
    s->probe_len++;
}

int orc_run(orc_sim* s, long long n_coarse_steps)
{
    for (long long t = 0; t < n_coarse_steps; ++t) {
        if (advance(s, 0, 0) != 0) return -1;
        s->coarse_steps++;
        probe_sample(s);
    }
    return s->error ? -1 : 0;
}

static int get_field(const orc_sim* s, int l, const double* src, int ncomp, double* out)
{
    if (l < 0 || l >= s->nlev) return -1;
    const level_t* v = &s->lv[l];
    for (long long q = 0; q < v->N; ++q)
        for (int i = 0; i < ncomp; ++i)
            out[(long long)i * v->N + q] = v->cls[q] == C_HOLE ? NAN : src[q * ncomp + i];
    return 0;
}

int orc_get_f(const orc_sim* s, int l, double* out) { return get_field(s, l, s->lv[l].f, s->L.Q, out); }
int orc_get_pre(const orc_sim* s, int l, double* out) { return get_field(s, l, s->lv[l].pre, s->L.Q, out); }

int orc_get_x(const orc_sim* s, int l, double* out)
{
    if (l < 0 || l >= s->nlev) return -1;
    const level_t* v = &s->lv[l];
    for (long long q = 0; q < v->N; ++q)
        for (int a = 0; a < 4; ++a) {
            int shared = v->cls[q] == C_TFF || v->cls[q] == C_TFC;
            out[(long long)a * v->N + q] = shared ? v->X[q * 4 + a] : NAN;
        }
    return 0;
}

int orc_set_f(orc_sim* s, int l, const double* in)
{
    if (l < 0 || l >= s->nlev) return -1;
    level_t* v = &s->lv[l];
    for (long long q = 0; q < v->N; ++q)
        for (int i = 0; i < s->L.Q; ++i) v->f[q * s->L.Q + i] = in[(long long)i * v->N + q];
    return 0;
}

long long orc_get_probes(const orc_sim* s, double* out)
{
    if (out) memcpy(out, s->probe_series, sizeof(double) * s->probe_len * s->n_probes);
    return s->probe_len;
}

/* FP64 mass, momentum and kinetic energy over the nodes each level owns
 * (the finest level containing a point owns it), weighted by cell volume. */
int orc_balance(const orc_sim* s, double out[5])
{
    const lattice_t* L = &s->L;
    for (int a = 0; a < 5; ++a) out[a] = 0.0;
    for (int l = 0; l < s->nlev; ++l) {
        const level_t* v = &s->lv[l];
        double vol = 1.0;
        for (int a = 0; a < L->D; ++a) vol /= (double)(1 << l);
        for (long long q = 0; q < v->N; ++q) {
            if (v->cls[q] == C_HOLE || v->cls[q] == C_TFC) continue;
            double rho = 0.0, j[3] = {0, 0, 0};
            for (int i = 0; i < L->Q; ++i) {
                double fi = v->f[q * L->Q + i];
                rho += fi;
                for (int a = 0; a < L->D; ++a) j[a] += L->xi[i][a] * fi;
            }
            out[0] += vol * rho;
            double e = 0.0;
            for (int a = 0; a < L->D; ++a) {
                out[1 + a] += vol * j[a];
                e += j[a] * j[a];
            }
            out[4] += vol * 0.5 * e / rho;
        }
    }
    return 0;
}

/* Threads the node loops run on: the OpenMP thread count when built with
 * OpenMP (the CPU-baseline build), else 1.  Every node's arithmetic is the
 * same either way; only the loops over independent nodes are shared out. */
int orc_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Thread count of the node loops (OpenMP builds only; a no-op otherwise). */
void orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

void orc_newton_stats(const orc_sim* s, long long* calls, int* max_iters, long long hist[8])
{
    *calls = s->newton_calls;
    *max_iters = s->newton_max_iters;
    for (int k = 0; k < 8; ++k) hist[k] = s->newton_iter_hist[k];
}

/* ---------------- stand-alone pieces, for pinning ---------------- */

int orc_lattice(int lattice, int* Q, int* D, int* xi, double* w)
{
    lattice_t L;
    if (make_lattice(lattice, &L) != 0) return -1;
    *Q = L.Q;
    *D = L.D;
    for (int i = 0; i < L.Q; ++i) {
        for (int a = 0; a < 3; ++a) xi[3 * i + a] = L.xi[i][a];
        w[i] = L.w[i];
    }
    return 0;
}

int orc_feq(int lattice, int eq_order, double rho, const double* u, double* out)
{
    lattice_t L;
    if (make_lattice(lattice, &L) != 0) return -1;
    double uu[3] = {0, 0, 0};
    for (int a = 0; a < L.D; ++a) uu[a] = u[a];
    for (int i = 0; i < L.Q; ++i) out[i] = feq_i(&L, eq_order, i, rho, uu);
    return 0;
}

int orc_newton(int lattice, int eq_order, const double* h, const double* G, double tol, int maxit,
               double* X, int* iters)
{
    lattice_t L;
    if (make_lattice(lattice, &L) != 0) return -1;
    return newton(&L, eq_order, h, G, tol, maxit, X, iters);
}

int orc_residual(int lattice, int eq_order, const double* h, const double* G, const double* X, double* F)
{
    lattice_t L;
    if (make_lattice(lattice, &L) != 0) return -1;
    double XX[4] = {X[0], X[1], X[2], L.D == 3 ? X[3] : 0.0};
    residual(&L, eq_order, h, G, XX, F);
    return 0;
}

int orc_sets(int lattice, unsigned Kf, unsigned Kc, int coupling, unsigned out[6])
{
    lattice_t L;
    if (make_lattice(lattice, &L) != 0) return -1;
    return sets_from_known(&L, Kf, Kc, coupling, &out[0], &out[1], &out[2], &out[3], &out[4], &out[5]);
}

int orc_node_masks(const orc_sim* s, int l, const int k[3], unsigned* Kf, unsigned* Kc)
{
    if (l < 1 || l >= s->nlev) return -1;
    const level_t* v = &s->lv[l];
    for (int a = 0; a < 3; ++a)
        if (k[a] < 0 || k[a] >= v->n[a]) return -1;
    if (v->cls[nid(v, k[0], k[1], k[2])] != C_TFF) return -2;
    known_masks(s, l, k, Kf, Kc);
    return 0;
}

void orc_line_stencil(int k, int N, int* pos, double* w) { line_stencil(k, N, pos, w); }

double orc_time_interp(long long captures, int substep, double Hm, double H0, double Hp)
{
    return time_interp(captures, substep, Hm, H0, Hp);
}
