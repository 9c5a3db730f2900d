/*
 * dclbm_oracle.h -- TEST INFRASTRUCTURE: the FP64 CPU oracle of the
 * direct-coupling lattice Boltzmann step (arXiv:2004.14887).  Used only by the
 * test suite, the smoke check and the benchmark's CPU-baseline leg; the HIP
 * library never includes or links this.
 */
#ifndef DCLBM_ORACLE_H
#define DCLBM_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_D2Q9 = 0, ORC_D3Q19 = 1 };

typedef struct orc_sim orc_sim;

/* boxes: (n_levels-1) x {lo[3], hi[3]}, each in the parent level's node
 * coordinates; probes: n_probes x 3 level-0 node coordinates. */
orc_sim* orc_create(int lattice, int eq_order, int coupling, const int n0[3], int n_levels,
                    const int* boxes, double tau0, int n_probes, const int* probes,
                    long long probe_capacity, char* err, int errlen);
void orc_destroy(orc_sim* s);
int orc_level_dims(const orc_sim* s, int l, int dims[3]);
int orc_level_tau(const orc_sim* s, int l, double* tau);
int orc_classes(const orc_sim* s, int l, unsigned char* out);
void orc_set_newton(orc_sim* s, double tol, int maxit);
void orc_plant_R(orc_sim* s, double R);
int orc_set_collision(orc_sim* s, int kind, double sigma, int psi_on);
/* Absorbing layer on level 0: width in cells, strength 0..1 at the domain's
 * outermost nodes, target velocity [3] (target density 1).  The child's box
 * must lie outside the layer.  0 on success, -1 on a bad argument. */
int orc_set_sponge(orc_sim* s, int width, double sigma_max, const double* u_target);
/* Refined region of level 1 as a mask of level-0 cells over its box (x
 * fastest, 1 = refined); two levels, 2-D, BGK, before initialisation.
 * 0 on success, -1 on a bad argument, -2 on a region the coupling cannot
 * handle. */
int orc_set_region(orc_sim* s, const unsigned char* mask);
/* H-RR gradient tensors of level l from the current state, [N][2][3][3]:
 * d_b u_a, then sum_g d_g Psi_abg (test access) */
int orc_hrr_gradients(orc_sim* s, int l, int substep, double* out);
/* rho: [n], u: [D][n], dense over the level's nodes */
int orc_init(orc_sim* s, int l, const double* rho, const double* u);
int orc_run(orc_sim* s, long long n_coarse_steps);
int orc_get_f(const orc_sim* s, int l, double* out);   /* [Q][n], holes NaN */
int orc_get_pre(const orc_sim* s, int l, double* out); /* [Q][n] */
int orc_get_x(const orc_sim* s, int l, double* out);   /* [4][n], NaN off co-located nodes */
int orc_set_f(orc_sim* s, int l, const double* in);   /* [Q][n] */
long long orc_get_probes(const orc_sim* s, double* out);
int orc_balance(const orc_sim* s, double out[5]);
void orc_newton_stats(const orc_sim* s, long long* calls, int* max_iters, long long hist[8]);
int orc_threads(void);
void orc_set_threads(int n);

int orc_lattice(int lattice, int* Q, int* D, int* xi, double* w);
int orc_feq(int lattice, int eq_order, double rho, const double* u, double* out);
int orc_newton(int lattice, int eq_order, const double* h, const double* G, double tol, int maxit,
               double* X, int* iters);
int orc_residual(int lattice, int eq_order, const double* h, const double* G, const double* X, double* F);
int orc_sets(int lattice, unsigned Kf, unsigned Kc, int coupling, unsigned out[6]);
int orc_node_masks(const orc_sim* s, int l, const int k[3], unsigned* Kf, unsigned* Kc);
void orc_line_stencil(int k, int N, int* pos, double* w);
double orc_time_interp(long long captures, int substep, double Hm, double H0, double Hp);

#ifdef __cplusplus
}
#endif
#endif
