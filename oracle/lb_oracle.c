/*
 * lb_oracle.c -- plain FP64 reference recurrence of the linear lattice
 * Boltzmann scheme for linear acoustic waves (Dhuri, Hanasoge, Perlekar,
 * Robertsson, "Numerical analysis of the lattice Boltzmann method for
 * simulation of linear acoustic waves", arXiv:1704.03172).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle: the tests, the smoke
 * check and the CPU-baseline leg of the benchmark call it; the product
 * library never includes, links or calls it, and it shares no code, table
 * or header with the GPU path.  It is written to be read against the paper,
 * not to be fast: one node at a time, explicit loops, no blocking, FP64.
 *
 * State convention: g[i][y][x] holds the pre-collision populations at an
 * integer time n (x fastest).  One call of orc_step() advances n -> n+1:
 *   1. moments rho = sum_i g_i, J = sum_i c_i g_i      (Sec. II B, moments)
 *   2. per-node weights from c_s^2(x)                  (Sec. II C, weight
 *      constraints and rest-particle weight)
 *   3. linear equilibrium g_i^eq = w_i/c^2 (p + c_i.J), p = c^2 rho
 *                                                       (eq. linear eqm dist,
 *                                                        eq. state)
 *   4. collision g* = g - C (g - g^eq), C = M^-1 S M     (eq. MRT-LB; BGK is
 *      C = I/tau, eq. BGK-LB)
 *   5. source g*_i += w_i S(n) at the source node       (eq. MRT-LB linear
 *                                                        acoustic)
 *   6. sponge g* <- (1 - sigma(x)) g*                   (Sec. IV, sponge
 *      layers: reduced by a fraction at each collision)
 *   7. stream g_i(x + c_i, n+1) = g*_i(x), periodic wrap (eq. BGK-LB lhs)
 * The collision matrix C is built by the Python side of the oracle from the
 * transformation matrices of Appendix A and passed in.
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>

typedef struct {
    int32_t nx, ny, q;         /* grid size; q = 5 (D2Q5) or 9 (D2Q9)        */
    int32_t cx[9], cy[9];      /* lattice velocities, Table I / Appendix A  */
    double coll[81];           /* collision matrix C, q x q, row major      */
    double ratio;              /* D2Q9 only: w5 / w1 (weight family)        */
    int32_t sponge_width;      /* L: sponge frame width in nodes (0 = none) */
    double sponge_sigma_max;   /* sigma at the outermost node               */
    int32_t src_x, src_y;      /* source node, or -1 for none               */
} orc_params;

/*
 * Lattice weights at one node from its squared sound speed c2 (Sec. II C):
 * sum_i w_i = 1 and sum_i w_i c_ia c_ib = c2 delta_ab, with equal weights on
 * symmetric velocities.  D2Q5: 2 w1 = c2, w0 = 1 - 4 w1 (this is
 * w0 = 1 - eta^2 with c_s,max^2 = 1/2, Appendix D).  D2Q9 is
 * under-determined (Sec. III C); the family fixes w5 = ratio * w1, so that
 * 2 w1 + 4 w5 = c2.
 */
void orc_node_weights(const orc_params *p, double c2, double *w)
{
    if (p->q == 5) {
        double w1 = 0.5 * c2;
        w[0] = 1.0 - 4.0 * w1;
        for (int i = 1; i < 5; ++i) w[i] = w1;
    } else {
        double w1 = c2 / (2.0 + 4.0 * p->ratio);
        double w5 = p->ratio * w1;
        w[0] = 1.0 - 4.0 * w1 - 4.0 * w5;
        for (int i = 1; i < 5; ++i) w[i] = w1;
        for (int i = 5; i < 9; ++i) w[i] = w5;
    }
}

/*
 * Sponge strength at node (x, y) (Sec. IV, overlap/sponge paragraph: at a
 * sponge node the distribution is reduced by a fraction of its value at
 * every collision).  The paper does not give the profile; the reading used
 * is sigma = sigma_max ((L - d) / L)^2 for d < L, where d is the distance in
 * nodes to the nearest outer edge of the grid.
 */
double orc_sponge_sigma(const orc_params *p, int x, int y)
{
    int L = p->sponge_width;
    if (L <= 0) return 0.0;
    int d = x;
    if (y < d) d = y;
    if (p->nx - 1 - x < d) d = p->nx - 1 - x;
    if (p->ny - 1 - y < d) d = p->ny - 1 - y;
    if (d >= L) return 0.0;
    double f = (double)(L - d) / (double)L;
    return p->sponge_sigma_max * f * f;
}

/*
 * Linear equilibrium (eq. linear eqm dist) of a population vector at one
 * node: g_i^eq = (w_i / c2) [p + c_i . J] with p = c2 rho (eq. state).
 */
void orc_equilibrium(const orc_params *p, double c2, double rho, double jx,
                     double jy, double *geq)
{
    double w[9];
    orc_node_weights(p, c2, w);
    double pr = c2 * rho;
    for (int i = 0; i < p->q; ++i)
        geq[i] = w[i] / c2 * (pr + p->cx[i] * jx + p->cy[i] * jy);
}

/* Fill a whole field with the equilibrium of given rho, Jx, Jy fields. */
void orc_equilibrium_field(const orc_params *p, const double *c2,
                           const double *rho, const double *jx,
                           const double *jy, double *g)
{
    const long n = (long)p->nx * p->ny;
    for (long node = 0; node < n; ++node) {
        double geq[9];
        orc_equilibrium(p, c2[node], rho[node], jx ? jx[node] : 0.0,
                        jy ? jy[node] : 0.0, geq);
        for (int i = 0; i < p->q; ++i) g[(long)i * n + node] = geq[i];
    }
}

/*
 * Steps 1-6 of the update at one node: moments, equilibrium, collision,
 * source (amount s_here, zero away from the source node) and sponge.
 */
void orc_collide_node(const orc_params *p, const double *gi, double c2,
                      double s_here, double sigma, double *gs)
{
    const int q = p->q;
    double rho = 0.0, jx = 0.0, jy = 0.0;
    for (int i = 0; i < q; ++i) {
        rho += gi[i];
        jx += p->cx[i] * gi[i];
        jy += p->cy[i] * gi[i];
    }
    double geq[9], w[9];
    orc_equilibrium(p, c2, rho, jx, jy, geq);
    orc_node_weights(p, c2, w);
    for (int i = 0; i < q; ++i) {
        double acc = 0.0;
        for (int j = 0; j < q; ++j) acc += p->coll[i * q + j] * (gi[j] - geq[j]);
        gs[i] = gi[i] - acc;
    }
    for (int i = 0; i < q; ++i) gs[i] += w[i] * s_here;
    for (int i = 0; i < q; ++i) gs[i] *= (1.0 - sigma);
}

/*
 * One time step n -> n+1 of the whole grid (steps 1-7 above).  g and gn are
 * [q][ny][nx] arrays and must not alias.  s_n is the source amplitude S(n)
 * added at the source node.
 */
void orc_step(const orc_params *p, const double *g, double *gn,
              const double *c2, double s_n)
{
    const int nx = p->nx, ny = p->ny, q = p->q;
    const long n = (long)nx * ny;
#pragma omp parallel for schedule(static)
    for (int y = 0; y < ny; ++y) {
        for (int x = 0; x < nx; ++x) {
            long node = (long)y * nx + x;
            double gi[9], gs[9];
            for (int i = 0; i < q; ++i) gi[i] = g[(long)i * n + node];
            double s_here = (x == p->src_x && y == p->src_y) ? s_n : 0.0;
            orc_collide_node(p, gi, c2[node], s_here,
                             orc_sponge_sigma(p, x, y), gs);
            for (int i = 0; i < q; ++i) {
                int xd = ((x + p->cx[i]) % nx + nx) % nx;
                int yd = ((y + p->cy[i]) % ny + ny) % ny;
                gn[(long)i * n + (long)yd * nx + xd] = gs[i];
            }
        }
    }
}

/* Number of OpenMP threads the step uses (reported with CPU timings). */
int orc_num_threads(void)
{
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Sets the OpenMP threads of later steps (timing only: the result of a step
   does not depend on it, each node being written by one thread). */
void orc_set_num_threads(int n)
{
#ifdef _OPENMP
    extern void omp_set_num_threads(int);
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
