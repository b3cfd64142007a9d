/*
 * lbm_oracle.c -- plain FP64 CPU reference of the reactive lattice Boltzmann step.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test suite, the smoke check and the benchmark's CPU
 * baseline leg use it.  It shares no code, header or table with the GPU path.
 *
 * What it computes (Weinmiller et al., "General Local Reactive Boundary
 * Condition for Dissolution and Precipitation Using the Lattice Boltzmann
 * Method"):
 *   - fluid lattice: BGK collision with the second-order equilibrium
 *     (Sec. 2.1, eqs. fluid_BGK, fluid_Equilib, fluid_BGK_visc); a body force
 *     enters through Guo's forcing with the half-force velocity shift (the
 *     paper names no forcing scheme, Guo's is the standard one for BGK);
 *     halfway bounce-back at solid neighbours.
 *   - solute lattice: advection-diffusion BGK with the linear equilibrium
 *     g_eq = C w_i (1 + u.e_i / c_s^2), u the fluid velocity of the same node
 *     and step (Sec. 2.1, eqs. solute_BGK, solute_equilibrium_function,
 *     solute_diffu).
 *   - solute velocity set: the paper's reduced lattices D2Q5 / D3Q7 (appendix,
 *     velocity sets; rest vector and the axis vectors), or the fluid's own
 *     D2Q9 / D3Q19.  A reduced set is located inside the fluid set by its
 *     vectors, so both lattices pull along the same geometry.
 *   - rest fraction (Sec. 2.2, eqs. RestFraction, RestFractionCs2): on D2Q5 /
 *     D3Q7 exactly the paper's w_0 = J0, w_i = c_s^2/2, c_s^2 = (1 - J0)/dim;
 *     on D2Q9 / D3Q19 w_0 = J0 and the moving weights scaled by
 *     (1 - J0)/(1 - w0_std), c_s^2 likewise (keeps sum w e e = c_s^2 I).
 *   - reactive boundary condition (Sec. 2.3, eq. general_RBC and the k_i of
 *     eqs. k_i_S_Ve, k_i_S2, k_i_S_New; gamma of eq. gammaAppendix):
 *        g_out = k/(1+k) 2 w C_eq + (1-k)/(1+k) g_src
 *     with the anti-bounce-back limit for k -> infinity and plain bounce-back
 *     for k = 0 (Sec. 2.3, limits); the anti-bounce-back scheme applies at
 *     solid nodes with k_r > 0 (a non-reactive wall stays bounce-back).
 *   - open channel (Sec. 3.3, reactive object in a channel flow: plug velocity
 *     at the inlet, fixed density at the outlet; the paper names no scheme):
 *     at the inlet face an incoming population is the node's own opposite one
 *     plus 2 w_i rho_out (e_i.u_in)/c_s^2 (bounce-back from a wall moving with
 *     u_in, which carries exactly rho_out u_in per inlet node), at the outlet
 *     face minus the node's own opposite one plus 2 w_i rho_out
 *     (anti-bounce-back at density rho_out, dropping O(u^2) terms).
 *   - solid fraction (Sec. 2.4, eq. solidFractionUpdate) fed by the mass
 *     actually exchanged over each reactive link; dissolution is charged to
 *     the solid node, precipitation credited to the fluid node.
 *
 * Storage is array-of-structures [node][direction], FP64, two buffers.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_QMAX 19

enum { ORC_MECH_PRE = 0, ORC_MECH_POST = 1 };
enum { ORC_SNEW = 0, ORC_SV = 1, ORC_SPJ = 2, ORC_ABB = 3 };
enum { ORC_BGK = 0, ORC_TRT = 1 };
/* the TRT "magic" parameter (Sec. 2.1, eq. fluid_TRT_visc): 3/16 puts
 * bounce-back walls exactly halfway */
#define ORC_MAGIC (3.0 / 16.0)

typedef struct {
    int dim, nx, ny, nz, q;
    int mechanics, scheme;
    double tau_ns, tau_ad, j0;
    double force[3];
    double c_eq, k_r, v_m, a_m;
    int periodic[3];
    int xwrap_shift_y;
    int inlet_axis;
    double c_in;
    int phase_change;
    int collision;          /* ORC_BGK | ORC_TRT */
    int qs;                 /* solute lattice: 0 or q (the fluid's), 5 (D2Q5 with
                               D2Q9) or 7 (D3Q7 with D3Q19) */
    int fluid_open;         /* 1: the fluid enters at the inlet face with the plug
                               velocity u_in and leaves at the outlet face at
                               density rho_out (inlet axis not periodic) */
    double u_in, rho_out;
} orc_params;

typedef struct {
    orc_params p;
    int Q;
    int QS;                /* solute directions                           */
    int sd[ORC_QMAX];      /* solute direction s is fluid direction sd[s] */
    uint8_t ins[ORC_QMAX]; /* fluid direction i belongs to the solute set */
    long N;
    int e[ORC_QMAX][3];
    int opp[ORC_QMAX];
    double wf[ORC_QMAX];   /* fluid weights: standard lattice            */
    double ws[ORC_QMAX];   /* solute weights: rest-fraction lattice, by
                              fluid direction (0 outside the solute set)  */
    double cs2f, cs2s;
    double gamma;          /* tau_AD / (tau_AD - 1/2)                     */
    uint8_t *solid;
    double *nrm;           /* [N][3] */
    double *ceq;           /* [N] per-node C_eq of the reaction, or NULL (c_eq) */
    double *kr;            /* [N]    */
    double *phi;           /* [N]    */
    double *f, *fn, *g, *gn; /* [N][Q] post-collision populations       */
    double *qx;            /* [N][Q] mass exchanged over the link last step */
    uint8_t *kind;         /* [N][Q] link classification of last step   */
    double inlet_ex, outlet_ex, wall_ex; /* cumulative exchanges            */
    long step, n_events;
    double *uh;            /* if set, [N][3]: the fluid velocity each node's
                              solute collision used in the current step    */
} orc;

/* link classes of an incoming solute population */
enum { K_KNOWN = 0, K_RBC = 1, K_WALL = 2, K_INLET = 3, K_OUTLET = 4 };

/* the solute runs on the reduced D2Q5 / D3Q7 set */
static int orc_reduced(const orc_params *p)
{
    return (p->q == 9 && p->qs == 5) || (p->q == 19 && p->qs == 7);
}

static void set_lattice(orc *o)
{
    int Q = o->p.q;
    o->Q = Q;
    if (Q == 9) {
        /* paper, appendix (velocity sets): D2Q9 in the paper's order */
        static const int E[9][2] = {{0, 0}, {-1, 1}, {-1, 0}, {-1, -1}, {0, -1},
                                    {1, -1}, {1, 0},  {1, 1},  {0, 1}};
        static const double W[9] = {4. / 9, 1. / 36, 1. / 9, 1. / 36, 1. / 9,
                                    1. / 36, 1. / 9, 1. / 36, 1. / 9};
        for (int i = 0; i < 9; i++) {
            o->e[i][0] = E[i][0];
            o->e[i][1] = E[i][1];
            o->e[i][2] = 0;
            o->wf[i] = W[i];
        }
    } else {
        /* D3Q19: rest, then nine vectors and their negatives (e_{i+9} = -e_i) */
        static const int E[10][3] = {{0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {0, 0, 1},
                                     {1, 1, 0}, {1, -1, 0}, {1, 0, 1}, {1, 0, -1},
                                     {0, 1, 1}, {0, 1, -1}};
        for (int i = 0; i < 10; i++)
            for (int d = 0; d < 3; d++) o->e[i][d] = E[i][d];
        for (int i = 1; i < 10; i++)
            for (int d = 0; d < 3; d++) o->e[i + 9][d] = -E[i][d];
        for (int i = 0; i < 19; i++) {
            int s = abs(o->e[i][0]) + abs(o->e[i][1]) + abs(o->e[i][2]);
            o->wf[i] = s == 0 ? 1. / 3 : (s == 1 ? 1. / 18 : 1. / 36);
        }
    }
    for (int i = 0; i < Q; i++)
        for (int j = 0; j < Q; j++)
            if (o->e[j][0] == -o->e[i][0] && o->e[j][1] == -o->e[i][1] &&
                o->e[j][2] == -o->e[i][2])
                o->opp[i] = j;
    o->cs2f = 1.0 / 3.0;
    for (int i = 0; i < Q; i++) o->ws[i] = 0.0;
    if (orc_reduced(&o->p)) {
        /* D2Q5 in the paper's appendix order; D3Q7 as the rest vector, the
         * three axis vectors and their negatives */
        static const int E5[5][3] = {{0, 0, 0}, {-1, 0, 0}, {0, -1, 0}, {1, 0, 0}, {0, 1, 0}};
        static const int E7[7][3] = {{0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {0, 0, 1},
                                     {-1, 0, 0}, {0, -1, 0}, {0, 0, -1}};
        const int dim = Q == 9 ? 2 : 3;
        o->QS = Q == 9 ? 5 : 7;
        for (int s = 0; s < o->QS; s++) {
            const int *v = Q == 9 ? E5[s] : E7[s];
            for (int i = 0; i < Q; i++)
                if (o->e[i][0] == v[0] && o->e[i][1] == v[1] && o->e[i][2] == v[2]) o->sd[s] = i;
        }
        /* eqs. RestFraction, RestFractionCs2; without a rest fraction the
         * common lattice (J0 = 1/3 on D2Q5, 1/4 on D3Q7) */
        const double j0 = o->p.j0 < 0 ? (dim == 2 ? 1.0 / 3.0 : 1.0 / 4.0) : o->p.j0;
        o->cs2s = (1.0 - j0) / dim;
        o->ws[o->sd[0]] = j0;
        for (int s = 1; s < o->QS; s++) o->ws[o->sd[s]] = o->cs2s / 2.0;
    } else {
        o->QS = Q;
        for (int i = 0; i < Q; i++) o->sd[i] = i;
        /* rest fraction: J0 < 0 keeps the standard weights */
        double w0 = o->wf[0];
        if (o->p.j0 < 0) {
            for (int i = 0; i < Q; i++) o->ws[i] = o->wf[i];
            o->cs2s = 1.0 / 3.0;
        } else {
            double sc = (1.0 - o->p.j0) / (1.0 - w0);
            o->ws[0] = o->p.j0;
            for (int i = 1; i < Q; i++) o->ws[i] = o->wf[i] * sc;
            o->cs2s = (1.0 / 3.0) * sc;
        }
    }
    for (int i = 0; i < Q; i++) o->ins[i] = 0;
    for (int s = 0; s < o->QS; s++) o->ins[o->sd[s]] = 1;
    o->gamma = o->p.tau_ad / (o->p.tau_ad - 0.5);
}

static long idx(const orc *o, int x, int y, int z)
{
    return (long)x + (long)o->p.nx * ((long)y + (long)o->p.ny * (long)z);
}

static void coords(const orc *o, long n, int *x, int *y, int *z)
{
    *x = (int)(n % o->p.nx);
    *y = (int)((n / o->p.nx) % o->p.ny);
    *z = (int)(n / ((long)o->p.nx * o->p.ny));
}

static int floordiv(int a, int b)
{
    int q = a / b;
    if ((a % b != 0) && ((a < 0) != (b < 0))) q--;
    return q;
}

/*
 * Site reached from (x,y,z) by (dx,dy,dz).  Periodic axes wrap; a wrap in x
 * also moves y by the shift (the torus of a tilted channel).  The solute sees
 * the inlet axis as non-periodic.  Returns -1 when the step leaves the domain
 * through a face, which is reported as 2*axis + (1 if the high side).
 */
static long site(const orc *o, int x, int y, int z, int dx, int dy, int dz, int solute,
                 int *face)
{
    int c[3] = {x + dx, y + dy, z + dz};
    int n[3] = {o->p.nx, o->p.ny, o->p.nz};
    *face = -1;
    for (int a = 0; a < 3; a++) {
        int per = o->p.periodic[a] && !(solute && o->p.inlet_axis == a);
        if (c[a] >= 0 && c[a] < n[a]) continue;
        if (!per) {
            *face = 2 * a + (c[a] >= n[a] ? 1 : 0);
            return -1;
        }
        int k = floordiv(c[a], n[a]);
        c[a] -= k * n[a];
        if (a == 0) c[1] += k * o->p.xwrap_shift_y;
    }
    return idx(o, c[0], c[1], c[2]);
}

/* ------------------------------------------------------------------------- */

static void fd_normal(orc *o, long s);

orc *orc_create(const orc_params *p, const uint8_t *solid, const double *normals,
                const double *k_r, const double *phi0)
{
    if (!(p->qs == 0 || p->qs == p->q || orc_reduced(p))) return NULL;
    orc *o = (orc *)calloc(1, sizeof(orc));
    o->p = *p;
    set_lattice(o);
    o->N = (long)p->nx * p->ny * p->nz;
    long N = o->N, Q = o->Q;
    o->solid = (uint8_t *)malloc(N);
    memcpy(o->solid, solid, N);
    o->nrm = (double *)calloc(N * 3, sizeof(double));
    if (normals) {
        memcpy(o->nrm, normals, sizeof(double) * N * 3);
    } else {
        /* no normals given: isotropic lattice gradient of the solid indicator
         * (the paper computes wall normals with an isotropic finite difference,
         * Sec. 3.2) */
        for (long n = 0; n < N; n++)
            if (o->solid[n]) fd_normal(o, n);
    }
    o->kr = (double *)malloc(sizeof(double) * N);
    for (long n = 0; n < N; n++) o->kr[n] = k_r ? k_r[n] : p->k_r;
    o->phi = (double *)malloc(sizeof(double) * N);
    for (long n = 0; n < N; n++) o->phi[n] = phi0 ? phi0[n] : (solid[n] ? 1.0 : 0.0);
    o->f = (double *)calloc(N * Q, sizeof(double));
    o->fn = (double *)calloc(N * Q, sizeof(double));
    o->g = (double *)calloc(N * Q, sizeof(double));
    o->gn = (double *)calloc(N * Q, sizeof(double));
    o->qx = (double *)calloc(N * Q, sizeof(double));
    o->kind = (uint8_t *)calloc(N * Q, 1);
    return o;
}

void orc_destroy(orc *o)
{
    if (!o) return;
    free(o->solid); free(o->nrm); free(o->kr); free(o->phi); free(o->ceq);
    free(o->f); free(o->fn); free(o->g); free(o->gn); free(o->qx); free(o->kind);
    free(o);
}

static double feq(const orc *o, int i, double rho, const double u[3])
{
    double eu = o->e[i][0] * u[0] + o->e[i][1] * u[1] + o->e[i][2] * u[2];
    double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    double c = o->cs2f;
    return o->wf[i] * rho * (1.0 + eu / c + eu * eu / (2.0 * c * c) - uu / (2.0 * c));
}

static double geq(const orc *o, int i, double C, const double u[3])
{
    double eu = o->e[i][0] * u[0] + o->e[i][1] * u[1] + o->e[i][2] * u[2];
    return o->ws[i] * C * (1.0 + eu / o->cs2s);
}

/* Initial state: equilibrium of the given fields written as the post-collision
 * populations (NULL fields: rho = 1, u = 0, C = 0).  Solid nodes hold zeros. */
void orc_init(orc *o, const double *rho, const double *u, const double *c)
{
    long N = o->N;
    int Q = o->Q;
    for (long n = 0; n < N; n++) {
        for (int i = 0; i < Q; i++) {
            o->f[n * Q + i] = 0.0;
            o->g[n * Q + i] = 0.0;
        }
        if (o->solid[n]) continue;
        double r = rho ? rho[n] : 1.0;
        double uu[3] = {0, 0, 0};
        if (u) { uu[0] = u[3 * n]; uu[1] = u[3 * n + 1]; uu[2] = u[3 * n + 2]; }
        double C = c ? c[n] : 0.0;
        for (int i = 0; i < Q; i++) {
            o->f[n * Q + i] = feq(o, i, r, uu);
            o->g[n * Q + i] = geq(o, i, C, uu);
        }
    }
    o->step = 0;
    o->inlet_ex = o->outlet_ex = o->wall_ex = 0.0;
}

/* k_i of the selected scheme for the link entering fluid node x from solid s
 * along e_i (e_i points from s to x); INFINITY encodes anti-bounce-back. */
static double link_k(const orc *o, long s, int i)
{
    const double *n = o->nrm + 3 * s;
    double en = o->e[i][0] * n[0] + o->e[i][1] * n[1] + o->e[i][2] * n[2];
    double kr = o->kr[s];
    switch (o->p.scheme) {
    case ORC_SV:   return en > 0 ? kr * en / o->cs2s : 0.0;
    case ORC_SPJ:  return en > 0 ? o->gamma * kr / (o->cs2s * en) : 0.0;
    /* anti-bounce-back is the limit k -> infinity of the rate condition (Sec.
     * 3.1, extended PeDa range); a solid node without reaction (k_r = 0)
     * keeps plain bounce-back */
    case ORC_ABB:  return kr > 0 ? INFINITY : 0.0;
    default:       return en > 0 ? o->gamma * kr * en / o->cs2s : 0.0;
    }
}

static void update_node(orc *o, long x)
{
    const int Q = o->Q;
    const orc_params *p = &o->p;
    int X, Y, Z, face;
    coords(o, x, &X, &Y, &Z);
    double *fo = o->f, *go = o->g;

    /* fluid: pull with halfway bounce-back; an open channel's inlet and
     * outlet faces instead impose the plug velocity and the outlet density */
    double fp[ORC_QMAX];
    for (int i = 0; i < Q; i++) {
        long y = site(o, X, Y, Z, -o->e[i][0], -o->e[i][1], -o->e[i][2], 0, &face);
        if (y >= 0 && !o->solid[y]) fp[i] = fo[y * Q + i];
        else fp[i] = fo[x * Q + o->opp[i]];
        if (y < 0 && p->fluid_open && p->inlet_axis >= 0) {
            const int a = p->inlet_axis;
            if (face == 2 * a)
                fp[i] += 2.0 * o->wf[i] * p->rho_out * (o->e[i][a] * p->u_in) / o->cs2f;
            else if (face == 2 * a + 1)
                fp[i] = -fp[i] + 2.0 * o->wf[i] * p->rho_out;
        }
    }
    double rho = 0, j[3] = {0, 0, 0};
    for (int i = 0; i < Q; i++) {
        rho += fp[i];
        for (int d = 0; d < 3; d++) j[d] += fp[i] * o->e[i][d];
    }
    double u[3];
    for (int d = 0; d < 3; d++) u[d] = (j[d] + 0.5 * p->force[d]) / rho;
    if (o->uh)
        for (int d = 0; d < 3; d++) o->uh[3 * x + d] = u[d];
    double c = o->cs2f;
    double uF = u[0] * p->force[0] + u[1] * p->force[1] + u[2] * p->force[2];
    double fe[ORC_QMAX], S[ORC_QMAX];
    for (int i = 0; i < Q; i++) {
        double eu = o->e[i][0] * u[0] + o->e[i][1] * u[1] + o->e[i][2] * u[2];
        double eF = o->e[i][0] * p->force[0] + o->e[i][1] * p->force[1] +
                    o->e[i][2] * p->force[2];
        S[i] = o->wf[i] * ((eF - uF) / c + eu * eF / (c * c));
        fe[i] = feq(o, i, rho, u);
    }
    if (p->collision == ORC_TRT) {
        /* TRT (Sec. 2.1, eqs. fluid_TRT, fluid_TRT_terms, fluid_TRT_visc):
         * the parts of f, f_eq even and odd in e_i relax with tau+ (viscosity)
         * and tau- (from the magic parameter); the Guo source term is split the
         * same way, each part with its own factor 1 - 1/(2 tau) (reading: the
         * paper gives no TRT forcing) */
        const double tp = p->tau_ns, tm = 0.5 + ORC_MAGIC / (p->tau_ns - 0.5);
        for (int i = 0; i < Q; i++) {
            const int ob = o->opp[i];
            const double fpl = 0.5 * (fp[i] + fp[ob]), fmi = 0.5 * (fp[i] - fp[ob]);
            const double epl = 0.5 * (fe[i] + fe[ob]), emi = 0.5 * (fe[i] - fe[ob]);
            const double spl = 0.5 * (S[i] + S[ob]), smi = 0.5 * (S[i] - S[ob]);
            o->fn[x * Q + i] = fp[i] - (fpl - epl) / tp - (fmi - emi) / tm +
                               (1.0 - 0.5 / tp) * spl + (1.0 - 0.5 / tm) * smi;
        }
    } else {
        for (int i = 0; i < Q; i++)
            o->fn[x * Q + i] = fp[i] - (fp[i] - fe[i]) / p->tau_ns + (1.0 - 0.5 / p->tau_ns) * S[i];
    }

    /* solute: pull, plane conditions, then the reactive links; only the
     * directions of the solute set (a fluid direction outside it carries no
     * solute population and no link) */
    double gp[ORC_QMAX];
    uint8_t kd[ORC_QMAX];
    long sol[ORC_QMAX];
    for (int i = 0; i < Q; i++) {
        gp[i] = 0.0;
        kd[i] = K_KNOWN;
        sol[i] = -1;
    }
    for (int s = 0; s < o->QS; s++) {
        const int i = o->sd[s];
        long y = site(o, X, Y, Z, -o->e[i][0], -o->e[i][1], -o->e[i][2], 1, &face);
        if (y >= 0) {
            if (!o->solid[y]) { gp[i] = go[y * Q + i]; kd[i] = K_KNOWN; }
            else { kd[i] = K_RBC; sol[i] = y; gp[i] = 0.0; }
        } else if (p->inlet_axis >= 0 && face == 2 * p->inlet_axis) {
            gp[i] = geq(o, i, p->c_in, u);
            kd[i] = K_INLET;
        } else if (p->inlet_axis >= 0 && face == 2 * p->inlet_axis + 1) {
            /* zero-gradient outlet: copy from the outlet-plane site upstream */
            int a = p->inlet_axis, ex[3] = {0, 0, 0};
            ex[a] = 1;
            int f2;
            long y2 = site(o, X, Y, Z, -o->e[i][0] - ex[0], -o->e[i][1] - ex[1],
                           -o->e[i][2] - ex[2], 1, &f2);
            if (y2 >= 0 && !o->solid[y2]) gp[i] = go[y2 * Q + i];
            else gp[i] = go[x * Q + o->opp[i]];
            kd[i] = K_OUTLET;
        } else {
            gp[i] = go[x * Q + o->opp[i]];
            kd[i] = K_WALL;
        }
    }
    for (int i = 0; i < Q; i++) {
        o->kind[x * Q + i] = kd[i];
        /* inlet and outlet faces: incoming minus the population lost there */
        o->qx[x * Q + i] = (kd[i] == K_INLET || kd[i] == K_OUTLET)
                               ? gp[i] - go[x * Q + o->opp[i]] : 0.0;
        if (kd[i] != K_RBC) continue;
        int ob = o->opp[i];
        double k = link_k(o, sol[i], i);
        double src;
        if (p->mechanics == ORC_MECH_PRE && kd[ob] != K_RBC) {
            src = gp[ob];
        } else {
            src = go[x * Q + ob];
            /* a one-node gap under the pre-collision reading falls back to the
             * post-collision source, whose effective rate is gamma times larger */
            if (p->mechanics == ORC_MECH_PRE) k = k / o->gamma;
        }
        /* the equilibrium concentration of the solid node's reaction */
        const double ceq = o->ceq ? o->ceq[sol[i]] : p->c_eq;
        double gout;
        if (isinf(k)) gout = 2.0 * o->ws[i] * ceq - src;
        else gout = k / (1.0 + k) * 2.0 * o->ws[i] * ceq + (1.0 - k) / (1.0 + k) * src;
        gp[i] = gout;
        o->qx[x * Q + i] = gout - go[x * Q + ob];
    }
    double C = 0;
    for (int s = 0; s < o->QS; s++) C += gp[o->sd[s]];
    if (p->collision == ORC_TRT) {
        /* TRT for the solute (Sec. 2.1, eqs. solute_TRT, solute_TRT_terms,
         * solute_TRT_visc): the even parts relax with 1/tau-, the odd parts
         * with 1/tau+; D = c_s^2 (tau+ - 1/2) sets tau+ = tau_AD */
        const double tp = p->tau_ad, tm = 0.5 + ORC_MAGIC / (p->tau_ad - 0.5);
        double ge[ORC_QMAX];
        for (int i = 0; i < Q; i++) ge[i] = geq(o, i, C, u);
        for (int s = 0; s < o->QS; s++) {
            const int i = o->sd[s], ob = o->opp[i];
            const double gpl = 0.5 * (gp[i] + gp[ob]), gmi = 0.5 * (gp[i] - gp[ob]);
            const double epl = 0.5 * (ge[i] + ge[ob]), emi = 0.5 * (ge[i] - ge[ob]);
            o->gn[x * Q + i] = gp[i] - (gpl - epl) / tm - (gmi - emi) / tp;
        }
    } else {
        for (int s = 0; s < o->QS; s++) {
            const int i = o->sd[s];
            o->gn[x * Q + i] = gp[i] - (gp[i] - geq(o, i, C, u)) / p->tau_ad;
        }
    }
}

static void apply_phase_change(orc *o);

void orc_step(orc *o, int nsteps)
{
    const long N = o->N;
    const int Q = o->Q;
    for (int t = 0; t < nsteps; t++) {
        long n;
#ifdef _OPENMP
        /* threads only for large lattices: on small ones the per-step fork and
         * barrier cost more than the work (nodes are independent either way) */
#pragma omp parallel for schedule(static) if (N >= 32768)
#endif
        for (n = 0; n < N; n++) {
            if (o->solid[n]) {
                for (int i = 0; i < Q; i++) {
                    o->fn[n * Q + i] = 0.0;
                    o->gn[n * Q + i] = 0.0;
                    o->qx[n * Q + i] = 0.0;
                    o->kind[n * Q + i] = K_KNOWN;
                }
                continue;
            }
            update_node(o, n);
        }
        /* solid fraction, in node order; link sums in ascending direction */
        const double vma = o->p.v_m * o->p.a_m;
        double wall = 0.0;
        for (n = 0; n < N; n++) {
            int X, Y, Z, face;
            coords(o, n, &X, &Y, &Z);
            if (o->solid[n]) {
                double s = 0.0;
                for (int i = 1; i < Q; i++) {
                    long x = site(o, X, Y, Z, o->e[i][0], o->e[i][1], o->e[i][2], 1, &face);
                    if (x < 0 || o->solid[x] || o->kind[x * Q + i] != K_RBC) continue;
                    double qv = o->qx[x * Q + i];
                    if (qv > 0) s += qv;
                }
                o->phi[n] -= vma * s;
            } else {
                double s = 0.0;
                for (int i = 1; i < Q; i++) {
                    int kd = o->kind[n * Q + i];
                    if (kd == K_INLET) o->inlet_ex += o->qx[n * Q + i];
                    if (kd == K_OUTLET) o->outlet_ex += o->qx[n * Q + i];
                    if (kd != K_RBC) continue;
                    double qv = o->qx[n * Q + i];
                    wall += qv;
                    if (qv < 0) s += -qv;
                }
                o->phi[n] += vma * s;
            }
        }
        o->wall_ex += wall;
        double *t1 = o->f; o->f = o->fn; o->fn = t1;
        double *t2 = o->g; o->g = o->gn; o->gn = t2;
        o->step++;
        if (o->p.phase_change) apply_phase_change(o);
    }
}

/* ------------------------------------------------------------------------- */
/* Phase change (Sec. 2.4: thresholds phi = 0 for dissolution and phi = 1 for
 * precipitation; the local concentration is turned into phi, the excess goes
 * to the surrounding fluid cells, and a dissolved cell starts at the mean
 * concentration of its fluid neighbours, paid for by the surrounding solid
 * cells).  The paper states the rules in words only.  Reading taken here: a
 * dissolving solid node (with at least one fluid neighbour) becomes fluid
 * with C and rho the means over its fluid neighbours and equilibrium
 * populations at rest, and V_m C - phi is taken from its solid neighbours in
 * proportion to their rate constants k_r (equal shares if all are 0; kept by
 * the node as a negative phi if it has no solid neighbour); a precipitating
 * fluid node becomes solid, adds V_m C to phi and passes phi - 1 in equal
 * shares to its fluid neighbours (the rate that weights the shares is the
 * precipitating cell's own, the same for every share).  Both keep the solute
 * plus solid mass.  Events are taken in node-index order; a node pushed over
 * its threshold by an earlier event is taken when the loop reaches it. */

static double node_C(const orc *o, long n)
{
    double C = 0;
    for (int i = 0; i < o->Q; i++) C += o->g[n * o->Q + i];
    return C;
}

static double node_rho(const orc *o, long n)
{
    double r = 0;
    for (int i = 0; i < o->Q; i++) r += o->f[n * o->Q + i];
    return r;
}

/* lattice-gradient normal of the solid indicator: n = -grad(phi_s)/|grad| */
static void fd_normal(orc *o, long s)
{
    int X, Y, Z, face;
    coords(o, s, &X, &Y, &Z);
    double gr[3] = {0, 0, 0};
    for (int i = 1; i < o->Q; i++) {
        long y = site(o, X, Y, Z, o->e[i][0], o->e[i][1], o->e[i][2], 0, &face);
        double ind = (y < 0) ? 1.0 : (o->solid[y] ? 1.0 : 0.0);
        for (int d = 0; d < 3; d++) gr[d] += o->wf[i] * o->e[i][d] * ind / o->cs2f;
    }
    double m = sqrt(gr[0] * gr[0] + gr[1] * gr[1] + gr[2] * gr[2]);
    for (int d = 0; d < 3; d++) o->nrm[3 * s + d] = m > 0 ? -gr[d] / m : 0.0;
}

static void apply_phase_change(orc *o)
{
    const long N = o->N;
    const int Q = o->Q;
    const double vm = o->p.v_m;
    long nev = 0;
    long *changed = NULL;
    long nch = 0, cap = 0;
    for (long n = 0; n < N; n++) {
        int X, Y, Z, face;
        coords(o, n, &X, &Y, &Z);
        if (o->solid[n] && o->phi[n] <= 0.0) {
            /* dissolution: needs at least one fluid neighbour */
            double csum = 0, rsum = 0;
            int nf = 0;
            double wsum = 0;
            for (int i = 1; i < Q; i++) {
                long y = site(o, X, Y, Z, o->e[i][0], o->e[i][1], o->e[i][2], 1, &face);
                if (y < 0) continue;
                if (!o->solid[y]) { csum += node_C(o, y); rsum += node_rho(o, y); nf++; }
            }
            if (nf == 0) continue;
            double Cs = csum / nf, rs = rsum / nf;
            /* take V_m C_s - phi_s from the solid neighbours, weighted by k */
            double need = vm * Cs - o->phi[n];
            long nb[ORC_QMAX];
            double wt[ORC_QMAX];
            int nn = 0;
            for (int i = 1; i < Q; i++) {
                long y = site(o, X, Y, Z, o->e[i][0], o->e[i][1], o->e[i][2], 1, &face);
                if (y < 0 || !o->solid[y]) continue;
                nb[nn] = y;
                wt[nn] = o->kr[y];
                wsum += o->kr[y];
                nn++;
            }
            o->solid[n] = 0;
            o->phi[n] = 0.0;
            double u0[3] = {0, 0, 0};
            for (int i = 0; i < Q; i++) {
                o->f[n * Q + i] = feq(o, i, rs, u0);
                o->g[n * Q + i] = geq(o, i, Cs, u0);
            }
            if (nn > 0) {
                for (int k = 0; k < nn; k++)
                    o->phi[nb[k]] -= need * (wsum > 0 ? wt[k] / wsum : 1.0 / nn);
            } else {
                /* no solid neighbour left: the deficit stays with the new fluid
                 * node as a negative solid fraction (keeps mass exact) */
                o->phi[n] -= need;
            }
            nev++;
            if (nch == cap) { cap = cap ? 2 * cap : 64; changed = (long *)realloc(changed, cap * sizeof(long)); }
            changed[nch++] = n;
        } else if (!o->solid[n] && o->phi[n] >= 1.0) {
            /* precipitation */
            double Cx = node_C(o, n);
            o->phi[n] += vm * Cx;
            double excess = o->phi[n] - 1.0;
            long nb[ORC_QMAX];
            int nn = 0;
            for (int i = 1; i < Q; i++) {
                long y = site(o, X, Y, Z, o->e[i][0], o->e[i][1], o->e[i][2], 1, &face);
                if (y < 0 || o->solid[y]) continue;
                nb[nn++] = y;
            }
            /* the weight is the precipitating cell's own rate, one value for
             * every share: the shares are equal */
            if (nn > 0) {
                for (int k = 0; k < nn; k++) o->phi[nb[k]] += excess / nn;
                o->phi[n] = 1.0;
            }
            o->solid[n] = 1;
            for (int i = 0; i < Q; i++) { o->f[n * Q + i] = 0.0; o->g[n * Q + i] = 0.0; }
            nev++;
            if (nch == cap) { cap = cap ? 2 * cap : 64; changed = (long *)realloc(changed, cap * sizeof(long)); }
            changed[nch++] = n;
        }
    }
    /* refresh normals of solid nodes within two sites of a change */
    for (long c = 0; c < nch; c++) {
        int X, Y, Z, face;
        coords(o, changed[c], &X, &Y, &Z);
        int r = 2, zr = o->p.dim == 3 ? 2 : 0;
        for (int dz = -zr; dz <= zr; dz++)
            for (int dy = -r; dy <= r; dy++)
                for (int dx = -r; dx <= r; dx++) {
                    long y = site(o, X, Y, Z, dx, dy, dz, 0, &face);
                    if (y >= 0 && o->solid[y]) fd_normal(o, y);
                }
    }
    free(changed);
    o->n_events += nev;
}

/* ------------------------------------------------------------------------- */
/* Read-outs.  rho = sum f*, u = (sum e f* - F/2)/rho (the velocity that entered
 * the last collision), C = sum g*; solid nodes read as zero. */
/* ------------------------------------------------------------------------- */
/* Adjoint of the solute lattice with respect to the rate constants k_r of the
 * solid nodes, by reverse-mode differentiation of the steps above.  The fluid
 * does not depend on k_r; its velocity is recorded during the forward run and
 * held fixed.  The solute step is affine in the populations for a given
 * velocity history, so the adjoint populations lambda(t) = dL/dg*(t) follow
 * from lambda(t+1) by the transpose of one step, and dL/dk_r collects, over
 * every step and reactive link, lambda of the link's incoming population times
 * the derivative of the rate condition (Sec. 2.3, eq. general_RBC) with
 * respect to k, times dk/dk_r of the scheme (eqs. k_i_S_Ve, k_i_S2,
 * k_i_S_New). */

/* dk/dk_r of link_k (all schemes are linear in k_r; anti-bounce-back has no k) */
static double link_dk(const orc *o, long s, int i)
{
    const double *n = o->nrm + 3 * s;
    double en = o->e[i][0] * n[0] + o->e[i][1] * n[1] + o->e[i][2] * n[2];
    switch (o->p.scheme) {
    case ORC_SV:   return en > 0 ? en / o->cs2s : 0.0;
    case ORC_SPJ:  return en > 0 ? o->gamma / (o->cs2s * en) : 0.0;
    case ORC_ABB:  return 0.0;
    default:       return en > 0 ? o->gamma * en / o->cs2s : 0.0;
    }
}

/* One fluid node x of the transposed step.  go: the post-collision solute
 * populations the forward step started from; u: the velocity the node's
 * collision used; mu: lambda(t+1) at x.  Adds into lam = lambda(t) and grad. */
static void adjoint_node(const orc *o, long x, const double *go, const double *u,
                         const double *mu, double *lam, double *grad)
{
    const int Q = o->Q;
    const orc_params *p = &o->p;
    int X, Y, Z, face;
    coords(o, x, &X, &Y, &Z);
    /* where every pre-collision value came from (the forward pull):
     * population src_d[i] of node src_n[i], or a constant (src_n = -1) */
    long src_n[ORC_QMAX], sol[ORC_QMAX];
    int src_d[ORC_QMAX], kd[ORC_QMAX];
    double gp[ORC_QMAX];
    for (int i = 0; i < Q; i++) {
        sol[i] = -1;
        if (!o->ins[i]) {
            /* outside the solute set: no population, no link */
            kd[i] = K_KNOWN;
            src_n[i] = -1;
            gp[i] = 0.0;
            continue;
        }
        long y = site(o, X, Y, Z, -o->e[i][0], -o->e[i][1], -o->e[i][2], 1, &face);
        src_n[i] = x;
        src_d[i] = o->opp[i];
        if (y >= 0) {
            if (!o->solid[y]) { kd[i] = K_KNOWN; src_n[i] = y; src_d[i] = i; }
            else { kd[i] = K_RBC; sol[i] = y; }
        } else if (p->inlet_axis >= 0 && face == 2 * p->inlet_axis) {
            kd[i] = K_INLET;
            src_n[i] = -1;
        } else if (p->inlet_axis >= 0 && face == 2 * p->inlet_axis + 1) {
            int a = p->inlet_axis, ex[3] = {0, 0, 0};
            ex[a] = 1;
            int f2;
            long y2 = site(o, X, Y, Z, -o->e[i][0] - ex[0], -o->e[i][1] - ex[1],
                           -o->e[i][2] - ex[2], 1, &f2);
            kd[i] = K_OUTLET;
            if (y2 >= 0 && !o->solid[y2]) { src_n[i] = y2; src_d[i] = i; }
        } else {
            kd[i] = K_WALL;
        }
        if (kd[i] == K_INLET) gp[i] = geq(o, i, p->c_in, u);
        else if (kd[i] == K_RBC) gp[i] = 0.0;
        else gp[i] = go[src_n[i] * Q + src_d[i]];
    }
    /* collision, BGK: g*_i = (1 - 1/tau) p_i + (1/tau) w_i C (1 + e_i.u/c_s^2),
     * C = sum_j p_j.  TRT (Sec. 2.1, eqs. solute_TRT, solute_TRT_terms) with
     * the even rate we = 1/tau- and the odd rate wo = 1/tau_AD:
     *   g*_i = (1 - (we + wo)/2) p_i + ((wo - we)/2) p_opp(i)
     *          + w_i C (we + wo e_i.u/c_s^2),
     * which is the BGK form when we = wo.  Its transpose: */
    double we = 1.0 / p->tau_ad, wo = 1.0 / p->tau_ad;
    if (p->collision == ORC_TRT) we = 1.0 / (0.5 + ORC_MAGIC / (p->tau_ad - 0.5));
    double m = 0.0;
    for (int i = 0; i < Q; i++) {
        double eu = o->e[i][0] * u[0] + o->e[i][1] * u[1] + o->e[i][2] * u[2];
        m += mu[i] * o->ws[i] * (we + wo * eu / o->cs2s);
    }
    double nu[ORC_QMAX];
    for (int i = 0; i < Q; i++)
        nu[i] = (1.0 - 0.5 * (we + wo)) * mu[i] + 0.5 * (wo - we) * mu[o->opp[i]] + m;
    /* reactive links: p_i = k/(1+k) 2 w_i C_eq + (1-k)/(1+k) src */
    for (int i = 0; i < Q; i++) {
        if (kd[i] != K_RBC) continue;
        int ob = o->opp[i];
        double k = link_k(o, sol[i], i);
        double dk = link_dk(o, sol[i], i);
        int pulled = p->mechanics == ORC_MECH_PRE && kd[ob] != K_RBC;
        double src = pulled ? gp[ob] : go[x * Q + ob];
        if (!pulled && p->mechanics == ORC_MECH_PRE) { k = k / o->gamma; dk = dk / o->gamma; }
        double csrc;
        if (isinf(k)) {
            csrc = -1.0;
        } else {
            csrc = (1.0 - k) / (1.0 + k);
            double dpdk = 2.0 * (o->ws[i] * p->c_eq - src) / ((1.0 + k) * (1.0 + k));
            grad[sol[i]] += nu[i] * dpdk * dk;
        }
        if (pulled) nu[ob] += csrc * nu[i];          /* through p_ob to its source */
        else lam[x * Q + ob] += csrc * nu[i];        /* the node's own population */
    }
    for (int i = 0; i < Q; i++) {
        if (kd[i] == K_RBC || src_n[i] < 0) continue;
        lam[src_n[i] * Q + src_d[i]] += nu[i];
    }
}

/* Run nsteps forward from the current state, recording every solute state and
 * velocity, then the adjoint of the loss whose gradient with respect to the
 * final concentrations C_T = sum_i g*_i(T) is dLdC [N].  Writes dL/dk_r into
 * grad [N] (zero away from solid interface nodes) and, if lam0 is not NULL,
 * dL/dg*(0) into lam0 [N][Q] (zero outside the solute set).  Leaves the state at step T.  Returns 0, or -1
 * (out of memory), -2 (phase change enabled). */
int orc_adjoint(orc *o, int nsteps, const double *dLdC, double *grad, double *lam0)
{
    const long N = o->N;
    const int Q = o->Q;
    if (o->p.phase_change) return -2;
    if (o->ceq) return -5;                      /* ... with a uniform C_eq */
    double *G = (double *)malloc(sizeof(double) * (size_t)(nsteps > 0 ? nsteps : 1) * N * Q);
    double *U = (double *)malloc(sizeof(double) * (size_t)(nsteps > 0 ? nsteps : 1) * N * 3);
    double *lam = (double *)calloc((size_t)N * Q, sizeof(double));
    double *lnew = (double *)calloc((size_t)N * Q, sizeof(double));
    if (!G || !U || !lam || !lnew) {
        free(G); free(U); free(lam); free(lnew);
        return -1;
    }
    for (int t = 0; t < nsteps; t++) {
        memcpy(G + (size_t)t * N * Q, o->g, sizeof(double) * N * Q);
        memset(U + (size_t)t * N * 3, 0, sizeof(double) * N * 3);
        o->uh = U + (size_t)t * N * 3;
        orc_step(o, 1);
        o->uh = NULL;
    }
    for (long n = 0; n < N; n++) {
        grad[n] = 0.0;
        if (o->solid[n]) continue;
        for (int i = 0; i < Q; i++) lam[n * Q + i] = o->ins[i] ? dLdC[n] : 0.0;
    }
    for (int t = nsteps - 1; t >= 0; t--) {
        memset(lnew, 0, sizeof(double) * N * Q);
        const double *go = G + (size_t)t * N * Q;
        const double *ut = U + (size_t)t * N * 3;
        for (long n = 0; n < N; n++)
            if (!o->solid[n]) adjoint_node(o, n, go, ut + 3 * n, lam + n * Q, lnew, grad);
        double *tmp = lam; lam = lnew; lnew = tmp;
    }
    if (lam0) memcpy(lam0, lam, sizeof(double) * N * Q);
    free(G); free(U); free(lam); free(lnew);
    return 0;
}

void orc_get_fields(const orc *o, double *rho, double *u, double *c, double *phi,
                    uint8_t *type)
{
    const int Q = o->Q;
    for (long n = 0; n < o->N; n++) {
        double r = 0, j[3] = {0, 0, 0}, C = 0;
        if (!o->solid[n]) {
            for (int i = 0; i < Q; i++) {
                double fi = o->f[n * Q + i];
                r += fi;
                for (int d = 0; d < 3; d++) j[d] += fi * o->e[i][d];
                C += o->g[n * Q + i];
            }
        }
        if (rho) rho[n] = r;
        if (u) for (int d = 0; d < 3; d++)
            u[3 * n + d] = o->solid[n] ? 0.0 : (j[d] - 0.5 * o->p.force[d]) / r;
        if (c) c[n] = C;
        if (phi) phi[n] = o->phi[n];
        if (type) type[n] = o->solid[n];
    }
}

/* post-collision populations, structure-of-arrays: f [Q][N], g [QS][N] in
 * the solute set's order */
void orc_get_pops(const orc *o, double *f, double *g)
{
    const int Q = o->Q;
    for (long n = 0; n < o->N; n++) {
        for (int i = 0; i < Q; i++)
            if (f) f[(long)i * o->N + n] = o->f[n * Q + i];
        for (int s = 0; s < o->QS; s++)
            if (g) g[(long)s * o->N + n] = o->g[n * Q + o->sd[s]];
    }
}

void orc_set_pops(orc *o, const double *f, const double *g)
{
    const int Q = o->Q;
    for (long n = 0; n < o->N; n++) {
        for (int i = 0; i < Q; i++)
            if (f) o->f[n * Q + i] = f[(long)i * o->N + n];
        for (int s = 0; s < o->QS; s++)
            if (g) o->g[n * Q + o->sd[s]] = g[(long)s * o->N + n];
    }
}

/* per-node equilibrium concentration of the reaction at solid nodes [N]
 * (NULL: the uniform c_eq) */
void orc_set_ceq(orc *o, const double *ceq)
{
    free(o->ceq);
    o->ceq = NULL;
    if (!ceq) return;
    o->ceq = (double *)malloc(sizeof(double) * o->N);
    memcpy(o->ceq, ceq, sizeof(double) * o->N);
}

/* the solute set: its size, and the fluid direction of each solute direction */
int orc_get_solute_set(const orc *o, int *sd)
{
    for (int s = 0; s < o->QS; s++) sd[s] = o->sd[s];
    return o->QS;
}

/* mass exchanged over each reactive link in the last step, [N][Q] */
void orc_get_exchange(const orc *o, double *q, uint8_t *kind)
{
    long NQ = o->N * o->Q;
    if (q) memcpy(q, o->qx, sizeof(double) * NQ);
    if (kind) memcpy(kind, o->kind, NQ);
}

/* k_i per (fluid node, direction) of the current geometry, [N][Q]; -1 where
 * the incoming population is not a reactive link (a direction outside the
 * solute set has weight 0 and no link) */
void orc_get_link_k(const orc *o, double *k)
{
    const int Q = o->Q;
    for (long n = 0; n < o->N; n++) {
        int X, Y, Z, face;
        coords(o, n, &X, &Y, &Z);
        for (int i = 0; i < Q; i++) {
            k[n * Q + i] = -1.0;
            if (o->solid[n]) continue;
            long y = site(o, X, Y, Z, -o->e[i][0], -o->e[i][1], -o->e[i][2], 1, &face);
            if (y >= 0 && o->solid[y] && o->ws[i] > 0.0) k[n * Q + i] = link_k(o, y, i);
        }
    }
}

void orc_get_normals(const orc *o, double *nrm)
{
    memcpy(nrm, o->nrm, sizeof(double) * 3 * o->N);
}

void orc_get_lattice(const orc *o, int *e, double *wf, double *ws, double *cs2)
{
    for (int i = 0; i < o->Q; i++) {
        for (int d = 0; d < 3; d++) e[3 * i + d] = o->e[i][d];
        wf[i] = o->wf[i];
        ws[i] = o->ws[i];
    }
    cs2[0] = o->cs2f;
    cs2[1] = o->cs2s;
}

/* diagnostics: [0] sum C, [1] sum phi, [2] cumulative reactive-wall exchange,
 * [3] cumulative inlet exchange, [4] cumulative outlet exchange, [5] step,
 * [6] events */
void orc_diag(const orc *o, double *d)
{
    double mc = 0, mp = 0;
    for (long n = 0; n < o->N; n++) {
        if (!o->solid[n]) mc += node_C(o, n);
        mp += o->phi[n];
    }
    d[0] = mc;
    d[1] = mp;
    d[2] = o->wall_ex;
    d[3] = o->inlet_ex;
    d[4] = o->outlet_ex;
    d[5] = (double)o->step;
    d[6] = (double)o->n_events;
}

/* threads of the node loop (timing of the CPU baseline) */
void orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int orc_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
