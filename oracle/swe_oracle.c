/*
 * swe_oracle.c -- plain, slow, FP64 CPU reference of the explicit
 * finite-volume step for the shallow-water equations on unstructured
 * triangles, after Delmas & Soulaimani, "Multi-GPU implementation of a
 * time-explicit finite volume solver for the Shallow-Water Equations using
 * CUDA and a CUDA-Aware version of OpenMPI" (arXiv 2010.14416), sections 2-3.
 *
 * TEST INFRASTRUCTURE ONLY. The test suite, the smoke check and the CPU
 * baseline leg of the benchmark are the only callers. It shares no source,
 * header, table or helper with the GPU library and includes nothing of it.
 *
 * Every function names the passage of the paper it follows. Where the paper
 * is silent, ambiguous or garbled, the comment says "reading:" and states the
 * interpretation taken.
 *
 * reading (rounding order, which the paper leaves open): a quotient by one
 * denominator that a formula uses more than once (the cell area of eq. 37,
 * the depth in the velocities and in the friction Jacobian of eq. 35, |q|,
 * the determinant of the 2x2 solve, S_R - S_L in the star flux of eq. 18)
 * is evaluated as one correctly rounded reciprocal and products. Equal in
 * exact arithmetic to the divisions as printed; one division instead of
 * several.
 *
 * Pins of each function are in tests/test_oracle_*.py; the wall under
 * impinging flow and the fixed-depth / fixed-stage ghosts,
 * which have no closed form, are pinned by balance laws and by equivalent
 * interior edges.
 *
 * Structure of one step, in the paper's order:
 *   1. time step from the current state (eq. 15, per-cell form of sec. 5.3.2)
 *   2. edge loop: hydrostatic reconstruction (eq. 28), rotation (eq. 12),
 *      HLLC flux (eqs. 17-26), back-rotation, bed-slope terms (eq. 30),
 *      boundary fluxes (sec. 3.1)
 *   3. cell loop: sum of the three edge contributions, semi-implicit Manning
 *      friction (eqs. 31-36), explicit Euler update (eq. 37), positivity
 *   4. t += dt
 * Loops 2 and 3 run over independent iterations (OpenMP, static schedule);
 * each cell sums its own three edges in fixed order, so the results do not
 * depend on the number of threads.
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -shared -fPIC swe_oracle.c -lm
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORA_MAX_TAG 1024

enum { K_WALL = 0, K_TRANSMISSIVE = 1, K_INFLOW = 2, K_FIXED_DEPTH = 3,
       K_FIXED_STAGE = 4 };

typedef struct {
    int kind;
    double value;   /* Q [m^3/s], depth [m] or surface elevation [m] */
    double q;       /* inflow per unit length, Q / (sum of edge lengths) */
} ora_bc;

typedef struct ora {
    int64_t nn, nc, ne, nb;
    double *x, *y;
    int32_t *tri;                 /* 3*nc, counter-clockwise */
    double *area, *inr;           /* |Omega_i| and inscribed radius R_i */
    int32_t *e_left, *e_right;    /* right = -1 on the boundary */
    int32_t *e_tag;
    double *e_nx, *e_ny, *e_len;  /* unit normal from left to right cell */
    int32_t *c_edge;              /* 3*nc: edge of local side k */
    int8_t *c_right;              /* 3*nc: 1 if the cell is that edge's right */
    double *z, *man, *h, *hu, *hv;
    double *cl, *cr;              /* 3*ne contributions to left / right cell */
    double *clamp;                /* per cell, mass added by positivity */
    /* monitors: per edge (boundary edges only) the outward volume rate of
       the last step and the volume since the reset; per cell the highest
       depth and the first time with h > h_dry (INFINITY: never) */
    double *brate, *bvol, *hmax, *twet;
    ora_bc bc[ORA_MAX_TAG];
    double g, cfl, h_dry, dt_max;
    double t, last_dt, ledger;
    int64_t step;
    char err[512];
} ora;

/* ---------------------------------------------------------------------- */
/* numerics of one edge                                                   */
/* ---------------------------------------------------------------------- */

/* Star-region depth, both sides wet (sec. 3.2, eqs. 21-23).
 * reading: in eqs. 21-22 the velocity difference is that of the normal
 * velocities u_R - u_L (the extraction prints "U_R - U_L").
 * reading: the two-rarefaction bracket of eq. 22 is clamped at zero before
 * squaring; a negative bracket means a vacuum forms and h* = 0.
 * reading: ties h0 == min(hL, hR) take the rarefaction branch, as printed. */
void ora_star_depth(double g, double hL, double uL, double hR, double uR,
                    double *h0_out, double *hs_out, int *branch)
{
    double aL = sqrt(g * hL), aR = sqrt(g * hR);
    double h0 = 0.5 * (hL + hR) - (uR - uL) * (hL + hR) / (4.0 * (aL + aR));
    double hs;
    double hmin = hL < hR ? hL : hR;
    if (h0 <= hmin) {
        double b = 0.5 * (aL + aR) + 0.25 * (uL - uR);
        if (b < 0.0) b = 0.0;
        hs = b * b / g;
        if (branch) *branch = 0;
    } else {
        double gL = sqrt(g * (h0 + hL) / (2.0 * h0 * hL));
        double gR = sqrt(g * (h0 + hR) / (2.0 * h0 * hR));
        hs = (hL * gL + hR * gR + uL - uR) / (gL + gR);
        if (branch) *branch = 1;
    }
    if (h0_out) *h0_out = h0;
    if (hs_out) *hs_out = hs;
}

/* Wave-speed factor of eq. 20.
 * reading: the printed "[h*(h*+h_k)/2]^{1/2}/2" is taken as
 * [h*(h*+h_k)/2]^{1/2}/h_k, the dimensionless form that equals 1 at
 * h* = h_k (continuity with the second case). */
static double wave_factor(double hs, double hk)
{
    if (hs > hk) return sqrt(hs * (hs + hk) / 2.0) / hk;
    return 1.0;
}

/* Wave speeds S_L, S_R and contact speed S* (eqs. 19-20, 25, 26).
 * Inputs are already the dry-zeroed states. Returns 0 if both sides dry.
 * reading: the second line of eq. 26 is the right-dry case h_R = 0 (the
 * extraction prints h_L = 0 twice). */
int ora_wave_speeds(double g, double hL, double uL, double hR, double uR,
                    int wetL, int wetR, double *SL, double *SR, double *Ss)
{
    double aL = sqrt(g * hL), aR = sqrt(g * hR);
    if (!wetL && !wetR) return 0;
    if (!wetL) {
        *SL = uR - 2.0 * aR;
        *SR = uR + aR;
        *Ss = *SL;
    } else if (!wetR) {
        *SL = uL - aL;
        *SR = uL + 2.0 * aL;
        *Ss = *SR;
    } else {
        double hs;
        ora_star_depth(g, hL, uL, hR, uR, NULL, &hs, NULL);
        *SL = uL - aL * wave_factor(hs, hL);
        *SR = uR + aR * wave_factor(hs, hR);
        *Ss = (*SL * hR * (uR - *SR) - *SR * hL * (uL - *SL))
            / (hR * (uR - *SR) - hL * (uL - *SL));
    }
    return 1;
}

/* Same with the star depth supplied by the caller (used by the tests to check
 * eqs. 19-20 against exact shock speeds). */
void ora_wave_speeds_given_hs(double g, double hL, double uL, double hR,
                              double uR, double hs, double *SL, double *SR)
{
    *SL = uL - sqrt(g * hL) * wave_factor(hs, hL);
    *SR = uR + sqrt(g * hR) * wave_factor(hs, hR);
}

/* One-dimensional flux along the normal, G of eq. 1 written in the rotated
 * frame: (h u, h u^2 + g h^2 / 2, h u v) with u normal, v tangential.
 * reading: eq. 12 writes G(T U); in the rotated frame the Riemann problem is
 * along the first axis, so the second component is the normal momentum and
 * the third the passive tangential one, which is what eq. 24 acts on. */
static void phys_flux(double g, double h, double u, double v, double G[3])
{
    G[0] = h * u;
    G[1] = h * u * u + 0.5 * g * h * h;
    G[2] = h * u * v;
}

/* HLLC flux of sec. 3.2 (eqs. 17-18, 24-26) in the rotated frame.
 * A side with h <= h_dry is dry: its depth and velocities are taken as 0.
 * reading (eq. 24): the passive tangential velocity is taken from the
 * upwind side of the contact, v_L when S* >= 0 and v_R when S* < 0 (the
 * printed assignment is the downwind one); the third component is only
 * replaced in the star region S_L < 0 < S_R, the full side flux applies
 * outside it (eq. 17). */
void ora_hllc(double g, double h_dry, double hL, double uL, double vL,
              double hR, double uR, double vR, double G[3])
{
    int wetL = hL > h_dry, wetR = hR > h_dry;
    double SL, SR, Ss, FL[3], FR[3];
    if (!wetL) { hL = 0.0; uL = 0.0; vL = 0.0; }
    if (!wetR) { hR = 0.0; uR = 0.0; vR = 0.0; }
    if (!ora_wave_speeds(g, hL, uL, hR, uR, wetL, wetR, &SL, &SR, &Ss)) {
        G[0] = G[1] = G[2] = 0.0;
        return;
    }
    phys_flux(g, hL, uL, vL, FL);
    phys_flux(g, hR, uR, vR, FR);
    if (SL >= 0.0) {
        G[0] = FL[0]; G[1] = FL[1]; G[2] = FL[2];
    } else if (SR <= 0.0) {
        G[0] = FR[0]; G[1] = FR[1]; G[2] = FR[2];
    } else {
        /* one reciprocal of S_R - S_L for both components (header) */
        double rS = 1.0 / (SR - SL);
        G[0] = (SR * FL[0] - SL * FR[0] + SR * SL * (hR - hL)) * rS;
        G[1] = (SR * FL[1] - SL * FR[1] + SR * SL * (hR * uR - hL * uL))
             * rS;
        G[2] = G[0] * (Ss >= 0.0 ? vL : vR);
    }
}

/* Back-rotation T^{-1} of eq. 12. */
static void rotate_back(const double G[3], double nx, double ny, double F[3])
{
    F[0] = G[0];
    F[1] = G[1] * nx - G[2] * ny;
    F[2] = G[1] * ny + G[2] * nx;
}

static void velocity(double h_dry, double h, double hu, double hv,
                     double *u, double *v)
{
    /* one reciprocal of h for both velocities (header) */
    if (h > h_dry) { double r = 1.0 / h; *u = hu * r; *v = hv * r; }
    else { *u = 0.0; *v = 0.0; }
}

/* Interior edge between left cell i and right cell j, unit normal n from i
 * to j, length L (eqs. 12-13, 28-30). Writes the contributions to the
 * right-hand side L * (...) of each cell:
 *   cl = -L F + L (g/2)(h_ij**^2 - h_i^2) (0, n)
 *   cr = +L F - L (g/2)(h_ji**^2 - h_j^2) (0, n)
 * reading (eq. 30): the bed-slope term carries g/2, from grad(g h^2 / 2) of
 * eq. 29 (the extraction prints g); only g/2 balances the hydrostatic flux.
 * reading (eq. 37): the flux is evaluated on the reconstructed states U** of
 * eq. 28, as in the method of Audusse and Ata that the section follows.
 * The interface depth max(0, h_i + z_i - z_ij) is evaluated as
 * max(0, h_i - (z_ij - z_i)), equal in exact arithmetic, so that the
 * reconstruction is the identity on a flat bed.
 * reading (wet/dry, not in the paper): an interface depth at or below h_dry
 * counts as zero both in the Riemann problem and in the bed-slope term, so
 * that still water stays still next to films thinner than h_dry. */
void ora_interior_edge(double g, double h_dry,
                       double hi, double hui, double hvi, double zi,
                       double hj, double huj, double hvj, double zj,
                       double nx, double ny, double L,
                       double cl[3], double cr[3])
{
    double ui, vi, uj, vj, G[3], F[3];
    double zs = zi > zj ? zi : zj;
    double hLs = hi - (zs - zi);
    double hRs = hj - (zs - zj);
    if (hLs <= h_dry) hLs = 0.0;
    if (hRs <= h_dry) hRs = 0.0;
    velocity(h_dry, hi, hui, hvi, &ui, &vi);
    velocity(h_dry, hj, huj, hvj, &uj, &vj);
    ora_hllc(g, h_dry,
             hLs, ui * nx + vi * ny, -ui * ny + vi * nx,
             hRs, uj * nx + vj * ny, -uj * ny + vj * nx, G);
    rotate_back(G, nx, ny, F);
    double pL = 0.5 * g * (hLs * hLs - hi * hi);
    double pR = 0.5 * g * (hRs * hRs - hj * hj);
    cl[0] = L * (-F[0]);
    cl[1] = L * (pL * nx - F[1]);
    cl[2] = L * (pL * ny - F[2]);
    cr[0] = L * F[0];
    cr[1] = L * (F[1] - pR * nx);
    cr[2] = L * (F[2] - pR * ny);
}

/* Boundary edge of cell i, outward unit normal n, length L (sec. 3.1).
 * On the boundary z_ij = z_i, so the reconstruction is the identity and the
 * bed-slope term vanishes.
 *  wall:         G = (0, g h^2 / 2, 0)
 *  transmissive: U_R = U_L, i.e. the exact normal flux of U_i
 *  inflow:       G = (-q, q^2 / h + g h^2 / 2, 0), q = Q / (total length of
 *                the tag's edges); q^2/h is dropped on a dry cell
 *  fixed depth:  HLLC with a ghost (h_b, u_n, u_t) of the cell's velocity
 *  fixed stage:  the same with h_b = max(0, value - z_i)
 * reading: the paper prints (g h_l)^2 / 2 for the hydrostatic term; the
 * dimensionally consistent g h_l^2 / 2 is used. The inflow mass flux is -q in
 * the outward-normal frame (water enters). The fixed-depth and fixed-stage
 * kinds are not in the paper; they realise a downstream water level. */
void ora_boundary_edge(double g, double h_dry, int kind, double value,
                       double q, double hi, double hui, double hvi, double zi,
                       double nx, double ny, double L, double cl[3])
{
    double ui, vi, G[3], F[3];
    velocity(h_dry, hi, hui, hvi, &ui, &vi);
    double un = ui * nx + vi * ny, ut = -ui * ny + vi * nx;
    switch (kind) {
    case K_TRANSMISSIVE:
        phys_flux(g, hi, un, ut, G);
        break;
    case K_INFLOW:
        G[0] = -q;
        G[1] = (hi > h_dry ? q * q / hi : 0.0) + 0.5 * g * hi * hi;
        G[2] = 0.0;
        break;
    case K_FIXED_DEPTH:
        ora_hllc(g, h_dry, hi, un, ut, value, un, ut, G);
        break;
    case K_FIXED_STAGE: {
        double hb = value - zi;
        if (hb < 0.0) hb = 0.0;
        ora_hllc(g, h_dry, hi, un, ut, hb, un, ut, G);
        break;
    }
    default: /* wall */
        G[0] = 0.0;
        G[1] = 0.5 * g * hi * hi;
        G[2] = 0.0;
        break;
    }
    rotate_back(G, nx, ny, F);
    cl[0] = L * (-F[0]);
    cl[1] = L * (-F[1]);
    cl[2] = L * (-F[2]);
}

/* Cell update of eq. 37 with semi-implicit Manning friction (eqs. 31-36).
 * R is the sum of the three edge contributions, A the cell area.
 * Friction, for a wet cell with q = (hu, hv) != 0 (eq. 5 in conservative
 * variables):  S_f = -c |q| q,  c = g m^2 h^{-7/3};
 * its Jacobian (eq. 35):  dS_f/dh = (7/3) c |q| q / h,
 *                         dS_f/dq = -c (|q| I + q q^T / |q|).
 * The first row of J is zero, so [I - dt/2 J] dU = dt (R/A + S_f) gives
 * dh = dt R_h / A and the 2x2 system
 *   (I - dt/2 dS_f/dq) dq = dt (R_q / A + S_f) + dt/2 (dS_f/dh) dh.
 * reading: dt multiplies the whole bracket of eq. 37 and the source terms are
 * not scaled by |Omega_i| (the factors printed in eq. 16 are not those of
 * eq. 27).
 * Positivity (not in the paper; reading): a negative depth is set to zero and
 * the mass so added, -A h, is returned in *clamp; at h <= h_dry the
 * discharges are zeroed. */
void ora_cell_update(double g, double h_dry, double dt, double A,
                     double h, double hu, double hv, double m,
                     const double R[3], double out[3], double *clamp)
{
    /* each denominator used several times (|Omega_i|, h, |q|, the
     * determinant) is inverted once (header) */
    double rA = 1.0 / A;
    double bh = R[0] * rA, bx = R[1] * rA, by = R[2] * rA;
    double dh = dt * bh, dqx, dqy;
    double qn = sqrt(hu * hu + hv * hv);
    if (h > h_dry && qn > 0.0) {
        double c = g * m * m / (h * h * cbrt(h));
        double sfx = -c * qn * hu, sfy = -c * qn * hv;
        double rh = 1.0 / h, rq = 1.0 / qn;
        double jhx = (7.0 / 3.0) * c * qn * hu * rh;
        double jhy = (7.0 / 3.0) * c * qn * hv * rh;
        double jxx = -c * (qn + hu * hu * rq);
        double jxy = -c * hu * hv * rq;
        double jyy = -c * (qn + hv * hv * rq);
        double m11 = 1.0 - 0.5 * dt * jxx;
        double m12 = -0.5 * dt * jxy;
        double m22 = 1.0 - 0.5 * dt * jyy;
        double rx = dt * (bx + sfx) + 0.5 * dt * jhx * dh;
        double ry = dt * (by + sfy) + 0.5 * dt * jhy * dh;
        double det = m11 * m22 - m12 * m12;
        double rd = 1.0 / det;
        dqx = (rx * m22 - m12 * ry) * rd;
        dqy = (m11 * ry - m12 * rx) * rd;
    } else {
        dqx = dt * bx;
        dqy = dt * by;
    }
    double hn = h + dh, hun = hu + dqx, hvn = hv + dqy;
    *clamp = 0.0;
    if (hn < 0.0) {
        *clamp = -A * hn;
        hn = 0.0;
    }
    if (hn <= h_dry) {
        hun = 0.0;
        hvn = 0.0;
    }
    out[0] = hn;
    out[1] = hun;
    out[2] = hvn;
}

/* ---------------------------------------------------------------------- */
/* mesh                                                                   */
/* ---------------------------------------------------------------------- */

typedef struct { int32_t a, b, cell, k, fwd; } half_edge;

static int cmp_he(const void *p, const void *q)
{
    const half_edge *u = p, *v = q;
    if (u->a != v->a) return u->a < v->a ? -1 : 1;
    if (u->b != v->b) return u->b < v->b ? -1 : 1;
    if (u->cell != v->cell) return u->cell < v->cell ? -1 : 1;
    return u->k < v->k ? -1 : (u->k > v->k);
}

typedef struct { int32_t a, b, tag; } seg;

static int cmp_seg(const void *p, const void *q)
{
    const seg *u = p, *v = q;
    if (u->a != v->a) return u->a < v->a ? -1 : 1;
    if (u->b != v->b) return u->b < v->b ? -1 : 1;
    return 0;
}

void ora_destroy(ora *o)
{
    if (!o) return;
    free(o->x); free(o->y); free(o->tri); free(o->area); free(o->inr);
    free(o->e_left); free(o->e_right); free(o->e_tag);
    free(o->e_nx); free(o->e_ny); free(o->e_len);
    free(o->c_edge); free(o->c_right);
    free(o->z); free(o->man); free(o->h); free(o->hu); free(o->hv);
    free(o->cl); free(o->cr); free(o->clamp);
    free(o->brate); free(o->bvol); free(o->hmax); free(o->twet);
    free(o);
}

/* Builds the cell-centred finite-volume mesh of sec. 3.1 from nodes and
 * triangles: orients each triangle counter-clockwise, finds the edges shared
 * by two cells (interior) or owned by one (boundary), the unit normal of each
 * edge (from its left cell to its right cell; outward on the boundary), the
 * areas |Omega_i| and the inscribed radius R_i = 2|Omega_i| / perimeter used
 * by the time-step rule of sec. 3.1.
 * The left cell of an interior edge is the one whose counter-clockwise
 * boundary runs along the edge from its lower to its higher node number.
 * Boundary segments (node pairs with a tag) select the boundary condition;
 * unlisted boundary edges carry tag 0. Returns NULL and fills err on error. */
ora *ora_create(int64_t nn, const double *xy, int64_t nc, const int32_t *tri,
                int64_t nseg, const int32_t *seg_nodes, const int32_t *seg_tag,
                char *err, int errlen)
{
    ora *o = calloc(1, sizeof(ora));
    half_edge *he = NULL;
    seg *sg = NULL;
    if (!o) { snprintf(err, errlen, "out of memory"); return NULL; }
#define FAIL(...) do { snprintf(err, errlen, __VA_ARGS__); goto fail; } while (0)
    if (nn < 3 || nc < 1) FAIL("mesh needs at least 3 nodes and 1 cell");
    o->nn = nn; o->nc = nc;
    o->x = malloc(nn * sizeof(double));
    o->y = malloc(nn * sizeof(double));
    o->tri = malloc(3 * nc * sizeof(int32_t));
    o->area = malloc(nc * sizeof(double));
    o->inr = malloc(nc * sizeof(double));
    if (!o->x || !o->y || !o->tri || !o->area || !o->inr) FAIL("out of memory");
    for (int64_t n = 0; n < nn; ++n) {
        o->x[n] = xy[2 * n];
        o->y[n] = xy[2 * n + 1];
        if (!isfinite(o->x[n]) || !isfinite(o->y[n]))
            FAIL("node %lld has a non-finite coordinate", (long long)n);
    }
    for (int64_t c = 0; c < nc; ++c) {
        int32_t v0 = tri[3 * c], v1 = tri[3 * c + 1], v2 = tri[3 * c + 2];
        if (v0 < 0 || v1 < 0 || v2 < 0 || v0 >= nn || v1 >= nn || v2 >= nn)
            FAIL("cell %lld references a node out of range", (long long)c);
        if (v0 == v1 || v1 == v2 || v0 == v2)
            FAIL("cell %lld repeats a node", (long long)c);
        double a2 = (o->x[v1] - o->x[v0]) * (o->y[v2] - o->y[v0])
                  - (o->x[v2] - o->x[v0]) * (o->y[v1] - o->y[v0]);
        if (a2 == 0.0) FAIL("cell %lld has zero area", (long long)c);
        if (a2 < 0.0) { int32_t t = v1; v1 = v2; v2 = t; a2 = -a2; }
        o->tri[3 * c] = v0; o->tri[3 * c + 1] = v1; o->tri[3 * c + 2] = v2;
        o->area[c] = 0.5 * a2;
        double per = 0.0;
        for (int k = 0; k < 3; ++k) {
            int32_t p = o->tri[3 * c + k], q = o->tri[3 * c + (k + 1) % 3];
            double dx = o->x[q] - o->x[p], dy = o->y[q] - o->y[p];
            per += sqrt(dx * dx + dy * dy);
        }
        o->inr[c] = 2.0 * o->area[c] / per;
    }

    /* edges from sorted half-edges */
    he = malloc(3 * nc * sizeof(half_edge));
    if (!he) FAIL("out of memory");
    for (int64_t c = 0; c < nc; ++c)
        for (int k = 0; k < 3; ++k) {
            int32_t p = o->tri[3 * c + k], q = o->tri[3 * c + (k + 1) % 3];
            half_edge *h = &he[3 * c + k];
            h->a = p < q ? p : q;
            h->b = p < q ? q : p;
            h->cell = (int32_t)c;
            h->k = k;
            h->fwd = p < q;
        }
    qsort(he, 3 * nc, sizeof(half_edge), cmp_he);
    int64_t ne = 0, nb = 0;
    for (int64_t i = 0; i < 3 * nc;) {
        int64_t j = i + 1;
        while (j < 3 * nc && he[j].a == he[i].a && he[j].b == he[i].b) ++j;
        if (j - i > 2)
            FAIL("edge (%d,%d) is shared by more than two cells", he[i].a,
                 he[i].b);
        if (j - i == 2 && he[i].fwd == he[i + 1].fwd)
            FAIL("cells %d and %d overlap along edge (%d,%d)", he[i].cell,
                 he[i + 1].cell, he[i].a, he[i].b);
        if (j - i == 1) ++nb;
        ++ne;
        i = j;
    }
    o->ne = ne; o->nb = nb;
    o->e_left = malloc(ne * sizeof(int32_t));
    o->e_right = malloc(ne * sizeof(int32_t));
    o->e_tag = calloc(ne, sizeof(int32_t));
    o->e_nx = malloc(ne * sizeof(double));
    o->e_ny = malloc(ne * sizeof(double));
    o->e_len = malloc(ne * sizeof(double));
    o->c_edge = malloc(3 * nc * sizeof(int32_t));
    o->c_right = malloc(3 * nc * sizeof(int8_t));
    if (!o->e_left || !o->e_right || !o->e_tag || !o->e_nx || !o->e_ny ||
        !o->e_len || !o->c_edge || !o->c_right)
        FAIL("out of memory");

    /* boundary segments, sorted for lookup */
    if (nseg > 0) {
        sg = malloc(nseg * sizeof(seg));
        if (!sg) FAIL("out of memory");
        for (int64_t s = 0; s < nseg; ++s) {
            int32_t p = seg_nodes[2 * s], q = seg_nodes[2 * s + 1];
            if (p < 0 || q < 0 || p >= nn || q >= nn || p == q)
                FAIL("boundary segment %lld has invalid nodes", (long long)s);
            if (seg_tag[s] < 0 || seg_tag[s] >= ORA_MAX_TAG)
                FAIL("boundary segment %lld has tag %d out of [0,%d)",
                     (long long)s, seg_tag[s], ORA_MAX_TAG);
            sg[s].a = p < q ? p : q;
            sg[s].b = p < q ? q : p;
            sg[s].tag = seg_tag[s];
        }
        qsort(sg, nseg, sizeof(seg), cmp_seg);
        for (int64_t s = 1; s < nseg; ++s)
            if (sg[s].a == sg[s - 1].a && sg[s].b == sg[s - 1].b)
                FAIL("boundary segment (%d,%d) listed twice", sg[s].a, sg[s].b);
    }
    int64_t nseg_found = 0;
    int64_t e = 0;
    for (int64_t i = 0; i < 3 * nc; ++e) {
        int64_t j = i + 1;
        while (j < 3 * nc && he[j].a == he[i].a && he[j].b == he[i].b) ++j;
        const half_edge *hl, *hr = NULL;
        if (j - i == 2) {
            hl = he[i].fwd ? &he[i] : &he[i + 1];
            hr = he[i].fwd ? &he[i + 1] : &he[i];
        } else {
            hl = &he[i];
        }
        /* the left cell runs along the edge from p to q, counter-clockwise;
           its outward normal is (dy, -dx) / L */
        int32_t p = o->tri[3 * hl->cell + hl->k];
        int32_t q = o->tri[3 * hl->cell + (hl->k + 1) % 3];
        double dx = o->x[q] - o->x[p], dy = o->y[q] - o->y[p];
        double L = sqrt(dx * dx + dy * dy);
        o->e_len[e] = L;
        o->e_nx[e] = dy / L;
        o->e_ny[e] = -dx / L;
        o->e_left[e] = hl->cell;
        o->c_edge[3 * hl->cell + hl->k] = (int32_t)e;
        o->c_right[3 * hl->cell + hl->k] = 0;
        if (hr) {
            o->e_right[e] = hr->cell;
            o->c_edge[3 * hr->cell + hr->k] = (int32_t)e;
            o->c_right[3 * hr->cell + hr->k] = 1;
        } else {
            o->e_right[e] = -1;
            if (nseg > 0) {
                seg key = { he[i].a, he[i].b, 0 };
                seg *f = bsearch(&key, sg, nseg, sizeof(seg), cmp_seg);
                if (f) { o->e_tag[e] = f->tag; ++nseg_found; }
            }
        }
        i = j;
    }
    if (nseg_found != nseg)
        FAIL("%lld boundary segment(s) are not boundary edges of the mesh",
             (long long)(nseg - nseg_found));
    free(he); he = NULL;
    free(sg); sg = NULL;

    o->z = calloc(nc, sizeof(double));
    o->man = calloc(nc, sizeof(double));
    o->h = calloc(nc, sizeof(double));
    o->hu = calloc(nc, sizeof(double));
    o->hv = calloc(nc, sizeof(double));
    o->cl = malloc(3 * ne * sizeof(double));
    o->cr = malloc(3 * ne * sizeof(double));
    o->clamp = malloc(nc * sizeof(double));
    o->brate = calloc(ne, sizeof(double));
    o->bvol = calloc(ne, sizeof(double));
    o->hmax = calloc(nc, sizeof(double));
    o->twet = malloc(nc * sizeof(double));
    if (!o->z || !o->man || !o->h || !o->hu || !o->hv || !o->cl || !o->cr ||
        !o->clamp || !o->brate || !o->bvol || !o->hmax || !o->twet)
        FAIL("out of memory");
    for (int64_t i = 0; i < nc; ++i) o->twet[i] = INFINITY;
    for (int k = 0; k < ORA_MAX_TAG; ++k) o->bc[k].kind = K_WALL;
    o->g = 9.81; o->cfl = 0.9; o->h_dry = 1e-6; o->dt_max = INFINITY;
    return o;
fail:
#undef FAIL
    free(he);
    free(sg);
    ora_destroy(o);
    return NULL;
}

int ora_set_bc(ora *o, int tag, int kind, double value)
{
    if (tag < 0 || tag >= ORA_MAX_TAG || kind < 0 || kind > 4 ||
        !isfinite(value)) return -1;
    if (kind == K_FIXED_DEPTH && value < 0.0) return -1;
    o->bc[tag].kind = kind;
    o->bc[tag].value = value;
    return 0;
}

int ora_set_params(ora *o, double g, double cfl, double h_dry, double dt_max)
{
    if (!(g > 0.0) || !(cfl > 0.0) || !(h_dry >= 0.0) || !(dt_max > 0.0))
        return -1;
    o->g = g; o->cfl = cfl; o->h_dry = h_dry; o->dt_max = dt_max;
    return 0;
}

int ora_set_fields(ora *o, const double *z, const double *man)
{
    for (int64_t i = 0; i < o->nc; ++i)
        if (!isfinite(z[i]) || !(man[i] >= 0.0) || !isfinite(man[i]))
            return -1;
    memcpy(o->z, z, o->nc * sizeof(double));
    memcpy(o->man, man, o->nc * sizeof(double));
    return 0;
}

void ora_reset_monitors(ora *o);

int ora_set_state(ora *o, const double *h, const double *hu, const double *hv)
{
    for (int64_t i = 0; i < o->nc; ++i)
        if (!(h[i] >= 0.0) || !isfinite(h[i]) || !isfinite(hu[i]) ||
            !isfinite(hv[i]))
            return -1;
    memcpy(o->h, h, o->nc * sizeof(double));
    memcpy(o->hu, hu, o->nc * sizeof(double));
    memcpy(o->hv, hv, o->nc * sizeof(double));
    ora_reset_monitors(o);
    return 0;
}

/* Monitors of the outflow / inflow rates (sec. 5.3.2) and of the flooded
 * area (flood lines, sec. 6.4.3), restarted from the current state: zero
 * rates and volumes, h_max = h, t_wet = t on wet cells. */
void ora_reset_monitors(ora *o)
{
    memset(o->brate, 0, o->ne * sizeof(double));
    memset(o->bvol, 0, o->ne * sizeof(double));
    for (int64_t i = 0; i < o->nc; ++i) {
        o->hmax[i] = o->h[i];
        o->twet[i] = o->h[i] > o->h_dry ? o->t : INFINITY;
    }
}

/* Rate [m^3/s] of the last step and volume [m^3] since the reset leaving
 * the domain through the boundary edges of one tag, summed in edge order. */
void ora_discharge(const ora *o, int tag, double *rate, double *volume)
{
    double r = 0.0, v = 0.0;
    for (int64_t e = 0; e < o->ne; ++e)
        if (o->e_right[e] < 0 && o->e_tag[e] == tag) {
            r += o->brate[e];
            v += o->bvol[e];
        }
    *rate = r;
    *volume = v;
}

void ora_envelope(const ora *o, double *hmax, double *twet)
{
    memcpy(hmax, o->hmax, o->nc * sizeof(double));
    memcpy(twet, o->twet, o->nc * sizeof(double));
}

void ora_get_state(const ora *o, double *h, double *hu, double *hv)
{
    memcpy(h, o->h, o->nc * sizeof(double));
    memcpy(hu, o->hu, o->nc * sizeof(double));
    memcpy(hv, o->hv, o->nc * sizeof(double));
}

void ora_set_time(ora *o, double t, int64_t step)
{
    o->t = t;
    o->step = step;
}

void ora_get_time(const ora *o, double *t, double *last_dt, int64_t *step,
                  double *ledger)
{
    *t = o->t;
    *last_dt = o->last_dt;
    *step = o->step;
    *ledger = o->ledger;
}

void ora_counts(const ora *o, int64_t *nn, int64_t *nc, int64_t *ne,
                int64_t *nb)
{
    *nn = o->nn; *nc = o->nc; *ne = o->ne; *nb = o->nb;
}

void ora_geometry(const ora *o, double *area, double *inr, int32_t *tri_ccw)
{
    memcpy(area, o->area, o->nc * sizeof(double));
    memcpy(inr, o->inr, o->nc * sizeof(double));
    memcpy(tri_ccw, o->tri, 3 * o->nc * sizeof(int32_t));
}

void ora_edges(const ora *o, int32_t *left, int32_t *right, int32_t *tag,
               double *nx, double *ny, double *len, int32_t *c_edge,
               int8_t *c_right)
{
    memcpy(left, o->e_left, o->ne * sizeof(int32_t));
    memcpy(right, o->e_right, o->ne * sizeof(int32_t));
    memcpy(tag, o->e_tag, o->ne * sizeof(int32_t));
    memcpy(nx, o->e_nx, o->ne * sizeof(double));
    memcpy(ny, o->e_ny, o->ne * sizeof(double));
    memcpy(len, o->e_len, o->ne * sizeof(double));
    memcpy(c_edge, o->c_edge, 3 * o->nc * sizeof(int32_t));
    memcpy(c_right, o->c_right, 3 * o->nc * sizeof(int8_t));
}

/* ---------------------------------------------------------------------- */
/* time stepping                                                          */
/* ---------------------------------------------------------------------- */

/* min over wet cells of R_i / (sqrt(g h_i) + |V_i|): the time-step rule of
 * eq. 15 with d = R_i (sec. 3.1), taken per cell as in sec. 5.3.2.
 * reading: the maximum and minimum of eq. 15 are taken together per cell,
 * dt = CFL * min_i R_i / s_i, the form the paper computes ("a local time step
 * for each cell", then a minimum reduction). Returns +inf if no cell is wet. */
double ora_min_rs(const ora *o)
{
    double m = INFINITY;
    const double g = o->g, h_dry = o->h_dry;
#pragma omp parallel for schedule(static) reduction(min : m)
    for (int64_t i = 0; i < o->nc; ++i) {
        double h = o->h[i];
        if (h > h_dry) {
            double rh = 1.0 / h;
            double u = o->hu[i] * rh, v = o->hv[i] * rh;
            double s = sqrt(g * h) + sqrt(u * u + v * v);
            double r = o->inr[i] / s;
            if (r < m) m = r;
        }
    }
    return m;
}

double ora_mass(const ora *o)
{
    double m = 0.0;
    for (int64_t i = 0; i < o->nc; ++i) m += o->area[i] * o->h[i];
    return m;
}

/* Advances up to max_steps explicit steps, stopping when t reaches t_end
 * (the last step is shortened to land on t_end exactly). nthreads <= 0 keeps
 * the OpenMP default. Returns 0, or -1 with a message (ora_error) on a
 * non-finite state or an unbounded time step. */
static int run_steps(ora *o, int64_t max_steps, double t_end,
                     const double *dt_fixed, int nthreads,
                     int64_t *steps_done, double *t_now);

int ora_run(ora *o, int64_t max_steps, double t_end, int nthreads,
            int64_t *steps_done, double *t_now)
{
    return run_steps(o, max_steps, t_end, NULL, nthreads, steps_done, t_now);
}

/* n steps with a frozen schedule: step k takes dt[k] as its time step
 * (the forward pass whose time steps an adjoint keeps fixed). */
int ora_run_dt(ora *o, int64_t n, const double *dt, int nthreads)
{
    int64_t done;
    double t;
    return run_steps(o, n, INFINITY, dt, nthreads, &done, &t);
}

static int run_steps(ora *o, int64_t max_steps, double t_end,
                     const double *dt_fixed, int nthreads,
                     int64_t *steps_done, double *t_now)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
    const double g = o->g, h_dry = o->h_dry;
    /* inflow per unit length of each tag */
    double lsum[ORA_MAX_TAG];
    memset(lsum, 0, sizeof(lsum));
    for (int64_t e = 0; e < o->ne; ++e)
        if (o->e_right[e] < 0) lsum[o->e_tag[e]] += o->e_len[e];
    for (int k = 0; k < ORA_MAX_TAG; ++k)
        o->bc[k].q = (o->bc[k].kind == K_INFLOW && lsum[k] > 0.0)
                         ? o->bc[k].value / lsum[k] : 0.0;
    int64_t done = 0;
    while (done < max_steps && o->t < t_end) {
        double dt, tn;
        if (dt_fixed) {
            dt = dt_fixed[done];
            tn = o->t + dt;
        } else {
            double m = ora_min_rs(o);
            dt = o->cfl * m;
            if (dt > o->dt_max) dt = o->dt_max;
            double rem = t_end - o->t;
            if (dt >= rem) { dt = rem; tn = t_end; }
            else tn = o->t + dt;
        }
        if (!(dt < INFINITY)) {
            snprintf(o->err, sizeof o->err,
                     "step %lld: no wet cell and no bound on the time step",
                     (long long)o->step);
            return -1;
        }
        /* edge loop */
#pragma omp parallel for schedule(static)
        for (int64_t e = 0; e < o->ne; ++e) {
            int32_t i = o->e_left[e], j = o->e_right[e];
            if (j >= 0) {
                ora_interior_edge(g, h_dry, o->h[i], o->hu[i], o->hv[i],
                                  o->z[i], o->h[j], o->hu[j], o->hv[j],
                                  o->z[j], o->e_nx[e], o->e_ny[e],
                                  o->e_len[e], &o->cl[3 * e], &o->cr[3 * e]);
            } else {
                const ora_bc *b = &o->bc[o->e_tag[e]];
                ora_boundary_edge(g, h_dry, b->kind, b->value, b->q, o->h[i],
                                  o->hu[i], o->hv[i], o->z[i], o->e_nx[e],
                                  o->e_ny[e], o->e_len[e], &o->cl[3 * e]);
            }
        }
        /* monitors: a boundary edge's contribution to its cell is
           cl = -L F with F_1 = G_1, the outward normal mass flux, so the
           volume leaving per unit time is L G_1 = -cl_1 */
        for (int64_t e = 0; e < o->ne; ++e)
            if (o->e_right[e] < 0) {
                o->brate[e] = -o->cl[3 * e];
                o->bvol[e] += dt * o->brate[e];
            }
        /* cell loop: the new state is written in place once every edge of
           the step has been evaluated */
        int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
        for (int64_t i = 0; i < o->nc; ++i) {
            double R[3] = { 0.0, 0.0, 0.0 }, out[3];
            for (int k = 0; k < 3; ++k) {
                int32_t e = o->c_edge[3 * i + k];
                const double *c = o->c_right[3 * i + k] ? &o->cr[3 * e]
                                                        : &o->cl[3 * e];
                R[0] += c[0];
                R[1] += c[1];
                R[2] += c[2];
            }
            ora_cell_update(g, h_dry, dt, o->area[i], o->h[i], o->hu[i],
                            o->hv[i], o->man[i], R, out, &o->clamp[i]);
            o->h[i] = out[0];
            o->hu[i] = out[1];
            o->hv[i] = out[2];
            if (out[0] > o->hmax[i]) o->hmax[i] = out[0];
            if (o->twet[i] == INFINITY && out[0] > h_dry) o->twet[i] = tn;
            if (!isfinite(out[0]) || !isfinite(out[1]) || !isfinite(out[2]))
                bad = 1;
        }
        double cs = 0.0;
        for (int64_t i = 0; i < o->nc; ++i) cs += o->clamp[i];
        o->ledger += cs;
        o->t = tn;
        o->last_dt = dt;
        o->step += 1;
        ++done;
        if (bad) {
            snprintf(o->err, sizeof o->err,
                     "step %lld: non-finite state", (long long)o->step);
            *steps_done = done;
            *t_now = o->t;
            return -1;
        }
    }
    *steps_done = done;
    *t_now = o->t;
    return 0;
}

const char *ora_error(const ora *o) { return o->err; }
