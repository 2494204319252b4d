/*
 * FP64 reference implementation ("oracle") of the qubit lattice algorithm
 * (QLA) for the 2D curl-Maxwell equations in a diagonal-tensor dielectric,
 * after G. Vahala et al., "Qubit Lattice Algorithm Simulations of Maxwell's
 * Equations for Scattering from Anisotropic Dielectric Objects",
 * arXiv:2301.13601 (2023).
 *
 * TEST INFRASTRUCTURE. This file exists to check the HIP library: only the
 * test suite, the package's smoke check and the benchmark's CPU-baseline leg
 * may load it. It shares no source, header, table or helper with the HIP
 * library, and the library never calls it.
 *
 * Plain, slow and literal by design: one full pass over the lattice per
 * operator, in the order the paper writes the operator products, all in
 * double precision with libm sin/cos. No fusion, blocking or reordering.
 *
 * Data layout: q[c][y][x] for c = 0..5 (Q = (n_x E_x, n_y E_y, n_z E_z,
 * B_x, B_y, B_z), Eq. (15)) and n[c][y][x] for c = 0..2 (n_x, n_y, n_z);
 * x is the fastest index. The lattice is periodic in x and y.
 *
 * Readings of the paper taken here (each is argued in the design notes):
 *  - Components are numbered q0..q5 (Eq. (16)); matrix rows/columns of
 *    Eq. (17), (19), (21), (22) map to q0..q5.
 *  - Operator products act right to left (the rightmost factor first).
 *  - Streaming "pulls": S^{+x}_{ab} replaces q_a, q_b at site x by their
 *    values at x+1 (and S^{-x} by the values at x-1). This is the
 *    direction under which Eq. (17)-(20) reproduce the signs of Eq. (16).
 *  - Eq. (19), row 2: the sin(theta_2) entry sits in column 3 (the printed
 *    column 4 makes C_Y non-orthogonal).
 *  - Eq. (22): the "o" in row 0 is 0, and row 3 reads
 *    q3' = sin(beta_3) q2 + cos(beta_3) q3 (the form Eq. (26) requires).
 *  - Collision angles are evaluated at the collision site; C and C^dagger
 *    at a site use the same angle.
 *  - Eq. (25): the derivative of n is the periodic central difference in
 *    cells, scaled by kappa: kappa = delta (lattice spacing delta in the
 *    coordinates of Eq. (25)), kappa = delta^2 (per-cell derivative), or
 *    kappa = 0 (no potentials: the pure collide-stream sequence).
 *  - Eq. (28): the interleaved potentials use half angles and act after the
 *    8th and after the 16th operator of each directional sequence; the
 *    x potentials act before U_Y.
 *
 * Besides the printed potentials the oracle holds one variant the paper
 * names as future work but does not specify (a unitary potential): the
 * skew-symmetric part of V_X, V_Y. The printed V at angle b differs from the
 * identity, to first order in b, by b times a matrix G with a single entry
 * per coupled pair; the variant replaces V by exp(b (G - G^T) / 2), which
 * is a rotation by b/2 in the same pair and in the sense of the printed
 * coupling. It is orthogonal, so with it every step conserves Eq. (27).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { POT_EQ23 = 0, POT_EQ28 = 1 };
enum { BETA_PHYS = 0, BETA_LATTICE = 1, BETA_OFF = 2 };
enum { V_PRINTED = 0, V_SKEW = 1 };

typedef struct {
    int nx, ny;
    int64_t sites;
    double *theta;   /* theta[c][site], c = 0,1,2: Eq. (24)            */
    double *beta;    /* beta[k][site],  k = 0..3:  Eq. (25)            */
    double *tmp;     /* one plane of scratch for the streaming shifts  */
    int v_form;      /* V_PRINTED or V_SKEW                             */
} lattice;

#define AT(plane, c, s, L) ((plane)[(int64_t)(c) * (L)->sites + (s)])

static int wrap(int i, int n) {
    int r = i % n;
    return r < 0 ? r + n : r;
}

/* ---------------------------------------------------------------------------
 * Angles.
 * Eq. (24): theta_0 = delta/(4 n_x), theta_1 = delta/(4 n_y),
 *           theta_2 = delta/(4 n_z).
 * Eq. (25): beta_0 = kappa * D_x n_y / n_y^2, beta_1 = kappa * D_y n_x / n_x^2,
 *           beta_2 = kappa * D_x n_z / n_z^2, beta_3 = kappa * D_y n_z / n_z^2,
 * with D_x f(x,y) = (f(x+1,y) - f(x-1,y))/2 (periodic) and likewise D_y.
 * ------------------------------------------------------------------------- */
static void compute_angles(lattice *L, const double *n, double delta, double kappa) {
    const int nx = L->nx, ny = L->ny;
    for (int y = 0; y < ny; ++y) {
        for (int x = 0; x < nx; ++x) {
            const int64_t s = (int64_t)y * nx + x;
            for (int c = 0; c < 3; ++c)
                AT(L->theta, c, s, L) = delta / (4.0 * AT(n, c, s, L));
            const int64_t sxp = (int64_t)y * nx + wrap(x + 1, nx);
            const int64_t sxm = (int64_t)y * nx + wrap(x - 1, nx);
            const int64_t syp = (int64_t)wrap(y + 1, ny) * nx + x;
            const int64_t sym = (int64_t)wrap(y - 1, ny) * nx + x;
            const double nxs = AT(n, 0, s, L), nys = AT(n, 1, s, L), nzs = AT(n, 2, s, L);
            const double dx_ny = 0.5 * (AT(n, 1, sxp, L) - AT(n, 1, sxm, L));
            const double dy_nx = 0.5 * (AT(n, 0, syp, L) - AT(n, 0, sym, L));
            const double dx_nz = 0.5 * (AT(n, 2, sxp, L) - AT(n, 2, sxm, L));
            const double dy_nz = 0.5 * (AT(n, 2, syp, L) - AT(n, 2, sym, L));
            AT(L->beta, 0, s, L) = kappa * dx_ny / (nys * nys);
            AT(L->beta, 1, s, L) = kappa * dy_nx / (nxs * nxs);
            AT(L->beta, 2, s, L) = kappa * dx_nz / (nzs * nzs);
            AT(L->beta, 3, s, L) = kappa * dy_nz / (nzs * nzs);
        }
    }
}

/* Rotation of the pair (a, b) by phi: a' = cos(phi) a - sin(phi) b,
 * b' = sin(phi) a + cos(phi) b. */
static void rotate(double *a, double *b, double phi) {
    const double c = cos(phi), s = sin(phi);
    const double a0 = *a, b0 = *b;
    *a = c * a0 - s * b0;
    *b = s * a0 + c * b0;
}

/* ---------------------------------------------------------------------------
 * Eq. (17): C_X rotates (q1, q5) by theta_1 and (q2, q4) by theta_2.
 * sign = +1 applies C_X, sign = -1 applies C_X^dagger (angles negated).
 * ------------------------------------------------------------------------- */
static void collide_x(lattice *L, double *q, int sign) {
    const int64_t N = L->sites;
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < N; ++s) {
        const double th1 = sign * AT(L->theta, 1, s, L);
        const double th2 = sign * AT(L->theta, 2, s, L);
        rotate(&AT(q, 1, s, L), &AT(q, 5, s, L), th1);
        rotate(&AT(q, 2, s, L), &AT(q, 4, s, L), th2);
    }
}

/* ---------------------------------------------------------------------------
 * Eq. (19): C_Y. Row 0 is q0' = cos(theta_0) q0 + sin(theta_0) q5 and row 5
 * is q5' = -sin(theta_0) q0 + cos(theta_0) q5, i.e. (q0, q5) rotated by
 * -theta_0; rows 2 and 3 rotate (q2, q3) by -theta_2. sign = -1 applies
 * C_Y^dagger.
 * ------------------------------------------------------------------------- */
static void collide_y(lattice *L, double *q, int sign) {
    const int64_t N = L->sites;
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < N; ++s) {
        const double th0 = -sign * AT(L->theta, 0, s, L);
        const double th2 = -sign * AT(L->theta, 2, s, L);
        rotate(&AT(q, 0, s, L), &AT(q, 5, s, L), th0);
        rotate(&AT(q, 2, s, L), &AT(q, 3, s, L), th2);
    }
}

/* ---------------------------------------------------------------------------
 * Streaming S^{(dx,dy)}_{ab} (Sec. 3): components a and b move one lattice
 * cell; the other four are unchanged. Pull form: the new value at (x, y) is
 * the old value at (x + dx, y + dy), periodic.
 * ------------------------------------------------------------------------- */
static void stream_one(lattice *L, double *q, int c, int dx, int dy) {
    const int nx = L->nx, ny = L->ny;
    double *plane = q + (int64_t)c * L->sites;
    memcpy(L->tmp, plane, sizeof(double) * (size_t)L->sites);
#pragma omp parallel for schedule(static)
    for (int y = 0; y < ny; ++y) {
        const int ys = wrap(y + dy, ny);
        for (int x = 0; x < nx; ++x) {
            const int xs = wrap(x + dx, nx);
            plane[(int64_t)y * nx + x] = L->tmp[(int64_t)ys * nx + xs];
        }
    }
}

static void stream(lattice *L, double *q, int a, int b, int dx, int dy) {
    stream_one(L, q, a, dx, dy);
    stream_one(L, q, b, dx, dy);
}

/* ---------------------------------------------------------------------------
 * Eq. (21): V_X. Row 4: q4' = -sin(beta_2) q2 + cos(beta_2) q4.
 *                 Row 5: q5' =  sin(beta_0) q1 + cos(beta_0) q5.
 * The inputs q1, q2 are rows the operator leaves unchanged, so the two rows
 * can be applied in either order. ``frac`` scales the angles (1/2 for the
 * interleaved form of Eq. (28)).
 * ------------------------------------------------------------------------- */
static void potential_x(lattice *L, double *q, double frac) {
    const int64_t N = L->sites;
    const int skew = L->v_form == V_SKEW;
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < N; ++s) {
        const double b0 = frac * AT(L->beta, 0, s, L);
        const double b2 = frac * AT(L->beta, 2, s, L);
        if (skew) {
            /* row 4 couples -q2 into q4: rotate (q4, q2) by b2/2;
             * row 5 couples +q1 into q5: rotate (q1, q5) by b0/2 */
            rotate(&AT(q, 4, s, L), &AT(q, 2, s, L), 0.5 * b2);
            rotate(&AT(q, 1, s, L), &AT(q, 5, s, L), 0.5 * b0);
            continue;
        }
        const double q1 = AT(q, 1, s, L), q2 = AT(q, 2, s, L);
        const double q4 = AT(q, 4, s, L), q5 = AT(q, 5, s, L);
        AT(q, 4, s, L) = -sin(b2) * q2 + cos(b2) * q4;
        AT(q, 5, s, L) = sin(b0) * q1 + cos(b0) * q5;
    }
}

/* ---------------------------------------------------------------------------
 * Eq. (22): V_Y. Row 3: q3' =  sin(beta_3) q2 + cos(beta_3) q3.
 *                 Row 5: q5' = -sin(beta_1) q0 + cos(beta_1) q5.
 * ------------------------------------------------------------------------- */
static void potential_y(lattice *L, double *q, double frac) {
    const int64_t N = L->sites;
    const int skew = L->v_form == V_SKEW;
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < N; ++s) {
        const double b1 = frac * AT(L->beta, 1, s, L);
        const double b3 = frac * AT(L->beta, 3, s, L);
        if (skew) {
            /* row 3 couples +q2 into q3: rotate (q2, q3) by b3/2;
             * row 5 couples -q0 into q5: rotate (q5, q0) by b1/2 */
            rotate(&AT(q, 2, s, L), &AT(q, 3, s, L), 0.5 * b3);
            rotate(&AT(q, 5, s, L), &AT(q, 0, s, L), 0.5 * b1);
            continue;
        }
        const double q0 = AT(q, 0, s, L), q2 = AT(q, 2, s, L);
        const double q3 = AT(q, 3, s, L), q5 = AT(q, 5, s, L);
        AT(q, 3, s, L) = sin(b3) * q2 + cos(b3) * q3;
        AT(q, 5, s, L) = -sin(b1) * q0 + cos(b1) * q5;
    }
}

/* ---------------------------------------------------------------------------
 * Eq. (18), applied right to left. The product splits into two halves of
 * eight operators; Eq. (28) inserts a potential after each half.
 *   first half:  C^dag, S^{-}_{14}, C, S^{+}_{14}, C^dag, S^{+}_{25}, C, S^{-}_{25}
 *   second half: C, S^{+}_{14}, C^dag, S^{-}_{14}, C, S^{-}_{25}, C^dag, S^{+}_{25}
 * ------------------------------------------------------------------------- */
static void sweep_x_first_half(lattice *L, double *q) {
    collide_x(L, q, -1);
    stream(L, q, 1, 4, -1, 0);
    collide_x(L, q, +1);
    stream(L, q, 1, 4, +1, 0);
    collide_x(L, q, -1);
    stream(L, q, 2, 5, +1, 0);
    collide_x(L, q, +1);
    stream(L, q, 2, 5, -1, 0);
}

static void sweep_x_second_half(lattice *L, double *q) {
    collide_x(L, q, +1);
    stream(L, q, 1, 4, +1, 0);
    collide_x(L, q, -1);
    stream(L, q, 1, 4, -1, 0);
    collide_x(L, q, +1);
    stream(L, q, 2, 5, -1, 0);
    collide_x(L, q, -1);
    stream(L, q, 2, 5, +1, 0);
}

/* Eq. (20): Eq. (18) with S_{14} -> S_{03}, x -> y and C_X -> C_Y. */
static void sweep_y_first_half(lattice *L, double *q) {
    collide_y(L, q, -1);
    stream(L, q, 0, 3, 0, -1);
    collide_y(L, q, +1);
    stream(L, q, 0, 3, 0, +1);
    collide_y(L, q, -1);
    stream(L, q, 2, 5, 0, +1);
    collide_y(L, q, +1);
    stream(L, q, 2, 5, 0, -1);
}

static void sweep_y_second_half(lattice *L, double *q) {
    collide_y(L, q, +1);
    stream(L, q, 0, 3, 0, +1);
    collide_y(L, q, -1);
    stream(L, q, 0, 3, 0, -1);
    collide_y(L, q, +1);
    stream(L, q, 2, 5, 0, -1);
    collide_y(L, q, -1);
    stream(L, q, 2, 5, 0, +1);
}

/* One time step.
 * Eq. (23): Q <- V_Y V_X U_Y U_X Q.
 * Eq. (28): Q <- V_Y' U_Y^(2) V_Y' U_Y^(1) V_X' U_X^(2) V_X' U_X^(1) Q, where
 *           U^(1), U^(2) are the halves above and V' uses beta/2. */
static void full_step(lattice *L, double *q, int pot_mode) {
    if (pot_mode == POT_EQ23) {
        sweep_x_first_half(L, q);
        sweep_x_second_half(L, q);
        sweep_y_first_half(L, q);
        sweep_y_second_half(L, q);
        potential_x(L, q, 1.0);
        potential_y(L, q, 1.0);
    } else {
        sweep_x_first_half(L, q);
        potential_x(L, q, 0.5);
        sweep_x_second_half(L, q);
        potential_x(L, q, 0.5);
        sweep_y_first_half(L, q);
        potential_y(L, q, 0.5);
        sweep_y_second_half(L, q);
        potential_y(L, q, 0.5);
    }
}

/* ---------------------------------------------------------------------------
 * Exported entry points (C ABI, double precision in and out).
 * Return 0 on success, -1 on invalid arguments, -2 on allocation failure.
 * ------------------------------------------------------------------------- */
static double kappa_of(double delta, int beta_scale) {
    if (beta_scale == BETA_PHYS) return delta;
    if (beta_scale == BETA_LATTICE) return delta * delta;
    return 0.0;
}

static int lattice_init(lattice *L, int nx, int ny) {
    L->nx = nx;
    L->ny = ny;
    L->sites = (int64_t)nx * ny;
    L->theta = (double *)malloc(sizeof(double) * 3 * (size_t)L->sites);
    L->beta = (double *)malloc(sizeof(double) * 4 * (size_t)L->sites);
    L->tmp = (double *)malloc(sizeof(double) * (size_t)L->sites);
    L->v_form = V_PRINTED;
    return (L->theta && L->beta && L->tmp) ? 0 : -2;
}

static void lattice_free(lattice *L) {
    free(L->theta);
    free(L->beta);
    free(L->tmp);
}

static int check_args(int nx, int ny, double delta, int pot_mode, int beta_scale,
                      const double *n) {
    if (nx < 1 || ny < 1 || !(delta > 0.0) || !isfinite(delta)) return -1;
    if (pot_mode != POT_EQ23 && pot_mode != POT_EQ28) return -1;
    if (beta_scale < BETA_PHYS || beta_scale > BETA_OFF) return -1;
    const int64_t total = (int64_t)3 * nx * ny;
    for (int64_t i = 0; i < total; ++i)
        if (!(n[i] > 0.0) || !isfinite(n[i])) return -1;
    return 0;
}

/* Advance q (6*ny*nx doubles, in place) by nsteps full steps, with the
 * potentials in form v_form (V_PRINTED or V_SKEW). */
int qla_oracle_run_form(int nx, int ny, double delta, int pot_mode, int beta_scale, int v_form,
                        const double *n, double *q, int64_t nsteps, int nthreads) {
    if (!n || !q || nsteps < 0) return -1;
    if (v_form != V_PRINTED && v_form != V_SKEW) return -1;
    int rc = check_args(nx, ny, delta, pot_mode, beta_scale, n);
    if (rc) return rc;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
    lattice L;
    rc = lattice_init(&L, nx, ny);
    if (rc == 0) {
        L.v_form = v_form;
        compute_angles(&L, n, delta, kappa_of(delta, beta_scale));
        for (int64_t t = 0; t < nsteps; ++t) full_step(&L, q, pot_mode);
    }
    lattice_free(&L);
    return rc;
}

/* Advance q by nsteps full steps with the printed potentials. */
int qla_oracle_run(int nx, int ny, double delta, int pot_mode, int beta_scale,
                   const double *n, double *q, int64_t nsteps, int nthreads) {
    return qla_oracle_run_form(nx, ny, delta, pot_mode, beta_scale, V_PRINTED, n, q, nsteps,
                               nthreads);
}

/* One potential operator alone: V_X (axis 0) or V_Y (axis 1) with its
 * angles scaled by frac, in form v_form, applied to q in place. */
int qla_oracle_potential(int nx, int ny, double delta, int beta_scale, int v_form, int axis,
                         double frac, const double *n, double *q) {
    if (!n || !q || (axis != 0 && axis != 1)) return -1;
    if (v_form != V_PRINTED && v_form != V_SKEW) return -1;
    int rc = check_args(nx, ny, delta, POT_EQ28, beta_scale, n);
    if (rc) return rc;
    lattice L;
    rc = lattice_init(&L, nx, ny);
    if (rc == 0) {
        L.v_form = v_form;
        compute_angles(&L, n, delta, kappa_of(delta, beta_scale));
        if (axis == 0)
            potential_x(&L, q, frac);
        else
            potential_y(&L, q, frac);
    }
    lattice_free(&L);
    return rc;
}

/* The angles of Eq. (24) and (25) as the oracle uses them:
 * theta (3*ny*nx) and beta (4*ny*nx). */
int qla_oracle_angles(int nx, int ny, double delta, int beta_scale, const double *n,
                      double *theta, double *beta) {
    if (!n || !theta || !beta) return -1;
    int rc = check_args(nx, ny, delta, POT_EQ28, beta_scale, n);
    if (rc) return rc;
    lattice L;
    rc = lattice_init(&L, nx, ny);
    if (rc == 0) {
        compute_angles(&L, n, delta, kappa_of(delta, beta_scale));
        memcpy(theta, L.theta, sizeof(double) * 3 * (size_t)L.sites);
        memcpy(beta, L.beta, sizeof(double) * 4 * (size_t)L.sites);
    }
    lattice_free(&L);
    return rc;
}

/* Number of OpenMP threads a parallel region would use (1 without OpenMP). */
int qla_oracle_threads(int nthreads) {
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
    return omp_get_max_threads();
#else
    (void)nthreads;
    return 1;
#endif
}
