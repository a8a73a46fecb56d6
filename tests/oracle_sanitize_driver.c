/* Runs the oracle's entry points on small problems of every model and option
 * under AddressSanitizer and UndefinedBehaviorSanitizer (test infrastructure:
 * built and run by tests/test_oracle_sanitize.py).  Exit status 0 when every
 * result is finite; the sanitizers abort on an invalid access, overflow or
 * leak. */
#include "../oracle/oracle.c"

#include <stdio.h>

static double frand(uint64_t *s)
{
    *s = *s * 6364136223846793005ull + 1442695040888963407ull;
    return (double)(*s >> 11) * (1.0 / 9007199254740992.0);
}

/* a smooth-ish random admissible primitive field */
static void fill_w(const orc_cfg *c, double *W, uint64_t seed)
{
    int nc = orc_ncomp(c);
    long n = (long)c->nx * c->ny * c->nz;
    uint64_t s = seed;
    for (long q = 0; q < n; q++) {
        double r = frand(&s);
        if (c->model == M_DIM) {
            double a = 0.02 + 0.96 * frand(&s);
            W[0 * n + q] = a * (0.5 + r);
            W[1 * n + q] = (1.0 - a) * (1.0 + r);
            W[2 * n + q] = 0.3 * frand(&s) - 0.15;
            W[3 * n + q] = 0.3 * frand(&s) - 0.15;
            W[4 * n + q] = 0.3 * frand(&s) - 0.15;
            W[5 * n + q] = 1.0 + r;
            W[6 * n + q] = a;
        } else {
            W[0 * n + q] = 0.5 + r;
            W[1 * n + q] = 0.3 * frand(&s) - 0.15;
            W[2 * n + q] = 0.3 * frand(&s) - 0.15;
            W[3 * n + q] = 0.3 * frand(&s) - 0.15;
            W[4 * n + q] = 1.0 + frand(&s);
        }
    }
    (void)nc;
}

static int finite_all(const double *a, long n)
{
    for (long q = 0; q < n; q++)
        if (!isfinite(a[q])) return 0;
    return 1;
}

static int run(orc_cfg c, uint64_t seed)
{
    int nc = orc_ncomp(&c);
    long n = (long)c.nx * c.ny * c.nz, N = nc * n;
    double *W = malloc(sizeof(double) * N), *U = malloc(sizeof(double) * N), *R = malloc(sizeof(double) * N);
    double *U1 = malloc(sizeof(double) * N);
    long nf = orc_face_count(&c, 0) + orc_face_count(&c, 1) + orc_face_count(&c, 2);
    uint8_t *fl = malloc(nf);
    fill_w(&c, W, seed);
    orc_prim_to_cons(&c, W, U);
    orc_cons_to_prim(&c, U, W);
    double dt = orc_dt(&c, U, 0.3);
    orc_rhs(&c, U, R, dt, fl);
    int ok = finite_all(R, N);
    int64_t cells[3] = {0, n / 2, n - 1};
    double Rc[3 * 7];
    uint8_t fc[3 * 6];
    orc_rhs_cells(&c, U, cells, 3, Rc, dt, fc);
    ok = ok && finite_all(Rc, 3 * nc);
    orc_rk3_stage(&c, 1, U, U, U1, dt);
    ok = ok && finite_all(U1, N);
    orc_advance(&c, U, 2, 0.0, 0.3);
    ok = ok && finite_all(U, N);
    free(W);
    free(U);
    free(R);
    free(U1);
    free(fl);
    return ok;
}

int main(void)
{
    const int grids[4][3] = {{5, 4, 3}, {1, 6, 1}, {7, 1, 1}, {3, 3, 3}};
    int bad = 0, runs = 0;
    for (int model = 0; model < 3; model++)
        for (int g = 0; g < 4; g++)
            for (int var = 0; var < 6; var++) {
                orc_cfg c;
                memset(&c, 0, sizeof c);
                c.nx = grids[g][0];
                c.ny = grids[g][1];
                c.nz = grids[g][2];
                c.model = model;
                for (int k = 0; k < 6; k++) c.bc[k] = (k / 2 + g) % 3;
                for (int a = 0; a < 3; a++) {
                    const int na = a == 0 ? c.nx : (a == 1 ? c.ny : c.nz);
                    if (na < 3 && c.bc[2 * a] == BC_SYMMETRY) c.bc[2 * a] = c.bc[2 * a + 1] = BC_ZEROGRAD;
                    if ((c.bc[2 * a] == BC_PERIODIC) != (c.bc[2 * a + 1] == BC_PERIODIC))
                        c.bc[2 * a] = c.bc[2 * a + 1] = BC_PERIODIC;
                }
                c.dx = 0.1;
                c.dy = 0.2;
                c.dz = 0.15;
                c.gamma1 = 1.4;
                c.gamma2 = 1.66;
                c.pinf1 = model == M_DIM ? 0.1 : 0.0;
                c.mu = model == M_NS ? 0.01 : 0.0;
                c.prandtl = 0.72;
                c.eps_rho = 1e-12;
                c.eps_rhoc2 = 1e-10;
                c.eps_alpha = 1e-12;
                c.weno_eps = 1e-40;
                c.T_ref = 1.0;
                c.gas_R = 1.0;
                c.positivity = (var & 1) || model == M_DIM;
                c.recon = var >= 2 && var < 4;
                c.scheme = var >= 3;
                c.thinc = model == M_DIM && var >= 4;
                c.visc_order = model == M_NS && var == 5 ? 6 : 4;
                c.visc_law = model == M_NS ? var % 3 : 0;
                runs++;
                if (!run(c, 17 + 31 * runs)) {
                    printf("non-finite: model %d grid %d variant %d\n", model, g, var);
                    bad++;
                }
            }
    printf("%d runs, %d non-finite\n", runs, bad);
    return bad != 0;
}
