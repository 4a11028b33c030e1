/* The oracle (oracle/swe_oracle.c) under AddressSanitizer and
 * UndefinedBehaviorSanitizer: one input file (the mesh format of
 * mesh_driver.cpp followed by the fields and boundary conditions) is run
 * through set-up, steps to an end time, frozen-schedule steps, monitors,
 * geometry and edge queries, and a state reset. Exit status 0 when every
 * call succeeds; a sanitizer report aborts the program.
 *
 * After the mesh part: double z[n], man[n], h[n], hu[n], hv[n]; int32 n_bc;
 * n_bc x (int32 tag, int32 kind, double value). */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

typedef struct ora ora;
ora *ora_create(int64_t nn, const double *xy, int64_t nc, const int32_t *tri,
                int64_t nb, const int32_t *bnd, const int32_t *bnd_tag,
                char *err, int errlen);
void ora_destroy(ora *o);
int ora_set_bc(ora *o, int tag, int kind, double value);
int ora_set_params(ora *o, double g, double cfl, double h_dry, double dt_max);
int ora_set_fields(ora *o, const double *z, const double *man);
int ora_set_state(ora *o, const double *h, const double *hu,
                  const double *hv);
void ora_get_state(const ora *o, double *h, double *hu, double *hv);
int ora_run(ora *o, int64_t max_steps, double t_end, int nthreads,
            int64_t *done, double *t);
int ora_run_dt(ora *o, int64_t n, const double *dt, int nthreads);
void ora_discharge(const ora *o, int tag, double *rate, double *volume);
void ora_envelope(const ora *o, double *hmax, double *twet);
void ora_set_time(ora *o, double t, int64_t step);
double ora_mass(const ora *o);
void ora_geometry(const ora *o, double *area, double *inr, int32_t *tri_ccw);
const char *ora_error(const ora *o);

static void *take(FILE *f, size_t n, size_t size)
{
    void *p = malloc(n * size + 1);
    if (!p || (n && fread(p, size, n, f) != n)) {
        fprintf(stderr, "short input\n");
        exit(2);
    }
    return p;
}

static int64_t take_i64(FILE *f)
{
    int64_t x;
    if (fread(&x, 8, 1, f) != 1) exit(2);
    return x;
}

int main(int argc, char **argv)
{
    if (argc != 2) return 2;
    FILE *f = fopen(argv[1], "rb");
    if (!f) return 2;
    const int64_t nn = take_i64(f);
    double *xy = take(f, 2 * nn, 8);
    const int64_t nc = take_i64(f);
    int32_t *tri = take(f, 3 * nc, 4);
    const int64_t nb = take_i64(f);
    int32_t *bnd = take(f, 2 * nb, 4);
    int32_t *btag = take(f, nb, 4);
    const int64_t ne = take_i64(f);
    free(take(f, 5 * ne, 4));
    free(take(f, nc, 1));
    double *z = take(f, nc, 8), *man = take(f, nc, 8);
    double *h = take(f, nc, 8), *hu = take(f, nc, 8), *hv = take(f, nc, 8);
    int32_t nbc;
    if (fread(&nbc, 4, 1, f) != 1) return 2;
    char err[512];
    ora *o = ora_create(nn, xy, nc, tri, nb, bnd, btag, err, 512);
    if (!o) {
        fprintf(stderr, "ora_create: %s\n", err);
        return 1;
    }
    for (int32_t k = 0; k < nbc; ++k) {
        int32_t tag, kind;
        double value;
        if (fread(&tag, 4, 1, f) != 1 || fread(&kind, 4, 1, f) != 1 ||
            fread(&value, 8, 1, f) != 1)
            return 2;
        if (ora_set_bc(o, tag, kind, value)) return 1;
    }
    fclose(f);
    if (ora_set_params(o, 9.81, 0.9, 1e-6, INFINITY) ||
        ora_set_fields(o, z, man) || ora_set_state(o, h, hu, hv))
        return 1;
    int64_t done = 0;
    double t = 0.0;
    if (ora_run(o, 25, INFINITY, 2, &done, &t) || done != 25) {
        fprintf(stderr, "run: %s\n", ora_error(o));
        return 1;
    }
    if (ora_run(o, 1000000, t + 0.05, 1, &done, &t)) return 1;
    double dts[7] = {1e-3, 2e-3, 0.0, 1e-3, 5e-4, 1e-3, 2e-3};
    if (ora_run_dt(o, 7, dts, 2)) return 1;
    double rate, vol;
    for (int tag = 0; tag < 4; ++tag) ora_discharge(o, tag, &rate, &vol);
    double *a = malloc(nc * 8), *b = malloc(nc * 8);
    int32_t *ccw = malloc(nc * 12);
    ora_envelope(o, a, b);
    ora_geometry(o, a, b, ccw);
    ora_get_state(o, h, hu, hv);
    ora_set_time(o, 0.0, 0);
    if (ora_set_state(o, h, hu, hv)) return 1;
    if (ora_run(o, 3, INFINITY, 1, &done, &t)) return 1;
    printf("steps %lld t %.6g mass %.12g\n", (long long)done, t, ora_mass(o));
    ora_destroy(o);
    free(a);
    free(b);
    free(ccw);
    free(xy);
    free(tri);
    free(bnd);
    free(btag);
    free(z);
    free(man);
    free(h);
    free(hu);
    free(hv);
    return 0;
}
