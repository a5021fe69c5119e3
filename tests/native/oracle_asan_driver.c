/* Host sanitizer run of the oracle: built with -fsanitize=address,undefined together with
 * oracle/pr_oracle.c, it evaluates every state mode and the diffusion coefficients on a
 * mechanism read from a text file (species constants as plain numbers, then the k_ij
 * matrix) and seeded cells, including non-physical ones.  Exit status 0 and no sanitizer
 * report is the pass condition; the values themselves are checked by the Python tests. */
#include <stdio.h>
#include <stdlib.h>

#include "../../oracle/pr_oracle.c"

static double urand(unsigned long long *s)
{
    /* splitmix64 -> [0, 1) */
    unsigned long long z = (*s += 0x9E3779B97F4A7C15ULL);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    z ^= z >> 31;
    return (double)(z >> 11) * (1.0 / 9007199254740992.0);
}

int main(int argc, char **argv)
{
    if (argc < 2) return 2;
    FILE *f = fopen(argv[1], "r");
    if (!f) return 2;
    orc_mech m;
    memset(&m, 0, sizeof(m));
    if (fscanf(f, "%d", &m.ns) != 1 || m.ns < 1 || m.ns > ORC_MAXNS) return 2;
    for (int i = 0; i < m.ns; i++) {
        orc_species *s = &m.sp[i];
        double *v[8] = {&s->W, &s->Tc, &s->Pc, &s->Vc, &s->omega, &s->dipole, &s->kappa, &s->Tmid};
        for (int k = 0; k < 8; k++)
            if (fscanf(f, "%lf", v[k]) != 1) return 2;
        for (int k = 0; k < 7; k++)
            if (fscanf(f, "%lf", &s->lo[k]) != 1) return 2;
        for (int k = 0; k < 7; k++)
            if (fscanf(f, "%lf", &s->hi[k]) != 1) return 2;
    }
    for (int k = 0; k < m.ns * m.ns; k++)
        if (fscanf(f, "%lf", &m.kij[k]) != 1) return 2;
    fclose(f);

    const int64_t n = 257;
    double *P = malloc(n * sizeof(double)), *T = malloc(n * sizeof(double));
    double *Y = malloc((size_t)m.ns * n * sizeof(double)), *D = malloc((size_t)m.ns * n * sizeof(double));
    double *in0 = malloc(n * sizeof(double)), *in1 = malloc(n * sizeof(double));
    orc_cell *c = malloc(n * sizeof(orc_cell)), *c2 = malloc(n * sizeof(orc_cell));
    unsigned long long seed = 12345;
    for (int64_t k = 0; k < n; k++) {
        P[k] = 1e5 + 2e7 * urand(&seed);
        T[k] = 80.0 + 3000.0 * urand(&seed);
        double s = 0.0;
        for (int i = 0; i < m.ns; i++) s += (Y[i * n + k] = urand(&seed));
        for (int i = 0; i < m.ns; i++) Y[i * n + k] /= s;
    }
    P[0] = -1.0;          /* non-physical cells take the error paths */
    T[1] = 0.0;
    Y[2] = -0.5;
    int rc = orc_eval(&m, 0, n, P, T, Y, 1, c, 1);
    for (int64_t k = 0; k < n; k++) {
        in0[k] = c[k].rho;
        in1[k] = c[k].e;
    }
    rc |= orc_eval(&m, 1, n, in0, in1, Y, 1, c2, 1);
    for (int64_t k = 0; k < n; k++) {
        in0[k] = c[k].v;
        in1[k] = T[k];
    }
    rc |= orc_eval(&m, 2, n, in0, in1, Y, 1, c2, 1);
    for (int64_t k = 0; k < n; k++) {
        in0[k] = c[k].h;
        in1[k] = P[k];
    }
    rc |= orc_eval(&m, 3, n, in0, in1, Y, 1, c2, 1);
    rc |= orc_eval_mixdiff(&m, n, P, T, Y, D, 1);
    double chk = 0.0;
    for (int64_t k = 3; k < n; k++) chk += c2[k].T + D[k];
    printf("rc %d checksum %.6e\n", rc, chk);
    free(P), free(T), free(Y), free(D), free(in0), free(in1), free(c), free(c2);
    return rc != 0;
}
