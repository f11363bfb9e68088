/*
 * oracle_driver.c -- runs the fp64 oracle (oracle/gp_oracle.c, linked in
 * directly) on a population read from a file, so the test suite can build
 * it with the host's AddressSanitizer and UndefinedBehaviorSanitizer and
 * compare its results with the normal build bit for bit.
 *
 * TEST INFRASTRUCTURE.  Input (binary, little endian): int64 P, n_nodes,
 * n_consts, n_vars, n_cases; uint32 nodes[n_nodes]; int64 offsets[P + 1];
 * float consts[n_consts]; float X[n_vars][n_cases]; float y[n_cases].
 * Output: status[P] (int32), max_depth[P] (int32), then float64 per program:
 * F (M64, tax 1e-3), F (M32E_RAND + 1), mse (M64), correlation score and r,
 * reward (power 8), and int64 c1, c2 per program.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int oracle_fitness(const uint32_t*, const int64_t*, int64_t, const float*, int64_t,
                   const float*, int32_t, int64_t, const float*, int64_t, double, uint32_t,
                   int, int, double*, double*, int32_t*);
int oracle_correlation(const uint32_t*, const int64_t*, int64_t, const float*, int64_t,
                       const float*, int32_t, int64_t, const float*, int64_t, double, uint32_t,
                       int, int, double*, double*, int64_t*, int32_t*);
int oracle_reward(const uint32_t*, const int64_t*, int64_t, const float*, int64_t,
                  const float*, int32_t, int64_t, const float*, int64_t, double, int, uint32_t,
                  int, int, double*, int32_t*);
void oracle_validate(const uint32_t*, const int64_t*, int64_t, int64_t, int32_t, uint32_t,
                     int32_t*, int32_t*);

static void* rd(FILE* f, size_t elem, int64_t n)
{
    void* p = malloc(elem * (size_t)(n > 0 ? n : 1));
    if (!p || (n > 0 && fread(p, elem, (size_t)n, f) != (size_t)n)) exit(2);
    return p;
}

int main(int argc, char** argv)
{
    if (argc != 4) return 2;
    const uint32_t mask = (uint32_t)strtoul(argv[3], NULL, 0);
    FILE* in = fopen(argv[1], "rb");
    if (!in) return 2;
    int64_t* hd = rd(in, 8, 5);
    const int64_t P = hd[0], NN = hd[1], NC = hd[2], NV = hd[3], N = hd[4];
    uint32_t* nodes = rd(in, 4, NN);
    int64_t* off = rd(in, 8, P + 1);
    float* consts = rd(in, 4, NC);
    float* X = rd(in, 4, NV * N);
    float* y = rd(in, 4, N);
    fclose(in);
    int32_t* st = malloc(4 * (size_t)P);
    int32_t* md = malloc(4 * (size_t)P);
    int32_t* st2 = malloc(4 * (size_t)P);
    double* out = malloc(8 * 6 * (size_t)P);
    int64_t* c12 = malloc(16 * (size_t)P);
    if (!st || !md || !st2 || !out || !c12) return 2;
    oracle_validate(nodes, off, P, NC, (int32_t)NV, mask, st, md);
    oracle_fitness(nodes, off, P, consts, NC, X, (int32_t)NV, N, y, N, 1e-3, mask, 0, 4,
                   out, out + 2 * P, st2);
    oracle_fitness(nodes, off, P, consts, NC, X, (int32_t)NV, N, y, N, 1e-3, mask, 17, 4,
                   out + P, out + 5 * P, st2);     /* the mse slot is scratch here */
    oracle_correlation(nodes, off, P, consts, NC, X, (int32_t)NV, N, y, N, 1e4, mask, 0, 4,
                       out + 3 * P, out + 4 * P, c12, st2);
    oracle_reward(nodes, off, P, consts, NC, X, (int32_t)NV, N, y, N, 1e4, 8, mask, 0, 4,
                  out + 5 * P, st2);
    FILE* o = fopen(argv[2], "wb");
    if (!o) return 2;
    fwrite(st, 4, (size_t)P, o);
    fwrite(md, 4, (size_t)P, o);
    fwrite(out, 8, 6 * (size_t)P, o);
    fwrite(c12, 8, 2 * (size_t)P, o);
    fclose(o);
    free(hd); free(nodes); free(off); free(consts); free(X); free(y);
    free(st); free(md); free(st2); free(out); free(c12);
    return 0;
}
