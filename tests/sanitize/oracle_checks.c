/* Runs the CPU oracle on the problems stored in a binary file, for a build of
 * oracle.c with AddressSanitizer and UndefinedBehaviorSanitizer (test
 * infrastructure).  Input: a sequence of problems, each
 *   int64 n, pL, ng, nt, ncells, var_conv, threads
 *   double Phi[n*n], XL[n*pL], G[n*ng], Y[n*nt], h2[nt], s2[nt]
 *   int64 snp[ncells], trait[ncells]
 * (column-major, leading dimension n).  Output: per problem the int32 return
 * code of oracle_gls, then (if 0) b[ncells*p], var[ncells*p*p], flag[ncells].
 * Also checks that bad arguments are refused.  Exit status 0 on success. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include "oracle.h"

static int read_all(FILE* f, void* dst, size_t bytes) { return fread(dst, 1, bytes, f) == bytes; }

static void* xmalloc(size_t bytes) {
  void* p = malloc(bytes ? bytes : 1);
  if (!p) {
    fprintf(stderr, "out of memory\n");
    exit(3);
  }
  return p;
}

static int bad_arguments(void) {
  double one = 1.0, h2 = 0.5, s2 = 1.0, b[2], var[4];
  int64_t zero = 0;
  int32_t flag;
  int fails = 0;
  /* n = 0, a negative cell count, null outputs, a leading dimension below n */
  fails += oracle_gls(0, 1, &one, 1, &one, 1, &one, 1, &one, 1, &h2, &s2, 1, &zero, &zero, 0, b, var, &flag, 1) != -1;
  fails += oracle_gls(1, 0, &one, 1, NULL, 1, &one, 1, &one, 1, &h2, &s2, -1, &zero, &zero, 0, b, var, &flag, 1) != -1;
  fails += oracle_gls(1, 0, &one, 1, NULL, 1, &one, 1, &one, 1, &h2, &s2, 1, &zero, &zero, 0, NULL, var, &flag, 1) != -1;
  fails += oracle_gls(2, 0, &one, 1, NULL, 2, &one, 2, &one, 2, &h2, &s2, 1, &zero, &zero, 0, b, var, &flag, 1) != -1;
  return fails;
}

int main(int argc, char** argv) {
  if (argc != 3) {
    fprintf(stderr, "usage: oracle_checks <input> <output>\n");
    return 2;
  }
  if (bad_arguments()) {
    fprintf(stderr, "oracle_gls accepted a bad argument\n");
    return 1;
  }
  FILE* in = fopen(argv[1], "rb");
  FILE* out = fopen(argv[2], "wb");
  if (!in || !out) return 2;
  int problems = 0;
  int64_t hdr[7];
  while (read_all(in, hdr, sizeof hdr)) {
    const int64_t n = hdr[0], pL = hdr[1], ng = hdr[2], nt = hdr[3], nc = hdr[4], p = pL + 1;
    double* Phi = xmalloc(sizeof(double) * n * n);
    double* XL = pL ? xmalloc(sizeof(double) * n * pL) : NULL;
    double* G = xmalloc(sizeof(double) * n * ng);
    double* Y = xmalloc(sizeof(double) * n * nt);
    double* h2 = xmalloc(sizeof(double) * nt);
    double* s2 = xmalloc(sizeof(double) * nt);
    int64_t* snp = xmalloc(sizeof(int64_t) * nc);
    int64_t* trait = xmalloc(sizeof(int64_t) * nc);
    if (!read_all(in, Phi, sizeof(double) * n * n) || (pL && !read_all(in, XL, sizeof(double) * n * pL)) ||
        !read_all(in, G, sizeof(double) * n * ng) || !read_all(in, Y, sizeof(double) * n * nt) ||
        !read_all(in, h2, sizeof(double) * nt) || !read_all(in, s2, sizeof(double) * nt) ||
        !read_all(in, snp, sizeof(int64_t) * nc) || !read_all(in, trait, sizeof(int64_t) * nc)) {
      fprintf(stderr, "truncated input\n");
      return 2;
    }
    double* b = xmalloc(sizeof(double) * nc * p);
    double* var = xmalloc(sizeof(double) * nc * p * p);
    int32_t* flag = xmalloc(sizeof(int32_t) * nc);
    const int32_t rc = oracle_gls(n, pL, Phi, n, XL, n, G, n, Y, n, h2, s2, nc, snp, trait, (int)hdr[5], b, var,
                                  flag, (int)hdr[6]);
    fwrite(&rc, sizeof rc, 1, out);
    if (rc == 0) {
      fwrite(b, sizeof(double), nc * p, out);
      fwrite(var, sizeof(double), nc * p * p, out);
      fwrite(flag, sizeof(int32_t), nc, out);
    }
    free(Phi), free(XL), free(G), free(Y), free(h2), free(s2), free(snp), free(trait), free(b), free(var),
        free(flag);
    ++problems;
  }
  fclose(in);
  fclose(out);
  printf("oracle_checks: %d problems\n", problems);
  return 0;
}
