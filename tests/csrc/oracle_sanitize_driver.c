/* Command-line driver for the sanitizer build of the FP64 reference simulator
 * (test use only): reads a case file (the layout of sanitize_driver.cpp),
 * applies its ops with oracle_apply, and writes the resulting state. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int oracle_apply(double *psi_d, int n, const void *ops_raw, uint64_t n_ops, const double *params);

int main(int argc, char **argv)
{
    if (argc != 3) return 2;
    FILE *f = fopen(argv[1], "rb");
    if (!f) return 2;
    int32_t hdr[6];
    uint64_t cnt[2];
    if (fread(hdr, sizeof hdr, 1, f) != 1 || fread(cnt, sizeof cnt, 1, f) != 1) return 2;
    const int n = hdr[0];
    if (n < 1 || n > 24) return 2;
    unsigned char *ops = malloc(cnt[0] * 40 + 1);
    double *params = malloc((cnt[1] + 1) * sizeof(double));
    double *psi = malloc((2ull << n) * sizeof(double));
    if (!ops || !params || !psi) return 2;
    if (fread(ops, 40, cnt[0], f) != cnt[0]) return 2;
    if (cnt[1] && fread(params, sizeof(double), cnt[1], f) != cnt[1]) return 2;
    if (fread(psi, sizeof(double), 2ull << n, f) != (2ull << n)) return 2;
    fclose(f);
    if (oracle_apply(psi, n, ops, cnt[0], params) != 0) return 3;
    FILE *g = fopen(argv[2], "wb");
    if (!g || fwrite(psi, sizeof(double), 2ull << n, g) != (2ull << n)) return 2;
    fclose(g);
    free(ops);
    free(params);
    free(psi);
    return 0;
}
