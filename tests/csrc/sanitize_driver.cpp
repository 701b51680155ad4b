// Command-line driver for the sanitizer build of the host code (test use
// only).  It reads one circuit case from a binary file, runs it through the
// planner and the CPU emulation of the launch steps (tests/csrc/plan_emu.cpp),
// and writes the resulting state.  Built with AddressSanitizer and
// UndefinedBehaviorSanitizer, so an out-of-bounds access or undefined
// operation anywhere on that path aborts the process.
//
// Case file layout (little-endian): int32 n, dtype, mode, b, rb, dense_min_ops;
// uint64 n_ops, n_params; n_ops 40-byte op records; n_params doubles; 2^n
// complex128 amplitudes (interleaved re, im).  SAN_ROUND_PARAMS=1 in the
// environment rounds complex64 parameters as the library uploads them, and
// SAN_SPLIT_REAL sets sv_apply_opts.split_real.
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "sv.h"

extern "C" int emu_run(int n, int dtype, const sv_op *ops, size_t n_ops, const double *params, int mode, int b,
                       int rb, double *psi, uint64_t *stats, int dense_min_ops);
extern "C" void emu_set_param_rounding(int on);
extern "C" void emu_set_split_real(int v);

int main(int argc, char **argv)
{
    if (argc != 3) {
        std::fprintf(stderr, "usage: %s case.bin out.bin\n", argv[0]);
        return 2;
    }
    FILE *f = std::fopen(argv[1], "rb");
    if (!f) return 2;
    int32_t hdr[6];
    uint64_t cnt[2];
    if (std::fread(hdr, sizeof hdr, 1, f) != 1 || std::fread(cnt, sizeof cnt, 1, f) != 1) return 2;
    const int n = hdr[0];
    if (n < 1 || n > 24) return 2;
    std::vector<sv_op> ops(cnt[0]);
    std::vector<double> params(cnt[1] ? cnt[1] : 1);
    std::vector<double> psi(2ull << n);
    if (std::fread(ops.data(), sizeof(sv_op), ops.size(), f) != ops.size()) return 2;
    if (cnt[1] && std::fread(params.data(), sizeof(double), cnt[1], f) != cnt[1]) return 2;
    if (std::fread(psi.data(), sizeof(double), psi.size(), f) != psi.size()) return 2;
    std::fclose(f);
    if (const char *v = std::getenv("SAN_ROUND_PARAMS")) emu_set_param_rounding(std::atoi(v));
    if (const char *v = std::getenv("SAN_SPLIT_REAL")) emu_set_split_real(std::atoi(v));
    uint64_t stats[7] = {0, 0, 0, 0, 0, 0, 0};
    const int rc = emu_run(n, hdr[1], ops.data(), ops.size(), params.data(), hdr[2], hdr[3], hdr[4], psi.data(),
                           stats, hdr[5]);
    if (rc != 0) {
        std::fprintf(stderr, "emulation check failed with code %d\n", rc);
        return 3;
    }
    FILE *g = std::fopen(argv[2], "wb");
    if (!g || std::fwrite(psi.data(), sizeof(double), psi.size(), g) != psi.size()) return 2;
    std::fclose(g);
    return 0;
}
