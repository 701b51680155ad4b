// Host-side check of the specialised tile-pass sources (test use only): plans
// a circuit, generates the kernel source of every distinct pass, and compiles
// it for gfx950 with hiprtc (no device needed), returning the number of
// distinct kernels or a negative code; the source and the compiler log can be
// written to files for inspection.
#include <hip/hiprtc.h>

#include <cstdio>
#include <fstream>
#include <set>
#include <string>

#include "plan_types.h"

namespace svi {
std::string jit_preamble(int dtype);
std::string jit_pass_body(const sv_plan &p, uint32_t pi, uint32_t *param_base, bool persistent);
std::string jit_kernel(const std::string &name, const std::string &body, int threads, bool persistent);
}  // namespace svi

using namespace svi;

// sv_apply_opts.split_real of the plans jit_check builds (SV_SPLIT_REAL_AUTO by default).
static int g_split_real = SV_SPLIT_REAL_AUTO;
extern "C" void jit_check_set_split_real(int v) { g_split_real = v; }

extern "C" int jit_check(int n, int dtype, const sv_op *ops, size_t n_ops, const double *params, int tile_qubits,
                         int reg_qubits, int persistent, const char *src_out, const char *code_out)
{
    sv_plan p;
    p.n = n;
    p.dtype = dtype;
    sv_apply_opts o{};
    o.mode = SV_MODE_FUSED;
    o.tile_qubits = tile_qubits;
    o.reg_qubits = reg_qubits;
    o.split_real = g_split_real;
    std::string err;
    if (build_plan(&p, ops, n_ops, params, o, err) != SV_OK) return -1;
    std::set<std::string> bodies;
    std::string src = jit_preamble(dtype);
    int k = 0;
    for (uint32_t pi = 0; pi < p.passes.size(); ++pi) {
        uint32_t pb = 0;
        const std::string body = jit_pass_body(p, pi, &pb, persistent != 0);
        if (!bodies.insert(body).second) continue;
        src += jit_kernel("tile_pass_" + std::to_string(k++), body, 1 << (p.b - p.rb), persistent != 0);
    }
    if (src_out) std::ofstream(src_out) << src;
    hiprtcProgram prog;
    if (hiprtcCreateProgram(&prog, src.c_str(), "tile_passes.hip", 0, nullptr, nullptr) != HIPRTC_SUCCESS) return -2;
    const char *opts[] = {"--offload-arch=gfx950", "-O3", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"};
    const hiprtcResult r = hiprtcCompileProgram(prog, 6, opts);
    if (r != HIPRTC_SUCCESS) {
        size_t m = 0;
        hiprtcGetProgramLogSize(prog, &m);
        std::string log(m, '\0');
        if (m) hiprtcGetProgramLog(prog, &log[0]);
        std::fprintf(stderr, "%s\n", log.substr(0, 8000).c_str());
        hiprtcDestroyProgram(&prog);
        return -3;
    }
    if (code_out) {
        size_t m = 0;
        hiprtcGetCodeSize(prog, &m);
        std::string code(m, '\0');
        hiprtcGetCode(prog, &code[0]);
        std::ofstream(code_out, std::ios::binary) << code;
    }
    hiprtcDestroyProgram(&prog);
    return k;
}
