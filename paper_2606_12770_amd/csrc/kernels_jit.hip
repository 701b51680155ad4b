// Specialised tile-pass kernels at run time: generate (tile_codegen.cpp),
// compile for the current device's architecture (the HIP compiler in child
// processes, in parallel; hiprtc in this process where that is unavailable),
// load, launch.
//
// Identical pass sources share one kernel (a process-wide cache keyed by the
// source text, per device), so a QSVT ladder compiles each distinct U_L pass
// once however many calls it holds.  Translation units of several kernels
// are compiled in parallel on host threads.
#include <hip/hip_runtime.h>
#include <hip/hiprtc.h>
#include <fcntl.h>
#include <spawn.h>
#include <sys/wait.h>
#include <unistd.h>

#include <algorithm>
#include <cerrno>
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <iterator>
#include <map>
#include <sstream>
#include <tuple>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "sv_internal.h"

namespace svi {

std::string jit_preamble(int dtype);
std::string jit_pass_body(const sv_plan &p, uint32_t pi, uint32_t *param_base, bool persistent);
std::string jit_kernel(const std::string &name, const std::string &body, int threads, bool persistent);

namespace {

std::mutex g_mu;
// (device, dtype, kernel source) -> function
std::map<std::tuple<int, int, std::string>, hipFunction_t> g_fn;
std::vector<hipModule_t> g_modules;  // kept loaded until the process ends
uint64_t g_serial = 0;

std::string arch_of(int dev)
{
    hipDeviceProp_t prop{};
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return "gfx950";
    std::string a = prop.gcnArchName;
    const size_t c = a.find(':');
    return c == std::string::npos ? a : a.substr(0, c);
}

// Compile one translation unit; returns the code object or an error message.
bool compile_unit(const std::string &src, const std::string &arch, std::vector<char> &code, std::string &err)
{
    hiprtcProgram prog;
    if (hiprtcCreateProgram(&prog, src.c_str(), "tile_passes.hip", 0, nullptr, nullptr) != HIPRTC_SUCCESS) {
        err = "hiprtcCreateProgram failed";
        return false;
    }
    const std::string off = "--offload-arch=" + arch;
    // packed FP32 instructions stay off, as in the library's own build
    const char *opts[] = {off.c_str(), "-O3", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"};
    const hiprtcResult r = hiprtcCompileProgram(prog, 6, opts);
    if (r != HIPRTC_SUCCESS) {
        size_t n = 0;
        hiprtcGetProgramLogSize(prog, &n);
        std::string log(n, '\0');
        if (n) hiprtcGetProgramLog(prog, &log[0]);
        err = std::string("hiprtc: ") + hiprtcGetErrorString(r) + "\n" + log.substr(0, 4000);
        hiprtcDestroyProgram(&prog);
        return false;
    }
    size_t n = 0;
    hiprtcGetCodeSize(prog, &n);
    code.resize(n);
    hiprtcGetCode(prog, code.data());
    hiprtcDestroyProgram(&prog);
    return true;
}

// The HIP compiler of the ROCm installation, for compiling in child
// processes: hiprtc serialises compilations inside one process, so the
// translation units of a plan compile one after another there.
std::string clang_path()
{
    const char *root = std::getenv("ROCM_PATH");
    const std::string c = std::string(root && *root ? root : "/opt/rocm") + "/lib/llvm/bin/clang++";
    return access(c.c_str(), X_OK) == 0 ? c : std::string();
}

// Compile one translation unit with the HIP compiler in a child process
// (device code only, one code object); false with a message when the
// compiler cannot be run or fails (the caller then uses hiprtc).
bool compile_unit_process(const std::string &clang, const std::string &src, const std::string &arch,
                          std::vector<char> &code, std::string &err)
{
    const char *tmp = std::getenv("TMPDIR");
    std::string dir = std::string(tmp && *tmp ? tmp : "/tmp") + "/svjit.XXXXXX";
    std::vector<char> dbuf(dir.begin(), dir.end());
    dbuf.push_back('\0');
    if (!mkdtemp(dbuf.data())) {
        err = "mkdtemp failed";
        return false;
    }
    dir = dbuf.data();
    const std::string in = dir + "/unit.hip", out = dir + "/unit.co", log = dir + "/unit.log";
    {
        std::ofstream f(in);
        f << "#include <hip/hip_runtime.h>\n" << src;
        if (!f) {
            err = "cannot write " + in;
            std::remove(in.c_str());
            rmdir(dir.c_str());
            return false;
        }
    }
    const char *root = std::getenv("ROCM_PATH");
    const std::string inc = std::string("-I") + (root && *root ? root : "/opt/rocm") + "/include";
    const std::string off = "--offload-arch=" + arch;
    std::vector<std::string> args = {clang, "-x", "hip", off, "--offload-device-only", "--no-gpu-bundle-output",
                                     "-O3", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", inc,
                                     "-c", in, "-o", out};
    std::vector<char *> argv;
    for (auto &a : args) argv.push_back(&a[0]);
    argv.push_back(nullptr);
    posix_spawn_file_actions_t fa;
    posix_spawn_file_actions_init(&fa);
    posix_spawn_file_actions_addopen(&fa, 1, log.c_str(), O_WRONLY | O_CREAT | O_TRUNC, 0600);
    posix_spawn_file_actions_adddup2(&fa, 1, 2);
    pid_t pid = 0;
    int rc = posix_spawn(&pid, clang.c_str(), &fa, nullptr, argv.data(), environ);
    posix_spawn_file_actions_destroy(&fa);
    int status = 0;
    pid_t w = -1;
    if (rc == 0)
        do w = waitpid(pid, &status, 0);
        while (w == -1 && errno == EINTR);
    bool ok = rc == 0 && w == pid && WIFEXITED(status) && WEXITSTATUS(status) == 0;
    if (ok) {
        std::ifstream f(out, std::ios::binary);
        code.assign(std::istreambuf_iterator<char>(f), std::istreambuf_iterator<char>());
        ok = !code.empty();
    }
    if (!ok) {
        std::ifstream f(log);
        std::stringstream ss;
        ss << f.rdbuf();
        err = "HIP compiler: " + ss.str().substr(0, 4000);
    }
    std::remove(in.c_str());
    std::remove(out.c_str());
    std::remove(log.c_str());
    rmdir(dir.c_str());
    return ok;
}

}  // namespace

// Generates, compiles and loads the specialised kernels of every tile pass of
// `p` (on the current device); fills p->jit_fn / p->jit_prm.  SV_OK, or an
// error code with a message in err (the plan is then left without them).
int jit_prepare(sv_plan *p, std::string &err)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        err = "hipGetDevice failed";
        return SV_EDEVICE;
    }
    const size_t np = p->passes.size();
    p->jit_fn.assign(np, nullptr);
    p->jit_prm.assign(np, 0);
    if (!np) return SV_OK;
    const int threads = 1 << (p->b - p->rb);
    const bool persistent = p->tile_launch == SV_TILE_LAUNCH_PERSISTENT;
    // distinct bodies of this plan
    std::vector<std::string> bodies;
    std::unordered_map<std::string, uint32_t> index;
    std::vector<uint32_t> pass_body(np);
    for (size_t pi = 0; pi < np; ++pi) {
        uint32_t pb = 0;
        std::string body = jit_pass_body(*p, (uint32_t)pi, &pb, persistent);
        p->jit_prm[pi] = pb;
        auto it = index.find(body);
        if (it == index.end()) {
            it = index.emplace(body, (uint32_t)bodies.size()).first;
            bodies.push_back(std::move(body));
        }
        pass_body[pi] = it->second;
    }
    p->info.n_compiled_kernels = bodies.size();
    // the ones not yet compiled on this device
    std::vector<hipFunction_t> fn(bodies.size(), nullptr);
    std::vector<uint32_t> todo;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        for (uint32_t i = 0; i < bodies.size(); ++i) {
            auto it = g_fn.find(std::make_tuple(dev, p->dtype, bodies[i]));
            if (it != g_fn.end())
                fn[i] = it->second;
            else
                todo.push_back(i);
        }
    }
    if (!todo.empty()) {
        // translation units of up to 24 kernels, compiled on parallel threads
        const size_t per_unit = 24;
        const size_t units = (todo.size() + per_unit - 1) / per_unit;
        std::vector<std::string> names(bodies.size());
        uint64_t serial0;
        {
            std::lock_guard<std::mutex> lk(g_mu);
            serial0 = g_serial;
            g_serial += bodies.size();
        }
        for (uint32_t i : todo) names[i] = "tile_pass_" + std::to_string(serial0 + i);
        const std::string pre = jit_preamble(p->dtype);
        const std::string arch = arch_of(dev);
        // child processes pay off from two units up (each starts a compiler and
        // reads the HIP headers, about a second); a single unit goes to hiprtc
        const std::string clang = units > 1 ? clang_path() : std::string();
        std::vector<std::vector<char>> code(units);
        std::vector<std::string> errs(units);
        std::vector<char> ok(units, 0);
        const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
        const size_t nthreads = std::min<size_t>(units, std::min<unsigned>(hw, 16u));
        std::vector<std::thread> pool;
        std::mutex qmu;
        size_t next = 0;
        for (size_t t = 0; t < nthreads; ++t) {
            pool.emplace_back([&]() {
                for (;;) {
                    size_t u;
                    {
                        std::lock_guard<std::mutex> lk(qmu);
                        if (next >= units) return;
                        u = next++;
                    }
                    std::string src = pre;
                    for (size_t j = u * per_unit; j < std::min(todo.size(), (u + 1) * per_unit); ++j)
                        src += jit_kernel(names[todo[j]], bodies[todo[j]], threads,
                                          bodies[todo[j]].compare(0, 13, "// persistent") == 0);
                    // a child process per unit (parallel), else hiprtc in this process
                    std::string perr;
                    ok[u] = (!clang.empty() && compile_unit_process(clang, src, arch, code[u], perr)) ||
                                    compile_unit(src, arch, code[u], errs[u])
                                ? 1
                                : 0;
                }
            });
        }
        for (auto &th : pool) th.join();
        for (size_t u = 0; u < units; ++u)
            if (!ok[u]) {
                err = "compiling specialised tile passes failed: " + errs[u];
                return SV_EUNSUPPORTED;
            }
        std::lock_guard<std::mutex> lk(g_mu);
        for (size_t u = 0; u < units; ++u) {
            hipModule_t mod = nullptr;
            hipError_t e = hipModuleLoadData(&mod, code[u].data());
            if (e != hipSuccess) {
                err = std::string("hipModuleLoadData: ") + hipGetErrorString(e);
                return SV_EDEVICE;
            }
            g_modules.push_back(mod);
            for (size_t j = u * per_unit; j < std::min(todo.size(), (u + 1) * per_unit); ++j) {
                const uint32_t i = todo[j];
                hipFunction_t f = nullptr;
                e = hipModuleGetFunction(&f, mod, names[i].c_str());
                if (e != hipSuccess) {
                    err = std::string("hipModuleGetFunction: ") + hipGetErrorString(e);
                    return SV_EDEVICE;
                }
                fn[i] = f;
                g_fn.emplace(std::make_tuple(dev, p->dtype, bodies[i]), f);
            }
        }
    }
    for (size_t pi = 0; pi < np; ++pi) p->jit_fn[pi] = (void *)fn[pass_body[pi]];
    return SV_OK;
}

// Resident workgroups of a persistent compiled pass kernel on the whole device.
static uint64_t resident_grid(hipFunction_t f, uint32_t block)
{
    int dev = 0, cus = 256, per_cu = 1;
    if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (hipModuleOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, f, (int)block, 0) != hipSuccess || per_cu < 1)
        per_cu = 1;
    (void)hipGetLastError();
    return (uint64_t)cus * (uint64_t)per_cu;
}

// Launch the specialised kernel of tile pass `pi` on `psi`: one workgroup per
// tile, or (persistent plans) the device's resident workgroups walking them.
int launch_jit_pass(const sv_plan *p, uint32_t pi, void *psi, hipStream_t st)
{
    const TilePass &P = p->passes[pi];
    const uint64_t tiles = 1ull << P.ntile;
    const size_t es = p->dtype == SV_C64 ? sizeof(float) : sizeof(double);
    void *prm = (char *)p->d_tparams + (size_t)p->jit_prm[pi] * es;
    hipFunction_t f = (hipFunction_t)p->jit_fn[pi];
    const uint32_t block = 1u << P.nthr;
    hipError_t e;
    if (p->tile_launch == SV_TILE_LAUNCH_PERSISTENT) {
        uint64_t n_tiles = tiles;
        const uint64_t g = std::min<uint64_t>(tiles, resident_grid(f, block));
        void *args[] = {&psi, &prm, &n_tiles};
        e = hipModuleLaunchKernel(f, (uint32_t)g, 1, 1, block, 1, 1, 0, st, args, nullptr);
    } else {
        const uint32_t gx = tiles > 65536 ? 65536u : (uint32_t)tiles;
        const uint32_t gy = (uint32_t)(tiles / gx);
        void *args[] = {&psi, &prm};
        e = hipModuleLaunchKernel(f, gx, gy, 1, block, 1, 1, 0, st, args, nullptr);
    }
    return e == hipSuccess ? SV_OK : SV_EDEVICE;
}

}  // namespace svi
