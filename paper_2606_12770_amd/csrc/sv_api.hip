// C ABI of libsv: argument validation, state and plan lifetime, execution.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <set>
#include <string>
#include <vector>

#include "sv_internal.h"

namespace svi {
int tile_kernel_setup();
int jit_prepare(sv_plan *p, std::string &err);
int launch_jit_pass(const sv_plan *p, uint32_t pi, void *psi, hipStream_t st);

struct Arena {
    void *d_mem = nullptr;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int refs = 0;
};
}  // namespace svi

struct sv_batch {
    // concurrent form (compiled plans): instance i runs its own plan's launches
    // on side stream stream_of[i]; the side streams fork from and join back to
    // `stream`, so one execution is one graph with a branch per stream
    bool concurrent = false;
    std::vector<sv_plan *> plans;
    std::vector<hipStream_t> side;
    std::vector<uint32_t> stream_of;
    std::vector<hipEvent_t> events;     // fork event, then one join event per side stream
    uint64_t launches = 0;
    // level-synchronous form
    svi::BatchTables tables{};
    std::vector<void *> d_tables;       // concatenated plan tables owned by the batch
    hipStream_t stream = nullptr;
    std::vector<uint32_t> n_items;      // per level
    std::vector<uint64_t> total;        // per level
    std::vector<uint8_t> gate_runs;     // per level: some pass of the level holds gate runs
    std::vector<uint8_t> stream_state;  // per level: nontemporal state accesses (the level's total state bytes)
    std::vector<svi::BatchItem *> d_items;
    std::vector<sv_state *> states;
    bool use_graph = false;
    bool graph_ready = false;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    uint64_t gates = 0;
    size_t groups = 0;
};

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string &msg)
{
    g_last_error = msg;
    return code;
}

int hip_fail(hipError_t e, const char *what)
{
    return fail(SV_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIP_TRY(call)                                  \
    do {                                               \
        hipError_t e_ = (call);                        \
        if (e_ != hipSuccess) return hip_fail(e_, #call); \
    } while (0)

// Staging buffer of sv_amplitudes_noalloc: a fixed device array, so that call
// allocates nothing.  Each device holds its own copy until the process ends;
// host code must use the per-device address from hipGetSymbolAddress, never
// the array's name (on the host that name is only a stand-in).
constexpr uint64_t kScratchAmps = 1ull << 18;  // complex128 amplitudes: 4 MiB
__device__ __align__(256) double2 scratch[kScratchAmps];

std::mutex g_setup_mu;
std::map<int, void *> g_scratch;  // device -> address of `scratch` on it

int ensure_device_setup(int dev)
{
    static std::set<int> ready;
    std::lock_guard<std::mutex> lk(g_setup_mu);
    if (ready.count(dev)) return SV_OK;
    int rc = svi::tile_kernel_setup();
    if (rc != SV_OK) return fail(rc, "could not raise the LDS limit of the tile kernels");
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    g_scratch[dev] = ptr;
    ready.insert(dev);
    return SV_OK;
}

void *scratch_on(int dev)
{
    std::lock_guard<std::mutex> lk(g_setup_mu);
    auto it = g_scratch.find(dev);
    return it == g_scratch.end() ? nullptr : it->second;
}

int validate_ops(int n, const sv_op *ops, size_t n_ops, const double *params, size_t n_params)
{
    if (n_ops && !ops) return fail(SV_EINVAL, "ops is NULL");
    const uint64_t all = (n >= 64) ? ~0ull : ((1ull << n) - 1ull);
    char buf[256];
    for (size_t k = 0; k < n_ops; ++k) {
        const sv_op &o = ops[k];
        auto bad = [&](const char *why) {
            snprintf(buf, sizeof buf, "op %zu (kind %u): %s", k, o.kind, why);
            return fail(SV_EINVAL, buf);
        };
        if (o.kind > SV_OP_PROJPHASE) return bad("unknown kind");
        if (o.flags != 0) return bad("flags must be 0");
        if (o.ctrl_val & ~o.ctrl_mask) return bad("ctrl_val has bits outside ctrl_mask");
        if (o.ctrl_mask & ~all) return bad("control qubit >= n");
        size_t np = 0;
        switch (o.kind) {
        case SV_OP_U: np = 8; break;
        case SV_OP_PHASE:
        case SV_OP_RY:
        case SV_OP_PROJPHASE: np = 1; break;
        default: break;
        }
        // (unsigned comparisons written so that no sum can wrap around)
        if (np && (!params || n_params < np || o.param > (uint64_t)(n_params - np)))
            return bad("parameter offset out of range");
        switch (o.kind) {
        case SV_OP_U:
        case SV_OP_X:
        case SV_OP_PHASE:
        case SV_OP_RY:
        case SV_OP_PROJPHASE:
            if (o.target >= (uint32_t)n) return bad("target qubit >= n");
            if ((o.ctrl_mask >> o.target) & 1ull) return bad("target is also a control");
            if (o.width != 0) return bad("width must be 0");
            break;
        case SV_OP_INC:
        case SV_OP_DEC: {
            if (o.width < 1 || o.width > 24) return bad("register width must be in [1, 24]");
            if (o.target >= (uint32_t)n || o.width > (uint32_t)n - o.target)
                return bad("register exceeds the qubit count");
            const uint64_t reg = ((1ull << o.width) - 1ull) << o.target;
            if (reg & o.ctrl_mask) return bad("register overlaps the controls");
            break;
        }
        case SV_OP_SWAP:
            if (o.target >= (uint32_t)n || o.width >= (uint32_t)n) return bad("swap qubit >= n");
            if (o.target == o.width) return bad("swap of a qubit with itself");
            if (((o.ctrl_mask >> o.target) & 1ull) || ((o.ctrl_mask >> o.width) & 1ull))
                return bad("swap qubit is also a control");
            break;
        }
    }
    return SV_OK;
}

size_t esize(int dtype) { return dtype == SV_C64 ? 8 : 16; }

struct Scratch {
    double *d_partial = nullptr;  // kReduceBlocks * 2 doubles + 2 result doubles
    double *d_out() { return d_partial + 2 * svi::kReduceBlocks; }
};

// per-state reduction scratch, allocated with the state
struct StateExt {
    sv_state s;
    Scratch scratch;
};

StateExt *ext(const sv_state *s) { return reinterpret_cast<StateExt *>(const_cast<sv_state *>(s)); }

int upload_plan(sv_plan *p)
{
    HIP_TRY(hipGetDevice(&p->device));
    auto up = [&](void **dst, const void *src, size_t bytes) -> int {
        if (!bytes) bytes = 16;
        HIP_TRY(hipMalloc(dst, bytes));
        if (src) HIP_TRY(hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice));
        return SV_OK;
    };
    int rc;
    if ((rc = up(&p->d_passes, p->passes.empty() ? nullptr : p->passes.data(),
                 p->passes.size() * sizeof(svi::TilePass))) != SV_OK)
        return rc;
    if ((rc = up(&p->d_stages, p->stages.empty() ? nullptr : p->stages.data(),
                 p->stages.size() * sizeof(svi::TileStage))) != SV_OK)
        return rc;
    if ((rc = up(&p->d_tops, p->tops.empty() ? nullptr : p->tops.data(), p->tops.size() * sizeof(svi::TileOp))) !=
        SV_OK)
        return rc;
    if (p->dtype == SV_C64) {
        const std::vector<float> f = svi::tile_params_c64(p->tops, p->tparams);
        rc = up(&p->d_tparams, f.empty() ? nullptr : f.data(), f.size() * sizeof(float));
    } else {
        rc = up(&p->d_tparams, p->tparams.empty() ? nullptr : p->tparams.data(), p->tparams.size() * sizeof(double));
    }
    if (rc != SV_OK) return rc;
    if (!p->dense.empty()) {
        if ((rc = up(&p->d_dense, p->dense.data(), p->dense.size() * sizeof(svi::DensePass))) != SV_OK) return rc;
        if (p->dtype == SV_C64) {
            std::vector<float> f(p->dparams.begin(), p->dparams.end());
            rc = up(&p->d_dparams, f.data(), f.size() * sizeof(float));
        } else {
            rc = up(&p->d_dparams, p->dparams.data(), p->dparams.size() * sizeof(double));
        }
    }
    return rc;
}

void release_plan(sv_plan *p)
{
    if (p->d_passes) (void)hipFree(p->d_passes);
    if (p->d_stages) (void)hipFree(p->d_stages);
    if (p->d_tops) (void)hipFree(p->d_tops);
    if (p->d_tparams) (void)hipFree(p->d_tparams);
    if (p->d_dense) (void)hipFree(p->d_dense);
    if (p->d_dparams) (void)hipFree(p->d_dparams);
    p->d_passes = p->d_stages = p->d_tops = p->d_tparams = p->d_dense = p->d_dparams = nullptr;
}

int run_plan_on(const sv_plan *p, sv_state *s, hipStream_t stream)
{
    for (const auto &st : p->steps) {
        int rc = st.type == 0   ? svi::launch_plain(p->plain[st.index], s->n, s->dtype, s->d_psi, stream)
                 : st.type == 1 ? (p->compiled ? svi::launch_jit_pass(p, st.index, s->d_psi, stream)
                                               : svi::launch_tile_pass(p, st.index, s->d_psi, stream))
                                : svi::launch_dense_pass(p, st.index, s->d_psi, stream);
        if (rc != SV_OK) return fail(rc, "kernel launch failed");
    }
    return SV_OK;
}

int run_plan_once(const sv_plan *p, sv_state *s) { return run_plan_on(p, s, s->stream); }

// A plan is released when its last holder lets go: the caller (sv_plan_free)
// and every concurrent batch that runs it.
void plan_release(sv_plan *p)
{
    if (--p->refs > 0) return;
    release_plan(p);
    delete p;
}

int check_plan_state(const sv_plan *p, const sv_state *s)
{
    if (!p || !s) return fail(SV_EINVAL, "NULL plan or state");
    if (p->n != s->n || p->dtype != s->dtype) return fail(SV_EINVAL, "plan and state differ in size or precision");
    return SV_OK;
}

}  // namespace

extern "C" {

const char *sv_strerror(int code)
{
    switch (code) {
    case SV_OK: return "ok";
    case SV_EINVAL: return "invalid argument";
    case SV_ENOMEM: return "out of device memory";
    case SV_EZEROPROB: return "post-selection on a zero-probability subspace";
    case SV_EDEVICE: return "HIP runtime error";
    case SV_EUNSUPPORTED: return "unsupported request";
    default: return "unknown error";
    }
}

const char *sv_last_error(void) { return g_last_error.c_str(); }

int sv_alloc(int n_qubits, int dtype, const double *init, void *stream, sv_state **out)
{
    if (!out) return fail(SV_EINVAL, "out is NULL");
    *out = nullptr;
    if (n_qubits < 1 || n_qubits > 36) return fail(SV_EINVAL, "n_qubits must be in [1, 36]");
    if (dtype != SV_C64 && dtype != SV_C128) return fail(SV_EINVAL, "dtype must be SV_C64 or SV_C128");
    const size_t bytes = esize(dtype) << n_qubits;
    size_t free_b = 0, total_b = 0;
    HIP_TRY(hipMemGetInfo(&free_b, &total_b));
    if (bytes + (64ull << 20) > free_b) return fail(SV_ENOMEM, "state does not fit in free device memory");
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    int rc = ensure_device_setup(dev);
    if (rc != SV_OK) return rc;

    StateExt *e = new (std::nothrow) StateExt();
    if (!e) return fail(SV_ENOMEM, "host allocation failed");
    e->s.n = n_qubits;
    e->s.dtype = dtype;
    e->s.device = dev;
    hipError_t he = hipMalloc(&e->s.d_psi, bytes);
    if (he != hipSuccess) {
        delete e;
        (void)hipGetLastError();
        return fail(SV_ENOMEM, "hipMalloc of the state failed");
    }
    he = hipMalloc((void **)&e->scratch.d_partial, sizeof(double) * (2 * svi::kReduceBlocks + 2));
    if (he != hipSuccess) {
        (void)hipFree(e->s.d_psi);
        delete e;
        return fail(SV_ENOMEM, "hipMalloc of the reduction scratch failed");
    }
    if (stream) {
        e->s.stream = (hipStream_t)stream;
    } else {
        he = hipStreamCreateWithFlags(&e->s.stream, hipStreamNonBlocking);
        if (he != hipSuccess) {
            (void)hipFree(e->s.d_psi);
            (void)hipFree(e->scratch.d_partial);
            delete e;
            return hip_fail(he, "hipStreamCreateWithFlags");
        }
        e->s.own_stream = true;
    }
    if (init) {
        rc = sv_set_amplitudes(&e->s, 0, 1ull << n_qubits, init);
    } else {
        rc = svi::launch_init_basis(e->s.d_psi, n_qubits, dtype, e->s.stream);
        if (rc == SV_OK && hipStreamSynchronize(e->s.stream) != hipSuccess) rc = fail(SV_EDEVICE, "init failed");
    }
    if (rc != SV_OK) {
        sv_free(&e->s);
        return rc;
    }
    *out = &e->s;
    return SV_OK;
}

int sv_free(sv_state *s)
{
    if (!s) return SV_OK;
    StateExt *e = ext(s);
    (void)hipStreamSynchronize(s->stream);
    if (s->arena) {
        svi::Arena *a = s->arena;
        if (--a->refs == 0) {
            (void)hipFree(a->d_mem);
            if (a->own_stream) (void)hipStreamDestroy(a->stream);
            delete a;
        }
    } else {
        if (s->d_psi) (void)hipFree(s->d_psi);
        if (s->own_stream) (void)hipStreamDestroy(s->stream);
    }
    if (e->scratch.d_partial) (void)hipFree(e->scratch.d_partial);
    delete e;
    return SV_OK;
}

int sv_info(const sv_state *s, int *n_qubits, int *dtype)
{
    if (!s) return fail(SV_EINVAL, "NULL state");
    if (n_qubits) *n_qubits = s->n;
    if (dtype) *dtype = s->dtype;
    return SV_OK;
}

int sv_plan_create(int n_qubits, int dtype, const sv_op *ops, size_t n_ops, const double *params, size_t n_params,
                   const sv_apply_opts *opts, sv_plan **out)
{
    if (!out) return fail(SV_EINVAL, "out is NULL");
    *out = nullptr;
    if (n_qubits < 1 || n_qubits > 36) return fail(SV_EINVAL, "n_qubits must be in [1, 36]");
    if (dtype != SV_C64 && dtype != SV_C128) return fail(SV_EINVAL, "dtype must be SV_C64 or SV_C128");
    sv_apply_opts o{};
    o.mode = SV_MODE_FUSED;
    if (opts) o = *opts;
    if (o.mode != SV_MODE_PLAIN && o.mode != SV_MODE_FUSED) return fail(SV_EINVAL, "unknown mode");
    if (o.tile_launch < SV_TILE_LAUNCH_AUTO || o.tile_launch > SV_TILE_LAUNCH_PERSISTENT)
        return fail(SV_EINVAL, "unknown tile_launch");
    if (o.plain_split != SV_PLAIN_SPLIT_AUTO && o.plain_split != SV_PLAIN_SPLIT_OFF)
        return fail(SV_EINVAL, "unknown plain_split");
    if (o.compile != SV_COMPILE_AUTO && o.compile != SV_COMPILE_OFF && o.compile != SV_COMPILE_ON)
        return fail(SV_EINVAL, "unknown compile");
    if (o.dense_bf16 != 0 && o.dense_bf16 != 1) return fail(SV_EINVAL, "dense_bf16 must be 0 or 1");
    if (o.peephole != SV_PEEPHOLE_AUTO && o.peephole != SV_PEEPHOLE_OFF && o.peephole != SV_PEEPHOLE_ON)
        return fail(SV_EINVAL, "peephole must be SV_PEEPHOLE_AUTO, _OFF or _ON");
    if (o.split_real < SV_SPLIT_REAL_AUTO || o.split_real > SV_SPLIT_REAL_ON)
        return fail(SV_EINVAL, "split_real must be SV_SPLIT_REAL_AUTO, _OFF or _ON");
    int rc = validate_ops(n_qubits, ops, n_ops, params, n_params);
    if (rc != SV_OK) return rc;
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    rc = ensure_device_setup(dev);
    if (rc != SV_OK) return rc;
    sv_plan *p = new (std::nothrow) sv_plan();
    if (!p) return fail(SV_ENOMEM, "host allocation failed");
    p->n = n_qubits;
    p->dtype = dtype;
    p->tile_launch = o.tile_launch == SV_TILE_LAUNCH_AUTO ? svi::kDefaultTileLaunch : o.tile_launch;
    p->dense_bf16 = o.dense_bf16 == 1 && dtype == SV_C64;
    std::string err;
    rc = svi::build_plan(p, ops, n_ops, params, o, err);
    if (rc != SV_OK) {
        delete p;
        return fail(rc, err);
    }
    rc = upload_plan(p);
    if (rc != SV_OK) {
        release_plan(p);
        delete p;
        return rc;
    }
    // specialised pass kernels: on request, or automatically for states of 21
    // qubits and more (LDS of a pass up to 64 KiB)
    const bool can = o.mode == SV_MODE_FUSED && p->b > 0 && !p->passes.empty() && ((size_t)8 << p->b) <= 65536;
    // (tiles of 512 threads exist only as compiled passes: AUTO compiles them at any size)
    const bool wide = p->b > 0 && p->b - p->rb > 8;
    const bool want = o.compile == SV_COMPILE_ON || (o.compile == SV_COMPILE_AUTO && (n_qubits >= 21 || wide));
    if (can && want) {
        std::string jerr;
        rc = svi::jit_prepare(p, jerr);
        if (rc == SV_OK) {
            p->compiled = true;
        } else if (o.compile == SV_COMPILE_ON) {
            release_plan(p);
            delete p;
            return fail(rc, jerr);
        } else {
            p->jit_fn.clear();
            p->jit_prm.clear();
            p->info.n_compiled_kernels = 0;
        }
    } else if (o.compile == SV_COMPILE_ON && o.mode == SV_MODE_FUSED && p->b > 0 && !p->passes.empty()) {
        release_plan(p);
        delete p;
        return fail(SV_EUNSUPPORTED, "compiled tile passes need at most 64 KiB of LDS per tile");
    }
    if (!p->compiled && wide && !p->passes.empty()) {
        release_plan(p);
        delete p;
        return fail(SV_EUNSUPPORTED, "tiles of 512 threads run only as compiled passes (compilation unavailable)");
    }
    *out = p;
    return SV_OK;
}

int sv_plan_free(sv_plan *p)
{
    if (!p) return SV_OK;
    plan_release(p);
    return SV_OK;
}

int sv_plan_get_info(const sv_plan *p, sv_plan_info *info)
{
    if (!p || !info) return fail(SV_EINVAL, "NULL argument");
    *info = p->info;
    return SV_OK;
}

int sv_plan_execute(sv_plan *p, sv_state *s, int repeat)
{
    int rc = check_plan_state(p, s);
    if (rc != SV_OK) return rc;
    if (repeat < 0) return fail(SV_EINVAL, "repeat < 0");
    for (int r = 0; r < repeat; ++r)
        if ((rc = run_plan_once(p, s)) != SV_OK) return rc;
    HIP_TRY(hipStreamSynchronize(s->stream));
    return SV_OK;
}

int sv_plan_execute_seq(sv_plan *const *plans, size_t n_plans, const int32_t *seq, size_t seq_len, sv_state *s)
{
    if (!plans || (!seq && seq_len)) return fail(SV_EINVAL, "NULL argument");
    for (size_t k = 0; k < seq_len; ++k)
        if (seq[k] < 0 || (size_t)seq[k] >= n_plans) return fail(SV_EINVAL, "sequence entry outside the plan array");
    for (size_t k = 0; k < seq_len; ++k) {
        int rc = check_plan_state(plans[seq[k]], s);
        if (rc != SV_OK) return rc;
    }
    for (size_t k = 0; k < seq_len; ++k) {
        int rc = run_plan_once(plans[seq[k]], s);
        if (rc != SV_OK) return rc;
    }
    HIP_TRY(hipStreamSynchronize(s->stream));
    return SV_OK;
}

int sv_plan_time(sv_plan *p, sv_state *s, int repeat, double *ms)
{
    int rc = check_plan_state(p, s);
    if (rc != SV_OK) return rc;
    if (!ms || repeat < 1) return fail(SV_EINVAL, "ms is NULL or repeat < 1");
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    HIP_TRY(hipEventRecord(e0, s->stream));
    for (int r = 0; r < repeat && rc == SV_OK; ++r) rc = run_plan_once(p, s);
    HIP_TRY(hipEventRecord(e1, s->stream));
    HIP_TRY(hipEventSynchronize(e1));
    float f = 0.f;
    HIP_TRY(hipEventElapsedTime(&f, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *ms = f;
    return rc;
}

int sv_apply_circuit(sv_state *s, const sv_op *ops, size_t n_ops, const double *params, size_t n_params,
                     const sv_apply_opts *opts)
{
    if (!s) return fail(SV_EINVAL, "NULL state");
    sv_plan *p = nullptr;
    int rc = sv_plan_create(s->n, s->dtype, ops, n_ops, params, n_params, opts, &p);
    if (rc != SV_OK) return rc;
    rc = sv_plan_execute(p, s, 1);
    sv_plan_free(p);
    return rc;
}

int sv_postselect(sv_state *s, uint64_t mask, uint64_t value, int keep, int renormalize, double *prob_out)
{
    if (!s) return fail(SV_EINVAL, "NULL state");
    const uint64_t all = (1ull << s->n) - 1ull;
    if ((mask & ~all) || (value & ~mask)) return fail(SV_EINVAL, "mask/value outside the state or value not in mask");
    Scratch &sc = ext(s)->scratch;
    int rc = svi::launch_prob(s->d_psi, s->n, s->dtype, mask, value, sc.d_partial, svi::kReduceBlocks, sc.d_out(),
                              s->stream);
    if (rc != SV_OK) return fail(rc, "reduction launch failed");
    double P = 0.0;
    HIP_TRY(hipMemcpyAsync(&P, sc.d_out(), sizeof(double), hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    if (prob_out) *prob_out = P;
    if (!keep) return SV_OK;
    if (!(P > 0.0)) return fail(SV_EZEROPROB, "post-selected subspace has probability 0");
    const double scale = renormalize ? 1.0 / std::sqrt(P) : 1.0;
    rc = svi::launch_keep_scale(s->d_psi, s->n, s->dtype, mask, value, scale, s->stream);
    if (rc != SV_OK) return fail(rc, "post-selection launch failed");
    HIP_TRY(hipStreamSynchronize(s->stream));
    return SV_OK;
}

static const uint64_t kChunk = 1ull << 22;  // amplitudes per staged copy (64 MiB of complex128)

int sv_amplitudes(const sv_state *s, uint64_t offset, uint64_t count, double *out)
{
    if (!s || (!out && count)) return fail(SV_EINVAL, "NULL argument");
    const uint64_t dim = 1ull << s->n;
    if (offset > dim || count > dim - offset) return fail(SV_EINVAL, "range outside the state");
    if (!count) return SV_OK;
    void *stage = nullptr;
    const uint64_t cap = count < kChunk ? count : kChunk;
    HIP_TRY(hipMalloc(&stage, cap * 16));
    int rc = SV_OK;
    for (uint64_t k = 0; k < count && rc == SV_OK; k += cap) {
        const uint64_t m = (count - k) < cap ? (count - k) : cap;
        rc = svi::launch_to_c128(s->d_psi, s->dtype, stage, offset + k, m, s->stream);
        if (rc == SV_OK && hipMemcpyAsync(out + 2 * k, stage, m * 16, hipMemcpyDeviceToHost, s->stream) != hipSuccess)
            rc = fail(SV_EDEVICE, "device-to-host copy failed");
        if (rc == SV_OK && hipStreamSynchronize(s->stream) != hipSuccess) rc = fail(SV_EDEVICE, "sync failed");
    }
    (void)hipFree(stage);
    return rc;
}

int sv_amplitudes_noalloc(const sv_state *s, uint64_t offset, uint64_t count, double *out)
{
    if (!s || (!out && count)) return fail(SV_EINVAL, "NULL argument");
    const uint64_t dim = 1ull << s->n;
    if (offset > dim || count > dim - offset) return fail(SV_EINVAL, "range outside the state");
    if (count > kScratchAmps)
        return fail(SV_EINVAL, "count exceeds the static staging buffer of sv_amplitudes_noalloc (262144 amplitudes)");
    if (!count) return SV_OK;
    void *stage = scratch_on(s->device);  // set when the state was allocated on its device
    if (!stage) return fail(SV_EDEVICE, "the static staging buffer was not set up on the state's device");
    int rc = svi::launch_to_c128(s->d_psi, s->dtype, stage, offset, count, s->stream);
    if (rc != SV_OK) return fail(rc, "conversion launch failed");
    HIP_TRY(hipMemcpyAsync(out, stage, count * 16, hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    return SV_OK;
}

int sv_set_amplitudes(sv_state *s, uint64_t offset, uint64_t count, const double *in)
{
    if (!s || (!in && count)) return fail(SV_EINVAL, "NULL argument");
    const uint64_t dim = 1ull << s->n;
    if (offset > dim || count > dim - offset) return fail(SV_EINVAL, "range outside the state");
    if (!count) return SV_OK;
    void *stage = nullptr;
    const uint64_t cap = count < kChunk ? count : kChunk;
    HIP_TRY(hipMalloc(&stage, cap * 16));
    int rc = SV_OK;
    for (uint64_t k = 0; k < count && rc == SV_OK; k += cap) {
        const uint64_t m = (count - k) < cap ? (count - k) : cap;
        if (hipMemcpyAsync(stage, in + 2 * k, m * 16, hipMemcpyHostToDevice, s->stream) != hipSuccess)
            rc = fail(SV_EDEVICE, "host-to-device copy failed");
        if (rc == SV_OK) rc = svi::launch_from_c128(s->d_psi, s->dtype, stage, offset + k, m, s->stream);
        if (rc == SV_OK && hipStreamSynchronize(s->stream) != hipSuccess) rc = fail(SV_EDEVICE, "sync failed");
    }
    (void)hipFree(stage);
    return rc;
}

int sv_copy(sv_state *dst, const sv_state *src)
{
    if (!dst || !src) return fail(SV_EINVAL, "NULL state");
    if (dst->n != src->n) return fail(SV_EINVAL, "states differ in qubit count");
    HIP_TRY(hipStreamSynchronize(src->stream));
    int rc = svi::launch_copy(dst->d_psi, dst->dtype, src->d_psi, src->dtype, dst->n, dst->stream);
    if (rc != SV_OK) return fail(rc, "copy launch failed");
    HIP_TRY(hipStreamSynchronize(dst->stream));
    return SV_OK;
}

int sv_inner(const sv_state *a, const sv_state *b, double *re, double *im)
{
    if (!a || !b) return fail(SV_EINVAL, "NULL state");
    if (a->n != b->n) return fail(SV_EINVAL, "states differ in qubit count");
    HIP_TRY(hipStreamSynchronize(b->stream));
    Scratch &sc = ext(a)->scratch;
    int rc = svi::launch_inner(a->d_psi, a->dtype, b->d_psi, b->dtype, a->n, sc.d_partial, svi::kReduceBlocks,
                               sc.d_out(), a->stream);
    if (rc != SV_OK) return fail(rc, "inner-product launch failed");
    double v[2] = {0, 0};
    HIP_TRY(hipMemcpyAsync(v, sc.d_out(), sizeof v, hipMemcpyDeviceToHost, a->stream));
    HIP_TRY(hipStreamSynchronize(a->stream));
    if (re) *re = v[0];
    if (im) *im = v[1];
    return SV_OK;
}


int sv_alloc_batch(int count, const int *n_qubits, int dtype, void *stream, sv_state **out)
{
    if (count < 1 || !n_qubits || !out) return fail(SV_EINVAL, "count < 1 or NULL argument");
    if (dtype != SV_C64 && dtype != SV_C128) return fail(SV_EINVAL, "dtype must be SV_C64 or SV_C128");
    for (int i = 0; i < count; ++i) {
        out[i] = nullptr;
        if (n_qubits[i] < 1 || n_qubits[i] > 36) return fail(SV_EINVAL, "n_qubits must be in [1, 36]");
    }
    const uint64_t align = 2ull << 20;  // 2 MiB: states start on large-page boundaries
    std::vector<uint64_t> off(count);
    uint64_t total = 0;
    for (int i = 0; i < count; ++i) {
        off[i] = total;
        const uint64_t bytes = (uint64_t)esize(dtype) << n_qubits[i];
        total += (bytes + align - 1) / align * align;
    }
    size_t free_b = 0, total_b = 0;
    HIP_TRY(hipMemGetInfo(&free_b, &total_b));
    if (total + (64ull << 20) + (uint64_t)count * sizeof(double) * (2 * svi::kReduceBlocks + 2) > free_b)
        return fail(SV_ENOMEM, "the batch does not fit in free device memory");
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    int rc = ensure_device_setup(dev);
    if (rc != SV_OK) return rc;
    svi::Arena *a = new (std::nothrow) svi::Arena();
    if (!a) return fail(SV_ENOMEM, "host allocation failed");
    if (hipMalloc(&a->d_mem, total) != hipSuccess) {
        (void)hipGetLastError();
        delete a;
        return fail(SV_ENOMEM, "hipMalloc of the arena failed");
    }
    if (stream) {
        a->stream = (hipStream_t)stream;
    } else if (hipStreamCreateWithFlags(&a->stream, hipStreamNonBlocking) != hipSuccess) {
        (void)hipFree(a->d_mem);
        delete a;
        return fail(SV_EDEVICE, "hipStreamCreateWithFlags failed");
    } else {
        a->own_stream = true;
    }
    for (int i = 0; i < count; ++i) {
        StateExt *e = new (std::nothrow) StateExt();
        if (e && hipMalloc((void **)&e->scratch.d_partial, sizeof(double) * (2 * svi::kReduceBlocks + 2)) != hipSuccess) {
            delete e;
            e = nullptr;
        }
        if (!e) {
            if (i == 0) {  // no state holds the arena yet
                (void)hipFree(a->d_mem);
                if (a->own_stream) (void)hipStreamDestroy(a->stream);
                delete a;
            } else {       // the last sv_free releases the arena
                for (int j = 0; j < i; ++j) {
                    sv_free(out[j]);
                    out[j] = nullptr;
                }
            }
            return fail(SV_ENOMEM, "allocation of a batch state failed");
        }
        e->s.n = n_qubits[i];
        e->s.dtype = dtype;
        e->s.device = dev;
        e->s.d_psi = (char *)a->d_mem + off[i];
        e->s.stream = a->stream;
        e->s.arena = a;
        a->refs += 1;
        out[i] = &e->s;
        rc = svi::launch_init_basis(e->s.d_psi, e->s.n, dtype, a->stream);
        if (rc != SV_OK) {
            for (int j = 0; j <= i; ++j) {
                sv_free(out[j]);
                out[j] = nullptr;
            }
            return fail(rc, "state initialisation failed");
        }
    }
    HIP_TRY(hipStreamSynchronize(a->stream));
    return SV_OK;
}

namespace {
// Concurrent form: instances assigned to side streams largest first, each to
// the stream with the least modelled work so far (its plans' algorithmic
// bytes plus a fixed cost per launch), so small instances overlap the large
// ones and each other instead of running one after another.
int batch_create_concurrent(sv_state *const *states, sv_plan *const *plans, size_t count, int use_graph,
                            sv_batch **out)
{
    constexpr size_t kSideStreams = 4;  // the device's hardware queues per process
    sv_batch *B = new (std::nothrow) sv_batch();
    if (!B) return fail(SV_ENOMEM, "host allocation failed");
    B->concurrent = true;
    B->stream = states[0]->stream;
    B->use_graph = use_graph != 0;
    B->states.assign(states, states + count);
    B->plans.assign(plans, plans + count);
    const size_t k = std::min(count, kSideStreams);
    auto cleanup = [&]() {
        for (hipStream_t st : B->side) (void)hipStreamDestroy(st);
        for (hipEvent_t e : B->events) (void)hipEventDestroy(e);
        delete B;
    };
    for (size_t j = 0; j < k; ++j) {
        hipStream_t st = nullptr;
        if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
            cleanup();
            return fail(SV_EDEVICE, "hipStreamCreateWithFlags failed");
        }
        B->side.push_back(st);
    }
    for (size_t j = 0; j <= k; ++j) {
        hipEvent_t e = nullptr;
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
            cleanup();
            return fail(SV_EDEVICE, "hipEventCreateWithFlags failed");
        }
        B->events.push_back(e);
    }
    std::vector<size_t> order(count);
    for (size_t i = 0; i < count; ++i) order[i] = i;
    auto cost = [&](size_t i) { return (double)plans[i]->info.bytes_moved / 4.0e6 + 8.0 * plans[i]->steps.size(); };
    std::stable_sort(order.begin(), order.end(), [&](size_t a, size_t b) { return cost(a) > cost(b); });
    std::vector<double> load(k, 0.0);
    B->stream_of.assign(count, 0);
    for (size_t i : order) {
        const size_t j = (size_t)(std::min_element(load.begin(), load.end()) - load.begin());
        B->stream_of[i] = (uint32_t)j;
        load[j] += cost(i);
    }
    for (size_t i = 0; i < count; ++i) {
        B->gates += plans[i]->info.n_ops;
        B->launches += plans[i]->steps.size();
    }
    for (size_t i = 0; i < count; ++i) plans[i]->refs += 1;  // released with the batch
    B->groups = k;
    *out = B;
    return SV_OK;
}

int batch_launch_concurrent(sv_batch *B)
{
    HIP_TRY(hipEventRecord(B->events[0], B->stream));
    for (hipStream_t st : B->side) HIP_TRY(hipStreamWaitEvent(st, B->events[0], 0));
    // instances in submission order of each stream (largest first, as assigned)
    for (size_t j = 0; j < B->side.size(); ++j)
        for (size_t i = 0; i < B->plans.size(); ++i)
            if (B->stream_of[i] == j) {
                int rc = run_plan_on(B->plans[i], B->states[i], B->side[j]);
                if (rc != SV_OK) return rc;
            }
    for (size_t j = 0; j < B->side.size(); ++j) {
        HIP_TRY(hipEventRecord(B->events[j + 1], B->side[j]));
        HIP_TRY(hipStreamWaitEvent(B->stream, B->events[j + 1], 0));
    }
    return SV_OK;
}
}  // namespace

int sv_batch_create(sv_state *const *states, sv_plan *const *plans, size_t count, int use_graph,
                    uint64_t group_bytes, sv_batch **out)
{
    if (!states || !plans || !out || count == 0) return fail(SV_EINVAL, "NULL argument or empty batch");
    *out = nullptr;
    bool all_compiled = true;
    for (size_t i = 0; i < count; ++i) {
        int rc = check_plan_state(plans[i], states[i]);
        if (rc != SV_OK) return rc;
        all_compiled = all_compiled && plans[i]->compiled;
        for (size_t j = 0; j < i; ++j)
            if (states[j] == states[i]) return fail(SV_EINVAL, "a state appears twice in the batch");
        if (states[i]->device != states[0]->device) return fail(SV_EINVAL, "batched states must share one device");
    }
    if (all_compiled) return batch_create_concurrent(states, plans, count, use_graph, out);
    const sv_plan *p0 = plans[0];
    svi::Arena *arena = states[0] ? states[0]->arena : nullptr;
    if (!arena) return fail(SV_EINVAL, "batched states must come from one sv_alloc_batch arena");
    for (size_t i = 0; i < count; ++i) {
        int rc = check_plan_state(plans[i], states[i]);
        if (rc != SV_OK) return rc;
        const sv_plan *p = plans[i];
        if (p->b == 0 || p->b != p0->b || p->rb != p0->rb || p->dtype != p0->dtype)
            return fail(SV_EINVAL, "batched plans must be fused with one tile geometry and one precision");
        if (p->b - p->rb > 8)
            return fail(SV_EUNSUPPORTED, "the level-synchronous batch runs tiles of at most 256 threads");
        for (const auto &st : p->steps)
            if (st.type != 1) return fail(SV_EUNSUPPORTED, "batched plans must consist of tile passes only");
        if (states[i]->arena != arena) return fail(SV_EINVAL, "batched states must come from one sv_alloc_batch arena");
        for (size_t j = 0; j < i; ++j)
            if (states[j] == states[i]) return fail(SV_EINVAL, "a state appears twice in the batch");
    }
    sv_batch *B = new (std::nothrow) sv_batch();
    if (!B) return fail(SV_ENOMEM, "host allocation failed");
    B->stream = states[0]->stream;
    B->use_graph = use_graph != 0;
    B->states.assign(states, states + count);
    for (size_t i = 0; i < count; ++i) B->gates += plans[i]->info.n_ops;

    // one copy of every distinct plan's tables, indices rebased
    std::vector<svi::TilePass> passes;
    std::vector<svi::TileStage> stages;
    std::vector<svi::TileOp> tops;
    std::vector<double> prm;
    std::vector<float> prmf;  // complex64: each plan's parameters as its own upload rounds them
    std::vector<const sv_plan *> seen;
    std::vector<uint64_t> pass_base(count);
    for (size_t i = 0; i < count; ++i) {
        const sv_plan *p = plans[i];
        size_t k = 0;
        while (k < seen.size() && seen[k] != p) ++k;
        if (k < seen.size()) {  // same plan as instance j: same tables
            for (size_t j = 0; j < i; ++j)
                if (plans[j] == p) pass_base[i] = pass_base[j];
            continue;
        }
        seen.push_back(p);
        const uint32_t so = (uint32_t)stages.size(), to = (uint32_t)tops.size();
        pass_base[i] = passes.size();
        for (svi::TilePass P : p->passes) {
            P.stage_begin += so;
            P.stage_end += so;
            P.fperm_begin += to;
            P.fperm_end += to;
            passes.push_back(P);
        }
        for (svi::TileStage S : p->stages) {
            S.op_begin += to;
            S.op_end += to;
            S.perm_begin += to;
            S.perm_end += to;
            stages.push_back(S);
        }
        for (svi::TileOp t : p->tops) {
            t.param += to * (uint32_t)svi::kParamStride;
            tops.push_back(t);
        }
        prm.insert(prm.end(), p->tparams.begin(), p->tparams.end());
        prm.resize(tops.size() * svi::kParamStride, 0.0);
        if (p->dtype == SV_C64) {
            const std::vector<float> f = svi::tile_params_c64(p->tops, p->tparams);
            prmf.insert(prmf.end(), f.begin(), f.end());
            prmf.resize(tops.size() * svi::kParamStride, 0.0f);
        }
    }
    auto cleanup = [&]() {
        for (auto *d : B->d_items) (void)hipFree(d);
        for (void *d : B->d_tables) (void)hipFree(d);
        delete B;
    };
    auto upload = [&](const void *src, size_t bytes) -> void * {
        void *d = nullptr;
        if (hipMalloc(&d, bytes ? bytes : 16) != hipSuccess) return nullptr;
        if (bytes && hipMemcpy(d, src, bytes, hipMemcpyHostToDevice) != hipSuccess) {
            (void)hipFree(d);
            return nullptr;
        }
        B->d_tables.push_back(d);
        return d;
    };
    svi::BatchTables &T = B->tables;
    T.arena = arena->d_mem;
    T.dtype = p0->dtype;
    T.b = p0->b;
    T.rb = p0->rb;
    T.nthr = p0->b - p0->rb;
    T.passes = upload(passes.data(), passes.size() * sizeof(svi::TilePass));
    T.stages = upload(stages.data(), stages.size() * sizeof(svi::TileStage));
    T.ops = upload(tops.data(), tops.size() * sizeof(svi::TileOp));
    if (p0->dtype == SV_C64) {
        T.prm = upload(prmf.data(), prmf.size() * sizeof(float));
    } else {
        T.prm = upload(prm.data(), prm.size() * sizeof(double));
    }
    if (!T.passes || !T.stages || !T.ops || !T.prm) {
        cleanup();
        return fail(SV_ENOMEM, "upload of the batch tables failed");
    }

    // Groups: instances sorted by state size are packed greedily into groups
    // whose states together stay within group_bytes, so a group that fits the
    // device's last-level cache keeps its states there across its levels; each
    // group runs level by level, groups one after another.
    if (group_bytes == 0) group_bytes = 192ull << 20;
    std::vector<size_t> order(count);
    for (size_t i = 0; i < count; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](size_t a, size_t b) { return states[a]->n < states[b]->n; });
    std::vector<std::vector<size_t>> groups;
    uint64_t acc = 0;
    for (size_t i : order) {
        const uint64_t bytes = (uint64_t)esize(states[i]->dtype) << states[i]->n;
        if (groups.empty() || (acc + bytes > group_bytes && !groups.back().empty())) {
            groups.emplace_back();
            acc = 0;
        }
        groups.back().push_back(i);
        acc += bytes;
    }
    const size_t es = esize(p0->dtype);
    for (const auto &grp : groups) {
        size_t glevels = 0;
        for (size_t i : grp) glevels = std::max(glevels, plans[i]->steps.size());
        for (size_t lv = 0; lv < glevels; ++lv) {
            std::vector<svi::BatchItem> items;
            uint64_t total = 0;
            uint8_t runs = 0;
            uint64_t level_bytes = 0;
            for (size_t i : grp) {
                const sv_plan *p = plans[i];
                if (lv >= p->steps.size()) continue;
                const uint32_t pi = p->steps[lv].index;
                runs |= p->passes[pi].gate_runs;
                level_bytes += (uint64_t)es << p->n;
                svi::BatchItem it{};
                it.psi_off = (uint64_t)((char *)states[i]->d_psi - (char *)arena->d_mem) / es;
                it.pass_index = pass_base[i] + pi;
                it.item_begin = total;
                total += 1ull << p->passes[pi].ntile;
                items.push_back(it);
            }
            svi::BatchItem *d = nullptr;
            if (hipMalloc((void **)&d, items.size() * sizeof(svi::BatchItem)) != hipSuccess ||
                hipMemcpy(d, items.data(), items.size() * sizeof(svi::BatchItem), hipMemcpyHostToDevice) != hipSuccess) {
                if (d) (void)hipFree(d);
                cleanup();
                return fail(SV_ENOMEM, "upload of the batch tables failed");
            }
            B->d_items.push_back(d);
            B->n_items.push_back((uint32_t)items.size());
            B->total.push_back(total);
            B->gate_runs.push_back(runs);
            B->stream_state.push_back(svi::stream_state_bytes(level_bytes) ? 1 : 0);
        }
    }
    B->groups = groups.size();
    *out = B;
    return SV_OK;
}

namespace {
int batch_launch_all(sv_batch *B)
{
    if (B->concurrent) return batch_launch_concurrent(B);
    for (size_t lv = 0; lv < B->d_items.size(); ++lv) {
        int rc = svi::launch_tile_batch(B->tables, B->d_items[lv], B->n_items[lv], B->total[lv], B->gate_runs[lv] != 0,
                                        B->stream_state[lv] != 0, B->stream);
        if (rc != SV_OK) return fail(rc, "batched launch failed");
    }
    return SV_OK;
}

int batch_run_once(sv_batch *B)
{
    if (!B->use_graph) return batch_launch_all(B);
    if (!B->graph_ready) {
        HIP_TRY(hipStreamBeginCapture(B->stream, hipStreamCaptureModeThreadLocal));
        int rc = batch_launch_all(B);
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(B->stream, &g);
        if (rc != SV_OK) {
            if (g) (void)hipGraphDestroy(g);
            return rc;
        }
        if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
        e = hipGraphInstantiate(&B->exec, g, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            (void)hipGraphDestroy(g);
            return hip_fail(e, "hipGraphInstantiate");
        }
        B->graph = g;
        B->graph_ready = true;
    }
    HIP_TRY(hipGraphLaunch(B->exec, B->stream));
    return SV_OK;
}
}  // namespace

int sv_batch_execute(sv_batch *B, int repeat)
{
    if (!B || repeat < 0) return fail(SV_EINVAL, "NULL batch or repeat < 0");
    for (int r = 0; r < repeat; ++r) {
        int rc = batch_run_once(B);
        if (rc != SV_OK) return rc;
    }
    HIP_TRY(hipStreamSynchronize(B->stream));
    return SV_OK;
}

int sv_batch_time(sv_batch *B, int repeat, double *ms)
{
    if (!B || !ms || repeat < 1) return fail(SV_EINVAL, "NULL argument or repeat < 1");
    if (B->use_graph && !B->graph_ready) {  // capture outside the timed region
        int rc = batch_run_once(B);
        if (rc != SV_OK) return rc;
        HIP_TRY(hipStreamSynchronize(B->stream));
    }
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    HIP_TRY(hipEventRecord(e0, B->stream));
    int rc = SV_OK;
    for (int r = 0; r < repeat && rc == SV_OK; ++r) rc = batch_run_once(B);
    HIP_TRY(hipEventRecord(e1, B->stream));
    HIP_TRY(hipEventSynchronize(e1));
    float f = 0.f;
    HIP_TRY(hipEventElapsedTime(&f, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *ms = f;
    return rc;
}

int sv_batch_levels(const sv_batch *B, uint64_t *launches, uint64_t *groups, uint64_t *gates)
{
    if (!B) return fail(SV_EINVAL, "NULL batch");
    if (launches) *launches = B->concurrent ? B->launches : B->d_items.size();
    if (groups) *groups = B->groups;
    if (gates) *gates = B->gates;
    return SV_OK;
}

int sv_batch_free(sv_batch *B)
{
    if (!B) return SV_OK;
    (void)hipStreamSynchronize(B->stream);
    if (B->exec) (void)hipGraphExecDestroy(B->exec);
    if (B->graph) (void)hipGraphDestroy(B->graph);
    for (auto *d : B->d_items) (void)hipFree(d);
    for (void *d : B->d_tables) (void)hipFree(d);
    for (hipStream_t st : B->side) {
        (void)hipStreamSynchronize(st);
        (void)hipStreamDestroy(st);
    }
    for (hipEvent_t e : B->events) (void)hipEventDestroy(e);
    for (sv_plan *p : B->plans) plan_release(p);
    delete B;
    return SV_OK;
}

}  // extern "C"
