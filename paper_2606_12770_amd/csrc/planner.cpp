// Host planner: turns a validated op list into launch steps.
//
// Plain mode: one step per op.
// Fused mode: ops are grouped into tile passes.  An op can join a pass whose
// resident ("local") qubit set S contains the qubits it moves amplitudes
// along (target of U/X, register of INC/DEC, both qubits of SWAP); diagonal
// ops (PHASE, PROJPHASE) and all control qubits impose nothing, because tile
// qubits are constant inside a workgroup and conditions on them are uniform.
// Ops may be moved ahead of earlier ops they commute with: two ops commute
// when every qubit they share is diagonal-type (control or phase) in both, or
// the target of an X in both.
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstring>

#include "plan_types.h"

namespace svi {

namespace {

struct OpInfo {
    uint32_t kind;
    uint32_t target, width;
    uint64_t mask, val;
    double m[8];
    uint64_t req;   // qubits that must be resident
    uint64_t z, x, g;
};

OpInfo normalize(const sv_op &o, const double *params)
{
    OpInfo r{};
    r.kind = o.kind;
    r.target = o.target;
    r.width = o.width;
    r.mask = o.ctrl_mask;
    r.val = o.ctrl_val;
    const double *p = params + o.param;
    const uint64_t tb = 1ull << o.target;
    switch (o.kind) {
    case SV_OP_U:
        for (int k = 0; k < 8; ++k) r.m[k] = p[k];
        r.req = tb;
        r.g = tb;
        r.z = o.ctrl_mask;
        break;
    case SV_OP_RY: {
        const double c = std::cos(0.5 * p[0]), s = std::sin(0.5 * p[0]);
        r.kind = SV_OP_U;
        const double m[8] = {c, 0, -s, 0, s, 0, c, 0};
        std::memcpy(r.m, m, sizeof m);
        r.req = tb;
        r.g = tb;
        r.z = o.ctrl_mask;
        break;
    }
    case SV_OP_X:
        r.req = tb;
        r.x = tb;
        r.z = o.ctrl_mask;
        break;
    case SV_OP_PHASE:
        r.m[0] = p[0];
        r.z = o.ctrl_mask | tb;
        break;
    case SV_OP_PROJPHASE:
        r.m[0] = p[0];
        r.z = o.ctrl_mask | tb;
        break;
    case SV_OP_INC:
    case SV_OP_DEC: {
        const uint64_t reg = ((1ull << o.width) - 1ull) << o.target;
        r.req = reg;
        r.g = reg;
        r.z = o.ctrl_mask;
        break;
    }
    case SV_OP_SWAP: {
        const uint64_t ab = tb | (1ull << o.width);
        r.req = ab;
        r.g = ab;
        r.z = o.ctrl_mask;
        break;
    }
    default:
        break;
    }
    return r;
}

PlainOp to_plain(const OpInfo &o)
{
    PlainOp p{};
    p.kind = o.kind;
    p.target = o.target;
    p.width = o.width;
    p.mask = o.mask;
    p.val = o.val;
    std::memcpy(p.m, o.m, sizeof p.m);
    return p;
}

uint64_t plain_bytes(const OpInfo &o, int n, int s)
{
    const int c = __builtin_popcountll(o.mask);
    switch (o.kind) {
    case SV_OP_U:
    case SV_OP_X:
        return 2ull * (1ull << (n - c)) * s;
    case SV_OP_PHASE:
        return 2ull * (1ull << (n - 1 - c)) * s;
    case SV_OP_SWAP:
        return 2ull * (1ull << (n - 1 - c)) * s;
    case SV_OP_INC:
    case SV_OP_DEC:
        return 2ull * (1ull << (n - c)) * s;
    default:
        return 2ull * (1ull << n) * s;
    }
}

// Bytes a plain launch of the op moves at cache-line granularity (128 B): a
// control (or a phase/swap condition) on one of the qubits inside a line
// does not reduce the lines touched.
uint64_t touched_bytes(const OpInfo &o, int n, int s)
{
    const int line_bits = s == 8 ? 4 : 3;
    const uint64_t in_line = (1ull << line_bits) - 1ull;
    const int c = __builtin_popcountll(o.mask & ~in_line);
    const uint64_t all = 2ull * (1ull << n) * s;
    switch (o.kind) {
    case SV_OP_U:
    case SV_OP_X:
    case SV_OP_INC:
    case SV_OP_DEC:
        return all >> c;
    case SV_OP_PHASE:
        return all >> (c + (o.target >= (uint32_t)line_bits ? 1 : 0));
    case SV_OP_SWAP:
        return all >> (c + (o.target >= (uint32_t)line_bits && o.width >= (uint32_t)line_bits ? 1 : 0));
    default:
        return all;
    }
}

// Modelled device time (microseconds) of a tile pass and of one plain launch:
// a fixed cost per launch (launch, fill and drain of a small grid) plus bytes
// at the sustained rate of each kernel family.  A plain register shift wider
// than 8 qubits walks its orbit serially, one dependent access per value.
constexpr double kTileFixedUs = 8.0, kTileBytesPerUs = 3.8e6;
constexpr double kPlainFixedUs = 4.0, kPlainBytesPerUs = 4.0e6;
// Cost of one op inside a tile pass: every tile reads its record and checks its
// tile condition (register moves and scalar work per wave, measured about
// 0.3 ns per tile and op), and the amplitudes it applies to cost about 0.32 ps
// each (the VALU work of a complex 2 x 2 gate in the fused kernel).
constexpr double kOpPerTileUs = 0.31e-3, kOpPerAmpUs = 0.32e-6;
// A dense 5-qubit block pass: a fixed cost per launch plus one sweep of the
// state at the rate the matrix-core pass sustains (measured 4.7 TB/s complex64
// and 4.9 TB/s complex128 on 28 qubits).
constexpr double kDenseFixedUs = 8.0, kDenseBytesPerUs = 4.7e6, kDenseFp32FlopPerUs = 9.0e7;
constexpr int kLookahead = 8;  // candidate resident-set widenings compared per step
constexpr int kMinGateRun = 6;  // shortest run of ops with one tile mask worth a bisection
double plain_us(const OpInfo &o, int n, int s)
{
    double t = kPlainFixedUs + (double)touched_bytes(o, n, s) / kPlainBytesPerUs;
    if ((o.kind == SV_OP_INC || o.kind == SV_OP_DEC) && o.width > 8) t += 0.3 * (double)(1ull << o.width);
    return t;
}

// j commutes with every op whose roles are accumulated in (Z, X, G)
inline bool commutes_with_all(const OpInfo &o, uint64_t Z, uint64_t X, uint64_t G)
{
    const uint64_t fp = o.z | o.x | o.g;
    return (fp & G) == 0 && (o.g & (Z | X)) == 0 && (o.z & X) == 0 && (o.x & Z) == 0;
}

struct PassBuild {
    uint64_t S = 0;
    std::vector<uint32_t> ops;
};

uint64_t touched_qubits(const OpInfo &o) { return o.z | o.x | o.g | (1ull << o.target); }

// Fold an uncontrolled single-qubit matrix into the previous op on its qubit
// when that op is also an uncontrolled single-qubit matrix on it: no op in
// between touches the qubit, so the later gate commutes back to the earlier
// one and the two become one matrix (later x earlier).
std::vector<OpInfo> fold_single_qubit_runs(const std::vector<OpInfo> &in)
{
    std::vector<OpInfo> out;
    out.reserve(in.size());
    long last[64];
    for (long &v : last) v = -1;
    for (const OpInfo &o : in) {
        if (o.kind == SV_OP_U && o.mask == 0) {
            const long j = last[o.target];
            if (j >= 0 && out[j].kind == SV_OP_U && out[j].mask == 0 && out[j].target == o.target) {
                const double *a = o.m, *b = out[j].m;  // new = a . b (complex 2x2, row-major re/im pairs)
                double r[8];
                for (int i = 0; i < 2; ++i)
                    for (int k = 0; k < 2; ++k) {
                        double re = 0.0, im = 0.0;
                        for (int l = 0; l < 2; ++l) {
                            const double ar = a[2 * (2 * i + l)], ai = a[2 * (2 * i + l) + 1];
                            const double br = b[2 * (2 * l + k)], bi = b[2 * (2 * l + k) + 1];
                            re += ar * br - ai * bi;
                            im += ar * bi + ai * br;
                        }
                        r[2 * (2 * i + k)] = re;
                        r[2 * (2 * i + k) + 1] = im;
                    }
                std::memcpy(out[j].m, r, sizeof r);
                continue;
            }
        }
        out.push_back(o);
        const uint64_t t = touched_qubits(o);
        for (int q = 0; q < 64; ++q)
            if ((t >> q) & 1ull) last[q] = (long)out.size() - 1;
    }
    return out;
}

// Peephole cancellation (Sec. III.F.2 post-processes the compiled circuits by
// dropping adjacent identical Toffoli pairs and X-X pairs).  Here: any two
// multi-controlled X gates, any two SWAPs, or an INC and a DEC of one register,
// with identical targets and identical controls (mask and polarity), that are
// adjacent on their qubits: the later op's qubits (targets and controls) are
// exactly the earlier op's, and no op in between acts on any of them.  Such a
// pair is the identity.  Each qubit keeps a stack of the live ops acting on
// it, so removing a pair exposes the ops before it, and nested pairs (A B B^-1
// A^-1, the ripples of an INC followed by its DEC) cancel in turn.
bool inverse_pair(const OpInfo &a, const OpInfo &b)
{
    if (a.mask != b.mask || a.val != b.val) return false;
    if (a.kind == SV_OP_X && b.kind == SV_OP_X) return a.target == b.target;
    if (a.kind == SV_OP_SWAP && b.kind == SV_OP_SWAP)
        return (a.target == b.target && a.width == b.width) || (a.target == b.width && a.width == b.target);
    if ((a.kind == SV_OP_INC && b.kind == SV_OP_DEC) || (a.kind == SV_OP_DEC && b.kind == SV_OP_INC))
        return a.target == b.target && a.width == b.width;
    return false;
}

size_t cancel_inverse_pairs(std::vector<OpInfo> &ops)
{
    std::vector<std::vector<uint32_t>> on(64);
    std::vector<char> live(ops.size(), 1);
    size_t dropped = 0;
    for (size_t k = 0; k < ops.size(); ++k) {
        const uint64_t t = touched_qubits(ops[k]);
        long top = -2;  // the one op on top of every stack of t, -1 if none
        for (uint64_t r = t; r; r &= r - 1) {
            const int q = __builtin_ctzll(r);
            const long j = on[q].empty() ? -1 : (long)on[q].back();
            if (top == -2) top = j;
            else if (top != j) { top = -1; break; }
        }
        if (top >= 0 && touched_qubits(ops[top]) == t && inverse_pair(ops[top], ops[k])) {
            live[top] = live[k] = 0;
            for (uint64_t r = t; r; r &= r - 1) on[__builtin_ctzll(r)].pop_back();
            dropped += 2;
            continue;
        }
        for (uint64_t r = t; r; r &= r - 1) on[__builtin_ctzll(r)].push_back((uint32_t)k);
    }
    if (dropped) {
        size_t w = 0;
        for (size_t k = 0; k < ops.size(); ++k)
            if (live[k]) ops[w++] = ops[k];
        ops.resize(w);
    }
    return dropped;
}

// Hadamard-like matrices in complex64 plans.  An uncontrolled 2x2 matrix whose
// entries are 0, +-1/sqrt(2) or +-i/sqrt(2) (H, and its products with X, Z,
// S, S^dagger) becomes, rounded to FP32, the same matrix times fp32(1/sqrt 2)
// sqrt(2) = 1 - 1.7e-8: each such gate shrinks the whole state by that factor,
// always in the same direction.  The label Hadamards of every U_L call (ten
// per call) then drain the norm, and with it the post-selection probability,
// by 3.4e-7 per call: 2.4% over a ladder of 71,001 calls.  Instead, in program
// order the first of each pair stores sqrt(2) M (entries 0, +-1, +-i) and the
// second M / sqrt(2) (entries 0, +-1/2, +-i/2), all exact in FP32: each
// gate's factor is an exact global scalar, and a pair's product is 1.  The
// gates are uncontrolled, so these scalars commute with every op, and the
// planner may place the two anywhere.  An odd one out keeps its matrix.
bool hadamard_like(const OpInfo &o)
{
    if (o.kind != SV_OP_U || o.mask != 0) return false;
    bool any = false;
    for (int k = 0; k < 8; k += 2) {
        const double re = o.m[k] * std::sqrt(2.0), im = o.m[k + 1] * std::sqrt(2.0);
        const double are = std::fabs(re), aim = std::fabs(im);
        const bool re0 = are < 1e-12, im0 = aim < 1e-12;
        const bool re1 = std::fabs(are - 1.0) < 1e-12, im1 = std::fabs(aim - 1.0) < 1e-12;
        if (!((re0 && im0) || (re1 && im0) || (re0 && im1))) return false;
        any = any || !(re0 && im0);
    }
    return any;
}

int exact_hadamard_pairs(std::vector<OpInfo> &ops)
{
    std::vector<size_t> at;
    for (size_t k = 0; k < ops.size(); ++k)
        if (hadamard_like(ops[k])) at.push_back(k);
    for (size_t j = 0; j + 1 < at.size(); j += 2) {
        OpInfo &a = ops[at[j]], &b = ops[at[j + 1]];
        for (int k = 0; k < 8; ++k) {
            a.m[k] = std::round(a.m[k] * std::sqrt(2.0));         // 0, +-1
            b.m[k] = 0.5 * std::round(b.m[k] * std::sqrt(2.0));   // 0, +-1/2
        }
    }
    return (int)(at.size() / 2);
}

// Bound on how far the FP32 rounding of the plan's real 2x2 gates can move
// the norm: for each gate, the largest change of a column's squared norm when
// its entries are rounded to nearest, summed over the gates.
double real_gate_norm_bound(const std::vector<OpInfo> &ops)
{
    double sum = 0.0;
    for (const OpInfo &o : ops) {
        if (o.kind != SV_OP_U || o.m[1] != 0.0 || o.m[3] != 0.0 || o.m[5] != 0.0 || o.m[7] != 0.0) continue;
        double d = 0.0;
        for (int c = 0; c < 2; ++c) {
            const double a = o.m[2 * c], b = o.m[2 * c + 4];
            const double fa = (float)a, fb = (float)b;
            d = std::max(d, std::fabs((fa * fa + fb * fb) - (a * a + b * b)));
        }
        sum += d;
    }
    return sum;
}

// ---- dense k-qubit blocks -------------------------------------------------
// The block matrix of a run of ops whose qubits (targets and controls) lie in
// blk[0..dk-1] (ascending): column j is the run applied to the basis vector
// e_j, bit k of the index standing for qubit blk[k].
using cplx = std::complex<double>;

void apply_small(std::vector<cplx> &v, const OpInfo &o, const int *blk, int dk)
{
    auto mapbits = [&](uint64_t m) {
        uint32_t r = 0;
        for (int k = 0; k < dk; ++k)
            if ((m >> blk[k]) & 1ull) r |= 1u << k;
        return r;
    };
    auto pos = [&](int q) {
        for (int k = 0; k < dk; ++k)
            if (blk[k] == q) return k;
        return -1;
    };
    const uint32_t mask = mapbits(o.mask), val = mapbits(o.val);
    const int N = 1 << dk;
    const std::vector<cplx> in = v;
    switch (o.kind) {
    case SV_OP_U: {
        const int t = pos(o.target);
        const cplx m00(o.m[0], o.m[1]), m01(o.m[2], o.m[3]), m10(o.m[4], o.m[5]), m11(o.m[6], o.m[7]);
        for (int i = 0; i < N; ++i) {
            if ((i >> t) & 1 || (i & mask) != val) continue;
            const int i1 = i | (1 << t);
            v[i] = m00 * in[i] + m01 * in[i1];
            v[i1] = m10 * in[i] + m11 * in[i1];
        }
        break;
    }
    case SV_OP_X: {
        const int t = pos(o.target);
        for (int i = 0; i < N; ++i)
            if (!((i >> t) & 1) && (i & mask) == val) std::swap(v[i], v[i | (1 << t)]);
        break;
    }
    case SV_OP_PHASE: {
        const int t = pos(o.target);
        const cplx ph(std::cos(o.m[0]), std::sin(o.m[0]));
        for (int i = 0; i < N; ++i)
            if (((i >> t) & 1) && (i & mask) == val) v[i] *= ph;
        break;
    }
    case SV_OP_PROJPHASE: {
        const int t = pos(o.target);
        for (int i = 0; i < N; ++i) {
            const int z = (i & mask) == val, sb = (i >> t) & 1;
            const double th = o.m[0] * (1 - 2 * (sb ^ z));
            v[i] *= cplx(std::cos(th), std::sin(th));
        }
        break;
    }
    case SV_OP_INC:
    case SV_OP_DEC: {
        const int base = pos(o.target), w = (int)o.width;
        const uint32_t rm = ((1u << w) - 1u) << base;
        for (int i = 0; i < N; ++i) {
            if ((i & mask) != val) continue;
            uint32_t r = ((uint32_t)i & rm) >> base;
            r = (o.kind == SV_OP_INC ? r + 1 : r - 1) & ((1u << w) - 1u);
            v[((uint32_t)i & ~rm) | (r << base)] = in[i];
        }
        break;
    }
    case SV_OP_SWAP: {
        const int a = pos(o.target), b = pos((int)o.width);
        for (int i = 0; i < N; ++i) {
            if ((i & mask) != val) continue;
            const int j = ((((i >> a) ^ (i >> b)) & 1) ? i ^ ((1 << a) | (1 << b)) : i);
            v[j] = in[i];
        }
        break;
    }
    default:
        break;
    }
}

}  // namespace

int build_plan(sv_plan *p, const sv_op *ops, size_t n_ops, const double *params, const sv_apply_opts &opts,
               std::string &err)
{
    const int n = p->n;
    const int esize = p->dtype == SV_C64 ? 8 : 16;
    std::vector<OpInfo> info(n_ops);
    for (size_t k = 0; k < n_ops; ++k) info[k] = normalize(ops[k], params);

    p->info = sv_plan_info{};
    p->info.n_ops = n_ops;

    // ---- tile geometry ----
    int rb = opts.reg_qubits ? opts.reg_qubits : 4;
    int b = opts.tile_qubits ? opts.tile_qubits : (p->dtype == SV_C64 ? 12 : 12);
    bool fused = opts.mode == SV_MODE_FUSED;
    if (fused) {
        if (rb < 4 || rb > kMaxRB) {
            err = "reg_qubits must be 4 or 5";
            return SV_EINVAL;
        }
        if (b > n) b = n;
        if (b > kMaxB || (size_t)esize << b > 160 * 1024) {
            err = "tile_qubits too large for LDS";
            return SV_EINVAL;
        }
        // 512 threads (nine thread bits) only as compiled passes: the generic
        // tile kernels are built for at most 256
        if (b - rb > 9 || (b - rb == 9 && opts.compile == SV_COMPILE_OFF)) {
            err = "tile_qubits - reg_qubits must be at most 8 (256 threads), or 9 (512) with compiled passes";
            return SV_EINVAL;
        }
        if (b - rb < 6) fused = false;  // fewer than 64 threads: use plain launches
        if (n - b > 48) {
            err = "too many tile qubits";
            return SV_EUNSUPPORTED;
        }
    }
    if (opts.coalesce_qubits < 0 || opts.coalesce_qubits > 8) {
        err = "coalesce_qubits must be 0 (automatic) or 1 to 8";
        return SV_EINVAL;
    }
    if (opts.split_real < SV_SPLIT_REAL_AUTO || opts.split_real > SV_SPLIT_REAL_ON) {
        err = "split_real must be SV_SPLIT_REAL_AUTO, _OFF or _ON";
        return SV_EINVAL;
    }
    if (opts.dense_qubits != 0 && opts.dense_qubits != 5 && opts.dense_qubits != 6) {
        err = "dense_qubits must be 0, 5 or 6";
        return SV_EINVAL;
    }
    if (opts.dense_qubits == 6 && p->dtype != SV_C64) {
        err = "six-qubit dense blocks are complex64 only";
        return SV_EUNSUPPORTED;
    }
    p->dense_k = opts.dense_qubits == 6 ? 6 : 5;
    p->b = fused ? b : 0;
    p->rb = fused ? rb : 0;
    p->info.tile_qubits = p->b;
    p->info.reg_qubits = p->rb;

    p->steps.clear();
    p->plain.clear();
    p->passes.clear();
    p->stages.clear();
    p->tops.clear();
    p->tparams.clear();
    p->dense.clear();
    p->dparams.clear();

    auto add_plain = [&](const OpInfo &o) {
        p->steps.push_back(Step{0, (uint32_t)p->plain.size()});
        p->plain.push_back(to_plain(o));
        p->info.bytes_moved += plain_bytes(o, n, esize);
        p->info.touched_bytes += touched_bytes(o, n, esize);
    };

    const bool peephole = opts.peephole == SV_PEEPHOLE_ON || (opts.peephole == SV_PEEPHOLE_AUTO && fused);
    if (peephole) {
        p->info.n_cancelled_ops = cancel_inverse_pairs(info);
        n_ops = info.size();
    }

    if (!fused) {
        if (p->dtype == SV_C64) exact_hadamard_pairs(info);
        for (size_t k = 0; k < n_ops; ++k) add_plain(info[k]);
        p->info.n_launches = p->steps.size();
        return SV_OK;
    }

    // single-qubit runs are folded on the host before grouping (fused mode only:
    // the per-gate path stays one launch per IR op)
    info = fold_single_qubit_runs(info);
    n_ops = info.size();
    if (p->dtype == SV_C64) exact_hadamard_pairs(info);
    const bool split_real = p->dtype == SV_C64 &&
                            (opts.split_real == SV_SPLIT_REAL_ON ||
                             (opts.split_real == SV_SPLIT_REAL_AUTO && real_gate_norm_bound(info) > kSplitRealBound));

    const int nthr = b - rb;
    // lowest qubits resident in every pass (each tile's runs of contiguous
    // amplitudes): 256 bytes by default; fewer leave more room for other qubits
    const int L0 = std::min(nthr, opts.coalesce_qubits ? opts.coalesce_qubits : (p->dtype == SV_C64 ? 5 : 4));
    const int lowb = 4;  // LDS swizzle width: 8-byte elements (a complex64, or half a complex128)
    const uint64_t lowmask = (1ull << L0) - 1ull;
    const size_t W = 1024;
    const bool plain_split = opts.plain_split != SV_PLAIN_SPLIT_OFF;
    // resident-set lookahead for states whose passes are bound by HBM sweeps
    // (planning cost grows by the candidates times the window per widening)
    const bool lookahead = n >= 24;
    // two steps (pairs of widenings) while the planning cost stays small
    const bool lookahead2 = lookahead && n_ops <= 200000;
    // X gates as flips of their local bit on exchanges that apply permutations
    const bool x_flips = true;

    // ---- dense k-qubit runs: maximal runs of consecutive ops whose qubits fit
    // in k (5, or 6 for complex64), kept when at least dense_min_ops long ----
    const int dk = p->dense_k;
    std::vector<int> dense_id(n_ops, -1);
    std::vector<std::pair<size_t, size_t>> runs;
    std::vector<uint64_t> run_support;
    // automatic (negative dense_min_ops): a run becomes a block when its ops
    // inside tile passes (each read by every tile and applied to the
    // amplitudes it touches) are modelled dearer than one dense pass
    int dense_min = opts.dense_min_ops;
    if (dense_min < 0) {
        double dense_us = kDenseFixedUs + (double)(2ull << n) * esize / kDenseBytesPerUs;
        // six-qubit blocks on FP32 matrix cores: 512 flop per amplitude, bound by the products
        if (dk == 6 && !p->dense_bf16)
            dense_us = std::max(dense_us, kDenseFixedUs + (double)(1ull << n) * 512.0 / kDenseFp32FlopPerUs);
        const double op_us = kOpPerTileUs * (double)(1ull << (n > b ? n - b : 0)) + kOpPerAmpUs * (double)(1ull << n);
        dense_min = (int)std::min(1e6, std::ceil(dense_us / op_us));
    }
    p->info.dense_min_ops = dense_min;
    if (dense_min > 0 && n >= 12) {
        size_t ws = 0;
        uint64_t S = 0;
        auto close = [&](size_t end) {
            if (end - ws >= (size_t)dense_min && S) {
                for (size_t k = ws; k < end; ++k) dense_id[k] = (int)runs.size();
                runs.emplace_back(ws, end);
                run_support.push_back(S);
            }
        };
        for (size_t i = 0; i < n_ops; ++i) {
            const uint64_t T = touched_qubits(info[i]);
            if (__builtin_popcountll(S | T) <= dk) {
                S |= T;
                continue;
            }
            close(i);
            ws = i;
            S = __builtin_popcountll(T) <= dk ? T : 0;
            if (!S) ws = i + 1;  // an op wider than a block starts no run
        }
        close(n_ops);
    }
    auto emit_dense = [&](int rid) {
        const uint64_t S = run_support[rid];
        int blk[kMaxDenseK];
        {
            uint64_t B = S;
            for (int q = 0; q < n && __builtin_popcountll(B) < dk; ++q) B |= 1ull << q;
            int k = 0;
            for (int q = 0; q < n; ++q)
                if ((B >> q) & 1ull) blk[k++] = q;
        }
        uint64_t R = 0;
        for (int k = 0; k < dk; ++k) R |= 1ull << blk[k];
        for (int q = 0; q < n && __builtin_popcountll(R) < 12; ++q) R |= 1ull << q;
        DensePass D{};
        D.k = (uint32_t)dk;
        TilePass &P = D.map;
        P.b = 12;
        P.rb = 4;
        P.nthr = 8;
        P.ntile = (uint8_t)(n - 12);
        int lpos[64];
        for (int q = 0; q < 64; ++q) lpos[q] = -1;
        {
            int k = 0, t = 0;
            for (int q = 0; q < n; ++q) {
                if ((R >> q) & 1ull) {
                    P.spos[k] = (uint8_t)q;
                    lpos[q] = k++;
                } else {
                    P.tpos[t++] = (uint8_t)q;
                }
            }
        }
        const int dl = p->dtype == SV_C64 ? 4 : 3;  // LDS swizzle width of the amplitude size
        for (int s2 = 0; s2 < 16; ++s2) {
            uint64_t off = 0;
            for (int k = 0; k < 4; ++k)
                if ((s2 >> k) & 1) off |= 1ull << P.spos[8 + k];
            P.goff[s2] = off;
            P.swz0[s2] = lds_swizzle((uint32_t)s2 << 8, dl);
        }
        P.n_tile_runs = (uint32_t)bit_runs(P.tpos, P.ntile, [&](int src, int dst, int w) {
            const int r = (int)P.n_tile_runs++;
            P.tile_shift[r] = (uint32_t)src | ((uint32_t)dst << 8);
            P.tile_mask[r] = (w >= 64) ? ~0ull : ((1ull << w) - 1ull);
        });
        P.n_gthr_runs = (uint32_t)bit_runs(P.spos, 8, [&](int src, int dst, int w) {
            const int r = (int)P.n_gthr_runs++;
            P.gthr_shift[r] = (uint32_t)src | ((uint32_t)dst << 8);
            P.gthr_mask[r] = (1u << w) - 1u;
        });
        const int N = 1 << dk;
        for (int j = 0; j < N; ++j) {
            uint32_t off = 0;
            for (int k = 0; k < dk; ++k)
                if ((j >> k) & 1) off |= 1u << lpos[blk[k]];
            D.joff[j] = off;
        }
        uint8_t nb[8];
        {
            int c = 0;
            for (int l = 0; l < 12; ++l) {
                bool inblk = false;
                for (int k = 0; k < dk; ++k) inblk = inblk || lpos[blk[k]] == l;
                if (!inblk) nb[c++] = (uint8_t)l;
            }
        }
        D.n_grp_runs = 0;
        bit_runs(nb, 12 - dk, [&](int src, int dst, int w) {
            D.grp_run[D.n_grp_runs++] = pack_run16((uint32_t)src, (uint32_t)dst, (1u << w) - 1u);
        });
        // the block matrix, column by column
        D.mat = (uint32_t)p->dparams.size();
        p->dparams.resize(p->dparams.size() + 2 * (size_t)N * N, 0.0);
        for (int j = 0; j < N; ++j) {
            std::vector<cplx> v(N, cplx(0.0, 0.0));
            v[j] = 1.0;
            for (size_t k = runs[rid].first; k < runs[rid].second; ++k) apply_small(v, info[k], blk, dk);
            for (int i = 0; i < N; ++i) {
                p->dparams[D.mat + 2 * (N * i + j)] = v[i].real();
                p->dparams[D.mat + 2 * (N * i + j) + 1] = v[i].imag();
            }
        }
        p->steps.push_back(Step{2, (uint32_t)p->dense.size()});
        p->dense.push_back(D);
        p->info.n_dense_passes += 1;
        p->info.n_dense_ops += runs[rid].second - runs[rid].first;
        p->info.bytes_moved += 2ull * (1ull << n) * esize;
        p->info.touched_bytes += 2ull * (1ull << n) * esize;
    };

    std::vector<char> done(n_ops, 0);
    size_t first = 0;
    while (true) {
        while (first < n_ops && done[first]) ++first;
        if (first >= n_ops) break;
        if (dense_id[first] >= 0) {  // every earlier op is done: the block goes now
            const int rid = dense_id[first];
            emit_dense(rid);
            for (size_t k = runs[rid].first; k < runs[rid].second; ++k) done[k] = 1;
            continue;
        }
        if (__builtin_popcountll(info[first].req | lowmask) > b) {
            // cannot be made resident: its own launch (all earlier ops are done)
            add_plain(info[first]);
            done[first] = 1;
            continue;
        }
        PassBuild pb;
        pb.S = lowmask;
        const size_t wend = std::min(n_ops, first + W);
        // Once every qubit is blocked (acted on non-diagonally by a skipped op,
        // or both an X target and diagonal in skipped ops), no later op of the
        // window commutes with all skipped ones: every op touches a qubit, and
        // commutes_with_all fails on any blocked qubit.  The scans stop there.
        const uint64_t allq = n >= 64 ? ~0ull : (1ull << n) - 1ull;
        auto all_blocked = [&](uint64_t Z, uint64_t X, uint64_t G) { return ((G | (X & Z)) & allq) == allq; };
        // ops of the window that a resident set S would let into the pass now
        auto gain = [&](uint64_t S) {
            uint64_t Z = 0, X = 0, G = 0;
            int cnt = 0;
            for (size_t j = first; j < wend; ++j) {
                if (done[j]) continue;
                const OpInfo &o = info[j];
                if (dense_id[j] < 0 && (o.req & ~S) == 0 && commutes_with_all(o, Z, X, G)) {
                    ++cnt;
                    continue;
                }
                Z |= o.z;
                X |= o.x;
                G |= o.g;
                if (all_blocked(Z, X, G)) break;
            }
            return cnt;
        };
        while (true) {
            uint64_t Z = 0, X = 0, G = 0;
            long cand = -1;
            uint64_t alt[kLookahead];
            int n_alt = 0;
            for (size_t j = first; j < wend; ++j) {
                if (done[j]) continue;
                const OpInfo &o = info[j];
                if (dense_id[j] >= 0) {  // belongs to a dense block: never taken, blocks what it touches
                    Z |= o.z;
                    X |= o.x;
                    G |= o.g;
                    continue;
                }
                const bool ready = commutes_with_all(o, Z, X, G);
                if (ready && (o.req & ~pb.S) == 0) {
                    done[j] = 1;
                    pb.ops.push_back((uint32_t)j);
                    continue;
                }
                if (ready && __builtin_popcountll(pb.S | o.req) <= b) {
                    if (cand < 0) cand = (long)j;
                    const uint64_t m = o.req & ~pb.S;
                    bool seen = false;
                    for (int a = 0; a < n_alt; ++a) seen = seen || alt[a] == m;
                    if (!seen && n_alt < kLookahead) alt[n_alt++] = m;
                }
                Z |= o.z;
                X |= o.x;
                G |= o.g;
                if (all_blocked(Z, X, G)) break;
            }
            if (cand < 0) break;
            if (lookahead && n_alt > 1) {
                // widen the resident set by the candidate that admits the most ops
                // per added qubit, alone or followed by a second candidate
                double best = -1.0;
                uint64_t pick = alt[0];
                for (int a = 0; a < n_alt; ++a) {
                    double v = (double)gain(pb.S | alt[a]) / (double)__builtin_popcountll(alt[a]);
                    for (int c = 0; c < (lookahead2 ? n_alt : 0); ++c) {
                        const uint64_t u = alt[a] | alt[c];
                        if (c == a || __builtin_popcountll(pb.S | u) > b) continue;
                        const double v2 = (double)gain(pb.S | u) / (double)__builtin_popcountll(u);
                        if (v2 > v) v = v2;
                    }
                    if (v > best) {
                        best = v;
                        pick = alt[a];
                    }
                }
                pb.S |= pick;
            } else {
                pb.S |= info[cand].req;
            }
        }
        // Ops cheaper as plain launches (each sweeps only its controlled
        // subspace) than inside the pass leave it: to the front when they
        // commute with every op kept before them, else to the back when they
        // commute with every op kept after them.  If what remains is cheaper
        // as plain launches than one pass over the state, the pass goes too.
        std::vector<uint32_t> tail_plain;
        if (plain_split) {
            const double tile_us = kTileFixedUs + (double)(2ull * (1ull << n) * esize) / kTileBytesPerUs;
            const double tiles = (double)(1ull << (n - b));
            auto leaves = [&](const OpInfo &o) {
                // inside the pass every tile walks the op record, and the tiles
                // meeting the op's non-resident controls do its arithmetic
                const int g = __builtin_popcountll(o.mask & ~pb.S);
                const double in_pass = kOpPerTileUs * tiles + kOpPerAmpUs * (double)(1ull << (n - g));
                return plain_us(o, n, esize) < in_pass;
            };
            std::vector<uint32_t> front, keep, back, kept;
            uint64_t Z = 0, X = 0, G = 0;
            for (uint32_t j : pb.ops) {
                const OpInfo &o = info[j];
                if (leaves(o) && commutes_with_all(o, Z, X, G)) {
                    front.push_back(j);
                    continue;
                }
                keep.push_back(j);
                Z |= o.z;
                X |= o.x;
                G |= o.g;
            }
            Z = X = G = 0;
            for (size_t i = keep.size(); i-- > 0;) {
                const OpInfo &o = info[keep[i]];
                if (leaves(o) && commutes_with_all(o, Z, X, G)) {
                    back.push_back(keep[i]);
                    continue;
                }
                kept.push_back(keep[i]);
                Z |= o.z;
                X |= o.x;
                G |= o.g;
            }
            std::reverse(kept.begin(), kept.end());
            std::reverse(back.begin(), back.end());
            for (uint32_t j : front) add_plain(info[j]);
            p->info.n_split_ops += front.size() + back.size();
            double t = 0.0;
            for (uint32_t j : kept) t += plain_us(info[j], n, esize);
            if (kept.empty() || t < tile_us) {
                for (uint32_t j : kept) add_plain(info[j]);
                for (uint32_t j : back) add_plain(info[j]);
                p->info.n_split_ops += kept.size();
                continue;
            }
            pb.ops = kept;
            tail_plain = back;
        }
        // fill the resident set up to b qubits with the lowest unused ones
        for (int q = 0; q < n && __builtin_popcountll(pb.S) < b; ++q) pb.S |= 1ull << q;

        // ---- lay out the pass ----
        TilePass P{};
        P.n_tile_runs = 0;
        P.n_gthr_runs = 0;
        P.b = (uint8_t)b;
        P.rb = (uint8_t)rb;
        P.nthr = (uint8_t)nthr;
        P.ntile = (uint8_t)(n - b);
        // Commutation dependences inside the pass: op i follows every earlier op
        // of the pass it does not commute with.
        const size_t m = pb.ops.size();
        std::vector<std::vector<uint32_t>> pred(m);
        for (size_t i = 0; i < m; ++i) {
            const OpInfo &oi = info[pb.ops[i]];
            for (size_t j = 0; j < i; ++j) {
                const OpInfo &oj = info[pb.ops[j]];
                if (!commutes_with_all(oi, oj.z, oj.x, oj.g)) pred[i].push_back((uint32_t)j);
            }
        }
        std::vector<char> placed(m, 0);
        auto ready = [&](size_t i) {
            for (uint32_t j : pred[i])
                if (!placed[j]) return false;
            return true;
        };
        auto reg_kind = [](uint32_t k) { return k == SV_OP_U || k == SV_OP_X; };
        auto perm_kind = [](uint32_t k) { return k == SV_OP_INC || k == SV_OP_DEC || k == SV_OP_SWAP; };
        // Register qubits for the next stage: among `allowed`, the targets of the
        // most ready register ops (earlier first on ties), then those of `keep`,
        // then the highest allowed qubits.
        auto pick_regs = [&](uint64_t allowed, uint64_t keep) {
            int cnt[64] = {0}, first_at[64];
            for (int q = 0; q < 64; ++q) first_at[q] = 1 << 30;
            for (size_t i = 0; i < m; ++i) {
                if (placed[i] || !ready(i)) continue;
                const OpInfo &o = info[pb.ops[i]];
                if (!reg_kind(o.kind) || !((allowed >> o.target) & 1ull)) continue;
                cnt[o.target]++;
                first_at[o.target] = std::min(first_at[o.target], (int)i);
            }
            uint64_t r = 0;
            int c = 0;
            while (c < rb) {
                int best = -1;
                for (int q = 0; q < n; ++q)
                    if (cnt[q] > 0 && !((r >> q) & 1ull) &&
                        (best < 0 || cnt[q] > cnt[best] || (cnt[q] == cnt[best] && first_at[q] < first_at[best])))
                        best = q;
                if (best < 0) break;
                r |= 1ull << best;
                ++c;
            }
            for (int q = 0; q < n && c < rb; ++q)
                if (((keep & allowed) >> q & 1ull) && !((r >> q) & 1ull)) {
                    r |= 1ull << q;
                    ++c;
                }
            for (int q = n - 1; q >= 0 && c < rb; --q)
                if (((allowed >> q) & 1ull) && !((r >> q) & 1ull)) {
                    r |= 1ull << q;
                    ++c;
                }
            return r;
        };
        // Local bit order: the other resident qubits ascending (the lowest ones
        // first, so the load stays coalesced), then the first stage's registers.
        // Qubits of an incremented register stay out of the first registers, so
        // that every such register keeps consecutive local bits.
        uint64_t shifted = 0;
        for (uint32_t j : pb.ops)
            if (info[j].kind == SV_OP_INC || info[j].kind == SV_OP_DEC) shifted |= info[j].req;
        uint64_t init_regs = pick_regs(pb.S & ~lowmask & ~shifted, 0);
        if (__builtin_popcountll(init_regs) < rb) {  // too few free qubits: the highest ones, in order
            init_regs = 0;
            for (int q = n - 1, c = 0; q >= 0 && c < rb; --q)
                if ((pb.S >> q) & 1ull) {
                    init_regs |= 1ull << q;
                    ++c;
                }
        }
        int lpos[64];
        for (int q = 0; q < 64; ++q) lpos[q] = -1;
        {
            int k = 0, t = 0;
            for (int q = 0; q < n; ++q) {
                if (((pb.S >> q) & 1ull) && !((init_regs >> q) & 1ull)) {
                    P.spos[k] = (uint8_t)q;
                    lpos[q] = k++;
                } else if (!((pb.S >> q) & 1ull)) {
                    P.tpos[t++] = (uint8_t)q;
                }
            }
            for (int q = 0; q < n; ++q)
                if ((init_regs >> q) & 1ull) {
                    P.spos[k] = (uint8_t)q;
                    lpos[q] = k++;
                }
        }
        // Order the pass's ops for few register stages (list scheduling): an op
        // whose predecessors are placed runs as soon as its target is in the
        // current register set, and diagonal ops run in any stage.  When nothing
        // more fits, the ready permutations are placed (they ride on the
        // exchange) and the next register set is picked as above.
        {
            std::vector<uint32_t> order;
            order.reserve(m);
            uint64_t regs = init_regs;
            size_t left = m;
            while (left) {
                const size_t left_before = left;
                for (bool progress = true; progress;) {
                    progress = false;
                    for (size_t i = 0; i < m; ++i) {
                        if (placed[i] || !ready(i)) continue;
                        const OpInfo &o = info[pb.ops[i]];
                        if (perm_kind(o.kind) || (reg_kind(o.kind) && !((regs >> o.target) & 1ull))) continue;
                        // (an X whose target is a register runs in the stage; otherwise it
                        // waits for the exchange and flips its local bit there)
                        placed[i] = 1;
                        order.push_back(pb.ops[i]);
                        --left;
                        progress = true;
                    }
                }
                if (!left) break;
                // X gates ride along (as flips of their local bit) only on an
                // exchange that applies other permutations anyway
                bool perms_here = false;
                for (bool progress = true; progress;) {
                    progress = false;
                    for (size_t i = 0; i < m; ++i) {
                        if (placed[i] || !ready(i) || !perm_kind(info[pb.ops[i]].kind)) continue;
                        perms_here = true;
                        placed[i] = 1;
                        order.push_back(pb.ops[i]);
                        --left;
                        progress = true;
                    }
                }
                uint64_t next_regs = pick_regs(pb.S, regs);
                // X gates whose targets miss the next registers ride along (as flips of
                // their local bit) on an exchange that applies other permutations anyway
                for (bool progress = perms_here && x_flips; progress;) {
                    progress = false;
                    for (size_t i = 0; i < m; ++i) {
                        if (placed[i] || !ready(i)) continue;
                        const OpInfo &o = info[pb.ops[i]];
                        if (o.kind != SV_OP_X && !perm_kind(o.kind)) continue;
                        if (o.kind == SV_OP_X && ((next_regs >> o.target) & 1ull)) continue;
                        placed[i] = 1;
                        order.push_back(pb.ops[i]);
                        --left;
                        progress = true;
                    }
                    if (progress) next_regs = pick_regs(pb.S, regs);
                }
                if (left == left_before && next_regs == regs) {
                    // nothing placed and nothing will change: take the first ready op
                    // as it comes (the emission below accepts any order)
                    for (size_t i = 0; i < m; ++i)
                        if (!placed[i] && ready(i)) {
                            placed[i] = 1;
                            order.push_back(pb.ops[i]);
                            --left;
                            break;
                        }
                }
                regs = next_regs;
            }
            pb.ops = order;
        }
        for (int s = 0; s < (1 << rb); ++s) {
            uint64_t off = 0;
            for (int k = 0; k < rb; ++k)
                if ((s >> k) & 1) off |= 1ull << P.spos[nthr + k];
            P.goff[s] = off;
            P.swz0[s] = lds_swizzle((uint32_t)s << nthr, lowb);
        }
        P.n_tile_runs = (uint32_t)bit_runs(P.tpos, P.ntile, [&](int src, int dst, int w) {
            const int r = (int)P.n_tile_runs++;
            P.tile_shift[r] = (uint32_t)src | ((uint32_t)dst << 8);
            P.tile_mask[r] = (w >= 64) ? ~0ull : ((1ull << w) - 1ull);
        });
        P.n_gthr_runs = (uint32_t)bit_runs(P.spos, nthr, [&](int src, int dst, int w) {
            const int r = (int)P.n_gthr_runs++;
            P.gthr_shift[r] = (uint32_t)src | ((uint32_t)dst << 8);
            P.gthr_mask[r] = (1u << w) - 1u;
        });
        auto split = [&](uint64_t mask, uint64_t val, TileOp &t) {
            t.lmask = 0;
            t.lval = 0;
            for (int q = 0; q < n; ++q) {
                if (!((mask >> q) & 1ull) || !((pb.S >> q) & 1ull)) continue;
                t.lmask |= 1u << lpos[q];
                if ((val >> q) & 1ull) t.lval |= 1u << lpos[q];
            }
            t.gmask = mask & ~pb.S;
            t.gval = val & ~pb.S;
        };

        // register sets: slot k <-> local bit rs[k]
        std::vector<int> cur_rs(rb);
        for (int k = 0; k < rb; ++k) cur_rs[k] = nthr + k;
        auto open_stage = [&](const std::vector<int> &rs, uint32_t perm_b, uint32_t perm_e) {
            TileStage S{};
            S.op_begin = S.op_end = (uint32_t)p->tops.size();
            S.perm_begin = perm_b;
            S.perm_end = perm_e;
            std::vector<char> isreg(b, 0);
            for (int k = 0; k < rb; ++k) isreg[rs[k]] = 1;
            int j = 0;
            for (int l = 0; l < b; ++l)
                if (!isreg[l]) S.thrpos[j++] = (uint8_t)l;
            for (int s = 0; s < (1 << rb); ++s) {
                uint32_t off = 0;
                for (int k = 0; k < rb; ++k)
                    if ((s >> k) & 1) off |= 1u << rs[k];
                S.regoff[s] = (uint32_t)off;
                S.swz[s] = lds_swizzle(off, lowb);
            }
            S.n_thr_runs = 0;
            bit_runs(S.thrpos, nthr, [&](int src, int dst, int w) {
                S.thr_run[S.n_thr_runs++] = pack_run16((uint32_t)src, (uint32_t)dst, (1u << w) - 1u);
            });
            p->stages.push_back(S);
        };
        auto is_reg_kind = [&](uint32_t k) { return k == SV_OP_U || k == SV_OP_X; };
        auto is_perm_kind = [&](uint32_t k) { return k == SV_OP_INC || k == SV_OP_DEC || k == SV_OP_SWAP; };
        // parameters of the op about to be appended to tops live at a fixed stride
        // (kParamStride reals per tops entry), so the kernel can fetch them without
        // first reading the op record
        auto put_params = [&](const double *v, int cnt) {
            const size_t at = p->tops.size() * kParamStride;
            if (p->tparams.size() < at + kParamStride) p->tparams.resize(at + kParamStride, 0.0);
            for (int k = 0; k < cnt; ++k) p->tparams[at + k] = v[k];
            return (uint32_t)at;
        };

        P.stage_begin = (uint32_t)p->stages.size();
        // perms are collected in a side list and copied into tops when a stage opens
        std::vector<TileOp> pending;
        open_stage(cur_rs, 0, 0);
        auto flush_into_new_stage = [&](const std::vector<int> &rs) {
            // close current stage's op range, then append pending perms and open the next stage
            p->stages.back().op_end = (uint32_t)p->tops.size();
            const uint32_t pbeg = (uint32_t)p->tops.size();
            for (auto &t : pending) p->tops.push_back(t);
            const uint32_t pend = (uint32_t)p->tops.size();
            pending.clear();
            open_stage(rs, pbeg, pend);
            cur_rs = rs;
        };
        auto choose_rs = [&](size_t from) {
            std::vector<int> rs;
            for (size_t i = from; i < pb.ops.size() && (int)rs.size() < rb; ++i) {
                const OpInfo &o = info[pb.ops[i]];
                if (is_perm_kind(o.kind)) break;
                if (!is_reg_kind(o.kind)) continue;
                const int l = lpos[o.target];
                if (std::find(rs.begin(), rs.end(), l) == rs.end()) rs.push_back(l);
            }
            for (int k = 0; k < rb && (int)rs.size() < rb; ++k)
                if (std::find(rs.begin(), rs.end(), cur_rs[k]) == rs.end()) rs.push_back(cur_rs[k]);
            for (int l = 0; l < b && (int)rs.size() < rb; ++l)
                if (std::find(rs.begin(), rs.end(), l) == rs.end()) rs.push_back(l);
            std::sort(rs.begin(), rs.end());
            return rs;
        };

        // split a local condition (t.lmask, t.lval) for the current stage into the
        // register-slot part (slotmask over all 2^rb slots) and the thread part
        auto stage_split = [&](TileOp &t) {
            const TileStage &S = p->stages.back();
            uint32_t regbits = 0;
            for (int k = 0; k < rb; ++k) regbits |= 1u << cur_rs[k];
            const uint32_t rm = t.lmask & regbits;
            t.slotmask = 0;
            for (int s = 0; s < (1 << rb); ++s)
                if ((S.regoff[s] & rm) == (t.lval & rm)) t.slotmask |= 1u << s;
            t.tidmask = 0;
            t.tidval = 0;
            for (int j = 0; j < nthr; ++j) {
                const uint32_t bit = 1u << S.thrpos[j];
                if (t.lmask & bit) {
                    t.tidmask |= (uint16_t)(1u << j);
                    if (t.lval & bit) t.tidval |= (uint16_t)(1u << j);
                }
            }
        };
        for (size_t i = 0; i < pb.ops.size(); ++i) {
            const OpInfo &o = info[pb.ops[i]];
            TileOp t{};
            const bool x_flip = x_flips && o.kind == SV_OP_X && !pending.empty();
            if (x_flip) {  // a flip of the target's local bit, applied on the next exchange
                split(o.mask, o.val, t);
                t.kind = T_XFLIP;
                t.a = (uint8_t)lpos[o.target];
                pending.push_back(t);
                continue;
            }
            if (is_perm_kind(o.kind)) {
                split(o.mask, o.val, t);
                if (o.kind == SV_OP_SWAP) {
                    t.kind = T_SWAP;
                    t.a = (uint8_t)lpos[o.target];
                    t.b = (uint8_t)lpos[o.width];
                } else {
                    t.kind = o.kind == SV_OP_INC ? T_INC : T_DEC;
                    t.a = (uint8_t)lpos[o.target];
                    t.b = (uint8_t)o.width;
                }
                pending.push_back(t);
                continue;
            }
            if (is_reg_kind(o.kind)) {
                const int l = lpos[o.target];
                auto it = std::find(cur_rs.begin(), cur_rs.end(), l);
                if (it == cur_rs.end() || !pending.empty()) {
                    flush_into_new_stage(it == cur_rs.end() ? choose_rs(i) : cur_rs);
                    it = std::find(cur_rs.begin(), cur_rs.end(), l);
                }
                split(o.mask, o.val, t);
                stage_split(t);
                t.slot = (uint8_t)(it - cur_rs.begin());
                if (o.kind == SV_OP_U) {
                    const bool real = o.m[1] == 0.0 && o.m[3] == 0.0 && o.m[5] == 0.0 && o.m[7] == 0.0;
                    t.kind = real ? (split_real ? T_UR2 : T_UR) : T_U;
                    double v[8];
                    if (real) {
                        for (int k = 0; k < 4; ++k) v[k] = o.m[2 * k];
                    } else {
                        for (int k = 0; k < 8; ++k) v[k] = o.m[k];
                    }
                    t.param = put_params(v, real ? 4 : 8);
                } else {
                    t.kind = T_X;
                    t.param = put_params(nullptr, 0);
                }
                p->tops.push_back(t);
                continue;
            }
            // diagonal ops (after pending permutations, the new stage already takes
            // the registers the following ops need)
            if (!pending.empty()) flush_into_new_stage(choose_rs(i));
            if (o.kind == SV_OP_PHASE) {
                split(o.mask | (1ull << o.target), o.val | (1ull << o.target), t);
                t.kind = T_PHASE;
            } else {  // PROJPHASE
                split(o.mask, o.val, t);
                t.kind = T_PROJ;
                if (!((pb.S >> o.target) & 1ull)) {
                    t.a = 0;
                    t.b = (uint8_t)o.target;
                } else {
                    const int l = lpos[o.target];
                    auto it = std::find(cur_rs.begin(), cur_rs.end(), l);
                    if (it != cur_rs.end()) {
                        t.a = 1;
                        t.b = (uint8_t)(it - cur_rs.begin());
                    } else {
                        const TileStage &S = p->stages.back();
                        t.a = 2;
                        for (int j = 0; j < nthr; ++j)
                            if (S.thrpos[j] == l) t.b = (uint8_t)j;
                    }
                }
            }
            stage_split(t);
            const double cs[2] = {std::cos(o.m[0]), std::sin(o.m[0])};
            t.param = put_params(cs, 2);
            p->tops.push_back(t);
        }
        p->stages.back().op_end = (uint32_t)p->tops.size();
        P.stage_end = (uint32_t)p->stages.size();
        bool at_load_mapping = true;
        for (int k = 0; k < rb; ++k) at_load_mapping = at_load_mapping && cur_rs[k] == nthr + k;
        P.fperm_begin = (uint32_t)p->tops.size();
        for (auto &t : pending) p->tops.push_back(t);
        P.fperm_end = (uint32_t)p->tops.size();
        P.final_exchange = (!at_load_mapping || !pending.empty()) ? 1 : 0;
        P.stream = stream_state_bytes((p->dtype == SV_C64 ? 8ull : 16ull) << n) ? 1 : 0;
        pending.clear();

        p->steps.push_back(Step{1, (uint32_t)p->passes.size()});
        p->passes.push_back(P);
        p->info.n_tile_passes += 1;
        p->info.n_stages += P.stage_end - P.stage_begin;
        p->info.bytes_moved += 2ull * (1ull << n) * esize;
        p->info.touched_bytes += 2ull * (1ull << n) * esize;
        for (uint32_t j : tail_plain) add_plain(info[j]);
    }
    p->tparams.resize(p->tops.size() * kParamStride, 0.0);
    // Gate runs: within a stage, maximal runs of consecutive ops (no T_PROJ)
    // with one nonzero tile mask are sorted by tile value (stable, parameters
    // moved along) and their first op records the run length.  Used from 21
    // qubits up: the run kernel reads op records without the one-ahead
    // prefetch, which on the short passes of smaller states costs more than
    // the bisection saves (measured 6% slower at 19 qubits).
    for (TilePass &P : p->passes) {
        if (n < 21) break;
        for (uint32_t st = P.stage_begin; st < P.stage_end; ++st) {
            const TileStage &S = p->stages[st];
            uint32_t k = S.op_begin;
            while (k < S.op_end) {
                const TileOp &h = p->tops[k];
                uint32_t e = k + 1;
                if (h.kind != T_PROJ && h.gmask != 0)
                    while (e < S.op_end && p->tops[e].kind != T_PROJ && p->tops[e].gmask == h.gmask && e - k < 0xffffu) ++e;
                const uint32_t L = e - k;
                if (L >= (uint32_t)kMinGateRun) {
                    std::vector<uint32_t> idx(L);
                    for (uint32_t i = 0; i < L; ++i) idx[i] = k + i;
                    std::stable_sort(idx.begin(), idx.end(),
                                     [&](uint32_t a, uint32_t b) { return p->tops[a].gval < p->tops[b].gval; });
                    std::vector<TileOp> ro(L);
                    std::vector<double> rp((size_t)L * kParamStride);
                    for (uint32_t i = 0; i < L; ++i) {
                        ro[i] = p->tops[idx[i]];
                        for (int j = 0; j < kParamStride; ++j)
                            rp[(size_t)i * kParamStride + j] = p->tparams[(size_t)idx[i] * kParamStride + j];
                    }
                    for (uint32_t i = 0; i < L; ++i) {
                        TileOp t = ro[i];
                        t.param = (k + i) * (uint32_t)kParamStride;
                        t.a = i == 0 ? (uint8_t)(L & 0xffu) : 0;
                        t.b = i == 0 ? (uint8_t)(L >> 8) : 0;
                        p->tops[k + i] = t;
                        for (int j = 0; j < kParamStride; ++j)
                            p->tparams[(size_t)(k + i) * kParamStride + j] = rp[(size_t)i * kParamStride + j];
                    }
                    P.gate_runs = 1;
                }
                k = e;
            }
        }
    }
    p->info.tile_pass_bytes = 2ull * (1ull << n) * esize;
    p->info.n_launches = p->steps.size();
    return SV_OK;
}

// A projector phase multiplies every amplitude by c + i s or c - i s (the QSVT
// phase rotations of Sec. II.D.5), so with (cos, sin) rounded to FP32 it
// scales the norm of the whole state by c^2 + s^2, a few 1e-8 away from 1.  A
// QSVT sequence has one distinct phase per step, so these factors do not
// cancel: over the 71,002 phases of the second-order run of Sec. III.E.2 they
// multiply to 1 + 2.6e-5.  Being global scalars they commute with every op,
// and only their product matters.  Each pair is therefore rounded to the FP32
// pair with the smallest angle error among those within one ulp of the
// nearest rounding in each entry that keep the running product of the factors
// within kNormBand of 1; where none does, to the one that brings the product
// closest to 1.  Either way the angle error stays within the nearest
// rounding's bound (half an ulp of each entry), and most pairs keep their
// nearest rounding.
// A real 2x2 gate (the value-load rotations of the block encoding, Sec.
// II.D.2, II.D.3) applies the same matrix in every call of the sequence to its
// controlled subspace; rounded to FP32 its columns' norms differ from 1 by up
// to 5e-8 and that subspace gains or loses the same fraction in every call
// (7e-5 over the second-order run, measured with FP64 arithmetic).  Gates the
// planner marked T_UR2 therefore carry each entry as the FP32 rounding (hi,
// slots 0-3) plus the FP32 rounding of the remainder (lo, slots 4-7), and the
// kernels apply hi + lo.  All other parameters round to nearest.
std::vector<float> tile_params_c64(const std::vector<TileOp> &tops, const std::vector<double> &tparams)
{
    constexpr double kNormBand = 1e-7;
    std::vector<float> f(tparams.begin(), tparams.end());
    double acc = 0.0;  // sum of (factor - 1): the log of the running product, to first order
    for (const TileOp &t : tops) {
        if (t.kind == T_UR2) {  // hi in slots 0-3, the remainder of each entry in slots 4-7
            for (int k = 0; k < 4; ++k) f[t.param + 4 + k] = (float)(tparams[t.param + k] - (double)f[t.param + k]);
            continue;
        }
        if (t.kind != T_PROJ) continue;
        const double c = tparams[t.param], s = tparams[t.param + 1];
        const float cn = (float)c, sn = (float)s;
        const float cc[3] = {cn, std::nextafter(cn, -2.0f), std::nextafter(cn, 2.0f)};
        const float sc[3] = {sn, std::nextafter(sn, -2.0f), std::nextafter(sn, 2.0f)};
        // angle error of (c', s') to first order: c (s' - s) - s (c' - c)
        auto angle_err = [&](float a, float b) { return std::fabs(c * ((double)b - s) - s * ((double)a - c)); };
        const double ulp_c = (double)cc[2] - (double)cn, ulp_s = (double)sc[2] - (double)sn;
        const double lim = std::max(0.5 * (std::fabs(s) * ulp_c + std::fabs(c) * ulp_s), angle_err(cn, sn));
        int in_band = -1, closest = 0;
        double in_band_err = 0.0, closest_acc = 0.0;
        for (int k = 0; k < 9; ++k) {
            const float a = cc[k / 3], b = sc[k % 3];
            const double e = angle_err(a, b);
            if (e > lim) continue;
            const double na = std::fabs(acc + ((double)a * a + (double)b * b - 1.0));
            if (na <= kNormBand && (in_band < 0 || e < in_band_err)) {
                in_band = k;
                in_band_err = e;
            }
            if (k == 0 || na < closest_acc) {
                closest = k;
                closest_acc = na;
            }
        }
        const int k = in_band >= 0 ? in_band : closest;
        const float bc = cc[k / 3], bs = sc[k % 3];
        acc += (double)bc * bc + (double)bs * bs - 1.0;
        f[t.param] = bc;
        f[t.param + 1] = bs;
    }
    return f;
}

}  // namespace svi
