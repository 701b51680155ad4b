// CPU emulation of libsv's launch steps, used only by the host-side tests of
// the planner.  It runs the planner's tile programs exactly as the tile kernel
// does (same load mapping, register stages, LDS exchanges with permutations,
// final exchange) in double precision on a host array, and checks on the way
// that every global and LDS index is in range, that each exchange writes every
// LDS cell exactly once, and that each pass reads and writes every amplitude
// exactly once.  Return codes: 0 ok, >0 a violated check, <0 planner error.
#include <complex>
#include <cstring>
#include <vector>

#include "plan_types.h"

using cd = std::complex<double>;
using namespace svi;

namespace {

uint64_t deposit_zeros(uint64_t x, uint64_t fixed)
{
    for (int p = 0; p < 64; ++p) {
        if (!((fixed >> p) & 1ull)) continue;
        x = ((x >> p) << (p + 1)) | (x & ((1ull << p) - 1ull));
    }
    return x;
}

void emu_plain(const PlainOp &op, int n, cd *psi)
{
    const int c = __builtin_popcountll(op.mask);
    const uint64_t tb = 1ull << op.target;
    switch (op.kind) {
    case SV_OP_U: {
        const cd m0(op.m[0], op.m[1]), m1(op.m[2], op.m[3]), m2(op.m[4], op.m[5]), m3(op.m[6], op.m[7]);
        for (uint64_t w = 0; w < (1ull << (n - 1 - c)); ++w) {
            const uint64_t i0 = deposit_zeros(w, op.mask | tb) | op.val, i1 = i0 | tb;
            const cd a = psi[i0], b = psi[i1];
            psi[i0] = m0 * a + m1 * b;
            psi[i1] = m2 * a + m3 * b;
        }
        break;
    }
    case SV_OP_X:
        for (uint64_t w = 0; w < (1ull << (n - 1 - c)); ++w) {
            const uint64_t i0 = deposit_zeros(w, op.mask | tb) | op.val;
            std::swap(psi[i0], psi[i0 | tb]);
        }
        break;
    case SV_OP_PHASE:
        for (uint64_t w = 0; w < (1ull << (n - 1 - c)); ++w)
            psi[deposit_zeros(w, op.mask | tb) | op.val | tb] *= std::polar(1.0, op.m[0]);
        break;
    case SV_OP_SWAP: {
        const uint64_t ab = tb, bb = 1ull << op.width;
        for (uint64_t w = 0; w < (1ull << (n - 2 - c)); ++w) {
            const uint64_t i = deposit_zeros(w, op.mask | ab | bb) | op.val | ab;
            std::swap(psi[i], psi[i ^ ab ^ bb]);
        }
        break;
    }
    case SV_OP_INC:
    case SV_OP_DEC: {
        const uint64_t len = 1ull << op.width, reg = (len - 1) << op.target;
        for (uint64_t w = 0; w < (1ull << (n - (int)op.width - c)); ++w) {
            const uint64_t r = deposit_zeros(w, op.mask | reg) | op.val;
            std::vector<cd> cyc(len);
            for (uint64_t v = 0; v < len; ++v) cyc[v] = psi[r | (v << op.target)];
            for (uint64_t v = 0; v < len; ++v) {
                const uint64_t src = op.kind == SV_OP_INC ? (v + len - 1) % len : (v + 1) % len;
                psi[r | (v << op.target)] = cyc[src];
            }
        }
        break;
    }
    case SV_OP_PROJPHASE:
        for (uint64_t i = 0; i < (1ull << n); ++i) {
            const int z = (i & op.mask) == op.val, s = (i >> op.target) & 1;
            psi[i] *= std::polar(1.0, op.m[0] * (1 - 2 * (s ^ z)));
        }
        break;
    }
}

uint32_t perms(uint32_t l, const std::vector<TileOp> &ops, uint32_t pb, uint32_t pe, uint64_t base)
{
    for (uint32_t k = pb; k < pe; ++k) {
        const TileOp &p = ops[k];
        if ((base & p.gmask) != p.gval) continue;
        if ((l & p.lmask) != p.lval) continue;
        if (p.kind == T_INC || p.kind == T_DEC) {
            const uint32_t m = (1u << p.b) - 1u;
            uint32_t v = (l >> p.a) & m;
            v = (p.kind == T_INC ? v + 1u : v - 1u) & m;
            l = (l & ~(m << p.a)) | (v << p.a);
        } else if (p.kind == T_SWAP) {
            if (((l >> p.a) ^ (l >> p.b)) & 1u) l ^= (1u << p.a) | (1u << p.b);
        } else if (p.kind == T_XFLIP) {
            l ^= 1u << p.a;
        }
    }
    return l;
}

int check_pass_fields(const sv_plan &p, uint32_t pi)
{
    const TilePass &P = p.passes[pi];
    const int b = P.b, rb = P.rb, nthr = P.nthr, NR = 1 << rb, T = 1 << nthr;
    const int lowb = 4;
    // precomputed pass fields: run maps and swizzled slot offsets
    for (int s = 0; s < NR; ++s)
        if (P.swz0[s] != lds_swizzle((uint32_t)s << nthr, lowb)) return 20;
    for (int t = 0; t < T; ++t) {
        uint64_t g0 = 0, g1 = 0;
        for (int j = 0; j < nthr; ++j) g0 |= (uint64_t)((t >> j) & 1) << P.spos[j];
        for (uint32_t r = 0; r < P.n_gthr_runs; ++r)
            g1 |= (uint64_t)(((uint32_t)t >> (P.gthr_shift[r] & 0xffu)) & P.gthr_mask[r]) << (P.gthr_shift[r] >> 8);
        if (g0 != g1) return 21;
    }
    {
        // nontemporal state accesses for 16 MiB of state or less, or 256 MiB or more
        const uint64_t bytes = (p.dtype == SV_C64 ? 8ull : 16ull) << p.n;
        if (P.stream != ((bytes <= (16ull << 20) || bytes >= (256ull << 20)) ? 1 : 0)) return 37;
    }
    for (uint32_t st = P.stage_begin; st < P.stage_end; ++st) {
        const TileStage &S = p.stages[st];
        // the kernel reads the parameters of op k at k * kParamStride
        for (uint32_t k = S.op_begin; k < S.op_end; ++k)
            if (p.tops[k].param != k * (uint32_t)kParamStride || (k + 1) * kParamStride > p.tparams.size()) return 26;
        // gate runs: the run a head announces lies in the stage, shares the
        // head's tile mask, holds no T_PROJ and is sorted by tile value
        for (uint32_t k = S.op_begin; k < S.op_end; ++k) {
            const TileOp &t = p.tops[k];
            if (t.kind == T_PROJ) continue;
            const uint32_t L = (uint32_t)t.a | ((uint32_t)t.b << 8);
            if (L == 0) continue;
            if (!P.gate_runs || L < 2 || k + L > S.op_end || t.gmask == 0) return 27;
            for (uint32_t j = k + 1; j < k + L; ++j) {
                const TileOp &u = p.tops[j];
                if (u.kind == T_PROJ || u.gmask != t.gmask || u.gval < p.tops[j - 1].gval) return 28;
                if ((uint32_t)u.a | ((uint32_t)u.b << 8)) return 28;
            }
        }
        for (int s = 0; s < NR; ++s)
            if (S.swz[s] != lds_swizzle(S.regoff[s], lowb)) return 22;
        for (int t = 0; t < T; ++t) {
            uint32_t a = 0, c = 0;
            for (int j = 0; j < nthr; ++j) a |= (uint32_t)((t >> j) & 1) << S.thrpos[j];
            for (uint32_t r = 0; r < S.n_thr_runs; ++r) {
                const uint32_t w = S.thr_run[r];
                c |= (((uint32_t)t >> (w & 0xffu)) & (w >> 16)) << ((w >> 8) & 0xffu);
            }
            if (a != c) return 23;
            // the kernel's XOR form of the LDS address equals the swizzle of the local index
            for (int s = 0; s < NR; ++s) {
                const uint32_t lx = lds_swizzle(a, lowb) ^ S.swz[s];
                if (lx != lds_swizzle(a | S.regoff[s], lowb) || lx >= (1u << b)) return 24;
            }
        }
    }
    // tile runs on a sample of tile counters (all of them when few)
    const uint64_t ntiles = 1ull << P.ntile;
    const uint64_t step = ntiles > 4096 ? ntiles / 4096 + 1 : 1;
    for (uint64_t tile = 0; tile < ntiles; tile += step) {
        uint64_t base = 0, b2 = 0;
        for (int j = 0; j < P.ntile; ++j) base |= ((tile >> j) & 1ull) << P.tpos[j];
        for (uint32_t r = 0; r < P.n_tile_runs; ++r)
            b2 |= ((tile >> (P.tile_shift[r] & 0xffu)) & P.tile_mask[r]) << (P.tile_shift[r] >> 8);
        if (b2 != base) return 25;
    }
    return 0;
}

int emu_tile(const sv_plan &p, uint32_t pi, cd *psi, std::vector<int> &rd, std::vector<int> &wr)
{
    const TilePass &P = p.passes[pi];
    const int n = p.n, b = P.b, rb = P.rb, nthr = P.nthr, NR = 1 << rb, T = 1 << nthr;
    const uint64_t dim = 1ull << n;
    if (b != nthr + rb || P.ntile != n - b) return 1;
    std::fill(rd.begin(), rd.end(), 0);
    std::fill(wr.begin(), wr.end(), 0);
    std::vector<cd> x((size_t)T * NR), lds((size_t)1 << b);
    std::vector<int> filled((size_t)1 << b);
    std::vector<uint32_t> thr(T);
    std::vector<uint32_t> ro(NR);
    const int lowb = 4;
    {
        const int rc = check_pass_fields(p, pi);
        if (rc) return rc;
    }
    for (uint64_t tile = 0; tile < (1ull << P.ntile); ++tile) {
        uint64_t base = 0;
        for (int j = 0; j < P.ntile; ++j) base |= ((tile >> j) & 1ull) << P.tpos[j];
        {
            uint64_t b2 = 0;
            for (uint32_t r = 0; r < P.n_tile_runs; ++r)
                b2 |= ((tile >> (P.tile_shift[r] & 0xffu)) & P.tile_mask[r]) << (P.tile_shift[r] >> 8);
            if (b2 != base) return 25;
        }
        auto gidx = [&](int t, int s) {
            uint64_t g = 0;
            for (int j = 0; j < nthr; ++j) g |= (uint64_t)((t >> j) & 1) << P.spos[j];
            return base | g | P.goff[s];
        };
        for (int t = 0; t < T; ++t)
            for (int s = 0; s < NR; ++s) {
                const uint64_t g = gidx(t, s);
                if (g >= dim) return 2;
                rd[g]++;
                x[(size_t)t * NR + s] = psi[g];
            }
        for (int t = 0; t < T; ++t) thr[t] = t;
        for (int s = 0; s < NR; ++s) ro[s] = (uint32_t)s << nthr;
        auto exchange = [&](uint32_t pb, uint32_t pe, const uint8_t *thrpos, const uint32_t *regoff) -> int {
            std::fill(filled.begin(), filled.end(), 0);
            for (int t = 0; t < T; ++t)
                for (int s = 0; s < NR; ++s) {
                    const uint32_t l = perms(thr[t] | ro[s], p.tops, pb, pe, base);
                    if (l >= (1u << b)) return 3;
                    if (filled[l]++) return 4;
                    lds[l] = x[(size_t)t * NR + s];
                }
            for (int t = 0; t < T; ++t) {
                uint32_t t2 = 0;
                for (int j = 0; j < nthr; ++j) t2 |= (uint32_t)((t >> j) & 1) << thrpos[j];
                thr[t] = t2;
            }
            for (int s = 0; s < NR; ++s) ro[s] = regoff[s];
            for (int t = 0; t < T; ++t)
                for (int s = 0; s < NR; ++s) {
                    const uint32_t l = thr[t] | ro[s];
                    if (l >= (1u << b) || !filled[l]) return 5;
                    x[(size_t)t * NR + s] = lds[l];
                }
            return 0;
        };
        for (uint32_t st = P.stage_begin; st < P.stage_end; ++st) {
            const TileStage &S = p.stages[st];
            if (st != P.stage_begin) {
                int rc = exchange(S.perm_begin, S.perm_end, S.thrpos, S.regoff);
                if (rc) return rc;
            }
            for (uint32_t k = S.op_begin; k < S.op_end; ++k) {
                const TileOp &op = p.tops[k];
                const double *prm = p.tparams.data() + op.param;
                // the slot/thread split of the condition must agree with the local condition
                for (int t = 0; t < T; ++t)
                    for (int s = 0; s < NR; ++s) {
                        const uint32_t l = thr[t] | ro[s];
                        const bool split_ok = ((op.slotmask >> s) & 1u) && ((t & op.tidmask) == op.tidval);
                        if (split_ok != ((l & op.lmask) == op.lval)) return 10;
                    }
                if (op.kind == T_PROJ) {
                    const bool zg = (base & op.gmask) == op.gval;
                    for (int t = 0; t < T; ++t) {
                        const bool tc = (t & op.tidmask) == op.tidval;
                        for (int s = 0; s < NR; ++s) {
                            const uint32_t z = (zg && tc && ((op.slotmask >> s) & 1u)) ? 1u : 0u;
                            uint32_t sb = 0;
                            if (op.a == 0) sb = (uint32_t)((base >> op.b) & 1ull);
                            else if (op.a == 1) sb = ((uint32_t)s >> op.b) & 1u;
                            else if (op.a == 2) sb = ((uint32_t)t >> op.b) & 1u;
                            else return 11;
                            x[(size_t)t * NR + s] *= cd(prm[0], (sb ^ z) ? -prm[1] : prm[1]);
                        }
                    }
                    continue;
                }
                if ((base & op.gmask) != op.gval) continue;
                for (int t = 0; t < T; ++t) {
                    if ((t & op.tidmask) != op.tidval) continue;
                    if (op.kind == T_PHASE) {
                        for (int s = 0; s < NR; ++s)
                            if ((op.slotmask >> s) & 1u) x[(size_t)t * NR + s] *= cd(prm[0], prm[1]);
                        continue;
                    }
                    if (op.slot >= rb) return 6;
                    const int K = op.slot;
                    for (int s = 0; s < NR; ++s) {
                        if (s & (1 << K)) continue;
                        if (!((op.slotmask >> s) & 1u)) continue;
                        cd &a = x[(size_t)t * NR + s];
                        cd &bb = x[(size_t)t * NR + (s | (1 << K))];
                        const cd a0 = a, b0 = bb;
                        if (op.kind == T_U) {
                            a = cd(prm[0], prm[1]) * a0 + cd(prm[2], prm[3]) * b0;
                            bb = cd(prm[4], prm[5]) * a0 + cd(prm[6], prm[7]) * b0;
                        } else if (op.kind == T_UR || op.kind == T_UR2) {
                            a = prm[0] * a0 + prm[1] * b0;
                            bb = prm[2] * a0 + prm[3] * b0;
                        } else if (op.kind == T_X) {
                            std::swap(a, bb);
                        } else {
                            return 7;
                        }
                    }
                }
            }
        }
        // the last stage must leave the load mapping unless a final exchange follows
        if (P.final_exchange) {
            uint8_t thrpos0[16];
            uint32_t regoff0[1 << kMaxRB];
            for (int j = 0; j < nthr; ++j) thrpos0[j] = (uint8_t)j;
            for (int s = 0; s < NR; ++s) regoff0[s] = (uint32_t)(s << nthr);
            int rc = exchange(P.fperm_begin, P.fperm_end, thrpos0, regoff0);
            if (rc) return rc;
        } else {
            for (int t = 0; t < T; ++t)
                if (thr[t] != (uint32_t)t) return 8;
            for (int s = 0; s < NR; ++s)
                if (ro[s] != ((uint32_t)s << nthr)) return 8;
        }
        for (int t = 0; t < T; ++t)
            for (int s = 0; s < NR; ++s) {
                const uint64_t g = gidx(t, s);
                wr[g]++;
                psi[g] = x[(size_t)t * NR + s];
            }
    }
    for (uint64_t i = 0; i < dim; ++i)
        if (rd[i] != 1 || wr[i] != 1) return 9;
    return 0;
}

// Dense block pass: gather each tile through the load mapping, multiply every
// group's 32 amplitudes by the block matrix (double precision), scatter back.
// Checks: group and block offsets tile the 4096 local indices exactly once, and
// every amplitude is read and written exactly once over the pass.
int emu_dense(const sv_plan &p, uint32_t di, cd *psi, std::vector<int> &rd, std::vector<int> &wr)
{
    const DensePass &D = p.dense[di];
    const TilePass &P = D.map;
    const int n = p.n;
    const uint64_t dim = 1ull << n;
    if (P.b != 12 || P.nthr != 8 || P.rb != 4 || P.ntile != n - 12) return 30;
    // LDS swizzle width of the amplitude size (8 B complex64, 16 B complex128)
    const int dl = p.dtype == SV_C64 ? 4 : 3;
    for (int s = 0; s < 16; ++s)
        if (P.swz0[s] != lds_swizzle((uint32_t)s << 8, dl)) return 36;
    std::fill(rd.begin(), rd.end(), 0);
    std::fill(wr.begin(), wr.end(), 0);
    if (D.k != 5 && D.k != 6) return 37;
    if (D.k == 6 && p.dtype != SV_C64) return 38;
    const int N = 1 << D.k, NG = 4096 >> D.k;
    // group offsets from the runs, and the exact cover of the local indices
    uint32_t goffl[128];
    std::vector<int> cover(4096, 0);
    for (int g = 0; g < NG; ++g) {
        uint32_t o = 0;
        for (uint32_t r = 0; r < D.n_grp_runs; ++r) {
            const uint32_t w = D.grp_run[r];
            o |= (((uint32_t)g >> (w & 0xffu)) & (w >> 16)) << ((w >> 8) & 0xffu);
        }
        goffl[g] = o;
        for (int j = 0; j < N; ++j) {
            const uint32_t l = o | D.joff[j];
            if (l >= 4096 || (o & D.joff[j])) return 31;
            cover[l]++;
        }
    }
    for (int l = 0; l < 4096; ++l)
        if (cover[l] != 1) return 32;
    if (D.mat + 2 * (size_t)N * N > p.dparams.size()) return 33;
    const double *G = p.dparams.data() + D.mat;
    std::vector<cd> x(4096), y(4096);
    for (uint64_t tile = 0; tile < (1ull << P.ntile); ++tile) {
        uint64_t base = 0;
        for (uint32_t r = 0; r < P.n_tile_runs; ++r)
            base |= ((tile >> (P.tile_shift[r] & 0xffu)) & P.tile_mask[r]) << (P.tile_shift[r] >> 8);
        auto gidx = [&](uint32_t l) {
            uint64_t g = 0;
            for (int k = 0; k < 12; ++k)
                if ((l >> k) & 1u) g |= 1ull << P.spos[k];
            return base | g;
        };
        for (uint32_t l = 0; l < 4096; ++l) {
            const uint64_t g = gidx(l);
            if (g >= dim) return 34;
            rd[g]++;
            x[l] = psi[g];
        }
        for (int g = 0; g < NG; ++g)
            for (int i = 0; i < N; ++i) {
                cd acc(0.0, 0.0);
                for (int j = 0; j < N; ++j)
                    acc += cd(G[2 * (N * i + j)], G[2 * (N * i + j) + 1]) * x[goffl[g] | D.joff[j]];
                y[goffl[g] | D.joff[i]] = acc;
            }
        for (uint32_t l = 0; l < 4096; ++l) {
            const uint64_t g = gidx(l);
            wr[g]++;
            psi[g] = y[l];
        }
    }
    for (uint64_t i = 0; i < dim; ++i)
        if (rd[i] != 1 || wr[i] != 1) return 35;
    return 0;
}

}  // namespace

// When set, complex64 plans run with their parameters rounded to float, as
// the library uploads them (tile parameters as the upload rounds them, dense
// parameters to nearest, plain-op matrices as hi + lo pairs; phase angles'
// cosines and sines are computed from the rounded values only where the
// kernels do the same); the arithmetic stays double.
static int g_round_params_f32 = 0;
extern "C" void emu_set_param_rounding(int on) { g_round_params_f32 = on; }

// sv_apply_opts.peephole of the plans emu_run builds (SV_PEEPHOLE_AUTO by default).
static int g_peephole = SV_PEEPHOLE_AUTO;
extern "C" void emu_set_peephole(int v) { g_peephole = v; }

// sv_apply_opts.dense_qubits of the plans emu_run builds (0: five).
static int g_dense_qubits = 0;
extern "C" void emu_set_dense_qubits(int v) { g_dense_qubits = v; }

// sv_apply_opts.coalesce_qubits of the plans emu_run builds (0: automatic).
static int g_coalesce_qubits = 0;
extern "C" void emu_set_coalesce_qubits(int v) { g_coalesce_qubits = v; }

// sv_apply_opts.split_real of the plans emu_run builds (SV_SPLIT_REAL_AUTO by default).
static int g_split_real = SV_SPLIT_REAL_AUTO;
extern "C" void emu_set_split_real(int v) { g_split_real = v; }

// Plans the op list and runs the plan on psi_io (interleaved re, im).  stats,
// when given, receives 7 entries: launches, tile passes, register stages,
// algorithmic bytes, ops split to plain launches, ops inside gate runs, ops
// dropped by the peephole pass.
extern "C" int emu_run(int n, int dtype, const sv_op *ops, size_t n_ops, const double *params, int mode,
                       int tile_qubits, int reg_qubits, double *psi_io, uint64_t *stats, int dense_min_ops)
{
    sv_plan p;
    p.n = n;
    p.dtype = dtype;
    sv_apply_opts o{mode, tile_qubits, reg_qubits, dense_min_ops};
    o.peephole = g_peephole;
    o.dense_qubits = g_dense_qubits;
    o.coalesce_qubits = g_coalesce_qubits;
    o.split_real = g_split_real;
    std::string err;
    int rc = build_plan(&p, ops, n_ops, params, o, err);
    if (rc != SV_OK) return rc;
    if (g_round_params_f32 && dtype == SV_C64) {
        const std::vector<float> f = tile_params_c64(p.tops, p.tparams);
        for (size_t k = 0; k < f.size(); ++k) p.tparams[k] = f[k];
        for (const TileOp &t : p.tops)  // split real 2x2 gates apply hi + lo
            if (t.kind == T_UR2)
                for (int k = 0; k < 4; ++k) p.tparams[t.param + k] += (double)f[t.param + 4 + k];
        for (double &v : p.dparams) v = (double)(float)v;
        for (PlainOp &op : p.plain)  // plain launches carry their matrix as hi + lo FP32 pairs
            if (op.kind == SV_OP_U)
                for (double &v : op.m) {
                    const float hi = (float)v;
                    v = (double)hi + (double)(float)(v - (double)hi);
                }
    }
    cd *psi = reinterpret_cast<cd *>(psi_io);
    std::vector<int> rd(1ull << n), wr(1ull << n);
    for (const auto &st : p.steps) {
        if (st.type == 0) {
            emu_plain(p.plain[st.index], n, psi);
        } else if (st.type == 1) {
            rc = emu_tile(p, st.index, psi, rd, wr);
            if (rc) return 100 + rc;
        } else {
            rc = emu_dense(p, st.index, psi, rd, wr);
            if (rc) return 200 + rc;
        }
    }
    if (stats) {
        stats[0] = p.info.n_launches;
        stats[1] = p.info.n_tile_passes;
        stats[2] = p.info.n_stages;
        stats[3] = p.info.bytes_moved;
        stats[4] = p.info.n_split_ops;
        uint64_t in_runs = 0;  // ops that gate runs cover
        for (const TileStage &S : p.stages)
            for (uint32_t k = S.op_begin; k < S.op_end; ++k)
                if (p.tops[k].kind != T_PROJ) in_runs += (uint32_t)p.tops[k].a | ((uint32_t)p.tops[k].b << 8);
        stats[5] = in_runs;
        stats[6] = p.info.n_cancelled_ops;
    }
    return 0;
}

// Plan only (no emulation): launch/pass/stage counts and algorithmic bytes.
extern "C" int emu_plan_stats(int n, int dtype, const sv_op *ops, size_t n_ops, const double *params, int mode,
                              int tile_qubits, int reg_qubits, uint64_t *stats)
{
    sv_plan p;
    p.n = n;
    p.dtype = dtype;
    sv_apply_opts o{mode, tile_qubits, reg_qubits, 0};
    std::string err;
    int rc = build_plan(&p, ops, n_ops, params, o, err);
    if (rc != SV_OK) return rc;
    stats[0] = p.info.n_launches;
    stats[1] = p.info.n_tile_passes;
    stats[2] = p.info.n_stages;
    stats[3] = p.info.bytes_moved;
    return 0;
}

// Plan only, then check the precomputed fields of every tile pass (any size).
extern "C" int emu_check_fields(int n, int dtype, const sv_op *ops, size_t n_ops, const double *params,
                                int tile_qubits, int reg_qubits)
{
    sv_plan p;
    p.n = n;
    p.dtype = dtype;
    sv_apply_opts o{SV_MODE_FUSED, tile_qubits, reg_qubits, 0};
    std::string err;
    int rc = build_plan(&p, ops, n_ops, params, o, err);
    if (rc != SV_OK) return rc;
    for (uint32_t pi = 0; pi < p.passes.size(); ++pi)
        if ((rc = check_pass_fields(p, pi)) != 0) return 100 + rc;
    return 0;
}
