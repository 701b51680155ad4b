// Specialised tile-pass kernels: HIP source for one tile pass of a plan, with
// the pass's op list written out as straight-line code.
//
// The generic tile kernel (kernels_tile.hip) interprets a pass's op records at
// run time: every op costs scalar record loads, a branch tree over kind and
// register slot, per-slot condition tests and register copies at the merges
// of those branches.  Here the same pass (the planner's TilePass, TileStage
// and TileOp tables, unchanged) becomes a kernel in which every op is a
// compile-time block: its slots, register bits, conditions and permutations
// are constants, so what remains at run time is the gate arithmetic, the
// per-lane and per-tile condition tests, the LDS exchanges and the parameter
// loads (uniform, scalar).  The arithmetic is the generic kernel's, written
// the same way operation for operation, so both give bit-identical states.
//
// Passes with the same structure (the U_L and U_L^dagger passes repeated by a
// QSVT ladder) give the same source: parameters are read relative to the
// pass's own parameter block, passed at launch.
//
// Host-only code (no HIP types): the runtime side (compilation, loading,
// launch) is in kernels_jit.hip.
#include <cstdio>
#include <cstring>
#include <sstream>
#include <string>

#include "plan_types.h"

namespace svi {

namespace {

std::string hex64(uint64_t v)
{
    char b[32];
    std::snprintf(b, sizeof b, "0x%llxull", (unsigned long long)v);
    return b;
}

std::string hex32(uint32_t v)
{
    char b[24];
    std::snprintf(b, sizeof b, "0x%xu", v);
    return b;
}

struct Gen {
    const sv_plan &p;
    const TilePass &P;
    bool dbl;
    int NR;
    uint32_t pbase;  // the pass's first parameter (reals)
    std::ostringstream o;
    int tmp = 0;

    Gen(const sv_plan &plan, const TilePass &pass, uint32_t param_base)
        : p(plan), P(pass), dbl(plan.dtype != SV_C64), NR(1 << pass.rb), pbase(param_base)
    {
    }

    const char *R() const { return dbl ? "double" : "float"; }

    // thread bits of `tid` -> local index bits, as packed runs
    std::string thr_expr(const uint32_t *runs, uint32_t n)
    {
        std::string e = "0u";
        for (uint32_t r = 0; r < n; ++r) {
            const uint32_t w = runs[r];
            const uint32_t src = w & 0xffu, dst = (w >> 8) & 0xffu, m = w >> 16;
            e += " | (((tid >> " + std::to_string(src) + ") & " + hex32(m) + ") << " + std::to_string(dst) + ")";
        }
        return e;
    }

    // condition prefix/suffix for a uniform tile condition (gmask, gval)
    std::string tile_if(uint64_t gm, uint64_t gv)
    {
        if (!gm) return "{";
        return "if ((base & " + hex64(gm) + ") == " + hex64(gv) + ") {";
    }

    // Local indices of all slots after the permutations [pb, pe), starting
    // from l_s = thr | regoff[s].  Written per slot with constants: the
    // compiler folds every test that involves register bits only (it knows
    // which bits the thread part can hold).
    void perm_indices(const uint32_t *regoff, uint32_t pb, uint32_t pe)
    {
        for (int s = 0; s < NR; ++s) o << "  l[" << s << "] = thr | " << hex32(regoff[s]) << ";\n";
        for (uint32_t k = pb; k < pe; ++k) {
            const TileOp &t = p.tops[k];
            o << "  " << tile_if(t.gmask, t.gval) << "\n";
            o << "   for (int s = 0; s < " << NR << "; ++s) {\n";
            o << "    const u32 v = l[s];\n";
            o << "    const bool c = (v & " << hex32(t.lmask) << ") == " << hex32(t.lval) << ";\n";
            switch (t.kind) {
            case T_INC:
            case T_DEC: {
                const uint32_t m = ((1u << t.b) - 1u) << t.a;
                const uint32_t step = (t.kind == T_INC ? 1u : (uint32_t)-1) << t.a;
                o << "    const u32 w = ((v & " << hex32(m) << ") + " << hex32(step) << ") & " << hex32(m) << ";\n";
                o << "    l[s] = c ? ((v & " << hex32(~m) << ") | w) : v;\n";
                break;
            }
            case T_SWAP: {
                const uint32_t both = (1u << t.a) | (1u << t.b);
                o << "    const bool h = c && ((((v >> " << (int)t.a << ") ^ (v >> " << (int)t.b << ")) & 1u) != 0u);\n";
                o << "    l[s] = h ? (v ^ " << hex32(both) << ") : v;\n";
                break;
            }
            case T_XFLIP:
                o << "    l[s] = c ? (v ^ " << hex32(1u << t.a) << ") : v;\n";
                break;
            default:
                break;
            }
            o << "   }\n  }\n";
        }
    }

    // One exchange through LDS: write under the old mapping (thread part
    // `thr`, slot offsets wregoff/wswz, or the permuted indices l[]), barrier,
    // read under the new mapping (thread runs `runs`, slot swizzles rswz).
    void exchange(bool perms, const uint32_t *wswz, const uint32_t *rruns, uint32_t nrruns, const uint32_t *rswz,
                  bool to_load_mapping)
    {
        o << "  bar();\n";
        const std::string t2 = to_load_mapping ? std::string("tid") : thr_expr(rruns, nrruns);
        if (!dbl) {
            if (perms) {
                o << "  for (int s = 0; s < " << NR << "; ++s) lds[swz(l[s])] = x[s];\n";
            } else {
                o << "  { const u32 tw = opq(swz(thr) * 8u);\n";
                for (int s = 0; s < NR; ++s)
                    o << "    *(C *)(lb + (tw ^ " << hex32(wswz[s] * 8u) << ")) = x[" << s << "];\n";
                o << "  }\n";
            }
            o << "  bar();\n";
            o << "  thr = " << t2 << ";\n";
            o << "  { const u32 tr = opq(swz(thr) * 8u);\n";
            for (int s = 0; s < NR; ++s)
                o << "    x[" << s << "] = *(const C *)(lb + (tr ^ " << hex32(rswz[s] * 8u) << "));\n";
            o << "  }\n";
            return;
        }
        // complex128: real parts through an LDS array of doubles, then the
        // imaginary parts (half the tile's bytes)
        o << "  { const u32 t2 = " << t2 << ";\n";
        o << "    const u32 tr = opq(swz(t2) * 8u);\n";
        if (perms) {
            o << "    u32 wa[" << NR << "];\n";
            o << "    for (int s = 0; s < " << NR << "; ++s) wa[s] = swz(l[s]) * 8u;\n";
        } else {
            o << "    const u32 tw = opq(swz(thr) * 8u);\n";
        }
        for (int half = 0; half < 2; ++half) {
            const char *f = half ? "y" : "x";
            if (half) o << "    bar();\n";
            for (int s = 0; s < NR; ++s) {
                if (perms)
                    o << "    *(double *)(lb + wa[" << s << "]) = x[" << s << "]." << f << ";\n";
                else
                    o << "    *(double *)(lb + (tw ^ " << hex32(wswz[s] * 8u) << ")) = x[" << s << "]." << f << ";\n";
            }
            o << "    bar();\n";
            for (int s = 0; s < NR; ++s)
                o << "    x[" << s << "]." << f << " = *(const double *)(lb + (tr ^ " << hex32(rswz[s] * 8u) << "));\n";
        }
        o << "    thr = t2;\n  }\n";
    }

    std::string prm(uint32_t param, int j) { return "prm[" + std::to_string(param - pbase + (uint32_t)j) + "]"; }

    // One register-level op (the generic kernel's tile_compute op loop body).
    void op(const TileOp &t)
    {
        const std::string tc = t.tidmask ? "(tid & " + hex32(t.tidmask) + ") == " + hex32(t.tidval) : "true";
        if (t.kind == T_PROJ) {
            o << "  { const R c = " << prm(t.param, 0) << ", sn = " << prm(t.param, 1) << ";\n";
            o << "    const bool zg = " << (t.gmask ? "(base & " + hex64(t.gmask) + ") == " + hex64(t.gval) : "true")
              << ";\n";
            o << "    const bool z0 = zg && (" << tc << ");\n";
            o << "    const u32 sg = " << (t.a == 2 ? "((tid >> " + std::to_string(t.b) + ") & 1u)" : std::string("0u"))
              << " ^ " << (t.a == 0 ? "(u32)((base >> " + std::to_string(t.b) + ") & 1ull)" : std::string("0u")) << ";\n";
            for (int s = 0; s < NR; ++s) {
                const bool in = (t.slotmask >> s) & 1u;
                const uint32_t ss = t.a == 1 ? (((uint32_t)s >> t.b) & 1u) : 0u;
                o << "    proj(x[" << s << "], c, ((sg ^ " << ss << "u ^ (" << (in ? "z0" : "false") << " ? 1u : 0u)) != 0u) ? -sn : sn);\n";
            }
            o << "  }\n";
            return;
        }
        o << "  " << tile_if(t.gmask, t.gval);
        if (t.tidmask) o << " if (" << tc << ") {";
        o << "\n";
        const int K = t.slot;
        switch (t.kind) {
        case T_U: {
            o << "    const R m0 = " << prm(t.param, 0);
            for (int j = 1; j < 8; ++j) o << ", m" << j << " = " << prm(t.param, j);
            o << ";\n";
            for (int s = 0; s < NR; ++s) {
                if (s & (1 << K) || !((t.slotmask >> s) & 1u)) continue;
                o << "    gu(x[" << s << "], x[" << (s | (1 << K)) << "], m0, m1, m2, m3, m4, m5, m6, m7);\n";
            }
            break;
        }
        case T_UR:
        case T_UR2: {  // T_UR2 (complex64): hi m0..m3 + lo m4..m7
            const bool two = t.kind == T_UR2;
            o << "    const R m0 = " << prm(t.param, 0);
            for (int j = 1; j < (two ? 8 : 4); ++j) o << ", m" << j << " = " << prm(t.param, j);
            o << ";\n";
            for (int s = 0; s < NR; ++s) {
                if (s & (1 << K) || !((t.slotmask >> s) & 1u)) continue;
                o << "    " << (two ? "gur2" : "gur") << "(x[" << s << "], x[" << (s | (1 << K))
                  << "], m0, m1, m2, m3" << (two ? ", m4, m5, m6, m7" : "") << ");\n";
            }
            break;
        }
        case T_X:
            for (int s = 0; s < NR; ++s) {
                if (s & (1 << K) || !((t.slotmask >> s) & 1u)) continue;
                o << "    { const C a = x[" << s << "]; x[" << s << "] = x[" << (s | (1 << K)) << "]; x["
                  << (s | (1 << K)) << "] = a; }\n";
            }
            break;
        case T_PHASE: {
            o << "    const R c = " << prm(t.param, 0) << ", sn = " << prm(t.param, 1) << ";\n";
            for (int s = 0; s < NR; ++s)
                if ((t.slotmask >> s) & 1u) o << "    proj(x[" << s << "], c, sn);\n";
            break;
        }
        default:
            break;
        }
        o << "  }";
        if (t.tidmask) o << "}";
        o << "\n";
    }

    // The register-level ops of one stage.  Consecutive ops that share a
    // nonzero tile mask (no projector phase among them) go into one switch on
    // the tile's value of those qubits, grouped by value: ops with different
    // values never act in the same tile, so they commute.
    void stage_ops(uint32_t ob, uint32_t oe)
    {
        uint32_t k = ob;
        while (k < oe) {
            const TileOp &h = p.tops[k];
            uint32_t e = k + 1;
            if (h.kind != T_PROJ && h.gmask != 0)
                while (e < oe && p.tops[e].kind != T_PROJ && p.tops[e].gmask == h.gmask) ++e;
            if (e - k < 3) {
                for (; k < e; ++k) op(p.tops[k]);
                continue;
            }
            o << "  switch (base & " << hex64(h.gmask) << ") {\n";
            std::vector<char> done(e - k, 0);
            for (uint32_t i = k; i < e; ++i) {
                if (done[i - k]) continue;
                const uint64_t v = p.tops[i].gval;
                o << "  case " << hex64(v) << ": {\n";
                for (uint32_t j = i; j < e; ++j) {
                    if (done[j - k] || p.tops[j].gval != v) continue;
                    done[j - k] = 1;
                    TileOp t = p.tops[j];
                    t.gmask = 0;  // the case label holds the tile condition
                    t.gval = 0;
                    op(t);
                }
                o << "  } break;\n";
            }
            o << "  default: break;\n  }\n";
            k = e;
        }
    }

    // absolute index bits of tile `t` (runs of the tile counter)
    std::string base_expr(const char *t)
    {
        std::string e = "0ull";
        for (uint32_t r = 0; r < P.n_tile_runs; ++r) {
            const uint32_t sh = P.tile_shift[r];
            e += " | ((" + std::string(t) + " >> " + std::to_string(sh & 0xffu) + ") & " + hex64(P.tile_mask[r]) +
                 ") << " + std::to_string(sh >> 8);
        }
        return e;
    }

    void loads(const char *dst, const char *ptr)
    {
        for (int s = 0; s < NR; ++s)
            o << " " << dst << "[" << s << "] = " << (P.stream ? "ldnt" : "ld") << "(" << ptr << " + "
              << hex64(P.goff[s]) << ");\n";
    }

    // persistent: one resident set of workgroups walks the tiles (tile, tile +
    // gridDim.x, ...) and issues the loads of its next tile before computing
    // the current one; the tiles are disjoint, so a prefetch never reads what
    // another workgroup writes, and the first LDS exchange of every tile starts
    // with a barrier that orders it after the previous tile's LDS reads
    void body(bool persistent)
    {
        const int b = P.b;
        o << " __shared__ " << (dbl ? "double" : "C") << " lds[" << (1u << b) << "];\n";
        o << " unsigned char *const lb = (unsigned char *)lds;\n";
        o << " const u32 tid = threadIdx.x;\n";
        o << " const u64 gthr = 0ull";
        for (uint32_t r = 0; r < P.n_gthr_runs; ++r) {
            const uint32_t sh = P.gthr_shift[r];
            o << " | ((u64)((tid >> " << (sh & 0xffu) << ") & " << hex32(P.gthr_mask[r]) << ") << " << (sh >> 8) << ")";
        }
        o << ";\n";
        if (persistent) {
            o << " u64 tile = (u64)blockIdx.x;\n";
            o << " if (tile >= n_tiles) return;\n";
            o << " u64 base_n = " << base_expr("tile") << ";\n";
            o << " C xn[" << NR << "];\n";
            o << " { C *const q = psi + (base_n | gthr);\n";
            loads("xn", "q");
            o << " }\n";
            o << " for (;;) {\n";
            o << " C x[" << NR << "];\n";
            for (int s = 0; s < NR; ++s) o << " x[" << s << "] = xn[" << s << "];\n";
            o << " const u64 base = base_n;\n";
            o << " const u64 next = tile + (u64)gridDim.x;\n";
            o << " if (next < n_tiles) {\n  base_n = " << base_expr("next") << ";\n";
            o << "  C *const q = psi + (base_n | gthr);\n";
            loads("xn", "q");
            o << " }\n";
        } else {
            if (P.ntile > 16)
                o << " const u64 tile = (u64)blockIdx.x + (u64)blockIdx.y * (u64)gridDim.x;\n";
            else
                o << " const u64 tile = (u64)blockIdx.x;\n";
            o << " const u64 base = " << base_expr("tile") << ";\n";
            o << " C x[" << NR << "];\n";
            o << " { C *const q = psi + (base | gthr);\n";
            loads("x", "q");
            o << " }\n";
        }
        o << " C *const pt = psi + (base | gthr);\n";
        o << " u32 thr = tid;\n";
        o << " u32 l[" << NR << "];\n (void)l;\n";
        for (uint32_t st = P.stage_begin; st < P.stage_end; ++st) {
            const TileStage &S = p.stages[st];
            o << " // stage " << (st - P.stage_begin) << "\n";
            if (st != P.stage_begin) {
                const TileStage &Pv = p.stages[st - 1];
                const bool perms = S.perm_begin != S.perm_end;
                o << " {\n";
                if (perms) perm_indices(Pv.regoff, S.perm_begin, S.perm_end);
                exchange(perms, Pv.swz, S.thr_run, S.n_thr_runs, S.swz, false);
                o << " }\n";
            }
            stage_ops(S.op_begin, S.op_end);
        }
        if (P.final_exchange) {
            const TileStage &Lst = p.stages[P.stage_end - 1];
            const bool perms = P.fperm_begin != P.fperm_end;
            o << " // back to the load mapping\n {\n";
            if (perms) perm_indices(Lst.regoff, P.fperm_begin, P.fperm_end);
            exchange(perms, Lst.swz, nullptr, 0, P.swz0, true);
            o << " }\n";
        }
        for (int s = 0; s < NR; ++s)
            o << " " << (P.stream ? "stnt" : "st") << "(pt + " << hex64(P.goff[s]) << ", x[" << s << "]);\n";
        if (persistent) o << " if (next >= n_tiles) break;\n tile = next;\n }\n";
    }
};

}  // namespace

// Shared definitions at the top of every generated translation unit.
std::string jit_preamble(int dtype)
{
    const bool dbl = dtype != SV_C64;
    std::ostringstream o;
    o << "typedef unsigned int u32;\ntypedef unsigned long long u64;\n";
    o << "typedef " << (dbl ? "double" : "float") << " R;\n";
    o << "typedef R C __attribute__((ext_vector_type(2)));\n";
    // fused multiply-add in the amplitude precision (no promotion to double)
    o << "#define FMA " << (dbl ? "__builtin_fma" : "__builtin_fmaf") << "\n";
    o << "__device__ __forceinline__ u32 opq(u32 v) { asm volatile(\"\" : \"+v\"(v)); return v; }\n";
    // Workgroup barrier that orders LDS accesses only.  __syncthreads() also
    // fences global memory, which makes every wave wait for its outstanding
    // global loads at the barrier: in the persistent form those are the next
    // tile's prefetch.  The tiles' global accesses are disjoint, so the LDS is
    // all a barrier here has to order.
    o << "__device__ __forceinline__ void bar() {\n"
         "  __builtin_amdgcn_fence(__ATOMIC_RELEASE, \"workgroup\", \"local\");\n"
         "  __builtin_amdgcn_s_barrier();\n"
         "  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, \"workgroup\", \"local\");\n}\n";
    o << "__device__ __forceinline__ u32 swz(u32 l) {\n"
         "  const u32 h = (l >> 4) ^ (l >> 8) ^ (l >> 12) ^ (l >> 16);\n"
         "  return l ^ (h & 15u);\n}\n";
    o << "__device__ __forceinline__ C ld(const C *q) { return *q; }\n";
    o << "__device__ __forceinline__ C ldnt(const C *q) { return __builtin_nontemporal_load(q); }\n";
    o << "__device__ __forceinline__ void st(C *q, C v) { *q = v; }\n";
    o << "__device__ __forceinline__ void stnt(C *q, C v) { __builtin_nontemporal_store(v, q); }\n";
    // the generic kernel's arithmetic, operation for operation
    o << "__device__ __forceinline__ C row2(R ar, R ai, R br, R bi, C a, C b) {\n"
         "  C r;\n"
         "  r.x = FMA(ar, a.x, FMA(-ai, a.y, FMA(br, b.x, -bi * b.y)));\n"
         "  r.y = FMA(ar, a.y, FMA(ai, a.x, FMA(br, b.y, bi * b.x)));\n"
         "  return r;\n}\n";
    o << "__device__ __forceinline__ void gu(C &x0, C &x1, R m0, R m1, R m2, R m3, R m4, R m5, R m6, R m7) {\n"
         "  const C a = x0, b = x1;\n"
         "  x0 = row2(m0, m1, m2, m3, a, b);\n"
         "  x1 = row2(m4, m5, m6, m7, a, b);\n}\n";
    o << "__device__ __forceinline__ void gur(C &x0, C &x1, R m0, R m1, R m2, R m3) {\n"
         "  const C a = x0, b = x1;\n"
         "  C r0, r1;\n"
         "  r0.x = FMA(m0, a.x, m1 * b.x);\n"
         "  r0.y = FMA(m0, a.y, m1 * b.y);\n"
         "  r1.x = FMA(m2, a.x, m3 * b.x);\n"
         "  r1.y = FMA(m2, a.y, m3 * b.y);\n"
         "  x0 = r0;\n  x1 = r1;\n}\n";
    // hi (m) + lo (l)
    o << "__device__ __forceinline__ void gur2(C &x0, C &x1, R m0, R m1, R m2, R m3, R l0, R l1, R l2, R l3) {\n"
         "  const C a = x0, b = x1;\n"
         "  C r0, r1;\n"
         "  r0.x = FMA(m0, a.x, FMA(m1, b.x, FMA(l0, a.x, l1 * b.x)));\n"
         "  r0.y = FMA(m0, a.y, FMA(m1, b.y, FMA(l0, a.y, l1 * b.y)));\n"
         "  r1.x = FMA(m2, a.x, FMA(m3, b.x, FMA(l2, a.x, l3 * b.x)));\n"
         "  r1.y = FMA(m2, a.y, FMA(m3, b.y, FMA(l2, a.y, l3 * b.y)));\n"
         "  x0 = r0;\n  x1 = r1;\n}\n";
    o << "__device__ __forceinline__ void proj(C &x, R c, R si) {\n"
         "  const C a = x;\n"
         "  C r;\n"
         "  r.x = FMA(a.x, c, -a.y * si);\n"
         "  r.y = FMA(a.x, si, a.y * c);\n"
         "  x = r;\n}\n";
    return o.str();
}

// Kernel body (between the braces) of tile pass `pi`, and its parameter base;
// `persistent` selects the form that walks the tiles with a prefetch.
std::string jit_pass_body(const sv_plan &p, uint32_t pi, uint32_t *param_base, bool persistent)
{
    const TilePass &P = p.passes[pi];
    uint32_t lo = p.stages[P.stage_begin].op_begin;
    const uint32_t pb = lo * (uint32_t)kParamStride;
    Gen g(p, P, pb);
    g.body(persistent);
    if (param_base) *param_base = pb;
    return (persistent ? "// persistent\n" : "") + g.o.str();
}

// Full kernel definition named `name` around a body of jit_pass_body; the
// persistent form takes the tile count as a third argument.
std::string jit_kernel(const std::string &name, const std::string &body, int threads, bool persistent)
{
    std::ostringstream o;
    o << "extern \"C\" __global__ void __launch_bounds__(" << threads << ") " << name
      << "(C *__restrict__ psi, const R *__restrict__ prm" << (persistent ? ", const u64 n_tiles" : "") << ") {\n"
      << body << "}\n";
    return o.str();
}

}  // namespace svi
