// Fused tile-pass kernel: one HBM read and one HBM write of the state for a
// whole run of gates.
//
// Workgroup = one tile = the 2^b amplitudes that agree on the n-b tile qubits.
// Thread count 2^(b-RB); each thread keeps 2^RB amplitudes in registers.
//   load   : register slot s <- local index (s << nthr) | tid   (coalesced on the
//            lowest local qubits, which are the lowest qubits of the index)
//   stages : gates on register bits run in registers (unrolled per slot bit);
//            between stages the tile goes through LDS, where permutation gates
//            are applied to the write address
//   store  : back through the load mapping
// Gate conditions are split into a local part (checked per amplitude on the
// local index) and a tile part (uniform per workgroup: the whole gate is
// skipped when it fails).

#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <utility>

#include "state_access.h"
#include "sv_internal.h"

namespace svi {

template <typename R> struct CTT;
template <> struct CTT<float> { using T = float2; static constexpr int LOWB = 4; };
template <> struct CTT<double> { using T = double2; static constexpr int LOWB = 4; };  // 8-byte halves in LDS


// LDS element at byte offset `off` (the swizzle XOR is done on byte offsets:
// shifting the uniform slot part happens in scalar registers, so each access
// costs the one vector XOR with the thread part)
template <typename C>
__device__ __forceinline__ C &lds_at(C *lds, uint32_t off)
{
    return *reinterpret_cast<C *>(reinterpret_cast<unsigned char *>(lds) + off);
}

// Byte offset of the thread part of an LDS address, hidden from the
// optimiser: otherwise it rewrites (t << 3) ^ (s << 3) as ((t ^ s) << 3) with
// the swizzle term XORed in separately, three vector ops per access instead of
// one.  The empty asm only pins the value in a register.
__device__ __forceinline__ uint32_t opaque_offset(uint32_t v)
{
    asm volatile("" : "+v"(v));
    return v;
}

template <typename C, typename R>
__device__ __forceinline__ C row2(R ar, R ai, R br, R bi, C a, C b)
{
    C r;
    r.x = fma(ar, a.x, fma(-ai, a.y, fma(br, b.x, -bi * b.y)));
    r.y = fma(ar, a.y, fma(ai, a.x, fma(br, b.y, bi * b.x)));
    return r;
}

// First word of an op record (kind, slot, a, b), read whole: sub-dword fields
// would be fetched with per-lane vector loads (there are no 8- or 16-bit
// scalar loads), whose waits also drain every older vector load in flight.
__device__ __forceinline__ uint32_t op_head(const TileOp *op)
{
    const void *src = __builtin_assume_aligned(op, 8);
    uint32_t w;
    __builtin_memcpy(&w, src, sizeof(w));
    return w;
}

// The permutations of an LDS exchange applied to the local index l[s] of every
// register slot.  The op records are read once per op, outside any per-lane
// branch (so as scalar loads), and each slot is updated without branches.
template <int NR>
__device__ __forceinline__ void apply_perms(uint32_t (&l)[NR], const TileOp *__restrict__ perms, uint32_t pb,
                                            uint32_t pe, uint64_t base)
{
    for (uint32_t k = pb; k < pe; ++k) {
        const TileOp &p = perms[k];
        if ((base & p.gmask) != p.gval) continue;
        const uint32_t lmask = p.lmask, lval = p.lval;
        const uint32_t head = op_head(&p);
        const uint32_t kind = head & 0xffu, pa = (head >> 16) & 0xffu, pbits = head >> 24;
        switch (kind) {
        case T_INC:
        case T_DEC: {
            const uint32_t m = ((1u << pbits) - 1u) << pa;
            const uint32_t step = (kind == T_INC ? 1u : (uint32_t)-1) << pa;
#pragma unroll
            for (int s = 0; s < NR; ++s) {
                const uint32_t v = ((l[s] & m) + step) & m;
                l[s] = ((l[s] & lmask) == lval) ? ((l[s] & ~m) | v) : l[s];
            }
            break;
        }
        case T_SWAP: {
            const uint32_t a = pa, b = pbits, both = (1u << a) | (1u << b);
#pragma unroll
            for (int s = 0; s < NR; ++s) {
                const bool hit = ((l[s] & lmask) == lval) && ((((l[s] >> a) ^ (l[s] >> b)) & 1u) != 0u);
                l[s] = hit ? (l[s] ^ both) : l[s];
            }
            break;
        }
        case T_XFLIP: {
            const uint32_t f = 1u << pa;
#pragma unroll
            for (int s = 0; s < NR; ++s) l[s] = ((l[s] & lmask) == lval) ? (l[s] ^ f) : l[s];
            break;
        }
        default:
            break;
        }
    }
}

// Register-level ops: slot s (with the target slot bit clear) is processed when
// bit s of the uniform slotmask is set; the thread part of the condition has
// already been applied by the caller.
template <int K, int NR, bool FULL, typename C, typename R>
__device__ __forceinline__ void reg_u(C (&x)[NR], const R *m, uint32_t slotmask)
{
#pragma unroll
    for (int s = 0; s < NR; ++s) {
        if (s & (1 << K)) continue;
        if (!FULL && !((slotmask >> s) & 1u)) continue;
        const int s1 = s | (1 << K);
        const C a = x[s], b = x[s1];
        x[s] = row2(m[0], m[1], m[2], m[3], a, b);
        x[s1] = row2(m[4], m[5], m[6], m[7], a, b);
    }
}

template <int K, int NR, bool FULL, typename C, typename R>
__device__ __forceinline__ void reg_ur(C (&x)[NR], const R *m, uint32_t slotmask)
{
#pragma unroll
    for (int s = 0; s < NR; ++s) {
        if (s & (1 << K)) continue;
        if (!FULL && !((slotmask >> s) & 1u)) continue;
        const int s1 = s | (1 << K);
        const C a = x[s], b = x[s1];
        C r0, r1;
        r0.x = fma(m[0], a.x, m[1] * b.x);
        r0.y = fma(m[0], a.y, m[1] * b.y);
        r1.x = fma(m[2], a.x, m[3] * b.x);
        r1.y = fma(m[2], a.y, m[3] * b.y);
        x[s] = r0;
        x[s1] = r1;
    }
}

// T_UR2: the real matrix as hi m[0..3] + lo m[4..7]
template <int K, int NR, bool FULL, typename C, typename R>
__device__ __forceinline__ void reg_ur2(C (&x)[NR], const R *m, uint32_t slotmask)
{
#pragma unroll
    for (int s = 0; s < NR; ++s) {
        if (s & (1 << K)) continue;
        if (!FULL && !((slotmask >> s) & 1u)) continue;
        const int s1 = s | (1 << K);
        const C a = x[s], b = x[s1];
        C r0, r1;
        r0.x = fma(m[0], a.x, fma(m[1], b.x, fma(m[4], a.x, m[5] * b.x)));
        r0.y = fma(m[0], a.y, fma(m[1], b.y, fma(m[4], a.y, m[5] * b.y)));
        r1.x = fma(m[2], a.x, fma(m[3], b.x, fma(m[6], a.x, m[7] * b.x)));
        r1.y = fma(m[2], a.y, fma(m[3], b.y, fma(m[6], a.y, m[7] * b.y)));
        x[s] = r0;
        x[s1] = r1;
    }
}

template <int K, int NR, bool FULL, typename C>
__device__ __forceinline__ void reg_x(C (&x)[NR], uint32_t slotmask)
{
#pragma unroll
    for (int s = 0; s < NR; ++s) {
        if (s & (1 << K)) continue;
        if (!FULL && !((slotmask >> s) & 1u)) continue;
        const int s1 = s | (1 << K);
        const C a = x[s];
        x[s] = x[s1];
        x[s1] = a;
    }
}

#define SV_SLOT_DISPATCH1(FN, F, ...)                                   \
    switch (op.slot) {                                                  \
    case 0: FN<0, NR, F>(__VA_ARGS__); break;                           \
    case 1: FN<1, NR, F>(__VA_ARGS__); break;                           \
    case 2: FN<2, NR, F>(__VA_ARGS__); break;                           \
    case 3: FN<3, NR, F>(__VA_ARGS__); break;                           \
    default:                                                            \
        if constexpr (RB > 4) FN<(RB > 4 ? 4 : 0), NR, F>(__VA_ARGS__); \
        break;                                                          \
    }
// ops whose condition holds on every register slot skip the per-slot tests
#define SV_SLOT_DISPATCH(FN, ...)                                       \
    if (op.slotmask == kAllSlots) {                                     \
        SV_SLOT_DISPATCH1(FN, true, __VA_ARGS__)                        \
    } else {                                                            \
        SV_SLOT_DISPATCH1(FN, false, __VA_ARGS__)                       \
    }

// Absolute index bits of a tile (uniform): bit runs of the tile counter.
__device__ __forceinline__ uint64_t tile_base(const TilePass *__restrict__ pass, uint64_t tile)
{
    uint64_t base = 0;
    for (uint32_t r = 0; r < pass->n_tile_runs; ++r) {
        const uint32_t sh = pass->tile_shift[r];
        base |= ((tile >> (sh & 0xffu)) & pass->tile_mask[r]) << (sh >> 8);
    }
    return base;
}

// Load mapping: thread bits = local bits [0, nthr), slots = local bits [nthr, b).
__device__ __forceinline__ uint64_t tile_thread_offset(const TilePass *__restrict__ pass, uint32_t tid)
{
    uint64_t gthr = 0;
    for (uint32_t r = 0; r < pass->n_gthr_runs; ++r) {
        const uint32_t sh = pass->gthr_shift[r];
        gthr |= (uint64_t)((tid >> (sh & 0xffu)) & pass->gthr_mask[r]) << (sh >> 8);
    }
    return gthr;
}

// One complex128 exchange in two halves through an LDS array of doubles: the
// real parts (write at byte offsets wa[s], barrier, read at tr ^ 8 swz[s]),
// then the imaginary parts the same way.  The caller has passed the barrier
// that ends the previous use of the LDS.
// Write offsets come from `wr(s)` (recomputed or looked up, as the caller
// chooses); the new real part lands in x[s].x once the old one is in LDS.
template <int NR, typename W>
__device__ __forceinline__ void exchange_halves(double2 (&x)[NR], unsigned char *lds, W wr, uint32_t tr,
                                                const uint32_t *__restrict__ swz)
{
#pragma unroll
    for (int s = 0; s < NR; ++s) *reinterpret_cast<double *>(lds + wr(s)) = x[s].x;
    __syncthreads();
#pragma unroll
    for (int s = 0; s < NR; ++s) x[s].x = *reinterpret_cast<const double *>(lds + (tr ^ (swz[s] * 8u)));
    __syncthreads();
#pragma unroll
    for (int s = 0; s < NR; ++s) *reinterpret_cast<double *>(lds + wr(s)) = x[s].y;
    __syncthreads();
#pragma unroll
    for (int s = 0; s < NR; ++s) x[s].y = *reinterpret_cast<const double *>(lds + (tr ^ (swz[s] * 8u)));
}

// The register stages and LDS exchanges of one tile, on amplitudes already in
// registers (load mapping in, load mapping out).  Every thread of the
// workgroup calls this.  Every pointer comes straight from kernel arguments
// (plus uniform offsets), so the compiler knows the address spaces and reads
// the plan tables with scalar loads; pointers read from memory would turn
// those into per-lane flat loads.
template <typename R, int RB, bool GR = false>
__device__ __forceinline__ void tile_compute(typename CTT<R>::T (&x)[1 << RB],
                                             const TilePass *__restrict__ pass,
                                             const TileStage *__restrict__ stages,
                                             const TileOp *__restrict__ ops, const R *__restrict__ prm,
                                             uint64_t base, bool final_exchange, typename CTT<R>::T *lds)
{
    using C = typename CTT<R>::T;
    constexpr int NR = 1 << RB;
    constexpr int LOWB = CTT<R>::LOWB;
    constexpr int PG = (NR == 16) ? 16 : 4;  // slots per permutation group
    constexpr uint32_t kAllSlots = (NR >= 32) ? 0xffffffffu : ((1u << NR) - 1u);

    const uint32_t tid = threadIdx.x;
    // current mapping: local index of slot s = thr | regoff[s] (disjoint bits);
    // the LDS swizzle is GF(2)-linear, so its slot part comes precomputed
    uint32_t thr = tid;
    const uint32_t se = pass->stage_end;
    for (uint32_t st = pass->stage_begin; st < se; ++st) {
        const TileStage &S = stages[st];
        if (st != pass->stage_begin) {
            const TileStage &P = stages[st - 1];
            __syncthreads();
            if constexpr (sizeof(R) == 8) {
                // complex128: the real parts go through LDS, then the imaginary
                // parts, in an array of doubles half the tile's size, so that
                // three workgroups share a CU where whole amplitudes allow two
                uint32_t t2 = 0;
                for (uint32_t r = 0; r < S.n_thr_runs; ++r) {
                    const uint32_t w = S.thr_run[r];
                    t2 |= ((tid >> (w & 0xffu)) & (w >> 16)) << ((w >> 8) & 0xffu);
                }
                const uint32_t tr = opaque_offset(lds_swizzle(t2, LOWB) * 8u);
                unsigned char *const lb = reinterpret_cast<unsigned char *>(lds);
                if (S.perm_begin == S.perm_end) {
                    const uint32_t tw = opaque_offset(lds_swizzle(thr, LOWB) * 8u);
                    exchange_halves<NR>(x, lb, [&](int s) { return tw ^ (P.swz[s] * 8u); }, tr, S.swz);
                } else {
                    uint32_t wa[NR];
#pragma unroll
                    for (int g = 0; g < NR; g += PG) {
                        uint32_t l[PG];
#pragma unroll
                        for (int s = 0; s < PG; ++s) l[s] = thr | P.regoff[g + s];
                        apply_perms<PG>(l, ops, S.perm_begin, S.perm_end, base);
#pragma unroll
                        for (int s = 0; s < PG; ++s) wa[g + s] = lds_swizzle(l[s], LOWB) * 8u;
                    }
                    exchange_halves<NR>(x, lb, [&](int s) { return wa[s]; }, tr, S.swz);
                }
                thr = t2;
            } else if (S.perm_begin == S.perm_end) {
                const uint32_t tw = opaque_offset(lds_swizzle(thr, LOWB) * (uint32_t)sizeof(C));
#pragma unroll
                for (int s = 0; s < NR; ++s) lds_at(lds, tw ^ (P.swz[s] * (uint32_t)sizeof(C))) = x[s];
            } else {
                // all 16 slot indices at once, so the permutation records are
                // walked once (measured faster even where the indices cost the
                // complex64 tile a wave of occupancy); 32-slot tiles in groups of 4
#pragma unroll
                for (int g = 0; g < NR; g += PG) {
                    uint32_t l[PG];
#pragma unroll
                    for (int s = 0; s < PG; ++s) l[s] = thr | P.regoff[g + s];
                    apply_perms<PG>(l, ops, S.perm_begin, S.perm_end, base);
#pragma unroll
                    for (int s = 0; s < PG; ++s) lds[lds_swizzle(l[s], LOWB)] = x[g + s];
                }
            }
            if constexpr (sizeof(R) == 4) {
                __syncthreads();
                uint32_t t2 = 0;
                for (uint32_t r = 0; r < S.n_thr_runs; ++r) {
                    const uint32_t w = S.thr_run[r];
                    t2 |= ((tid >> (w & 0xffu)) & (w >> 16)) << ((w >> 8) & 0xffu);
                }
                thr = t2;
                const uint32_t tr = opaque_offset(lds_swizzle(thr, LOWB) * (uint32_t)sizeof(C));
#pragma unroll
                for (int s = 0; s < NR; ++s) x[s] = lds_at(lds, tr ^ (S.swz[s] * (uint32_t)sizeof(C)));
            }
        }
        // op records are prefetched one ahead; parameters sit at a fixed stride,
        // so their loads do not wait for the record
        TileOp nxt;
        if (!GR && S.op_begin < S.op_end) nxt = ops[S.op_begin];
        uint32_t run_end = 0;  // gate runs: end of the run whose matching ops are being applied
        uint64_t run_v = 0;
        for (uint32_t k = S.op_begin; k < S.op_end; ++k) {
            TileOp op;
            if constexpr (GR) {
                // (record reads without the one-ahead prefetch, which the jumps
                // below would make per-lane; readfirstlane keeps the indices and
                // so the record reads scalar)
                op = ops[k];
                if (run_end != 0 && (k >= run_end || op.gval != run_v)) {
                    // the run's ops for this tile are done: continue after the run
                    k = __builtin_amdgcn_readfirstlane(run_end);
                    run_end = 0;
                    if (k >= S.op_end) break;
                    op = ops[k];
                }
                const uint32_t L = (uint32_t)op.a | ((uint32_t)op.b << 8);
                if (run_end == 0 && L >= 2 && op.kind != T_PROJ) {
                    // ops k .. k + L - 1 share op's tile mask, sorted by tile value:
                    // bisect for the first whose value is this tile's
                    const uint64_t v = base & op.gmask;
                    uint32_t lo = k, hi = k + L;
                    while (lo < hi) {
                        const uint32_t mid = __builtin_amdgcn_readfirstlane((lo + hi) >> 1);
                        if (ops[mid].gval < v) lo = mid + 1; else hi = mid;
                    }
                    if (lo >= k + L || ops[lo].gval != v) {  // no op of the run acts on this tile
                        k += L - 1;
                        continue;
                    }
                    run_end = k + L;
                    run_v = v;
                    k = __builtin_amdgcn_readfirstlane(lo);
                    op = ops[k];
                }
            } else {
                op = nxt;
                if (k + 1 < S.op_end) nxt = ops[k + 1];
            }
            const R *__restrict__ pk = prm + (size_t)k * kParamStride;
            // tile condition first: a uniform branch taken before any per-lane work
            const bool zg = (base & op.gmask) == op.gval;
            if (!zg && op.kind != T_PROJ) continue;
            const bool tc = (tid & op.tidmask) == op.tidval;
            if (op.kind == T_PROJ) {
                const R c = pk[0], sn = pk[1];
                const uint32_t sig_thread = op.a == 2 ? ((tid >> op.b) & 1u) : 0u;
                const uint32_t sig_tile = op.a == 0 ? (uint32_t)((base >> op.b) & 1ull) : 0u;
#pragma unroll
                for (int s = 0; s < NR; ++s) {
                    const uint32_t z = (zg && tc && ((op.slotmask >> s) & 1u)) ? 1u : 0u;
                    const uint32_t sig_slot = op.a == 1 ? (((uint32_t)s >> op.b) & 1u) : 0u;
                    const R si = ((sig_thread ^ sig_tile ^ sig_slot) ^ z) ? -sn : sn;
                    const C a = x[s];
                    C r;
                    r.x = fma(a.x, c, -a.y * si);
                    r.y = fma(a.x, si, a.y * c);
                    x[s] = r;
                }
                continue;
            }
            if (!tc) continue;
            if (op.kind == T_U) {
                R m[8];
#pragma unroll
                for (int j = 0; j < 8; ++j) m[j] = pk[j];
                SV_SLOT_DISPATCH(reg_u, x, m, op.slotmask)
            } else if (op.kind == T_UR) {
                R m[4];
#pragma unroll
                for (int j = 0; j < 4; ++j) m[j] = pk[j];
                SV_SLOT_DISPATCH(reg_ur, x, m, op.slotmask)
            } else if (op.kind == T_UR2) {  // complex64 plans only
                R m[8];
#pragma unroll
                for (int j = 0; j < 8; ++j) m[j] = pk[j];
                SV_SLOT_DISPATCH(reg_ur2, x, m, op.slotmask)
            } else if (op.kind == T_X) {
                SV_SLOT_DISPATCH(reg_x, x, op.slotmask)
            } else if (op.kind == T_PHASE) {
                const R c = pk[0], sn = pk[1];
#pragma unroll
                for (int s = 0; s < NR; ++s) {
                    if (!((op.slotmask >> s) & 1u)) continue;
                    const C a = x[s];
                    C r;
                    r.x = fma(a.x, c, -a.y * sn);
                    r.y = fma(a.x, sn, a.y * c);
                    x[s] = r;
                }
            }
        }
    }

    if (final_exchange) {
        const TileStage &L = stages[se - 1];
        __syncthreads();
        if constexpr (sizeof(R) == 8) {
            const uint32_t tr = opaque_offset(lds_swizzle(tid, LOWB) * 8u);
            unsigned char *const lb = reinterpret_cast<unsigned char *>(lds);
            if (pass->fperm_begin == pass->fperm_end) {
                const uint32_t tw = opaque_offset(lds_swizzle(thr, LOWB) * 8u);
                exchange_halves<NR>(x, lb, [&](int s) { return tw ^ (L.swz[s] * 8u); }, tr, pass->swz0);
            } else {
                uint32_t wa[NR];
#pragma unroll
                for (int g = 0; g < NR; g += PG) {
                    uint32_t l[PG];
#pragma unroll
                    for (int s = 0; s < PG; ++s) l[s] = thr | L.regoff[g + s];
                    apply_perms<PG>(l, ops, pass->fperm_begin, pass->fperm_end, base);
#pragma unroll
                    for (int s = 0; s < PG; ++s) wa[g + s] = lds_swizzle(l[s], LOWB) * 8u;
                }
                exchange_halves<NR>(x, lb, [&](int s) { return wa[s]; }, tr, pass->swz0);
            }
            return;
        }
        if (pass->fperm_begin == pass->fperm_end) {
            const uint32_t tw = opaque_offset(lds_swizzle(thr, LOWB) * (uint32_t)sizeof(C));
#pragma unroll
            for (int s = 0; s < NR; ++s) lds_at(lds, tw ^ (L.swz[s] * (uint32_t)sizeof(C))) = x[s];
        } else {
#pragma unroll
            for (int g = 0; g < NR; g += PG) {
                uint32_t l[PG];
#pragma unroll
                for (int s = 0; s < PG; ++s) l[s] = thr | L.regoff[g + s];
                apply_perms<PG>(l, ops, pass->fperm_begin, pass->fperm_end, base);
#pragma unroll
                for (int s = 0; s < PG; ++s) lds[lds_swizzle(l[s], LOWB)] = x[g + s];
            }
        }
        __syncthreads();
        const uint32_t tr = opaque_offset(lds_swizzle(tid, LOWB) * (uint32_t)sizeof(C));
#pragma unroll
        for (int s = 0; s < NR; ++s) x[s] = lds_at(lds, tr ^ (pass->swz0[s] * (uint32_t)sizeof(C)));
    }
}

// The pass's final-exchange flag, read as a whole aligned word (the flag and
// its padding at offset 20) before any barrier, so that it is a scalar load.
__device__ __forceinline__ bool pass_final_exchange(const TilePass *__restrict__ pass)
{
    uint32_t w;
    __builtin_memcpy(&w, __builtin_assume_aligned(&pass->final_exchange, 4), sizeof(w));
    return (w & 0xffu) != 0u;
}

// One tile of one pass: load, register stages with LDS exchanges, store.
template <typename R, int RB, bool GR = false, bool NT = false>
__device__ __forceinline__ void tile_pass_body(typename CTT<R>::T *__restrict__ psi,
                                               const TilePass *__restrict__ pass,
                                               const TileStage *__restrict__ stages,
                                               const TileOp *__restrict__ ops, const R *__restrict__ prm,
                                               uint64_t tile, typename CTT<R>::T *lds)
{
    using C = typename CTT<R>::T;
    constexpr int NR = 1 << RB;
    const uint64_t base = tile_base(pass, tile);
    C *const pt = psi + (base | tile_thread_offset(pass, threadIdx.x));
    C x[NR];
#pragma unroll
    for (int s = 0; s < NR; ++s) x[s] = load_state<NT>(pt + pass->goff[s]);
    tile_compute<R, RB, GR>(x, pass, stages, ops, prm, base, pass_final_exchange(pass), lds);
#pragma unroll
    for (int s = 0; s < NR; ++s) store_state<NT>(pt + pass->goff[s], x[s]);
}

// Persistent form: each workgroup walks tiles blockIdx.x, + gridDim.x, ...
// and issues the loads of its next tile before computing the current one, so
// the HBM reads of one tile overlap the arithmetic of the previous one.  The
// tiles are disjoint, so the prefetch never reads what another tile writes.
// The first LDS exchange of every tile begins with a barrier, which orders it
// after the previous tile's last LDS reads.
template <typename R, int RB>
__global__ void __launch_bounds__(256)
k_tile_pass_pipe(typename CTT<R>::T *__restrict__ psi, const TilePass *__restrict__ pass,
                 const TileStage *__restrict__ stages, const TileOp *__restrict__ ops, const R *__restrict__ prm,
                 uint64_t n_tiles)
{
    using C = typename CTT<R>::T;
    constexpr int NR = 1 << RB;
    extern __shared__ unsigned char smem_raw[];
    C *const lds = reinterpret_cast<C *>(smem_raw);
    uint64_t tile = blockIdx.x;
    if (tile >= n_tiles) return;
    const uint64_t stride = gridDim.x;
    const uint64_t gthr = tile_thread_offset(pass, threadIdx.x);
    const bool fx = pass_final_exchange(pass);
    uint64_t base_next = tile_base(pass, tile);
    C xn[NR];
    {
        const C *const pn = psi + (base_next | gthr);
#pragma unroll
        for (int s = 0; s < NR; ++s) xn[s] = pn[pass->goff[s]];
    }
    for (;;) {
        C x[NR];
#pragma unroll
        for (int s = 0; s < NR; ++s) x[s] = xn[s];
        const uint64_t base = base_next;
        const uint64_t next = tile + stride;
        if (next < n_tiles) {
            base_next = tile_base(pass, next);
            const C *const pn = psi + (base_next | gthr);
#pragma unroll
            for (int s = 0; s < NR; ++s) xn[s] = pn[pass->goff[s]];
        }
        tile_compute<R, RB>(x, pass, stages, ops, prm, base, fx, lds);
        C *const pt = psi + (base | gthr);
#pragma unroll
        for (int s = 0; s < NR; ++s) pt[pass->goff[s]] = x[s];
        if (next >= n_tiles) break;
        tile = next;
    }
}

// GR: the pass holds gate runs (a separate instantiation, so passes without
// them keep the plain op loop with its one-ahead record prefetch).  NT: the
// pass's `stream` flag (nontemporal state loads and stores).
template <typename R, int RB, bool GR, bool NT>
__global__ void __launch_bounds__(256)
k_tile_pass(typename CTT<R>::T *__restrict__ psi, const TilePass *__restrict__ pass,
            const TileStage *__restrict__ stages, const TileOp *__restrict__ ops, const R *__restrict__ prm)
{
    using C = typename CTT<R>::T;
    extern __shared__ unsigned char smem_raw[];
    const uint64_t tile = (uint64_t)blockIdx.x + (uint64_t)blockIdx.y * gridDim.x;
    tile_pass_body<R, RB, GR, NT>(psi, pass, stages, ops, prm, tile, reinterpret_cast<C *>(smem_raw));
}

// Batched tile passes: one launch runs pass `level` of every instance of a
// group.  The batch owns one concatenated copy of its plans' tables (indices
// rebased) and its states live in one arena, so an item is only offsets:
// the state's first amplitude in the arena, its pass in the table and its first
// work index.  Workgroup w finds its item by binary search over item_begin and
// runs that tile.  Instances of a launch share the geometry (b, RB).
template <typename R, int RB, bool GR, bool NT>
__global__ void __launch_bounds__(256)
k_tile_batch(typename CTT<R>::T *__restrict__ arena, const TilePass *__restrict__ passes,
             const TileStage *__restrict__ stages, const TileOp *__restrict__ ops, const R *__restrict__ prm,
             const BatchItem *__restrict__ items, uint32_t n_items, uint64_t total)
{
    using C = typename CTT<R>::T;
    extern __shared__ unsigned char smem_raw[];
    const uint64_t w = (uint64_t)blockIdx.x + (uint64_t)blockIdx.y * gridDim.x;
    if (w >= total) return;  // padding of the last grid row: the whole workgroup leaves together
    uint32_t lo = 0, hi = n_items;  // last item with item_begin <= w
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (items[mid].item_begin <= w) lo = mid; else hi = mid;
    }
    const BatchItem &B = items[lo];
    tile_pass_body<R, RB, GR, NT>(arena + B.psi_off, passes + B.pass_index, stages, ops, prm, w - B.item_begin,
                                  reinterpret_cast<C *>(smem_raw));
}

// Resident workgroups of the persistent kernel on the whole device, cached per
// (kernel, block, LDS) shape.
template <typename R, int RB>
static uint64_t pipe_grid(uint32_t block, size_t lds)
{
    static std::mutex mu;
    static std::map<std::pair<uint32_t, size_t>, uint64_t> cache;
    std::lock_guard<std::mutex> lk(mu);
    const auto key = std::make_pair(block, lds);
    auto it = cache.find(key);
    if (it != cache.end()) return it->second;
    int dev = 0, cus = 256, per_cu = 1;
    if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)k_tile_pass_pipe<R, RB>, (int)block,
                                                     lds) != hipSuccess || per_cu < 1)
        per_cu = 1;
    (void)hipGetLastError();
    const uint64_t g = (uint64_t)cus * (uint64_t)per_cu;
    cache[key] = g;
    return g;
}

template <typename R, int RB>
static int launch_tile_t(const sv_plan *p, uint32_t pi, void *psi, hipStream_t st)
{
    using C = typename CTT<R>::T;
    const TilePass &P = p->passes[pi];
    const uint64_t tiles = 1ull << P.ntile;
    if (p->tile_launch == SV_TILE_LAUNCH_PERSISTENT) {
        const uint32_t block = 1u << P.nthr;
        const size_t lds = (size_t)8 << P.b;  // 8 bytes per amplitude: a complex64, or half a complex128
        const uint64_t g = std::min<uint64_t>(tiles, pipe_grid<R, RB>(block, lds));
        hipLaunchKernelGGL((k_tile_pass_pipe<R, RB>), dim3((uint32_t)g), dim3(block), lds, st, (C *)psi,
                           (const TilePass *)p->d_passes + pi, (const TileStage *)p->d_stages,
                           (const TileOp *)p->d_tops, (const R *)p->d_tparams, tiles);
        return hipGetLastError() == hipSuccess ? SV_OK : SV_EDEVICE;
    }
    const uint32_t gx = tiles > 65536 ? 65536u : (uint32_t)tiles;
    const uint32_t gy = (uint32_t)(tiles / gx);
    const dim3 grid(gx, gy);
    const dim3 block(1u << P.nthr);
    const size_t lds = (size_t)8 << P.b;
    auto go = [&](auto kernel) {
        hipLaunchKernelGGL(kernel, grid, block, lds, st, (C *)psi, (const TilePass *)p->d_passes + pi,
                           (const TileStage *)p->d_stages, (const TileOp *)p->d_tops, (const R *)p->d_tparams);
    };
    if (P.gate_runs)
        P.stream ? go(k_tile_pass<R, RB, true, true>) : go(k_tile_pass<R, RB, true, false>);
    else
        P.stream ? go(k_tile_pass<R, RB, false, true>) : go(k_tile_pass<R, RB, false, false>);
    return hipGetLastError() == hipSuccess ? SV_OK : SV_EDEVICE;
}

template <typename R, int RB>
static int launch_batch_t(const BatchTables &T, const BatchItem *d_items, uint32_t n_items, uint64_t total,
                          bool gate_runs, bool stream, hipStream_t st)
{
    using C = typename CTT<R>::T;
    const uint32_t gx = total > 65536 ? 65536u : (uint32_t)total;
    const uint64_t gy = (total + gx - 1) / gx;
    if (gy > 65535) return SV_EUNSUPPORTED;
    auto go = [&](auto kernel) {
        hipLaunchKernelGGL(kernel, dim3(gx, (uint32_t)gy), dim3(1u << T.nthr), (size_t)8 << T.b, st, (C *)T.arena,
                           (const TilePass *)T.passes, (const TileStage *)T.stages, (const TileOp *)T.ops,
                           (const R *)T.prm, d_items, n_items, total);
    };
    // a level holding gate runs takes the bisecting instantiation (it runs every
    // other pass of the level correctly too, without the record prefetch)
    if (gate_runs)
        stream ? go(k_tile_batch<R, RB, true, true>) : go(k_tile_batch<R, RB, true, false>);
    else
        stream ? go(k_tile_batch<R, RB, false, true>) : go(k_tile_batch<R, RB, false, false>);
    return hipGetLastError() == hipSuccess ? SV_OK : SV_EDEVICE;
}

int launch_tile_batch(const BatchTables &T, const BatchItem *d_items, uint32_t n_items, uint64_t total_work,
                      bool gate_runs, bool stream, hipStream_t st)
{
    if (!n_items || !total_work) return SV_OK;
    if (T.dtype == SV_C64)
        return T.rb == 5 ? launch_batch_t<float, 5>(T, d_items, n_items, total_work, gate_runs, stream, st)
                         : launch_batch_t<float, 4>(T, d_items, n_items, total_work, gate_runs, stream, st);
    return T.rb == 5 ? launch_batch_t<double, 5>(T, d_items, n_items, total_work, gate_runs, stream, st)
                     : launch_batch_t<double, 4>(T, d_items, n_items, total_work, gate_runs, stream, st);
}

int launch_tile_pass(const sv_plan *p, uint32_t pi, void *psi, hipStream_t st)
{
    if (p->dtype == SV_C64)
        return p->rb == 5 ? launch_tile_t<float, 5>(p, pi, psi, st) : launch_tile_t<float, 4>(p, pi, psi, st);
    return p->rb == 5 ? launch_tile_t<double, 5>(p, pi, psi, st) : launch_tile_t<double, 4>(p, pi, psi, st);
}

template <typename R, int RB>
static void set_lds_limit(int bytes)
{
    const void *const kernels[] = {
        (const void *)k_tile_pass<R, RB, false, false>, (const void *)k_tile_pass<R, RB, false, true>,
        (const void *)k_tile_pass<R, RB, true, false>,  (const void *)k_tile_pass<R, RB, true, true>,
        (const void *)k_tile_batch<R, RB, false, false>, (const void *)k_tile_batch<R, RB, false, true>,
        (const void *)k_tile_batch<R, RB, true, false>,  (const void *)k_tile_batch<R, RB, true, true>,
        (const void *)k_tile_pass_pipe<R, RB>};
    for (const void *k : kernels) (void)hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
}

// LDS above 64 KiB per workgroup must be requested per kernel.  A refusal is
// not fatal: a launch that then exceeds the limit fails with a runtime error.
int tile_kernel_setup()
{
    const int big = 160 * 1024;
    set_lds_limit<float, 4>(big);
    set_lds_limit<float, 5>(big);
    set_lds_limit<double, 4>(big);
    set_lds_limit<double, 5>(big);
    (void)hipGetLastError();
    return SV_OK;
}

}  // namespace svi
