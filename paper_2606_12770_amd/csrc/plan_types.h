// Plan structures of libsv shared by the planner (host) and the kernels.
// Free of HIP types so host-only code can include it.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "sv.h"

namespace svi {

// ---------------------------------------------------------------------------
// Fused tile passes.
//
// A tile pass keeps b "local" qubits of the index resident on chip: one
// workgroup loads the 2^b amplitudes that share the values of the other n-b
// ("tile") qubits, applies a whole run of gates to them, and writes them back
// once.  Local qubit k of a pass is qubit spos[k] (ascending), so local bit
// positions preserve the order of the qubits.
//
// Inside the workgroup each thread holds 2^RB amplitudes in registers.  A
// "stage" fixes which RB local bits index the register slots (regoff[s] is the
// local index offset of slot s) and which b-RB local bits index the thread
// (thrpos).  Gates whose target is a register bit are applied in registers;
// moving to the next stage exchanges the tile through LDS, and permutation
// gates (INC/DEC/SWAP/X on local bits) are applied to the LDS address during
// that exchange.
// ---------------------------------------------------------------------------

enum : uint8_t {
    T_U = 0,      // complex 2x2 matrix on register slot bit `slot` (8 reals)
    T_X = 1,      // exchange on register slot bit `slot`
    T_PHASE = 2,  // diagonal phase (cos, sin) where the condition holds
    T_PROJ = 3,   // projector phase (cos, sin); signal: a = 0 tile qubit b,
                  // a = 1 register slot bit b, a = 2 thread bit b
    T_INC = 4,    // permutation: local register [a, a+b) += 1
    T_DEC = 5,    // permutation: local register [a, a+b) -= 1
    T_SWAP = 6,   // permutation: exchange local bits a and b
    T_XFLIP = 7,  // permutation: flip local bit a
    T_UR = 8,     // real 2x2 matrix on register slot bit `slot` (4 reals)
    T_UR2 = 9,    // the same, complex64 only, as hi (reals 0-3) + lo (reals 4-7)
};

// SV_SPLIT_REAL_AUTO splits the real gates of a complex64 plan when the sum of
// their FP32 matrices' column-norm errors exceeds this bound.
constexpr double kSplitRealBound = 1e-4;

// Conditions of register-level ops are pre-split for the stage they run in:
//   slotmask bit s : the register-slot part of the condition holds for slot s
//   (tid & tidmask) == tidval : the thread part holds
//   (tile base & gmask) == gval : the tile part holds (uniform)
// Permutations keep the condition on the whole local index (lmask, lval).
// Gate runs: in a pass with gate_runs set, a register op or T_PHASE whose
// (a | b << 8) = L >= 2 heads a run of L consecutive ops of its stage that share
// its tile mask (gmask) and are sorted by tile value (gval); none is a T_PROJ.
// A tile applies only the ops of the run whose gval is its own, so it can find
// them by bisection and pass over the rest.  (Ops with different tile values
// never act in the same tile, so sorting them changes nothing.)
struct TileOp {
    uint8_t kind;
    uint8_t slot;
    uint8_t a;
    uint8_t b;
    uint32_t param;   // offset (in reals) into the plan's parameter array
    uint32_t slotmask;
    uint16_t tidmask;
    uint16_t tidval;
    uint32_t lmask;
    uint32_t lval;
    uint64_t gmask;
    uint64_t gval;
};
static_assert(sizeof(TileOp) == 40, "TileOp layout");

constexpr int kMaxRB = 5;
constexpr int kMaxB = 14;
constexpr int kMaxThrRuns = 10;  // runs of up to nine thread bits (512 threads)
constexpr int kMaxTileRuns = 16;
constexpr int kParamStride = 8;
constexpr int kDefaultTileLaunch = SV_TILE_LAUNCH_GRID;  // what SV_TILE_LAUNCH_AUTO resolves to  // reals of parameters reserved per tile op (op k at k * 8)

// LDS placement of local index l: XOR-fold the higher bits into the lowest
// `lowb` bits so that threads strided by any power of two hit different banks.
// GF(2)-linear, so swz(a | b) = swz(a) ^ swz(b) for disjoint a, b: the planner
// stores swz(register offset) per slot and the kernel XORs in swz(thread part).
constexpr uint32_t lds_swizzle(uint32_t l, int lowb)
{
    const uint32_t h = (l >> lowb) ^ (l >> (2 * lowb)) ^ (l >> (3 * lowb)) ^ (l >> (4 * lowb));
    return l ^ (h & ((1u << lowb) - 1u));
}

// A run of consecutive source bits moved as one block: out |= ((in >> src) & mask) << dst.
// Thread-to-local runs pack (src, dst, mask) into one word: src | dst << 8 | mask << 16.
constexpr uint32_t pack_run16(uint32_t src, uint32_t dst, uint32_t mask) { return src | (dst << 8) | (mask << 16); }

struct TileStage {
    uint32_t op_begin, op_end;      // register-level ops of the stage
    uint32_t perm_begin, perm_end;  // permutations applied on entry to the stage
    uint32_t n_thr_runs;            // thread bits -> local bits, as runs
    uint32_t thr_run[kMaxThrRuns];
    uint32_t swz[1 << kMaxRB];      // lds_swizzle(regoff[s])
    uint8_t thrpos[16];             // local bit index of thread bit j
    uint32_t regoff[1 << kMaxRB];   // local index offset of register slot s (32-bit: read with scalar loads)
};

// Whether tile passes stream a state of `bytes` (all the states of a batched
// level together) with nontemporal loads and stores.  16 MiB or less, or
// 256 MiB or more, takes the hint; a state in between stays in the last-level
// cache from pass to pass, and the hint would send it back to HBM.  Measured on
// MI355X: the 19-qubit first-order ladders (4 and 8 MiB) 4-10% faster with it,
// the 28- and 31-qubit circuits (2 and 16 GiB) 2% faster, the 23-qubit
// second-order ladder (64 and 128 MiB) 3-7% slower.
inline bool stream_state_bytes(uint64_t bytes)
{
    return bytes <= (16ull << 20) || bytes >= (256ull << 20);
}

struct TilePass {
    uint32_t stage_begin, stage_end;
    uint32_t fperm_begin, fperm_end;  // permutations on the final exchange
    uint8_t b, rb, nthr, ntile;
    uint8_t final_exchange;           // 1: exchange back to the load mapping before the store
    uint8_t gate_runs;                // 1: some stage holds gate runs (see TileOp)
    uint8_t stream;                   // 1: state loads and stores carry the nontemporal hint
    uint8_t pad[1];
    uint32_t n_tile_runs;             // tile counter bits -> absolute index bits, as runs
    uint32_t n_gthr_runs;             // thread bits -> absolute index bits (load mapping), as runs
    uint32_t tile_shift[kMaxTileRuns];  // src | dst << 8
    uint64_t tile_mask[kMaxTileRuns];
    uint32_t gthr_shift[kMaxThrRuns];
    uint32_t gthr_mask[kMaxThrRuns];
    uint32_t swz0[1 << kMaxRB];       // lds_swizzle(s << nthr): load-mapping slots
    uint8_t spos[kMaxB];              // local bit -> qubit
    uint8_t pad2[2];
    uint8_t tpos[48];                 // tile bit -> qubit
    uint64_t goff[1 << kMaxRB];       // absolute index offset of load-mapping register slot s
};

// Runs of a bit map src bit j -> dst position pos[j] (pos ascending): each
// maximal stretch with pos[j+1] = pos[j] + 1 becomes one (src, dst, width).
template <typename F>
inline int bit_runs(const uint8_t *pos, int count, F &&emit)
{
    int runs = 0;
    int j = 0;
    while (j < count) {
        int w = 1;
        while (j + w < count && pos[j + w] == pos[j] + w) ++w;
        emit(j, (int)pos[j], w);
        ++runs;
        j += w;
    }
    return runs;
}

// ---------------------------------------------------------------------------
// Plain per-gate launches.
// ---------------------------------------------------------------------------
struct PlainOp {
    uint32_t kind;       // SV_OP_* (RY already turned into U)
    uint32_t target, width;
    uint64_t mask, val;
    double m[8];         // U matrix or phase angle in m[0]
};

struct Step {
    int type;            // 0 = plain op, 1 = tile pass, 2 = dense block pass
    uint32_t index;
};

// Dense k-qubit block (k = 5 or 6): the 2^12 amplitudes of a tile (the k block
// qubits and 12 - k others) go through LDS; a group is one value of the other
// local qubits, and every group's 2^k amplitudes are multiplied by the block
// matrix.  `map` carries the load/store mapping (spos, tpos, runs, goff, swz0)
// of a tile pass with b = 12 and 4 register qubits; its stage fields are unused.
constexpr int kMaxDenseK = 6;
struct DensePass {
    TilePass map;
    uint32_t k;                       // block qubits
    uint32_t mat;                     // offset (reals) of the matrix: (row i, column j), re, im
    uint32_t n_grp_runs;              // group index (12 - k bits) -> local offset, as pack_run16 runs
    uint32_t grp_run[kMaxThrRuns];
    uint32_t joff[1 << kMaxDenseK];   // local offset of block value j (bit k of j -> block qubit k)
};

// One instance of a batched launch: where its state starts in the arena (in
// amplitudes), the pass it runs at this level (index into the batch's
// concatenated pass table) and the first work index it owns.
struct BatchItem {
    uint64_t psi_off;
    uint64_t pass_index;
    uint64_t item_begin;
};
static_assert(sizeof(BatchItem) == 24, "BatchItem layout");

// Device tables shared by all launches of a batch.
struct BatchTables {
    void *arena;
    const void *passes, *stages, *ops, *prm;
    int dtype, b, rb, nthr;
};

}  // namespace svi



struct sv_plan {
    int n = 0;
    int dtype = SV_C64;
    int b = 0, rb = 0;
    int tile_launch = 1;              // SV_TILE_LAUNCH_GRID or SV_TILE_LAUNCH_PERSISTENT (resolved)
    std::vector<svi::Step> steps;
    std::vector<svi::PlainOp> plain;
    std::vector<svi::TilePass> passes;
    std::vector<svi::TileStage> stages;
    std::vector<svi::TileOp> tops;
    std::vector<double> tparams;      // host copy (double); converted on upload
    std::vector<svi::DensePass> dense;
    std::vector<double> dparams;      // dense block matrices (double); converted on upload
    void *d_passes = nullptr, *d_stages = nullptr, *d_tops = nullptr, *d_tparams = nullptr;
    void *d_dense = nullptr, *d_dparams = nullptr;
    int device = -1;
    sv_plan_info info{};
    // specialised tile-pass kernels (compiled plans): function per pass and
    // the pass's first parameter (reals into the device parameter array)
    bool compiled = false;
    bool dense_bf16 = false;          // complex64 dense blocks on BF16 matrix cores (split operands)
    int dense_k = 5;                  // qubits per dense block (5, or 6 for complex64)
    int refs = 1;                     // the caller's handle, plus each concurrent batch that runs it
    std::vector<void *> jit_fn;
    std::vector<uint32_t> jit_prm;
};

namespace svi {
// Builds steps/passes/stages/ops on the host; returns SV_OK or an error code.
int build_plan(sv_plan *p, const sv_op *ops, size_t n_ops, const double *params,
               const sv_apply_opts &opts, std::string &err);
// Complex64 copy of a plan's tile parameters: projector phases rounded so that
// the product of their norm factors stays next to 1, the rest to nearest.
std::vector<float> tile_params_c64(const std::vector<TileOp> &tops, const std::vector<double> &tparams);
}  // namespace svi
