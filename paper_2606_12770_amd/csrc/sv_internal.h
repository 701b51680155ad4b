// Internal declarations of libsv: device state and kernel launch wrappers.
#pragma once

#include <hip/hip_runtime.h>

#include "plan_types.h"

namespace svi {
struct Arena;  // shared device allocation of states made by sv_alloc_batch
}

struct sv_state {
    int n = 0;
    int dtype = SV_C64;
    void *d_psi = nullptr;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int device = 0;
    svi::Arena *arena = nullptr;  // non-null: d_psi lives in an arena, freed with its last state
};

namespace svi {

// kernels (launch wrappers), all on `stream`
int launch_plain(const PlainOp &op, int n, int dtype, void *psi, hipStream_t stream);
int launch_tile_pass(const sv_plan *p, uint32_t pass_index, void *psi, hipStream_t stream);
int launch_dense_pass(const sv_plan *p, uint32_t dense_index, void *psi, hipStream_t stream);
int launch_init_basis(void *psi, int n, int dtype, hipStream_t stream);
int launch_from_c128(void *psi, int dtype, const void *d_src, uint64_t offset, uint64_t count,
                     hipStream_t stream);
int launch_to_c128(const void *psi, int dtype, void *d_dst, uint64_t offset, uint64_t count,
                   hipStream_t stream);
int launch_prob(const void *psi, int n, int dtype, uint64_t mask, uint64_t val, double *d_partial,
                int max_blocks, double *d_out, hipStream_t stream);
int launch_keep_scale(void *psi, int n, int dtype, uint64_t mask, uint64_t val, double scale,
                      hipStream_t stream);
int launch_inner(const void *a, int dta, const void *b, int dtb, int n, double *d_partial,
                 int max_blocks, double *d_out, hipStream_t stream);
int launch_copy(void *dst, int dtd, const void *src, int dts, int n, hipStream_t stream);

constexpr int kReduceBlocks = 2048;

// batched tile passes: items of one level, on `stream`; `gate_runs` when some
// pass of the level holds gate runs, `stream_state` for nontemporal state accesses
int launch_tile_batch(const BatchTables &tables, const BatchItem *d_items, uint32_t n_items, uint64_t total_work,
                      bool gate_runs, bool stream_state, hipStream_t stream);

}  // namespace svi
