// Dense block passes on matrix cores: five-qubit blocks in FP32 or split BF16
// for complex64 states and in FP64 for complex128 states; six-qubit blocks in
// FP32 or split BF16 for complex64 states.
//
// A workgroup stages one tile of 2^12 amplitudes in LDS (five block qubits and
// seven others, loaded through the coalesced tile mapping).  Each of the four
// waves takes 32 groups (values of the seven other local qubits) and computes
// Y = G X for their 32-amplitude columns as a real 32 x 64 by 64 x 32 product
// per part:
//   Y_re = [G_re | -G_im] [X_re; X_im],   Y_im = [G_im | G_re] [X_re; X_im],
// with v_mfma_f32_32x32x2f32 (32 K-steps of 2 per part).  Operand layout of
// that instruction: lane l holds A[l % 32][k = l / 32] and B[k = l / 32][l % 32];
// result register t of lane l is D[8 (t / 4) + 4 (l / 32) + t % 4][l % 32].
// Lane (c, h) = (l % 32, l / 32) therefore reads the amplitudes j = 2i + h of
// group c and ends up holding rows 8 (t / 4) + 4 h + t % 4 of that group.
#include <hip/hip_runtime.h>

#include "sv_internal.h"

namespace svi {

typedef float v16f __attribute__((ext_vector_type(16)));

// Absolute index bits of a tile: bit runs of the tile counter.
__device__ __forceinline__ uint64_t dense_tile_base(const TilePass &P, uint64_t tile)
{
    uint64_t base = 0;
    for (uint32_t r = 0; r < P.n_tile_runs; ++r) {
        const uint32_t sh = P.tile_shift[r];
        base |= ((tile >> (sh & 0xffu)) & P.tile_mask[r]) << (sh >> 8);
    }
    return base;
}

// Persistent: a workgroup loads its matrix operands once (64 values per lane)
// and then strides over tiles, so the 8 KiB block matrix is not fetched again
// for every tile.
__global__ void __launch_bounds__(256)
k_dense_pass(float2 *__restrict__ psi, const DensePass *__restrict__ dp, const float *__restrict__ mats,
             uint64_t n_tiles)
{
    extern __shared__ unsigned char smem_raw[];
    float2 *lds = reinterpret_cast<float2 *>(smem_raw);
    const DensePass &D = *dp;
    const TilePass &P = D.map;
    const uint32_t tid = threadIdx.x;

    // A operands of this lane: row c of [G_re | -G_im] and of [G_im | G_re],
    // columns 2 kk + h
    const uint32_t lane = tid & 63u, wave = tid >> 6;
    const uint32_t c = lane & 31u, h = lane >> 5;
    const float *G = mats + D.mat;
    float a1[32], a2[32];
#pragma unroll
    for (int kk = 0; kk < 32; ++kk) {
        const uint32_t q = 2u * kk + h;
        if (kk < 16) {
            a1[kk] = G[2 * (32 * c + q)];
            a2[kk] = G[2 * (32 * c + q) + 1];
        } else {
            a1[kk] = -G[2 * (32 * c + q - 32) + 1];
            a2[kk] = G[2 * (32 * c + q - 32)];
        }
    }
    uint64_t gthr = 0;
    for (uint32_t r = 0; r < P.n_gthr_runs; ++r) {
        const uint32_t sh = P.gthr_shift[r];
        gthr |= (uint64_t)((tid >> (sh & 0xffu)) & P.gthr_mask[r]) << (sh >> 8);
    }
    const uint32_t g = wave * 32u + c;
    uint32_t gl = 0;
    for (uint32_t r = 0; r < D.n_grp_runs; ++r) {
        const uint32_t w = D.grp_run[r];
        gl |= ((g >> (w & 0xffu)) & (w >> 16)) << ((w >> 8) & 0xffu);
    }
    const uint32_t tw = lds_swizzle(tid, 4);

    // the amplitudes of the next tile are loaded while the current one is multiplied
    float2 x[16];
    if (blockIdx.x < n_tiles) {
        const float2 *p0 = psi + (dense_tile_base(P, blockIdx.x) | gthr);
#pragma unroll
        for (int s = 0; s < 16; ++s) x[s] = p0[P.goff[s]];
    }
    for (uint64_t tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
        float2 *const pt = psi + (dense_tile_base(P, tile) | gthr);
#pragma unroll
        for (int s = 0; s < 16; ++s) lds[tw ^ P.swz0[s]] = x[s];
        __syncthreads();
        if (tile + gridDim.x < n_tiles) {
            const float2 *pn = psi + (dense_tile_base(P, tile + gridDim.x) | gthr);
#pragma unroll
            for (int s = 0; s < 16; ++s) x[s] = pn[P.goff[s]];
        }

        float2 xb[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) xb[i] = lds[lds_swizzle(gl | D.joff[2 * i + h], 4)];
        v16f acc_re = {0.f}, acc_im = {0.f};
#pragma unroll
        for (int kk = 0; kk < 16; ++kk) {
            acc_re = __builtin_amdgcn_mfma_f32_32x32x2f32(a1[kk], xb[kk].x, acc_re, 0, 0, 0);
            acc_im = __builtin_amdgcn_mfma_f32_32x32x2f32(a2[kk], xb[kk].x, acc_im, 0, 0, 0);
        }
#pragma unroll
        for (int kk = 16; kk < 32; ++kk) {
            acc_re = __builtin_amdgcn_mfma_f32_32x32x2f32(a1[kk], xb[kk - 16].y, acc_re, 0, 0, 0);
            acc_im = __builtin_amdgcn_mfma_f32_32x32x2f32(a2[kk], xb[kk - 16].y, acc_im, 0, 0, 0);
        }
        __syncthreads();
#pragma unroll
        for (int t = 0; t < 16; ++t)
            lds[lds_swizzle(gl | D.joff[8u * (t / 4) + 4u * h + (t % 4)], 4)] = make_float2(acc_re[t], acc_im[t]);
        __syncthreads();
        float2 y[16];
#pragma unroll
        for (int s = 0; s < 16; ++s) y[s] = lds[tw ^ P.swz0[s]];
#pragma unroll
        for (int s = 0; s < 16; ++s) pt[P.goff[s]] = y[s];
        __syncthreads();  // the next tile overwrites the LDS
    }
}

// Complex64 in split BF16: the same product on BF16 matrix cores with
// v_mfma_f32_32x32x8bf16_1k (K = 8 per instruction, FP32 accumulation).  Each
// FP32 value v is split into hi = bf16(v) and lo = bf16(v - hi), both rounded
// to nearest even, and G X is taken as Gh Xh + Gh Xl + Gl Xh: the dropped
// Gl Xl term and the rounding of the lo parts leave about 2^-16 of each
// product, against 2^-24 on FP32 matrix cores, for 48 BF16 products per tile
// and wave instead of 64 FP32 ones.  Operand layout of the instruction
// (checked on the device with integer operands): lane l holds
// A[l % 32][4 (l / 32) + j] and B[4 (l / 32) + j][l % 32], j = 0..3; result
// register t of lane l is D[8 (t / 4) + 4 (l / 32) + t % 4][l % 32], as for
// the FP32 instruction.  K chunk q (0..7) of the real product covers columns
// 8 q .. 8 q + 7 of [G_re | -G_im] (rows of Y_re) and [G_im | G_re] (Y_im):
// chunks 0-3 take X_re, 4-7 X_im, of the amplitudes 8 (q % 4) + 4 h + j.
typedef short s4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ short bf16_rn(float f)
{
    uint32_t u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);  // round to nearest even (amplitudes and gates are finite)
    return (short)(u >> 16);
}

__device__ __forceinline__ float bf16_f(short h) { return __uint_as_float((uint32_t)(uint16_t)h << 16); }

__global__ void __launch_bounds__(256)
k_dense_pass_bf16(float2 *__restrict__ psi, const DensePass *__restrict__ dp, const float *__restrict__ mats,
                  uint64_t n_tiles)
{
    extern __shared__ unsigned char smem_raw[];
    float2 *lds = reinterpret_cast<float2 *>(smem_raw);
    const DensePass &D = *dp;
    const TilePass &P = D.map;
    const uint32_t tid = threadIdx.x;
    const uint32_t lane = tid & 63u, wave = tid >> 6;
    const uint32_t c = lane & 31u, h = lane >> 5;
    const float *G = mats + D.mat;

    // A operands, split: [part][chunk] of 4 values (columns 8 q + 4 h + j)
    s4 ah[2][8], al[2][8];
#pragma unroll
    for (int q = 0; q < 8; ++q)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const uint32_t col = 8u * (uint32_t)(q & 3) + 4u * h + (uint32_t)j;  // block value of the column
            const float gre = G[2 * (32 * c + col)], gim = G[2 * (32 * c + col) + 1];
            const float v0 = q < 4 ? gre : -gim;  // [G_re | -G_im]
            const float v1 = q < 4 ? gim : gre;   // [G_im | G_re]
            ah[0][q][j] = bf16_rn(v0);
            al[0][q][j] = bf16_rn(v0 - bf16_f(ah[0][q][j]));
            ah[1][q][j] = bf16_rn(v1);
            al[1][q][j] = bf16_rn(v1 - bf16_f(ah[1][q][j]));
        }
    uint64_t gthr = 0;
    for (uint32_t r = 0; r < P.n_gthr_runs; ++r) {
        const uint32_t sh = P.gthr_shift[r];
        gthr |= (uint64_t)((tid >> (sh & 0xffu)) & P.gthr_mask[r]) << (sh >> 8);
    }
    const uint32_t g = wave * 32u + c;
    uint32_t gl = 0;
    for (uint32_t r = 0; r < D.n_grp_runs; ++r) {
        const uint32_t w = D.grp_run[r];
        gl |= ((g >> (w & 0xffu)) & (w >> 16)) << ((w >> 8) & 0xffu);
    }
    const uint32_t tw = lds_swizzle(tid, 4);

    for (uint64_t tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
        float2 *const pt = psi + (dense_tile_base(P, tile) | gthr);
        {
            float2 x[16];
#pragma unroll
            for (int s = 0; s < 16; ++s) x[s] = pt[P.goff[s]];
#pragma unroll
            for (int s = 0; s < 16; ++s) lds[tw ^ P.swz0[s]] = x[s];
        }
        __syncthreads();
        // B operands, split: the amplitudes 8 q + 4 h + j of this lane's group
        s4 bh[8], bl[8];
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const float2 xv = lds[lds_swizzle(gl | D.joff[8 * q + 4 * h + j], 4)];
                bh[q][j] = bf16_rn(xv.x);
                bl[q][j] = bf16_rn(xv.x - bf16_f(bh[q][j]));
                bh[q + 4][j] = bf16_rn(xv.y);
                bl[q + 4][j] = bf16_rn(xv.y - bf16_f(bh[q + 4][j]));
            }
        v16f acc_re = {0.f}, acc_im = {0.f};
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            acc_re = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(ah[0][q], bh[q], acc_re, 0, 0, 0);
            acc_re = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(ah[0][q], bl[q], acc_re, 0, 0, 0);
            acc_re = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(al[0][q], bh[q], acc_re, 0, 0, 0);
            acc_im = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(ah[1][q], bh[q], acc_im, 0, 0, 0);
            acc_im = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(ah[1][q], bl[q], acc_im, 0, 0, 0);
            acc_im = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(al[1][q], bh[q], acc_im, 0, 0, 0);
        }
        __syncthreads();  // every wave has read its X before Y overwrites it
#pragma unroll
        for (int t = 0; t < 16; ++t)
            lds[lds_swizzle(gl | D.joff[8u * (t / 4) + 4u * h + (t % 4)], 4)] = make_float2(acc_re[t], acc_im[t]);
        __syncthreads();
        float2 y[16];
#pragma unroll
        for (int s = 0; s < 16; ++s) y[s] = lds[tw ^ P.swz0[s]];
#pragma unroll
        for (int s = 0; s < 16; ++s) pt[P.goff[s]] = y[s];
        __syncthreads();  // the next tile overwrites the LDS
    }
}

// Six-qubit blocks (complex64): a tile holds 64 groups (values of the six other
// local qubits) of 64 amplitudes, and Y = G X is a real 64 x 128 by 128 x 64
// product per part.  Wave w takes the 32 x 32 corner of rows 32 (w >> 1) ..
// 32 (w >> 1) + 31 and groups 32 (w & 1) .. 32 (w & 1) + 31, for Y_re and for
// Y_im: 64 K-steps of v_mfma_f32_32x32x2f32 per part (the operand layout of
// the five-qubit kernel).  [G_im | G_re] is [G_re | -G_im] with its halves
// exchanged and one negated, so a lane keeps only the 64 values of the latter
// in registers for the whole persistent launch and negates X_re instead:
//   Y_re = G_re X_re + (-G_im) X_im,   Y_im = (-G_im)(-X_re) + G_re X_im.
// At 512 flop per amplitude this form is bound by the FP32 matrix cores.
__global__ void __launch_bounds__(256)
k_dense6_pass(float2 *__restrict__ psi, const DensePass *__restrict__ dp, const float *__restrict__ mats,
              uint64_t n_tiles)
{
    extern __shared__ unsigned char smem_raw[];
    float2 *lds = reinterpret_cast<float2 *>(smem_raw);
    const DensePass &D = *dp;
    const TilePass &P = D.map;
    const uint32_t tid = threadIdx.x;
    const uint32_t lane = tid & 63u, wave = tid >> 6;
    const uint32_t c = lane & 31u, h = lane >> 5;
    const uint32_t mb = wave >> 1, nb = wave & 1u;
    const uint32_t row = 32u * mb + c;
    const float *G = mats + D.mat;
    float a1[64];  // columns 2 kk + h of [G_re | -G_im]
#pragma unroll
    for (int kk = 0; kk < 64; ++kk) {
        const uint32_t q = 2u * kk + h;
        a1[kk] = kk < 32 ? G[2 * (64 * row + q)] : -G[2 * (64 * row + q - 64) + 1];
    }
    uint64_t gthr = 0;
    for (uint32_t r = 0; r < P.n_gthr_runs; ++r) {
        const uint32_t sh = P.gthr_shift[r];
        gthr |= (uint64_t)((tid >> (sh & 0xffu)) & P.gthr_mask[r]) << (sh >> 8);
    }
    const uint32_t g = 32u * nb + c;
    uint32_t gl = 0;
    for (uint32_t r = 0; r < D.n_grp_runs; ++r) {
        const uint32_t w = D.grp_run[r];
        gl |= ((g >> (w & 0xffu)) & (w >> 16)) << ((w >> 8) & 0xffu);
    }
    const uint32_t tw = lds_swizzle(tid, 4);

    for (uint64_t tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
        float2 *const pt = psi + (dense_tile_base(P, tile) | gthr);
        {
            float2 x[16];
#pragma unroll
            for (int s = 0; s < 16; ++s) x[s] = pt[P.goff[s]];
#pragma unroll
            for (int s = 0; s < 16; ++s) lds[tw ^ P.swz0[s]] = x[s];
        }
        __syncthreads();
        v16f acc_re = {0.f}, acc_im = {0.f};
#pragma unroll
        for (int half = 0; half < 2; ++half) {
            // amplitudes 2 i + h of the group, i in [16 half, 16 half + 16)
            float2 xb[16];
#pragma unroll
            for (int i = 0; i < 16; ++i) xb[i] = lds[lds_swizzle(gl | D.joff[2 * (16 * half + i) + h], 4)];
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const int kk = 16 * half + i;
                acc_re = __builtin_amdgcn_mfma_f32_32x32x2f32(a1[kk], xb[i].x, acc_re, 0, 0, 0);
                acc_im = __builtin_amdgcn_mfma_f32_32x32x2f32(a1[kk + 32], -xb[i].x, acc_im, 0, 0, 0);
                acc_re = __builtin_amdgcn_mfma_f32_32x32x2f32(a1[kk + 32], xb[i].y, acc_re, 0, 0, 0);
                acc_im = __builtin_amdgcn_mfma_f32_32x32x2f32(a1[kk], xb[i].y, acc_im, 0, 0, 0);
            }
        }
        __syncthreads();  // every wave has read its X before Y overwrites it
#pragma unroll
        for (int t = 0; t < 16; ++t) {
            const uint32_t r = 32u * mb + 8u * (t / 4) + 4u * h + (t % 4);
            lds[lds_swizzle(gl | D.joff[r], 4)] = make_float2(acc_re[t], acc_im[t]);
        }
        __syncthreads();
        float2 y[16];
#pragma unroll
        for (int s = 0; s < 16; ++s) y[s] = lds[tw ^ P.swz0[s]];
#pragma unroll
        for (int s = 0; s < 16; ++s) pt[P.goff[s]] = y[s];
        __syncthreads();  // the next tile overwrites the LDS
    }
}

// Six-qubit blocks in split BF16: the corner of k_dense6_pass on
// v_mfma_f32_32x32x8bf16_1k, hi and lo parts as in k_dense_pass_bf16.  K chunk
// q (0..15) covers columns 8 q .. 8 q + 7 of [G_re | -G_im] and [G_im | G_re]:
// chunks 0-7 take X_re, 8-15 X_im, of the amplitudes 8 (q % 8) + 4 h + j.
// As in the FP32 form only the split [G_re | -G_im] stays in registers (the
// split of a negated value is the negated split), and Y_im takes -X_re.
// 96 BF16 products per tile and wave replace 256 FP32 ones.
__global__ void __launch_bounds__(256)
k_dense6_pass_bf16(float2 *__restrict__ psi, const DensePass *__restrict__ dp, const float *__restrict__ mats,
                   uint64_t n_tiles)
{
    extern __shared__ unsigned char smem_raw[];
    float2 *lds = reinterpret_cast<float2 *>(smem_raw);
    const DensePass &D = *dp;
    const TilePass &P = D.map;
    const uint32_t tid = threadIdx.x;
    const uint32_t lane = tid & 63u, wave = tid >> 6;
    const uint32_t c = lane & 31u, h = lane >> 5;
    const uint32_t mb = wave >> 1, nb = wave & 1u;
    const uint32_t row = 32u * mb + c;
    const float *G = mats + D.mat;

    s4 ah[16], al[16];  // [G_re | -G_im], chunk q: columns 8 q + 4 h + j
#pragma unroll
    for (int q = 0; q < 16; ++q)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const uint32_t col = 8u * (uint32_t)(q & 7) + 4u * h + (uint32_t)j;  // block value of the column
            const float v0 = q < 8 ? G[2 * (64 * row + col)] : -G[2 * (64 * row + col) + 1];
            ah[q][j] = bf16_rn(v0);
            al[q][j] = bf16_rn(v0 - bf16_f(ah[q][j]));
        }
    uint64_t gthr = 0;
    for (uint32_t r = 0; r < P.n_gthr_runs; ++r) {
        const uint32_t sh = P.gthr_shift[r];
        gthr |= (uint64_t)((tid >> (sh & 0xffu)) & P.gthr_mask[r]) << (sh >> 8);
    }
    const uint32_t g = 32u * nb + c;
    uint32_t gl = 0;
    for (uint32_t r = 0; r < D.n_grp_runs; ++r) {
        const uint32_t w = D.grp_run[r];
        gl |= ((g >> (w & 0xffu)) & (w >> 16)) << ((w >> 8) & 0xffu);
    }
    const uint32_t tw = lds_swizzle(tid, 4);

    for (uint64_t tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
        float2 *const pt = psi + (dense_tile_base(P, tile) | gthr);
        {
            float2 x[16];
#pragma unroll
            for (int s = 0; s < 16; ++s) x[s] = pt[P.goff[s]];
#pragma unroll
            for (int s = 0; s < 16; ++s) lds[tw ^ P.swz0[s]] = x[s];
        }
        __syncthreads();
        v16f acc_re = {0.f}, acc_im = {0.f};
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            // chunk q (real parts, and their negation for Y_im) and chunk q + 8 (imaginary parts)
            s4 bhr, blr, nhr, nlr, bhi, bli;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const float2 xv = lds[lds_swizzle(gl | D.joff[8 * q + 4 * h + j], 4)];
                bhr[j] = bf16_rn(xv.x);
                blr[j] = bf16_rn(xv.x - bf16_f(bhr[j]));
                nhr[j] = (short)(bhr[j] ^ (short)0x8000);
                nlr[j] = (short)(blr[j] ^ (short)0x8000);
                bhi[j] = bf16_rn(xv.y);
                bli[j] = bf16_rn(xv.y - bf16_f(bhi[j]));
            }
            acc_re = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(ah[q], bhr, acc_re, 0, 0, 0);
            acc_re = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(ah[q], blr, acc_re, 0, 0, 0);
            acc_re = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(al[q], bhr, acc_re, 0, 0, 0);
            acc_im = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(ah[q + 8], nhr, acc_im, 0, 0, 0);
            acc_im = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(ah[q + 8], nlr, acc_im, 0, 0, 0);
            acc_im = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(al[q + 8], nhr, acc_im, 0, 0, 0);
            acc_re = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(ah[q + 8], bhi, acc_re, 0, 0, 0);
            acc_re = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(ah[q + 8], bli, acc_re, 0, 0, 0);
            acc_re = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(al[q + 8], bhi, acc_re, 0, 0, 0);
            acc_im = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(ah[q], bhi, acc_im, 0, 0, 0);
            acc_im = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(ah[q], bli, acc_im, 0, 0, 0);
            acc_im = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(al[q], bhi, acc_im, 0, 0, 0);
        }
        __syncthreads();  // every wave has read its X before Y overwrites it
#pragma unroll
        for (int t = 0; t < 16; ++t) {
            const uint32_t r = 32u * mb + 8u * (t / 4) + 4u * h + (t % 4);
            lds[lds_swizzle(gl | D.joff[r], 4)] = make_float2(acc_re[t], acc_im[t]);
        }
        __syncthreads();
        float2 y[16];
#pragma unroll
        for (int s = 0; s < 16; ++s) y[s] = lds[tw ^ P.swz0[s]];
#pragma unroll
        for (int s = 0; s < 16; ++s) pt[P.goff[s]] = y[s];
        __syncthreads();  // the next tile overwrites the LDS
    }
}

// Complex128: the same product on FP64 matrix cores, v_mfma_f64_16x16x4f64
// (M = 16 block rows, N = 16 groups, K = 4 block values per instruction).
// Operand layout of that instruction (checked on the device): lane l holds
// A[l % 16][l / 16] and B[l / 16][l % 16]; result t of lane l is
// D[4 t + l / 16][l % 16].  A tile holds 128 groups; wave w takes groups
// 32 w .. 32 w + 31 as two N blocks, both 16-row halves of the block matrix,
// and keeps the A operands (G_re, G_im for 2 halves x 8 K steps) in registers.
//   Y_re += G_re X_re + G_im (-X_im),   Y_im += G_im X_re + G_re X_im.
typedef double v4d __attribute__((ext_vector_type(4)));

__global__ void __launch_bounds__(256)
k_dense_pass_f64(double2 *__restrict__ psi, const DensePass *__restrict__ dp, const double *__restrict__ mats,
                 uint64_t n_tiles)
{
    extern __shared__ unsigned char smem_raw[];
    double2 *lds = reinterpret_cast<double2 *>(smem_raw);
    const DensePass &D = *dp;
    const TilePass &P = D.map;
    const uint32_t tid = threadIdx.x;
    const uint32_t lane = tid & 63u, wave = tid >> 6;
    const uint32_t r16 = lane & 15u, k4 = lane >> 4;

    const double *G = mats + D.mat;
    double gre[2][8], gim[2][8];
#pragma unroll
    for (int mb = 0; mb < 2; ++mb)
#pragma unroll
        for (int ks = 0; ks < 8; ++ks) {
            const uint32_t idx = 32u * (16u * mb + r16) + 4u * ks + k4;
            gre[mb][ks] = G[2 * idx];
            gim[mb][ks] = G[2 * idx + 1];
        }
    uint64_t gthr = 0;
    for (uint32_t r = 0; r < P.n_gthr_runs; ++r) {
        const uint32_t sh = P.gthr_shift[r];
        gthr |= (uint64_t)((tid >> (sh & 0xffu)) & P.gthr_mask[r]) << (sh >> 8);
    }
    uint32_t gl[2];
#pragma unroll
    for (int nb = 0; nb < 2; ++nb) {
        const uint32_t g = wave * 32u + 16u * nb + r16;
        uint32_t o = 0;
        for (uint32_t r = 0; r < D.n_grp_runs; ++r) {
            const uint32_t w = D.grp_run[r];
            o |= ((g >> (w & 0xffu)) & (w >> 16)) << ((w >> 8) & 0xffu);
        }
        gl[nb] = o;
    }
    const uint32_t tw = lds_swizzle(tid, 3);

    for (uint64_t tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
        double2 *const pt = psi + (dense_tile_base(P, tile) | gthr);
        {
            double2 x[16];
#pragma unroll
            for (int s = 0; s < 16; ++s) x[s] = pt[P.goff[s]];
#pragma unroll
            for (int s = 0; s < 16; ++s) lds[tw ^ P.swz0[s]] = x[s];
        }
        __syncthreads();

        v4d yre[2][2], yim[2][2];  // [N block][M half]
#pragma unroll
        for (int nb = 0; nb < 2; ++nb) {
#pragma unroll
            for (int mb = 0; mb < 2; ++mb) {
                yre[nb][mb] = (v4d){0.0, 0.0, 0.0, 0.0};
                yim[nb][mb] = (v4d){0.0, 0.0, 0.0, 0.0};
            }
#pragma unroll
            for (int ks = 0; ks < 8; ++ks) {
                const double2 xv = lds[lds_swizzle(gl[nb] | D.joff[4 * ks + k4], 3)];
                const double xim_neg = -xv.y;
#pragma unroll
                for (int mb = 0; mb < 2; ++mb) {
                    yre[nb][mb] = __builtin_amdgcn_mfma_f64_16x16x4f64(gre[mb][ks], xv.x, yre[nb][mb], 0, 0, 0);
                    yre[nb][mb] = __builtin_amdgcn_mfma_f64_16x16x4f64(gim[mb][ks], xim_neg, yre[nb][mb], 0, 0, 0);
                    yim[nb][mb] = __builtin_amdgcn_mfma_f64_16x16x4f64(gim[mb][ks], xv.x, yim[nb][mb], 0, 0, 0);
                    yim[nb][mb] = __builtin_amdgcn_mfma_f64_16x16x4f64(gre[mb][ks], xv.y, yim[nb][mb], 0, 0, 0);
                }
            }
        }
        __syncthreads();  // every wave has read its X before Y overwrites it
#pragma unroll
        for (int nb = 0; nb < 2; ++nb)
#pragma unroll
            for (int mb = 0; mb < 2; ++mb)
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const uint32_t row = 16u * mb + 4u * t + k4;
                    lds[lds_swizzle(gl[nb] | D.joff[row], 3)] = make_double2(yre[nb][mb][t], yim[nb][mb][t]);
                }
        __syncthreads();
        {
            double2 x[16];
#pragma unroll
            for (int s = 0; s < 16; ++s) x[s] = lds[tw ^ P.swz0[s]];
#pragma unroll
            for (int s = 0; s < 16; ++s) pt[P.goff[s]] = x[s];
        }
        __syncthreads();  // the next tile overwrites the LDS
    }
}

int launch_dense_pass(const sv_plan *p, uint32_t di, void *psi, hipStream_t st)
{
    const DensePass &D = p->dense[di];
    const uint64_t tiles = 1ull << D.map.ntile;
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    const uint64_t cap = (uint64_t)cus * 2;  // resident workgroups per CU at these kernels' register and LDS use
    const uint32_t grid = (uint32_t)(tiles < cap ? tiles : cap);
    if (p->dtype == SV_C64 && D.k == 6 && p->dense_bf16)
        hipLaunchKernelGGL(k_dense6_pass_bf16, dim3(grid), dim3(256), sizeof(float2) << 12, st, (float2 *)psi,
                           (const DensePass *)p->d_dense + di, (const float *)p->d_dparams, tiles);
    else if (p->dtype == SV_C64 && D.k == 6)
        hipLaunchKernelGGL(k_dense6_pass, dim3(grid), dim3(256), sizeof(float2) << 12, st, (float2 *)psi,
                           (const DensePass *)p->d_dense + di, (const float *)p->d_dparams, tiles);
    else if (p->dtype == SV_C64 && p->dense_bf16)
        hipLaunchKernelGGL(k_dense_pass_bf16, dim3(grid), dim3(256), sizeof(float2) << 12, st, (float2 *)psi,
                           (const DensePass *)p->d_dense + di, (const float *)p->d_dparams, tiles);
    else if (p->dtype == SV_C64)
        hipLaunchKernelGGL(k_dense_pass, dim3(grid), dim3(256), sizeof(float2) << 12, st, (float2 *)psi,
                           (const DensePass *)p->d_dense + di, (const float *)p->d_dparams, tiles);
    else
        hipLaunchKernelGGL(k_dense_pass_f64, dim3(grid), dim3(256), sizeof(double2) << 12, st, (double2 *)psi,
                           (const DensePass *)p->d_dense + di, (const double *)p->d_dparams, tiles);
    return hipGetLastError() == hipSuccess ? SV_OK : SV_EDEVICE;
}

}  // namespace svi
