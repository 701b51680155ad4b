// Plain per-gate kernels (one launch = one sweep of the subspace a gate
// touches), FP64 reductions, post-selection and conversions.
//
// Work items are enumerated over the free index bits only: a compact counter
// w is spread into an index by inserting zero bits at the sorted positions of
// the target/register/control bits, then the control values are OR-ed in.  A
// gate with c controls therefore reads and writes 2^(n-c) amplitudes, not 2^n.
// Consecutive threads take consecutive counters, so accesses are coalesced on
// the lowest free qubits.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "state_access.h"
#include "sv_internal.h"

namespace svi {

template <typename R> struct CT;
template <> struct CT<float> { using T = float2; };
template <> struct CT<double> { using T = double2; };

// The spread as bit runs: each maximal stretch of consecutive free qubits takes
// a stretch of counter bits, so a register or a block of adjacent controls
// costs one run, not one step per fixed bit.  Run r moves counter bits
// [src, src + width) to index bits [dst, dst + width); packed src | dst << 8 |
// width << 16.
struct Deposit {
    uint32_t n;
    uint32_t run[20];
};

__device__ __forceinline__ uint64_t deposit_zeros(uint64_t x, const Deposit &d)
{
    uint64_t out = 0;
    for (uint32_t k = 0; k < d.n; ++k) {
        const uint32_t r = d.run[k];
        const uint32_t src = r & 0xffu, dst = (r >> 8) & 0xffu, w = r >> 16;
        out |= ((x >> src) & ((1ull << w) - 1ull)) << dst;
    }
    return out;
}

template <typename R> struct Mat2 { R v[8]; };

template <typename C, typename R>
__device__ __forceinline__ C mat_row(R ar, R ai, R br, R bi, C a, C b)
{
    // (ar + i ai) a + (br + i bi) b
    C r;
    r.x = fma(ar, a.x, fma(-ai, a.y, fma(br, b.x, -bi * b.y)));
    r.y = fma(ar, a.y, fma(ai, a.x, fma(br, b.y, bi * b.x)));
    return r;
}

// Workgroups of a grid-stride launch: one item per thread up to 2^20
// workgroups (2^28 threads), so most launches run a single pass of their loop.
// Measured against a cap of 16,384 workgroups: the plain complex128 28-qubit
// circuit 15% faster, the plain 31-qubit ladder 8%, the split launches of the
// fused 31- and 34-qubit ladders 2-3% (the blocked shift keeps its own cap:
// 4,096 workgroups were faster there than one workgroup per block).
static inline int grid_for(uint64_t work, int block)
{
    uint64_t g = (work + block - 1) / block;
    if (g > (1ull << 20)) g = 1ull << 20;
    if (g < 1) g = 1;
    return (int)g;
}

// The same row with every coefficient given as hi + lo (lo the FP32 rounding of
// the FP64 coefficient's remainder), so the matrix the row applies is exact to
// about 2^-48 and only the arithmetic rounds.
template <typename C, typename R>
__device__ __forceinline__ C mat_row2(const R *h, const R *l, C a, C b)
{
    const R lx = fma(l[0], a.x, fma(-l[1], a.y, fma(l[2], b.x, -l[3] * b.y)));
    const R ly = fma(l[0], a.y, fma(l[1], a.x, fma(l[2], b.y, l[3] * b.x)));
    C r;
    r.x = fma(h[0], a.x, fma(-h[1], a.y, fma(h[2], b.x, fma(-h[3], b.y, lx))));
    r.y = fma(h[0], a.y, fma(h[1], a.x, fma(h[2], b.y, fma(h[3], b.x, ly))));
    return r;
}

template <typename R, bool NT>
__global__ void __launch_bounds__(256) k_gate_u(typename CT<R>::T *__restrict__ psi, uint64_t nwork,
                                                Deposit d, uint64_t cval, uint64_t tbit, Mat2<R> m)
{
    using C = typename CT<R>::T;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t w = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; w < nwork; w += stride) {
        const uint64_t i0 = deposit_zeros(w, d) | cval;
        const uint64_t i1 = i0 | tbit;
        const C a = load_state<NT>(psi + i0), b = load_state<NT>(psi + i1);
        store_state<NT>(psi + i0, mat_row(m.v[0], m.v[1], m.v[2], m.v[3], a, b));
        store_state<NT>(psi + i1, mat_row(m.v[4], m.v[5], m.v[6], m.v[7], a, b));
    }
}

// Complex64 form: the matrix as hi + lo FP32 pairs.  A plain launch often
// applies the same gate in every call of a long sequence (a value-load
// rotation of each block-encoding call), and with its matrix rounded to FP32
// the gate scales its subspace by the same factor every time, a drift that adds
// up linearly; carried as hi + lo, the matrix keeps the norm to about 2^-48.
// Plain launches move state through HBM, so the four extra FMAs per amplitude
// cost nothing.
template <bool NT>
__global__ void __launch_bounds__(256) k_gate_u2(float2 *__restrict__ psi, uint64_t nwork, Deposit d,
                                                 uint64_t cval, uint64_t tbit, Mat2<float> m, Mat2<float> lo)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t w = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; w < nwork; w += stride) {
        const uint64_t i0 = deposit_zeros(w, d) | cval;
        const uint64_t i1 = i0 | tbit;
        const float2 a = load_state<NT>(psi + i0), b = load_state<NT>(psi + i1);
        store_state<NT>(psi + i0, mat_row2(m.v, lo.v, a, b));
        store_state<NT>(psi + i1, mat_row2(m.v + 4, lo.v + 4, a, b));
    }
}

template <typename R, bool NT>
__global__ void __launch_bounds__(256) k_gate_x(typename CT<R>::T *__restrict__ psi, uint64_t nwork,
                                                Deposit d, uint64_t cval, uint64_t tbit)
{
    using C = typename CT<R>::T;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t w = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; w < nwork; w += stride) {
        const uint64_t i0 = deposit_zeros(w, d) | cval;
        const uint64_t i1 = i0 | tbit;
        const C a = load_state<NT>(psi + i0), b = load_state<NT>(psi + i1);
        store_state<NT>(psi + i0, b);
        store_state<NT>(psi + i1, a);
    }
}

// multiply by (c, s) every amplitude whose target bit is 1 and controls hold
template <typename R, bool NT>
__global__ void __launch_bounds__(256) k_gate_phase(typename CT<R>::T *__restrict__ psi, uint64_t nwork,
                                                    Deposit d, uint64_t setbits, R c, R s)
{
    using C = typename CT<R>::T;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t w = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; w < nwork; w += stride) {
        const uint64_t i = deposit_zeros(w, d) | setbits;
        const C a = load_state<NT>(psi + i);
        C r;
        r.x = fma(a.x, c, -a.y * s);
        r.y = fma(a.x, s, a.y * c);
        store_state<NT>(psi + i, r);
    }
}

// exchange amplitude i (bit a = 1, bit b = 0) with i ^ abit ^ bbit
template <typename R, bool NT>
__global__ void __launch_bounds__(256) k_gate_swap(typename CT<R>::T *__restrict__ psi, uint64_t nwork,
                                                   Deposit d, uint64_t cval, uint64_t abit, uint64_t bbit)
{
    using C = typename CT<R>::T;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t w = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; w < nwork; w += stride) {
        const uint64_t i = deposit_zeros(w, d) | cval | abit;
        const uint64_t j = i ^ abit ^ bbit;
        const C x = load_state<NT>(psi + i), y = load_state<NT>(psi + j);
        store_state<NT>(psi + i, y);
        store_state<NT>(psi + j, x);
    }
}

// cyclic shift of the register [b, b+w) on one orbit per work item
template <typename R>
__global__ void __launch_bounds__(256) k_gate_shift(typename CT<R>::T *__restrict__ psi, uint64_t nwork,
                                                    Deposit d, uint64_t cval, int base, int width, int up)
{
    using C = typename CT<R>::T;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    const uint64_t len = 1ull << width;
    for (uint64_t w = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; w < nwork; w += stride) {
        const uint64_t r = deposit_zeros(w, d) | cval;
        if (up) {  // new[v] = old[v-1]
            C prev = psi[r | ((len - 1) << base)];
            for (uint64_t v = 0; v < len; ++v) {
                const uint64_t i = r | (v << base);
                const C cur = psi[i];
                psi[i] = prev;
                prev = cur;
            }
        } else {   // new[v] = old[v+1]
            C prev = psi[r];
            for (uint64_t v = len; v-- > 0;) {
                const uint64_t i = r | (v << base);
                const C cur = psi[i];
                psi[i] = prev;
                prev = cur;
            }
        }
    }
}

// The same shift for registers of at most 8 qubits, with every amplitude of an
// orbit read before any is written: a workgroup owns P = 2^(12 - width) whole
// orbits (4,096 amplitudes, 16 per thread), loads them into registers, waits at
// a barrier and stores them shifted, so no thread walks an orbit serially.
// Item i = tid + 256 k of a workgroup is orbit o at register value v; the split
// of i into (o, v) puts consecutive lanes on whichever index lies on the lower
// qubits, so that accesses are coalesced.  The index spread is linear over
// disjoint counter bits, so it is taken apart once: the workgroup's orbit base
// (uniform), the thread's own bits (once per thread) and the 16 per-item parts
// (computed on the host, passed in `it`).
struct ShiftItems {
    uint64_t kdep[16];  // spread counter bits of item k's orbit part
    uint32_t kv[16];    // register-value bits of item k
    uint32_t sh_o, m_o; // thread part of the orbit counter: (tid >> sh_o) & m_o
    uint32_t sh_v, m_v; // thread part of the register value: (tid >> sh_v) & m_v
};

template <typename R, bool NT>
__global__ void __launch_bounds__(256) k_gate_shift_blk(typename CT<R>::T *__restrict__ psi, uint64_t nblk,
                                                        Deposit d, uint64_t cval, int base, int width, int up,
                                                        ShiftItems it)
{
    using C = typename CT<R>::T;
    const uint32_t len_mask = (1u << width) - 1u;
    const int lg_p = 12 - width;
    const uint32_t tid = threadIdx.x;
    const uint64_t dep_t = deposit_zeros((tid >> it.sh_o) & it.m_o, d) | cval;
    const uint32_t v_t = (tid >> it.sh_v) & it.m_v;
    for (uint64_t blk = blockIdx.x; blk < nblk; blk += gridDim.x) {  // uniform per workgroup
        const uint64_t r0 = deposit_zeros(blk << lg_p, d) | dep_t;
        C x[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            const uint32_t v = v_t | it.kv[k];
            const uint32_t src = (up ? v - 1u : v + 1u) & len_mask;  // new[v] = old[v -+ 1]
            x[k] = load_state<NT>(psi + (r0 | it.kdep[k] | ((uint64_t)src << base)));
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < 16; ++k) store_state<NT>(psi + (r0 | it.kdep[k] | ((uint64_t)(v_t | it.kv[k]) << base)), x[k]);
        __syncthreads();
    }
}

// exp(i theta (1 - 2 (s xor z))), z = [(i & mask) == val], s = bit `sig`
template <typename R>
__global__ void __launch_bounds__(256) k_projphase(typename CT<R>::T *__restrict__ psi, uint64_t dim,
                                                   uint64_t mask, uint64_t val, int sig, R c, R s)
{
    using C = typename CT<R>::T;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < dim; i += stride) {
        const uint32_t z = (i & mask) == val;
        const uint32_t sb = (uint32_t)(i >> sig) & 1u;
        const R sn = (sb ^ z) ? -s : s;
        const C a = psi[i];
        C r;
        r.x = fma(a.x, c, -a.y * sn);
        r.y = fma(a.x, sn, a.y * c);
        psi[i] = r;
    }
}

// The device spread of deposit_zeros, on the host (for per-item constants).
static uint64_t deposit_host(uint64_t x, const Deposit &d)
{
    uint64_t out = 0;
    for (uint32_t k = 0; k < d.n; ++k) {
        const uint32_t r = d.run[k];
        const uint32_t src = r & 0xffu, dst = (r >> 8) & 0xffu, w = r >> 16;
        out |= ((x >> src) & ((1ull << w) - 1ull)) << dst;
    }
    return out;
}

static Deposit make_deposit(uint64_t fixed_bits, int n)
{
    // free qubits of an n-qubit index, ascending, grouped into runs (at most
    // n / 2 + 1 <= 19 of them); callers enumerate counters below 2^(free qubits)
    Deposit d{};
    d.n = 0;
    uint32_t src = 0;
    int q = 0;
    while (q < n) {
        if ((fixed_bits >> q) & 1ull) {
            ++q;
            continue;
        }
        int e = q;
        while (e < n && !((fixed_bits >> e) & 1ull)) ++e;
        const uint32_t w = (uint32_t)(e - q);
        d.run[d.n++] = src | ((uint32_t)q << 8) | (w << 16);
        src += w;
        q = e;
    }
    return d;
}

template <typename R, bool NT>
static int launch_plain_t(const PlainOp &op, int n, void *psi_v, hipStream_t st)
{
    using C = typename CT<R>::T;
    C *psi = (C *)psi_v;
    const int B = 256;
    const int c = __builtin_popcountll(op.mask);
    switch (op.kind) {
    case SV_OP_U: {
        const uint64_t nwork = 1ull << (n - 1 - c);
        Mat2<R> m;
        for (int k = 0; k < 8; ++k) m.v[k] = (R)op.m[k];
        if constexpr (std::is_same<R, float>::value) {
            Mat2<float> lo;
            for (int k = 0; k < 8; ++k) lo.v[k] = (float)(op.m[k] - (double)m.v[k]);
            hipLaunchKernelGGL((k_gate_u2<NT>), dim3(grid_for(nwork, B)), dim3(B), 0, st, psi, nwork,
                               make_deposit(op.mask | (1ull << op.target), n), op.val, 1ull << op.target, m, lo);
        } else {
            hipLaunchKernelGGL((k_gate_u<R, NT>), dim3(grid_for(nwork, B)), dim3(B), 0, st, psi, nwork,
                               make_deposit(op.mask | (1ull << op.target), n), op.val, 1ull << op.target, m);
        }
        break;
    }
    case SV_OP_X: {
        const uint64_t nwork = 1ull << (n - 1 - c);
        hipLaunchKernelGGL((k_gate_x<R, NT>), dim3(grid_for(nwork, B)), dim3(B), 0, st, psi, nwork,
                           make_deposit(op.mask | (1ull << op.target), n), op.val, 1ull << op.target);
        break;
    }
    case SV_OP_PHASE: {
        const uint64_t nwork = 1ull << (n - 1 - c);
        hipLaunchKernelGGL((k_gate_phase<R, NT>), dim3(grid_for(nwork, B)), dim3(B), 0, st, psi, nwork,
                           make_deposit(op.mask | (1ull << op.target), n), op.val | (1ull << op.target),
                           (R)cos(op.m[0]), (R)sin(op.m[0]));
        break;
    }
    case SV_OP_SWAP: {
        const uint64_t ab = 1ull << op.target, bb = 1ull << op.width;
        const uint64_t nwork = 1ull << (n - 2 - c);
        hipLaunchKernelGGL((k_gate_swap<R, NT>), dim3(grid_for(nwork, B)), dim3(B), 0, st, psi, nwork,
                           make_deposit(op.mask | ab | bb, n), op.val, ab, bb);
        break;
    }
    case SV_OP_INC:
    case SV_OP_DEC: {
        const uint64_t reg = ((1ull << op.width) - 1ull) << op.target;
        const int lg_orb = n - (int)op.width - c;  // log2 of the number of orbits
        const uint64_t nwork = 1ull << lg_orb;
        if (op.width <= 8 && lg_orb + (int)op.width >= 12) {
            const int w = (int)op.width;
            const int lg_p = 12 - w;  // orbits per workgroup, 4096 amplitudes in all
            const uint64_t fixed = op.mask | reg;
            const uint64_t free_bits = ~fixed & ((n >= 64) ? ~0ull : ((1ull << n) - 1ull));
            const int low_free = free_bits ? __builtin_ctzll(free_bits) : 64;
            const bool v_fast = (int)op.target < low_free;  // the register lies below every free qubit
            const Deposit d = make_deposit(fixed, n);
            // item i = tid + 256 k -> (orbit o, value v), split into thread and item parts
            ShiftItems it{};
            for (int k = 0; k < 16; ++k) {
                uint64_t o_k;
                uint32_t v_k;
                if (v_fast) {             // v = i mod 2^w, o = i >> w
                    o_k = (uint64_t)k << (8 - w);
                    v_k = 0;
                } else if (lg_p >= 8) {   // o = i mod P (P >= 256), v = i / P
                    o_k = (uint64_t)(k & ((1 << (lg_p - 8)) - 1)) << 8;
                    v_k = (uint32_t)k >> (lg_p - 8);
                } else {                  // P < 256: o = tid mod P, v = i / P
                    o_k = 0;
                    v_k = (uint32_t)k << (8 - lg_p);
                }
                it.kdep[k] = deposit_host(o_k, d);
                it.kv[k] = v_k;
            }
            if (v_fast) {
                it.sh_o = (uint32_t)w; it.m_o = 0xffu; it.sh_v = 0; it.m_v = (1u << w) - 1u;
            } else if (lg_p >= 8) {
                it.sh_o = 0; it.m_o = 0xffu; it.sh_v = 0; it.m_v = 0;
            } else {
                it.sh_o = 0; it.m_o = (1u << lg_p) - 1u; it.sh_v = (uint32_t)lg_p; it.m_v = 0xffu;
            }
            const uint64_t nblk = 1ull << (lg_orb - lg_p);
            const int grid = (int)std::min<uint64_t>(nblk, 4096);
            hipLaunchKernelGGL((k_gate_shift_blk<R, NT>), dim3(grid), dim3(B), 0, st, psi, nblk, d, op.val, (int)op.target, w,
                               op.kind == SV_OP_INC ? 1 : 0, it);
        } else {
            hipLaunchKernelGGL(k_gate_shift<R>, dim3(grid_for(nwork, B)), dim3(B), 0, st, psi, nwork,
                               make_deposit(op.mask | reg, n), op.val, (int)op.target, (int)op.width,
                               op.kind == SV_OP_INC ? 1 : 0);
        }
        break;
    }
    case SV_OP_PROJPHASE: {
        const uint64_t dim = 1ull << n;
        hipLaunchKernelGGL(k_projphase<R>, dim3(grid_for(dim, B)), dim3(B), 0, st, psi, dim, op.mask,
                           op.val, (int)op.target, (R)cos(op.m[0]), (R)sin(op.m[0]));
        break;
    }
    default:
        return SV_EINVAL;
    }
    return hipGetLastError() == hipSuccess ? SV_OK : SV_EDEVICE;
}

int launch_plain(const PlainOp &op, int n, int dtype, void *psi, hipStream_t stream)
{
    // nontemporal state accesses by the size rule of the tile passes
    const bool nt = stream_state_bytes((dtype == SV_C64 ? 8ull : 16ull) << n);
    if (dtype == SV_C64)
        return nt ? launch_plain_t<float, true>(op, n, psi, stream) : launch_plain_t<float, false>(op, n, psi, stream);
    return nt ? launch_plain_t<double, true>(op, n, psi, stream) : launch_plain_t<double, false>(op, n, psi, stream);
}

// ---------------------------------------------------------------------------
// reductions (FP64 accumulation for every precision)
// ---------------------------------------------------------------------------
__device__ __forceinline__ double block_sum(double v)
{
    __shared__ double red[16];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) red[wid] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0) {
        const int nw = (blockDim.x + 63) >> 6;
        for (int k = 0; k < nw; ++k) t += red[k];
    }
    return t;  // valid in thread 0
}

template <typename R>
__global__ void __launch_bounds__(256) k_prob(const typename CT<R>::T *__restrict__ psi, uint64_t nwork,
                                              Deposit d, uint64_t val, double *__restrict__ partial)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    double acc = 0.0;
    for (uint64_t w = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; w < nwork; w += stride) {
        const auto a = psi[deposit_zeros(w, d) | val];
        const double x = (double)a.x, y = (double)a.y;
        acc = fma(x, x, fma(y, y, acc));
    }
    const double t = block_sum(acc);
    if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

__global__ void __launch_bounds__(256) k_sum_partials(const double *__restrict__ partial, int count, int stride2,
                                                      double *__restrict__ out)
{
    // sums partial[k*stride2 + j] over k for j in [0, stride2); stride2 <= 2
    for (int j = 0; j < stride2; ++j) {
        double acc = 0.0;
        for (int k = threadIdx.x; k < count; k += blockDim.x) acc += partial[k * stride2 + j];
        const double t = block_sum(acc);
        if (threadIdx.x == 0) out[j] = t;
        __syncthreads();
    }
}

template <typename R>
__global__ void __launch_bounds__(256) k_keep_scale(typename CT<R>::T *__restrict__ psi, uint64_t dim,
                                                    uint64_t mask, uint64_t val, R scale)
{
    using C = typename CT<R>::T;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < dim; i += stride) {
        C a = psi[i];
        if ((i & mask) == val) {
            a.x *= scale;
            a.y *= scale;
        } else {
            a.x = 0;
            a.y = 0;
        }
        psi[i] = a;
    }
}

template <typename RA, typename RB>
__global__ void __launch_bounds__(256) k_inner(const typename CT<RA>::T *__restrict__ a,
                                               const typename CT<RB>::T *__restrict__ b, uint64_t dim,
                                               double *__restrict__ partial)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    double re = 0.0, im = 0.0;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < dim; i += stride) {
        const double ax = a[i].x, ay = a[i].y, bx = b[i].x, by = b[i].y;
        re = fma(ax, bx, fma(ay, by, re));   // conj(a) b
        im = fma(ax, by, fma(-ay, bx, im));
    }
    const double tr = block_sum(re);
    __syncthreads();
    const double ti = block_sum(im);
    if (threadIdx.x == 0) {
        partial[2 * blockIdx.x] = tr;
        partial[2 * blockIdx.x + 1] = ti;
    }
}

template <typename RS, typename RD>
__global__ void __launch_bounds__(256) k_convert(typename CT<RD>::T *__restrict__ dst,
                                                 const typename CT<RS>::T *__restrict__ src, uint64_t count)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) {
        typename CT<RD>::T v;
        v.x = (RD)src[i].x;
        v.y = (RD)src[i].y;
        dst[i] = v;
    }
}

template <typename R>
__global__ void __launch_bounds__(256) k_basis0(typename CT<R>::T *__restrict__ psi, uint64_t dim)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < dim; i += stride) {
        typename CT<R>::T v;
        v.x = (i == 0) ? (R)1 : (R)0;
        v.y = 0;
        psi[i] = v;
    }
}

static int status() { return hipGetLastError() == hipSuccess ? SV_OK : SV_EDEVICE; }

int launch_init_basis(void *psi, int n, int dtype, hipStream_t st)
{
    const uint64_t dim = 1ull << n;
    if (dtype == SV_C64)
        hipLaunchKernelGGL(k_basis0<float>, dim3(grid_for(dim, 256)), dim3(256), 0, st, (float2 *)psi, dim);
    else
        hipLaunchKernelGGL(k_basis0<double>, dim3(grid_for(dim, 256)), dim3(256), 0, st, (double2 *)psi, dim);
    return status();
}

int launch_from_c128(void *psi, int dtype, const void *d_src, uint64_t offset, uint64_t count,
                     hipStream_t st)
{
    if (dtype == SV_C64)
        hipLaunchKernelGGL((k_convert<double, float>), dim3(grid_for(count, 256)), dim3(256), 0, st,
                           (float2 *)psi + offset, (const double2 *)d_src, count);
    else
        hipLaunchKernelGGL((k_convert<double, double>), dim3(grid_for(count, 256)), dim3(256), 0, st,
                           (double2 *)psi + offset, (const double2 *)d_src, count);
    return status();
}

int launch_to_c128(const void *psi, int dtype, void *d_dst, uint64_t offset, uint64_t count,
                   hipStream_t st)
{
    if (dtype == SV_C64)
        hipLaunchKernelGGL((k_convert<float, double>), dim3(grid_for(count, 256)), dim3(256), 0, st,
                           (double2 *)d_dst, (const float2 *)psi + offset, count);
    else
        hipLaunchKernelGGL((k_convert<double, double>), dim3(grid_for(count, 256)), dim3(256), 0, st,
                           (double2 *)d_dst, (const double2 *)psi + offset, count);
    return status();
}

// Same-precision copy in 16-byte vectors; count16 = bytes / 16.
__global__ void __launch_bounds__(256) k_copy16(uint4 *__restrict__ dst, const uint4 *__restrict__ src,
                                                uint64_t count16)
{
    // one 16-byte element per thread: every wave's loads are in flight at once
    // (measured faster than grid-stride loops with several elements per thread);
    // nontemporal hints: 6.5 TB/s on a 2 GiB copy against 6.1 without
    typedef unsigned v4 __attribute__((ext_vector_type(4)));
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count16)
        __builtin_nontemporal_store(__builtin_nontemporal_load(reinterpret_cast<const v4 *>(src) + i),
                                    reinterpret_cast<v4 *>(dst) + i);
}

int launch_copy(void *dst, int dtd, const void *src, int dts, int n, hipStream_t st)
{
    const uint64_t dim = 1ull << n;
    const dim3 g(grid_for(dim, 256)), b(256);
    if (dts == dtd && (dim * (dts == SV_C64 ? 8 : 16)) % 16 == 0) {
        const uint64_t c16 = dim * (dts == SV_C64 ? 8 : 16) / 16;
        const uint64_t blocks = (c16 + 255) / 256;  // at most 2^28 for 36 qubits in complex128
        hipLaunchKernelGGL(k_copy16, dim3((uint32_t)blocks), dim3(256), 0, st, (uint4 *)dst, (const uint4 *)src, c16);
    } else if (dts == SV_C64 && dtd == SV_C64)
        hipLaunchKernelGGL((k_convert<float, float>), g, b, 0, st, (float2 *)dst, (const float2 *)src, dim);
    else if (dts == SV_C64)
        hipLaunchKernelGGL((k_convert<float, double>), g, b, 0, st, (double2 *)dst, (const float2 *)src, dim);
    else if (dtd == SV_C64)
        hipLaunchKernelGGL((k_convert<double, float>), g, b, 0, st, (float2 *)dst, (const double2 *)src, dim);
    else
        hipLaunchKernelGGL((k_convert<double, double>), g, b, 0, st, (double2 *)dst, (const double2 *)src, dim);
    return status();
}

int launch_prob(const void *psi, int n, int dtype, uint64_t mask, uint64_t val, double *d_partial,
                int max_blocks, double *d_out, hipStream_t st)
{
    const int c = __builtin_popcountll(mask);
    const uint64_t nwork = 1ull << (n - c);
    uint64_t g = (nwork + 255) / 256;
    if (g > (uint64_t)max_blocks) g = max_blocks;
    const Deposit d = make_deposit(mask, n);
    if (dtype == SV_C64)
        hipLaunchKernelGGL(k_prob<float>, dim3(g), dim3(256), 0, st, (const float2 *)psi, nwork, d, val, d_partial);
    else
        hipLaunchKernelGGL(k_prob<double>, dim3(g), dim3(256), 0, st, (const double2 *)psi, nwork, d, val, d_partial);
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, st, (const double *)d_partial, (int)g, 1, d_out);
    return status();
}

int launch_keep_scale(void *psi, int n, int dtype, uint64_t mask, uint64_t val, double scale,
                      hipStream_t st)
{
    const uint64_t dim = 1ull << n;
    if (dtype == SV_C64)
        hipLaunchKernelGGL(k_keep_scale<float>, dim3(grid_for(dim, 256)), dim3(256), 0, st, (float2 *)psi, dim,
                           mask, val, (float)scale);
    else
        hipLaunchKernelGGL(k_keep_scale<double>, dim3(grid_for(dim, 256)), dim3(256), 0, st, (double2 *)psi, dim,
                           mask, val, scale);
    return status();
}

int launch_inner(const void *a, int dta, const void *b, int dtb, int n, double *d_partial, int max_blocks,
                 double *d_out, hipStream_t st)
{
    const uint64_t dim = 1ull << n;
    uint64_t g = (dim + 255) / 256;
    if (g > (uint64_t)max_blocks) g = max_blocks;
    const dim3 G(g), B(256);
    if (dta == SV_C64 && dtb == SV_C64)
        hipLaunchKernelGGL((k_inner<float, float>), G, B, 0, st, (const float2 *)a, (const float2 *)b, dim, d_partial);
    else if (dta == SV_C64)
        hipLaunchKernelGGL((k_inner<float, double>), G, B, 0, st, (const float2 *)a, (const double2 *)b, dim, d_partial);
    else if (dtb == SV_C64)
        hipLaunchKernelGGL((k_inner<double, float>), G, B, 0, st, (const double2 *)a, (const float2 *)b, dim, d_partial);
    else
        hipLaunchKernelGGL((k_inner<double, double>), G, B, 0, st, (const double2 *)a, (const double2 *)b, dim, d_partial);
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, st, (const double *)d_partial, (int)g, 2, d_out);
    return status();
}

}  // namespace svi
