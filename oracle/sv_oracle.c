/*
 * FP64 reference state-vector simulator.  TEST INFRASTRUCTURE ONLY: it is
 * called from tests, from the package smoke check and from the CPU-baseline
 * leg of the benchmark, never from the product path.  It shares no code with
 * the HIP library.
 *
 * Every op is applied by the plainest possible loop: visit every basis index
 * i of the 2^n-entry state, test whether the op touches i, and update.  No
 * blocking, no fusion, no reordering.  Amplitudes are C99 double complex,
 * index bit j = qubit j.
 *
 * What each op computes is the definition of that gate acting on the
 * computational basis (the elementary gate set of Sec. III: X/CNOT/Toffoli and
 * their multi-controlled forms, H, R_Y, S, S^dagger, plus the projector phase
 * of the QSVT circuit figure, Sec. II.D.5).  The record layout is read as
 * 40-byte little-endian records:
 *   u32 kind, u32 target, u32 width, u32 flags, u64 mask, u64 val, u64 param.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

typedef struct {
    uint32_t kind, target, width, flags;
    uint64_t mask, val, param;
} orc_op;

enum { K_U = 0, K_X = 1, K_PHASE = 2, K_RY = 3, K_INC = 4, K_DEC = 5, K_SWAP = 6, K_PROJPHASE = 7 };

static int controls_hold(uint64_t i, const orc_op *op) { return (i & op->mask) == op->val; }

/* 2x2 matrix m = {m00, m01, m10, m11} on the pair (i with bit t clear, i with bit t set). */
static void apply_matrix(cplx *psi, int n, const orc_op *op, const cplx m[4])
{
    const uint64_t dim = 1ull << n;
    const uint64_t tb = 1ull << op->target;
#pragma omp parallel for schedule(static)
    for (int64_t ii = 0; ii < (int64_t)dim; ++ii) {
        uint64_t i = (uint64_t)ii;
        if (i & tb) continue;
        if (!controls_hold(i, op)) continue;
        uint64_t j = i | tb;
        cplx a0 = psi[i], a1 = psi[j];
        psi[i] = m[0] * a0 + m[1] * a1;
        psi[j] = m[2] * a0 + m[3] * a1;
    }
}

static void apply_x(cplx *psi, int n, const orc_op *op)
{
    const uint64_t dim = 1ull << n;
    const uint64_t tb = 1ull << op->target;
#pragma omp parallel for schedule(static)
    for (int64_t ii = 0; ii < (int64_t)dim; ++ii) {
        uint64_t i = (uint64_t)ii;
        if (i & tb) continue;
        if (!controls_hold(i, op)) continue;
        uint64_t j = i | tb;
        cplx tmp = psi[i];
        psi[i] = psi[j];
        psi[j] = tmp;
    }
}

static void apply_phase(cplx *psi, int n, const orc_op *op, double theta)
{
    const uint64_t dim = 1ull << n;
    const uint64_t tb = 1ull << op->target;
    const cplx ph = cexp(I * theta);
#pragma omp parallel for schedule(static)
    for (int64_t ii = 0; ii < (int64_t)dim; ++ii) {
        uint64_t i = (uint64_t)ii;
        if ((i & tb) && controls_hold(i, op)) psi[i] *= ph;
    }
}

/* Cyclic shift of the register value v = bits [b, b+w) of i, by +1 (INC) or -1
 * (DEC) modulo 2^w, on the basis states whose controls hold.  Each orbit
 * (fixed bits outside the register) is rotated in place. */
static void apply_shift(cplx *psi, int n, const orc_op *op, int up)
{
    const uint64_t dim = 1ull << n;
    const int b = (int)op->target, w = (int)op->width;
    const uint64_t len = 1ull << w;
    const uint64_t regmask = (len - 1) << b;
#pragma omp parallel for schedule(static)
    for (int64_t ii = 0; ii < (int64_t)dim; ++ii) {
        uint64_t r = (uint64_t)ii;
        if (r & regmask) continue;          /* one representative per orbit */
        if (!controls_hold(r, op)) continue;
        if (up) {   /* new[v] = old[v-1] */
            cplx last = psi[r | ((len - 1) << b)];
            for (uint64_t v = len - 1; v >= 1; --v)
                psi[r | (v << b)] = psi[r | ((v - 1) << b)];
            psi[r] = last;
        } else {    /* new[v] = old[v+1] */
            cplx first = psi[r];
            for (uint64_t v = 0; v + 1 < len; ++v)
                psi[r | (v << b)] = psi[r | ((v + 1) << b)];
            psi[r | ((len - 1) << b)] = first;
        }
    }
}

static void apply_swap(cplx *psi, int n, const orc_op *op)
{
    const uint64_t dim = 1ull << n;
    const uint64_t ba = 1ull << op->target, bb = 1ull << op->width;
#pragma omp parallel for schedule(static)
    for (int64_t ii = 0; ii < (int64_t)dim; ++ii) {
        uint64_t i = (uint64_t)ii;
        /* visit the member of each exchanged pair with qubit a = 1, qubit b = 0 */
        if (!(i & ba) || (i & bb)) continue;
        if (!controls_hold(i, op)) continue;
        uint64_t j = (i & ~ba) | bb;
        cplx tmp = psi[i];
        psi[i] = psi[j];
        psi[j] = tmp;
    }
}

/* The projector phase taken literally as three gates: MCX (condition ->
 * signal), exp(i theta Z) on the signal, the same MCX. */
static void apply_projphase(cplx *psi, int n, const orc_op *op, double theta)
{
    orc_op mcx = *op;
    mcx.kind = K_X;
    apply_x(psi, n, &mcx);
    orc_op z = *op;
    z.mask = 0;
    z.val = 0;
    const cplx m[4] = {cexp(I * theta), 0.0, 0.0, cexp(-I * theta)};
    apply_matrix(psi, n, &z, m);
    apply_x(psi, n, &mcx);
}

int oracle_apply(double *psi_d, int n, const void *ops_raw, uint64_t n_ops, const double *params)
{
    cplx *psi = (cplx *)psi_d;
    const orc_op *ops = (const orc_op *)ops_raw;
    for (uint64_t k = 0; k < n_ops; ++k) {
        const orc_op *op = &ops[k];
        const double *p = params + op->param;
        switch (op->kind) {
        case K_U: {
            const cplx m[4] = {p[0] + I * p[1], p[2] + I * p[3], p[4] + I * p[5], p[6] + I * p[7]};
            apply_matrix(psi, n, op, m);
            break;
        }
        case K_X: apply_x(psi, n, op); break;
        case K_PHASE: apply_phase(psi, n, op, p[0]); break;
        case K_RY: {
            const double c = cos(0.5 * p[0]), s = sin(0.5 * p[0]);
            const cplx m[4] = {c, -s, s, c};
            apply_matrix(psi, n, op, m);
            break;
        }
        case K_INC: apply_shift(psi, n, op, 1); break;
        case K_DEC: apply_shift(psi, n, op, 0); break;
        case K_SWAP: apply_swap(psi, n, op); break;
        case K_PROJPHASE: apply_projphase(psi, n, op, p[0]); break;
        default: return -1;
        }
    }
    return 0;
}

/* sum |psi_i|^2 over the i with (i & mask) == val */
double oracle_prob(const double *psi_d, int n, uint64_t mask, uint64_t val)
{
    const cplx *psi = (const cplx *)psi_d;
    const uint64_t dim = 1ull << n;
    double acc = 0.0;
#pragma omp parallel for reduction(+ : acc) schedule(static)
    for (int64_t ii = 0; ii < (int64_t)dim; ++ii) {
        uint64_t i = (uint64_t)ii;
        if ((i & mask) == val) acc += creal(psi[i]) * creal(psi[i]) + cimag(psi[i]) * cimag(psi[i]);
    }
    return acc;
}

/* Keep the subspace (i & mask) == val, zero the rest; divide by sqrt(P) if
 * renormalize.  Returns P (the state is left untouched when P == 0). */
double oracle_postselect(double *psi_d, int n, uint64_t mask, uint64_t val, int renormalize)
{
    cplx *psi = (cplx *)psi_d;
    const uint64_t dim = 1ull << n;
    const double P = oracle_prob(psi_d, n, mask, val);
    if (P == 0.0) return 0.0;
    const double s = renormalize ? 1.0 / sqrt(P) : 1.0;
#pragma omp parallel for schedule(static)
    for (int64_t ii = 0; ii < (int64_t)dim; ++ii) {
        uint64_t i = (uint64_t)ii;
        psi[i] = ((i & mask) == val) ? psi[i] * s : 0.0;
    }
    return P;
}

/* <a|b> = sum conj(a_i) b_i, written to out[0] (re), out[1] (im) */
void oracle_inner(const double *a_d, const double *b_d, int n, double *out)
{
    const cplx *a = (const cplx *)a_d, *b = (const cplx *)b_d;
    const uint64_t dim = 1ull << n;
    double re = 0.0, im = 0.0;
#pragma omp parallel for reduction(+ : re, im) schedule(static)
    for (int64_t ii = 0; ii < (int64_t)dim; ++ii) {
        cplx z = conj(a[ii]) * b[ii];
        re += creal(z);
        im += cimag(z);
    }
    out[0] = re;
    out[1] = im;
}

int oracle_threads(void)
{
#ifdef _OPENMP
    int t = 1;
#pragma omp parallel
    {
#pragma omp single
        t = omp_get_num_threads();
    }
    return t;
#else
    return 1;
#endif
}

/*
 * QSP polynomial p(x) = <0| e^{i phi_0 Z} W(x) e^{i phi_1 Z} ... W(x) e^{i phi_d Z} |0>
 * with W(x) = [[x, i s], [i s, x]], s = sqrt(1 - x^2) (the W_x convention of
 * the QSVT construction, Sec. II.D.5), at n_x points: the first row of the
 * running product of the 2x2 matrices, left to right, one point per loop
 * iteration.  phases has d + 1 entries; out holds n_x complex values.
 */
void oracle_qsp_poly(const double *phases, uint64_t d, const double *x, uint64_t n_x, double *out_d)
{
    cplx *out = (cplx *)out_d;
    cplx *e = (cplx *)malloc((d + 1) * sizeof(cplx));
    if (!e) {
        for (uint64_t k = 0; k < n_x; ++k) out[k] = NAN;
        return;
    }
    for (uint64_t j = 0; j <= d; ++j) e[j] = cexp(I * phases[j]);
#pragma omp parallel for schedule(static)
    for (int64_t kk = 0; kk < (int64_t)n_x; ++kk) {
        const double xv = x[kk];
        const double s = sqrt(fmax(0.0, 1.0 - xv * xv));
        cplx r0 = e[0], r1 = 0.0;
        for (uint64_t j = 1; j <= d; ++j) {
            /* [r0, r1] . W(x) . diag(e^{i phi_j}, e^{-i phi_j}) */
            const cplx n0 = (r0 * xv + r1 * (I * s)) * e[j];
            const cplx n1 = (r0 * (I * s) + r1 * xv) * conj(e[j]);
            r0 = n0;
            r1 = n1;
        }
        out[kk] = r0;
    }
    free(e);
}
