/*
 * libsv — state-vector simulation of elementary-gate circuits on one MI355X
 * (gfx950), the simulator behind the explicit circuit demonstration of the
 * Carleman-linearised lattice Boltzmann QSVT solver (Sec. III.E; the circuit
 * itself is built in Sec. II.D: block encodings, the L-matrix encoding and
 * the QSVT ladder).
 *
 * Conventions shared by every entry point
 *   - Qubit j is bit j of the amplitude index (little-endian).
 *   - Host amplitude buffers are interleaved complex128: re0, im0, re1, im1, ...
 *   - Every function returns SV_OK (0) or a negative SV_E* code.  Arguments are
 *     validated on the host before any launch; on an error nothing is launched
 *     and the state is unchanged.  sv_last_error() gives a message for the
 *     calling thread's last failure.
 *   - Calls are synchronous with respect to the host: when a call returns, its
 *     device work has completed.  Work is issued on the state's stream.
 *   - The library owns all device memory it allocates.  Host buffers passed in
 *     belong to the caller and are only read or written during the call.
 *   - Calls that use one sv_state must not overlap in time (no internal locks).
 */
#ifndef SV_H
#define SV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- error codes ---------------------------------------------------------- */
#define SV_OK            0
#define SV_EINVAL       -1  /* bad argument: qubit >= n, target among controls, overlap, bad kind ... */
#define SV_ENOMEM       -2  /* the device cannot hold the requested state or plan */
#define SV_EZEROPROB    -3  /* post-selection on a subspace of probability 0; state unchanged */
#define SV_EDEVICE      -4  /* a HIP runtime call failed */
#define SV_EUNSUPPORTED -5  /* valid request outside what the library implements */

/* ---- amplitude precision -------------------------------------------------- */
#define SV_C64  0   /* complex64: float re, im (8 bytes per amplitude)   */
#define SV_C128 1   /* complex128: double re, im (16 bytes per amplitude) */

/* ---- gate IR --------------------------------------------------------------
 * One op is a 40-byte POD record.  A gate with controls acts only on the basis
 * states i with (i & ctrl_mask) == ctrl_val (ctrl_val must be a subset of
 * ctrl_mask; a 0 under a mask bit is an open control).  `param` is an offset
 * into the caller's float64 parameter pool.
 *
 *  kind             target      width        params  action
 *  SV_OP_U          qubit t     0            8       2x2 complex matrix (u00,u01,u10,u11 as re,im)
 *                                                    on each pair (i, i|2^t), i with bit t = 0
 *  SV_OP_X          qubit t     0            0       exchange the two amplitudes of each pair
 *  SV_OP_PHASE      qubit t     0            1       multiply by exp(i theta) where bit t = 1
 *  SV_OP_RY         qubit t     0            1       [[cos th/2, -sin th/2],[sin th/2, cos th/2]]
 *  SV_OP_INC        base b      width w      0       register v = bits [b,b+w): v -> v+1 mod 2^w
 *  SV_OP_DEC        base b      width w      0       v -> v-1 mod 2^w
 *  SV_OP_SWAP       qubit a     qubit b      0       exchange qubits a and b
 *  SV_OP_PROJPHASE  signal s    0            1       multiply by exp(i theta (1 - 2 (s xor z))),
 *                                                    z = [(i & ctrl_mask) == ctrl_val]: the
 *                                                    projector-controlled phase of one QSVT step
 *                                                    (QSVT circuit figure, Sec. II.D.5); here
 *                                                    ctrl_* is the projector condition
 * The elementary gate set of Sec. III.F.2 (Toffoli, CNOT, H, X, R_Y, S, S^dagger and
 * their multi-controlled forms) maps onto U, X, RY and PHASE.
 *
 * Complex64 plans compute in FP32 and choose the FP32 form of each parameter so
 * that long sequences keep the norm: uncontrolled Hadamard-type matrices in
 * pairs of exactly representable scaled matrices whose scales multiply to 1;
 * projector phases rounded, within an ulp of the nearest and no further in
 * angle, so that their norm factors multiply to 1 within 1e-7; real 2x2
 * matrices in tile passes as hi + lo pairs when sv_apply_opts.split_real asks;
 * the 2x2 matrices of plain launches always as hi + lo pairs.
 */
#define SV_OP_U          0
#define SV_OP_X          1
#define SV_OP_PHASE      2
#define SV_OP_RY         3
#define SV_OP_INC        4
#define SV_OP_DEC        5
#define SV_OP_SWAP       6
#define SV_OP_PROJPHASE  7

typedef struct {
    uint32_t kind;
    uint32_t target;
    uint32_t width;
    uint32_t flags;      /* must be 0 */
    uint64_t ctrl_mask;
    uint64_t ctrl_val;
    uint64_t param;
} sv_op;

/* ---- execution options ---------------------------------------------------- */
#define SV_MODE_PLAIN 0   /* one kernel launch per gate, each a sweep of the touched subspace */
#define SV_MODE_FUSED 1   /* gates grouped into LDS-resident tile passes (one HBM sweep each) */

typedef struct {
    int mode;          /* SV_MODE_PLAIN or SV_MODE_FUSED                                  */
    int tile_qubits;   /* fused: qubits resident per tile, 0 = automatic                   */
    int reg_qubits;    /* fused: qubits held in registers per thread, 0 = automatic; the
                          workgroup has 2^(tile_qubits - reg_qubits) threads, 64 to 256,
                          or 512 for compiled plans                                  */
    int dense_min_ops; /* fused: a run of at least this many consecutive ops acting
                          inside dense_qubits qubits (targets and controls) becomes one
                          dense block applied on matrix cores (FP32 or split BF16 for
                          complex64, FP64 for complex128); 0 = never; negative = the
                          planner's cost model picks the length (one dense sweep of the
                          state against the run's ops inside tile passes)            */
    int tile_launch;   /* fused: how tile passes are launched. SV_TILE_LAUNCH_AUTO (0),
                          SV_TILE_LAUNCH_GRID (1): one workgroup per tile,
                          SV_TILE_LAUNCH_PERSISTENT (2): one resident workgroup set that
                          walks the tiles, loading the next tile while computing one.
                          Results are identical; only the timing differs.            */
    int plain_split;   /* fused: SV_PLAIN_SPLIT_AUTO (0): a group of ops whose plain
                          launches (each sweeping only its controlled subspace) are
                          modelled cheaper than one tile pass over the whole state runs
                          as those launches; SV_PLAIN_SPLIT_OFF (1): tile passes only
                          (required for plans given to sv_batch_create)              */
    int compile;       /* fused: how tile passes run.  SV_COMPILE_OFF (1): the generic
                          tile kernel, which reads each pass's op records at run time;
                          SV_COMPILE_ON (2): every distinct pass is compiled at plan
                          creation (hiprtc, for the current device) into a kernel with
                          its op list written out, and runs as that kernel (same
                          arithmetic, bit-identical states; plan creation takes
                          longer), in either launch form; SV_COMPILE_AUTO (0): ON for
                          states of at least 21 qubits and for tiles of 512 threads,
                          OFF otherwise, and OFF if compilation is unavailable (then a
                          512-thread plan is refused with SV_EUNSUPPORTED)            */
    int dense_bf16;    /* fused, complex64: 0 = dense blocks on FP32 matrix cores;
                          1 = on BF16 matrix cores with split operands (each FP32
                          value as a BF16 high part plus a BF16 low part, three
                          products, FP32 accumulation: about 2^-16 relative
                          error per block instead of 2^-24)                          */
    int peephole;      /* cancellation of adjacent inverse pairs (Sec. III.F.2: identical
                          Toffoli pairs and X-X pairs, here every multi-controlled X, and
                          also SWAP pairs and an INC next to the DEC of the same register,
                          all with identical controls), adjacent meaning that no op in
                          between acts on any of the pair's qubits: the pair is the
                          identity and is dropped before planning.  SV_PEEPHOLE_AUTO (0):
                          on in fused mode, off in plain mode (which keeps one launch per
                          op); SV_PEEPHOLE_OFF (1); SV_PEEPHOLE_ON (2): on in both modes */
    int dense_qubits;  /* fused: qubits per dense block: 0 or 5 = five (32 x 32 blocks);
                          6 = six (64 x 64 blocks, complex64 only: SV_EUNSUPPORTED for
                          complex128), on FP32 or split-BF16 matrix cores as dense_bf16
                          says                                                       */
    int coalesce_qubits; /* fused: the lowest qubits kept resident in every tile pass, so that
                          each tile reads and writes runs of 2^coalesce_qubits contiguous
                          amplitudes; 0 = automatic (256-byte runs: 5 for complex64, 4
                          for complex128), else 1 to 8.  Fewer leave more of the tile to
                          other qubits (fewer passes, each applying more gates); runs
                          shorter than a 128-byte line cost extra HBM traffic         */
    int split_real;    /* fused, complex64: real 2x2 gates (rotations such as the value
                          loads of a block encoding, Sec. II.D.2, II.D.3) in tile passes
                          carry each matrix entry as its FP32 rounding plus the FP32
                          rounding of the remainder, so their matrices hold the norm to
                          about 2^-48 instead of 2^-24 (four more FMAs per amplitude
                          pair).  A gate repeated in every call of a long sequence
                          otherwise scales its controlled subspace by the same factor
                          each time.  SV_SPLIT_REAL_AUTO (0): on when the sum over the
                          plan's real gates of their FP32 matrices' column-norm errors
                          exceeds 1e-4 (a bound on the norm change they can cause);
                          SV_SPLIT_REAL_OFF (1); SV_SPLIT_REAL_ON (2).  Plain launches of
                          complex64 plans always carry their matrices this way       */
} sv_apply_opts;

#define SV_TILE_LAUNCH_AUTO 0
#define SV_TILE_LAUNCH_GRID 1
#define SV_TILE_LAUNCH_PERSISTENT 2

#define SV_PLAIN_SPLIT_AUTO 0
#define SV_PLAIN_SPLIT_OFF 1

#define SV_COMPILE_AUTO 0
#define SV_COMPILE_OFF 1
#define SV_COMPILE_ON 2

#define SV_PEEPHOLE_AUTO 0
#define SV_PEEPHOLE_OFF 1
#define SV_PEEPHOLE_ON 2

#define SV_SPLIT_REAL_AUTO 0
#define SV_SPLIT_REAL_OFF 1
#define SV_SPLIT_REAL_ON 2

typedef struct sv_state sv_state;
typedef struct sv_plan sv_plan;

typedef struct {
    uint64_t n_ops;           /* IR ops planned                                      */
    uint64_t n_launches;      /* kernel launches per execution                       */
    uint64_t n_tile_passes;   /* launches that are fused tile passes                 */
    uint64_t n_stages;        /* register stages summed over tile passes             */
    uint64_t bytes_moved;     /* algorithmic HBM bytes per execution (reads+writes)  */
    uint64_t tile_pass_bytes; /* algorithmic HBM bytes of one tile pass              */
    int      tile_qubits;     /* b actually used (fused)                             */
    int      reg_qubits;      /* register qubits actually used (fused)               */
    uint64_t n_dense_passes;  /* launches that apply a dense 5-qubit block           */
    uint64_t n_dense_ops;     /* IR ops absorbed into dense blocks                   */
    uint64_t n_split_ops;     /* fused: IR ops run as plain launches by the cost model */
    uint64_t n_compiled_kernels; /* compiled plans: distinct specialised pass kernels; 0 otherwise */
    int      dense_min_ops;   /* fused: the run length that makes a dense block (0: none) */
    uint64_t n_cancelled_ops; /* IR ops dropped as adjacent inverse pairs (peephole)  */
    uint64_t touched_bytes;   /* HBM bytes per execution at 128-byte line granularity: a
                                 plain launch whose controls sit on qubits inside a line
                                 still reads and writes whole lines (>= bytes_moved)   */
} sv_plan_info;

/* ---- state lifetime ------------------------------------------------------- */

/* sv_alloc — the simulated register of the circuit of Sec. II.D (system
 * register: Carleman index, Taylor index k and time step m; row labels i_L and
 * i_A, target t; the QSVT signal qubit of Sec. II.D.5), as 2^n_qubits
 * amplitudes in device memory (1 <= n_qubits <= 36; the qubit counts of
 * Sec. III.F.1).  init: NULL for |0...0>, else 2^n interleaved complex128
 * host values, converted to the state's precision: this is how the
 * right-hand side b is loaded, f(0) in the m = 0 block and zero elsewhere
 * (Sec. II.D.5).  stream: a hipStream_t to issue work on, or NULL for one the
 * library creates.  On success *out owns the state (free with sv_free).
 * Errors: SV_EINVAL (bad n_qubits or dtype, out NULL), SV_ENOMEM (the state
 * does not fit the free device memory), SV_EDEVICE. */
int sv_alloc(int n_qubits, int dtype, const double *init, void *stream, sv_state **out);

/* sv_free — releases a state of sv_alloc / sv_alloc_batch (the register of
 * Sec. II.D) and its stream if the library created it.  NULL is accepted. */
int sv_free(sv_state *s);

/* sv_info — qubit count (Sec. III.F.1) and precision of a state; either
 * output pointer may be NULL.  SV_EINVAL for a NULL state. */
int sv_info(const sv_state *s, int *n_qubits, int *dtype);

/* ---- circuits ------------------------------------------------------------- */

/* sv_apply_circuit — applies ops[0..n_ops) in order: the elementary gate set
 * of Sec. III.F.2 (Toffoli, CNOT, H, X, R_Y, S, S^dagger) and the
 * multi-controlled forms the block encodings of Sec. II.D.1-II.D.4 are built
 * from (value loads R_Y, controlled increments and decrements for streaming
 * and the k, m counters, register swaps), plus the projector-controlled phase
 * of the QSVT ladder (Sec. II.D.5).  params is the float64 parameter pool the
 * ops index (n_params reals); both arrays are the caller's and only read.
 * opts NULL = fused.  The call plans, runs and frees a plan.  Errors:
 * SV_EINVAL (an op fails validation: nothing is launched and the state is
 * unchanged), SV_ENOMEM, SV_EDEVICE, SV_EUNSUPPORTED. */
int sv_apply_circuit(sv_state *s, const sv_op *ops, size_t n_ops,
                     const double *params, size_t n_params, const sv_apply_opts *opts);

/* sv_plan_create — plans an op list once for states of n_qubits qubits and
 * precision dtype so that it can run many times: the QSVT ladder of
 * Sec. II.D.5 applies the same U_L and U_L^dagger op lists d times, so its
 * elementary gate count is linear in d (Sec. III.F.2).  The plan copies what
 * it needs from ops and params.  Errors as sv_apply_circuit; *out owns the
 * plan (free with sv_plan_free). */
int sv_plan_create(int n_qubits, int dtype, const sv_op *ops, size_t n_ops,
                   const double *params, size_t n_params, const sv_apply_opts *opts,
                   sv_plan **out);

/* sv_plan_free — releases a plan of sv_plan_create (the reusable U_L or
 * U_L^dagger of Sec. II.D.5).  NULL is accepted. */
int sv_plan_free(sv_plan *p);

/* sv_plan_get_info — launch and byte counts of a plan (the per-call cost of
 * the U_L oracle, Sec. III.F.2).  SV_EINVAL for NULL arguments. */
int sv_plan_get_info(const sv_plan *p, sv_plan_info *info);

/* sv_plan_execute — runs a plan `repeat` times on a state of matching size and
 * precision (repeated U_L calls of the ladder, Sec. II.D.5).  SV_EINVAL on a
 * size or precision mismatch or repeat < 0 (nothing launched). */
int sv_plan_execute(sv_plan *p, sv_state *s, int repeat);

/* sv_plan_execute_seq — runs plans[seq[0]], plans[seq[1]], ... (seq_len
 * entries) in one host call: the QSVT ladder of Sec. II.D.5 as phase, U_L,
 * phase, U_L^dagger, ...  plans holds n_plans entries; every seq entry must
 * lie in [0, n_plans), and every referenced plan must match the state, or the
 * call returns SV_EINVAL before any launch. */
int sv_plan_execute_seq(sv_plan *const *plans, size_t n_plans, const int32_t *seq, size_t seq_len,
                        sv_state *s);

/* sv_plan_time — as sv_plan_execute (the ladder's repeated oracle calls,
 * Sec. II.D.5), bracketed by HIP events on the state's stream; *ms is the
 * elapsed device time of all repeats.  SV_EINVAL for ms NULL or repeat < 1. */
int sv_plan_time(sv_plan *p, sv_state *s, int repeat, double *ms);

/* ---- reductions, post-selection, read-out (all accumulate in FP64) ---------- */

/* sv_postselect — the post-selection that completes the QSVT solve: the
 * solution sits in the block where every block-encoding ancilla (the row
 * labels and the target) and the QSVT signal qubit are 0 (Sec. II.D.5), and
 * the final-time state in the rows m >= N_t of the time-step register, which
 * the terminal-copy rows of L fill (Sec. II.D.4); the success probability of
 * that projection scales as 1/kappa (Sec. IV.D.1).
 * *prob_out = P = sum of |a_i|^2 over (i & mask) == value, in FP64 for either
 * precision.  keep != 0: the other amplitudes are set to zero; renormalize
 * != 0 then divides the kept ones by sqrt(P).  mask = 0, value = 0, keep = 0
 * returns the squared norm (norm drift check).  Errors: SV_EINVAL (mask or
 * value outside the state, value not inside mask), SV_EZEROPROB (P == 0 with
 * keep != 0; the state is unchanged). */
int sv_postselect(sv_state *s, uint64_t mask, uint64_t value, int keep, int renormalize,
                  double *prob_out);

/* sv_amplitudes — read-out of amplitudes [offset, offset+count) to the
 * caller's host buffer `out` (2 count doubles, interleaved complex128): the
 * simulated output state that Sec. III.E compares with the classical Taylor
 * solution (a full read-out that only a classical simulation affords,
 * Sec. IV.D.1).  Allocates a device staging buffer per call.  SV_EINVAL for a
 * range outside the state. */
int sv_amplitudes(const sv_state *s, uint64_t offset, uint64_t count, double *out);

/* sv_amplitudes_noalloc — sv_amplitudes for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc): it calls no allocating routine and stages through a
 * fixed device array of 262144 complex128 amplitudes (4 MiB), which each
 * device holds from the library's set-up (the first sv_alloc or
 * sv_plan_create on it) until the process ends.  Same arguments, layout and
 * result as sv_amplitudes; count may be at most 262144 (a larger count, or a
 * range outside the state, gives SV_EINVAL and copies nothing).  Every call on
 * one device shares that array: calls that overlap in time on one device
 * (from several host threads, or on several streams) race and must not be
 * made. */
int sv_amplitudes_noalloc(const sv_state *s, uint64_t offset, uint64_t count, double *out);

/* sv_set_amplitudes — overwrites amplitudes [offset, offset+count) from the
 * caller's host interleaved complex128 values: the right-hand side b, f(0) in
 * the m = 0 block (Sec. II.D.5).  SV_EINVAL for a range outside the state. */
int sv_set_amplitudes(sv_state *s, uint64_t offset, uint64_t count, const double *in);

/* sv_copy — copies the amplitudes of src into dst (same qubit count;
 * precisions may differ): a reference state kept beside a run, for the
 * comparisons of Sec. III.E.  SV_EINVAL on a size mismatch. */
int sv_copy(sv_state *dst, const sv_state *src);

/* sv_inner — <a|b> = sum conj(a_i) b_i in FP64 (same qubit count; precisions
 * may differ): the overlap behind the fidelity of a run against a reference
 * state, the agreement measure of Sec. III.E.  SV_EINVAL on a size mismatch. */
int sv_inner(const sv_state *a, const sv_state *b, double *re, double *im);

/* ---- batches of independent circuits ---------------------------------------
 * Many independent instances of the circuit of Sec. II.D (different grid
 * sizes, Taylor orders and step counts, hence different qubit counts, as in
 * the parameter scans of Sec. III.D-III.E) run together on one device. */

/* sv_alloc_batch — `count` registers of the circuit of Sec. II.D, of
 * n_qubits[i] qubits and precision dtype, in one device arena (each state
 * starts on a 2 MiB boundary), all on one stream (stream, or a library-created
 * one when NULL), each initialised to |0...0>.  out[i] receives the states;
 * free each with sv_free (the arena goes with the last one).  On an error no
 * state is returned and nothing stays allocated. */
int sv_alloc_batch(int count, const int *n_qubits, int dtype, void *stream, sv_state **out);

typedef struct sv_batch sv_batch;

/* sv_batch_create — binds plans[i] (each the ladder or oracle of one instance
 * of Sec. II.D.5) to states[i] for i < count; the states must be distinct and
 * on one device.  Two forms:
 *  - compiled plans (sv_apply_opts.compile): every instance runs its own plan,
 *    the instances spread over four side streams (largest first, each to the
 *    least-loaded stream by modelled work) that fork from and join back to the
 *    first state's stream, so small instances run alongside each other and the
 *    large ones.  The batch holds the plans until sv_batch_free (sv_plan_free
 *    may be called earlier); group_bytes is not used.
 *  - otherwise: every plan must be fused (tile passes only), with one tile
 *    geometry and precision across the batch, and the states must come from
 *    one sv_alloc_batch arena.  Instances, ordered by size, are packed into
 *    groups of at most group_bytes of state (0: 192 MiB, about what the
 *    last-level cache holds; UINT64_MAX: one group); a group runs level by
 *    level, each level one launch over the tiles of all its instances.  The
 *    batch keeps its own copy of the plans' tables (the plans may be freed).
 * use_graph != 0 captures one execution in a HIP graph on first execution and
 * replays it afterwards.  The batch points into the states: free it before
 * them. */
int sv_batch_create(sv_state *const *states, sv_plan *const *plans, size_t count, int use_graph,
                    uint64_t group_bytes, sv_batch **out);

/* sv_batch_execute — runs every instance's plan (Sec. II.D.5 ladders)
 * `repeat` times; returns when the work is done. */
int sv_batch_execute(sv_batch *b, int repeat);

/* sv_batch_time — as sv_batch_execute (Sec. II.D.5 ladders), bracketed by HIP
 * events (graph capture, if any, happens before the timed region); *ms is the
 * device time of all repeats. */
int sv_batch_time(sv_batch *b, int repeat, double *ms);

/* sv_batch_levels — launches and groups of one execution, and the total IR
 * ops (elementary gates of Sec. III.F.2) it applies. */
int sv_batch_levels(const sv_batch *b, uint64_t *launches, uint64_t *groups, uint64_t *gates);

/* sv_batch_free — releases a batch (its copies of the Sec. II.D.5 plans). */
int sv_batch_free(sv_batch *b);

/* ---- diagnostics (library-defined; no passage of the paper) --------------- */
const char *sv_strerror(int code);
const char *sv_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SV_H */
