/*
 * tanq.h -- C ABI of the MI355X (gfx950) density-matrix superoperator engine.
 *
 * Method (TANQ-Sim, arXiv 2404.13184):
 *   - rho is stored as the column-stacked vector vec(rho) of length 4^n (Sec. 3.1):
 *     element rho[r][c] sits at index r + c * 2^n.  Qubit q is bit q of r (and bit q + n
 *     of the vec index for the column), as in the strided index map of Sec. 3.1.
 *   - A gate or Kraus channel K_i on j qubits becomes the superoperator
 *     S = sum_i conj(K_i) (x) K_i (Sec. 3.1, from vec(A B C) = (C^T (x) A) vec(B)), and the
 *     simulation is |rho(t)> = S |rho(t-1)> (Eq. eq:sp).
 *   - Applying S is a batched small complex GEMM over the 4^(n-k) groups of amplitudes
 *     that differ only in the 2k target bits (Sec. 3.1 "im2col" view, Sec. 3.2 tensor-core
 *     mapping); consecutive operations are fused into k-qubit blocks (Sec. 3.3).
 *
 * Conventions used by every entry point:
 *   - Complex numbers are interleaved (re, im).  FP64 state = complex128 (16 B/element),
 *     FP32 state = complex64 (8 B/element).
 *   - A j-qubit matrix on qubits (q_0..q_{j-1}) is row-major, M[out * 2^j + in], and its
 *     local basis index is sum_t b_{q_t} 2^t (the first listed qubit is the least
 *     significant bit).
 *   - A k-qubit superoperator S is row-major 4^k x 4^k complex128, and its local index is
 *     row_local + 2^k * col_local, with row_local/col_local as above.
 *   - Every call returns TANQ_OK (0) or a negative tanq_status; no C++ exception crosses
 *     the ABI.  On error, tanq_last_error() describes the failure (per calling thread).
 *   - Calls that take a tanq_dm run stream-ordered on the stream given at creation and
 *     return before the GPU finishes unless documented as synchronising.
 *   - Handles are not thread-safe: one handle must not be used by two threads at once.
 */
#ifndef TANQ_H
#define TANQ_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int tanq_status;

#define TANQ_OK 0
#define TANQ_E_ARG (-1)         /* invalid argument (bad n, qubits, sizes, NULL pointer) */
#define TANQ_E_OOM (-2)         /* device or pinned-host allocation failed or over budget */
#define TANQ_E_HIP (-3)         /* a HIP runtime call failed */
#define TANQ_E_STATE (-4)       /* handle in the wrong state (e.g. mismatched precision) */
#define TANQ_E_UNSUPPORTED (-5) /* valid request that this build does not implement */
#define TANQ_E_AGAIN (-6)       /* server: result not ready yet */
#define TANQ_E_CANCELED (-7)    /* server: the request was cancelled (tanq_server_cancel) */
#define TANQ_E_TIMEOUT (-8)     /* server: the request did not finish within the server's timeout */

typedef enum { TANQ_F64 = 0, TANQ_F32 = 1 } tanq_prec;

/* Fusion modes for tanq_fuse(max_width): */
#define TANQ_FUSE_AUTO 0    /* choose 2 or 3 by the autotuner's measured cost model */
#define TANQ_FUSE_NONE (-1) /* plain method: one superoperator per operation, no fusion */
#define TANQ_FUSE_PAPER (-2) /* Sec. 3.3: merge consecutive 1q ops on one qubit, then
                                consecutive 2q ops on the same ordered pair */
/* 1, 2, 3: greedy blocks of at most that many qubits (Sec. 3.3 generalised). */

typedef struct tanq_dm_s* tanq_dm;
typedef struct tanq_circuit_s* tanq_circuit;
typedef struct tanq_fused_s* tanq_fused;

/* Text of the last error on the calling thread ("" if none).  Owned by the library. */
const char* tanq_last_error(void);

/* Library version as 10000*major + 100*minor + patch. */
int tanq_version(void);

/* ---------------------------------------------------------------------------------------
 * Density matrices (Sec. 2.1; storage vec(rho), Sec. 3.1).
 * ------------------------------------------------------------------------------------- */

/* Allocate a device-resident vec(rho) of 4^n elements of precision p and set
 * rho = |0..0><0..0|.  hip_stream: a hipStream_t (NULL = the null stream) on which every
 * later call on this handle is ordered; the caller keeps the stream alive.  The handle
 * owns the memory.  Errors: TANQ_E_ARG if n < 1 or n > 17 or out == NULL; TANQ_E_OOM if
 * the footprint exceeds free device memory. */
tanq_status tanq_dm_init(int n, tanq_prec p, void* hip_stream, tanq_dm* out);

/* Wrap caller-owned device memory (4^n contiguous complex128 or complex64 elements, e.g.
 * a PyTorch tensor).  The contents are left as they are; the caller keeps the memory alive
 * until tanq_dm_free.  Same errors as tanq_dm_init, plus TANQ_E_ARG for a NULL pointer or
 * a pointer not 16-byte aligned. */
tanq_status tanq_dm_wrap(int n, tanq_prec p, void* dev_ptr, void* hip_stream, tanq_dm* out);

/* Release the handle (and its memory if owned).  Synchronises the handle's stream. */
tanq_status tanq_dm_free(tanq_dm d);

/* rho = |0..0><0..0| (stream-ordered). */
tanq_status tanq_dm_reset(tanq_dm d);

/* rho <- factor * rho in place (stream-ordered), e.g. factor = 1/tr to renormalise the state
 * itself rather than its outputs.  Every element is read once and written once with 16-byte
 * accesses and nothing else, so the call is also the plain in-place streaming pass over the
 * state buffer against which the apply kernels' bandwidth is measured.  TANQ_E_ARG if factor
 * is not finite.  In FP32 the factor is rounded to float. */
tanq_status tanq_dm_scale(tanq_dm d, double factor);

/* The matrix units' sustained rate on the current device, in TFLOP/s, in the shape of the
 * pass kernels' multiplication loop (Sec. 3.2's batched GEMM on the matrix units) but with
 * nothing else: one workgroup of eight waves per CU, each repeating 16x16x4 products of
 * precision p (FP64, or FP32 for TANQ_F32) in three independent accumulation chains with
 * register operands, plus the 3M combination.  This is the ceiling that kernel's products can
 * reach on this device and clock, next to the datasheet peak.  Allocates and frees a small
 * device buffer, uses a stream of its own and synchronises it (about 0.1 s).  E_ARG for a bad
 * precision or a NULL pointer. */
tanq_status tanq_mfma_rate(tanq_prec p, double* tflops);

/* Number of qubits, precision, element count (4^n) and device pointer of a handle. */
tanq_status tanq_dm_query(tanq_dm d, int* n, int* prec, uint64_t* elements, void** dev_ptr);

/* Copy vec(rho) to / from host memory (bytes must equal 4^n * element size).  Both
 * synchronise the stream before returning. */
tanq_status tanq_dm_read(tanq_dm d, void* host, size_t bytes);
tanq_status tanq_dm_write(tanq_dm d, const void* host, size_t bytes);

/* Fill vec(rho) with seeded pseudo-random complex values (not a density matrix): element
 * e gets re = u(2x), im = u(2x + 1) with x = (seed << 40) + e and u(c) the top 53 bits of
 * SplitMix64(c) (Steele, Lea & Flood 2014) scaled to [-0.5, 0.5).  Input generator for
 * linearity checks of single applies at full size.  Stream-ordered. */
tanq_status tanq_dm_fill_random(tanq_dm d, uint64_t seed);

/* Copy `count` elements of vec(rho) at the vec indices idx[0..count-1] (host array) into
 * host_out (count complex values of the handle's precision).  A gather kernel reads them on
 * the device, so only the sampled elements cross PCIe.  TANQ_E_ARG if an index >= 4^n.
 * Synchronises. */
tanq_status tanq_dm_gather(tanq_dm d, size_t count, const uint64_t* idx, void* host_out);

/* Block until all work queued on the handle's stream is done. */
tanq_status tanq_sync(tanq_dm d);

/* ---------------------------------------------------------------------------------------
 * Circuits: an ordered list of gates and Kraus channels (the transformations of Eq.
 * eq:dmsim; noise as Kraus sets, Sec. 3.5).
 * ------------------------------------------------------------------------------------- */

/* Create an empty circuit on n qubits (1 <= n <= 17). */
tanq_status tanq_circuit_create(int n, tanq_circuit* out);
tanq_status tanq_circuit_free(tanq_circuit c);

/* Append a j-qubit gate U (2^j x 2^j complex128, row-major) on qubits[0..j-1].
 * j in {1, 2, 3}; qubits distinct and < n.  Arrays are copied. */
tanq_status tanq_circuit_add_gate(tanq_circuit c, int j, const int* qubits, const double* U);

/* Append a j-qubit channel given by m >= 1 Kraus matrices K (m consecutive 2^j x 2^j
 * complex128 row-major matrices).  The channel is rho -> sum_i K_i rho K_i^dagger.  The set
 * need not be trace preserving: a post-selection (a projector) lowers the trace to the
 * probability of the selected outcomes, which tanq_probs reports as the trace. */
tanq_status tanq_circuit_add_kraus(tanq_circuit c, int j, const int* qubits, int m, const double* K);

/* Append `count` operations at once.  Operation i acts on qubits[3i .. 3i + j[i] - 1] with
 * m[i] Kraus matrices (2^j[i] x 2^j[i] complex128 row-major each; m[i] = 1 with a unitary is a
 * gate) stored at pool[koff[i] ..] (offsets in doubles).  pool (pool_doubles doubles) is copied
 * once and shared by the operations, so a channel repeated through a circuit costs one copy.
 * All-or-nothing: on TANQ_E_ARG (bad width, qubit, count or offset) nothing is appended. */
tanq_status tanq_circuit_add_ops(tanq_circuit c, int count, const int* j, const int* qubits, const int* m,
                                 const int64_t* koff, const double* pool, size_t pool_doubles);

/* Number of operations appended so far. */
tanq_status tanq_circuit_size(tanq_circuit c, int* count);

/* ---------------------------------------------------------------------------------------
 * Fusion (Sec. 3.3) and superoperator construction (Sec. 3.1).
 * ------------------------------------------------------------------------------------- */

typedef struct {
  int count;       /* number of fused superoperators */
  int count_k[4];  /* how many have k = 1, 2, 3 qubits (index 0 unused) */
  int source_ops;  /* operations absorbed */
  int max_width;   /* width actually used (1, 2 or 3), or TANQ_FUSE_NONE / TANQ_FUSE_PAPER */
  int prec;        /* tanq_prec the fused list is packed for */
  int n;           /* qubits of the circuit */
} tanq_fused_info_t;

/* Plan blocks on the host, then on the GPU: build each operation's superoperator
 * S = sum_i conj(K_i) (x) K_i and compose the operations of each block, in circuit order,
 * in FP64; finally pack each block for the apply kernel of precision p (FP32 blocks are
 * rounded once from the FP64 composition).  max_width: TANQ_FUSE_AUTO, TANQ_FUSE_NONE,
 * TANQ_FUSE_PAPER or 1..3.  The result is device-resident and usable with any tanq_dm of
 * the same n and precision.  Synchronises hip_stream before returning. */
tanq_status tanq_fuse(tanq_circuit c, int max_width, tanq_prec p, void* hip_stream, tanq_fused* out);
tanq_status tanq_fused_info(tanq_fused f, tanq_fused_info_t* info);
/* Waits for all work queued on f's device (applies of f may be in flight on any stream), then
 * releases its device memory. */
tanq_status tanq_fused_free(tanq_fused f);

/* Host-only planning query (no GPU needed): the block that each operation of c joins under
 * max_width (same modes as tanq_fuse except TANQ_FUSE_AUTO, which is rejected).
 * op_block receives one block index per operation (size of c); *nblocks the block count.
 * Blocks are applied in increasing index order; operations inside a block keep circuit
 * order. */
tanq_status tanq_fuse_plan(tanq_circuit c, int max_width, int* op_block, int* nblocks);
/* The block assignment tanq_fuse(c, max_width, p) makes under the current pass limit: as
 * tanq_fuse_plan, then ordered for multi-superoperator passes (commuting blocks moved next to
 * each other; see tanq_set_pass_limit).  Host only. */
tanq_status tanq_fuse_plan_ordered(tanq_circuit c, int max_width, tanq_prec p, int* op_block, int* nblocks);

/* Copy fused superoperator idx back to the host: *k, qubits[0..k-1] (ascending) and the
 * FP64 composition S (4^k x 4^k complex128 row-major, caller provides 2*16^k doubles). */
tanq_status tanq_fused_get(tanq_fused f, int idx, int* k, int* qubits, double* S);

/* ---------------------------------------------------------------------------------------
 * Applying superoperators (Eq. eq:sp; Sec. 3.1-3.2).
 * ------------------------------------------------------------------------------------- */

/* In place: for every group g of the 4^(n-k) groups, x <- S x on the 4^k amplitudes whose
 * target bits (q_t and q_t + n) take every value.  S: host 4^k x 4^k complex128 (copied
 * into a pinned ring before return; FP32 handles round it once).  k in {1, 2, 3}, k <= n,
 * qubits distinct and < n.  Stream-ordered, asynchronous. */
tanq_status tanq_apply_superop(tanq_dm d, int k, const int* qubits, const double* S);

/* Apply every fused superoperator of f in order (or those with index in [begin, end)).
 * f must have been built for d's n and precision (TANQ_E_STATE otherwise). */
tanq_status tanq_apply_fused(tanq_dm d, tanq_fused f);
tanq_status tanq_apply_fused_range(tanq_dm d, tanq_fused f, int begin, int end);

/* ---------------------------------------------------------------------------------------
 * Autotuning of the apply kernels (tile shape, workgroup size and staging per qubit count,
 * width and precision).
 * ------------------------------------------------------------------------------------- */

typedef struct {
  int k;          /* superoperator width (2 or 3) */
  int prec;       /* tanq_prec */
  int tile_bits;  /* log2 of the elements one workgroup stages per tile */
  int threads;    /* workgroup size */
  int staging;    /* 0: tiles staged through registers; 1: direct global-to-LDS loads into two
                     LDS buffers (full tiles; partial tiles use staging 0) */
} tanq_variant_t;

/* Number of apply-kernel variants for width k (2 or 3) and precision p; k = 1 has one. */
tanq_status tanq_variant_count(int k, tanq_prec p, int* count);
tanq_status tanq_variant_get(int k, tanq_prec p, int index, tanq_variant_t* out);
/* Process-wide choice used by every later apply of that width and precision (it also clears
 * the autotuned entries of that width and precision). */
tanq_status tanq_variant_select(int k, tanq_prec p, int index);
tanq_status tanq_variant_selected(int k, tanq_prec p, int* index);

/* Time every variant of every width k <= min(3, n) on d (reps applies of the identity
 * superoperator on a low and a high qubit placement, so finite contents of d are left
 * unchanged), record the fastest of each width as the variant for (n, k, precision) -- it
 * takes precedence over the process-wide choice for states of n qubits until the next
 * tanq_variant_select of that (k, precision) -- and record the best milliseconds per apply.
 * Where passes apply (see tanq_set_pass_limit), also time passes of 2..limit superoperators on
 * the four highest qubits and record milliseconds per pass.  TANQ_FUSE_AUTO then chooses the
 * fusion width that minimises the sum of these costs over the launches tanq_apply_fused would
 * make for each planned width.  ms_per_apply (may be NULL) receives 4 values, index k = 1..3
 * (0 where k > n).  Synchronises. */
tanq_status tanq_autotune(tanq_dm d, int reps, double* ms_per_apply);

/* As tanq_autotune, but timed on dense data: d is first overwritten with the seeded
 * pseudo-random values of tanq_dm_fill_random (seed 1) and the applies use a fixed dense
 * unitary superoperator instead of the identity.  Dense operands draw more power in the
 * matrix units than a mostly-zero state does, so these costs are the ones real circuits see.
 * d's contents are replaced (call tanq_dm_reset afterwards).  Synchronises. */
tanq_status tanq_autotune_dense(tanq_dm d, int reps, double* ms_per_apply);

/* Multi-superoperator passes.  tanq_apply_fused and tanq_apply_fused_range apply each run of
 * consecutive 2-qubit blocks whose qubits together number at most 6 in one pass over vec(rho):
 * every tile of the state is read into LDS once, multiplied by each superoperator of the run in
 * circuit order (in 3M form: three real products per complex one, where a single apply uses the
 * real-block form; results agree with applying the blocks one by one to rounding), and written
 * back once.  This cuts HBM traffic, the
 * bound of 2-qubit applies (Sec. 3.2: a 2-qubit superoperator is memory-bound).  Passes are
 * used on states of at least 10 (FP64) or 11 (FP32) qubits, for runs whose tiles keep whole
 * 128-byte lines of vec(rho), with at most 4 (FP64) or 6 (FP32) superoperators.  With passes
 * enabled, tanq_fuse also orders commuting blocks so that blocks sharing a pass are adjacent,
 * and widens 1-qubit blocks that join a pass to 2 qubits (the identity on the added qubit).  The limit is
 * the most superoperators per pass, 1..8 (1 = no passes; default 8), process-wide. */
tanq_status tanq_set_pass_limit(int max_superops);
tanq_status tanq_get_pass_limit(int* max_superops);
/* How tanq_apply_fused groups f's blocks under the current limit: *passes receives the number
 * of multi-superoperator passes and *in_passes the blocks they apply (the other blocks are
 * applied one by one).  Host only. */
tanq_status tanq_fused_passes(tanq_fused f, int* passes, int* in_passes);
/* The launches tanq_apply_fused makes for f, in order: run_len[i] blocks (1 = a single apply,
 * >= 2 = a pass) starting where launch i - 1 ended.  *count receives the number of launches;
 * run_len may be NULL to query it (E_ARG if cap is smaller).  Applying f launch by launch with
 * tanq_apply_fused_range over these ranges gives the same launches.  Host only. */
tanq_status tanq_fused_launches(tanq_fused f, int* run_len, int cap, int* count);
/* Diagnostics of one pass layout (host only): m 2-qubit superoperators on n qubits, qubits =
 * m pairs; *conflict_free receives how many of the 2 m LDS access patterns (the MFMA operand
 * reads and the result writes of each superoperator) the chosen swizzle keeps free of bank
 * conflicts, *achievable an upper bound of that number over all swizzles of the kernels' form
 * (in FP32 a pattern can be conflict-free only if its lowest free bits include tile bit 0).
 * E_ARG if the pass is not valid (qubits out of range or repeated within a block, more than 6
 * distinct qubits, m outside 1..8, too small a state). */
tanq_status tanq_pass_layout_info(int n, int m, const int* qubits, tanq_prec p, int* conflict_free, int* achievable);

/* The variant applies of width k on n-qubit states use (the autotuned one, else the
 * process-wide choice). */
tanq_status tanq_variant_for(int n, int k, tanq_prec p, int* index);

/* The autotuning cache as text, to keep tuning results across processes: one line per tuned
 * (n, k, precision), "tune <n> <k> <f64|f32> <tile_bits> <threads> <staging> <ms per apply>"
 * (tile bits, threads and staging are 0 for k = 1), and one per timed pass length,
 * "pass <n> <f64|f32> <superoperators> <ms per pass>".  buf may be NULL to query; *len
 * receives the size needed, including the terminating NUL; E_ARG if cap is smaller. */
tanq_status tanq_tuning_export(char* buf, size_t cap, size_t* len);
/* Load text written by tanq_tuning_export (blank lines and lines starting with '#' are
 * skipped).  Every line is validated first -- E_ARG names a malformed line or a variant this
 * build does not have -- and nothing changes unless all lines are valid. */
tanq_status tanq_tuning_import(const char* text);

/* ---------------------------------------------------------------------------------------
 * Measurement statistics (Sec. 2.1: rho gives the probability of every outcome).
 * ------------------------------------------------------------------------------------- */

/* Z-basis probabilities p_x = Re rho[x][x] (divided by the trace if renormalize != 0),
 * reduced in FP64 on the GPU; host_out receives 2^n doubles, *trace_out (may be NULL) the
 * trace.  Synchronises. */
tanq_status tanq_probs(tanq_dm d, double* host_out, int renormalize, double* trace_out);

/* Z-basis probabilities seen through a classical readout-error model (Sec. 3.5, measurement
 * error): qubit t is read as 0 when it is 1 with probability p01[t] (P(0|1)) and as 1 when it
 * is 0 with p10[t] (P(1|0)), independently, i.e. q = (x)_t [[1 - p10, p01], [p10, 1 - p01]] p
 * with p the renormalised probabilities.  The paper's averaged model is p01 = p10.  FP64 on
 * the GPU; host_out receives 2^n doubles.  Synchronises. */
tanq_status tanq_probs_readout(tanq_dm d, const double* p01, const double* p10, double* host_out);

/* Measure all qubits `shots` times (the all-measure operation): outcome i is the smallest x
 * with cdf(x) > u_i * cdf(2^n - 1), cdf the FP64 prefix sums of the probabilities (after the
 * readout model when p01/p10 are given, else both NULL) and u_i the top 53 bits of
 * SplitMix64((seed << 40) + i) scaled to [0, 1).  host_out receives shots outcomes (bit t of an
 * outcome = qubit t).  seed < 2^23.  Synchronises. */
tanq_status tanq_sample(tanq_dm d, uint64_t shots, uint64_t seed, const double* p01, const double* p10,
                        uint64_t* host_out);

/* tanq_sample without any device allocation, for callers that cannot allocate: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  Same arguments, draws
 * and outcomes as tanq_sample.  The CDF and the outcomes live in a fixed 2 MiB device array of
 * the library (one per GPU, held until the process ends), so n <= 17 and shots <= 2^17 per call;
 * beyond that TANQ_E_ARG.  Calls on one GPU share that array: calls that overlap there (from
 * several threads, or on streams that are not drained in between) race.  Synchronises. */
tanq_status tanq_sample_noalloc(tanq_dm d, uint64_t shots, uint64_t seed, const double* p01, const double* p10,
                                uint64_t* host_out);

/* rho = |r><c| (a basis operator; not a state unless r == c).  Input of process tomography,
 * where the channel is linear in its input.  Stream-ordered. */
tanq_status tanq_dm_set_basis(tanq_dm d, uint64_t r, uint64_t c);

/* Reduced density matrix on k <= 4 qubits keep[0..k-1] (keep[0] = least significant bit of
 * the result's index): out[a][b] = sum_f rho[a|f][b|f] over the other qubits' values f.  FP64
 * reduction on the GPU; host_out receives 4^k complex values (row-major, interleaved).
 * Synchronises. */
tanq_status tanq_reduced_dm(tanq_dm d, int k, const int* keep, double* host_out);

/* Process tomography of a one-qubit channel defined by a circuit (Sec. 5, teleportation case
 * study): for each basis operator |a><b| placed on in_qubit (every other qubit |0><0|), fuse
 * and simulate the circuit on the GPU, reduce to out_qubit, and assemble the channel's 4 x 4
 * superoperator S (column a + 2b = vec of the output).  chi_out receives the process matrix in
 * the Pauli basis (I, X, Y, Z), E(rho) = sum_ij chi_ij sigma_i rho sigma_j, as 4 x 4 complex
 * row-major; superop_out (may be NULL) receives S.  Synchronises. */
tanq_status tanq_process_chi_1q(tanq_circuit c, int max_width, tanq_prec p, int in_qubit, int out_qubit,
                                double* chi_out, double* superop_out);

/* Re Tr(P rho) for the Pauli string P = (x)_t sigma_{pauli[t]}, pauli = n characters of
 * "IXYZ", character t acting on qubit t.  FP64 reduction.  Synchronises. */
tanq_status tanq_expect_pauli(tanq_dm d, const char* pauli, double* out);

/* Tr(P rho) with its imaginary part (zero for Hermitian rho). */
tanq_status tanq_expect_pauli_c(tanq_dm d, const char* pauli, double* re, double* im);

/* count Pauli strings at once (one launch); out_re/out_im receive count values each
 * (out_im may be NULL). */
tanq_status tanq_expect_pauli_batch(tanq_dm d, int count, const char* const* paulis, double* out_re,
                                    double* out_im);

/* Compare two density matrices of the same n (any precisions), reduced in FP64 on the GPU:
 * out[0] = ||a - b||_F, out[1] = max_ij |a_ij - b_ij|, out[2] = ||a||_F.  The trace distance
 * obeys (1/2)||a - b||_1 <= (1/2) 2^(n/2) ||a - b||_F.  Both handles must live on the same
 * device; work is ordered on a's stream after b's stream is synchronised.  Synchronises. */
tanq_status tanq_dm_compare(tanq_dm a, tanq_dm b, double* out3);

/* ---------------------------------------------------------------------------------------
 * Serving: continuous batching of many small noisy circuits.
 *
 * Requests are admitted in arrival order while a slot is free and their device footprint
 * (vec(rho) plus packed superoperators plus fusion temporaries, known at submit) fits in the
 * budget.  Each admitted request's state stays resident on the device until its results are
 * read back.  A scheduler thread applies, per batched launch, the next fused superoperator of
 * every resident request at once (steps_per_launch such launches per iteration, optionally
 * captured once in a hipGraph and replayed); requests arriving meanwhile join at the next
 * iteration.  A request's arithmetic does not depend on the other requests in the batch, so
 * its results are the same alone and in the mix.  All blocks are widened to the server's
 * fusion width (2 or 3).  Errors on the scheduler thread fail the affected requests with
 * TANQ_E_HIP and the server stops accepting work.
 * ------------------------------------------------------------------------------------- */

typedef struct tanq_server_s* tanq_server;

typedef struct {
  size_t hbm_budget;    /* device bytes the server may use for states and operands (>= 64 MiB) */
  int max_slots;        /* requests resident at once, 1..4096 */
  int prec;             /* tanq_prec of the states */
  int width;            /* fusion width 2 or 3 (0 = 2) */
  int steps_per_launch; /* batched applies per scheduler iteration, 1..64 */
  int use_graphs;       /* nonzero: replay the iteration's launches from a captured hipGraph */
  size_t cohort_bytes;  /* 0: every resident request advances in every iteration.  Otherwise each
                           iteration advances a cohort of resident requests, taken round-robin,
                           whose states total at most cohort_bytes (at least one request), so
                           that the iteration's consecutive passes over those states can hit the
                           device's last-level cache */
  double request_timeout_s; /* > 0: a request not finished this many seconds after its submission
                               is dropped with status TANQ_E_TIMEOUT (queued: taken off the queue;
                               resident: no further batched applies, its slot and memory freed
                               once the launches already queued for it have run); 0: no timeout */
} tanq_server_config;

typedef struct {
  int probs;                 /* nonzero: return the 2^n probabilities, divided by the trace */
  int npauli;                /* number of Pauli strings (0..1024) */
  const char* const* paulis; /* n characters of "IXYZ" each, character t acting on qubit t */
} tanq_outputs;

typedef struct {
  int status;            /* TANQ_OK or the request's error */
  int n;
  double trace;
  const double* probs;   /* 2^n values or NULL; owned by the server until release */
  const double* pauli;   /* npauli values Re Tr(P rho) */
  int npauli;
  int fused_applies;     /* fused superoperators applied */
  double t_submit, t_admit, t_done; /* seconds on the server clock */
} tanq_result;

typedef struct {
  uint64_t submitted, admitted, completed, rejected; /* completed: finished with outputs */
  uint64_t launches;     /* scheduler iterations (each steps_per_launch batched applies) */
  uint64_t steps;        /* batched applies that had work */
  size_t bytes_in_use, peak_bytes, budget_bytes;
  int active, pending;
  double clock;          /* seconds since creation */
  uint64_t tiles;        /* tile multiplications of the batched launches so far (one tile of one
                            state by one fused superoperator) */
  uint64_t chunks;       /* work-list chunks those launches claimed */
  uint64_t dropped;      /* requests cancelled or timed out */
} tanq_server_stats;

/* Create a server on the current device with its own stream and scheduler thread.
 * TANQ_E_OOM if the budget exceeds free device memory. */
tanq_status tanq_server_create(const tanq_server_config* cfg, tanq_server* out);

/* Queue a circuit (copied; c may be freed afterwards) with the outputs wanted.  Never blocks on
 * the GPU: plans the fusion on the calling thread and returns a ticket.  TANQ_E_ARG if n is
 * outside [width, 14]; TANQ_E_OOM if the request alone exceeds the budget (it could never be
 * admitted).  A circuit with no operations completes with the outputs of |0..0><0..0|. */
tanq_status tanq_server_submit(tanq_server s, tanq_circuit c, const tanq_outputs* outs, uint64_t* ticket);

/* Cancel a request.  A queued request leaves the queue at once; a resident one gets no further
 * batched applies and frees its slot and device memory once the launches already queued for it
 * have run.  Its result then has status TANQ_E_CANCELED and no outputs.  A request that has
 * already finished keeps its result (TANQ_OK, nothing changes).  TANQ_E_ARG for an unknown
 * ticket.  Never blocks on the GPU. */
tanq_status tanq_server_cancel(tanq_server s, uint64_t ticket);

/* Result of a finished request (TANQ_E_AGAIN while it is not finished); wait blocks. */
tanq_status tanq_server_poll(tanq_server s, uint64_t ticket, tanq_result* out);
tanq_status tanq_server_wait(tanq_server s, uint64_t ticket, tanq_result* out);

/* Drop a finished request and its result buffers. */
tanq_status tanq_server_release(tanq_server s, uint64_t ticket);

tanq_status tanq_server_stats_get(tanq_server s, tanq_server_stats* out);

/* Finish queued work, stop the scheduler and free everything. */
tanq_status tanq_server_destroy(tanq_server s);

#ifdef __cplusplus
}
#endif

#endif /* TANQ_H */
