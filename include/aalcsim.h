/*
 * aalcsim.h -- C ABI of libaalcsim.so: amplitude-aware lossy-compressed
 * state-vector simulation on one AMD Instinct MI355X (gfx950).
 *
 * Method: Wu, Di, Cappello, Finkel, Alexeev, Chong, "Amplitude-Aware Lossy
 * Compression for Quantum Circuit Simulation".  The state vector of n qubits
 * (2^n complex doubles, Sec. II) is never held uncompressed: it is split into
 * blocks ("strides", Sec. III) of 2^b amplitudes, each stored as a compressed
 * block stream in device memory.  Every gate runs the loop of Alg. 2 on every
 * block: decompress, normalise, apply the gate, compress at the error bounds
 * delta_0 < delta_1 < ... of the ladder until the ratio reaches theta.
 *
 * Conventions for every entry point
 *   - Qubit q is bit q of the amplitude index.
 *   - Pointers named host_* or documented as host are host memory, borrowed
 *     for the duration of the call only.  Device memory is owned by the
 *     sim and released by sim_destroy: either allocated by the library
 *     (sim_create, sim_create_ex) or carved from a caller-owned device
 *     buffer (sim_context_create + sim_create_in), in which case the sim
 *     and every call on it allocate no device memory of their own.
 *   - Calls on one sim are ordered on that sim's HIP stream.  sim_apply_gate
 *     is asynchronous; every call that returns data to the host synchronises
 *     the stream first.  A sim is not thread-safe; different sims are
 *     independent.
 *   - Return codes are SIM_OK (0) or a negative SIM_E* code.  Validation
 *     failures leave the state unchanged.  sim_last_error() gives a
 *     thread-local text for the last failure.
 *   - Errors found on the device during an asynchronous pass (arena
 *     overflow) are reported by the next synchronising call: the state is
 *     rolled back to the input of the failing gate and that gate and the ones
 *     queued after it are dropped; the call returns SIM_ENOMEM.
 */
#ifndef AALCSIM_H
#define AALCSIM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sim sim_t;

enum {
    SIM_OK = 0,
    SIM_EINVAL = -1,        /* bad argument */
    SIM_ENOMEM = -2,        /* device allocation or arena capacity exhausted */
    SIM_EBUDGET = -3,       /* the sim's memory context cannot hold a request */
    SIM_EDEVICE = -4,       /* HIP runtime error */
    SIM_ECOLLAPSED = -5,    /* N^2 of the stored state was 0 or not finite */
    SIM_EUNSUPPORTED = -6   /* valid request that the library does not implement */
};

/* Gate kinds.  u is a 2x2 complex matrix, row-major, (re, im) pairs:
 * u00=(u[0],u[1]) u01=(u[2],u[3]) u10=(u[4],u[5]) u11=(u[6],u[7]).
 * Matrices and phases are computed by the caller; the library applies them
 * with one IEEE binary64 rounding per multiply and add (no fused
 * multiply-add), so results are reproducible bit for bit. */
enum {
    G_U = 1,          /* u on qubit q0: pair update of Sec. II */
    G_DIAG1 = 2,      /* diag(1, u11) on qubit q0 (T, S, Z, phase) */
    G_CU = 3,         /* u on target q1 where control q0 is 1 (Sec. II) */
    G_CPHASE = 4,     /* amplitude with bits q0 and q1 set times u11 */
    G_CZ = 5,         /* amplitude with bits q0 and q1 set negated */
    G_SWAP = 6,       /* exchange qubits q0 and q1 */
    G_X = 7,          /* exchange the two amplitudes of each pair on q0 */
    G_PHASE_FLIP = 8, /* amplitude at `index` negated (Grover oracle, Sec. IV) */
    G_DIFFUSE = 9     /* 2|s><s| - I on all qubits (Grover diffusion) */
};

typedef struct {
    uint32_t kind;
    int32_t q0, q1;
    uint32_t pad;     /* must be 0 */
    uint64_t index;   /* G_PHASE_FLIP only */
    double u[8];
} sim_gate_t;

typedef struct {
    double normsq;             /* N^2 of the stored state after the last pass */
    double scale;              /* s = 1/sqrt(N^2), applied at the next decode */
    int32_t collapsed;         /* N^2 was 0 or not finite at some pass */
    int32_t compressed;        /* 0 for the uncompressed path */
    uint64_t resident_bytes;   /* bytes of block streams now (compressed) */
    uint64_t peak_resident;    /* max over passes of resident_bytes */
    double min_ratio;          /* min over passes of 16*2^n / resident_bytes */
    double last_ratio;
    uint64_t passes;           /* gates applied since the last set_basis */
    uint64_t level_hist[8];    /* blocks encoded at each ladder level */
    uint64_t arena_bytes;      /* capacity of each of the two arenas */
    uint64_t device_bytes;     /* all device memory held by the sim (not the
                                  pass kernels' staging of a sim outside a
                                  context: one buffer per GPU, shared) */
    uint64_t replays;          /* blocks re-encoded because the level chosen
                                  differed from the one speculated */
    uint64_t escalations;      /* blocks whose first sized levels all missed
                                  theta, so the rest of the ladder was sized */
    uint64_t arena_peak;       /* largest arena fill of any pass (bytes) */
} sim_stats_t;

/* Create an n-qubit state |0...0> with blocks of 2^block_log2 amplitudes
 * (the AALC decision unit; 6 <= block_log2 <= 20, clamped to n;
 * 6 <= n <= 40).
 *   error_bound > 0 : AALC ladder (0, eb/1000, eb/100, eb/10, eb), theta 4
 *                     (Alg. 2: lossless first, then growing bounds).
 *   error_bound == 0: lossless only.
 *   error_bound < 0 : uncompressed FP64 state vector (n <= 34), the
 *                     "no compression" comparator of Sec. IV.
 * Two arenas of compressed streams are allocated (ping-pong between
 * passes); their size is min(2.1 * 16 * 2^n + 1 MiB, 8 GiB) each unless
 * sim_create_ex gives one.  The first compressed sim (or batch) on a GPU
 * also allocates the pass kernels' staging for that GPU (1.2 GB, indexed by
 * hardware wave slot and shared by every sim and batch of the process on
 * that GPU; held until the process ends).  Returns NULL on failure
 * (sim_last_error()). */
sim_t *sim_create(int n_qubits, int block_log2, double error_bound);

/* As sim_create, with an explicit capacity per arena (0 = default) and a
 * HIP stream (NULL = a stream created and owned by the sim). */
sim_t *sim_create_ex(int n_qubits, int block_log2, double error_bound,
                     uint64_t arena_bytes, void *hip_stream);

void sim_destroy(sim_t *sim);

/* Memory contexts: device memory that the caller owns (for example the
 * storage of a torch tensor), from which sims created in the context take
 * all of their device memory -- arenas, descriptors, size tables, staging,
 * reduction buffers and the temporaries of queries.  The sim path itself
 * then calls no hipMalloc.  Nothing else of the method changes.  */
typedef struct sim_ctx sim_ctx_t;

/* Wrap dev_buf (device memory of the current GPU, >= 4096 bytes, owned by
 * the caller and kept alive until sim_context_destroy) as a context.  Sims
 * created in it use hip_stream (NULL: each creates its own stream).  The
 * buffer is carved first fit in 256-byte aligned ranges; ranges freed by
 * sim_destroy are reused.  SIM_EINVAL if dev_buf is not device memory.  A
 * context is not thread-safe: create and destroy its sims from one thread. */
int sim_context_create(void *dev_buf, size_t bytes, void *hip_stream, sim_ctx_t **ctx);

/* Release the context (not the buffer).  SIM_EINVAL while sims created in it
 * are alive. */
int sim_context_destroy(sim_ctx_t *ctx);

/* Bytes of the context: usable capacity, in use, peak in use, and the
 * largest free range (any pointer may be NULL). */
int sim_context_info(const sim_ctx_t *ctx, uint64_t *capacity, uint64_t *used,
                     uint64_t *peak, uint64_t *largest_free);

/* As sim_create_ex, with all device memory taken from ctx (on its GPU, on
 * its stream).  Returns SIM_OK and *out, or SIM_EBUDGET when the context
 * cannot hold the sim (nothing is kept), or another SIM_E* code.  Later
 * calls on the sim that need device memory (a longer ladder, a larger grid,
 * whole-state export and import, queries) take it from the context too and
 * return SIM_EBUDGET when it is exhausted, with the state unchanged. */
int sim_create_in(sim_ctx_t *ctx, int n_qubits, int block_log2, double error_bound,
                  uint64_t arena_bytes, sim_t **out);

/* Apply one gate (Alg. 2 for every block).  Asynchronous on the sim stream;
 * the gate record is copied.  Returns SIM_EINVAL for an invalid gate (qubit
 * out of range, equal qubits, index >= 2^n, unknown kind, pad != 0). */
int sim_apply_gate(sim_t *sim, const sim_gate_t *gate);

/* Apply `count` gates in order (same contract as sim_apply_gate; stops at
 * the first invalid gate, whose position is in sim_last_error()). */
int sim_apply_gates(sim_t *sim, const sim_gate_t *gates, size_t count);

/* Shortcuts of Sec. V (off by default, where every gate runs Alg. 2 on
 * every block):
 *   SIM_SC_PERMUTE: under a gate that only reorders amplitudes (X, SWAP, and
 *     CU whose matrix is exactly [[0, 1], [1, 0]], i.e. CNOT) each block is
 *     compressed at the ladder level its previous stream used; no other
 *     level is tried.
 *   SIM_SC_SKIP: a block that the gate leaves unchanged by its structure (a
 *     diagonal or controlled gate whose qubit at or above block_log2 is 0 in
 *     the block's index, PHASE_FLIP away from its index, SWAP of two such
 *     qubits that are equal there) keeps its stream; the pass's
 *     normalisation s is deferred into the block's scale, c_j <- fl(c_j s).
 *     A block is decoded with the factor fl(c_j s), weighs fl(normsq_j
 *     fl(c_j c_j)) in N^2 when c_j != 1, and returns to c_j = 1 when it is
 *     compressed again.  Exported streams of blocks with c_j != 1 set bit 0
 *     of header byte 5 and carry c_j as an f64 right after the header
 *     (counted in total_bytes); sim_import_state accepts them.
 * Both change which streams are produced (the results differ from Alg. 2's
 * where a skipped block would have been re-encoded at another level), so
 * they are opt-in.  Flags take effect from the next gate.  SIM_EINVAL for
 * unknown flags, SIM_EUNSUPPORTED on the uncompressed path. */
enum { SIM_SC_PERMUTE = 1, SIM_SC_SKIP = 2 };
int sim_set_shortcut(sim_t *sim, int flags);

/* Probabilities of every outcome of `qubits` (nq distinct qubits, 1..24):
 * probs[o] = sum over indices whose listed bits spell o (bit k of o is
 * qubit qubits[k]) of |a_i|^2 for the normalised amplitudes a = s * xhat.
 * probs is host memory of 2^nq doubles.  Synchronises. */
int sim_measure_probs(sim_t *sim, const int *qubits, int nq, double *probs);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * result as sim_measure_probs with no device allocation and no free.  The
 * outcome bins and the qubit list live in one array that the library holds
 * on each GPU until the process ends (2^16 doubles + 256 bytes), so nq is
 * limited to 1..16 (SIM_EINVAL above that).  Every call on one GPU shares
 * that array: calls that overlap on one GPU (sims on different streams,
 * several host threads) race and must be serialised by the caller.  Host
 * memory probs (2^nq doubles) is the caller's.  Synchronises. */
int sim_measure_probs_noalloc(sim_t *sim, const int *qubits, int nq, double *probs);

/* Fidelity of two states with the same n (Sec. II, with the modulus squared
 * and both norms divided out): F = |<a|b>|^2 / (<a|a><b|b>).  Either sim may
 * be compressed or uncompressed.  Synchronises. */
int sim_fidelity(sim_t *a, sim_t *b, double *F);

/* Replace the state by the basis state |x> (x < 2^n); resets stats. */
int sim_set_basis(sim_t *sim, uint64_t x);

/* Set the AALC ladder: L (1..8) levels, ladder[0] may be 0 (lossless), the
 * lossy levels all of one kind and growing: absolute bounds delta >= 2^-30
 * (|x - xhat| < delta per real component, Sec. III), or pointwise-relative
 * bounds given as -eps with eps in [2^-19, 0.05] and growing eps (|x - xhat|
 * < eps |x|, zeros kept exactly: log2|x| is quantised in steps of
 * 2 fl(1.4 eps) with the sign in the code's low bit, after the log transform
 * of the relative-bound reference the paper builds on; values that miss the
 * bound are stored exactly).  theta >= 1.  Takes effect for the next pass.
 * SIM_EINVAL otherwise, SIM_EUNSUPPORTED on the uncompressed path. */
int sim_set_aalc(sim_t *sim, const double *ladder, int L, double theta);

/* Turn the normalisation before each gate (Sec. III) on (default) or off. */
int sim_set_normalize(sim_t *sim, int on);

/* Copy normalised amplitudes s * xhat for indices [first, first+count) to
 * host memory `out` as interleaved (re, im) doubles.  Synchronises. */
int sim_get_amplitudes(sim_t *sim, uint64_t first, uint64_t count,
                       double *out);

/* Copy the canonical block stream v1 of block j to host memory buf (cap
 * bytes); *len receives its length (also when cap is too small, in which
 * case SIM_ENOMEM is returned).  Synchronises. */
int sim_export_block(sim_t *sim, uint64_t j, void *buf, size_t cap,
                     size_t *len);

/* Checkpoint of the whole state: the canonical block streams of every block,
 * block 0 first, concatenated into host memory buf (cap bytes); *len
 * receives the total (also when cap is too small or buf is NULL, in which
 * case SIM_ENOMEM is returned).  This is the state Alg. 1 keeps (each stride
 * stored compressed); the scale of the next gate follows from the normsq
 * fields, so these bytes are the whole resumable state.  The streams are
 * staged in the sim's idle arena (no device allocation).  Synchronises.
 * SIM_EUNSUPPORTED on the uncompressed path. */
int sim_export_state(sim_t *sim, void *buf, size_t cap, size_t *len);

/* Checkpoint through the entropy stage: as sim_export_state, but each
 * block's stream re-coded losslessly as a block entropy stream v1.  SZ, the
 * compressor of Sec. III, ends in entropy and dictionary coding; the
 * resident streams keep the fixed-width packer that the per-gate kernels
 * decode, and this stage is applied where streams leave the GPU.  Layout
 * (little-endian):
 *   header (32 B): the v1 header with magic 0x31454141 ("AAE1") and
 *                  total_bytes = the length of this stream
 *   u32 v1_bytes (length of the v1 stream) | u32 n_items
 *   [f64 scale]  iff header flag bit 0, as in v1
 *   n_items u32 tags, zero-padded to a multiple of 8 bytes; item bodies
 * Tag bit 31: a run of (tag & 0x7FFFFFFF) >= 1 planes, each plane's v1
 * record equal to the record two planes before it (never planes 0, 1), no
 * body.  Else one literal plane: bit 30 set: the body is the v1 record
 * itself, (tag & 0x3FFFFFFF) bytes; bit 30 clear: a coded body of tag bytes:
 *   i64 anchor | u32 payload_words (pw) | u32 n_outliers
 *   if pw > 0: u32 coded_words | u32 0 | C mode bytes (padded to 8) |
 *     u16 coded bit length of each chunk that is not fixed width (padded to
 *     8) | coded_words u64 words of chunk codes back to back (LSB first,
 *     zero-padded)
 *   outliers as in v1
 * Mode m: 128 + w fixed width w (0..64); 63 + w sparse of width w (1..64):
 * a 64-bit mask of the nonzero residuals, then those in w bits; k < 64
 * Golomb-Rice with parameter k: per residual z, z >> k one-bits, a zero bit,
 * the k low bits (the chunk's v1 width is the bit length of its largest z).
 * The encoder takes, per chunk of width w > 0, the shortest of fixed (64 w
 * bits), Rice (64 (k + 1) + sum (z >> k), the smallest best k) and sparse
 * (64 + nnz w), ties in that order; a literal whose coded body would not be
 * shorter than its record is stored verbatim.  Every block size the library
 * takes qualifies (at most 2^(20-10+1) planes).  *len and SIM_ENOMEM as for
 * sim_export_state; the streams are staged in the idle arena.  Synchronises. */
int sim_export_state_entropy(sim_t *sim, void *buf, size_t cap, size_t *len);

/* Resume from a checkpoint: replace the state by the concatenated block
 * streams in host memory buf[0..len) as sim_export_state or
 * sim_export_state_entropy write them (or any producer of block stream v1 or
 * block entropy stream v1, mixed freely; entropy streams are decoded on the
 * GPU, above the room their v1 streams take in the idle arena).  Every stream must have this sim's segment
 * and block sizes and a level of this sim's ladder whose bound equals its
 * delta bit for bit (set the ladder first with sim_set_aalc), its records
 * must be well formed (sizes, chunk widths, first residual 0, lossy anchors
 * within +-(2^30 - 1), ascending in-plane outlier indices, none in lossless
 * planes), and its normsq field must equal the normsq of its decoded values.
 * The host checks the headers, then the streams are copied into the idle
 * arena and checked there by kernels.  On success the sim holds that state:
 * N^2 and the scale of the next gate are recomputed from the decoded values
 * exactly as after a pass, the pass count restarts at 0, and the following
 * gates give the streams the exporting sim would have produced.  Returns
 * SIM_EINVAL (state unchanged) on a malformed or mismatched stream,
 * SIM_ENOMEM when the streams exceed the arena, SIM_ECOLLAPSED (state
 * replaced) when the imported N^2 is 0 or not finite.  Synchronises. */
int sim_import_state(sim_t *sim, const void *buf, size_t len);

/* Launch shape of the per-gate pass: at most max_workgroups workgroups
 * (64..65536, default 3072) loop over the segment pairs of the state.  A
 * tuning knob only: results do not depend on it. */
int sim_set_grid(sim_t *sim, int max_workgroups);

/* Copy the 32-byte stream headers (block stream v1, normsq field filled) of
 * blocks [first, first+count) to host memory buf (cap >= 32*count bytes).
 * The N^2 of the state is the pairwise sum of the normsq fields over all
 * blocks in index order (Sec. III normalisation).  Synchronises. */
int sim_export_headers(sim_t *sim, uint64_t first, uint64_t count, void *buf,
                       size_t cap);

/* out[0], out[1] = sums of the real and imaginary parts of the normalised
 * amplitudes s * xhat over all 2^n indices, as one perfect binary tree in
 * index order: the sum that the Grover diffusion 2|s><s| - I takes its mean
 * from (Sec. IV).  out is host memory of 2 doubles.  Synchronises. */
int sim_amplitude_sum(sim_t *sim, double *out);

/* Statistics of the stored state.  Synchronises. */
int sim_stats(sim_t *sim, sim_stats_t *st);

/* Wait for all queued work of the sim; reports device-side errors. */
int sim_sync(sim_t *sim);

/* Use `hip_stream` (a hipStream_t, e.g. a torch stream's handle) for all
 * later work of the sim.  The previous work is synchronised first. */
int sim_set_stream(sim_t *sim, void *hip_stream);

/* Per-kernel device time of one sim's launches. */
typedef struct {
    char name[32];       /* kernel name, NUL-terminated */
    uint64_t launches;
    double total_ms;     /* sum over launches of (end event - begin event) */
    double min_ms;
    double max_ms;
} sim_kernel_time_t;

/* HIP-event timing of this sim's kernels: 0 off, 1 every kernel, 2 only the
 * fused per-gate pass kernel (fewest events).  A begin and an end event are
 * recorded on the sim stream around each timed launch.  Synchronises. */
int sim_profile(sim_t *sim, int on);

/* Per-kernel totals of the launches timed since the last read (then reset).
 * Writes up to cap entries to host memory `out`, the number of kernels seen
 * to *count.  Synchronises. */
int sim_profile_read(sim_t *sim, sim_kernel_time_t *out, int cap, int *count);

/* Overlap with the Fourier basis state QFT|x> (Sec. IV QFT workload):
 * out[0] + i out[1] = sum over k of e^(-2 pi i x k / 2^n) a_k and out[2] =
 * sum of |a_k|^2, for the normalised amplitudes a (each sum one pairwise
 * tree in index order).  The fidelity to QFT|x> is
 * (out[0]^2 + out[1]^2) / (2^n out[2]).  out is host memory of 3 doubles.
 * Works on both paths.  Synchronises. */
int sim_fourier_overlap(sim_t *sim, uint64_t x, double *out);

/* Self-test hook for the normalisation scalar: out[i] = 1/sqrt(in[i])
 * computed on the device by the same code that derives s from N^2 (one
 * correctly rounded sqrt, one correctly rounded division).  in and out are
 * host arrays of count doubles.  Uses the default device. */
int sim_debug_rsqrt(const double *in, double *out, size_t count);

/* ---- batches: many states advanced by the same kernels -----------------
 *
 * A batch applies one gate to each of several sims per pass with one set of
 * kernel launches for all of them (the work items of every state share the
 * grid), and optionally records the passes as a HIP graph that is replayed
 * whenever the same shape comes again (the per-state arguments live in device
 * memory and are rewritten before each launch, so the graph's topology stays
 * fixed).  Every state computes exactly what sim_apply_gate computes for it:
 * a state's streams are the same alone and in a batch.  Work of the batch is
 * ordered after the work already queued on each sim's stream, and later work
 * on those streams after the batch. */
typedef struct sim_batch sim_batch_t;

/* A batch for up to max_states sims per call and max_passes passes per call
 * (each 1..4096), on `hip_stream` (NULL = a stream owned by the batch).
 * Allocates device and pinned host memory for the per-pass arguments.
 * Returns NULL on failure (sim_last_error()). */
sim_batch_t *sim_batch_create(int max_states, int max_passes, void *hip_stream);

void sim_batch_destroy(sim_batch_t *batch);

/* Apply passes x count gates: gates[p * count + k] to sims[k] in pass p,
 * passes in order.  A gate of kind 0 (all fields 0) leaves that sim alone in
 * that pass.  sims must be distinct compressed sims holding a state.  With
 * use_graph != 0 the passes are captured once per shape (count, passes,
 * which passes hold a diffusion, launch grids) and replayed as one graph
 * launch.  Asynchronous; validation failures (SIM_EINVAL, SIM_EUNSUPPORTED)
 * queue nothing.  Device-side errors of a sim are reported by that sim's next
 * synchronising call, as for sim_apply_gate. */
int sim_batch_apply(sim_batch_t *batch, sim_t *const *sims, int count,
                    const sim_gate_t *gates, int passes, int use_graph);

/* Wait for all work of the batch. */
int sim_batch_sync(sim_batch_t *batch);

/* HIP-event timing of the batch's kernels (modes as sim_profile).  While it
 * is on, sim_batch_apply launches the passes directly instead of replaying a
 * graph (events cannot time the kernels inside a graph launch). */
int sim_batch_profile(sim_batch_t *batch, int on);
int sim_batch_profile_read(sim_batch_t *batch, sim_kernel_time_t *out, int cap,
                           int *count);

/* Number of graphs captured and graph launches so far (either may be NULL). */
int sim_batch_info(sim_batch_t *batch, uint64_t *graph_builds,
                   uint64_t *graph_launches);

/* Thread-local message of the last failure on this thread ("" if none). */
const char *sim_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
