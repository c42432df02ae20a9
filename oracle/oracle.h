/*
 * oracle.h -- plain FP64 CPU reference for amplitude-aware lossy compressed
 * state-vector simulation (Wu, Di, Cappello, Finkel, Alexeev, Chong,
 * "Amplitude-Aware Lossy Compression for Quantum Circuit Simulation").
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this code; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no source with the GPU path: both are
 * written from the paper and from the block-stream format definition.
 *
 * Conventions
 *   - Qubit q is bit q of the amplitude index (little-endian).
 *   - A state of n qubits is 2^n complex doubles, stored interleaved (re, im).
 *   - A block (the paper's "stride", Sec. III) is 2^b consecutive amplitudes.
 *   - A segment is 2^s consecutive amplitudes inside a block (6 <= s <= b).
 *   - Every floating-point operation is one IEEE binary64 operation; the file
 *     is compiled with -ffp-contract=off so no fused multiply-add appears.
 */
#ifndef AALC_ORACLE_H
#define AALC_ORACLE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    OR_OK = 0,
    OR_EINVAL = -1,
    OR_ENOMEM = -2,
    OR_ECOLLAPSED = -5
};

/* Gate kinds (same numbering as the product header, defined independently). */
enum {
    OR_G_U = 1,          /* 2x2 unitary u on qubit q0 (Sec. II pair update) */
    OR_G_DIAG1 = 2,      /* diag(1, u11) on qubit q0 */
    OR_G_CU = 3,         /* u on target q1 where control q0 is 1 (Sec. II) */
    OR_G_CPHASE = 4,     /* amplitude with bits q0 and q1 set times u11 */
    OR_G_CZ = 5,         /* amplitude with bits q0 and q1 set negated */
    OR_G_SWAP = 6,       /* exchange qubits q0 and q1 */
    OR_G_X = 7,          /* exchange the pair on qubit q0 */
    OR_G_PHASE_FLIP = 8, /* amplitude at index `index` negated */
    OR_G_DIFFUSE = 9     /* 2|s><s| - I over all n qubits */
};

/* u holds a 2x2 complex matrix row-major: u00=(u[0],u[1]) u01=(u[2],u[3])
 * u10=(u[4],u[5]) u11=(u[6],u[7]). */
typedef struct {
    uint32_t kind;
    int32_t q0, q1;
    uint32_t pad;
    uint64_t index;
    double u[8];
} or_gate;

/* ---- building blocks, exposed so tests can pin each one ---------------- */

/* Perfect-binary-tree sum of m = 2^k values (m >= 1). */
double or_pairwise(const double *v, size_t m);

/* Encode one block (2^b interleaved complex values) at error bound `delta`
 * (0 = lossless) into the block stream v1.  `level` is recorded in the
 * header.  Writes up to cap bytes, sets *len to the stream length (also when
 * cap is too small, in which case OR_ENOMEM is returned and nothing useful is
 * written).  The header's normsq field is filled from the decoded values. */
int or_encode_block(const double *x, int b, int s, double delta, int level,
                    uint8_t *out, size_t cap, size_t *len);

/* Decode a block stream into 2^b interleaved complex values (the stored,
 * unnormalised x-hat).  Returns OR_EINVAL on a malformed stream. */
int or_decode_block(const uint8_t *stream, size_t len, double *x);

/* Alg. 2 inner loop on one block: compress at ladder levels 0,1,... in order
 * and stop at the first whose ratio 16*2^b / size reaches theta; otherwise the
 * last level.  sizes[k] receives the stream size of every level tried (the
 * untried ones are set to 0).  Returns the chosen level or a negative code. */
int or_aalc_encode(const double *x, int b, int s, const double *ladder, int L,
                   double theta, uint8_t *out, size_t cap, size_t *len,
                   uint64_t *sizes);

/* Plain state-vector gate on a full 2^n complex array (no compression, no
 * normalisation).  DIFFUSE uses the mean of the array itself. */
int or_sv_apply_gate(double *amp, int n, const or_gate *g);

/* ---- compressed simulator (Alg. 2 driver) ------------------------------ */

typedef struct or_sim or_sim;

/* ladder: L strictly increasing error bounds, ladder[0] may be 0 (lossless),
 * 1 <= L <= 8, theta >= 1.  The state starts as |0...0>. */
or_sim *or_create(int n, int b, int s, const double *ladder, int L,
                  double theta, int normalize);
void or_destroy(or_sim *sim);
int or_set_basis(or_sim *sim, uint64_t x);
int or_apply_gate(or_sim *sim, const or_gate *g);

/* Normalised amplitudes fl(xhat * scale) for indices [first, first+count). */
int or_get_amplitudes(const or_sim *sim, uint64_t first, uint64_t count,
                      double *out);
int or_export_block(const or_sim *sim, uint64_t j, uint8_t *buf, size_t cap,
                    size_t *len);

/* Replace the state by the concatenated block streams buf[0..len) (block 0
 * first, each as or_export_block writes it).  Every stream must match this
 * simulator's s, b and ladder (its delta equal to the bound of its level)
 * and decode cleanly, and its normsq field must equal the normsq of its
 * decoded values; otherwise OR_EINVAL and the state is unchanged.  Returns
 * OR_ECOLLAPSED (state replaced) when N^2 of the imported state is 0 or not
 * finite. */
int or_import_state(or_sim *sim, const uint8_t *buf, size_t len);

/* Entropy stage (block entropy stream v1, defined in oracle.c): lossless
 * re-coding of one block stream v1 (runs of plane records equal to the
 * record two planes before, Golomb-Rice or fixed-width chunk codes).  Both
 * set *olen to the output length (also when out is NULL or cap too small:
 * OR_ENOMEM).  The decoder returns OR_EINVAL for a malformed stream; what
 * it returns is a v1 stream whose own checks are or_decode_block's. */
int or_entropy_encode(const uint8_t *v1, size_t len, uint8_t *out, size_t cap,
                      size_t *olen);
int or_entropy_decode(const uint8_t *e, size_t len, uint8_t *out, size_t cap,
                      size_t *olen);

typedef struct {
    double normsq;           /* N^2 of the stored state after the last pass */
    double scale;            /* s applied at the next decode */
    int32_t collapsed;       /* N^2 was 0 or not finite */
    int32_t pad;
    uint64_t resident_bytes; /* sum of stream lengths */
    double min_ratio;        /* min over passes (and the initial encode) */
    double last_ratio;
    uint64_t passes;
    uint64_t level_hist[8];  /* blocks encoded at each level, all passes */
} or_stats;
int or_get_stats(const or_sim *sim, or_stats *st);

/* S[0], S[1] = pairwise sums of the re and im parts of the normalised
 * amplitudes over the whole state (the sum the Grover diffusion's mean is
 * taken from). */
int or_amplitude_sum(const or_sim *sim, double *S);

/* Probability of every outcome of the listed qubits (2^nq doubles). */
int or_measure_probs(const or_sim *sim, const int *qubits, int nq,
                     double *probs);

/* One group of Alg. 2 on its own: decode the input streams of the group
 * (block j0, and block j0 ^ (mask >> b) when the gate couples two blocks),
 * normalise with `scale`, apply the gate, re-encode each block with the
 * ladder.  tdiff holds 2*mean (re, im) for DIFFUSE.  Used for sampled parity
 * at sizes where the whole state does not fit in host memory. */
int or_process_group(int n, int b, int s, const double *ladder, int L,
                     double theta, double scale, const double *tdiff,
                     const or_gate *g, uint64_t j0, const uint8_t *in0,
                     size_t len0, const uint8_t *in1, size_t len1,
                     uint8_t *out0, size_t cap0, size_t *olen0, uint8_t *out1,
                     size_t cap1, size_t *olen1);

/* Shortcuts of the paper's Sec. V (off by default: Alg. 2 as written).
 *   OR_SC_PERMUTE: a gate that only reorders amplitudes (X, SWAP, and CU
 *     whose matrix is exactly [[0, 1], [1, 0]], i.e. CNOT) compresses each
 *     block at the ladder level its previous stream used, trying no other.
 *   OR_SC_SKIP: a block whose amplitudes the gate leaves unchanged (by the
 *     gate's structure: a diagonal or controlled gate whose qubit at or
 *     above b is 0 in the block index, PHASE_FLIP away from its index, SWAP
 *     where both bits are equal) keeps its stream; the normalisation s of
 *     that pass is deferred into the block's scale, c_j <- fl(c_j s).  A
 *     block is decoded with the factor fl(c_j s) (s when c_j = 1), its weight
 *     in N^2 is fl(normsq_j fl(c_j c_j)), and c_j returns to 1 when the block
 *     is compressed again.  An exported stream with c_j != 1 sets bit 0 of
 *     header byte 5 and carries c_j as an f64 right after the header. */
enum { OR_SC_PERMUTE = 1, OR_SC_SKIP = 2 };
int or_set_shortcut(or_sim *sim, int flags);

/* Threads for the block groups of a pass (OpenMP); returns the number in
 * effect (1 when built without OpenMP).  Results do not depend on it. */
int or_set_threads(int nthreads);

/* The codec's log2 (finite a > 0) and power of two, used by the
 * pointwise-relative levels (ladder entries -eps): exposed for the tests. */
double or_codec_log2(double a);
double or_codec_exp2(double y);

/* Fidelity |<a|b>|^2 / (<a|a><b|b>) of two 2^n complex arrays. */
double or_fidelity(const double *a, const double *b, int n);

#ifdef __cplusplus
}
#endif
#endif
