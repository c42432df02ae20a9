// device.h -- types shared by the host runtime and the gfx950 kernels of
// libaalcsim.so (internal; the public ABI is include/aalcsim.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace aalc {

// Block stream v1 constants (format of the compressed stride, Sec. III).
constexpr uint32_t kMagic = 0x31424141u;  // "AAB1"
constexpr uint32_t kHdrBytes = 32;
// Header byte 5, bit 0: the 8 bytes after the header hold the block's
// deferred scale c (finite, > 0, not 1), counted in total_bytes; the records
// follow.  Set only on streams of blocks kept by the skip shortcut.
constexpr uint32_t kHdrScaled = 1u;
constexpr uint32_t kScaleBytes = 8;
constexpr uint32_t kPlaneHdrBytes = 16;
constexpr uint32_t kOutlierBytes = 16;
constexpr int kChunk = 64;     // scalars per chunk: one wavefront
constexpr int kWG = 256;       // threads per workgroup: four wavefronts
constexpr int kMaxL = 8;       // ladder levels
constexpr int kMinS = 6;       // segment log2 range supported by the kernels
constexpr int kMaxS = 10;
// Blocks are at most 2^kMaxB amplitudes (sim_create refuses larger).
constexpr int kMaxB = 20;
// Largest |y| (exclusive) that quantises to a code: 2^30 - 1, so codes lie
// in [-(2^30 - 1), 2^30 - 1] and the Lorenzo residual of two codes always
// fits 32 signed bits (the format defines it in 64-bit arithmetic).
constexpr double kQMax = 1073741823.0;
// Per-wave staging of a plane's packed payload (at most 16 chunks x 64 words)
// and of its first kScratchOutl outliers, written while the encode level is
// sized and copied into the record once its arena offset is known.
constexpr uint32_t kScratchOutl = 64;
// Bytes reserved at the start of each arena (bump allocation starts there):
// [0, 16) holds the one all-zero plane record that every all-+0 plane of a
// pass points to.
constexpr uint64_t kArenaBase = 256;
// Where an arena's bump pointer starts after a reset: [kArenaBase, start)
// is reserved for the first chunk of each workgroup of a pass (workgroup i
// takes [kArenaBase + i c, kArenaBase + (i + 1) c), c = its chunk size, at
// most cap / (8 x grid), so all of them fit), which it uses without taking
// it from the bump pointer.
__host__ __device__ inline uint64_t arena_start(uint64_t cap)
{
    return kArenaBase + ((cap / 8) & ~255ull);
}
constexpr uint64_t kScratchPayload = 16 * 64 * 8;
constexpr uint64_t kScratchWave = kScratchPayload + kScratchOutl * 16;
// The staging can be indexed by the hardware slot its wave occupies (XCC,
// shader engine and array, CU, SIMD, wave buffer slot: 17 bits of the
// HW_ID and XCC_ID registers), which no two resident waves share.  One
// device-wide buffer then serves every unit kernel on the GPU, and only the
// waves resident at once touch it, so it stays in the L2 caches.
constexpr uint32_t kHwSlotBits = 17;
constexpr uint64_t kHwSlots = 1ull << kHwSlotBits;
// The device-wide slot-indexed staging of the current GPU (allocated at the
// first call for that GPU, held until the process ends).
hipError_t slot_staging(int device, uint8_t **ptr);

// Gate kinds (numbering of the public header).
enum : uint32_t {
    kNone = 0, kU = 1, kDiag1 = 2, kCU = 3, kCPhase = 4, kCZ = 5, kSwap = 6,
    kX = 7, kPhaseFlip = 8, kDiffuse = 9
};

struct GateArg {
    uint32_t kind;
    int32_t q0, q1;
    uint32_t pad;
    uint64_t index;
    uint64_t mask;  // amplitude i couples with i ^ mask (0: diagonal)
    double u[8];
};

struct Ladder {
    int32_t L;
    int32_t pad;
    double theta;
    double delta[kMaxL];  // 0 = lossless
    double e[kMaxL];      // 2 * delta (exact)
    double r[kMaxL];      // fl(1 / e), rounded on the host
};

// One descriptor set: the stream header of every block and where each plane
// record lives in the arena.  A block's canonical stream is its header
// followed by its plane records in plane order.
struct Desc {
    uint8_t *hdr;         // [nblocks][32] stream headers (block stream v1)
    uint32_t *blk_len;    // [nblocks] canonical stream bytes
    uint8_t *blk_level;   // [nblocks] ladder level of the stream
    uint32_t *plane_off;  // [2*nseg] offset of each plane record, in 8-byte units
    double *segnorm;      // [nseg] pairwise normsq of each segment's x-hat
    double *bscale;       // [nblocks] deferred scale c_j of each block (1 unless the
                          // block was kept by the skip shortcut)
};

// Plane records are 8-byte aligned, so their offsets are stored in 8-byte
// units: a 32-bit entry covers arenas of up to kMaxArenaBytes.
constexpr uint64_t kMaxArenaBytes = 32ull << 30;

__device__ __forceinline__ uint64_t rec_at(const Desc &d, uint64_t plane)
{
    return (uint64_t)d.plane_off[plane] << 3;
}

__device__ __forceinline__ void set_rec_at(const Desc &d, uint64_t plane, uint64_t off)
{
    d.plane_off[plane] = (uint32_t)(off >> 3);
}

// Device-resident scalars of one sim, read and written only by kernels.
// The counters that every workgroup of a pass updates atomically sit on
// their own 128-byte lines, away from the read-mostly scalars.
struct DevState {
    double normsq;          // N^2 of the stored state
    double scale;           // s applied at the next decode
    double tdiff[2];        // 2 * mean for DIFFUSE
    uint64_t resident;      // bytes of the current state
    uint64_t peak_resident;
    double min_ratio;
    double last_ratio;
    uint64_t passes;
    uint32_t err;           // sticky error bits (kErr*)
    uint32_t err_pass;      // pass index of the first error
    int32_t collapsed;
    int32_t normalize;
    double sum[2];          // amplitude sum query result
    uint8_t pad0[128 - 104];
    uint64_t arena_used[2]; // bump pointers of the two arenas
    uint64_t arena_peak;    // largest bump pointer reached (incl. replay waste)
    uint8_t pad1[128 - 24];
    uint32_t n_replay;      // blocks whose chosen level was not the speculated one
    uint32_t n_esc;         // blocks whose computed levels all missed theta
    uint64_t replays;       // cumulative count of replayed blocks
    uint64_t escalations;   // cumulative count of escalated blocks
    uint64_t level_hist[kMaxL];
    uint32_t red_ticket;    // workgroups of the wide reduction done (0 between passes)
    uint32_t pad2;
};

static_assert(offsetof(DevState, arena_used) == 128 && offsetof(DevState, n_replay) == 256,
              "DevState counters must start on their own 128-byte lines");

// kErrImport: an imported stream's records are inconsistent;
// kErrImportNorm: a block's normsq field differs from its decoded values'.
enum : uint32_t { kErrArena = 1u, kErrSize = 2u, kErrImport = 4u, kErrImportNorm = 8u };

// Pass index recorded by the basis-state encode (set_basis), which has no
// earlier state to fall back to.
constexpr uint64_t kBasisPass = 0xFFFFFFFFull;

struct Geo {
    int32_t n, b, s, pad;
    uint64_t nblocks;  // 2^(n-b)
    uint64_t nseg;     // 2^(n-s)
    uint64_t nunits;   // workgroup work items of a pass
};

// Everything a pass kernel needs.
struct PassArgs {
    Geo geo;
    Ladder lad;
    GateArg gate;
    Desc din, dout;
    const uint8_t *arena_in;
    uint8_t *arena_out;
    uint64_t arena_cap;
    int32_t out_arena;   // index of arena_out (bump pointer)
    int32_t in_arena;
    uint64_t pass;       // pass counter (for error reporting; kBasisPass for set_basis)
    uint64_t chunk_bytes;  // arena space a workgroup takes per bump-pointer update
    uint64_t basis;      // source state |basis> when src_basis != 0
    int32_t src_basis;
    int32_t unit_batch;  // units per workgroup round of the bulk phase (<= 1: none)
    // Sec. V shortcuts of this pass: sc_skip -- blocks the gate leaves
    // unchanged by its structure keep their records (copied), their scale
    // becomes fl(c_j s); sc_perm -- the gate only reorders amplitudes, so
    // every block is encoded at its previous level and no other is sized
    int32_t sc_skip;
    int32_t sc_perm;
    // some block of the input may carry a deferred scale (c_j != 1): the
    // unit kernels then read each block's scale (instances with SC = true)
    int32_t sc_scaled;
    int32_t sc_rel;      // the ladder has pointwise-relative levels
    int32_t stage_by_slot;  // scratch is the slot-indexed staging (else by workgroup)
    uint32_t *psz;       // [L][2*nseg]: payload words | n_outliers << 16
    uint8_t *scratch;    // staging: [kHwSlots][kScratchWave] by hardware wave slot
                         // (stage_by_slot), else [scratch_wgs * 4][kScratchWave]
                         // by workgroup and wave
    uint64_t scratch_wgs;  // workgroups the staging covers (grids must not exceed it)
    uint32_t *replay_list;  // [nblocks]
    uint32_t *esc_list;     // [nblocks]
    double *blknorm;     // [nblocks]
    double *segsum;      // [2][nseg] DIFFUSE pre-pass
    double *blksum;      // [2][nblocks]
    DevState *dev;
};

// Kernel identities for the optional per-launch event timer.
enum KernelId : int {
    kIdPass, kIdDecide, kIdEscSize, kIdEscDecide, kIdReplay, kIdBlockNorm,
    kIdReduce, kIdMean, kIdMeanTree, kIdMeanFinal, kIdInitState, kIdSvPair,
    kIdSvDiag, kIdSvPartial, kIdSvFinal, kIdExport, kIdImportScan, kIdImportCheck,
    kIdImportNorm, kIdImportBlocks, kIdPassBulk, kNumKernelIds
};
extern const char *const kKernelNames[kNumKernelIds];

// Host-side timer hook: when non-null, launchers bracket each kernel launch
// with begin/end on the launch stream.
struct Prof {
    virtual void begin(int id, hipStream_t st) = 0;
    virtual void end(int id, hipStream_t st) = 0;
    virtual ~Prof() {}
};

// Launchers (kernels.hip).
void launch_init_state(DevState *dev, int normalize, uint64_t arena_cap, hipStream_t st,
                       Prof *prof);
// Pairwise sums S (re, im) of the normalised amplitudes; out[c] = fl(S_c * mul)
// (device pointer).
void launch_mean(const PassArgs &a, double mul, double *out, hipStream_t st, Prof *prof);
// grid_cap: most workgroups of the unit kernels (they loop over units).
unsigned unit_grid_for(uint64_t units, unsigned cap);
void launch_pass(const PassArgs &a, unsigned grid_cap, hipStream_t st, Prof *prof);
void launch_encode_basis(const PassArgs &a, unsigned grid_cap, hipStream_t st, Prof *prof);
void launch_decode_range(const PassArgs &a, uint64_t first, uint64_t count,
                         double *out, hipStream_t st);
void launch_probs(const PassArgs &a, const int *qubits_dev, int nq,
                  double *probs_dev, hipStream_t st);
void launch_inner(const PassArgs &a, const PassArgs &b, const double *amp_a,
                  const double *amp_b, double *part, double *result,
                  hipStream_t st);
void launch_rsqrt(const double *in, double *out, uint64_t count,
                  hipStream_t st);
// part: 3 * 2^(n - min(n, 10)) doubles; result: 3 doubles (device).
void launch_fourier(const PassArgs &a, const double *amp, uint64_t x, double *part,
                    double *result, hipStream_t st);
void launch_export(const PassArgs &a, uint64_t j, uint8_t *out, hipStream_t st);
void launch_export_headers(const PassArgs &a, uint64_t first, uint64_t count, uint8_t *out,
                           hipStream_t st);
// Streams of blocks [first, first + count) into out, block first + k at
// out + offs[k] (device pointers).
void launch_export_range(const PassArgs &a, uint64_t first, uint64_t count,
                         const uint64_t *offs, uint8_t *out, hipStream_t st, Prof *prof);
// Entropy stage of checkpoints (entropy.hip), blocks of at most
// kEntropyMaxPlanes planes: entropy stream bytes of blocks [first, first +
// count) of the set a.din into elen[k]; the streams themselves into out +
// eoff[k]; and the v1 streams of count given streams (v1 ones copied,
// entropy ones decoded) from src + soff[k] into dst + doff[k] (soff and doff
// with count + 1 entries), errors in kErrImport.
constexpr uint32_t kEntropyMagic = 0x31454141u;  // "AAE1"
constexpr uint64_t kEntropyMaxPlanes = 4096;
void launch_entropy_size(const PassArgs &a, uint64_t first, uint64_t count, uint32_t *elen,
                         hipStream_t st);
void launch_entropy_write(const PassArgs &a, uint64_t first, uint64_t count,
                          const uint64_t *eoff, uint8_t *out, hipStream_t st);
void launch_entropy_expand(const PassArgs &a, uint64_t count, const uint8_t *src,
                           const uint64_t *soff, uint8_t *dst, const uint64_t *doff,
                           hipStream_t st);
// Checkpoint import: streams already copied to a.arena_out + kArenaBase + boff[j]
// become descriptor set a.dout; then N^2 and s as after a pass (a.src_basis
// set: no pass is counted).  Errors set kErrImport / kErrImportNorm.
void launch_import(const PassArgs &a, const uint64_t *boff, hipStream_t st, Prof *prof);

// One batched pass over nst states (device pointers; each prefix has nst + 1
// entries).  upre/bpre count the units/blocks of the states with a gate in
// this pass, mpre/mbpre those of the states whose gate is DIFFUSE.  Grids
// depend only on the set of states, so a captured sequence stays valid when
// the arrays are rewritten.
struct BatchLaunch {
    const PassArgs *args;
    const uint64_t *upre, *bpre, *mpre, *mbpre;
    uint32_t nst;
    unsigned grid_units, grid_blocks;
    bool any_mean, any_ladder;
    bool any_sc;  // some state skips blocks or holds scaled blocks
};
void launch_batch_pass(const BatchLaunch &b, hipStream_t st, Prof *prof);
// Arena chunk a workgroup takes per bump-pointer update.
uint64_t batch_chunk_bytes(uint64_t arena_cap, unsigned grid);

// Allocation-free marginals: the library-held device array (bins of up to
// 2^kNoAllocMaxQ outcomes, then the qubit list) of the current GPU, and a
// fill kernel that clears it (a kernel, so that a captured graph holds no
// memset node).
constexpr int kNoAllocMaxQ = 16;
constexpr uint64_t kNoAllocBinBytes = 8ull << kNoAllocMaxQ;
constexpr uint64_t kNoAllocBytes = kNoAllocBinBytes + 256;
hipError_t noalloc_scratch(int device, void **ptr);
void launch_zero_f64(double *p, uint64_t count, hipStream_t st);

// Uncompressed path (sv.hip).
void sv_set_basis(double *amp, int n, uint64_t x, hipStream_t st);
void sv_apply(double *amp, int n, const GateArg &g, double *scratch,
              double *tdiff_dev, hipStream_t st, Prof *prof);
void sv_probs(const double *amp, int n, const int *qubits_dev, int nq,
              double *probs_dev, hipStream_t st);
void sv_normsq(const double *amp, int n, double *scratch, double *out_dev,
               hipStream_t st);
void sv_sum(const double *amp, int n, double *scratch, double *out_dev, hipStream_t st);

}  // namespace aalc
