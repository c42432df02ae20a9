// sim.cpp -- host runtime behind the C ABI of include/aalcsim.h.
//
// A compressed sim owns two arenas of block streams (ping-pong: a pass reads
// one and writes the other), two descriptor sets locating every block stream
// and plane record, per-plane size tables for the ladder, and a small
// device-resident state (N^2, s, bump pointers, statistics, error bits).
// Passes are queued on the sim's stream without host synchronisation; the
// host learns about device-side errors at the next synchronising call and
// rolls the state back to the input of the failing pass.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <iterator>
#include <map>
#include <string>
#include <vector>

#include "../../include/aalcsim.h"
#include "device.h"

using namespace aalc;

namespace {

thread_local std::string g_err;
thread_local int g_code = SIM_OK;

int fail(int code, const char *fmt, ...)
{
    g_code = code;
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIPCHK(expr)                                                              \
    do {                                                                          \
        hipError_t e_ = (expr);                                                   \
        if (e_ != hipSuccess)                                                     \
            return fail(SIM_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_));     \
    } while (0)

constexpr uint64_t kMiB = 1ull << 20;
constexpr uint64_t kGiB = 1ull << 30;

// Per-launch event timer: a begin and an end event around every kernel,
// resolved into per-kernel totals when read.
struct EventProf final : Prof {
    struct Rec {
        int id;
        hipEvent_t a, b;
    };
    std::vector<Rec> recs;
    std::vector<hipEvent_t> pool;
    hipEvent_t pending = nullptr;
    int pending_id = -1;
    bool only_pass = false;  // time the fused pass kernel only

    hipEvent_t get()
    {
        if (!pool.empty()) {
            hipEvent_t e = pool.back();
            pool.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        // no system-scope fence on record: the events only time kernels
        if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess)
            return nullptr;
        return e;
    }
    void begin(int id, hipStream_t st) override
    {
        if (only_pass && id != kIdPass && id != kIdPassBulk)
            return;
        pending = get();
        pending_id = id;
        if (pending)
            (void)hipEventRecord(pending, st);
    }
    void end(int id, hipStream_t st) override
    {
        if (only_pass && id != kIdPass && id != kIdPassBulk)
            return;
        hipEvent_t e = get();
        if (!e || !pending || id != pending_id)
            return;
        (void)hipEventRecord(e, st);
        recs.push_back({id, pending, e});
        pending = nullptr;
    }
    ~EventProf() override
    {
        for (auto &r : recs) {
            (void)hipEventDestroy(r.a);
            (void)hipEventDestroy(r.b);
        }
        for (auto e : pool)
            (void)hipEventDestroy(e);
    }
};

}  // namespace

// A device-memory context: a caller-owned device buffer (for example a
// torch tensor's storage) that sims created in it carve all their device
// memory from.  First fit over an ordered free list with 256-byte
// alignment; freed ranges merge with their neighbours.
struct sim_ctx {
    uint8_t *base = nullptr;
    uint64_t cap = 0;
    hipStream_t stream = nullptr;  // stream of sims created in it (may be null)
    std::map<uint64_t, uint64_t> free_;  // offset -> bytes
    uint64_t used = 0, peak = 0;
    int nsims = 0;
    int device = 0;

    void *take(uint64_t bytes)
    {
        bytes = (bytes + 255) & ~255ull;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes)
                continue;
            const uint64_t off = it->first, len = it->second;
            free_.erase(it);
            if (len > bytes)
                free_[off + bytes] = len - bytes;
            used += bytes;
            peak = used > peak ? used : peak;
            return base + off;
        }
        return nullptr;
    }
    void give(void *p, uint64_t bytes)
    {
        bytes = (bytes + 255) & ~255ull;
        uint64_t off = (uint64_t)((uint8_t *)p - base);
        used -= bytes;
        auto next = free_.lower_bound(off);
        if (next != free_.end() && off + bytes == next->first) {
            bytes += next->second;
            next = free_.erase(next);
        }
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == off) {
                prev->second += bytes;
                return;
            }
        }
        free_[off] = bytes;
    }
    uint64_t largest_free() const
    {
        uint64_t m = 0;
        for (const auto &f : free_)
            m = f.second > m ? f.second : m;
        return m;
    }
};

struct sim {
    int n = 0, b = 0, s = 0;
    int device = 0;  // the GPU current when the sim was created
    bool compressed = true;
    int shortcut = 0;     // SIM_SC_* flags (Sec. V shortcuts), 0 = Alg. 2 as written
    bool scaled = false;  // some block may carry a deferred scale (after a skip pass
                          // or the import of scaled streams, until set_basis)
    int normalize = 1;
    Ladder lad{};
    Geo geo{};
    hipStream_t stream = nullptr;
    bool own_stream = false;
    // compressed path
    uint8_t *arena[2] = {nullptr, nullptr};
    uint64_t arena_cap = 0;
    Desc desc[2]{};
    uint32_t *psz = nullptr;
    int psz_levels = 0;
    uint8_t *scratch = nullptr;  // per-wave staging for the unit kernels
    uint64_t scratch_wgs = 0;
    bool stage_slot = false;  // scratch is the device-wide slot-indexed staging
    uint32_t *replay_list = nullptr, *esc_list = nullptr;
    double *blknorm = nullptr, *segsum = nullptr, *blksum = nullptr;
    DevState *dev = nullptr;
    int cur = 0;
    uint64_t passes = 0;
    int par = 0;  // arena of the state at passes == 0 (cur == (passes + par) & 1)
    uint64_t *xoff = nullptr;  // [nblocks] stream offsets for whole-state export/import
    bool valid = false;  // the current descriptor set holds a complete state
    unsigned grid_cap = 3072;  // workgroups of the per-gate unit kernels (three per
                               // resident slot of 256 CUs x 4)
    // uncompressed path
    double *amp = nullptr;
    double *sv_scratch = nullptr;
    double *sv_tdiff = nullptr;
    std::vector<std::pair<void *, uint64_t>> allocs;
    uint64_t device_bytes = 0;
    sim_ctx *ctx = nullptr;  // device memory comes from this context when set
    EventProf *prof = nullptr;
};

namespace {

// Device memory of a sim: from its context when it has one (SIM_EBUDGET
// when the context cannot hold it), else hipMalloc (SIM_ENOMEM).
int raw_alloc(sim *S, void **p, uint64_t bytes)
{
    *p = nullptr;
    if (bytes == 0)
        bytes = 8;
    if (S->ctx) {
        *p = S->ctx->take(bytes);
        if (!*p)
            return fail(SIM_EBUDGET, "context exhausted: %llu bytes requested, %llu of %llu "
                        "in use, largest free range %llu",
                        (unsigned long long)bytes, (unsigned long long)S->ctx->used,
                        (unsigned long long)S->ctx->cap,
                        (unsigned long long)S->ctx->largest_free());
        return SIM_OK;
    }
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        *p = nullptr;
        return fail(SIM_ENOMEM, "hipMalloc(%llu bytes) failed: %s",
                    (unsigned long long)bytes, hipGetErrorString(e));
    }
    return SIM_OK;
}

void raw_free(sim *S, void *p, uint64_t bytes)
{
    if (!p)
        return;
    if (S->ctx)
        S->ctx->give(p, bytes ? bytes : 8);
    else
        (void)hipFree(p);
}

// A buffer held for the life of the sim.
int dmalloc(sim *S, void **p, uint64_t bytes)
{
    int rc = raw_alloc(S, p, bytes);
    if (rc)
        return rc;
    S->allocs.push_back({*p, bytes});
    S->device_bytes += bytes;
    return SIM_OK;
}

// Release one buffer obtained from dmalloc (the stream must be idle).
void dfree(sim *S, void *p)
{
    for (auto it = S->allocs.begin(); it != S->allocs.end(); ++it)
        if (it->first == p) {
            raw_free(S, p, it->second);
            S->device_bytes -= it->second;
            S->allocs.erase(it);
            return;
        }
}

void free_all(sim *S)
{
    for (auto &a : S->allocs)
        raw_free(S, a.first, a.second);
    S->allocs.clear();
    S->device_bytes = 0;
}

// A temporary buffer of one call (from the context when the sim has one).
struct Tmp {
    sim *S;
    void *p = nullptr;
    uint64_t bytes = 0;
    explicit Tmp(sim *s) : S(s) {}
    int get(uint64_t n)
    {
        bytes = n;
        return raw_alloc(S, &p, n);
    }
    ~Tmp() { raw_free(S, p, bytes); }
};

// A ladder: optionally lossless first (0), then lossy levels of one kind --
// absolute bounds (>= 2^-30) strictly increasing, or pointwise-relative
// bounds (entries -eps, eps in [2^-19, 0.05]) with eps strictly increasing.
bool ladder_ok(const double *ladder, int L, double theta)
{
    if (!ladder || L < 1 || L > kMaxL || !(theta >= 1.0) || !std::isfinite(theta))
        return false;
    int kind = 0;  // 1 absolute, -1 relative
    for (int k = 0; k < L; ++k) {
        const double d = ladder[k];
        if (!std::isfinite(d))
            return false;
        if (d == 0.0) {
            if (k != 0)
                return false;
            continue;
        }
        const int kk = d > 0.0 ? 1 : -1;
        if (kind && kk != kind)
            return false;
        kind = kk;
        const double mag = std::fabs(d);
        if (mag < (kk < 0 ? 0x1p-19 : 0x1p-30) || (kk < 0 && mag > 0.05))
            return false;
        if (k > 0 && ladder[k - 1] != 0.0 && !(mag > std::fabs(ladder[k - 1])))
            return false;
    }
    return true;
}

// Per level: the bound, the step between codes e (2 delta; for a relative
// level -eps the log-domain step 2 fl(1.4 eps)) and r = fl(1/e).
void set_ladder(Ladder &lad, const double *ladder, int L, double theta)
{
    lad = Ladder{};
    lad.L = L;
    lad.theta = theta;
    for (int k = 0; k < L; ++k) {
        const double d = ladder[k];
        lad.delta[k] = d;
        if (d > 0.0) {
            lad.e[k] = 2.0 * d;
        } else if (d < 0.0) {
            const double dl = 1.4 * -d;
            lad.e[k] = 2.0 * dl;
        } else {
            lad.e[k] = 0.0;
        }
        lad.r[k] = d != 0.0 ? 1.0 / lad.e[k] : 0.0;
    }
}

int ensure_psz(sim *S, int L)
{
    if (S->psz_levels >= L)
        return SIM_OK;
    if (S->psz) {
        HIPCHK(hipStreamSynchronize(S->stream));
        dfree(S, S->psz);
        S->psz = nullptr;
    }
    int rc = dmalloc(S, (void **)&S->psz, (uint64_t)L * 2 * S->geo.nseg * 4);
    if (rc)
        return rc;
    S->psz_levels = L;
    return SIM_OK;
}

// Staging for `wgs` workgroups of the unit kernels (grown on demand).  A
// sim that allocates its own memory uses the device-wide staging indexed by
// hardware wave slot, which serves any grid; a sim in a caller's context
// takes workgroup-indexed staging from the context.
int ensure_scratch(sim *S, uint64_t wgs)
{
    if (!S->ctx) {
        if (!S->stage_slot) {
            const hipError_t e = slot_staging(S->device, &S->scratch);
            if (e != hipSuccess)
                return fail(SIM_ENOMEM, "slot staging of %llu bytes: %s",
                            (unsigned long long)(kHwSlots * kScratchWave),
                            hipGetErrorString(e));
            S->stage_slot = true;
            S->scratch_wgs = 0xFFFFFFFFull;
        }
        return SIM_OK;
    }
    if (S->scratch_wgs >= wgs)
        return SIM_OK;
    if (S->scratch) {
        HIPCHK(hipStreamSynchronize(S->stream));
        dfree(S, S->scratch);
        S->scratch = nullptr;
        S->scratch_wgs = 0;
    }
    int rc = dmalloc(S, (void **)&S->scratch, wgs * 4 * kScratchWave);
    if (rc)
        return rc;
    S->scratch_wgs = wgs;
    return SIM_OK;
}

// Workgroups of the unit kernels of a pass (as launch_pass computes them).
uint64_t unit_grid(const sim *S)
{
    const uint64_t u = S->geo.nunits;
    const uint64_t g = u < S->grid_cap ? u : S->grid_cap;
    return g ? g : 1;
}

uint64_t gate_mask(const sim_gate_t *g)
{
    switch (g->kind) {
    case G_U:
    case G_X:
        return 1ull << g->q0;
    case G_CU:
        return 1ull << g->q1;
    case G_SWAP:
        return (1ull << g->q0) | (1ull << g->q1);
    default:
        return 0;
    }
}

int check_gate(const sim *S, const sim_gate_t *g)
{
    if (!g)
        return fail(SIM_EINVAL, "gate is NULL");
    if (g->pad != 0)
        return fail(SIM_EINVAL, "gate pad must be 0");
    const int n = S->n;
    auto qok = [n](int q) { return q >= 0 && q < n; };
    switch (g->kind) {
    case G_U:
    case G_DIAG1:
    case G_X:
        if (!qok(g->q0))
            return fail(SIM_EINVAL, "qubit %d out of range for n=%d", g->q0, n);
        return SIM_OK;
    case G_CU:
    case G_CPHASE:
    case G_CZ:
    case G_SWAP:
        if (!qok(g->q0) || !qok(g->q1) || g->q0 == g->q1)
            return fail(SIM_EINVAL, "qubits (%d,%d) invalid for n=%d", g->q0, g->q1, n);
        return SIM_OK;
    case G_PHASE_FLIP:
        if (g->index >= (1ull << n))
            return fail(SIM_EINVAL, "index %llu >= 2^%d", (unsigned long long)g->index, n);
        return SIM_OK;
    case G_DIFFUSE:
        return SIM_OK;
    default:
        return fail(SIM_EINVAL, "unknown gate kind %u", g->kind);
    }
}

GateArg to_arg(const sim_gate_t *g)
{
    GateArg a{};
    a.kind = g->kind;
    a.q0 = g->q0;
    a.q1 = g->q1;
    a.index = g->index;
    a.mask = gate_mask(g);
    for (int k = 0; k < 8; ++k)
        a.u[k] = g->u[k];
    return a;
}

// Whether the gate can leave whole blocks of 2^b amplitudes unchanged by
// its structure (a diagonal or controlled gate with a qubit at or above b,
// PHASE_FLIP, SWAP of two qubits at or above b): only then does the skip
// shortcut have blocks to keep in the pass.
bool gate_may_keep(const GateArg &g, int b)
{
    switch (g.kind) {
    case kDiag1:
    case kCU:
        return g.q0 >= b;
    case kCPhase:
    case kCZ:
        return g.q0 >= b || g.q1 >= b;
    case kPhaseFlip:
        return true;
    case kSwap:
        return g.q0 >= b && g.q1 >= b;
    default:
        return false;
    }
}

// A gate that only reorders amplitudes: X, SWAP, and CU whose matrix is
// exactly [[0, 1], [1, 0]] (CNOT), compared bit for bit.
bool gate_permutes(const GateArg &g)
{
    if (g.kind == kX || g.kind == kSwap)
        return true;
    if (g.kind != kCU)
        return false;
    static const double x[8] = {0.0, 0.0, 1.0, 0.0, 1.0, 0.0, 0.0, 0.0};
    return memcmp(g.u, x, sizeof x) == 0;
}

PassArgs make_args(const sim *S, int in, int out, const GateArg &g)
{
    PassArgs a{};
    a.geo = S->geo;
    a.lad = S->lad;
    a.gate = g;
    a.din = S->desc[in];
    a.dout = S->desc[out];
    a.arena_in = S->arena[in];
    a.arena_out = S->arena[out];
    a.arena_cap = S->arena_cap;
    a.out_arena = out;
    a.in_arena = in;
    a.pass = S->passes;
    a.psz = S->psz;
    a.scratch = S->scratch;
    a.scratch_wgs = S->scratch_wgs;
    a.stage_by_slot = S->stage_slot ? 1 : 0;
    a.replay_list = S->replay_list;
    a.esc_list = S->esc_list;
    a.blknorm = S->blknorm;
    a.segsum = S->segsum;
    a.blksum = S->blksum;
    a.dev = S->dev;
    a.sc_skip = (S->shortcut & SIM_SC_SKIP) && gate_may_keep(g, S->b) ? 1 : 0;
    a.sc_perm = (S->shortcut & SIM_SC_PERMUTE) && gate_permutes(g) ? 1 : 0;
    a.sc_scaled = S->scaled ? 1 : 0;
    a.sc_rel = 0;
    for (int k = 0; k < S->lad.L; ++k)
        a.sc_rel |= S->lad.delta[k] < 0.0 ? 1 : 0;
    return a;
}

int reset_devstate(sim *S)
{
    launch_init_state(S->dev, S->normalize, S->arena_cap, S->stream, S->prof);
    HIPCHK(hipGetLastError());
    return SIM_OK;
}

// Synchronise, then surface device-side errors (rolling back on overflow).
int sync_check(sim *S)
{
    HIPCHK(hipStreamSynchronize(S->stream));
    if (!S->compressed)
        return SIM_OK;
    DevState d;
    HIPCHK(hipMemcpy(&d, S->dev, sizeof d, hipMemcpyDeviceToHost));
    if (d.err) {
        const uint64_t pe = d.err_pass;
        const uint32_t bits = d.err;
        if (pe == kBasisPass) {
            // the basis encode itself failed: there is no state to keep
            S->valid = false;
            S->passes = 0;
            S->cur = 0;
            S->par = 0;
            d.err = 0;
            d.err_pass = 0;
            d.passes = 0;
            d.arena_used[0] = d.arena_used[1] = arena_start(S->arena_cap);
            d.n_replay = d.n_esc = 0;
            HIPCHK(hipMemcpy(S->dev, &d, sizeof d, hipMemcpyHostToDevice));
            return fail(bits & kErrSize ? SIM_EDEVICE : SIM_ENOMEM,
                        "the basis state did not fit the %llu-byte arena; the sim holds "
                        "no state until sim_set_basis succeeds",
                        (unsigned long long)S->arena_cap);
        }
        S->passes = pe;
        S->cur = (int)((pe + (uint64_t)S->par) & 1);
        d.err = 0;
        d.err_pass = 0;
        d.passes = pe;
        d.arena_used[1 - S->cur] = arena_start(S->arena_cap);
        d.n_replay = d.n_esc = 0;
        HIPCHK(hipMemcpy(S->dev, &d, sizeof d, hipMemcpyHostToDevice));
        if (bits & kErrSize)
            return fail(SIM_EDEVICE, "internal size mismatch at pass %llu",
                        (unsigned long long)pe);
        return fail(SIM_ENOMEM,
                    "arena capacity %llu bytes exceeded at pass %llu; state rolled back "
                    "to the input of that gate",
                    (unsigned long long)S->arena_cap, (unsigned long long)pe);
    }
    if (d.collapsed)
        return fail(SIM_ECOLLAPSED, "N^2 of the stored state was 0 or not finite");
    return SIM_OK;
}

// Synchronise and require a complete state (for calls that read it).
int sync_state(sim *S)
{
    int rc = sync_check(S);
    if (rc && rc != SIM_ECOLLAPSED)
        return rc;
    if (S->compressed && !S->valid)
        return fail(SIM_EINVAL, "the sim holds no state (a basis encode failed); call "
                    "sim_set_basis");
    return rc;
}

int run_basis(sim *S, uint64_t x)
{
    if (!S->compressed) {
        sv_set_basis(S->amp, S->n, x, S->stream);
        S->passes = 0;
        HIPCHK(hipGetLastError());
        return SIM_OK;
    }
    int rc = reset_devstate(S);
    if (rc)
        return rc;
    GateArg none{};
    none.kind = kNone;
    S->scaled = false;  // every block of a basis state has scale 1
    PassArgs a = make_args(S, 1, 0, none);
    a.src_basis = 1;
    a.basis = x;
    a.pass = kBasisPass;
    launch_encode_basis(a, S->grid_cap, S->stream, S->prof);
    HIPCHK(hipGetLastError());
    S->cur = 0;
    S->par = 0;
    S->passes = 0;
    S->valid = true;  // until a synchronising call reports otherwise
    return SIM_OK;
}

sim *create(int n, int block_log2, double eb, uint64_t arena_bytes, void *stream,
            sim_ctx *ctx = nullptr)
{
    g_err.clear();
    g_code = SIM_OK;
    const bool compressed = !(eb < 0.0);
    if (std::isnan(eb)) {
        fail(SIM_EINVAL, "error_bound is NaN");
        return nullptr;
    }
    if (n < 6 || n > (compressed ? 40 : 34)) {
        fail(SIM_EINVAL, "n_qubits %d out of range", n);
        return nullptr;
    }
    if (block_log2 < 6 || block_log2 > kMaxB) {
        fail(SIM_EINVAL, "block_log2 %d outside [6, 20]", block_log2);
        return nullptr;
    }
    sim *S = new (std::nothrow) sim();
    if (!S) {
        fail(SIM_ENOMEM, "host allocation failed");
        return nullptr;
    }
    S->n = n;
    S->ctx = ctx;
    S->compressed = compressed;
    S->b = block_log2 > n ? n : block_log2;
    S->s = S->b < kMaxS ? S->b : kMaxS;
    if (hipGetDevice(&S->device) != hipSuccess) {
        fail(SIM_EDEVICE, "hipGetDevice failed");
        delete S;
        return nullptr;
    }
    if (ctx && ctx->device != S->device) {
        fail(SIM_EINVAL, "the context's buffer is on device %d, device %d is current",
             ctx->device, S->device);
        delete S;
        return nullptr;
    }
    if (stream) {
        S->stream = (hipStream_t)stream;
    } else {
        if (hipStreamCreateWithFlags(&S->stream, hipStreamNonBlocking) != hipSuccess) {
            fail(SIM_EDEVICE, "hipStreamCreate failed");
            delete S;
            return nullptr;
        }
        S->own_stream = true;
    }
    int rc = SIM_OK;
    if (!compressed) {
        const uint64_t N = 1ull << n;
        rc = dmalloc(S, (void **)&S->amp, 16 * N);
        if (!rc)
            rc = dmalloc(S, (void **)&S->sv_scratch, 16 * ((N >> 16) + 1) + 64);
        if (!rc)
            rc = dmalloc(S, (void **)&S->sv_tdiff, 64);
    } else {
        S->geo.n = n;
        S->geo.b = S->b;
        S->geo.s = S->s;
        S->geo.nblocks = 1ull << (n - S->b);
        S->geo.nseg = 1ull << (n - S->s);
        S->geo.nunits = S->geo.nseg == 1 ? 1 : S->geo.nseg / 2;
        if (eb > 0.0) {
            const double lad[5] = {0.0, eb / 1000.0, eb / 100.0, eb / 10.0, eb};
            if (!ladder_ok(lad, 5, 4.0)) {
                fail(SIM_EINVAL, "error_bound %g gives an invalid ladder (lossy bounds "
                     "must be >= 2^-30)", eb);
                delete S;
                return nullptr;
            }
            set_ladder(S->lad, lad, 5, 4.0);
        } else {
            const double lad[1] = {0.0};
            set_ladder(S->lad, lad, 1, 4.0);
        }
        uint64_t cap = arena_bytes;
        if (cap == 0) {
            // a pass may write a block twice (speculated level, then the chosen one)
            const double want = 2.1 * 16.0 * std::ldexp(1.0, n) + (double)kMiB;
            cap = want > (double)(8 * kGiB) ? 8 * kGiB : (uint64_t)want;
        }
        cap = (cap + 255) & ~255ull;
        if (cap > kMaxArenaBytes)
            rc = fail(SIM_EINVAL, "arena of %llu bytes exceeds the %llu bytes that plane "
                      "offsets address", (unsigned long long)cap,
                      (unsigned long long)kMaxArenaBytes);
        S->arena_cap = cap;
        const uint64_t nb = S->geo.nblocks, ns = S->geo.nseg;
        for (int k = 0; k < 2 && !rc; ++k) {
            rc = dmalloc(S, (void **)&S->arena[k], cap + 64);
            if (!rc)
                rc = dmalloc(S, (void **)&S->desc[k].hdr, 32 * nb);
            if (!rc)
                rc = dmalloc(S, (void **)&S->desc[k].blk_len, 4 * nb);
            if (!rc)
                rc = dmalloc(S, (void **)&S->desc[k].blk_level, nb);
            if (!rc)
                rc = dmalloc(S, (void **)&S->desc[k].plane_off, 4 * 2 * ns);
            if (!rc)
                rc = dmalloc(S, (void **)&S->desc[k].segnorm, 8 * ns);
            if (!rc)
                rc = dmalloc(S, (void **)&S->desc[k].bscale, 8 * nb);
            if (!rc && hipMemset(S->arena[k], 0, kArenaBase) != hipSuccess)
                rc = fail(SIM_EDEVICE, "arena initialisation failed");
        }
        if (!rc)
            rc = dmalloc(S, (void **)&S->replay_list, 4 * nb);
        if (!rc)
            rc = dmalloc(S, (void **)&S->esc_list, 4 * nb);

        if (!rc)
            rc = ensure_psz(S, S->lad.L);
        if (!rc)
            rc = ensure_scratch(S, unit_grid(S));
        if (!rc)
            rc = dmalloc(S, (void **)&S->blknorm, 8 * nb);
        if (!rc)
            rc = dmalloc(S, (void **)&S->segsum, 16 * ns);
        if (!rc)
            rc = dmalloc(S, (void **)&S->blksum, 16 * nb);
        if (!rc)
            rc = dmalloc(S, (void **)&S->dev, sizeof(DevState));
    }
    if (!rc)
        rc = run_basis(S, 0);
    if (!rc)
        rc = sync_state(S);  // the initial encode must fit the arena
    if (rc) {
        std::string keep = g_err;
        free_all(S);
        if (S->own_stream)
            (void)hipStreamDestroy(S->stream);
        delete S;
        g_err = keep;
        return nullptr;
    }
    if (ctx)
        ctx->nsims++;
    return S;
}

}  // namespace

extern "C" {

sim_t *sim_create(int n_qubits, int block_log2, double error_bound)
{
    return create(n_qubits, block_log2, error_bound, 0, nullptr);
}

sim_t *sim_create_ex(int n_qubits, int block_log2, double error_bound,
                     uint64_t arena_bytes, void *hip_stream)
{
    return create(n_qubits, block_log2, error_bound, arena_bytes, hip_stream);
}

int sim_context_create(void *dev_buf, size_t bytes, void *hip_stream, sim_ctx_t **ctx)
{
    g_code = SIM_OK;
    if (!ctx)
        return fail(SIM_EINVAL, "ctx is NULL");
    *ctx = nullptr;
    if (!dev_buf || bytes < 4096)
        return fail(SIM_EINVAL, "a context needs a device buffer of at least 4096 bytes");
    hipPointerAttribute_t at{};
    if (hipPointerGetAttributes(&at, dev_buf) != hipSuccess ||
        at.type != hipMemoryTypeDevice) {
        (void)hipGetLastError();
        return fail(SIM_EINVAL, "dev_buf is not device memory");
    }
    sim_ctx *C = new (std::nothrow) sim_ctx();
    if (!C)
        return fail(SIM_ENOMEM, "host allocation failed");
    // 256-byte aligned start; the tail that is not a multiple of 256 is unused
    const uint64_t a0 = ((uint64_t)(uintptr_t)dev_buf + 255) & ~255ull;
    const uint64_t skip = a0 - (uint64_t)(uintptr_t)dev_buf;
    C->base = (uint8_t *)(uintptr_t)a0;
    C->cap = bytes > skip ? ((bytes - skip) & ~255ull) : 0;
    C->stream = (hipStream_t)hip_stream;
    C->device = at.device;
    if (C->cap)
        C->free_[0] = C->cap;
    *ctx = C;
    return SIM_OK;
}

int sim_context_destroy(sim_ctx_t *C)
{
    if (!C)
        return fail(SIM_EINVAL, "ctx is NULL");
    if (C->nsims)
        return fail(SIM_EINVAL, "%d sims created in the context are still alive", C->nsims);
    delete C;
    return SIM_OK;
}

int sim_context_info(const sim_ctx_t *C, uint64_t *capacity, uint64_t *used, uint64_t *peak,
                     uint64_t *largest_free)
{
    if (!C)
        return fail(SIM_EINVAL, "ctx is NULL");
    if (capacity)
        *capacity = C->cap;
    if (used)
        *used = C->used;
    if (peak)
        *peak = C->peak;
    if (largest_free)
        *largest_free = C->largest_free();
    return SIM_OK;
}

int sim_create_in(sim_ctx_t *ctx, int n_qubits, int block_log2, double error_bound,
                  uint64_t arena_bytes, sim_t **out)
{
    if (!out)
        return fail(SIM_EINVAL, "out is NULL");
    *out = nullptr;
    if (!ctx)
        return fail(SIM_EINVAL, "ctx is NULL");
    sim *S = create(n_qubits, block_log2, error_bound, arena_bytes, ctx->stream, ctx);
    if (!S)
        return g_code ? g_code : SIM_EDEVICE;
    *out = S;
    return SIM_OK;
}

void sim_destroy(sim_t *S)
{
    if (!S)
        return;
    (void)hipStreamSynchronize(S->stream);
    delete S->prof;
    free_all(S);
    if (S->ctx)
        S->ctx->nsims--;
    if (S->own_stream)
        (void)hipStreamDestroy(S->stream);
    delete S;
}

int sim_apply_gate(sim_t *S, const sim_gate_t *gate)
{
    if (!S)
        return fail(SIM_EINVAL, "sim is NULL");
    int rc = check_gate(S, gate);
    if (rc)
        return rc;
    const GateArg g = to_arg(gate);
    if (!S->compressed) {
        sv_apply(S->amp, S->n, g, S->sv_scratch, S->sv_tdiff, S->stream, S->prof);
        HIPCHK(hipGetLastError());
        S->passes++;
        return SIM_OK;
    }
    if (!S->valid)
        return fail(SIM_EINVAL, "the sim holds no state (a basis encode failed); call "
                    "sim_set_basis");
    const int in = S->cur, out = 1 - S->cur;
    PassArgs a = make_args(S, in, out, g);
    if (g.kind == kDiffuse)
        launch_mean(a, ldexp(1.0, 1 - S->n), &S->dev->tdiff[0], S->stream, S->prof);
    launch_pass(a, S->grid_cap, S->stream, S->prof);
    HIPCHK(hipGetLastError());
    if (a.sc_skip)
        S->scaled = true;
    S->cur = out;
    S->passes++;
    return SIM_OK;
}

int sim_apply_gates(sim_t *S, const sim_gate_t *gates, size_t count)
{
    if (!S || (!gates && count))
        return fail(SIM_EINVAL, "NULL argument");
    for (size_t k = 0; k < count; ++k) {
        int rc = sim_apply_gate(S, &gates[k]);
        if (rc) {
            std::string m = g_err;
            return fail(rc, "gate %zu: %s", k, m.c_str());
        }
    }
    return SIM_OK;
}

int sim_set_basis(sim_t *S, uint64_t x)
{
    if (!S)
        return fail(SIM_EINVAL, "sim is NULL");
    if (x >= (1ull << S->n))
        return fail(SIM_EINVAL, "basis index out of range");
    HIPCHK(hipStreamSynchronize(S->stream));
    return run_basis(S, x);
}

int sim_set_aalc(sim_t *S, const double *ladder, int L, double theta)
{
    if (!S)
        return fail(SIM_EINVAL, "sim is NULL");
    if (!S->compressed)
        return fail(SIM_EUNSUPPORTED, "the uncompressed path has no ladder");
    if (!ladder_ok(ladder, L, theta))
        return fail(SIM_EINVAL, "invalid ladder or theta");
    int rc = ensure_psz(S, L);
    if (rc)
        return rc;
    set_ladder(S->lad, ladder, L, theta);
    return SIM_OK;
}

int sim_set_shortcut(sim_t *S, int flags)
{
    if (!S)
        return fail(SIM_EINVAL, "sim is NULL");
    if (flags & ~(SIM_SC_PERMUTE | SIM_SC_SKIP))
        return fail(SIM_EINVAL, "unknown shortcut flags %d", flags);
    if (!S->compressed)
        return fail(SIM_EUNSUPPORTED, "the uncompressed path has no shortcuts");
    S->shortcut = flags;
    return SIM_OK;
}

int sim_set_normalize(sim_t *S, int on)
{
    if (!S)
        return fail(SIM_EINVAL, "sim is NULL");
    if (!S->compressed)
        return fail(SIM_EUNSUPPORTED, "the uncompressed path does not normalise");
    S->normalize = on ? 1 : 0;
    const int32_t flag = S->normalize;
    HIPCHK(hipMemcpyAsync(&S->dev->normalize, &flag, sizeof flag, hipMemcpyHostToDevice,
                          S->stream));
    if (!on) {
        const double one = 1.0;
        HIPCHK(hipMemcpyAsync(&S->dev->scale, &one, sizeof one, hipMemcpyHostToDevice,
                              S->stream));
    }
    HIPCHK(hipStreamSynchronize(S->stream));
    return SIM_OK;
}

int sim_get_amplitudes(sim_t *S, uint64_t first, uint64_t count, double *out)
{
    if (!S || (!out && count))
        return fail(SIM_EINVAL, "NULL argument");
    const uint64_t N = 1ull << S->n;
    if (first > N || count > N - first)
        return fail(SIM_EINVAL, "range out of bounds");
    if (count == 0)
        return SIM_OK;
    if (!S->compressed) {
        HIPCHK(hipMemcpyAsync(out, S->amp + 2 * first, 16 * count, hipMemcpyDeviceToHost,
                              S->stream));
        HIPCHK(hipStreamSynchronize(S->stream));
        return SIM_OK;
    }
    int rc = sync_state(S);
    if (rc && rc != SIM_ECOLLAPSED)
        return rc;
    const uint64_t step = 1ull << 24;
    const uint64_t bcount = count < step ? count : step;
    Tmp tb(S);
    int ra = tb.get(16 * bcount);
    if (ra)
        return ra;
    double *buf = (double *)tb.p;
    PassArgs a = make_args(S, S->cur, 1 - S->cur, GateArg{});
    for (uint64_t off = 0; off < count; off += step) {
        const uint64_t c = count - off < step ? count - off : step;
        launch_decode_range(a, first + off, c, buf, S->stream);
        hipError_t e = hipMemcpyAsync(out + 2 * off, buf, 16 * c, hipMemcpyDeviceToHost,
                                      S->stream);
        if (e == hipSuccess)
            e = hipStreamSynchronize(S->stream);
        if (e != hipSuccess)
            return fail(SIM_EDEVICE, "decode range: %s", hipGetErrorString(e));
    }
    return rc;
}

int sim_export_block(sim_t *S, uint64_t j, void *buf, size_t cap, size_t *len)
{
    if (!S || !len)
        return fail(SIM_EINVAL, "NULL argument");
    if (!S->compressed)
        return fail(SIM_EUNSUPPORTED, "the uncompressed path has no block streams");
    if (j >= S->geo.nblocks)
        return fail(SIM_EINVAL, "block index out of range");
    int rc = sync_state(S);
    if (rc && rc != SIM_ECOLLAPSED)
        return rc;
    uint32_t l = 0;
    HIPCHK(hipMemcpy(&l, S->desc[S->cur].blk_len + j, 4, hipMemcpyDeviceToHost));
    if (l < 32 || l > S->arena_cap)
        return fail(SIM_EDEVICE, "block %llu has an implausible stream length %u",
                    (unsigned long long)j, l);
    *len = l;
    if (cap < l || !buf)
        return fail(SIM_ENOMEM, "buffer of %zu bytes too small for %u", cap, l);
    Tmp ts(S);
    int ra = ts.get(l);
    if (ra)
        return ra;
    uint8_t *stage = (uint8_t *)ts.p;
    launch_export(make_args(S, S->cur, 1 - S->cur, GateArg{}), j, stage, S->stream);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess)
        e = hipMemcpyAsync(buf, stage, l, hipMemcpyDeviceToHost, S->stream);
    if (e == hipSuccess)
        e = hipStreamSynchronize(S->stream);
    if (e != hipSuccess)
        return fail(SIM_EDEVICE, "export: %s", hipGetErrorString(e));
    return rc;
}

int sim_set_grid(sim_t *S, int max_workgroups)
{
    if (!S)
        return fail(SIM_EINVAL, "sim is NULL");
    if (max_workgroups < 64 || max_workgroups > (1 << 16))
        return fail(SIM_EINVAL, "max_workgroups %d outside [64, 65536]", max_workgroups);
    if (!S->compressed) {
        S->grid_cap = (unsigned)max_workgroups;
        return SIM_OK;
    }
    const unsigned old = S->grid_cap;
    S->grid_cap = (unsigned)max_workgroups;
    int rc = ensure_scratch(S, unit_grid(S));
    if (rc)
        S->grid_cap = old;
    return rc;
}

int sim_amplitude_sum(sim_t *S, double *out)
{
    if (!S || !out)
        return fail(SIM_EINVAL, "NULL argument");
    if (!S->compressed) {
        sv_sum(S->amp, S->n, S->sv_scratch, S->sv_tdiff + 2, S->stream);
        HIPCHK(hipMemcpyAsync(out, S->sv_tdiff + 2, 16, hipMemcpyDeviceToHost, S->stream));
        HIPCHK(hipStreamSynchronize(S->stream));
        return SIM_OK;
    }
    int rc = sync_state(S);
    if (rc && rc != SIM_ECOLLAPSED)
        return rc;
    PassArgs a = make_args(S, S->cur, 1 - S->cur, GateArg{});
    launch_mean(a, 1.0, &S->dev->sum[0], S->stream, nullptr);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(out, &S->dev->sum[0], 16, hipMemcpyDeviceToHost, S->stream));
    HIPCHK(hipStreamSynchronize(S->stream));
    return rc;
}

int sim_export_headers(sim_t *S, uint64_t first, uint64_t count, void *buf, size_t cap)
{
    if (!S || (!buf && count))
        return fail(SIM_EINVAL, "NULL argument");
    if (!S->compressed)
        return fail(SIM_EUNSUPPORTED, "the uncompressed path has no block streams");
    if (first > S->geo.nblocks || count > S->geo.nblocks - first)
        return fail(SIM_EINVAL, "block range out of bounds");
    if (cap < 32 * count)
        return fail(SIM_ENOMEM, "buffer of %zu bytes too small for %llu headers", cap,
                    (unsigned long long)count);
    if (count == 0)
        return SIM_OK;
    int rc = sync_state(S);
    if (rc && rc != SIM_ECOLLAPSED)
        return rc;
    Tmp ts(S);
    int ra = ts.get(32 * count);
    if (ra)
        return ra;
    uint8_t *stage = (uint8_t *)ts.p;
    launch_export_headers(make_args(S, S->cur, 1 - S->cur, GateArg{}), first, count, stage,
                          S->stream);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess)
        e = hipMemcpyAsync(buf, stage, 32 * count, hipMemcpyDeviceToHost, S->stream);
    if (e == hipSuccess)
        e = hipStreamSynchronize(S->stream);
    if (e != hipSuccess)
        return fail(SIM_EDEVICE, "export headers: %s", hipGetErrorString(e));
    return rc;
}

int sim_export_state(sim_t *S, void *buf, size_t cap, size_t *len)
{
    if (!S || !len)
        return fail(SIM_EINVAL, "NULL argument");
    if (!S->compressed)
        return fail(SIM_EUNSUPPORTED, "the uncompressed path has no block streams");
    int rc = sync_state(S);
    if (rc && rc != SIM_ECOLLAPSED)
        return rc;
    const uint64_t nb = S->geo.nblocks;
    std::vector<uint32_t> bl(nb);
    HIPCHK(hipMemcpy(bl.data(), S->desc[S->cur].blk_len, 4 * nb, hipMemcpyDeviceToHost));
    // the idle arena stages the streams (above its reserved head, which
    // holds the shared zero record of the next pass)
    const uint64_t room = S->arena_cap - kArenaBase;
    uint64_t total = 0;
    for (uint64_t j = 0; j < nb; ++j) {
        if (bl[j] < kHdrBytes || bl[j] > room)
            return fail(SIM_EDEVICE, "block %llu has an implausible stream length %u",
                        (unsigned long long)j, bl[j]);
        total += bl[j];
    }
    *len = (size_t)total;
    if (!buf || cap < total)
        return fail(SIM_ENOMEM, "buffer of %zu bytes too small for %llu", cap,
                    (unsigned long long)total);
    if (!S->xoff) {
        int r2 = dmalloc(S, (void **)&S->xoff, 8 * nb);
        if (r2)
            return r2;
    }
    uint8_t *stage = S->arena[1 - S->cur] + kArenaBase;
    const PassArgs a = make_args(S, S->cur, 1 - S->cur, GateArg{});
    std::vector<uint64_t> offs(nb);
    uint64_t done = 0;
    for (uint64_t j0 = 0; j0 < nb;) {
        // the longest run of blocks whose streams fit the staging area
        uint64_t j1 = j0, bytes = 0;
        while (j1 < nb && bytes + bl[j1] <= room) {
            offs[j1 - j0] = bytes;
            bytes += bl[j1];
            ++j1;
        }
        HIPCHK(hipMemcpyAsync(S->xoff, offs.data(), 8 * (j1 - j0), hipMemcpyHostToDevice,
                              S->stream));
        launch_export_range(a, j0, j1 - j0, S->xoff, stage, S->stream, S->prof);
        HIPCHK(hipGetLastError());
        HIPCHK(hipMemcpyAsync((uint8_t *)buf + done, stage, bytes, hipMemcpyDeviceToHost,
                              S->stream));
        HIPCHK(hipStreamSynchronize(S->stream));
        done += bytes;
        j0 = j1;
    }
    return rc;
}

int sim_export_state_entropy(sim_t *S, void *buf, size_t cap, size_t *len)
{
    if (!S || !len)
        return fail(SIM_EINVAL, "NULL argument");
    if (!S->compressed)
        return fail(SIM_EUNSUPPORTED, "the uncompressed path has no block streams");
    if ((2ull << (S->b - S->s)) > kEntropyMaxPlanes)
        return fail(SIM_EUNSUPPORTED, "the entropy stage takes blocks of at most %llu planes "
                    "(b - s <= 11)", (unsigned long long)kEntropyMaxPlanes);
    int rc = sync_state(S);
    if (rc && rc != SIM_ECOLLAPSED)
        return rc;
    const uint64_t nb = S->geo.nblocks;
    if (!S->xoff) {
        int r2 = dmalloc(S, (void **)&S->xoff, 8 * nb);
        if (r2)
            return r2;
    }
    // entropy stream lengths (4 bytes per block, in the offsets array's room)
    const PassArgs a = make_args(S, S->cur, 1 - S->cur, GateArg{});
    uint32_t *elen_dev = (uint32_t *)S->xoff;
    launch_entropy_size(a, 0, nb, elen_dev, S->stream);
    HIPCHK(hipGetLastError());
    std::vector<uint32_t> el(nb);
    HIPCHK(hipMemcpyAsync(el.data(), elen_dev, 4 * nb, hipMemcpyDeviceToHost, S->stream));
    HIPCHK(hipStreamSynchronize(S->stream));
    const uint64_t room = S->arena_cap - kArenaBase;
    uint64_t total = 0;
    for (uint64_t j = 0; j < nb; ++j) {
        if (el[j] < kHdrBytes + 8 || el[j] > room)
            return fail(SIM_EDEVICE, "block %llu has an implausible entropy stream length %u",
                        (unsigned long long)j, el[j]);
        total += el[j];
    }
    *len = (size_t)total;
    if (!buf || cap < total)
        return fail(SIM_ENOMEM, "buffer of %zu bytes too small for %llu", cap,
                    (unsigned long long)total);
    uint8_t *stage = S->arena[1 - S->cur] + kArenaBase;
    std::vector<uint64_t> offs(nb);
    uint64_t done = 0;
    for (uint64_t j0 = 0; j0 < nb;) {
        uint64_t j1 = j0, bytes = 0;
        while (j1 < nb && bytes + el[j1] <= room) {
            offs[j1 - j0] = bytes;
            bytes += el[j1];
            ++j1;
        }
        HIPCHK(hipMemcpyAsync(S->xoff, offs.data(), 8 * (j1 - j0), hipMemcpyHostToDevice,
                              S->stream));
        launch_entropy_write(a, j0, j1 - j0, S->xoff, stage, S->stream);
        HIPCHK(hipGetLastError());
        HIPCHK(hipMemcpyAsync((uint8_t *)buf + done, stage, bytes, hipMemcpyDeviceToHost,
                              S->stream));
        HIPCHK(hipStreamSynchronize(S->stream));
        done += bytes;
        j0 = j1;
    }
    return rc;
}

int sim_import_state(sim_t *S, const void *buf, size_t len)
{
    if (!S || (!buf && len))
        return fail(SIM_EINVAL, "NULL argument");
    if (!S->compressed)
        return fail(SIM_EUNSUPPORTED, "the uncompressed path has no block streams");
    const uint64_t nb = S->geo.nblocks;
    const uint8_t *p = (const uint8_t *)buf;
    // per block: where its stream starts in buf (soff) and where its v1
    // stream goes in the arena (boff); entropy streams are expanded there
    std::vector<uint64_t> boff(nb + 1), soff(nb + 1);
    uint64_t pos = 0, vpos = 0;
    bool scaled_any = false, any_entropy = false;
    const uint64_t planes = 2ull << (S->b - S->s);
    for (uint64_t j = 0; j < nb; ++j) {
        if (len - pos < kHdrBytes)
            return fail(SIM_EINVAL, "stream of block %llu truncated", (unsigned long long)j);
        const uint8_t *h = p + pos;
        uint32_t magic, total;
        double delta;
        memcpy(&magic, h, 4);
        memcpy(&total, h + 12, 4);
        memcpy(&delta, h + 16, 8);
        const int level = h[4];
        const bool ent = magic == kEntropyMagic;
        if ((magic != kMagic && !ent) || (h[5] & ~kHdrScaled) != 0 || h[6] != S->s ||
            h[7] != S->b)
            return fail(SIM_EINVAL, "block %llu: bad magic, flags or geometry (s %d, b %d "
                        "expected)", (unsigned long long)j, S->s, S->b);
        if (ent && planes > kEntropyMaxPlanes)
            return fail(SIM_EUNSUPPORTED, "block %llu: entropy streams take blocks of at most "
                        "%llu planes", (unsigned long long)j,
                        (unsigned long long)kEntropyMaxPlanes);
        // an entropy stream has its v1 length and item count after the header
        const uint32_t extra = ent ? 8u : 0u;
        uint32_t vlen = total;
        if (ent) {
            if (total < kHdrBytes + extra || total > len - pos)
                return fail(SIM_EINVAL, "block %llu: stream length %u invalid",
                            (unsigned long long)j, total);
            memcpy(&vlen, h + kHdrBytes, 4);
            const uint64_t vmin = kHdrBytes + ((h[5] & kHdrScaled) ? kScaleBytes : 0u) +
                                  (uint64_t)kPlaneHdrBytes * planes;
            if (vlen < vmin || vlen % 8 != 0)
                return fail(SIM_EINVAL, "block %llu: v1 length %u of an entropy stream invalid",
                            (unsigned long long)j, vlen);
            any_entropy = true;
        }
        if (h[5] & kHdrScaled) {
            // a deferred scale c after the header: finite, > 0 and not 1
            double c = 0.0;
            if (total < kHdrBytes + extra + kScaleBytes || total > len - pos)
                return fail(SIM_EINVAL, "block %llu: stream length %u invalid",
                            (unsigned long long)j, total);
            memcpy(&c, h + kHdrBytes + extra, 8);
            if (!std::isfinite(c) || !(c > 0.0) || c == 1.0)
                return fail(SIM_EINVAL, "block %llu: invalid deferred scale %.17g",
                            (unsigned long long)j, c);
            scaled_any = true;
        }
        if (level >= S->lad.L || memcmp(&delta, &S->lad.delta[level], 8) != 0)
            return fail(SIM_EINVAL, "block %llu: level %d with bound %.17g is not a level of "
                        "this sim's ladder", (unsigned long long)j, level, delta);
        if (total < kHdrBytes || total % 8 != 0 || total > len - pos)
            return fail(SIM_EINVAL, "block %llu: stream length %u invalid",
                        (unsigned long long)j, total);
        soff[j] = pos;
        boff[j] = vpos;
        pos += total;
        vpos += vlen;
    }
    soff[nb] = pos;
    boff[nb] = vpos;
    if (pos != len)
        return fail(SIM_EINVAL, "%llu bytes after the last block stream",
                    (unsigned long long)(len - pos));
    // entropy streams sit above the room of the v1 streams they expand to
    const uint64_t vroom = (vpos + 255) & ~255ull;
    const uint64_t need = any_entropy ? vroom + len : len;
    if (need > S->arena_cap - kArenaBase)
        return fail(SIM_ENOMEM, "%llu bytes of streams exceed the arena (%llu bytes)",
                    (unsigned long long)need, (unsigned long long)S->arena_cap);
    Tmp offs_dev(S);
    if (any_entropy) {
        int r2 = offs_dev.get(16 * (nb + 1));
        if (r2)
            return r2;
    }
    if (!S->xoff) {
        int r2 = dmalloc(S, (void **)&S->xoff, 8 * nb);
        if (r2)
            return r2;
    }
    // the current state (if any) stays intact in the other arena and
    // descriptor set until the import has passed every check
    HIPCHK(hipStreamSynchronize(S->stream));
    DevState keep;
    HIPCHK(hipMemcpy(&keep, S->dev, sizeof keep, hipMemcpyDeviceToHost));
    const int out = 1 - S->cur;
    DevState d{};
    d.scale = 1.0;
    d.normalize = S->normalize;
    d.arena_used[0] = d.arena_used[1] = arena_start(S->arena_cap);
    d.arena_used[out] = kArenaBase + vroom;
    HIPCHK(hipMemcpyAsync(S->dev, &d, sizeof d, hipMemcpyHostToDevice, S->stream));
    uint8_t *varea = S->arena[out] + kArenaBase;
    HIPCHK(hipMemcpyAsync(any_entropy ? varea + vroom : varea, buf, len, hipMemcpyHostToDevice,
                          S->stream));
    HIPCHK(hipMemcpyAsync(S->xoff, boff.data(), 8 * nb, hipMemcpyHostToDevice, S->stream));
    PassArgs a = make_args(S, out, out, GateArg{});
    if (any_entropy) {
        // v1 streams copied, entropy streams decoded, into their v1 places
        uint64_t *so = (uint64_t *)offs_dev.p, *vo = so + (nb + 1);
        HIPCHK(hipMemcpyAsync(so, soff.data(), 8 * (nb + 1), hipMemcpyHostToDevice,
                              S->stream));
        HIPCHK(hipMemcpyAsync(vo, boff.data(), 8 * (nb + 1), hipMemcpyHostToDevice,
                              S->stream));
        launch_entropy_expand(a, nb, varea + vroom, so, varea, vo, S->stream);
        HIPCHK(hipGetLastError());
    }
    a.in_arena = 1 - out;  // the reduction frees the previous state's arena
    a.pass = kBasisPass;
    launch_import(a, S->xoff, S->stream, S->prof);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(S->stream));
    HIPCHK(hipMemcpy(&d, S->dev, sizeof d, hipMemcpyDeviceToHost));
    if (d.err & (kErrImport | kErrImportNorm)) {
        HIPCHK(hipMemcpy(S->dev, &keep, sizeof keep, hipMemcpyHostToDevice));
        return fail(SIM_EINVAL, (d.err & kErrImport)
                                    ? "a plane record is malformed (sizes, widths, anchor "
                                      "or outliers); state unchanged"
                                    : "a block's normsq field differs from its decoded "
                                      "values; state unchanged");
    }
    if (d.err)
        return fail(SIM_EDEVICE, "device error %u during import", d.err);
    S->cur = out;
    S->par = out;
    S->passes = 0;
    S->valid = true;
    S->scaled = scaled_any;
    return sync_check(S);
}

int sim_stats(sim_t *S, sim_stats_t *st)
{
    if (!S || !st)
        return fail(SIM_EINVAL, "NULL argument");
    memset(st, 0, sizeof *st);
    st->device_bytes = S->device_bytes;
    st->passes = S->passes;
    if (!S->compressed) {
        double ns = 0.0;
        sv_normsq(S->amp, S->n, S->sv_scratch, S->sv_tdiff + 4, S->stream);
        HIPCHK(hipMemcpyAsync(&ns, S->sv_tdiff + 4, 8, hipMemcpyDeviceToHost, S->stream));
        HIPCHK(hipStreamSynchronize(S->stream));
        st->normsq = ns;
        st->scale = 1.0;
        st->compressed = 0;
        st->resident_bytes = 16ull << S->n;
        st->peak_resident = st->resident_bytes;
        st->min_ratio = st->last_ratio = 1.0;
        return SIM_OK;
    }
    int rc = sync_check(S);
    if (rc && rc != SIM_ECOLLAPSED)
        return rc;
    DevState d;
    HIPCHK(hipMemcpy(&d, S->dev, sizeof d, hipMemcpyDeviceToHost));
    st->normsq = d.normsq;
    st->scale = d.scale;
    st->collapsed = d.collapsed;
    st->compressed = 1;
    st->resident_bytes = d.resident;
    st->peak_resident = d.peak_resident;
    st->min_ratio = d.min_ratio;
    st->last_ratio = d.last_ratio;
    st->passes = d.passes;
    for (int k = 0; k < kMaxL; ++k)
        st->level_hist[k] = d.level_hist[k];
    st->arena_bytes = S->arena_cap;
    st->replays = d.replays;
    st->escalations = d.escalations;
    st->arena_peak = d.arena_peak;
    return rc;
}

int sim_sync(sim_t *S)
{
    if (!S)
        return fail(SIM_EINVAL, "sim is NULL");
    return sync_check(S);
}

int sim_set_stream(sim_t *S, void *hip_stream)
{
    if (!S)
        return fail(SIM_EINVAL, "sim is NULL");
    HIPCHK(hipStreamSynchronize(S->stream));
    if (S->own_stream)
        (void)hipStreamDestroy(S->stream);
    if (hip_stream) {
        S->stream = (hipStream_t)hip_stream;
        S->own_stream = false;
    } else {
        HIPCHK(hipStreamCreateWithFlags(&S->stream, hipStreamNonBlocking));
        S->own_stream = true;
    }
    return SIM_OK;
}

}  // extern "C"

namespace {

int probs_args_ok(const sim *S, const int *qubits, int nq, const double *probs, int max_nq)
{
    if (!S || !qubits || !probs)
        return fail(SIM_EINVAL, "NULL argument");
    if (nq < 1 || nq > max_nq)
        return fail(SIM_EINVAL, "nq %d out of range [1, %d]", nq, max_nq);
    for (int k = 0; k < nq; ++k) {
        if (qubits[k] < 0 || qubits[k] >= S->n)
            return fail(SIM_EINVAL, "qubit %d out of range", qubits[k]);
        for (int m = 0; m < k; ++m)
            if (qubits[m] == qubits[k])
                return fail(SIM_EINVAL, "qubit %d listed twice", qubits[k]);
    }
    return SIM_OK;
}

// The marginal probabilities with bins dp (2^nq doubles) and qubit list dq
// (nq ints) in device memory the caller provides; dp is cleared here.
hipError_t probs_into(sim *S, int *dq, double *dp, const int *qubits, int nq, double *probs)
{
    const size_t nb = (size_t)1 << nq;
    hipError_t e = hipMemcpyAsync(dq, qubits, sizeof(int) * nq, hipMemcpyHostToDevice,
                                  S->stream);
    if (e == hipSuccess) {
        launch_zero_f64(dp, nb, S->stream);
        e = hipGetLastError();
    }
    if (e == hipSuccess) {
        if (S->compressed)
            launch_probs(make_args(S, S->cur, 1 - S->cur, GateArg{}), dq, nq, dp, S->stream);
        else
            sv_probs(S->amp, S->n, dq, nq, dp, S->stream);
        e = hipGetLastError();
    }
    if (e == hipSuccess)
        e = hipMemcpyAsync(probs, dp, 8 * nb, hipMemcpyDeviceToHost, S->stream);
    if (e == hipSuccess)
        e = hipStreamSynchronize(S->stream);
    return e;
}

}  // namespace

extern "C" {

int sim_measure_probs(sim_t *S, const int *qubits, int nq, double *probs)
{
    int rc = probs_args_ok(S, qubits, nq, probs, 24);
    if (rc)
        return rc;
    rc = S->compressed ? sync_state(S) : SIM_OK;
    if (rc && rc != SIM_ECOLLAPSED)
        return rc;
    const size_t nb = (size_t)1 << nq;
    Tmp tp(S);
    int ra = tp.get(8 * nb + 256);
    if (ra)
        return ra;
    double *dp = (double *)tp.p;
    int *dq = (int *)((uint8_t *)tp.p + 8 * nb);
    hipError_t e = probs_into(S, dq, dp, qubits, nq, probs);
    if (e != hipSuccess)
        return fail(SIM_EDEVICE, "measure: %s", hipGetErrorString(e));
    return rc;
}

int sim_measure_probs_noalloc(sim_t *S, const int *qubits, int nq, double *probs)
{
    int rc = probs_args_ok(S, qubits, nq, probs, kNoAllocMaxQ);
    if (rc)
        return rc;
    rc = S->compressed ? sync_state(S) : SIM_OK;
    if (rc && rc != SIM_ECOLLAPSED)
        return rc;
    // the library-held array of the sim's GPU (its address is looked up on
    // the first call on that GPU, with that GPU current)
    int prev = -1;
    HIPCHK(hipGetDevice(&prev));
    if (prev != S->device)
        HIPCHK(hipSetDevice(S->device));
    void *base = nullptr;
    hipError_t e = noalloc_scratch(S->device, &base);
    if (e == hipSuccess) {
        double *dp = (double *)base;
        int *dq = (int *)((uint8_t *)base + kNoAllocBinBytes);
        e = probs_into(S, dq, dp, qubits, nq, probs);
    }
    if (prev != S->device)
        (void)hipSetDevice(prev);
    if (e != hipSuccess)
        return fail(SIM_EDEVICE, "measure (no allocation): %s", hipGetErrorString(e));
    return rc;
}

int sim_fidelity(sim_t *A, sim_t *B, double *F)
{
    if (!A || !B || !F)
        return fail(SIM_EINVAL, "NULL argument");
    if (A->n != B->n)
        return fail(SIM_EINVAL, "qubit counts differ (%d vs %d)", A->n, B->n);
    int ra = A->compressed ? sync_state(A) : SIM_OK;
    if (ra && ra != SIM_ECOLLAPSED)
        return ra;
    int rb = B->compressed ? sync_state(B) : SIM_OK;
    if (rb && rb != SIM_ECOLLAPSED)
        return rb;
    HIPCHK(hipStreamSynchronize(A->stream));
    HIPCHK(hipStreamSynchronize(B->stream));
    const int n = A->n;
    const int S = n < kMaxS ? n : kMaxS;
    const uint64_t nr = 1ull << (n - S);
    Tmp tp(A);
    int rt = tp.get(8 * (4 * nr + 8));
    if (rt)
        return rt;
    double *part = (double *)tp.p;
    PassArgs pa = A->compressed ? make_args(A, A->cur, 1 - A->cur, GateArg{}) : PassArgs{};
    PassArgs pb = B->compressed ? make_args(B, B->cur, 1 - B->cur, GateArg{}) : PassArgs{};
    pa.geo.n = n;
    launch_inner(pa, pb, A->compressed ? nullptr : A->amp, B->compressed ? nullptr : B->amp,
                 part, part + 4 * nr, A->stream);
    double res[5];
    hipError_t e = hipGetLastError();
    if (e == hipSuccess)
        e = hipMemcpyAsync(res, part + 4 * nr, sizeof res, hipMemcpyDeviceToHost, A->stream);
    if (e == hipSuccess)
        e = hipStreamSynchronize(A->stream);
    if (e != hipSuccess)
        return fail(SIM_EDEVICE, "fidelity: %s", hipGetErrorString(e));
    *F = res[0];
    return ra ? ra : rb;
}

int sim_fourier_overlap(sim_t *S, uint64_t x, double *out)
{
    if (!S || !out)
        return fail(SIM_EINVAL, "NULL argument");
    if (x >= (1ull << S->n))
        return fail(SIM_EINVAL, "x out of range");
    int rc = S->compressed ? sync_state(S) : SIM_OK;
    if (rc && rc != SIM_ECOLLAPSED)
        return rc;
    HIPCHK(hipStreamSynchronize(S->stream));
    const int n = S->n;
    const int Sg = n < kMaxS ? n : kMaxS;
    const uint64_t nr = 1ull << (n - Sg);
    Tmp tp(S);
    int rt = tp.get(8 * (3 * nr + 4));
    if (rt)
        return rt;
    double *part = (double *)tp.p;
    PassArgs pa = S->compressed ? make_args(S, S->cur, 1 - S->cur, GateArg{}) : PassArgs{};
    pa.geo.n = n;
    launch_fourier(pa, S->compressed ? nullptr : S->amp, x, part, part + 3 * nr, S->stream);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess)
        e = hipMemcpyAsync(out, part + 3 * nr, 3 * sizeof(double), hipMemcpyDeviceToHost,
                           S->stream);
    if (e == hipSuccess)
        e = hipStreamSynchronize(S->stream);
    if (e != hipSuccess)
        return fail(SIM_EDEVICE, "fourier overlap: %s", hipGetErrorString(e));
    return rc;
}

int sim_debug_rsqrt(const double *in, double *out, size_t count)
{
    if (!in || !out)
        return fail(SIM_EINVAL, "NULL argument");
    if (!count)
        return SIM_OK;
    double *d = nullptr;
    HIPCHK(hipMalloc((void **)&d, 16 * count));
    hipError_t e = hipMemcpy(d, in, 8 * count, hipMemcpyHostToDevice);
    if (e == hipSuccess) {
        launch_rsqrt(d, d + count, count, nullptr);
        e = hipGetLastError();
    }
    if (e == hipSuccess)
        e = hipMemcpy(out, d + count, 8 * count, hipMemcpyDeviceToHost);
    (void)hipFree(d);
    if (e != hipSuccess)
        return fail(SIM_EDEVICE, "rsqrt: %s", hipGetErrorString(e));
    return SIM_OK;
}

}  // extern "C"

namespace {

int prof_set(EventProf *&P, hipStream_t st, int on)
{
    HIPCHK(hipStreamSynchronize(st));
    if (on < 0 || on > 2)
        return fail(SIM_EINVAL, "profile mode %d", on);
    if (on && !P)
        P = new (std::nothrow) EventProf();
    if (on && !P)
        return fail(SIM_ENOMEM, "profiler allocation failed");
    if (on)
        P->only_pass = (on == 2);
    if (!on) {
        delete P;
        P = nullptr;
    }
    return SIM_OK;
}

int prof_read(EventProf *P, hipStream_t st, sim_kernel_time_t *out, int cap, int *count)
{
    if (!count || (cap > 0 && !out))
        return fail(SIM_EINVAL, "NULL argument");
    *count = 0;
    if (!P)
        return SIM_OK;
    HIPCHK(hipStreamSynchronize(st));
    sim_kernel_time_t acc[kNumKernelIds];
    memset(acc, 0, sizeof acc);
    for (auto &r : P->recs) {
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
            sim_kernel_time_t &k = acc[r.id];
            if (k.launches == 0 || ms < k.min_ms)
                k.min_ms = ms;
            if (ms > k.max_ms)
                k.max_ms = ms;
            k.total_ms += ms;
            k.launches += 1;
        }
        P->pool.push_back(r.a);
        P->pool.push_back(r.b);
    }
    P->recs.clear();
    int m = 0;
    for (int id = 0; id < kNumKernelIds; ++id) {
        if (!acc[id].launches)
            continue;
        if (m < cap) {
            out[m] = acc[id];
            snprintf(out[m].name, sizeof out[m].name, "%s", kKernelNames[id]);
        }
        ++m;
    }
    *count = m;
    return SIM_OK;
}

}  // namespace

extern "C" {

int sim_profile(sim_t *S, int on)
{
    if (!S)
        return fail(SIM_EINVAL, "sim is NULL");
    return prof_set(S->prof, S->stream, on);
}

int sim_profile_read(sim_t *S, sim_kernel_time_t *out, int cap, int *count)
{
    if (!S)
        return fail(SIM_EINVAL, "NULL argument");
    return prof_read(S->prof, S->stream, out, cap, count);
}

const char *sim_last_error(void) { return g_err.c_str(); }

}  // extern "C"

// ------------------------------------------------------------ batches -----

struct sim_batch {
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int max_states = 0, max_passes = 0;
    size_t slot_bytes = 0;     // one pass: PassArgs[max_states] + 4 prefixes
    uint8_t *dslots = nullptr; // device [max_passes] slots
    uint8_t *scratch = nullptr; // the device-wide slot-indexed staging (not owned)
    uint8_t *hslots = nullptr; // pinned host mirror
    hipEvent_t uploaded = nullptr;  // the last upload from hslots has finished
    hipEvent_t joined = nullptr;
    std::vector<hipEvent_t> sim_ev;
    struct Graph {
        std::vector<uint8_t> key;
        hipGraph_t g = nullptr;
        hipGraphExec_t exec = nullptr;
    };
    std::vector<Graph> graphs;
    uint64_t graph_launches = 0, graph_builds = 0;
    EventProf *prof = nullptr;  // when set, passes are launched directly and timed
};

namespace {

constexpr size_t kMaxGraphs = 16;
constexpr unsigned kMaxBatchGrid = 4096;

size_t slot_prefix_off(int max_states)
{
    return ((size_t)max_states * sizeof(PassArgs) + 255) & ~(size_t)255;
}

void destroy_graph(sim_batch::Graph &G)
{
    if (G.exec)
        (void)hipGraphExecDestroy(G.exec);
    if (G.g)
        (void)hipGraphDestroy(G.g);
    G.exec = nullptr;
    G.g = nullptr;
}

BatchLaunch slot_launch(const sim_batch *B, int p, uint32_t nst, unsigned gu, unsigned gb,
                        bool mean, bool ladder, bool sc)
{
    const uint8_t *base = B->dslots + (size_t)p * B->slot_bytes;
    const uint64_t *pre = (const uint64_t *)(base + slot_prefix_off(B->max_states));
    const size_t stride = (size_t)B->max_states + 1;
    BatchLaunch L{};
    L.args = (const PassArgs *)base;
    L.upre = pre;
    L.bpre = pre + stride;
    L.mpre = pre + 2 * stride;
    L.mbpre = pre + 3 * stride;
    L.nst = nst;
    L.grid_units = gu;
    L.grid_blocks = gb;
    L.any_mean = mean;
    L.any_ladder = ladder;
    L.any_sc = sc;
    return L;
}

void batch_free(sim_batch *B)
{
    if (B->stream)
        (void)hipStreamSynchronize(B->stream);
    for (auto &G : B->graphs)
        destroy_graph(G);
    for (auto e : B->sim_ev)
        (void)hipEventDestroy(e);
    if (B->uploaded)
        (void)hipEventDestroy(B->uploaded);
    if (B->joined)
        (void)hipEventDestroy(B->joined);
    if (B->dslots)
        (void)hipFree(B->dslots);
    if (B->hslots)
        (void)hipHostFree(B->hslots);
    delete B->prof;
    if (B->own_stream && B->stream)
        (void)hipStreamDestroy(B->stream);
    delete B;
}

}  // namespace

extern "C" {

sim_batch_t *sim_batch_create(int max_states, int max_passes, void *hip_stream)
{
    g_err.clear();
    if (max_states < 1 || max_states > 4096 || max_passes < 1 || max_passes > 4096) {
        fail(SIM_EINVAL, "max_states %d / max_passes %d out of range [1, 4096]", max_states,
             max_passes);
        return nullptr;
    }
    sim_batch *B = new (std::nothrow) sim_batch();
    if (!B) {
        fail(SIM_ENOMEM, "host allocation failed");
        return nullptr;
    }
    B->max_states = max_states;
    B->max_passes = max_passes;
    B->slot_bytes = (slot_prefix_off(max_states) + 4 * 8 * ((size_t)max_states + 1) + 255) &
                    ~(size_t)255;
    const size_t total = B->slot_bytes * (size_t)max_passes;
    bool ok = true;
    if (hip_stream) {
        B->stream = (hipStream_t)hip_stream;
    } else {
        ok = hipStreamCreateWithFlags(&B->stream, hipStreamNonBlocking) == hipSuccess;
        B->own_stream = ok;
    }
    ok = ok && hipMalloc((void **)&B->dslots, total) == hipSuccess;
    int dev = 0;
    ok = ok && hipGetDevice(&dev) == hipSuccess;
    ok = ok && slot_staging(dev, &B->scratch) == hipSuccess;
    ok = ok && hipHostMalloc((void **)&B->hslots, total, hipHostMallocDefault) == hipSuccess;
    ok = ok && hipEventCreateWithFlags(&B->uploaded, hipEventDisableTiming) == hipSuccess;
    ok = ok && hipEventCreateWithFlags(&B->joined, hipEventDisableTiming) == hipSuccess;
    if (!ok) {
        (void)hipGetLastError();
        fail(SIM_ENOMEM, "batch allocation of %zu bytes failed", total);
        batch_free(B);
        return nullptr;
    }
    return B;
}

void sim_batch_destroy(sim_batch_t *B)
{
    if (B)
        batch_free(B);
}

int sim_batch_apply(sim_batch_t *B, sim_t *const *sims, int count, const sim_gate_t *gates,
                    int passes, int use_graph)
{
    if (!B || !sims || !gates)
        return fail(SIM_EINVAL, "NULL argument");
    if (count < 1 || count > B->max_states || passes < 1 || passes > B->max_passes)
        return fail(SIM_EINVAL, "count %d / passes %d outside the batch's limits (%d, %d)",
                    count, passes, B->max_states, B->max_passes);
    // validate everything before queuing anything
    uint64_t units = 0, blocks = 0;
    bool ladder = false, sc = false;
    for (int k = 0; k < count; ++k) {
        sim *S = sims[k];
        if (!S)
            return fail(SIM_EINVAL, "sims[%d] is NULL", k);
        if (!S->compressed)
            return fail(SIM_EUNSUPPORTED, "sims[%d] is uncompressed", k);
        for (int m = 0; m < k; ++m)
            if (sims[m] == S)
                return fail(SIM_EINVAL, "sims[%d] repeats sims[%d]", k, m);
        if (!S->valid)
            return fail(SIM_EINVAL, "sims[%d] holds no state", k);
        units += S->geo.nunits;
        blocks += S->geo.nblocks;
        ladder = ladder || S->lad.L > 1;
        sc = sc || S->scaled || (S->shortcut & SIM_SC_SKIP);
        for (int k = 0; k < S->lad.L; ++k)
            sc = sc || S->lad.delta[k] < 0.0;
        for (int p = 0; p < passes; ++p) {
            const sim_gate_t *g = &gates[(size_t)p * count + k];
            if (g->kind == 0 && g->pad == 0)
                continue;
            const int rc = check_gate(S, g);
            if (rc)
                return fail(rc, "pass %d, sims[%d]: %s", p, k, std::string(g_err).c_str());
        }
    }
    const unsigned gu = unit_grid_for(units, kMaxBatchGrid);
    const unsigned gb = (unsigned)(blocks < (1u << 20) ? blocks : (1u << 20));
    // the host mirror may still be the source of the previous upload
    HIPCHK(hipEventSynchronize(B->uploaded));
    const size_t poff = slot_prefix_off(B->max_states);
    const size_t stride = (size_t)B->max_states + 1;
    std::vector<uint8_t> key;
    key.reserve(16 + passes);
    auto put = [&key](uint64_t v) {
        for (int i = 0; i < 8; ++i)
            key.push_back((uint8_t)(v >> (8 * i)));
    };
    put((uint64_t)count);
    put((uint64_t)passes);
    put((uint64_t)gu | ((uint64_t)gb << 32));
    put((uint64_t)ladder | ((uint64_t)sc << 1));
    std::vector<uint8_t> mean_of(passes, 0);
    for (int p = 0; p < passes; ++p) {
        uint8_t *slot = B->hslots + (size_t)p * B->slot_bytes;
        PassArgs *args = (PassArgs *)slot;
        uint64_t *pre = (uint64_t *)(slot + poff);
        uint64_t *upre = pre, *bpre = pre + stride, *mpre = pre + 2 * stride,
                 *mbpre = pre + 3 * stride;
        upre[0] = bpre[0] = mpre[0] = mbpre[0] = 0;
        for (int k = 0; k < count; ++k) {
            sim *S = sims[k];
            const sim_gate_t *g = &gates[(size_t)p * count + k];
            const bool on = g->kind != 0;
            const bool mean = on && g->kind == G_DIFFUSE;
            if (on) {
                args[k] = make_args(S, S->cur, 1 - S->cur, to_arg(g));
                S->cur = 1 - S->cur;
                S->passes++;
                if (args[k].sc_skip)
                    S->scaled = true;
            } else {
                GateArg none{};
                args[k] = make_args(S, S->cur, 1 - S->cur, none);
            }
            args[k].chunk_bytes = batch_chunk_bytes(S->arena_cap, gu);
            args[k].scratch = B->scratch;
            args[k].scratch_wgs = 0xFFFFFFFFull;
            args[k].stage_by_slot = 1;
            upre[k + 1] = upre[k] + (on ? S->geo.nunits : 0);
            bpre[k + 1] = bpre[k] + (on ? S->geo.nblocks : 0);
            mpre[k + 1] = mpre[k] + (mean ? S->geo.nunits : 0);
            mbpre[k + 1] = mbpre[k] + (mean ? S->geo.nblocks : 0);
            mean_of[p] = mean_of[p] || mean;
        }
        key.push_back(mean_of[p]);
    }
    // order after the work already queued on each sim's stream
    if (B->sim_ev.size() < (size_t)count) {
        while (B->sim_ev.size() < (size_t)count) {
            hipEvent_t e = nullptr;
            HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
            B->sim_ev.push_back(e);
        }
    }
    for (int k = 0; k < count; ++k) {
        if (sims[k]->stream == B->stream)
            continue;
        HIPCHK(hipEventRecord(B->sim_ev[k], sims[k]->stream));
        HIPCHK(hipStreamWaitEvent(B->stream, B->sim_ev[k], 0));
    }
    HIPCHK(hipMemcpyAsync(B->dslots, B->hslots, (size_t)passes * B->slot_bytes,
                          hipMemcpyHostToDevice, B->stream));
    HIPCHK(hipEventRecord(B->uploaded, B->stream));
    if (use_graph && !B->prof) {
        sim_batch::Graph *G = nullptr;
        for (auto &c : B->graphs)
            if (c.key == key) {
                G = &c;
                break;
            }
        if (!G) {
            if (B->graphs.size() >= kMaxGraphs) {
                destroy_graph(B->graphs.front());
                B->graphs.erase(B->graphs.begin());
            }
            sim_batch::Graph fresh;
            fresh.key = key;
            HIPCHK(hipStreamBeginCapture(B->stream, hipStreamCaptureModeThreadLocal));
            for (int p = 0; p < passes; ++p)
                launch_batch_pass(slot_launch(B, p, (uint32_t)count, gu, gb, mean_of[p] != 0,
                                              ladder, sc),
                                  B->stream, nullptr);
            hipError_t e = hipStreamEndCapture(B->stream, &fresh.g);
            if (e == hipSuccess)
                e = hipGraphInstantiate(&fresh.exec, fresh.g, nullptr, nullptr, 0);
            if (e != hipSuccess) {
                destroy_graph(fresh);
                return fail(SIM_EDEVICE, "graph capture: %s", hipGetErrorString(e));
            }
            B->graphs.push_back(fresh);
            G = &B->graphs.back();
            B->graph_builds++;
        }
        HIPCHK(hipGraphLaunch(G->exec, B->stream));
        B->graph_launches++;
    } else {
        for (int p = 0; p < passes; ++p)
            launch_batch_pass(slot_launch(B, p, (uint32_t)count, gu, gb, mean_of[p] != 0,
                                          ladder, sc),
                              B->stream, B->prof);
        HIPCHK(hipGetLastError());
    }
    // later work on each sim's stream waits for the batch
    HIPCHK(hipEventRecord(B->joined, B->stream));
    for (int k = 0; k < count; ++k)
        if (sims[k]->stream != B->stream)
            HIPCHK(hipStreamWaitEvent(sims[k]->stream, B->joined, 0));
    return SIM_OK;
}

int sim_batch_sync(sim_batch_t *B)
{
    if (!B)
        return fail(SIM_EINVAL, "batch is NULL");
    HIPCHK(hipStreamSynchronize(B->stream));
    return SIM_OK;
}

int sim_batch_profile(sim_batch_t *B, int on)
{
    if (!B)
        return fail(SIM_EINVAL, "batch is NULL");
    return prof_set(B->prof, B->stream, on);
}

int sim_batch_profile_read(sim_batch_t *B, sim_kernel_time_t *out, int cap, int *count)
{
    if (!B)
        return fail(SIM_EINVAL, "batch is NULL");
    return prof_read(B->prof, B->stream, out, cap, count);
}

int sim_batch_info(sim_batch_t *B, uint64_t *graph_builds, uint64_t *graph_launches)
{
    if (!B)
        return fail(SIM_EINVAL, "batch is NULL");
    if (graph_builds)
        *graph_builds = B->graph_builds;
    if (graph_launches)
        *graph_launches = B->graph_launches;
    return SIM_OK;
}

}  // extern "C"
