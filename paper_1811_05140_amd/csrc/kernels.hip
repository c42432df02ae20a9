// kernels.hip -- gfx950 kernels of the compressed path.
//
// One pass of a gate runs Alg. 2 of the paper (decompress, normalise,
// gateComputation, compress at delta_0, delta_1, ... until the ratio reaches
// theta) for every stride, as these kernels on the sim stream:
//   k_pass           per unit of two segments: decode + normalise + gate in
//                    LDS; the size of each plane record at ladder levels
//                    0 .. the block's previous level; encode at that level
//                    (the speculation), write the records, per-segment
//                    normsq.  k_pass<true> takes the units in bulk rounds
//                    (all-zero and one-value units settled one per thread);
//                    k_pass_const adds a one-value fast path per unit for
//                    DIFFUSE and PHASE_FLIP on smaller states
//   k_decide         per block: the first computed level whose ratio reaches
//                    theta; a block whose choice differs from the speculation
//                    joins the replay list, one whose computed levels all
//                    miss theta joins the escalation list
//   k_fix            replayed blocks: encode again at the chosen level;
//                    escalated blocks: size the remaining levels, choose,
//                    encode
//   k_segtree        per block: pairwise normsq from the segment sums
//   k_reduce         N^2 over blocks, s = 1/sqrt(N^2), statistics
// The level chosen is always exactly the one of Alg. 2 (the first level
// whose full-block ratio reaches theta, else the last); speculation only
// decides which records have to be written twice.  DIFFUSE adds a read-only
// mean pre-pass (k_mean + k_segtree + k_mean_final).  Checkpoints: k_export_range
// and the k_import_* kernels.
//
// Work decomposition: a workgroup of four wave64s takes one unit of two
// segments (2 x 2^s amplitudes); wave w decodes / encodes plane (w & 1) of
// segment (w >> 1), one 64-scalar chunk per wave instruction, with DPP row
// and wave operations for prefix sums, neighbours and widths.  The decoded
// unit sits in LDS (32 KiB at s = 10) for the gate butterflies, so four
// workgroups share a CU.  Units are segment pairs (g, g ^ (mask >> s)) when
// a gate couples segments, so every pair update of Sec. II finds both
// amplitudes in LDS.  Plane records are bump-allocated per unit in the
// output arena; a block's canonical stream is its header plus its records
// in plane order.
//
// Arithmetic: every floating-point operation is one IEEE binary64 rounding
// (contraction off), in the order the block-stream format and the gate
// definitions fix, so codes and streams match the CPU reference bit for bit.
#pragma clang fp contract(off)

#include <mutex>

#include "device.h"
#include "gates.h"

namespace aalc {

// ------------------------------------------------------------- helpers ----

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }

// ---- DPP wave primitives (gfx9 DPP: row shifts, row broadcasts, wave shift).
// update_dpp(old, v, ctrl, row_mask, bank_mask, bound_ctrl=false): lanes
// whose source is invalid, or whose row is masked off, receive `old`.
template <int CTRL, int ROWM = 0xF>
__device__ __forceinline__ uint32_t dpp32(uint32_t old, uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_update_dpp((int)old, (int)v, CTRL, ROWM, 0xF, false);
}

template <int CTRL, int ROWM = 0xF>
__device__ __forceinline__ uint64_t dpp64(uint64_t old, uint64_t v)
{
    const uint32_t lo = dpp32<CTRL, ROWM>((uint32_t)old, (uint32_t)v);
    const uint32_t hi = dpp32<CTRL, ROWM>((uint32_t)(old >> 32), (uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}

constexpr int kRowShr1 = 0x111, kRowShr2 = 0x112, kRowShr4 = 0x114, kRowShr8 = 0x118;
constexpr int kRowRor4 = 0x124, kRowRor8 = 0x128;
constexpr int kWaveShr1 = 0x138;
constexpr int kRowBcast15 = 0x142, kRowBcast31 = 0x143;
constexpr int kQuadXor1 = 0xB1;  // quad_perm [1,0,3,2]
constexpr int kQuadXor2 = 0x4E;  // quad_perm [2,3,0,1]

// Inclusive prefix sums over the 64 lanes: row-local Hillis-Steele, then
// row 0 -> row 1 and row 2 -> row 3 (bcast 15), then rows 0-1 -> rows 2-3
// (bcast 31).
__device__ __forceinline__ uint32_t wave_scan32(uint32_t v)
{
    v += dpp32<kRowShr1>(0u, v);
    v += dpp32<kRowShr2>(0u, v);
    v += dpp32<kRowShr4>(0u, v);
    v += dpp32<kRowShr8>(0u, v);
    v += dpp32<kRowBcast15, 0xA>(0u, v);
    v += dpp32<kRowBcast31, 0xC>(0u, v);
    return v;
}

__device__ __forceinline__ uint64_t wave_scan64(uint64_t v)
{
    v += dpp64<kRowShr1>(0ull, v);
    v += dpp64<kRowShr2>(0ull, v);
    v += dpp64<kRowShr4>(0ull, v);
    v += dpp64<kRowShr8>(0ull, v);
    v += dpp64<kRowBcast15, 0xA>(0ull, v);
    v += dpp64<kRowBcast31, 0xC>(0ull, v);
    return v;
}

// Maximum over the 64 lanes, returned as a wave-uniform value.
__device__ __forceinline__ uint32_t wave_max32(uint32_t v)
{
    uint32_t t;
    t = dpp32<kQuadXor1>(0u, v);
    v = v > t ? v : t;
    t = dpp32<kQuadXor2>(0u, v);
    v = v > t ? v : t;
    t = dpp32<kRowRor4>(0u, v);
    v = v > t ? v : t;
    t = dpp32<kRowRor8>(0u, v);
    v = v > t ? v : t;
    t = dpp32<kRowBcast15, 0xA>(0u, v);
    v = v > t ? v : t;
    t = dpp32<kRowBcast31, 0xC>(0u, v);
    v = v > t ? v : t;
    return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}

// Maximum over each row of 16 lanes, held by every lane of the row.
__device__ __forceinline__ uint32_t row_max32(uint32_t v)
{
    uint32_t t;
    t = dpp32<kQuadXor1>(0u, v);
    v = v > t ? v : t;
    t = dpp32<kQuadXor2>(0u, v);
    v = v > t ? v : t;
    t = dpp32<kRowRor4>(0u, v);
    v = v > t ? v : t;
    t = dpp32<kRowRor8>(0u, v);
    v = v > t ? v : t;
    return v;
}

// Inclusive prefix sums within each row of 16 lanes.
__device__ __forceinline__ uint32_t row_scan32(uint32_t v)
{
    v += dpp32<kRowShr1>(0u, v);
    v += dpp32<kRowShr2>(0u, v);
    v += dpp32<kRowShr4>(0u, v);
    v += dpp32<kRowShr8>(0u, v);
    return v;
}

__device__ __forceinline__ uint64_t readlane64(uint64_t v, int l)
{
    uint32_t lo = __builtin_amdgcn_readlane((int)(uint32_t)v, l);
    uint32_t hi = __builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), l);
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint32_t bitlen64(uint64_t z)
{
    return z ? 64u - (uint32_t)__builtin_clzll(z) : 0u;
}

__device__ __forceinline__ uint64_t zigzag64(uint64_t c)
{
    return (c << 1) ^ (uint64_t)((int64_t)c >> 63);
}

// |H| folded to H ^ (H >> 31), H the high word of the 64-bit residual d.
__device__ __forceinline__ uint32_t hi_mag(uint64_t d)
{
    const int32_t H = (int32_t)(uint32_t)(d >> 32);
    return (uint32_t)(H ^ (H >> 31));
}

__device__ __forceinline__ uint64_t unzigzag64(uint64_t z)
{
    return (z >> 1) ^ (0 - (z & 1));
}

__device__ __forceinline__ uint32_t pad8(uint32_t v) { return (v + 7u) & ~7u; }

// Bytes of a plane record from its (payload words, outliers) pair.
__device__ __forceinline__ uint64_t rec_bytes(uint32_t v, uint32_t padC)
{
    uint32_t pw = v & 0xFFFFu, no = v >> 16;
    return kPlaneHdrBytes + (pw ? padC : 0u) + 8ull * pw + (uint64_t)kOutlierBytes * no;
}

// s = 1/sqrt(N^2): one correctly rounded square root, one correctly
// rounded division.
__device__ __forceinline__ double inv_sqrt_exact(double x)
{
    double r = __builtin_sqrt(x);
    return 1.0 / r;
}

// ------------------------------------------------------------ units -------

struct Unit {
    uint64_t g[2];  // segments (g[0] < g[1] when coupled)
    int nsu;        // segments in the unit (1 only when the state has one)
    __device__ __forceinline__ uint64_t seg(int k) const { return k ? g[1] : g[0]; }
};

// The unit holding segment g: {g, g ^ Ms} for coupled segments, else the
// aligned pair {g & ~1, g | 1}.
__device__ __forceinline__ Unit unit_of_seg(uint64_t g, uint64_t nseg, uint64_t Ms)
{
    Unit r;
    if (nseg == 1) {
        r.g[0] = r.g[1] = 0;
        r.nsu = 1;
        return r;
    }
    r.nsu = 2;
    if (Ms) {
        const uint64_t g0 = (g ^ Ms) < g ? (g ^ Ms) : g;
        r.g[0] = g0;
        r.g[1] = g0 ^ Ms;
    } else {
        r.g[0] = g & ~1ull;
        r.g[1] = g | 1ull;
    }
    return r;
}

// The u-th unit of a pass.
__device__ __forceinline__ Unit unit_of(uint64_t u, uint64_t nseg, uint64_t Ms)
{
    if (nseg == 1 || Ms == 0)
        return unit_of_seg(2 * u, nseg, Ms);
    const int hb = 63 - __builtin_clzll(Ms);
    const uint64_t g0 = ((u >> hb) << (hb + 1)) | (u & ((1ull << hb) - 1));
    return unit_of_seg(g0, nseg, Ms);
}

typedef double Planes[2][2][1 << kMaxS];

// LDS position of in-plane scalar o.  Inside each 64-scalar chunk, o =
// 4p + i (lane p of a row, its i-th scalar) is stored at 32 (i >> 1) + 2p +
// (i & 1): the codec's 16-byte accesses of the 16 lanes of a row then sweep
// 256 contiguous bytes (all banks once), instead of a 32-byte lane stride.
__device__ __forceinline__ uint32_t sw(uint32_t o)
{
    return (o & ~63u) | ((o & 2u) << 4) | ((o >> 1) & 0x1Eu) | (o & 1u);
}

// In-plane scalar stored at LDS position pos (inverse of sw).
__device__ __forceinline__ uint32_t unsw(uint32_t pos)
{
    return (pos & ~63u) | (((pos >> 1) & 15u) << 2) | (((pos >> 5) & 1u) << 1) | (pos & 1u);
}

// sw is a permutation of the index bits (bit 0 stays, bit 1 -> 5, bits 2..5
// -> 1..4, higher bits stay), so it maps an xor mask to an xor mask and bit k
// of o to bit sw_bit(k) of the position.
__device__ __forceinline__ int sw_bit(int k)
{
    return k == 0 ? 0 : (k == 1 ? 5 : (k < 6 ? k - 1 : k));
}

// ---- codec layout: a wavefront works on four chunks at a time, row r
// (lanes 16r .. 16r+15) on chunk 4t + r in step t, lane p of the row on the
// four consecutive scalars 4p .. 4p+3 of that chunk.  Chunk widths are row
// maxima, prefix sums run in-lane then over rows, and the neighbour of a
// lane's first scalar is the previous lane's last one (wave shift by one).

// Field of width w (<= 32) at bit b of a little-endian dword stream.
__device__ __forceinline__ uint32_t field32(const uint32_t *P, uint32_t b, uint32_t w)
{
    const uint32_t k = b >> 5, sh = b & 31u;
    const uint32_t v = __builtin_amdgcn_alignbit(P[k + 1], P[k], sh);
    return w >= 32u ? v : (v & ((1u << w) - 1u));
}

// Field of width w (<= 64) at bit b (branch-free, so that a lane's four
// field loads can be issued together).
__device__ __forceinline__ uint64_t field64(const uint32_t *P, uint32_t b, uint32_t w)
{
    const uint32_t k = b >> 5, sh = b & 31u;
    const uint32_t d0 = P[k], d1 = P[k + 1], d2 = P[k + 2];
    const uint32_t lo = __builtin_amdgcn_alignbit(d1, d0, sh);
    const uint32_t hi = __builtin_amdgcn_alignbit(d2, d1, sh);
    const uint64_t v = ((uint64_t)hi << 32) | lo;
    return w >= 64u ? v : (v & ((1ull << w) - 1ull));
}

// ---- pointwise-relative levels: a ladder entry delta < 0 is the relative
// bound eps = -delta.  A value x != 0 is coded through log2|x| quantised in
// steps eL = 2 fl(1.4 eps) (a log-domain error below fl(1.4 eps) keeps the
// relative error below eps), code c = 2 (q + 2^28) + sign; c = 0 is +0.
// Every stored value is checked, |x - xhat| < eps |x|, else an outlier.  The
// log and the power of two are this codec's own, from IEEE additions,
// multiplications and one division in a fixed order, so that every device
// and the CPU reference give the same bits.
constexpr double kRelOff = 268435456.0;    // 2^28
constexpr double kRelRange = 268435455.0;  // |y| < 2^28 - 1: codes <= 2^30 - 1

// log2 a for finite a > 0: a = m 2^k with m in [sqrt(1/2), sqrt(2)), then
// ln m = 2 atanh t, t = (m - 1)/(m + 1), by its odd series up to t^15.
__device__ double codec_log2(double a)
{
    uint64_t bits = (uint64_t)__double_as_longlong(a);
    int e = (int)((bits >> 52) & 0x7FFu);
    if (e == 0) {  // subnormal: scale by 2^54 first (exact)
        bits = (uint64_t)__double_as_longlong(a * 0x1p54);
        e = (int)((bits >> 52) & 0x7FFu) - 54;
    }
    double m = __longlong_as_double(
        (long long)((bits & 0x000FFFFFFFFFFFFFull) | 0x3FF0000000000000ull));
    int k = e - 1023;
    if (m > 0x1.6a09e667f3bcdp+0) {  // sqrt 2
        m = m * 0.5;
        k = k + 1;
    }
    const double t = (m - 1.0) / (m + 1.0);
    const double t2 = t * t;
    double p = 0x1.1111111111111p-4;  // 1/15
    p = p * t2 + 0x1.3b13b13b13b14p-4;  // 1/13
    p = p * t2 + 0x1.745d1745d1746p-4;  // 1/11
    p = p * t2 + 0x1.c71c71c71c71cp-4;  // 1/9
    p = p * t2 + 0x1.2492492492492p-3;  // 1/7
    p = p * t2 + 0x1.999999999999ap-3;  // 1/5
    p = p * t2 + 0x1.5555555555555p-2;  // 1/3
    p = p * t2 + 1.0;
    const double lnm = (2.0 * t) * p;
    return (double)k + lnm * 0x1.71547652b82fep+0;  // 1/ln 2
}

// 2^y for finite y: y = k + f with f in [-1/2, 1/2]; 2^f = e^(f ln 2) by its
// Taylor series up to the 13th power; then times 2^k (exact, or one rounding
// into the subnormals).
__device__ double codec_exp2(double y)
{
    double k = __builtin_floor(y);
    double f = y - k;
    if (f > 0.5) {
        f = f - 1.0;
        k = k + 1.0;
    }
    const double z = f * 0x1.62e42fefa39efp-1;  // ln 2
    double p = 0x1.6124613a86d09p-33;          // 1/13!
    p = p * z + 0x1.1eed8eff8d898p-29;         // 1/12!
    p = p * z + 0x1.ae64567f544e4p-26;         // 1/11!
    p = p * z + 0x1.27e4fb7789f5cp-22;         // 1/10!
    p = p * z + 0x1.71de3a556c734p-19;         // 1/9!
    p = p * z + 0x1.a01a01a01a01ap-16;         // 1/8!
    p = p * z + 0x1.a01a01a01a01ap-13;         // 1/7!
    p = p * z + 0x1.6c16c16c16c17p-10;         // 1/6!
    p = p * z + 0x1.1111111111111p-7;          // 1/5!
    p = p * z + 0x1.5555555555555p-5;          // 1/4!
    p = p * z + 0x1.5555555555555p-3;          // 1/3!
    p = p * z + 0.5;
    p = p * z + 1.0;
    p = p * z + 1.0;
    if (k > 1023.0)
        return __longlong_as_double(0x7FF0000000000000ll);  // +inf
    if (k < -1022.0) {
        if (k < -1100.0)
            return 0.0;
        const double two = __longlong_as_double((long long)((uint64_t)((int)k + 600 + 1023) << 52));
        return (p * two) * 0x1p-600;
    }
    return p * __longlong_as_double((long long)((uint64_t)((int)k + 1023) << 52));
}

// Step between consecutive codes of a lossy level: 2 delta (absolute), or
// eL = 2 fl(1.4 eps) in the log domain (relative, delta = -eps).
__device__ __forceinline__ double level_step(double delta)
{
    if (delta > 0.0)
        return 2.0 * delta;
    const double dl = 1.4 * -delta;
    return 2.0 * dl;
}

// Value of relative-level code c with log step eL.
__device__ __forceinline__ double rel_value(int32_t c, double eL)
{
    const double qv = (double)((c >> 1) - (int32_t)kRelOff);
    const double mag = codec_exp2(qv * eL);
    return c == 0 ? 0.0 : ((c & 1) ? -mag : mag);
}

// Value of code c at a lossy level (e = level_step(delta)).
__device__ __forceinline__ double dequant(int32_t c, double delta, double e)
{
    return delta > 0.0 ? (double)c * e : rel_value(c, e);
}

// Decode one plane record into dst[0 .. 2^s) (one wavefront; dst is the
// wave's own LDS plane region), scaling each value by `scale` when do_scale
// (normalisation before the gate).  Lossy planes run the prefix sums in 32
// bits: a partial sum is the difference of two codes of magnitude at most
// 2^30 - 1, so it is exact.
// The payload is first copied into the top of dst (words 2^s - pw .. 2^s),
// every load in flight at once, together with the widths and the first 64
// outliers; the fields are then read from LDS.  A chunk's payload is at most
// 64 words and its decoded values exactly 64, so the values written in steps
// 0..t end below the payload of every chunk of a later step.
// REL: the instance that also decodes relative levels (the pass kernels
// without it are kept free of that code's registers).
template <bool REL = true>
__device__ uint32_t decode_plane(const uint8_t *rec, int s, double delta,
                                 double scale, bool do_scale, double *dst)
{
    const int lane = lane_id();
    const int r = lane >> 4, p = lane & 15;
    const int C = 1 << (s - 6);
    const int steps = (C + 3) >> 2;
    const uint64_t anchor = *(const uint64_t *)rec;
    const uint32_t pw = *(const uint32_t *)(rec + 8);
    const uint32_t nout = *(const uint32_t *)(rec + 12);
    const uint8_t *widths = rec + kPlaneHdrBytes;
    const uint2 *gpay = (const uint2 *)(rec + kPlaneHdrBytes + (pw ? pad8((uint32_t)C) : 0u));
    const uint8_t *outl = (const uint8_t *)(gpay + pw);
    // width byte of chunk `lane` (branch-free: without widths the load reads
    // the header and the value is dropped)
    const uint32_t wdw = *((const uint32_t *)(pw ? widths : rec) + ((lane >> 2) & 3));
    const bool o0 = (uint32_t)lane < nout;
    uint32_t oidx = 0;
    uint64_t obits = 0;
    if (o0) {
        oidx = *(const uint32_t *)(outl + (uint64_t)kOutlierBytes * lane);
        obits = *(const uint64_t *)(outl + (uint64_t)kOutlierBytes * lane + 8);
    }
    uint32_t *payload = (uint32_t *)dst + 2 * ((1u << s) - pw);
    // the first 256 words outside the loop, so that their loads go out with
    // the ones above
    {
        uint2 v[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const uint32_t k = (uint32_t)lane + 64u * (uint32_t)i;
            v[i] = k < pw ? gpay[k] : make_uint2(0u, 0u);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const uint32_t k = (uint32_t)lane + 64u * (uint32_t)i;
            if (k < pw) {
                payload[2 * k] = v[i].x;
                payload[2 * k + 1] = v[i].y;
            }
        }
    }
    for (uint32_t k0 = 256u; k0 < pw; k0 += 256u) {
        uint2 v[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const uint32_t k = k0 + (uint32_t)lane + 64u * (uint32_t)i;
            v[i] = k < pw ? gpay[k] : make_uint2(0u, 0u);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const uint32_t k = k0 + (uint32_t)lane + 64u * (uint32_t)i;
            if (k < pw) {
                payload[2 * k] = v[i].x;
                payload[2 * k + 1] = v[i].y;
            }
        }
    }
    const uint32_t wraw = (pw && lane < C) ? ((wdw >> (8 * (lane & 3))) & 0xFFu) : 0u;
    // chunk widths (lanes 0..C-1) and their exclusive prefix (payload word
    // offsets); lanes 0..15 of row 0 hold chunks 0..15
    const uint32_t wl = wraw;
    const uint32_t ol = row_scan32(wl) - wl;
    const double e = delta != 0.0 ? level_step(delta) : 0.0;
    uint64_t carry = anchor;
    for (int t = 0; t < steps; ++t) {
        const int c = 4 * t + r;
        const bool active = c < C;
        const int cs = active ? c : 0;
        const uint32_t w = active ? (uint32_t)__shfl((int)wl, cs, 64) : 0u;
        const uint32_t woff = (uint32_t)__shfl((int)ol, cs, 64);
        const uint32_t *P = payload + 2 * woff;
        const uint32_t b0 = (uint32_t)(4 * p) * w;
        double x[4];
        if (delta == 0.0) {
            // one branch around all four fields, so their loads are in flight together
            uint64_t d[4] = {0ull, 0ull, 0ull, 0ull};
            if (w) {
                uint64_t f[4];
                uint32_t bi = b0;
#pragma unroll
                for (int i = 0; i < 4; ++i, bi += w)
                    f[i] = field64(P, bi, w);
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    d[i] = unzigzag64(f[i]);
            }
            const uint64_t s1 = d[0] + d[1], s2 = s1 + d[2], s3 = s2 + d[3];
            const uint64_t incl = wave_scan64(s3);
            const uint64_t base = carry + (incl - s3);
            const uint64_t q0 = base + d[0], q1 = base + s1, q2 = base + s2, q3 = base + s3;
            carry = carry + readlane64(incl, 63);
            x[0] = __longlong_as_double((long long)q0);
            x[1] = __longlong_as_double((long long)q1);
            x[2] = __longlong_as_double((long long)q2);
            x[3] = __longlong_as_double((long long)q3);
        } else {
            uint32_t d[4] = {0u, 0u, 0u, 0u};
            if (w) {
                uint32_t z[4];
                uint32_t bi = b0;
#pragma unroll
                for (int i = 0; i < 4; ++i, bi += w)
                    z[i] = field32(P, bi, w);
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    d[i] = (z[i] >> 1) ^ (0u - (z[i] & 1u));
            }
            const uint32_t s1 = d[0] + d[1], s2 = s1 + d[2], s3 = s2 + d[3];
            const uint32_t incl = wave_scan32(s3);
            const uint32_t ex = incl - s3;
            const int32_t c32 = (int32_t)(uint32_t)carry;
            const int32_t q0 = c32 + (int32_t)(ex + d[0]), q1 = c32 + (int32_t)(ex + s1);
            const int32_t q2 = c32 + (int32_t)(ex + s2), q3 = c32 + (int32_t)(ex + s3);
            if (!REL || delta > 0.0) {
                x[0] = (double)q0 * e;
                x[1] = (double)q1 * e;
                x[2] = (double)q2 * e;
                x[3] = (double)q3 * e;
            } else {
                x[0] = rel_value(q0, e);
                x[1] = rel_value(q1, e);
                x[2] = rel_value(q2, e);
                x[3] = rel_value(q3, e);
            }
            carry = (uint64_t)(int64_t)(c32 + (int32_t)__builtin_amdgcn_readlane((int)incl, 63));
        }
        if (active) {
#pragma unroll
            for (int i = 0; i < 4; ++i)
                x[i] = do_scale ? x[i] * scale : x[i];
            double2 *pa = (double2 *)(dst + c * kChunk + 2 * p);
            pa[0] = make_double2(x[0], x[1]);
            pa[16] = make_double2(x[2], x[3]);
        }
    }
    if (o0) {
        double v = __longlong_as_double((long long)obits);
        if (do_scale)
            v = v * scale;
        dst[sw(oidx)] = v;
    }
    for (uint32_t k = 64u + (uint32_t)lane; k < nout; k += 64u) {
        const uint32_t idx = *(const uint32_t *)(outl + (uint64_t)kOutlierBytes * k);
        double v = *(const double *)(outl + (uint64_t)kOutlierBytes * k + 8);
        if (do_scale)
            v = v * scale;
        dst[sw(idx)] = v;
    }
    // whether some chunk of the plane has width 0 (a flat run of equal
    // codes, such as zeros): only then can the codec's step skips apply
    return __ballot(wraw == 0u && (uint32_t)lane < (uint32_t)C) != 0ull ? 1u : 0u;
}

// Decode (or synthesise, for the basis-state source) the planes of a unit
// into LDS; wave w owns plane (w & 1) of segment (w >> 1).  normalise: each
// value times its block's factor fl(c_j s) (the deferred scale c_j of the
// skip shortcut, 1 otherwise), else the stored x-hat as it is.
__device__ void load_unit(const PassArgs &a, const Unit &uc, Planes &X,
                          double scale, bool normalise)
{
    const int wave = threadIdx.x >> 6, lane = lane_id();
    const int us = wave >> 1, p = wave & 1;
    const int s = a.geo.s;
    if (us >= uc.nsu)
        return;
    const uint64_t g = uc.seg(us);
    double *dst = &X[us][p][0];
    if (a.src_basis) {
        for (int o = lane; o < (1 << s); o += 64)
            dst[sw(o)] = (p == 0 && ((g << s) | (uint64_t)o) == a.basis) ? 1.0 : 0.0;
        return;
    }
    const uint64_t j = g >> (a.geo.b - s);
    const double delta = *(const double *)(a.din.hdr + 32 * j + 16);
    const double fac = normalise ? a.din.bscale[j] * scale : 1.0;
    decode_plane(a.arena_in + rec_at(a.din, 2 * g + p), s, delta, fac, fac != 1.0, dst);
}

__device__ void gate_unit(const GateArg &G, const Unit &uc, int s, Planes &X,
                          const double *tdiff)
{
    // Loops run over LDS positions (consecutive lanes on consecutive
    // positions, conflict-free); the amplitude index of a position comes
    // from unsw, and a pair partner is an xor in position space too.
    const int tid = threadIdx.x;
    if (G.kind == kNone)
        return;
    const uint64_t M = G.mask;
    const uint64_t Ms = M >> s;
    const uint32_t S = 1u << s;
    const uint32_t Ml = (uint32_t)(M & (S - 1));
    const uint32_t Pl = sw(Ml);
    if (M == 0) {
        const uint32_t total = (uint32_t)uc.nsu << s;
        for (uint32_t t = tid; t < total; t += kWG) {
            const int us = (int)(t >> s);
            const uint32_t pos = t & (S - 1);
            const uint64_t i = (uc.seg(us) << s) | unsw(pos);
            double ar = X[us][0][pos], ai = X[us][1][pos];
            gate_diag(G, i, ar, ai, tdiff);
            X[us][0][pos] = ar;
            X[us][1][pos] = ai;
        }
    } else if (Ms) {
        for (uint32_t pos = tid; pos < S; pos += kWG) {
            const uint32_t pos2 = pos ^ Pl;
            const uint64_t i = (uc.g[0] << s) | unsw(pos);
            double ar = X[0][0][pos], ai = X[0][1][pos];
            double br = X[1][0][pos2], bi = X[1][1][pos2];
            gate_pair(G, i, ar, ai, br, bi);
            X[0][0][pos] = ar;
            X[0][1][pos] = ai;
            X[1][0][pos2] = br;
            X[1][1][pos2] = bi;
        }
    } else {
        // pairs (o, o ^ Ml) with bit hb of o clear: in positions, bit pb clear
        const int hb = 31 - __builtin_clz(Ml);
        const int pb = sw_bit(hb);
        const uint32_t half = S >> 1;
        const uint32_t total = (uint32_t)uc.nsu * half;
        for (uint32_t t = tid; t < total; t += kWG) {
            const int us = (int)(t >> (s - 1));
            const uint32_t r = t & (half - 1);
            const uint32_t pos = ((r >> pb) << (pb + 1)) | (r & ((1u << pb) - 1));
            const uint32_t pos2 = pos ^ Pl;
            const uint64_t i = (uc.seg(us) << s) | unsw(pos);
            double ar = X[us][0][pos], ai = X[us][1][pos];
            double br = X[us][0][pos2], bi = X[us][1][pos2];
            gate_pair(G, i, ar, ai, br, bi);
            X[us][0][pos] = ar;
            X[us][1][pos] = ai;
            X[us][0][pos2] = br;
            X[us][1][pos2] = bi;
        }
    }
}

// Lossy code of one scalar at one level: q the int32 code, `out` the outlier
// flag, xh the value a decoder reconstructs (the scalar itself for outliers).
// Code of x at a relative level (delta = -eps, eL = e, rL = r): code 0 for
// +-0 (decoded +0, never an outlier); non-finite values and log codes out of
// range become code 0 and outliers; otherwise an outlier iff the decoded
// value misses |x - xhat| < eps |x| (q is kept in the predictor).
__device__ __forceinline__ void rel_code(double x, double eps, double eL, double rL,
                                         int32_t &q, bool &out, double &xh)
{
    const double a = fabs(x);
    const bool zero = a == 0.0;
    const bool fin = a < __longlong_as_double(0x7FF0000000000000ll);  // false for inf, NaN
    const double y = codec_log2(fin && !zero ? a : 1.0) * rL;
    const bool in = fin && !zero && fabs(y) < kRelRange;
    const double qr = in ? __builtin_rint(y) : 0.0;
    const int32_t c = in ? 2 * ((int32_t)qr + (int32_t)kRelOff) + (x < 0.0 ? 1 : 0) : 0;
    const double mag = codec_exp2(in ? qr * eL : 0.0);
    const double v = in ? (x < 0.0 ? -mag : mag) : 0.0;
    out = !zero && (!in || !(fabs(x - v) < eps * a));
    q = c;
    xh = out ? x : v;
}

template <bool REL = true>
__device__ __forceinline__ void lossy_code(double x, double delta, double e, double r,
                                           int32_t &q, bool &out, double &xh)
{
    if (REL && delta < 0.0) {
        rel_code(x, -delta, e, r, q, out, xh);
        return;
    }
    // branch-free: a code out of range (or NaN) becomes 0 and an outlier
    const double y = x * r;
    const bool in = fabs(y) < kQMax;
    const double qr = in ? __builtin_rint(y) : 0.0;
    q = (int32_t)qr;
    const double xq = qr * e;
    out = !in || !(fabs(x - xq) < delta);
    xh = out ? x : xq;
}

__device__ __forceinline__ uint32_t zigzag32(int32_t d)
{
    return ((uint32_t)d << 1) ^ (uint32_t)(d >> 31);
}

__device__ __forceinline__ uint32_t bitlen32(uint32_t z)
{
    return z ? 32u - (uint32_t)__builtin_clz(z) : 0u;
}

// Step t's chunk widths (row r holds chunk 4t + r) into lanes 4t .. 4t+3.
__device__ __forceinline__ void gather_widths(uint32_t w, int t, uint32_t &wl)
{
    const int lane = lane_id();
    const uint32_t w0 = (uint32_t)__builtin_amdgcn_readlane((int)w, 0);
    const uint32_t w1 = (uint32_t)__builtin_amdgcn_readlane((int)w, 16);
    const uint32_t w2 = (uint32_t)__builtin_amdgcn_readlane((int)w, 32);
    const uint32_t w3 = (uint32_t)__builtin_amdgcn_readlane((int)w, 48);
    const uint32_t d = (uint32_t)(lane - 4 * t);
    const uint32_t ws = d == 0u ? w0 : (d == 1u ? w1 : (d == 2u ? w2 : w3));
    wl = d < 4u ? ws : wl;
}

// What the codec may skip in one plane, by step t (four chunks, row r on
// chunk 4t + r): key[t] bounds the largest |x| of the step from above (the
// high word of |x|, plus one when the low word is not zero, capped at the
// high word of +inf, so NaN and inf never look small) and bit t of zpos says
// that every value of the step is +0.  At a lossy level with bound delta a
// step whose values all have |x| < delta quantises to codes 0 with no
// outliers (|fl(x r)| <= 1/2, and |x - 0| < delta); at the lossless level a
// step of +0 has codes 0.  When the code before the step is 0 as well, every
// residual of the step is 0, so all four chunk widths are 0: the step adds
// nothing to the size and nothing to the payload.
struct StepSum {
    uint32_t k0, k1, k2, k3;
    uint32_t zpos;
};

__device__ StepSum step_summary(const double *x, int s)
{
    const int lane = lane_id();
    const int r = lane >> 4, p = lane & 15;
    const int C = 1 << (s - 6);
    const int steps = (C + 3) >> 2;
    StepSum q = {0x7FF00000u, 0x7FF00000u, 0x7FF00000u, 0x7FF00000u, 0u};
    for (int t = 0; t < steps; ++t) {
        const int c = 4 * t + r;
        const bool active = c < C;
        const double2 *pa = (const double2 *)(x + (active ? c : 0) * kChunk + 2 * p);
        const double2 v01 = pa[0], v23 = pa[16];
        const uint64_t b[4] = {(uint64_t)__double_as_longlong(v01.x),
                               (uint64_t)__double_as_longlong(v01.y),
                               (uint64_t)__double_as_longlong(v23.x),
                               (uint64_t)__double_as_longlong(v23.y)};
        uint32_t key = 0, any = 0;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const uint32_t lo = (uint32_t)b[i], hi = (uint32_t)(b[i] >> 32);
            const uint32_t ha = hi & 0x7FFFFFFFu;
            uint32_t kv = ha + (lo != 0u ? 1u : 0u);
            kv = ha >= 0x7FF00000u ? 0x7FF00000u : kv;
            key = kv > key ? kv : key;
            any |= lo | hi;
        }
        key = active ? key : 0u;
        any = active ? any : 0u;
        const uint32_t km = wave_max32(key);
        const bool zero = __ballot(any != 0u) == 0ull;
        if (t == 0)
            q.k0 = km;
        else if (t == 1)
            q.k1 = km;
        else if (t == 2)
            q.k2 = km;
        else
            q.k3 = km;
        q.zpos |= zero ? (1u << t) : 0u;
    }
    return q;
}

// Steps (bit t) whose four chunks have width 0 at a level with bound delta
// whenever the code before the step is 0: at a lossy level those whose
// values all lie below delta in magnitude, at the lossless level those of
// +0 only.
__device__ __forceinline__ uint32_t size_skip_mask(const StepSum &q, double delta)
{
    if (delta == 0.0)
        return q.zpos;
    if (delta < 0.0)  // relative: only +-0 has code 0
        return (q.k0 == 0u ? 1u : 0u) | (q.k1 == 0u ? 2u : 0u) | (q.k2 == 0u ? 4u : 0u) |
               (q.k3 == 0u ? 8u : 0u);
    const double d = delta;
    return (__hiloint2double((int)q.k0, 0) < d ? 1u : 0u) |
           (__hiloint2double((int)q.k1, 0) < d ? 2u : 0u) |
           (__hiloint2double((int)q.k2, 0) < d ? 4u : 0u) |
           (__hiloint2double((int)q.k3, 0) < d ? 8u : 0u);
}

// Steps the encoder may skip: besides width 0, every value must already be
// its own x-hat, which holds for +-0 at a lossy level (codes 0, x-hat of the
// same sign) and for +0 at the lossless level.
__device__ __forceinline__ uint32_t pack_skip_mask(const StepSum &q, double delta)
{
    if (delta == 0.0)
        return q.zpos;
    return (q.k0 == 0u ? 1u : 0u) | (q.k1 == 0u ? 2u : 0u) | (q.k2 == 0u ? 4u : 0u) |
           (q.k3 == 0u ? 8u : 0u);
}

// Sizes of one plane at ladder levels k0 .. k1 (one wavefront; levels outer
// so that only one level's state is live).  Returns the (payload words,
// outliers) word of level `want` when it lies in the range; lane c (< 16)
// of `wl` then holds that level's width of chunk c.
template <bool REL>
__device__ uint32_t size_levels(const double *x, int s, const Ladder &lad, int k0, int k1,
                                int want, uint32_t *psz, uint64_t plane, uint64_t nplanes,
                                uint32_t &wl, const StepSum &sum)
{
    const int lane = lane_id();
    const int r = lane >> 4, p = lane & 15;
    const int C = 1 << (s - 6);
    const int steps = (C + 3) >> 2;
    uint32_t wanted = 0;
    wl = 0;
    for (int k = k0; k <= k1; ++k) {
        const double delta = lad.delta[k];
        const uint32_t skip = size_skip_mask(sum, delta);
        uint32_t pw_acc = 0, no_acc = 0;
        if (delta == 0.0) {
            uint64_t carry = 0;
            for (int t = 0; t < steps; ++t) {
                if (((skip >> t) & 1u) && carry == 0ull)
                    continue;  // codes 0 after a code 0: widths 0 (carry stays 0)
                const int c = 4 * t + r;
                const bool active = c < C;
                const double2 *pa = (const double2 *)(x + (active ? c : 0) * kChunk + 2 * p);
                const double2 v01 = pa[0], v23 = pa[16];
                const uint64_t q0 = (uint64_t)__double_as_longlong(v01.x);
                const uint64_t q1 = (uint64_t)__double_as_longlong(v01.y);
                const uint64_t q2 = (uint64_t)__double_as_longlong(v23.x);
                const uint64_t q3 = (uint64_t)__double_as_longlong(v23.y);
                const uint64_t prev = dpp64<kWaveShr1>(t == 0 ? q0 : carry, q3);
                // A residual d whose high word H is not 0 or -1 has zigzag
                // width 33 + bitlen(H ^ (H >> 31)), every other one at most
                // 33: a row with such a residual has that width from the
                // high words alone; rows without one take the full widths.
                const uint32_t oh = hi_mag(q0 - prev) | hi_mag(q1 - q0) | hi_mag(q2 - q1) |
                                    hi_mag(q3 - q2);
                uint32_t w = row_max32(active && oh ? 33u + bitlen32(oh) : 0u);
                if (__ballot(active && w == 0u)) {
                    const uint64_t o = zigzag64(q0 - prev) | zigzag64(q1 - q0) |
                                       zigzag64(q2 - q1) | zigzag64(q3 - q2);
                    const uint32_t we = row_max32(active ? bitlen64(o) : 0u);
                    w = w ? w : we;
                }
                pw_acc += w;
                if (k == want)
                    gather_widths(w, t, wl);
                carry = readlane64(q3, 63);
            }
        } else {
            const double e = lad.e[k], rr = lad.r[k];
            int32_t carry = 0;
            for (int t = 0; t < steps; ++t) {
                if (((skip >> t) & 1u) && carry == 0)
                    continue;  // codes 0 after a code 0: widths 0, no outliers
                const int c = 4 * t + r;
                const bool active = c < C;
                const double2 *pa = (const double2 *)(x + (active ? c : 0) * kChunk + 2 * p);
                const double2 v01 = pa[0], v23 = pa[16];
                const double xs[4] = {v01.x, v01.y, v23.x, v23.y};
                int32_t q[4];
                bool out[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    double xh;
                    lossy_code<REL>(xs[i], delta, e, rr, q[i], out[i], xh);
                }
                const int32_t prev = (int32_t)dpp32<kWaveShr1>(
                    (uint32_t)(t == 0 ? q[0] : carry), (uint32_t)q[3]);
                const uint32_t o = zigzag32(q[0] - prev) | zigzag32(q[1] - q[0]) |
                                   zigzag32(q[2] - q[1]) | zigzag32(q[3] - q[2]);
                const uint32_t w = row_max32(active ? bitlen32(o) : 0u);
                pw_acc += w;
                if (active)
                    no_acc += (uint32_t)out[0] + (uint32_t)out[1] + (uint32_t)out[2] +
                              (uint32_t)out[3];
                if (k == want)
                    gather_widths(w, t, wl);
                carry = __builtin_amdgcn_readlane(q[3], 63);
            }
        }
        const uint32_t pw = (uint32_t)__builtin_amdgcn_readlane((int)pw_acc, 0) +
                            (uint32_t)__builtin_amdgcn_readlane((int)pw_acc, 16) +
                            (uint32_t)__builtin_amdgcn_readlane((int)pw_acc, 32) +
                            (uint32_t)__builtin_amdgcn_readlane((int)pw_acc, 48);
        const uint32_t no = (uint32_t)__builtin_amdgcn_readlane((int)wave_scan32(no_acc), 63);
        const uint32_t v = pw | (no << 16);
        if (lane == 0)
            psz[(uint64_t)k * nplanes + plane] = v;
        if (k == want)
            wanted = v;
    }
    return wanted;
}

// Dwords of one row of the packing buffer: a chunk of width w < 64 fills
// bits below 64 w, so dwords 0 .. 2 w - 1 <= 125.
constexpr int kPackRow = 126;

// OR `v` into the dword stream of LDS buffer pb at bit b (v < 2^32 >> 0;
// the bits above 32 - (b & 31) spill into the next dword).
__device__ __forceinline__ void or_bits32(uint32_t *pb, uint32_t b, uint32_t v)
{
    // branch-free: ORing 0 is harmless and cheaper than masking lanes off.
    // A spill into dword 126 is never non-zero (a chunk's bits end below
    // 64 * 63), so that index is clamped into the row.
    const uint32_t k = b >> 5, sh = b & 31u;
    atomicOr(&pb[k], v << sh);
    atomicOr(&pb[min(k + 1u, (uint32_t)kPackRow - 1u)], (uint32_t)(((uint64_t)v << sh) >> 32));
}

// Encode one plane at one level into its record (one wavefront).  Lane c
// (< 16) of wreg holds the level's width of chunk c from the sizing sweep.
// x is overwritten with the decoded values x-hat for the normsq.  pb is the
// wave's LDS packing buffer (4 rows of kPackRow dwords, zero on entry and on
// exit).
// The encode level in one pass over the plane: the chunk widths and outlier
// count (as size_levels computes them) and, step by step, each chunk's
// fields packed through the row's LDS buffer into this wave's staging
// payload at their final payload offsets (known as the widths accumulate),
// the first kScratchOutl outliers into the staging list, and x-hat written
// back over x.  Returns payload words | outliers << 16 (also stored to
// *psz_slot); wl = width of chunk `lane`; anchor = the plane's first code.
template <bool REL>
__device__ uint32_t size_pack_level(double *x, int s, double delta, double e, double r,
                                    uint32_t *psz_slot, uint8_t *stage, uint32_t *pb,
                                    uint32_t &wl, uint64_t &anchor, const StepSum &sum)
{
    const int lane = lane_id();
    const int row = lane >> 4, p = lane & 15;
    const int C = 1 << (s - 6);
    const int steps = (C + 3) >> 2;
    uint32_t *spay = (uint32_t *)stage;
    uint8_t *sout = stage + kScratchPayload;
    uint32_t *prow = pb + kPackRow * row;
    uint32_t base_w = 0, nout = 0;
    uint64_t carry = 0;
    wl = 0;
    anchor = 0;
    // payload word offset of this row's chunk; advances base_w, records widths
    auto place = [&](uint32_t w, int t) -> uint32_t {
        const uint32_t w0 = (uint32_t)__builtin_amdgcn_readlane((int)w, 0);
        const uint32_t w1 = (uint32_t)__builtin_amdgcn_readlane((int)w, 16);
        const uint32_t w2 = (uint32_t)__builtin_amdgcn_readlane((int)w, 32);
        const uint32_t w3 = (uint32_t)__builtin_amdgcn_readlane((int)w, 48);
        const uint32_t woff =
            base_w + (row > 0 ? w0 : 0u) + (row > 1 ? w1 : 0u) + (row > 2 ? w2 : 0u);
        base_w += w0 + w1 + w2 + w3;
        const uint32_t d = (uint32_t)(lane - 4 * t);
        const uint32_t ws = d == 0u ? w0 : (d == 1u ? w1 : (d == 2u ? w2 : w3));
        wl = d < 4u ? ws : wl;
        return woff;
    };
    const uint32_t skip = pack_skip_mask(sum, delta);
    for (int t = 0; t < steps; ++t) {
        // a step of codes 0 after a code 0: widths 0, no outliers, nothing
        // to pack, x-hat = x (anchor and carry stay 0)
        if (((skip >> t) & 1u) && carry == 0ull)
            continue;
        const int c = 4 * t + row;
        const bool active = c < C;
        const int cs = active ? c : 0;
        double2 *pa = (double2 *)(x + cs * kChunk + 2 * p);
        uint32_t w, woff;
        if (delta == 0.0) {
            uint64_t q[4];
            {
                const double2 v01 = pa[0], v23 = pa[16];
                q[0] = (uint64_t)__double_as_longlong(v01.x);
                q[1] = (uint64_t)__double_as_longlong(v01.y);
                q[2] = (uint64_t)__double_as_longlong(v23.x);
                q[3] = (uint64_t)__double_as_longlong(v23.y);
            }
            const uint64_t prev = dpp64<kWaveShr1>(t == 0 ? q[0] : carry, q[3]);
            if (t == 0)
                anchor = readlane64(q[0], 0);
            carry = readlane64(q[3], 63);
            uint64_t z[4];
            z[0] = zigzag64(q[0] - prev);
            z[1] = zigzag64(q[1] - q[0]);
            z[2] = zigzag64(q[2] - q[1]);
            z[3] = zigzag64(q[3] - q[2]);
            w = row_max32(active ? bitlen64(z[0] | z[1] | z[2] | z[3]) : 0u);
            woff = place(w, t);
            const uint32_t b0 = (uint32_t)(4 * p) * w;
            if (active && w == 64u) {
                uint64_t *dst = (uint64_t *)(spay + 2 * woff) + 4 * p;
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    dst[i] = z[i];
            } else if (active && w) {
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const uint32_t bi = b0 + (uint32_t)i * w;
                    const uint32_t sh = bi & 31u;
                    const uint32_t lo = (uint32_t)z[i], hi = (uint32_t)(z[i] >> 32);
                    or_bits32(prow, bi, lo);
                    if (hi) {
                        const uint32_t k = (bi >> 5) + 1;
                        atomicOr(&prow[k], hi << sh);
                        if (sh && (hi >> (32u - sh)))
                            atomicOr(&prow[k + 1], hi >> (32u - sh));
                    }
                }
            }
        } else {
            int32_t q[4];
            bool out[4];
            double xs[4], xh[4];
            {
                const double2 v01 = pa[0], v23 = pa[16];
                xs[0] = v01.x;
                xs[1] = v01.y;
                xs[2] = v23.x;
                xs[3] = v23.y;
            }
#pragma unroll
            for (int i = 0; i < 4; ++i)
                lossy_code<REL>(xs[i], delta, e, r, q[i], out[i], xh[i]);
            const int32_t prev =
                (int32_t)dpp32<kWaveShr1>((uint32_t)(t == 0 ? q[0] : (int32_t)carry),
                                          (uint32_t)q[3]);
            if (t == 0)
                anchor = (uint64_t)(int64_t)__builtin_amdgcn_readlane(q[0], 0);
            carry = (uint64_t)(int64_t)__builtin_amdgcn_readlane(q[3], 63);
            uint32_t z[4];
            z[0] = zigzag32(q[0] - prev);
            z[1] = zigzag32(q[1] - q[0]);
            z[2] = zigzag32(q[2] - q[1]);
            z[3] = zigzag32(q[3] - q[2]);
            w = row_max32(active ? bitlen32(z[0] | z[1] | z[2] | z[3]) : 0u);
            woff = place(w, t);
            const uint32_t b0 = (uint32_t)(4 * p) * w;
            if (active && w) {
                if (4u * w <= 32u) {
                    const uint32_t comb =
                        z[0] | (z[1] << w) | (z[2] << (2u * w)) | (z[3] << (3u * w));
                    or_bits32(prow, b0, comb);
                } else {
#pragma unroll
                    for (int i = 0; i < 4; ++i)
                        or_bits32(prow, b0 + (uint32_t)i * w, z[i]);
                }
            }
            // outliers, in plane index order (the first kScratchOutl staged)
            const uint32_t nl = active ? (uint32_t)out[0] + (uint32_t)out[1] +
                                             (uint32_t)out[2] + (uint32_t)out[3]
                                       : 0u;
            if (__ballot(nl != 0u)) {
                const uint32_t incl = wave_scan32(nl);
                uint32_t rank = nout + incl - nl;
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    if (active && out[i]) {
                        if (rank < kScratchOutl) {
                            uint8_t *ent = sout + (uint64_t)kOutlierBytes * rank;
                            *(uint32_t *)ent = (uint32_t)(c * kChunk + 4 * p + i);
                            *(uint32_t *)(ent + 4) = 0u;
                            *(uint64_t *)(ent + 8) = (uint64_t)__double_as_longlong(xs[i]);
                        }
                        ++rank;
                    }
                }
                nout += (uint32_t)__builtin_amdgcn_readlane((int)incl, 63);
            }
            if (active) {
                pa[0] = make_double2(xh[0], xh[1]);
                pa[16] = make_double2(xh[2], xh[3]);
            }
        }
        __builtin_amdgcn_wave_barrier();
        if (active && w && w < 64u) {
            uint32_t *sp = spay + 2 * woff;
            for (uint32_t k = (uint32_t)p; k < 2u * w; k += 16u) {
                sp[k] = prow[k];
                prow[k] = 0u;
            }
        }
        __builtin_amdgcn_wave_barrier();
    }
    const uint32_t v = base_w | (nout << 16);
    if (lane == 0)
        *psz_slot = v;
    return v;
}

// The plane record at rec from the staged payload and outliers (outliers at
// most kScratchOutl).
__device__ void emit_record(uint8_t *rec, int s, uint32_t pszv, uint32_t wl, uint64_t anchor,
                            const uint8_t *stage)
{
    const int lane = lane_id();
    const uint32_t C = 1u << (s - 6);
    const uint32_t pw = pszv & 0xFFFFu, no = pszv >> 16;
    if (lane == 0) {
        *(uint64_t *)rec = anchor;
        *(uint32_t *)(rec + 8) = pw;
        *(uint32_t *)(rec + 12) = no;
    }
    if (pw && (uint32_t)lane < pad8(C))
        rec[kPlaneHdrBytes + lane] = (uint32_t)lane < C ? (uint8_t)wl : (uint8_t)0;
    // payload words then outlier words, contiguous in the record; each
    // round issues all its loads before its stores
    uint64_t *__restrict__ dst = (uint64_t *)(rec + kPlaneHdrBytes + (pw ? pad8(C) : 0u));
    const uint64_t *__restrict__ src = (const uint64_t *)stage;
    const uint64_t *__restrict__ os = (const uint64_t *)(stage + kScratchPayload) - pw;
    const uint32_t total = pw + 2u * no;
    for (uint32_t k0 = 0; k0 < total; k0 += 256u) {
        uint64_t v[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const uint32_t k = k0 + (uint32_t)lane + 64u * (uint32_t)i;
            v[i] = k < pw ? src[k] : (k < total ? os[k] : 0ull);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const uint32_t k = k0 + (uint32_t)lane + 64u * (uint32_t)i;
            if (k < total)
                dst[k] = v[i];
        }
    }
}

template <bool REL>
__device__ void encode_plane(double *x, int s, double delta, double e, double r,
                             uint32_t pszv, uint32_t wreg, uint8_t *rec,
                             uint32_t *pb, uint32_t *err)
{
    const int lane = lane_id();
    const int row = lane >> 4, p = lane & 15;
    const int C = 1 << (s - 6);
    const int steps = (C + 3) >> 2;
    const uint32_t pw_total = pszv & 0xFFFFu, nout_total = pszv >> 16;
    uint8_t *widths = rec + kPlaneHdrBytes;
    uint32_t *payload =
        (uint32_t *)(rec + kPlaneHdrBytes + (pw_total ? pad8((uint32_t)C) : 0u));
    uint8_t *outl = (uint8_t *)(payload + 2 * pw_total);
    const uint32_t wl = lane < C ? wreg : 0u;
    const uint32_t ol = row_scan32(wl) - wl;
    const uint32_t wsum = (uint32_t)__builtin_amdgcn_readlane((int)(ol + wl), 15);
    if (lane == 0) {
        *(uint32_t *)(rec + 8) = pw_total;
        *(uint32_t *)(rec + 12) = nout_total;
    }
    if (pw_total && lane < (int)pad8((uint32_t)C))
        widths[lane] = lane < C ? (uint8_t)wl : (uint8_t)0;
    uint32_t *prow = pb + kPackRow * row;
    uint32_t nout = 0;
    uint64_t carry = 0;
    for (int t = 0; t < steps; ++t) {
        const int c = 4 * t + row;
        const bool active = c < C;
        const int cs = active ? c : 0;
        const uint32_t w = active ? (uint32_t)__shfl((int)wl, cs, 64) : 0u;
        const uint32_t woff = (uint32_t)__shfl((int)ol, cs, 64);
        const bool fits = woff + w <= pw_total;
        double2 *pa = (double2 *)(x + cs * kChunk + 2 * p);
        const double2 v01 = pa[0], v23 = pa[16];
        const double xs[4] = {v01.x, v01.y, v23.x, v23.y};
        const uint32_t b0 = (uint32_t)(4 * p) * w;
        if (delta == 0.0) {
            uint64_t q[4];
#pragma unroll
            for (int i = 0; i < 4; ++i)
                q[i] = (uint64_t)__double_as_longlong(xs[i]);
            const uint64_t prev = dpp64<kWaveShr1>(t == 0 ? q[0] : carry, q[3]);
            if (t == 0 && lane == 0)
                *(uint64_t *)rec = q[0];
            uint64_t z[4];
            z[0] = zigzag64(q[0] - prev);
            z[1] = zigzag64(q[1] - q[0]);
            z[2] = zigzag64(q[2] - q[1]);
            z[3] = zigzag64(q[3] - q[2]);
            carry = readlane64(q[3], 63);
            if (active && fits && w == 64u) {
                uint64_t *dst = (uint64_t *)payload + woff + 4 * p;
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    dst[i] = z[i];
            } else if (active && fits && w) {
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const uint32_t bi = b0 + (uint32_t)i * w;
                    const uint32_t sh = bi & 31u;
                    const uint32_t lo = (uint32_t)z[i], hi = (uint32_t)(z[i] >> 32);
                    or_bits32(prow, bi, lo);
                    // bits 32.. of the field start at bit bi + 32
                    if (hi) {
                        const uint32_t k = (bi >> 5) + 1;
                        atomicOr(&prow[k], hi << sh);
                        if (sh && (hi >> (32u - sh)))
                            atomicOr(&prow[k + 1], hi >> (32u - sh));
                    }
                }
            }
        } else {
            int32_t q[4];
            bool out[4];
            double xh[4];
#pragma unroll
            for (int i = 0; i < 4; ++i)
                lossy_code<REL>(xs[i], delta, e, r, q[i], out[i], xh[i]);
            const int32_t prev =
                (int32_t)dpp32<kWaveShr1>((uint32_t)(t == 0 ? q[0] : (int32_t)carry),
                                          (uint32_t)q[3]);
            if (t == 0 && lane == 0)
                *(int64_t *)rec = (int64_t)q[0];
            uint32_t z[4];
            z[0] = zigzag32(q[0] - prev);
            z[1] = zigzag32(q[1] - q[0]);
            z[2] = zigzag32(q[2] - q[1]);
            z[3] = zigzag32(q[3] - q[2]);
            carry = (uint64_t)(int64_t)__builtin_amdgcn_readlane(q[3], 63);
            if (active && fits && w) {
                if (4u * w <= 32u) {
                    const uint32_t comb = z[0] | (z[1] << w) | (z[2] << (2u * w)) |
                                          (z[3] << (3u * w));
                    or_bits32(prow, b0, comb);
                } else {
#pragma unroll
                    for (int i = 0; i < 4; ++i)
                        or_bits32(prow, b0 + (uint32_t)i * w, z[i]);
                }
            }
            // outliers, in plane index order
            uint32_t nl = active ? (uint32_t)out[0] + (uint32_t)out[1] + (uint32_t)out[2] +
                                       (uint32_t)out[3]
                                 : 0u;
            if (__ballot(nl != 0u)) {
                const uint32_t incl = wave_scan32(nl);
                uint32_t rank = nout + incl - nl;
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    if (active && out[i]) {
                        if (rank < nout_total) {
                            uint8_t *ent = outl + (uint64_t)kOutlierBytes * rank;
                            *(uint32_t *)ent = (uint32_t)(c * kChunk + 4 * p + i);
                            *(uint32_t *)(ent + 4) = 0u;
                            *(uint64_t *)(ent + 8) = (uint64_t)__double_as_longlong(xs[i]);
                        }
                        ++rank;
                    }
                }
                nout += (uint32_t)__builtin_amdgcn_readlane((int)incl, 63);
            }
            if (active) {
                pa[0] = make_double2(xh[0], xh[1]);
                pa[16] = make_double2(xh[2], xh[3]);
            }
        }
        __builtin_amdgcn_wave_barrier();
        // copy each row's packed words out and clear the buffer
        if (active && fits && w && w < 64u) {
            for (uint32_t k = (uint32_t)p; k < 2u * w; k += 16u) {
                payload[2 * woff + k] = prow[k];
                prow[k] = 0u;
            }
        }
        __builtin_amdgcn_wave_barrier();
    }
    if (lane == 0 && (wsum != pw_total || nout != nout_total))
        atomicOr(err, kErrSize);
}

// Pairwise sums of a unit's segments: leaf(o) for the amplitudes of segment
// us, tree over o; the two waves of a segment each reduce one half.
constexpr int kRowMirror = 0x140, kRowHalfMirror = 0x141;

// Perfect pairwise tree over the 64 lanes' values of a wave (exact order:
// xor-1 and xor-2 partners by quad permutes, then the other half-row and
// row by mirrors, each lane holding its aligned group's sum; rows combined
// as (r0 + r1) + (r2 + r3)).  Valid in every lane.
__device__ __forceinline__ double wave_tree_sum(double v)
{
    auto dv = [](uint64_t u) { return __longlong_as_double((long long)u); };
    auto du = [](double d) { return (uint64_t)__double_as_longlong(d); };
    v = v + dv(dpp64<kQuadXor1>(0ull, du(v)));
    v = v + dv(dpp64<kQuadXor2>(0ull, du(v)));
    v = v + dv(dpp64<kRowHalfMirror>(0ull, du(v)));
    v = v + dv(dpp64<kRowMirror>(0ull, du(v)));
    const double r0 = dv(readlane64(du(v), 0)), r1 = dv(readlane64(du(v), 16));
    const double r2 = dv(readlane64(du(v), 32)), r3 = dv(readlane64(du(v), 48));
    return (r0 + r1) + (r2 + r3);
}

// segment_tree for s = 10 with a leaf f(re, im) of both planes: lane L of
// a wave sums the 8 consecutive scalars 8L .. 8L+7 of its half segment, which
// sit in two 4-double runs of the swizzled layout.
template <class F>
__device__ double segment_tree10(const Unit &uc, const Planes &X, double *red, F f)
{
    const int wave = threadIdx.x >> 6, lane = lane_id();
    const int us = wave >> 1, half = wave & 1;
    double v = 0.0;
    if (us < uc.nsu) {
        const int base = (half * 8 + (lane >> 3)) * kChunk + 4 * (lane & 7);
        const double2 *ra = (const double2 *)&X[us][0][base];
        const double2 *rb = (const double2 *)&X[us][0][base + 32];
        const double2 *ia = (const double2 *)&X[us][1][base];
        const double2 *ib = (const double2 *)&X[us][1][base + 32];
        const double2 r01 = ra[0], r45 = ra[1], r23 = rb[0], r67 = rb[1];
        const double2 i01 = ia[0], i45 = ia[1], i23 = ib[0], i67 = ib[1];
        const double f0 = f(r01.x, i01.x), f1 = f(r01.y, i01.y);
        const double f2 = f(r23.x, i23.x), f3 = f(r23.y, i23.y);
        const double f4 = f(r45.x, i45.x), f5 = f(r45.y, i45.y);
        const double f6 = f(r67.x, i67.x), f7 = f(r67.y, i67.y);
        v = wave_tree_sum(((f0 + f1) + (f2 + f3)) + ((f4 + f5) + (f6 + f7)));
    }
    if (lane == 0)
        red[wave] = v;
    __syncthreads();
    double out = 0.0;
    if (threadIdx.x < (unsigned)uc.nsu)
        out = red[2 * threadIdx.x] + red[2 * threadIdx.x + 1];
    __syncthreads();
    return out;
}

template <class Leaf>
__device__ double segment_tree(const Unit &uc, int s, double *red, Leaf leaf)
{
    const int wave = threadIdx.x >> 6, lane = lane_id();
    const int us = wave >> 1, half = wave & 1;
    const int halfn = 1 << (s - 1);
    const int per = halfn >= 64 ? halfn / 64 : 1;
    const int active = halfn >= 64 ? 64 : halfn;
    double v = 0.0;
    if (us < uc.nsu) {
        if (lane < active) {
            const int base = half * halfn + lane * per;
            double t[8];
#pragma unroll
            for (int i = 0; i < 8; ++i)
                t[i] = (i < per) ? leaf(us, base + i) : 0.0;
#pragma unroll
            for (int st = 1; st < 8; st <<= 1)
                if (st < per) {
#pragma unroll
                    for (int i = 0; i < 8; i += 2 * st)
                        t[i] = t[i] + t[i + st];
                }
            v = t[0];
        }
        for (int d = 1; d < active; d <<= 1)
            v = v + __shfl_xor(v, d, 64);
    }
    if (lane == 0)
        red[wave] = v;
    __syncthreads();
    double out = 0.0;
    if (threadIdx.x < (unsigned)uc.nsu)
        out = red[2 * threadIdx.x] + red[2 * threadIdx.x + 1];
    __syncthreads();
    return out;
}

// --------------------------------------------------------- the pass -------

enum : int { kFused = 0, kEsc = 1, kReplay = 2 };

// Ladder level the block's previous stream used (0 for the basis source).
__device__ __forceinline__ int hint_level(const PassArgs &a, uint64_t j)
{
    if (a.src_basis)
        return 0;
    const int h = a.din.blk_level[j];
    return h < a.lad.L ? h : a.lad.L - 1;
}

// Whether the gate leaves every amplitude of block j as it is, by the
// gate's structure alone (Sec. V): a diagonal or controlled gate acts only
// where its qubits are 1, PHASE_FLIP only at its index, SWAP only where its
// two bits differ.  A qubit inside the block (below b) varies over the
// block, so only qubits at or above b can leave a whole block unchanged.
__device__ __forceinline__ bool block_untouched(const GateArg &G, int b, uint64_t j)
{
    auto hi = [&](int q) -> int { return q >= b ? (int)((j >> (q - b)) & 1u) : -1; };
    switch (G.kind) {
    case kDiag1:
    case kCU:
        return hi(G.q0) == 0;
    case kCPhase:
    case kCZ:
        return hi(G.q0) == 0 || hi(G.q1) == 0;
    case kPhaseFlip:
        return (G.index >> b) != j;
    case kSwap: {
        const int x = hi(G.q0), y = hi(G.q1);
        return x >= 0 && x == y;
    }
    default:
        return false;
    }
}

// A block whose stream this pass keeps (skip shortcut).
__device__ __forceinline__ bool block_kept(const PassArgs &a, uint64_t j)
{
    return a.sc_skip && !a.src_basis && block_untouched(a.gate, a.geo.b, j);
}

// Bytes of the plane record at rec.
__device__ __forceinline__ uint32_t record_bytes(const uint8_t *rec, uint32_t padC)
{
    const uint32_t pw = *(const uint32_t *)(rec + 8);
    const uint32_t no = *(const uint32_t *)(rec + 12);
    return kPlaneHdrBytes + (pw ? padC : 0u) + 8u * pw + kOutlierBytes * no;
}

// Copy a record of `bytes` (a multiple of 8) with one wavefront.
__device__ void copy_record(const uint8_t *src, uint8_t *dst, uint32_t bytes)
{
    const int lane = lane_id();
    const uint64_t *s8 = (const uint64_t *)src;
    uint64_t *d8 = (uint64_t *)dst;
    const uint32_t nw = bytes / 8;
    for (uint32_t k0 = 0; k0 < nw; k0 += 256u) {
        uint64_t v[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const uint32_t k = k0 + (uint32_t)lane + 64u * (uint32_t)i;
            v[i] = k < nw ? s8[k] : 0ull;
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const uint32_t k = k0 + (uint32_t)lane + 64u * (uint32_t)i;
            if (k < nw)
                d8[k] = v[i];
        }
    }
}

// Workgroup-shared storage of the pass kernels (40.9 KiB: four workgroups
// fit a CU).  After a unit's records are written, X doubles as scratch for
// the block decisions and reductions.
struct PassLds {
    alignas(16) Planes X;
    uint32_t pack[4][4 * kPackRow];
    uint64_t misc[9];  // segment sums, then record bytes + base
    uint64_t chunk[2]; // this workgroup's current arena chunk [cur, end)
};

// The hardware slot of the calling wave, < kHwSlots: HW_ID's wave slot
// [3:0], SIMD [5:4], CU [11:8], shader array [12] and engine [14:13], and
// XCC_ID [3:0].
__device__ __forceinline__ uint64_t hw_wave_slot()
{
    const uint32_t hw = __builtin_amdgcn_s_getreg((31 << 11) | (0 << 6) | 4);
    const uint32_t xcc = __builtin_amdgcn_s_getreg((3 << 11) | (0 << 6) | 20);
    return (uint64_t)((hw & 0x3Fu) | (((hw >> 8) & 0x7Fu) << 6) | ((xcc & 0xFu) << 13));
}

// Whether the gate maps amplitudes that are +0 in both components to +0 in
// both, for every amplitude index, as evaluated by the gate code itself (a
// product with a negative matrix entry or a negation yields -0, whose
// lossless code differs from +0's).  Then a unit whose input planes are all
// +0 has all-+0 output planes.
__device__ __forceinline__ bool zero_preserving(const GateArg &G)
{
    auto pz = [](double v) { return __double_as_longlong(v) == 0; };
    switch (G.kind) {
    case kX:
    case kSwap:
        return true;
    case kU:
    case kCU: {
        double ar = 0.0, ai = 0.0, br = 0.0, bi = 0.0;
        gate_pair(G, ~0ull, ar, ai, br, bi);
        return pz(ar) && pz(ai) && pz(br) && pz(bi);
    }
    case kDiag1:
    case kCPhase:
    case kCZ: {
        double ar = 0.0, ai = 0.0;
        gate_diag(G, ~0ull, ar, ai, nullptr);
        return pz(ar) && pz(ai);
    }
    default:
        return false;
    }
}

// Arena space is taken from the shared bump pointer in chunks of
// PassArgs::chunk_bytes (or one unit's need, if larger) and handed out unit by
// unit, so a pass issues far fewer device-scope atomics than it has units.
// The chunk is at most 32 KiB and at most 1/8 of the arena divided by the
// workgroup count, which bounds the unused chunk tails.

// One unit of a pass: decode + normalise + gate in LDS, then per plane
//   kFused:  sizes at levels 0..h (h = the block's previous level), encode
//            at h (the speculation);
//   kEsc:    for the planes of block jsel (whose sized levels 0..h all
//            missed theta): sizes at levels h+2 .. L-1, encode at h+1 (the
//            likeliest choice, kept when the block's decision takes it);
//   kReplay: encode the planes of block jsel at its chosen level;
// records are bump-allocated per unit; per-segment normsq of what was
// encoded.
// `tot` bytes from the workgroup's arena chunk, taking a new chunk from the
// arena's bump pointer when the current one is too small (one thread);
// ~0 when the arena is full (the error is recorded).
__device__ __forceinline__ uint64_t take_arena(const PassArgs &a, PassLds &S, uint64_t tot)
{
    if (S.chunk[0] + tot > S.chunk[1]) {
        const uint64_t want = tot > a.chunk_bytes ? tot : a.chunk_bytes;
        const uint64_t b0 = atomicAdd((unsigned long long *)&a.dev->arena_used[a.out_arena],
                                      (unsigned long long)want);
        S.chunk[0] = b0;
        S.chunk[1] = b0 + want;
    }
    const uint64_t base = S.chunk[0];
    S.chunk[0] += tot;
    if (base + tot > a.arena_cap) {
        if (atomicOr(&a.dev->err, kErrArena) == 0)
            a.dev->err_pass = (uint32_t)a.pass;
        return ~0ull;
    }
    return base;
}

// This workgroup's first arena chunk of a pass, from the reservation below
// arena_start (S.chunk, set by one thread); an empty chunk (the first
// allocation then takes one from the bump pointer) when the grid's chunks
// would not fit the reservation.
__device__ __forceinline__ void first_chunk(const PassArgs &a, PassLds &S)
{
    const uint64_t c = a.chunk_bytes;
    if ((uint64_t)gridDim.x * c <= arena_start(a.arena_cap) - kArenaBase) {
        S.chunk[0] = kArenaBase + (uint64_t)blockIdx.x * c;
        S.chunk[1] = S.chunk[0] + c;
    } else {
        S.chunk[0] = S.chunk[1] = 0;
    }
}

// Bump-allocate `mine ? bytes : 0` per wave for this unit's records (all
// threads); returns this wave's offset, or ~0 when the arena is full (the
// error is recorded).
__device__ uint64_t alloc_records(const PassArgs &a, PassLds &S, bool mine, uint64_t bytes)
{
    uint64_t *rbytes = S.misc;
    uint64_t &rbase = S.misc[8];
    const int wave = threadIdx.x >> 6, lane = lane_id();
    if (lane == 0)
        rbytes[wave] = mine ? bytes : 0;
    __syncthreads();
    if (threadIdx.x == 0) {
        const uint64_t tot = rbytes[0] + rbytes[1] + rbytes[2] + rbytes[3];
        rbase = tot ? take_arena(a, S, tot) : 0;
    }
    __syncthreads();
    if (rbase == ~0ull)
        return ~0ull;
    uint64_t off = rbase;
    for (int w2 = 0; w2 < wave; ++w2)
        off += rbytes[w2];
    return off;
}

// Output of a unit whose four input planes are all +0 under a zero-preserving
// gate: every plane is +0 at every level, so each sized level has no payload
// and no outliers, each record is its 16-byte header of zeros, and every
// segment's normsq is +0 -- exactly what the full path computes for it.
template <int MODE>
__device__ void zero_unit(const PassArgs &a, const Unit &uc, uint64_t jsel, PassLds &S, int lvl)
{
    const int s = a.geo.s;
    const int wave = threadIdx.x >> 6, lane = lane_id();
    const int us = wave >> 1, p = wave & 1;
    const int bs = a.geo.b - s;
    const uint64_t nplanes = 2 * a.geo.nseg;
    const bool active = us < uc.nsu;
    const uint64_t g = active ? uc.seg(us) : 0;
    const uint64_t j = g >> bs;
    const uint64_t plane = 2 * g + p;
    const bool mine = active && (MODE == kFused || j == jsel);
    if (mine && lane == 0) {
        int k0 = 0, k1 = lvl;
        if (MODE == kEsc) {
            k0 = lvl + 1;
            k1 = a.lad.L - 1;
        } else if (MODE == kReplay) {
            k0 = k1 = lvl;
        }
        for (int k = k0; k <= k1; ++k)
            a.psz[(uint64_t)k * nplanes + plane] = 0u;
        set_rec_at(a.dout, plane, 0);  // the shared all-zero record
    }
    if (threadIdx.x < (unsigned)uc.nsu) {
        const uint64_t gs = uc.seg((int)threadIdx.x);
        if (MODE == kFused || (gs >> bs) == jsel)
            a.dout.segnorm[gs] = 0.0;
    }
}

// SC: the general instance, for passes with the skip shortcut, states that
// may hold blocks with a deferred scale (reads each block's scale, keeps
// untouched blocks) and ladders with relative levels; the other instance has
// none of that code.
template <int MODE, bool SC>
__device__ void unit_body(const PassArgs &a, const Unit &uc, uint64_t jsel, PassLds &S,
                          double scale, const double *tdiff, bool zp,
                          const DevState *lazy = nullptr)
{
    Planes &X = S.X;
    double *red = (double *)S.misc;
    const int s = a.geo.s;
    const int wave = threadIdx.x >> 6, lane = lane_id();
    const int us = wave >> 1, p = wave & 1;
    const int L = a.lad.L;
    const uint64_t nplanes = 2 * a.geo.nseg;
    const int bs = a.geo.b - s;
    const uint32_t padC = pad8(1u << (s - 6));
    const bool active = us < uc.nsu;
    const uint64_t g = uc.seg(active ? us : 0);
    const uint64_t j = g >> bs;
    // The unit's reads that depend on nothing else, in one round trip: the
    // record offsets of its four planes (offset 0 is the shared all-zero
    // record, every other record lies at kArenaBase or above), the block's
    // error bound and its level (kReplay: the decided one; else the one
    // the previous pass chose, the speculated level here).
    uint64_t poff = 0, zoff = 1;
    double pdelta = 0.0, cin = 1.0;
    uint32_t lraw = 0;
    // lazy: s and 2*mean read here, with the unit's reads, instead of in a
    // round trip of their own at the kernel's start
    double tdl[2] = {0.0, 0.0};
    if (lazy) {
        scale = lazy->scale;
        tdl[0] = lazy->tdiff[0];
        tdl[1] = lazy->tdiff[1];
        tdiff = tdl;
    }
    if (MODE == kReplay)
        lraw = a.dout.blk_level[j];
    if (!a.src_basis) {
        pdelta = *(const double *)(a.din.hdr + 32 * j + 16);
        if (SC)
            cin = a.din.bscale[j];
        if (MODE != kReplay)
            lraw = a.din.blk_level[j];
        const uint64_t g0 = uc.seg(0), g1 = uc.seg(1);
        const uint64_t o00 = rec_at(a.din, 2 * g0), o01 = rec_at(a.din, 2 * g0 + 1);
        const uint64_t o10 = rec_at(a.din, 2 * g1), o11 = rec_at(a.din, 2 * g1 + 1);
        poff = us == 0 ? (p ? o01 : o00) : (p ? o11 : o10);
        zoff = o00 | o01 | o10 | o11;
        // keeps the compiler from sinking these loads to their first uses
        // (one wait for all of them instead of one round trip each)
        asm volatile("" ::"v"(zoff), "v"(poff), "v"(pdelta), "v"(lraw), "v"(scale), "v"(cin));
    }
    const int lvl = MODE == kReplay ? (int)lraw : ((int)lraw < L ? (int)lraw : L - 1);
    // skip shortcut: segments of blocks the gate leaves unchanged keep their
    // records (copied into the output arena) and their segment norms
    const bool keep0 = SC && MODE == kFused && block_kept(a, uc.seg(0) >> bs);
    const bool keep1 = SC && MODE == kFused && uc.nsu == 2 && block_kept(a, uc.seg(1) >> bs);
    const bool keep_me = SC && active && (us ? keep1 : keep0);
    if (SC && keep0 && (uc.nsu == 1 || keep1)) {
        const uint32_t rb = (active && poff) ? record_bytes(a.arena_in + poff, padC) : 0u;
        const uint64_t off = alloc_records(a, S, active && poff != 0, rb);
        if (active) {
            if (poff == 0) {
                if (lane == 0)
                    set_rec_at(a.dout, 2 * g + p, 0);
            } else if (off != ~0ull) {
                if (lane == 0)
                    set_rec_at(a.dout, 2 * g + p, off);
                copy_record(a.arena_in + poff, a.arena_out + off, rb);
            }
        }
        if (threadIdx.x < (unsigned)uc.nsu) {
            const uint64_t gs = uc.seg((int)threadIdx.x);
            a.dout.segnorm[gs] = a.din.segnorm[gs];
        }
        return;
    }
    if (a.src_basis) {
        // basis state: every unit but the one holding |basis> is all +0
        const uint64_t gb = a.basis >> s;
        bool holds = false;
        for (int k = 0; k < uc.nsu; ++k)
            holds = holds || uc.seg(k) == gb;
        if (!holds) {
            zero_unit<MODE>(a, uc, jsel, S, lvl);
            return;
        }
    } else if (zp && zoff == 0) {
        // every input plane of the unit is the all-zero record
        zero_unit<MODE>(a, uc, jsel, S, lvl);
        return;
    }
    uint32_t flat = 1;  // this plane's input has a chunk of width 0
    if (active && !keep_me) {
        double *dst = &X[us][p][0];
        if (a.src_basis) {
            for (int o = lane; o < (1 << s); o += 64)
                dst[sw(o)] = (p == 0 && ((g << s) | (uint64_t)o) == a.basis) ? 1.0 : 0.0;
        } else {
            // normalisation with the block's deferred scale: fl(c_j s)
            const double fac = SC ? cin * scale : scale;
            flat = decode_plane<SC>(a.arena_in + poff, s, pdelta, fac, fac != 1.0, dst);
        }
    }
    if (lane == 0)
        S.misc[4 + wave] = flat;
    __syncthreads();
    gate_unit(a.gate, uc, s, X, tdiff);
    __syncthreads();
    // a unit none of whose input planes has a flat chunk is dense: the gate
    // mixes within the unit only, so its output has no zero steps to skip
    // and the step summary is not formed
    const bool sparse = (S.misc[4] | S.misc[5] | S.misc[6] | S.misc[7]) != 0;
    const uint64_t plane = 2 * g + p;
    const bool mine = active && !keep_me && (MODE == kFused || j == jsel);
    int lev = 0;
    uint32_t pszv = 0, wreg = 0;
    uint64_t anchor = 0;
    uint8_t *stage =
        a.scratch +
        (a.stage_by_slot ? hw_wave_slot() : ((uint64_t)blockIdx.x * 4 + (uint64_t)wave)) *
            kScratchWave;
    if (mine) {
        const int h = lvl;
        const StepSum sum = sparse ? step_summary(&X[us][p][0], s)
                                   : StepSum{0x7FF00000u, 0x7FF00000u, 0x7FF00000u,
                                             0x7FF00000u, 0u};
        if (MODE == kEsc) {
            // an escalated block (h < L - 1): the levels above h + 1 are only
            // sized; h + 1 is sized and packed together
            lev = h + 1;
            if (lev < L - 1)
                size_levels<SC>(&X[us][p][0], s, a.lad, lev + 1, L - 1, -1, a.psz, plane,
                                nplanes, wreg, sum);
        } else {
            // kFused: levels below the speculated one are only sized; the
            // speculated level is sized and packed together
            lev = h;
            // (permutation shortcut: the previous level only, no other sized)
            if (MODE == kFused && h > 0 && !a.sc_perm)
                size_levels<SC>(&X[us][p][0], s, a.lad, 0, h - 1, -1, a.psz, plane, nplanes,
                            wreg, sum);
        }
        pszv = size_pack_level<SC>(&X[us][p][0], s, a.lad.delta[lev], a.lad.e[lev],
                                   a.lad.r[lev], a.psz + (uint64_t)lev * nplanes + plane, stage,
                                   &S.pack[wave][0], wreg, anchor, sum);
    }
    // bump-allocate this unit's records in the output arena (an all-zero
    // record is the shared one)
    const bool zrec = pszv == 0u && anchor == 0ull;
    // a kept segment of a unit whose other segment is processed (a unit over
    // two blocks): its records are copied
    const uint32_t kb = (SC && keep_me && poff) ? record_bytes(a.arena_in + poff, padC) : 0u;
    const uint64_t off = alloc_records(a, S, (mine && !zrec) || kb != 0u,
                                       keep_me ? kb : rec_bytes(pszv, padC));
    if (SC && keep_me) {
        if (poff == 0) {
            if (lane == 0)
                set_rec_at(a.dout, plane, 0);
        } else if (off != ~0ull) {
            if (lane == 0)
                set_rec_at(a.dout, plane, off);
            copy_record(a.arena_in + poff, a.arena_out + off, kb);
        }
    } else if (mine && zrec) {
        if (lane == 0)
            set_rec_at(a.dout, plane, 0);
    } else if (mine && off != ~0ull) {
        if (lane == 0)
            set_rec_at(a.dout, plane, off);
        if ((pszv >> 16) <= kScratchOutl)
            emit_record(a.arena_out + off, s, pszv, wreg, anchor, stage);
        else  // more outliers than staged: encode again from x-hat (same codes)
            encode_plane<SC>(&X[us][p][0], s, a.lad.delta[lev], a.lad.e[lev], a.lad.r[lev],
                         pszv, wreg, a.arena_out + off, &S.pack[wave][0], &a.dev->err);
    }
    __syncthreads();
    const double ns = s == kMaxS
        ? segment_tree10(uc, X, red, [](double re, double im) {
              const double rr = re * re;
              const double ii = im * im;
              return rr + ii;
          })
        : segment_tree(uc, s, red, [&](int su, int o) {
              const double re = X[su][0][sw(o)], im = X[su][1][sw(o)];
              const double rr = re * re;
              const double ii = im * im;
              return rr + ii;
          });
    if (threadIdx.x < (unsigned)uc.nsu) {
        const uint64_t gs = uc.seg((int)threadIdx.x);
        if (SC && (threadIdx.x ? keep1 : keep0))
            a.dout.segnorm[gs] = a.din.segnorm[gs];
        else if (MODE == kFused || (gs >> bs) == jsel)
            a.dout.segnorm[gs] = ns;
    }
}

__device__ bool decide_escalated(const PassArgs &a, uint64_t j, PassLds &S);

// ------------------------------------------------------- bulk rounds ----
//
// With many more units than workgroups (a.unit_batch > 1), a workgroup takes
// its units in rounds of unit_batch.  First each thread settles one unit on
// its own where it can, writing exactly what the unit body writes for it:
// an all-zero unit under a zero-preserving gate (in a basis encode, every
// unit without the basis index), or, in a DIFFUSE or PHASE_FLIP pass, a unit
// of one-value planes.  The units left are marked in per-wave masks and run
// through the unit body by the whole workgroup.  States of a few thousand
// units keep unit_batch 1: one unit per round, no first phase.

// Units per round for a state of nunits units on a grid of at most grid
// workgroups: 1 (no bulk rounds) below 16 units per workgroup, else the
// largest power of two up to one per thread that leaves every workgroup at
// least two rounds.
__host__ __device__ inline uint32_t unit_batch_for(uint64_t nunits, uint64_t grid)
{
    if (nunits < 16 * grid)
        return 1;
    uint32_t b = 1;
    while (b < (uint32_t)kWG && (uint64_t)b * 4 * grid <= nunits)
        b *= 2;
    return b;
}

// One thread's all-zero unit (see zero_unit).  Returns whether it was one.
__device__ bool bulk_zero_unit(const PassArgs &a, const Unit &uc)
{
    const int s = a.geo.s, bs = a.geo.b - s;
    const uint64_t nplanes = 2 * a.geo.nseg;
    if (a.src_basis) {
        const uint64_t gb = a.basis >> s;
        for (int k = 0; k < uc.nsu; ++k)
            if (uc.seg(k) == gb)
                return false;
    } else {
        uint64_t o = 0;
        for (int i = 0; i < 2 * uc.nsu; ++i)
            o |= rec_at(a.din, 2 * uc.seg(i >> 1) + (i & 1));
        if (o != 0)
            return false;
    }
    for (int k = 0; k < uc.nsu; ++k) {
        const uint64_t g = uc.seg(k);
        const int lvl = hint_level(a, g >> bs);
        for (int p = 0; p < 2; ++p) {
            const uint64_t plane = 2 * g + p;
            for (int l = 0; l <= lvl; ++l)
                a.psz[(uint64_t)l * nplanes + plane] = 0u;
            set_rec_at(a.dout, plane, 0);  // the shared all-zero record
        }
        a.dout.segnorm[g] = 0.0;
    }
    return true;
}

// Arena space for one bulk round: `bytes` from this thread, one allocation
// for the workgroup (all threads).  Returns this thread's offset, ~0 after an
// overflow (recorded).
__device__ uint64_t bulk_alloc(const PassArgs &a, PassLds &S, uint32_t bytes)
{
    uint32_t *cnt = (uint32_t *)&S.misc[0];
    if (threadIdx.x == 0)
        *cnt = 0u;
    __syncthreads();
    const uint32_t mine = bytes ? atomicAdd(cnt, bytes) : 0u;
    __syncthreads();
    if (threadIdx.x == 0) {
        const uint64_t tot = *cnt;
        S.misc[8] = tot ? take_arena(a, S, tot) : 0;
    }
    __syncthreads();
    const uint64_t base = S.misc[8];
    return base == ~0ull ? ~0ull : base + mine;
}

// One thread's one-value unit (see const_unit), from const_eval's results:
// sizes of levels 0..h, the records (the k-th nonzero anchor at rec + 16 k;
// rec is ~0 after an overflow), segment norms.
__device__ __forceinline__ void bulk_const_write(const PassArgs &a, const Unit &uc,
                                                 const double *y,
                                 const double *xh, const uint64_t *anc, const int *lev,
                                 uint64_t rec)
{
    const int s = a.geo.s;
    const uint64_t nplanes = 2 * a.geo.nseg;
    uint64_t at = rec;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const uint64_t plane = 2 * uc.seg(i >> 1) + (i & 1);
        const int h = lev[i >> 1];
        for (int k = 0; k <= h; ++k) {
            uint32_t v = 0;
            if (a.lad.delta[k] != 0.0) {
                int32_t q;
                bool out;
                double xq;
                lossy_code(y[i], a.lad.delta[k], a.lad.e[k], a.lad.r[k], q, out, xq);
                v = out ? (1u << s) << 16 : 0u;
            }
            a.psz[(uint64_t)k * nplanes + plane] = v;
        }
        if (anc[i] == 0ull) {
            set_rec_at(a.dout, plane, 0);
        } else {
            if (rec != ~0ull) {
                set_rec_at(a.dout, plane, at);
                uint4 r;
                r.x = (uint32_t)anc[i];
                r.y = (uint32_t)(anc[i] >> 32);
                r.z = 0u;
                r.w = 0u;
                *(uint4 *)(a.arena_out + at) = r;
            }
            at += kPlaneHdrBytes;
        }
    }
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const double rr = xh[2 * k] * xh[2 * k];
        const double ii = xh[2 * k + 1] * xh[2 * k + 1];
        a.dout.segnorm[uc.seg(k)] = (rr + ii) * (double)(1u << s);
    }
}

// The workgroup-uniform 64-bit mask of wave w's threads that left their unit
// to the unit body (published in S.misc[4 + w]).
__device__ __forceinline__ uint64_t left_mask(const PassLds &S, int w)
{
    const uint64_t m = S.misc[4 + w];
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)m);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(m >> 32));
    return ((uint64_t)hi << 32) | lo;
}

// The value of plane i (segment i >> 1, component i & 1) of a unit whose
// records hold one value each, after decode, normalisation and the gate
// (DIFFUSE: 2 mean - a; PHASE_FLIP outside its index: unchanged).
__device__ __forceinline__ double const_plane_value(const PassArgs &a, uint64_t anchor,
                                                    double delta_in, int comp, double scale,
                                                    double td)
{
    double x = delta_in == 0.0 ? __longlong_as_double((long long)anchor)
                               : dequant((int32_t)(uint32_t)anchor, delta_in,
                                         level_step(delta_in));
    if (scale != 1.0)
        x = x * scale;
    (void)comp;
    return a.gate.kind == kDiffuse ? td - x : x;
}

// Fast path of a DIFFUSE or PHASE_FLIP pass for a unit whose four input
// records carry neither payload nor outliers (Grover states are almost
// entirely such units).  Each plane then holds one value y after the gate,
// and its encoding follows from y alone: at every level all codes are equal
// (every Lorenzo residual and chunk width is 0, so no payload), a lossy level
// has either no outlier or all 2^s of them, and the record is the anchor.
// The segment normsq is 2^s times fl(fl(re^2) + fl(im^2)) of the x-hat
// values (the pairwise tree of equal leaves doubles exactly).  Units whose
// speculated level would hold outliers, and the unit holding PHASE_FLIP's
// index, take the full path.  Returns whether the unit was handled
// (workgroup-uniform).
// The evaluation half of const_unit, by one thread for a whole unit: whether
// the unit qualifies, and then each plane's value after the gate (y), its
// x-hat and output anchor at the speculated level, and the speculated level
// of each segment.
// Whether a gate applies the same operation to every position of a segment
// (with, for a pair gate, the partner at the same position of the coupled
// segment): DIFFUSE, PHASE_FLIP away from its index, and gates whose qubits
// are all at or above s.  Planes of one value then stay planes of one value.
__device__ __forceinline__ bool segment_uniform(const GateArg &G, int s)
{
    switch (G.kind) {
    case kDiffuse:
    case kPhaseFlip:
        return true;
    case kU:
    case kX:
    case kDiag1:
        return G.q0 >= s;
    case kCU:
    case kCPhase:
    case kCZ:
    case kSwap:
        return G.q0 >= s && G.q1 >= s;
    default:
        return false;
    }
}

__device__ __forceinline__ bool const_eval(const PassArgs &a, const Unit &uc, double scale,
                                           const double *tdiff, double *y, double *xh,
                                           uint64_t *anc_out, int *lev)
{
    if (a.src_basis)
        return false;
    const int s = a.geo.s, bs = a.geo.b - s, L = a.lad.L;
    if (a.gate.kind == kPhaseFlip) {
        const uint64_t gm = a.gate.index >> s;
        if (uc.seg(0) == gm || uc.seg(1) == gm)
            return false;
    }
    const uint64_t g0 = uc.seg(0), g1 = uc.seg(1);
    const uint64_t o[4] = {rec_at(a.din, 2 * g0), rec_at(a.din, 2 * g0 + 1),
                           rec_at(a.din, 2 * g1), rec_at(a.din, 2 * g1 + 1)};
    uint64_t hv = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i)
        hv |= *(const uint64_t *)(a.arena_in + o[i] + 8);  // payload words | outliers
    if (hv != 0)
        return false;
    bool ok = true;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const uint64_t g = (i >> 1) ? g1 : g0;
        const uint64_t j = g >> bs;
        const double delta_in = *(const double *)(a.din.hdr + 32 * j + 16);
        const int hl = a.din.blk_level[j];
        const int h = hl < L ? hl : L - 1;
        lev[i >> 1] = h;
        const uint64_t anc = *(const uint64_t *)(a.arena_in + o[i]);
        y[i] = const_plane_value(a, anc, delta_in, i & 1, a.din.bscale[j] * scale,
                                 tdiff[i & 1]);
    }
    // gates other than DIFFUSE and PHASE_FLIP: the value pair of each
    // position through the gate's own pair or diagonal update (every
    // position of a segment gets the same operation: segment_uniform)
    if (a.gate.kind != kDiffuse && a.gate.kind != kPhaseFlip) {
        if (a.gate.mask >> s) {
            gate_pair(a.gate, g0 << s, y[0], y[1], y[2], y[3]);
        } else {
            gate_diag(a.gate, g0 << s, y[0], y[1], tdiff);
            gate_diag(a.gate, g1 << s, y[2], y[3], tdiff);
        }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int h = lev[i >> 1];
        const double dh = a.lad.delta[h];
        if (dh == 0.0) {
            xh[i] = y[i];
            anc_out[i] = (uint64_t)__double_as_longlong(y[i]);
        } else {
            int32_t q;
            bool out;
            double xq;
            lossy_code(y[i], dh, a.lad.e[h], a.lad.r[h], q, out, xq);
            ok = ok && !out;
            xh[i] = xq;
            anc_out[i] = (uint64_t)(int64_t)q;
        }
    }
    return ok;
}

__device__ bool const_unit(const PassArgs &a, const Unit &uc, PassLds &S, double scale,
                           const double *tdiff)
{
    // every thread evaluates all four planes (a few scalars): the decision
    // below is then uniform without LDS
    double y[4], xh[4];
    uint64_t anc_out[4];
    int lev[2];
    if (!const_eval(a, uc, scale, tdiff, y, xh, anc_out, lev))
        return false;
    const int s = a.geo.s;
    const uint64_t g0 = uc.seg(0), g1 = uc.seg(1);
    const int wave = threadIdx.x >> 6, lane = lane_id();
    const int us = wave >> 1, p = wave & 1;
    const bool active = us < uc.nsu;
    const uint64_t g = us ? g1 : g0;
    const uint64_t plane = 2 * g + p;
    const uint64_t nplanes = 2 * a.geo.nseg;
    const int i = 2 * us + p;
    const double yi = i == 0 ? y[0] : (i == 1 ? y[1] : (i == 2 ? y[2] : y[3]));
    const uint64_t ai = i == 0 ? anc_out[0]
                               : (i == 1 ? anc_out[1] : (i == 2 ? anc_out[2] : anc_out[3]));
    const int h = us ? lev[1] : lev[0];
    // sizes of levels 0..h: no payload; a lossy level below h has 2^s
    // outliers when y misses its bound
    if (active && lane <= h) {
        const int k = lane;
        uint32_t v = 0;
        if (a.lad.delta[k] != 0.0) {
            int32_t q;
            bool out;
            double xq;
            lossy_code(yi, a.lad.delta[k], a.lad.e[k], a.lad.r[k], q, out, xq);
            v = out ? (1u << s) << 16 : 0u;
        }
        a.psz[(uint64_t)k * nplanes + plane] = v;
    }
    // the record: the anchor alone (the shared zero record when it is 0)
    const bool zrec = ai == 0ull;
    const uint64_t off = alloc_records(a, S, active && !zrec, kPlaneHdrBytes);
    if (active && lane == 0) {
        if (zrec) {
            set_rec_at(a.dout, plane, 0);
        } else if (off != ~0ull) {
            set_rec_at(a.dout, plane, off);
            uint4 r;
            r.x = (uint32_t)ai;
            r.y = (uint32_t)(ai >> 32);
            r.z = 0u;
            r.w = 0u;
            *(uint4 *)(a.arena_out + off) = r;
        }
    }
    if (threadIdx.x < (unsigned)uc.nsu) {
        const int k = (int)threadIdx.x;
        const double re = k ? xh[2] : xh[0], im = k ? xh[3] : xh[1];
        const double rr = re * re;
        const double ii = im * im;
        a.dout.segnorm[uc.seg(k)] = (rr + ii) * (double)(1u << s);
    }
    return true;
}

// Bulk rounds serve states whose last pass left a compression ratio of at
// least kBulkRatio (and every basis encode): mostly all-zero or one-value
// units.  For a state with many units both k_pass<true> and the one-unit
// kernel are launched and each reads the ratio at its start, so exactly one
// of them runs the pass: dense states keep the one-unit kernel's code.
constexpr double kBulkRatio = 32.0;

__device__ __forceinline__ bool bulk_turn(const PassArgs &a)
{
    return a.src_basis || a.dev->last_ratio >= kBulkRatio;
}

// The fused pass over all units.
// Four workgroups per CU (the LDS budget) need at most 128 VGPRs per lane.
// BULK: rounds of a.unit_batch units with the per-thread first phase (a
// kernel of its own, so that the one-unit-per-round form that smaller states
// run keeps exactly its earlier code).
template <bool BULK, bool SC>
__global__ __launch_bounds__(kWG) __attribute__((amdgpu_waves_per_eu(4, 4))) void k_pass(
    PassArgs a)
{
    if (gridDim.x > a.scratch_wgs) {  // launch larger than the staging (host bug)
        if (blockIdx.x == 0 && threadIdx.x == 0)
            atomicOr(&a.dev->err, kErrSize);
        return;
    }
    if (a.dev->err)
        return;
    if (BULK ? !bulk_turn(a) : (a.unit_batch > 1 && bulk_turn(a)))
        return;  // the other kernel of the pair runs this pass
    __shared__ PassLds S;
    for (int k = threadIdx.x; k < 4 * 4 * kPackRow; k += kWG)
        (&S.pack[0][0])[k] = 0u;
    if (threadIdx.x == 0)
        first_chunk(a, S);
    const uint64_t Ms = a.gate.mask >> a.geo.s;
    // s and 2*mean are read by each unit together with its own reads
    const bool zp = zero_preserving(a.gate);
    if (!BULK) {
        // grid-stride over the units; the launch makes the grid odd, so
        // nonzero units on a power-of-two stride (a QFT's first half) fall
        // on distinct workgroups
        for (uint64_t it = blockIdx.x; it < a.geo.nunits; it += gridDim.x) {
            const Unit uc = unit_of(it, a.geo.nseg, Ms);
            unit_body<kFused, SC>(a, uc, ~0ull, S, 1.0, nullptr, zp, a.dev);
            __syncthreads();
        }
        return;
    }
    const uint64_t B = a.unit_batch > 1 ? (uint64_t)a.unit_batch : 1;
    const uint64_t nu = a.geo.nunits;
    const int wave = threadIdx.x >> 6;
    const bool su = !a.src_basis && segment_uniform(a.gate, a.geo.s);
    const double scale = a.dev->scale;
    const double tdiff[2] = {a.dev->tdiff[0], a.dev->tdiff[1]};
    // A workgroup whose last two first phases settled no unit (a dense
    // state) skips the first phase, trying it again every 16th round: the
    // first phase is then no cost to states it cannot help.
    uint32_t quiet = 0, round = 0;
    for (uint64_t base = blockIdx.x * B; base < nu; base += gridDim.x * B, ++round) {
        const bool probe = quiet < 2 || (round & 15) == 0;
        uint64_t m0 = 1, m1 = 0, m2 = 0, m3 = 0;  // one unit per round: base
        if (B > 1 && !probe) {
            // every unit of the round goes to the unit body
            const uint64_t cnt = nu - base < B ? nu - base : B;
            auto bits = [&](int w) -> uint64_t {
                const uint64_t lo = 64ull * (uint64_t)w;
                if (cnt <= lo)
                    return 0ull;
                const uint64_t k = cnt - lo;
                return k >= 64 ? ~0ull : ((1ull << k) - 1);
            };
            m0 = bits(0);
            m1 = bits(1);
            m2 = bits(2);
            m3 = bits(3);
        }
        if (B > 1 && probe) {
            bool left = false, mine = false;
            double y[4], xh[4];
            uint64_t anc[4];
            int lev[2];
            Unit uc{};
            uint32_t bytes = 0;
            if (threadIdx.x < B && base + threadIdx.x < nu) {
                uc = unit_of(base + threadIdx.x, a.geo.nseg, Ms);
                // units of blocks kept by the skip shortcut go to the unit
                // body, which copies their records
                const int bs = a.geo.b - a.geo.s;
                const bool kept =
                    block_kept(a, uc.seg(0) >> bs) || block_kept(a, uc.seg(1) >> bs);
                if (kept) {
                    left = true;
                } else if (!((zp || a.src_basis) && bulk_zero_unit(a, uc))) {
                    mine = su && const_eval(a, uc, scale, tdiff, y, xh, anc, lev);
                    left = !mine;
                    if (mine)
#pragma unroll
                        for (int i = 0; i < 4; ++i)
                            bytes += anc[i] != 0ull ? kPlaneHdrBytes : 0u;
                }
            }
            const uint64_t rec = bulk_alloc(a, S, bytes);
            if (mine)
                bulk_const_write(a, uc, y, xh, anc, lev, rec);
            const uint64_t bw = __ballot(left);
            if (lane_id() == 0)
                S.misc[4 + wave] = bw;
            __syncthreads();
            m0 = left_mask(S, 0);
            m1 = left_mask(S, 1);
            m2 = left_mask(S, 2);
            m3 = left_mask(S, 3);
            __syncthreads();  // the masks are read before the next round writes them
            const uint64_t cnt = nu - base < B ? nu - base : B;
            const uint64_t nleft = (uint64_t)(__builtin_popcountll(m0) + __builtin_popcountll(m1) +
                                              __builtin_popcountll(m2) + __builtin_popcountll(m3));
            quiet = nleft == cnt ? quiet + 1 : 0;
        }
        // the units left, in wave-mask order, through one call site
        int w = 0;
        uint64_t mw = m0;
        for (;;) {
            while (mw == 0 && w < 3) {
                ++w;
                mw = w == 1 ? m1 : (w == 2 ? m2 : m3);
            }
            if (mw == 0)
                break;
            const uint64_t it = base + 64 * (uint64_t)w + (uint64_t)__builtin_ctzll(mw);
            mw &= mw - 1;
            const Unit uc = unit_of(it, a.geo.nseg, Ms);
            unit_body<kFused, SC>(a, uc, ~0ull, S, 1.0, nullptr, zp, a.dev);
            __syncthreads();
        }
    }
}

// The pass for DIFFUSE and PHASE_FLIP gates: k_pass with const_unit's fast
// path in front of the unit body.
template <bool SC>
__global__ __launch_bounds__(kWG) __attribute__((amdgpu_waves_per_eu(4, 4))) void k_pass_const(
    PassArgs a)
{
    if (gridDim.x > a.scratch_wgs) {  // launch larger than the staging (host bug)
        if (blockIdx.x == 0 && threadIdx.x == 0)
            atomicOr(&a.dev->err, kErrSize);
        return;
    }
    if (a.dev->err)
        return;
    if (a.unit_batch > 1 && bulk_turn(a))
        return;  // k_pass<true> runs this pass
    __shared__ PassLds S;
    for (int k = threadIdx.x; k < 4 * 4 * kPackRow; k += kWG)
        (&S.pack[0][0])[k] = 0u;
    if (threadIdx.x == 0)
        first_chunk(a, S);
    const double scale = a.dev->scale;
    const double tdiff[2] = {a.dev->tdiff[0], a.dev->tdiff[1]};
    const bool zp = zero_preserving(a.gate);
    const int bs = a.geo.b - a.geo.s;
    for (uint64_t it = blockIdx.x; it < a.geo.nunits; it += gridDim.x) {
        const Unit uc = unit_of(it, a.geo.nseg, 0);
        // units of blocks kept by the skip shortcut go to the unit body,
        // which copies their records
        const bool kept =
            SC && (block_kept(a, uc.seg(0) >> bs) || block_kept(a, uc.seg(1) >> bs));
        if (kept || !const_unit(a, uc, S, scale, tdiff))
            unit_body<kFused, SC>(a, uc, ~0ull, S, scale, tdiff, zp);
        __syncthreads();
    }
}

// Replays and escalations left by k_decide.  Items: (replayed block,
// segment) pairs, one unit each, encoded again at the chosen level; then one
// item per escalated block, whose workgroup sizes the block's remaining
// levels over all its units while encoding them at the first of those
// (kEsc), decides, and encodes the block's units again only when the level
// decided is a higher one.
// Workgroup wg of nwg working on one state's replays and escalations (the
// pack buffers of S must be zero).
template <bool SC>
__device__ void fix_body(const PassArgs &a, uint64_t wg, uint64_t nwg, PassLds &S)
{
    if (gridDim.x > a.scratch_wgs) {
        if (wg == 0 && threadIdx.x == 0)
            atomicOr(&a.dev->err, kErrSize);
        return;
    }
    // the error word and the list lengths in one round trip
    const uint32_t err = a.dev->err, nrep = a.dev->n_replay, nesc = a.dev->n_esc;
    if ((err != 0) | (nrep + nesc == 0))
        return;
    if (threadIdx.x == 0)
        S.chunk[0] = S.chunk[1] = 0;
    const int bs = a.geo.b - a.geo.s;
    const uint64_t spb = 1ull << bs;
    const uint64_t Ms = a.gate.mask >> a.geo.s;
    const uint64_t nrep_items = (uint64_t)nrep << bs;
    const uint64_t nitems = nrep_items + nesc;
    const double scale = a.dev->scale;
    const double tdiff[2] = {a.dev->tdiff[0], a.dev->tdiff[1]};
    const bool zp = zero_preserving(a.gate);
    // one call site per unit_body mode (keeps them inlined once each)
    for (uint64_t it = wg; it < nitems; it += nwg) {
        const bool rep = it < nrep_items;
        const uint64_t jsel = rep ? a.replay_list[it >> bs] : a.esc_list[it - nrep_items];
        const uint64_t t0 = rep ? (it & (spb - 1)) : 0;
        const uint64_t tn = rep ? t0 + 1 : spb;
        for (int phase = rep ? 1 : 0; phase < 2; ++phase) {
            if (phase == 1 && !rep && !decide_escalated(a, jsel, S))
                break;  // the block's encoding at the first remaining level stands
            for (uint64_t t = t0; t < tn; ++t) {
                const uint64_t g = (jsel << bs) | t;
                const Unit uc = unit_of_seg(g, a.geo.nseg, Ms);
                const uint64_t other = uc.nsu == 2 ? (uc.g[0] == g ? uc.g[1] : uc.g[0]) : g;
                if ((other >> bs) == jsel && other < g)
                    continue;  // the unit is handled with its first segment
                if (phase == 0)
                    unit_body<kEsc, SC>(a, uc, jsel, S, scale, tdiff, zp);
                else
                    unit_body<kReplay, SC>(a, uc, jsel, S, scale, tdiff, zp);
                __syncthreads();
            }
        }
    }
}

template <bool SC>
__global__ __launch_bounds__(kWG) __attribute__((amdgpu_waves_per_eu(3, 4))) void k_fix(
    PassArgs a)
{
    __shared__ PassLds S;
    for (int k = threadIdx.x; k < 4 * 4 * kPackRow; k += kWG)
        (&S.pack[0][0])[k] = 0u;
    fix_body<SC>(a, blockIdx.x, gridDim.x, S);
}

// Read-only DIFFUSE pre-pass: per-segment pairwise sums of the normalised
// re and im parts.
__device__ void mean_unit(const PassArgs &a, uint64_t u, Planes &X, double *red,
                          double scale)
{
    const Unit uc = unit_of(u, a.geo.nseg, 0);
    const int s = a.geo.s;
    // A unit whose plane records carry neither payload nor outliers holds
    // one value per plane (the anchor's: the bit pattern, or code times 2
    // delta), and the pairwise tree of 2^s equal values v is exactly 2^s v
    // (each addition doubles): its sums need no decode, LDS or barrier.
    // (Grover states are almost entirely such units.)
    {
        const uint64_t g0 = uc.seg(0), g1 = uc.seg(1);
        const uint64_t o0 = rec_at(a.din, 2 * g0), o1 = rec_at(a.din, 2 * g0 + 1);
        const uint64_t o2 = rec_at(a.din, 2 * g1), o3 = rec_at(a.din, 2 * g1 + 1);
        // payload words | outliers << 32 of each record
        const uint64_t h0 = *(const uint64_t *)(a.arena_in + o0 + 8);
        const uint64_t h1 = *(const uint64_t *)(a.arena_in + o1 + 8);
        const uint64_t h2 = *(const uint64_t *)(a.arena_in + o2 + 8);
        const uint64_t h3 = *(const uint64_t *)(a.arena_in + o3 + 8);
        if ((h0 | h1 | h2 | h3) == 0) {
            const unsigned t = threadIdx.x;
            if (t < 2u * (unsigned)uc.nsu) {
                const uint64_t g = (t >> 1) ? g1 : g0;
                const uint64_t o = t == 0 ? o0 : (t == 1 ? o1 : (t == 2 ? o2 : o3));
                const uint64_t anc = *(const uint64_t *)(a.arena_in + o);
                const uint64_t j = g >> (a.geo.b - s);
                const double delta = *(const double *)(a.din.hdr + 32 * j + 16);
                const double e = delta == 0.0 ? 0.0 : level_step(delta);
                double v = delta == 0.0 ? __longlong_as_double((long long)anc)
                                        : dequant((int32_t)(uint32_t)anc, delta, e);
                const double fac = a.din.bscale[j] * scale;
                if (fac != 1.0)
                    v = v * fac;
                a.segsum[(uint64_t)(t & 1) * a.geo.nseg + g] = v * (double)(1u << s);
            }
            return;
        }
    }
    load_unit(a, uc, X, scale, true);
    __syncthreads();
    for (int c = 0; c < 2; ++c) {
        const double sm = a.geo.s == kMaxS
            ? segment_tree10(uc, X, red, [c](double re, double im) { return c ? im : re; })
            : segment_tree(uc, a.geo.s, red, [&](int su, int o) { return X[su][c][sw(o)]; });
        if (threadIdx.x < (unsigned)uc.nsu)
            a.segsum[(uint64_t)c * a.geo.nseg + uc.seg((int)threadIdx.x)] = sm;
    }
    __syncthreads();
}

// mean_unit's one-value case by one thread for a whole unit (bulk rounds);
// returns whether the unit was one.
__device__ bool bulk_mean_unit(const PassArgs &a, uint64_t u, double scale)
{
    const Unit uc = unit_of(u, a.geo.nseg, 0);
    const int s = a.geo.s;
    uint64_t o[4];
    uint64_t hv = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        o[i] = i < 2 * uc.nsu ? rec_at(a.din, 2 * uc.seg(i >> 1) + (i & 1)) : 0ull;
        hv |= *(const uint64_t *)(a.arena_in + o[i] + 8);
    }
    if (hv != 0)
        return false;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        if (i >= 2 * uc.nsu)
            break;
        const uint64_t g = uc.seg(i >> 1);
        const uint64_t anc = *(const uint64_t *)(a.arena_in + o[i]);
        const uint64_t j = g >> (a.geo.b - s);
        const double delta = *(const double *)(a.din.hdr + 32 * j + 16);
        const double e = delta == 0.0 ? 0.0 : level_step(delta);
        double v = delta == 0.0 ? __longlong_as_double((long long)anc)
                                : dequant((int32_t)(uint32_t)anc, delta, e);
        const double fac = a.din.bscale[j] * scale;
        if (fac != 1.0)
            v = v * fac;
        a.segsum[(uint64_t)(i & 1) * a.geo.nseg + g] = v * (double)(1u << s);
    }
    return true;
}

template <bool BULK>
__global__ __launch_bounds__(kWG) void k_mean(PassArgs a)
{
    if (a.dev->err)
        return;
    __shared__ __attribute__((aligned(16))) Planes X;
    __shared__ double red[8];
    __shared__ uint64_t lmask[4];
    const double scale = a.dev->scale;
    // bulk rounds as in the pass: one-value units settled one per thread,
    // the others through mean_unit by the whole workgroup
    if (!BULK) {
        for (uint64_t u = blockIdx.x; u < a.geo.nunits; u += gridDim.x)
            mean_unit(a, u, X, red, scale);
        return;
    }
    const uint64_t B = a.unit_batch > 1 ? (uint64_t)a.unit_batch : 1;
    const uint64_t nu = a.geo.nunits;
    const int wave = threadIdx.x >> 6;
    auto mask = [&](int w) {
        const uint64_t v = lmask[w];
        const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
        const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(v >> 32));
        return ((uint64_t)hi << 32) | lo;
    };
    for (uint64_t base = blockIdx.x * B; base < nu; base += gridDim.x * B) {
        if (B > 1) {
            bool left = false;
            if (threadIdx.x < B && base + threadIdx.x < nu)
                left = !bulk_mean_unit(a, base + threadIdx.x, scale);
            const uint64_t bw = __ballot(left);
            if (lane_id() == 0)
                lmask[wave] = bw;
            __syncthreads();
        }
        int w = 0;
        uint64_t mw = B > 1 ? mask(0) : 1;
        for (;;) {
            while (mw == 0 && B > 1 && w < 3)
                mw = mask(++w);
            if (mw == 0)
                break;
            const uint64_t u = base + 64 * (uint64_t)w + (uint64_t)__builtin_ctzll(mw);
            mw &= mw - 1;
            mean_unit(a, u, X, red, scale);
        }
        __syncthreads();  // the masks are read before the next round writes them
    }
}

// ------------------------------------------------------ reductions --------

// Pairwise sum of PER consecutive values, fully unrolled in registers.
template <int PER, class Load>
__device__ __forceinline__ double seq_tree(Load load, uint64_t base)
{
    double v[PER];
#pragma unroll
    for (int i = 0; i < PER; ++i)
        v[i] = load(base + i);
#pragma unroll
    for (int st = 1; st < PER; st <<= 1) {
#pragma unroll
        for (int i = 0; i < PER; i += 2 * st)
            v[i] = v[i] + v[i + st];
    }
    return v[0];
}

// Pairwise sum of cnt (a power of two, at most 2^kCounterLevels) aligned
// subtrees of 32 values load(base ..): the subtrees are combined through a
// binary counter -- pend[l] holds the pending left operand of level l, and a
// new subtree carries up through the levels whose pending slot is full --
// which gives exactly the perfect tree over the run.  Every level is
// unrolled with a fixed index, so pend stays in registers (no private
// memory).
constexpr int kCounterLevels = 16;

template <class Load>
__device__ __forceinline__ double counter_tree(Load load, uint64_t base, uint64_t cnt)
{
    double pend[kCounterLevels + 1];
#pragma unroll
    for (int l = 0; l <= kCounterLevels; ++l)
        pend[l] = 0.0;
    for (uint64_t i = 0; i < cnt; ++i) {
        double x = seq_tree<32>(load, base + 32 * i);
        bool carry = true;
#pragma unroll
        for (int l = 0; l <= kCounterLevels; ++l) {
            const bool full = ((i >> l) & 1u) != 0;
            if (carry && full)
                x = pend[l] + x;
            else if (carry)
                pend[l] = x;
            carry = carry && full;
        }
    }
    // the whole run ends up in the slot of level log2(cnt)
    const int top = 63 - __builtin_clzll(cnt);
    double v = 0.0;
#pragma unroll
    for (int l = 0; l <= kCounterLevels; ++l)
        v = l == top ? pend[l] : v;
    return v;
}

// Pairwise sum of m = 2^k values load(0..m) by one workgroup: each thread
// sums m/256 consecutive values (an aligned subtree), then a tree in LDS.
template <class Load>
__device__ double wg_tree(Load load, uint64_t m, double *lds)
{
    const int t = threadIdx.x;
    uint64_t nact;
    if (m >= kWG) {
        const uint64_t per = m / kWG;
        const uint64_t base = t * per;
        double v;
        switch (per) {
        case 1: v = seq_tree<1>(load, base); break;
        case 2: v = seq_tree<2>(load, base); break;
        case 4: v = seq_tree<4>(load, base); break;
        case 8: v = seq_tree<8>(load, base); break;
        case 16: v = seq_tree<16>(load, base); break;
        case 32: v = seq_tree<32>(load, base); break;
        default:
            v = counter_tree(load, base, per / 32);
        }
        lds[t] = v;
        nact = kWG;
    } else {
        lds[t] = (t < (int)m) ? load((uint64_t)t) : 0.0;
        nact = m;
    }
    __syncthreads();
    for (uint64_t st = 1; st < nact; st <<= 1) {
        if ((t & (2 * st - 1)) == 0 && (uint64_t)t + st < nact)
            lds[t] = lds[t] + lds[t + st];
        __syncthreads();
    }
    const double r = lds[0];
    __syncthreads();
    return r;
}

// Pairwise sum of m = 2^k non-negative values src[0..m) by one wavefront
// (lanes take aligned runs of m/64, or one value each with zero padding
// when m < 64, which leaves every sum of real values unchanged).
__device__ double wave_pairwise(const double *src, uint64_t m)
{
    const int lane = lane_id();
    double v;
    if (m >= 64) {
        const uint64_t per = m / 64;
        const uint64_t base = lane * per;
        auto load = [&](uint64_t i) { return src[i]; };
        switch (per) {
        case 1: v = seq_tree<1>(load, base); break;
        case 2: v = seq_tree<2>(load, base); break;
        case 4: v = seq_tree<4>(load, base); break;
        case 8: v = seq_tree<8>(load, base); break;
        case 16: v = seq_tree<16>(load, base); break;
        case 32: v = seq_tree<32>(load, base); break;
        default:
            v = counter_tree(load, base, per / 32);
        }
    } else {
        v = (uint64_t)lane < m ? src[lane] : 0.0;
    }
    return wave_tree_sum(v);
}

// dst[j] = pairwise(src[j*per .. (j+1)*per)) for j < nout; with write_hdr,
// also the normsq field of block j's output header.
__global__ __launch_bounds__(kWG) void k_segtree(PassArgs a, const double *src,
                                                 double *dst, uint64_t per,
                                                 uint64_t nout, int write_hdr)
{
    if (a.dev->err)
        return;
    __shared__ double lds[kWG];
    for (uint64_t j = blockIdx.x; j < nout; j += gridDim.x) {
        const double *p = src + j * per;
        const double v = wg_tree([&](uint64_t i) { return p[i]; }, per, lds);
        if (threadIdx.x == 0) {
            dst[j] = v;
            if (write_hdr)
                *(double *)(a.dout.hdr + 32 * j + 24) = v;
        }
    }
}

// out[c] = fl(S_c * mul), S_c the pairwise sum over all amplitudes of
// component c (block sums are aligned subtrees of the one tree).
__global__ __launch_bounds__(kWG) void k_mean_final(PassArgs a, double mul, double *out)
{
    if (a.dev->err)
        return;
    __shared__ double lds[kWG];
    for (int c = 0; c < 2; ++c) {
        const double *p = a.blksum + (uint64_t)c * a.geo.nblocks;
        const double S = wg_tree([&](uint64_t i) { return p[i]; }, a.geo.nblocks, lds);
        if (threadIdx.x == 0)
            out[c] = S * mul;
    }
}

// ------------------------------------------------------ decisions --------

// Per-level block totals over levels k0..k1 into tot[]/nout[] (workgroup).
__device__ void block_totals(const PassArgs &a, uint64_t j, int k0, int k1, uint64_t *red,
                             uint64_t *tot, uint64_t *nout)
{
    const int t = threadIdx.x;
    const uint64_t npb = 2ull << (a.geo.b - a.geo.s);
    const uint64_t nplanes = 2 * a.geo.nseg;
    const uint32_t padC = pad8(1u << (a.geo.s - 6));
    const uint64_t base = j * npb;
    for (int k = k0; k <= k1; ++k) {
        uint64_t by = 0, no = 0;
        for (uint64_t q = t; q < npb; q += kWG) {
            const uint32_t v = a.psz[(uint64_t)k * nplanes + base + q];
            by += rec_bytes(v, padC);
            no += v >> 16;
        }
        for (int part = 0; part < 2; ++part) {
            red[t] = part ? no : by;
            __syncthreads();
            for (int st = kWG / 2; st > 0; st >>= 1) {
                if (t < st)
                    red[t] += red[t + st];
                __syncthreads();
            }
            if (t == 0) {
                if (part)
                    nout[k] = red[0];
                else
                    tot[k] = red[0] + kHdrBytes;
            }
            __syncthreads();
        }
    }
}

// Header, length and level of block j's output stream.
__device__ void finalize_block(const PassArgs &a, uint64_t j, int d, uint64_t len,
                               uint64_t nout)
{
    uint64_t *h = (uint64_t *)(a.dout.hdr + 32 * j);
    h[0] = (uint64_t)kMagic | ((uint64_t)d << 32) | ((uint64_t)a.geo.s << 48) |
           ((uint64_t)a.geo.b << 56);
    h[1] = (uint64_t)(uint32_t)nout | (len << 32);
    h[2] = (uint64_t)__double_as_longlong(a.lad.delta[d]);
    h[3] = 0;
    a.dout.blk_len[j] = (uint32_t)len;
    a.dout.blk_level[j] = (uint8_t)d;
    a.dout.bscale[j] = 1.0;
}

// A block kept by the skip shortcut (one wavefront): its header, level and
// records stay (the pass copied the records and segment norms); its scale
// becomes c' = fl(c s), which the stream carries after its header when it
// is not 1; its weight in N^2 is its normsq, times fl(c' c') when c' != 1.
__device__ void keep_block(const PassArgs &a, uint64_t j)
{
    const int lane = lane_id();
    const uint64_t spb = 1ull << (a.geo.b - a.geo.s);
    const double *segn = a.dout.segnorm + j * spb;
    const double sn0 = (spb <= 64 && (uint64_t)lane < spb) ? segn[lane] : 0.0;
    const double ns = spb <= 64 ? wave_tree_sum(sn0) : wave_pairwise(segn, spb);
    if (lane == 0) {
        const double cin = a.din.bscale[j];
        const double c = cin * a.dev->scale;
        const uint64_t *hi = (const uint64_t *)(a.din.hdr + 32 * j);
        uint64_t *ho = (uint64_t *)(a.dout.hdr + 32 * j);
        const uint64_t plain = (uint64_t)a.din.blk_len[j] - (cin != 1.0 ? kScaleBytes : 0u);
        const uint64_t len = plain + (c != 1.0 ? kScaleBytes : 0u);
        const uint64_t h0 = hi[0] & ~(0xFFull << 40);
        ho[0] = h0 | ((uint64_t)(c != 1.0 ? kHdrScaled : 0u) << 40);
        ho[1] = (hi[1] & 0xFFFFFFFFull) | (len << 32);
        ho[2] = hi[2];
        ho[3] = 0;
        a.dout.blk_len[j] = (uint32_t)len;
        a.dout.blk_level[j] = a.din.blk_level[j];
        a.dout.bscale[j] = c;
        double w = ns;
        if (c != 1.0) {
            const double c2 = c * c;
            w = ns * c2;
        }
        a.blknorm[j] = w;
    }
}

// Alg. 2's choice for each block over the levels the fused pass sized
// (0 .. h, h = the block's previous level): the first whose full-block ratio
// reaches theta.  When that is the speculated level h the block is done;
// another level sends the block to the replay list; when none qualifies and
// levels above h remain, the block joins the escalation list.
// h: the block's previous level (hint_level).
template <int VEC>
__device__ void decide_block(const PassArgs &a, uint64_t j, int h);

// One wavefront per block.
// VEC: 1 = blocks of 256 planes or more (vector loads), 0 = smaller blocks,
// -1 = either (chosen per block).
template <int VEC>
__global__ __launch_bounds__(kWG) void k_decide(PassArgs a)
{
    const uint64_t nw = (uint64_t)gridDim.x * (kWG / 64);
    const uint64_t j0 = (uint64_t)blockIdx.x * (kWG / 64) + (threadIdx.x >> 6);
    // the error word and the first block's previous level in one round trip
    const uint32_t err = a.dev->err;
    const int h0 = j0 < a.geo.nblocks ? hint_level(a, j0) : 0;
    asm volatile("" ::"v"(err), "v"(h0));
    if (err)
        return;
    for (uint64_t j = j0; j < a.geo.nblocks; j += nw)
        decide_block<VEC>(a, j, j == j0 ? h0 : hint_level(a, j));
}

template <int VEC>
__device__ void decide_block(const PassArgs &a, uint64_t j, int h)
{
    if (block_kept(a, j)) {
        keep_block(a, j);
        return;
    }
    // sizes of levels 0..h summed over the block's planes by one wavefront
    // (permutation shortcut: level h only, taken without the theta test)
    const int lane = lane_id();
    const int L = a.lad.L;
    const int k0 = a.sc_perm ? h : 0;
    const uint64_t npb = 2ull << (a.geo.b - a.geo.s);
    const uint64_t nplanes = 2 * a.geo.nseg;
    const uint32_t padC = pad8(1u << (a.geo.s - 6));
    const uint64_t base = j * npb;
    // the block's segment norms, loaded early (used when the block is final)
    const uint64_t spb = npb >> 1;
    const double *segn = a.dout.segnorm + j * spb;
    const double sn0 = (spb <= 64 && (uint64_t)lane < spb) ? segn[lane] : 0.0;
    uint64_t by[kMaxL];
    uint32_t no[kMaxL];
#pragma unroll
    for (int k = 0; k < kMaxL; ++k) {
        by[k] = 0;
        no[k] = 0;
    }
    if (VEC == 1 || (VEC < 0 && npb % 256 == 0)) {
        // blocks of 256 planes or more: four planes per lane per load, four
        // loads in flight (the sums are of integers: any order is exact)
#pragma unroll 4
        for (uint64_t q = 4 * (uint64_t)lane; q < npb; q += 256) {
#pragma unroll
            for (int k = 0; k < kMaxL; ++k) {
                if (k >= k0 && k <= h) {
                    const uint4 v = *(const uint4 *)(a.psz + (uint64_t)k * nplanes + base + q);
                    by[k] += rec_bytes(v.x, padC) + rec_bytes(v.y, padC) +
                             rec_bytes(v.z, padC) + rec_bytes(v.w, padC);
                    no[k] += (v.x >> 16) + (v.y >> 16) + (v.z >> 16) + (v.w >> 16);
                }
            }
        }
    } else {
        for (uint64_t q = lane; q < npb; q += 64) {
#pragma unroll
            for (int k = 0; k < kMaxL; ++k) {
                if (k >= k0 && k <= h) {
                    const uint32_t v = a.psz[(uint64_t)k * nplanes + base + q];
                    by[k] += rec_bytes(v, padC);
                    no[k] += v >> 16;
                }
            }
        }
    }
    const double raw = (double)(16ull << a.geo.b);
    int d = -1;
    uint64_t tot_d = 0, nout_d = 0;
#pragma unroll
    for (int k = 0; k < kMaxL; ++k) {
        if (k >= k0 && k <= h && d < 0) {
            const uint64_t tk = readlane64(wave_scan64(by[k]), 63) + kHdrBytes;
            if (raw >= a.lad.theta * (double)tk || (k == h && h == L - 1) || a.sc_perm) {
                d = k;
                tot_d = tk;
                nout_d = (uint32_t)__builtin_amdgcn_readlane((int)wave_scan32(no[k]), 63);
            }
        }
    }
    if (d < 0) {
        if (lane == 0) {
            const uint32_t slot = atomicAdd(&a.dev->n_esc, 1u);
            a.esc_list[slot] = (uint32_t)j;
            atomicAdd((unsigned long long *)&a.dev->escalations, 1ull);
        }
        return;
    }
    if (lane == 0) {
        finalize_block(a, j, d, tot_d, nout_d);
        if (d != h) {
            const uint32_t slot = atomicAdd(&a.dev->n_replay, 1u);
            a.replay_list[slot] = (uint32_t)j;
            atomicAdd((unsigned long long *)&a.dev->replays, 1ull);
        }
    }
    if (d == h) {
        // the block's streams are final: its normsq from its segment sums
        // (for up to 64 segments one per lane, zero-padded: norms are >= +0)
        const double v = spb <= 64 ? wave_tree_sum(sn0) : wave_pairwise(segn, spb);
        if (lane == 0)
            a.blknorm[j] = v;
    }
}

// Choice for an escalated block over levels h+1 .. L-1 (the first whose
// ratio reaches theta, else the last), once the workgroup has sized every
// unit of the block at those levels and encoded it at h+1.  Returns whether
// the choice is above h+1, so that the block's units have to be encoded
// again at the level chosen.
__device__ bool decide_escalated(const PassArgs &a, uint64_t j, PassLds &S)
{
    uint64_t *red = (uint64_t *)&S.X[0][0][0];
    uint64_t *tot = red + kWG;
    uint64_t *nout = tot + kMaxL;
    const int L = a.lad.L;
    const int h = hint_level(a, j);
    block_totals(a, j, h + 1, L - 1, red, tot, nout);
    if (threadIdx.x == 0) {
        const double raw = (double)(16ull << a.geo.b);
        int d = L - 1;
        for (int k = h + 1; k < L; ++k)
            if (raw >= a.lad.theta * (double)tot[k]) {
                d = k;
                break;
            }
        finalize_block(a, j, d, tot[d], nout[d]);
        atomicAdd((unsigned long long *)&a.dev->replays, 1ull);
        S.misc[0] = d != h + 1;
    }
    __syncthreads();
    const bool again = S.misc[0] != 0;
    __syncthreads();
    return again;
}

// N^2 (pairwise over all amplitudes: block and segment sums are aligned
// subtrees, so the tree runs over segment sums, or over block sums when
// k_segtree has formed them), s, statistics; frees the input arena.
// nrep, nesc: the replay and escalation list lengths.
__device__ void reduce_body(const PassArgs &a, double *lds, uint64_t *ures, uint32_t nrep,
                            uint32_t nesc);
__device__ void reduce_finish(const PassArgs &a, double N2, uint64_t res, const uint32_t *hist);

// Sum of v over the workgroup (integers: any order is exact).
__device__ uint64_t wg_sum_u64(uint64_t v, uint64_t *ures)
{
    const int t = threadIdx.x;
    ures[t] = v;
    __syncthreads();
    for (int st = kWG / 2; st > 0; st >>= 1) {
        if (t < st)
            ures[t] += ures[t + st];
        __syncthreads();
    }
    const uint64_t r = ures[0];
    __syncthreads();
    return r;
}

// The reduction of a state with many blocks by gridDim.x workgroups (a power
// of two dividing the block count): each takes an aligned run of blocks,
// whose pairwise sum is a subtree of the tree over all blocks, after
// recomputing the norms of the replayed blocks in its run; its partial sums
// go to blksum (free between the DIFFUSE pre-pass and the next pass); the
// workgroup that finishes last (a ticket taken after a device-scope release
// fence, then an acquire fence) sums the partials by the same tree -- the
// top of the tree over all blocks -- and finishes as k_reduce does.
__global__ __launch_bounds__(kWG) void k_reduce_wide(PassArgs a)
{
    const uint32_t err = a.dev->err, nrep = a.dev->n_replay, nesc = a.dev->n_esc;
    if (err)
        return;
    __shared__ double lds[kWG];
    __shared__ uint64_t ures[kWG];
    __shared__ uint32_t last;
    const int t = threadIdx.x, wave = t >> 6, lane = lane_id();
    const uint64_t G = gridDim.x, per = a.geo.nblocks / G;
    const uint64_t lo = (uint64_t)blockIdx.x * per, hi = lo + per;
    const uint64_t spb = 1ull << (a.geo.b - a.geo.s);
    for (uint32_t k = (uint32_t)wave; k < nrep + nesc; k += kWG / 64) {
        const uint64_t j = k < nrep ? a.replay_list[k] : a.esc_list[k - nrep];
        if (j < lo || j >= hi)
            continue;
        const double v = wave_pairwise(a.dout.segnorm + j * spb, spb);
        if (lane == 0)
            a.blknorm[j] = v;
    }
    __syncthreads();
    const double part = wg_tree([&](uint64_t i) { return a.blknorm[lo + i]; }, per, lds);
    uint64_t by = 0;
    uint32_t hist[kMaxL];
#pragma unroll
    for (int k = 0; k < kMaxL; ++k)
        hist[k] = 0;
    for (uint64_t j = lo + t; j < hi; j += kWG) {
        by += a.dout.blk_len[j];
        const int lv = a.dout.blk_level[j];
#pragma unroll
        for (int k = 0; k < kMaxL; ++k)
            hist[k] += lv == k;
    }
    by = wg_sum_u64(by, ures);
#pragma unroll
    for (int k = 0; k < kMaxL; ++k)
        hist[k] = (uint32_t)wg_sum_u64(hist[k], ures);
    // partials: G norms, G byte counts, G x kMaxL level counts
    double *pn = a.blksum;
    uint64_t *pb = (uint64_t *)(pn + G);
    uint32_t *ph = (uint32_t *)(pb + G);
    if (t == 0) {
        pn[blockIdx.x] = part;
        pb[blockIdx.x] = by;
        for (int k = 0; k < kMaxL; ++k)
            ph[blockIdx.x * kMaxL + k] = hist[k];
        __threadfence();
        const uint32_t before = atomicAdd(&a.dev->red_ticket, 1u);
        last = before == (uint32_t)(G - 1);
        if (last) {
            __threadfence();
            a.dev->red_ticket = 0u;
        }
    }
    __syncthreads();
    if (!last)
        return;
    const double N2 = wg_tree([&](uint64_t i) { return pn[i]; }, G, lds);
    uint64_t res = 0;
    uint32_t htot[kMaxL];
#pragma unroll
    for (int k = 0; k < kMaxL; ++k)
        htot[k] = 0;
    for (uint64_t g = t; g < G; g += kWG) {
        res += pb[g];
#pragma unroll
        for (int k = 0; k < kMaxL; ++k)
            htot[k] += ph[g * kMaxL + k];
    }
    res = wg_sum_u64(res, ures);
#pragma unroll
    for (int k = 0; k < kMaxL; ++k)
        htot[k] = (uint32_t)wg_sum_u64(htot[k], ures);
    if (t == 0)
        reduce_finish(a, N2, res, htot);
}

__global__ __launch_bounds__(kWG) void k_reduce(PassArgs a)
{
    // the error word and the list lengths in one round trip
    const uint32_t err = a.dev->err, nrep = a.dev->n_replay, nesc = a.dev->n_esc;
    asm volatile("" ::"v"(err), "v"(nrep), "v"(nesc));
    if (err)
        return;
    __shared__ double lds[kWG];
    __shared__ uint64_t ures[kWG];
    reduce_body(a, lds, ures, nrep, nesc);
}

__device__ void reduce_body(const PassArgs &a, double *lds, uint64_t *ures, uint32_t nrep,
                            uint32_t nesc)
{
    const int t = threadIdx.x, wave = t >> 6, lane = lane_id();
    // normsq of the blocks that were re-encoded after k_decide
    const uint64_t spb = 1ull << (a.geo.b - a.geo.s);
    const uint32_t nfix = nrep + nesc;
    for (uint32_t k = (uint32_t)wave; k < nfix; k += kWG / 64) {
        const uint64_t j = k < nrep ? a.replay_list[k] : a.esc_list[k - nrep];
        const double v = wave_pairwise(a.dout.segnorm + j * spb, spb);
        if (lane == 0)
            a.blknorm[j] = v;
    }
    __syncthreads();
    // N^2: one pairwise tree over the block norms (aligned subtrees)
    const uint64_t nb = a.geo.nblocks;
    double N2;
    uint64_t res = 0;
    // blocks per chosen level, for the statistics
    uint32_t hist[kMaxL];
#pragma unroll
    for (int k = 0; k < kMaxL; ++k)
        hist[k] = 0;
    if (nb <= 4096) {
        N2 = wave == 0 ? wave_pairwise(a.blknorm, nb) : 0.0;
        if (wave == 0) {
            uint64_t by = 0;
            for (uint64_t j = lane; j < nb; j += 64) {
                by += a.dout.blk_len[j];
                const int lv = a.dout.blk_level[j];
#pragma unroll
                for (int k = 0; k < kMaxL; ++k)
                    hist[k] += lv == k;
            }
            res = readlane64(wave_scan64(by), 63);
#pragma unroll
            for (int k = 0; k < kMaxL; ++k)
                hist[k] = (uint32_t)__builtin_amdgcn_readlane((int)wave_scan32(hist[k]), 63);
        }
    } else {
        N2 = wg_tree([&](uint64_t i) { return a.blknorm[i]; }, nb, lds);
        uint64_t by = 0;
#pragma unroll 8
        for (uint64_t j = t; j < nb; j += kWG) {
            by += a.dout.blk_len[j];
            const int lv = a.dout.blk_level[j];
#pragma unroll
            for (int k = 0; k < kMaxL; ++k)
                hist[k] += lv == k;
        }
        ures[t] = by;
        __syncthreads();
        for (int st = kWG / 2; st > 0; st >>= 1) {
            if (t < st)
                ures[t] += ures[t + st];
            __syncthreads();
        }
        res = ures[0];
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kMaxL; ++k) {
            ures[t] = hist[k];
            __syncthreads();
            for (int st = kWG / 2; st > 0; st >>= 1) {
                if (t < st)
                    ures[t] += ures[t + st];
                __syncthreads();
            }
            hist[k] = (uint32_t)ures[0];
            __syncthreads();
        }
    }
    if (t == 0)
        reduce_finish(a, N2, res, hist);
}

// N^2 and the pass's statistics into the sim's device state; frees the
// input arena and clears the replay lists (one thread).
__device__ void reduce_finish(const PassArgs &a, double N2, uint64_t res, const uint32_t *hist)
{
    DevState *d = a.dev;
    // every field this update reads, loaded before any store: one memory
    // round trip instead of one per read-modify-write
    const int32_t normalize = d->normalize;
    const uint64_t peak = d->peak_resident;
    const double minr = d->min_ratio;
    const uint64_t passes = d->passes;
    const uint64_t used_out = d->arena_used[a.out_arena];
    const uint64_t apeak = d->arena_peak;
    uint64_t lh[kMaxL];
#pragma unroll
    for (int k = 0; k < kMaxL; ++k)
        lh[k] = d->level_hist[k];
    d->normsq = N2;
    if (N2 > 0.0 && __builtin_isfinite(N2)) {
        if (normalize)
            d->scale = inv_sqrt_exact(N2);
    } else {
        d->collapsed = 1;
        d->scale = 1.0;
    }
    d->resident = res;
    if (res > peak)
        d->peak_resident = res;
    const double ratio = (double)(16ull << a.geo.n) / (double)res;
    d->last_ratio = ratio;
    if (a.src_basis) {
        d->min_ratio = ratio;
    } else {
        d->passes = passes + 1;
        if (ratio < minr)
            d->min_ratio = ratio;
#pragma unroll
        for (int k = 0; k < kMaxL; ++k)
            d->level_hist[k] = lh[k] + hist[k];
    }
    if (used_out > apeak)
        d->arena_peak = used_out;
    d->arena_used[a.in_arena] = arena_start(a.arena_cap);
    d->n_replay = 0;
    d->n_esc = 0;
}

// ---------------------------------------------------- queries -------------

__global__ __launch_bounds__(kWG) void k_decode_range(PassArgs a, uint64_t u0,
                                                      uint64_t u1, uint64_t first,
                                                      uint64_t count, double *out)
{
    __shared__ __attribute__((aligned(16))) Planes X;
    const int s = a.geo.s;
    const double scale = a.dev->scale;
    for (uint64_t u = u0 + blockIdx.x; u < u1; u += gridDim.x) {
        const Unit uc = unit_of(u, a.geo.nseg, 0);
        load_unit(a, uc, X, scale, true);
        __syncthreads();
        for (int us = 0; us < uc.nsu; ++us)
            for (uint32_t o = threadIdx.x; o < (1u << s); o += kWG) {
                const uint64_t i = (uc.seg(us) << s) | o;
                if (i >= first && i < first + count) {
                    out[2 * (i - first)] = X[us][0][sw(o)];
                    out[2 * (i - first) + 1] = X[us][1][sw(o)];
                }
            }
        __syncthreads();
    }
}

__global__ __launch_bounds__(kWG) void k_probs(PassArgs a, const int *qubits, int nq,
                                               double *probs)
{
    __shared__ __attribute__((aligned(16))) Planes X;
    __shared__ double bins[1024];
    const int s = a.geo.s;
    const double scale = a.dev->scale;
    const bool lds_bins = nq <= 10;
    const uint32_t nb = 1u << nq;
    if (lds_bins)
        for (uint32_t k = threadIdx.x; k < nb; k += kWG)
            bins[k] = 0.0;
    __syncthreads();
    for (uint64_t u = blockIdx.x; u < a.geo.nunits; u += gridDim.x) {
        const Unit uc = unit_of(u, a.geo.nseg, 0);
        load_unit(a, uc, X, scale, true);
        __syncthreads();
        for (int us = 0; us < uc.nsu; ++us)
            for (uint32_t o = threadIdx.x; o < (1u << s); o += kWG) {
                const uint64_t i = (uc.seg(us) << s) | o;
                uint32_t oc = 0;
                for (int k = 0; k < nq; ++k)
                    oc |= (uint32_t)bit_of(i, qubits[k]) << k;
                const double re = X[us][0][sw(o)], im = X[us][1][sw(o)];
                const double rr = re * re;
                const double ii = im * im;
                const double pv = rr + ii;
                if (lds_bins)
                    atomicAdd(&bins[oc], pv);
                else
                    atomicAdd(&probs[oc], pv);
            }
        __syncthreads();
    }
    if (lds_bins)
        for (uint32_t k = threadIdx.x; k < nb; k += kWG)
            if (bins[k] != 0.0)
                atomicAdd(&probs[k], bins[k]);
}

// Inner products of two states over ranges of 2^S amplitudes.  Planes of A
// go to X[0], of B to X[1]; an uncompressed state is read from its array.
__device__ void load_range(const PassArgs &a, const double *amp, uint64_t first,
                           int S, double *dst, int p, double scale)
{
    const int lane = lane_id();
    const int cnt = 1 << S;
    if (amp) {
        for (int o = lane; o < cnt; o += 64)
            dst[sw(o)] = amp[2 * (first + o) + p];
        return;
    }
    const int s = a.geo.s;
    for (int off = 0; off < cnt; off += (1 << s)) {
        const uint64_t g = (first + off) >> s;
        const uint64_t j = g >> (a.geo.b - s);
        const double delta = *(const double *)(a.din.hdr + 32 * j + 16);
        const double fac = a.din.bscale[j] * scale;  // fl(c_j s)
        decode_plane(a.arena_in + rec_at(a.din, 2 * g + p), s, delta, fac, fac != 1.0,
                     dst + off);
    }
}

__global__ __launch_bounds__(kWG) void k_inner(PassArgs A, PassArgs B,
                                               const double *ampA,
                                               const double *ampB, int S,
                                               uint64_t nranges, double *part)
{
    __shared__ __attribute__((aligned(16))) Planes X;
    __shared__ double lds[kWG];
    const int wave = threadIdx.x >> 6;
    const double sa = ampA ? 1.0 : A.dev->scale;
    const double sb = ampB ? 1.0 : B.dev->scale;
    for (uint64_t u = blockIdx.x; u < nranges; u += gridDim.x) {
        const uint64_t first = u << S;
        if (wave < 2)
            load_range(A, ampA, first, S, &X[0][wave][0], wave, sa);
        else
            load_range(B, ampB, first, S, &X[1][wave - 2][0], wave - 2, sb);
        __syncthreads();
        const uint64_t m = 1ull << S;
        for (int c = 0; c < 4; ++c) {
            const double v = wg_tree(
                [&](uint64_t o) {
                    const uint32_t so = sw((uint32_t)o);
                    const double ar = X[0][0][so], ai = X[0][1][so];
                    const double br = X[1][0][so], bi = X[1][1][so];
                    if (c == 0) {
                        const double p1 = ar * br, p2 = ai * bi;
                        return p1 + p2;
                    } else if (c == 1) {
                        const double p3 = ar * bi, p4 = ai * br;
                        return p3 - p4;
                    } else if (c == 2) {
                        const double q1 = ar * ar, q2 = ai * ai;
                        return q1 + q2;
                    }
                    const double q3 = br * br, q4 = bi * bi;
                    return q3 + q4;
                },
                m, lds);
            if (threadIdx.x == 0)
                part[(uint64_t)c * nranges + u] = v;
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(kWG) void k_inner_final(const double *part,
                                                     uint64_t nranges, double *res)
{
    __shared__ double lds[kWG];
    double v[4];
    for (int c = 0; c < 4; ++c) {
        const double *p = part + (uint64_t)c * nranges;
        v[c] = wg_tree([&](uint64_t i) { return p[i]; }, nranges, lds);
    }
    if (threadIdx.x == 0) {
        const double num = v[0] * v[0] + v[1] * v[1];
        res[0] = num / (v[2] * v[3]);
        res[1] = v[0];
        res[2] = v[1];
        res[3] = v[2];
        res[4] = v[3];
    }
}

// Overlap with a Fourier basis state: part[0..2][u] = pairwise over range u
// of re and im of e^(-2 pi i x k / 2^n) a_k and of |a_k|^2 (a = s * xhat, or
// amp when given).  The angle is formed from (x k) mod 2^n exactly.
__global__ __launch_bounds__(kWG) void k_fourier(PassArgs A, const double *amp, uint64_t x,
                                                 int S, uint64_t nranges, double *part)
{
    __shared__ __attribute__((aligned(16))) Planes X;
    __shared__ double lds[kWG];
    const int wave = threadIdx.x >> 6;
    const double sa = amp ? 1.0 : A.dev->scale;
    const int n = A.geo.n;
    const uint64_t mask = (n >= 64) ? ~0ull : ((1ull << n) - 1);
    const double inv = ldexp(1.0, 1 - n);
    for (uint64_t u = blockIdx.x; u < nranges; u += gridDim.x) {
        const uint64_t first = u << S;
        if (wave < 2)
            load_range(A, amp, first, S, &X[0][wave][0], wave, sa);
        __syncthreads();
        const uint64_t m = 1ull << S;
        for (int c = 0; c < 3; ++c) {
            const double v = wg_tree(
                [&](uint64_t o) {
                    const uint32_t so = sw((uint32_t)o);
                    const double ar = X[0][0][so], ai = X[0][1][so];
                    if (c == 2) {
                        const double q1 = ar * ar, q2 = ai * ai;
                        return q1 + q2;
                    }
                    const uint64_t r = (x * (first + o)) & mask;
                    double sn, cs;
                    sincospi((double)r * inv, &sn, &cs);
                    if (c == 0) {
                        const double p1 = cs * ar, p2 = sn * ai;
                        return p1 + p2;
                    }
                    const double p3 = cs * ai, p4 = sn * ar;
                    return p3 - p4;
                },
                m, lds);
            if (threadIdx.x == 0)
                part[(uint64_t)c * nranges + u] = v;
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(kWG) void k_fourier_final(const double *part, uint64_t nranges,
                                                       double *res)
{
    __shared__ double lds[kWG];
    for (int c = 0; c < 3; ++c) {
        const double *p = part + (uint64_t)c * nranges;
        const double v = wg_tree([&](uint64_t i) { return p[i]; }, nranges, lds);
        if (threadIdx.x == 0)
            res[c] = v;
    }
}

__global__ void k_rsqrt(const double *in, double *out, uint64_t count)
{
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < count;
         i += (uint64_t)gridDim.x * blockDim.x)
        out[i] = inv_sqrt_exact(in[i]);
}

// Canonical stream of block j (header + plane records in plane order) into
// `out` (one workgroup).
// Block j's canonical stream into out (its header, with the normsq field
// formed from the block's segment sums, then its plane records in plane
// order).  One workgroup; offs and red are workgroup scratch.
__device__ void export_body(const PassArgs &a, uint64_t j, uint8_t *out, uint64_t *offs,
                            uint64_t *poff, uint64_t *red, double *lds)
{
    const int t = threadIdx.x;
    const int s = a.geo.s;
    const uint64_t npb = 2ull << (a.geo.b - s);
    const uint32_t padC = pad8(1u << (s - 6));
    const uint64_t base = j * npb;
    const uint64_t per = (npb + kWG - 1) / kWG;
    // sizes of this thread's planes, from their record headers
    uint64_t local = 0;
    for (uint64_t q = t * per; q < (t + 1) * per && q < npb; ++q) {
        const uint64_t po = rec_at(a.din, base + q);
        const uint8_t *rec = a.arena_in + po;
        const uint32_t pw = *(const uint32_t *)(rec + 8);
        const uint32_t no = *(const uint32_t *)(rec + 12);
        const uint64_t sz = kPlaneHdrBytes + (pw ? padC : 0u) + 8ull * pw +
                            (uint64_t)kOutlierBytes * no;
        offs[q] = sz;
        poff[q] = po;
        local += sz;
    }
    red[t] = local;
    __syncthreads();
    for (int st = 1; st < kWG; st <<= 1) {
        const uint64_t add = t >= st ? red[t - st] : 0;
        __syncthreads();
        red[t] += add;
        __syncthreads();
    }
    // a block with a deferred scale carries it right after the header (its
    // header already has the flag and counts the 8 bytes)
    const double cj = a.din.bscale[j];
    const uint64_t rec0 = kHdrBytes + (cj != 1.0 ? kScaleBytes : 0u);
    uint64_t run = rec0 + red[t] - local;
    for (uint64_t q = t * per; q < (t + 1) * per && q < npb; ++q) {
        const uint64_t sz = offs[q];
        offs[q] = run;
        run += sz;
    }
    if (t < 3)
        ((uint64_t *)out)[t] = ((const uint64_t *)(a.din.hdr + 32 * j))[t];
    if (t == 3 && cj != 1.0)
        *(double *)(out + kHdrBytes) = cj;
    {
        // header normsq: pairwise over the block's segment sums
        const uint64_t spb = 1ull << (a.geo.b - s);
        const double *src = a.din.segnorm + j * spb;
        const double ns = wg_tree([&](uint64_t i) { return src[i]; }, spb, lds);
        if (t == 0)
            *(double *)(out + 24) = ns;
    }
    __syncthreads();
    const uint64_t nwords = ((uint64_t)a.din.blk_len[j] - rec0) / 8;
    if (nwords >= 32 * npb) {
        // records of 32 words or more on average: wave w copies records w,
        // w+4, ... with its 64 lanes
        const int wave = t >> 6, lane = lane_id();
        for (uint64_t q = wave; q < npb; q += 4) {
            const uint64_t *src = (const uint64_t *)(a.arena_in + poff[q]);
            const uint64_t end = (q + 1 < npb) ? offs[q + 1] : (uint64_t)a.din.blk_len[j];
            const uint64_t nw = (end - offs[q]) / 8;
            uint64_t *dst = (uint64_t *)(out + offs[q]);
            for (uint64_t k = lane; k < nw; k += 64)
                dst[k] = src[k];
        }
        __syncthreads();
        return;
    }
    // small records: the records as one run of words, thread t writing words
    // t, t+256, ... of the stream after the header (coalesced), each read
    // from the record holding it (binary search over the record starts)
    uint64_t *dst = (uint64_t *)(out + rec0);
    for (uint64_t k = t; k < nwords; k += kWG) {
        const uint64_t pos = rec0 + 8 * k;
        uint64_t lo = 0, hi = npb;  // offs[lo] <= pos < offs[hi] (offs[npb]: the end)
        while (hi - lo > 1) {
            const uint64_t mid = (lo + hi) >> 1;
            if (offs[mid] <= pos)
                lo = mid;
            else
                hi = mid;
        }
        dst[k] = *(const uint64_t *)(a.arena_in + poff[lo] + (pos - offs[lo]));
    }
    __syncthreads();
}

__global__ __launch_bounds__(kWG) void k_export(PassArgs a, uint64_t j, uint8_t *out)
{
    __shared__ uint64_t offs[2 << 10];  // planes per block: at most 2^(1 + 20 - 10)
    __shared__ uint64_t poff[2 << 10];
    __shared__ uint64_t red[kWG];
    __shared__ double lds[kWG];
    export_body(a, j, out, offs, poff, red, lds);
}

// Streams of blocks [first, first + count), block first + k at out + offs[k]
// (the exclusive prefix of their lengths): a whole-state checkpoint.
__global__ __launch_bounds__(kWG) void k_export_range(PassArgs a, uint64_t first,
                                                      uint64_t count,
                                                      const uint64_t *__restrict__ offs_out,
                                                      uint8_t *out)
{
    __shared__ uint64_t offs[2 << 10];
    __shared__ uint64_t poff[2 << 10];
    __shared__ uint64_t red[kWG];
    __shared__ double lds[kWG];
    for (uint64_t k = blockIdx.x; k < count; k += gridDim.x)
        export_body(a, first + k, out + offs_out[k], offs, poff, red, lds);
}

// ------------------------------------------------------ import ------------
//
// Checkpoint resume: concatenated block streams, copied into the arena that
// becomes the state's (arena_out, from kArenaBase on; block j's stream at
// kArenaBase + boff[j]), are turned into the descriptor set dout in place:
// every plane record stays where the copy put it.  The host has checked each
// block header (magic, s, b, level, delta, length within the buffer); these
// kernels check the records, and any failure sets an error bit that every
// later import kernel (and k_reduce) honours by doing nothing.

// One thread per block walks its plane records (each record's size follows
// from its own header), records where each one starts, and checks that the
// records fill the stream exactly and that their outlier counts add up to
// the header's.  Every read lies inside the block's stream: a record header
// is read only when 16 bytes remain, and a record is accepted only when it
// ends within the stream.
__global__ __launch_bounds__(kWG) void k_import_scan(PassArgs a, const uint64_t *__restrict__ boff)
{
    const uint64_t j = (uint64_t)blockIdx.x * kWG + threadIdx.x;
    if (j >= a.geo.nblocks)
        return;
    const int s = a.geo.s;
    const uint64_t npb = 2ull << (a.geo.b - s);
    const uint32_t C = 1u << (s - 6);
    const uint32_t padC = pad8(C);
    const uint8_t *base = a.arena_out;
    const uint64_t start = kArenaBase + boff[j];
    const uint64_t *h = (const uint64_t *)(base + start);
    const uint64_t h0 = h[0], h1 = h[1], h2 = h[2], h3 = h[3];
    uint64_t *hd = (uint64_t *)(a.dout.hdr + 32 * j);
    hd[0] = h0;
    hd[1] = h1;
    hd[2] = h2;
    hd[3] = h3;
    const uint32_t nout_hdr = (uint32_t)h1;
    const uint32_t total = (uint32_t)(h1 >> 32);
    a.dout.blk_len[j] = total;
    a.dout.blk_level[j] = (uint8_t)(h0 >> 32);
    const uint64_t end = start + total;
    // a deferred scale (checked by the host) sits between header and records
    const bool scaled = ((h0 >> 40) & kHdrScaled) != 0;
    a.dout.bscale[j] = scaled ? *(const double *)(base + start + kHdrBytes) : 1.0;
    uint64_t pos = start + kHdrBytes + (scaled ? kScaleBytes : 0u);
    uint64_t nsum = 0;
    bool ok = true;
    for (uint64_t q = 0; q < npb; ++q) {
        if (end - pos < kPlaneHdrBytes) {
            ok = false;
            break;
        }
        const uint64_t anc = *(const uint64_t *)(base + pos);
        const uint64_t v = *(const uint64_t *)(base + pos + 8);
        const uint32_t pw = (uint32_t)v, no = (uint32_t)(v >> 32);
        if (pw > 64u * C || no > (1u << s)) {
            ok = false;
            break;
        }
        const uint64_t sz = kPlaneHdrBytes + (pw ? padC : 0u) + 8ull * pw +
                            (uint64_t)kOutlierBytes * no;
        if (end - pos < sz) {
            ok = false;
            break;
        }
        // an all-zero record (anchor 0, no payload, no outliers) decodes to
        // all +0: point it at the shared zero record, as a pass does
        set_rec_at(a.dout, j * npb + q, (anc | v) == 0 ? 0 : pos);
        nsum += no;
        pos += sz;
    }
    if (!ok || pos != end || nsum != nout_hdr)
        atomicOr(&a.dev->err, kErrImport);
}

// One thread per plane record: the chunk widths (at most 32 bits for a lossy
// plane, 64 for a lossless one) sum to the payload words; the first residual
// of the plane is 0 (c_0 = 0 by definition); a lossy anchor is a code within
// +-(2^30 - 1); outlier indices lie in the plane and ascend strictly; a
// lossless plane has no outliers.  Reads stay inside the record, whose
// extent k_import_scan has checked.
__global__ __launch_bounds__(kWG) void k_import_check(PassArgs a)
{
    if (a.dev->err)
        return;
    const int s = a.geo.s, bs = a.geo.b - s;
    const uint32_t C = 1u << (s - 6);
    const uint32_t padC = pad8(C);
    const uint64_t nplanes = 2 * a.geo.nseg;
    for (uint64_t q = (uint64_t)blockIdx.x * kWG + threadIdx.x; q < nplanes;
         q += (uint64_t)gridDim.x * kWG) {
        const uint64_t off = rec_at(a.dout, q);
        if (off == 0)
            continue;
        const uint8_t *rec = a.arena_out + off;
        const int64_t anc = *(const int64_t *)rec;
        const uint32_t pw = *(const uint32_t *)(rec + 8);
        const uint32_t no = *(const uint32_t *)(rec + 12);
        const uint64_t j = (q >> 1) >> bs;
        const double delta = *(const double *)(a.dout.hdr + 32 * j + 16);
        const bool lossy = delta != 0.0;
        const int64_t qlim = (int64_t)kQMax;
        bool ok = lossy ? (anc >= -qlim && anc <= qlim) : no == 0;
        if (pw) {
            const uint32_t wmax = lossy ? 32u : 64u;
            uint32_t sum = 0;
            bool wok = true;
            for (uint32_t c = 0; c < C; ++c) {
                const uint32_t w = rec[kPlaneHdrBytes + c];
                sum += w;
                wok = wok && w <= wmax;
            }
            ok = ok && wok && sum == pw;
            const uint32_t w0 = rec[kPlaneHdrBytes];
            if (w0 && w0 <= 64u) {
                const uint64_t word0 = *(const uint64_t *)(rec + kPlaneHdrBytes + padC);
                const uint64_t m = w0 == 64u ? ~0ull : ((1ull << w0) - 1);
                ok = ok && (word0 & m) == 0;
            }
        }
        const uint8_t *ol = rec + kPlaneHdrBytes + (pw ? padC : 0u) + 8ull * pw;
        uint32_t last = 0;
        for (uint32_t k = 0; k < no; ++k) {
            const uint32_t idx = *(const uint32_t *)(ol + (uint64_t)kOutlierBytes * k);
            ok = ok && idx < (1u << s) && (k == 0 || idx > last);
            last = idx;
        }
        if (!ok)
            atomicOr(&a.dev->err, kErrImport);
    }
}

// Segment normsq of every unit, from the decoded (unscaled) values with the
// pass's own tree and leaf fl(fl(re^2) + fl(im^2)).  A unit whose records
// carry neither payload nor outliers holds one value per plane (the anchor's:
// its bit pattern, or code times 2 delta; +0 for the shared zero record), and
// the pairwise tree of 2^s equal leaves is 2^s times the leaf (each addition
// doubles): those units need no decode, as in the pass.  a.din/a.arena_in
// are the imported set (the same as dout).
__global__ __launch_bounds__(kWG) void k_import_norm(PassArgs a, uint32_t batch)
{
    if (a.dev->err)
        return;
    __shared__ __attribute__((aligned(16))) Planes X;
    __shared__ double red[8];
    __shared__ uint32_t list[kWG];
    __shared__ uint32_t nlist;
    const int s = a.geo.s, bs = a.geo.b - s;
    const uint64_t nu = a.geo.nunits;
    // `batch` units per round: one thread each settles a one-value unit on
    // its own; the others are queued and decoded by the whole workgroup
    for (uint64_t base = (uint64_t)blockIdx.x * batch; base < nu;
         base += (uint64_t)gridDim.x * batch) {
        if (threadIdx.x == 0)
            nlist = 0;
        __syncthreads();
        const uint64_t u = base + threadIdx.x;
        if (threadIdx.x < batch && u < nu) {
            const Unit uc = unit_of(u, a.geo.nseg, 0);
            uint64_t hv = 0;
            for (int i = 0; i < 2 * uc.nsu; ++i) {
                const uint64_t off = rec_at(a.din, 2 * uc.seg(i >> 1) + (i & 1));
                hv |= *(const uint64_t *)(a.arena_in + off + 8);  // payload words | outliers
            }
            if (hv == 0) {
                for (int k = 0; k < uc.nsu; ++k) {
                    const uint64_t g = uc.seg(k);
                    const double delta = *(const double *)(a.din.hdr + 32 * (g >> bs) + 16);
                    const double e = delta == 0.0 ? 0.0 : level_step(delta);
                    double v[2];
#pragma unroll
                    for (int p = 0; p < 2; ++p) {
                        const uint64_t off = rec_at(a.din, 2 * g + p);
                        const uint64_t anc = *(const uint64_t *)(a.arena_in + off);
                        v[p] = delta == 0.0 ? __longlong_as_double((long long)anc)
                                            : dequant((int32_t)(uint32_t)anc, delta, e);
                    }
                    const double rr = v[0] * v[0];
                    const double ii = v[1] * v[1];
                    a.din.segnorm[g] = (rr + ii) * (double)(1u << s);
                }
            } else {
                list[atomicAdd(&nlist, 1u)] = threadIdx.x;
            }
        }
        __syncthreads();
        const uint32_t cnt = nlist;
        for (uint32_t i = 0; i < cnt; ++i) {
            const Unit uc = unit_of(base + list[i], a.geo.nseg, 0);
            load_unit(a, uc, X, 1.0, false);
            __syncthreads();
            const double ns = s == kMaxS
                ? segment_tree10(uc, X, red, [](double re, double im) {
                      const double rr = re * re;
                      const double ii = im * im;
                      return rr + ii;
                  })
                : segment_tree(uc, s, red, [&](int su, int o) {
                      const double re = X[su][0][sw(o)], im = X[su][1][sw(o)];
                      const double rr = re * re;
                      const double ii = im * im;
                      return rr + ii;
                  });
            if (threadIdx.x < (unsigned)uc.nsu)
                a.din.segnorm[uc.seg((int)threadIdx.x)] = ns;
        }
        __syncthreads();
    }
}

// Block normsq (pairwise over the block's segment sums) for the reduction,
// checked bit for bit against the header's normsq field.
__global__ __launch_bounds__(kWG) void k_import_blocks(PassArgs a)
{
    if (a.dev->err)
        return;
    __shared__ double lds[kWG];
    const uint64_t spb = 1ull << (a.geo.b - a.geo.s);
    for (uint64_t j = blockIdx.x; j < a.geo.nblocks; j += gridDim.x) {
        const double *src = a.dout.segnorm + j * spb;
        const double v = wg_tree([&](uint64_t i) { return src[i]; }, spb, lds);
        if (threadIdx.x == 0) {
            // weight in N^2: times fl(c c) for a block with a deferred scale
            const double c = a.dout.bscale[j];
            double w = v;
            if (c != 1.0) {
                const double c2 = c * c;
                w = v * c2;
            }
            a.blknorm[j] = w;
            const uint64_t want = *(const uint64_t *)(a.dout.hdr + 32 * j + 24);
            if ((uint64_t)__double_as_longlong(v) != want)
                atomicOr(&a.dev->err, kErrImportNorm);
        }
    }
}

// Stream headers of blocks [first, first + count) into out[count][32], each
// with its normsq field (pairwise over the block's segment sums).
__global__ __launch_bounds__(kWG) void k_export_headers(PassArgs a, uint64_t first,
                                                        uint64_t count, uint8_t *out)
{
    __shared__ double lds[kWG];
    const uint64_t spb = 1ull << (a.geo.b - a.geo.s);
    for (uint64_t k = blockIdx.x; k < count; k += gridDim.x) {
        const uint64_t j = first + k;
        const double *src = a.din.segnorm + j * spb;
        const double ns = wg_tree([&](uint64_t i) { return src[i]; }, spb, lds);
        if (threadIdx.x < 3)
            ((uint64_t *)(out + 32 * k))[threadIdx.x] =
                ((const uint64_t *)(a.din.hdr + 32 * j))[threadIdx.x];
        if (threadIdx.x == 0)
            *(double *)(out + 32 * k + 24) = ns;
    }
}

// ------------------------------------------------------ batched pass ------
//
// One pass over many states at once: each state s has its own PassArgs
// (geometry, ladder, gate, buffers) in device memory and contributes
// pre[s+1] - pre[s] work items to the kernel's item range (0 for a state
// without a gate in this pass).  Items are handed out grid-stride; the state
// of an item is found by binary search over the prefix.  Everything a state
// computes is what the single-state kernels compute for it.

__device__ __forceinline__ uint32_t state_of(const uint64_t *__restrict__ pre, uint32_t nst,
                                             uint64_t it)
{
    uint32_t lo = 0, hi = nst;  // pre[lo] <= it < pre[hi]
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (pre[mid] <= it)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

template <bool SC>
__global__ __launch_bounds__(kWG) __attribute__((amdgpu_waves_per_eu(4, 4))) void k_bpass(
    const PassArgs *__restrict__ args, const uint64_t *__restrict__ upre, uint32_t nst)
{
    __shared__ PassLds S;
    for (int k = threadIdx.x; k < 4 * 4 * kPackRow; k += kWG)
        (&S.pack[0][0])[k] = 0u;
    const uint64_t total = upre[nst];
    uint32_t cur = ~0u;
    bool skip = false;
    double scale = 1.0, tdiff[2] = {0.0, 0.0};
    uint64_t Ms = 0;
    bool zp = false;
    uint64_t lo = 0, hi = 0;  // item range of state cur (a search only on leaving it)
    for (uint64_t it = blockIdx.x; it < total; it += gridDim.x) {
        uint32_t st = cur;
        if (it < lo || it >= hi) {
            st = state_of(upre, nst, it);
            lo = upre[st];
            hi = upre[st + 1];
        }
        const PassArgs &a = args[st];
        if (st != cur) {
            cur = st;
            if (threadIdx.x == 0)
                first_chunk(a, S);  // arena chunks belong to one state
            if (gridDim.x > a.scratch_wgs && threadIdx.x == 0)
                atomicOr(&a.dev->err, kErrSize);
            skip = a.dev->err != 0 || gridDim.x > a.scratch_wgs;
            scale = a.dev->scale;
            tdiff[0] = a.dev->tdiff[0];
            tdiff[1] = a.dev->tdiff[1];
            Ms = a.gate.mask >> a.geo.s;
            zp = zero_preserving(a.gate);
        }
        if (skip)
            continue;
        unit_body<kFused, SC>(a, unit_of(it - lo, a.geo.nseg, Ms), ~0ull, S, scale, tdiff,
                              zp);
        __syncthreads();
    }
}

__global__ __launch_bounds__(kWG) void k_bdecide(const PassArgs *__restrict__ args,
                                                 const uint64_t *__restrict__ bpre,
                                                 uint32_t nst)
{
    const uint64_t total = bpre[nst];
    const uint64_t nw = (uint64_t)gridDim.x * (kWG / 64);
    for (uint64_t it = (uint64_t)blockIdx.x * (kWG / 64) + (threadIdx.x >> 6); it < total;
         it += nw) {
        const uint32_t st = state_of(bpre, nst, it);
        const PassArgs &a = args[st];
        if (a.dev->err)
            continue;
        decide_block<-1>(a, it - bpre[st], hint_level(a, it - bpre[st]));
    }
}

// Every workgroup takes its share of the replay and escalation items of
// every state that has any.  The states are screened 64 at a time, one lane
// each; the resulting mask is the same in every wave.
template <bool SC>
__global__ __launch_bounds__(kWG) void k_bfix(const PassArgs *__restrict__ args,
                                              const uint64_t *__restrict__ upre, uint32_t nst)
{
    __shared__ PassLds S;
    for (int k = threadIdx.x; k < 4 * 4 * kPackRow; k += kWG)
        (&S.pack[0][0])[k] = 0u;
    for (uint32_t base = 0; base < nst; base += 64) {
        const uint32_t st = base + (uint32_t)lane_id();
        bool work = false;
        if (st < nst && upre[st + 1] != upre[st] && args[st].lad.L > 1) {
            const DevState *d = args[st].dev;
            work = d->err == 0 && d->n_replay + d->n_esc != 0;
        }
        uint64_t m = __ballot(work);
        while (m) {
            const int l = __builtin_ctzll(m);
            m &= m - 1;
            fix_body<SC>(args[base + l], blockIdx.x, gridDim.x, S);
            __syncthreads();
        }
    }
}

// One workgroup per state with a gate.
__global__ __launch_bounds__(kWG) void k_breduce(const PassArgs *__restrict__ args,
                                                 const uint64_t *__restrict__ upre)
{
    __shared__ double lds[kWG];
    __shared__ uint64_t ures[kWG];
    const uint32_t st = blockIdx.x;
    if (upre[st + 1] == upre[st])
        return;
    const DevState *d = args[st].dev;
    const uint32_t err = d->err, nrep = d->n_replay, nesc = d->n_esc;
    asm volatile("" ::"v"(err), "v"(nrep), "v"(nesc));
    if (err)
        return;
    reduce_body(args[st], lds, ures, nrep, nesc);
}

// DIFFUSE pre-pass of the states whose gate is DIFFUSE (items: units).
__global__ __launch_bounds__(kWG) void k_bmean(const PassArgs *__restrict__ args,
                                               const uint64_t *__restrict__ mpre, uint32_t nst)
{
    __shared__ __attribute__((aligned(16))) Planes X;
    __shared__ double red[8];
    const uint64_t total = mpre[nst];
    for (uint64_t it = blockIdx.x; it < total; it += gridDim.x) {
        const uint32_t st = state_of(mpre, nst, it);
        const PassArgs &a = args[st];
        if (a.dev->err)
            continue;
        mean_unit(a, it - mpre[st], X, red, a.dev->scale);
    }
}

// Block sums of both components (items: blocks of those states).
__global__ __launch_bounds__(kWG) void k_bmeantree(const PassArgs *__restrict__ args,
                                                   const uint64_t *__restrict__ mbpre,
                                                   uint32_t nst)
{
    __shared__ double lds[kWG];
    const uint64_t total = mbpre[nst];
    for (uint64_t it = blockIdx.x; it < total; it += gridDim.x) {
        const uint32_t st = state_of(mbpre, nst, it);
        const PassArgs &a = args[st];
        if (a.dev->err)
            continue;
        const uint64_t j = it - mbpre[st];
        const uint64_t spb = 1ull << (a.geo.b - a.geo.s);
        for (int c = 0; c < 2; ++c) {
            const double *src = a.segsum + (uint64_t)c * a.geo.nseg + j * spb;
            const double v = wg_tree([&](uint64_t i) { return src[i]; }, spb, lds);
            if (threadIdx.x == 0)
                a.blksum[(uint64_t)c * a.geo.nblocks + j] = v;
        }
    }
}

// 2 * mean of each DIFFUSE state (one workgroup per state).
__global__ __launch_bounds__(kWG) void k_bmeanfinal(const PassArgs *__restrict__ args,
                                                    const uint64_t *__restrict__ mpre)
{
    __shared__ double lds[kWG];
    const uint32_t st = blockIdx.x;
    if (mpre[st + 1] == mpre[st])
        return;
    const PassArgs &a = args[st];
    if (a.dev->err)
        return;
    const double mul = ldexp(1.0, 1 - a.geo.n);
    for (int c = 0; c < 2; ++c) {
        const double *p = a.blksum + (uint64_t)c * a.geo.nblocks;
        const double S = wg_tree([&](uint64_t i) { return p[i]; }, a.geo.nblocks, lds);
        if (threadIdx.x == 0)
            a.dev->tdiff[c] = S * mul;
    }
}

// ------------------------------------------------------- launchers --------

const char *const kKernelNames[kNumKernelIds] = {
    "pass", "decide", "esc_size", "esc_decide", "fix", "block_norm", "reduce",
    "mean", "mean_tree", "mean_final", "init_state", "sv_pair", "sv_diag",
    "sv_partial", "sv_final", "export", "import_scan", "import_check", "import_norm",
    "import_blocks", "pass_bulk"};

static unsigned grid_for(uint64_t items)
{
    const uint64_t cap = 1ull << 20;
    return (unsigned)(items < cap ? (items ? items : 1) : cap);
}

// Bracket one launch with the optional timer.
#define TIMED(prof, id, st, launch)                                              \
    do {                                                                         \
        if (prof)                                                                \
            (prof)->begin((id), (st));                                           \
        launch;                                                                  \
        if (prof)                                                                \
            (prof)->end((id), (st));                                             \
    } while (0)

__global__ void k_init_state(DevState *dev, int normalize, uint64_t arena_cap)
{
    if (threadIdx.x == 0) {
        DevState d = {};
        d.scale = 1.0;
        d.normalize = normalize;
        d.arena_used[0] = d.arena_used[1] = arena_start(arena_cap);
        *dev = d;
    }
}

void launch_init_state(DevState *dev, int normalize, uint64_t arena_cap, hipStream_t st,
                       Prof *prof)
{
    TIMED(prof, kIdInitState, st,
          hipLaunchKernelGGL(k_init_state, dim3(1), dim3(64), 0, st, dev, normalize,
                             arena_cap));
}

void launch_mean(const PassArgs &a, double mul, double *out, hipStream_t st, Prof *prof)
{
    PassArgs m = a;
    // up to 12288 workgroups: one unit each (the earlier launch shape); past
    // that, bulk rounds (unit_batch_for)
    const unsigned gm = grid_for(a.geo.nunits < 12288 ? a.geo.nunits : 12288);
    m.unit_batch = a.geo.nunits <= 12288 ? 1 : (int32_t)unit_batch_for(a.geo.nunits, gm);
    const unsigned gl = m.unit_batch > 1 ? gm : grid_for(a.geo.nunits);
    if (m.unit_batch > 1)
        TIMED(prof, kIdMean, st,
              hipLaunchKernelGGL(k_mean<true>, dim3(gl), dim3(kWG), 0, st, m));
    else
        TIMED(prof, kIdMean, st,
              hipLaunchKernelGGL(k_mean<false>, dim3(gl), dim3(kWG), 0, st, m));
    const uint64_t spb = 1ull << (a.geo.b - a.geo.s);
    for (int c = 0; c < 2; ++c)
        TIMED(prof, kIdMeanTree, st,
              hipLaunchKernelGGL(k_segtree, dim3(grid_for(a.geo.nblocks)), dim3(kWG), 0,
                                 st, m,
                                 (const double *)(a.segsum + (uint64_t)c * a.geo.nseg),
                                 a.blksum + (uint64_t)c * a.geo.nblocks, spb,
                                 a.geo.nblocks, 0));
    TIMED(prof, kIdMeanFinal, st,
          hipLaunchKernelGGL(k_mean_final, dim3(1), dim3(kWG), 0, st, m, mul, out));
}

uint64_t batch_chunk_bytes(uint64_t arena_cap, unsigned grid);

// Workgroups of a unit kernel over `units` units with at most `cap`: odd
// when the workgroups loop, so that units on a power-of-two stride spread
// over distinct workgroups instead of a 1/stride share of them.
unsigned unit_grid_for(uint64_t units, unsigned cap)
{
    if (units <= cap)
        return grid_for(units);
    return grid_for(cap > 1 ? ((cap - 1) | 1u) : 1u);
}

// The pass's reduction: one workgroup, or for more than 4096 blocks one
// workgroup per run of 1024 blocks (at most 256 workgroups, a power of two
// dividing the block count).
void launch_reduce(const PassArgs &a, hipStream_t st, Prof *prof)
{
    const uint64_t nb = a.geo.nblocks;
    if (nb <= 4096) {
        TIMED(prof, kIdReduce, st, hipLaunchKernelGGL(k_reduce, dim3(1), dim3(kWG), 0, st, a));
        return;
    }
    const uint64_t g = nb / 1024 < 256 ? nb / 1024 : 256;
    TIMED(prof, kIdReduce, st,
          hipLaunchKernelGGL(k_reduce_wide, dim3((unsigned)g), dim3(kWG), 0, st, a));
}

void launch_pass(const PassArgs &a0, unsigned grid_cap, hipStream_t st, Prof *prof)
{
    const unsigned gu = unit_grid_for(a0.geo.nunits, grid_cap);
    const unsigned gb = grid_for((a0.geo.nblocks + 3) / 4);
    // replays are a few blocks per pass at most; a small grid launches and
    // retires faster when there are none
    const unsigned gfix = gu < 256 ? gu : 256;
    PassArgs a = a0;
    a.chunk_bytes = batch_chunk_bytes(a.arena_cap, gu);
    a.unit_batch = (int32_t)unit_batch_for(a0.geo.nunits, gu);
    // states with many more units than workgroups: the bulk-round kernel
    // (every gate kind) beside the one-unit kernel, exactly one of which
    // runs (bulk_turn); the one-unit kernels have the one-value fast path
    // for DIFFUSE and PHASE_FLIP
    // the instances with the shortcut code only when this pass keeps blocks
    // or the state may hold scaled blocks
    const bool sc = a.sc_skip || a.sc_scaled || a.sc_rel;
    if (a.unit_batch > 1) {
        if (sc)
            TIMED(prof, kIdPassBulk, st,
                  hipLaunchKernelGGL((k_pass<true, true>), dim3(gu), dim3(kWG), 0, st, a));
        else
            TIMED(prof, kIdPassBulk, st,
                  hipLaunchKernelGGL((k_pass<true, false>), dim3(gu), dim3(kWG), 0, st, a));
    }
    if (a.gate.kind == kDiffuse || a.gate.kind == kPhaseFlip) {
        if (sc)
            TIMED(prof, kIdPass, st,
                  hipLaunchKernelGGL(k_pass_const<true>, dim3(gu), dim3(kWG), 0, st, a));
        else
            TIMED(prof, kIdPass, st,
                  hipLaunchKernelGGL(k_pass_const<false>, dim3(gu), dim3(kWG), 0, st, a));
    } else if (sc) {
        TIMED(prof, kIdPass, st,
              hipLaunchKernelGGL((k_pass<false, true>), dim3(gu), dim3(kWG), 0, st, a));
    } else {
        TIMED(prof, kIdPass, st,
              hipLaunchKernelGGL((k_pass<false, false>), dim3(gu), dim3(kWG), 0, st, a));
    }
    if ((2ull << (a.geo.b - a.geo.s)) % 256 == 0)
        TIMED(prof, kIdDecide, st,
              hipLaunchKernelGGL(k_decide<1>, dim3(gb), dim3(kWG), 0, st, a));
    else
        TIMED(prof, kIdDecide, st,
              hipLaunchKernelGGL(k_decide<0>, dim3(gb), dim3(kWG), 0, st, a));
    if (a.lad.L > 1) {
        if (sc)
            TIMED(prof, kIdReplay, st,
                  hipLaunchKernelGGL(k_fix<true>, dim3(gfix), dim3(kWG), 0, st, a));
        else
            TIMED(prof, kIdReplay, st,
                  hipLaunchKernelGGL(k_fix<false>, dim3(gfix), dim3(kWG), 0, st, a));
    }
    launch_reduce(a, st, prof);
}

void launch_batch_pass(const BatchLaunch &b, hipStream_t st, Prof *prof)
{
    if (b.any_mean) {
        TIMED(prof, kIdMean, st,
              hipLaunchKernelGGL(k_bmean, dim3(b.grid_units), dim3(kWG), 0, st, b.args, b.mpre,
                                 b.nst));
        TIMED(prof, kIdMeanTree, st,
              hipLaunchKernelGGL(k_bmeantree, dim3(b.grid_blocks), dim3(kWG), 0, st, b.args,
                                 b.mbpre, b.nst));
        TIMED(prof, kIdMeanFinal, st,
              hipLaunchKernelGGL(k_bmeanfinal, dim3(b.nst), dim3(kWG), 0, st, b.args, b.mpre));
    }
    if (b.any_sc)
        TIMED(prof, kIdPass, st,
              hipLaunchKernelGGL(k_bpass<true>, dim3(b.grid_units), dim3(kWG), 0, st, b.args,
                                 b.upre, b.nst));
    else
        TIMED(prof, kIdPass, st,
              hipLaunchKernelGGL(k_bpass<false>, dim3(b.grid_units), dim3(kWG), 0, st, b.args,
                                 b.upre, b.nst));
    TIMED(prof, kIdDecide, st,
          hipLaunchKernelGGL(k_bdecide, dim3((b.grid_blocks + 3) / 4), dim3(kWG), 0, st,
                             b.args, b.bpre, b.nst));
    if (b.any_ladder && b.any_sc)
        TIMED(prof, kIdReplay, st,
              hipLaunchKernelGGL(k_bfix<true>, dim3(b.grid_units), dim3(kWG), 0, st, b.args,
                                 b.upre, b.nst));
    else if (b.any_ladder)
        TIMED(prof, kIdReplay, st,
              hipLaunchKernelGGL(k_bfix<false>, dim3(b.grid_units), dim3(kWG), 0, st, b.args,
                                 b.upre, b.nst));
    TIMED(prof, kIdReduce, st,
          hipLaunchKernelGGL(k_breduce, dim3(b.nst), dim3(kWG), 0, st, b.args, b.upre));
}

uint64_t batch_chunk_bytes(uint64_t arena_cap, unsigned grid)
{
    uint64_t chunk = arena_cap / (8ull * grid);
    chunk = chunk > 32768 ? 32768 : chunk;
    chunk &= ~255ull;
    return chunk < 256 ? 256 : chunk;
}

void launch_encode_basis(const PassArgs &a, unsigned grid_cap, hipStream_t st, Prof *prof)
{
    launch_pass(a, grid_cap, st, prof);
}

void launch_decode_range(const PassArgs &a, uint64_t first, uint64_t count,
                         double *out, hipStream_t st)
{
    const int s = a.geo.s;
    uint64_t u0, u1;
    if (a.geo.nseg == 1) {
        u0 = 0;
        u1 = 1;
    } else {
        u0 = (first >> s) >> 1;
        u1 = (((first + count - 1) >> s) >> 1) + 1;
    }
    hipLaunchKernelGGL(k_decode_range, dim3(grid_for(u1 - u0)), dim3(kWG), 0, st, a, u0,
                       u1, first, count, out);
}

void launch_probs(const PassArgs &a, const int *qubits_dev, int nq, double *probs_dev,
                  hipStream_t st)
{
    hipLaunchKernelGGL(k_probs, dim3(grid_for(a.geo.nunits)), dim3(kWG), 0, st, a,
                       qubits_dev, nq, probs_dev);
}

void launch_inner(const PassArgs &a, const PassArgs &b, const double *amp_a,
                  const double *amp_b, double *part, double *result, hipStream_t st)
{
    const int n = a.geo.n;
    int S = kMaxS;
    if (S > n)
        S = n;
    const uint64_t nr = 1ull << (n - S);
    hipLaunchKernelGGL(k_inner, dim3(grid_for(nr)), dim3(kWG), 0, st, a, b, amp_a, amp_b,
                       S, nr, part);
    hipLaunchKernelGGL(k_inner_final, dim3(1), dim3(kWG), 0, st, (const double *)part, nr,
                       result);
}

void launch_fourier(const PassArgs &a, const double *amp, uint64_t x, double *part,
                    double *result, hipStream_t st)
{
    const int n = a.geo.n;
    const int S = n < kMaxS ? n : kMaxS;
    const uint64_t nr = 1ull << (n - S);
    hipLaunchKernelGGL(k_fourier, dim3(grid_for(nr)), dim3(kWG), 0, st, a, amp, x, S, nr,
                       part);
    hipLaunchKernelGGL(k_fourier_final, dim3(1), dim3(kWG), 0, st, (const double *)part, nr,
                       result);
}

void launch_rsqrt(const double *in, double *out, uint64_t count, hipStream_t st)
{
    hipLaunchKernelGGL(k_rsqrt, dim3(grid_for((count + kWG - 1) / kWG)), dim3(kWG), 0, st,
                       in, out, count);
}

void launch_export(const PassArgs &a, uint64_t j, uint8_t *out, hipStream_t st)
{
    hipLaunchKernelGGL(k_export, dim3(1), dim3(kWG), 0, st, a, j, out);
}

void launch_export_range(const PassArgs &a, uint64_t first, uint64_t count,
                         const uint64_t *offs, uint8_t *out, hipStream_t st, Prof *prof)
{
    TIMED(prof, kIdExport, st,
          hipLaunchKernelGGL(k_export_range, dim3(grid_for(count < 4096 ? count : 4096)),
                             dim3(kWG), 0, st, a, first, count, offs, out));
}

void launch_import(const PassArgs &a0, const uint64_t *boff, hipStream_t st, Prof *prof)
{
    // a: din = dout = the imported set, arena_in = arena_out = its arena; the
    // reduction alone runs as a state encode (no pass counted)
    PassArgs a = a0;
    a.src_basis = 0;
    PassArgs r = a0;
    r.src_basis = 1;
    TIMED(prof, kIdImportScan, st,
          hipLaunchKernelGGL(k_import_scan, dim3(grid_for((a.geo.nblocks + kWG - 1) / kWG)),
                             dim3(kWG), 0, st, a, boff));
    const uint64_t np = 2 * a.geo.nseg;
    const uint64_t gq = (np + kWG - 1) / kWG;
    TIMED(prof, kIdImportCheck, st,
          hipLaunchKernelGGL(k_import_check, dim3(grid_for(gq < 4096 ? gq : 4096)), dim3(kWG),
                             0, st, a));
    // units per workgroup round: enough that a grid of about 3072
    // workgroups covers the state, at most one per thread
    uint32_t batch = 1;
    while (batch < (uint32_t)kWG && (uint64_t)batch * 2 * 3072 <= a.geo.nunits)
        batch *= 2;
    const uint64_t rounds = (a.geo.nunits + batch - 1) / batch;
    const uint64_t gu = rounds < 12288 ? rounds : 12288;
    TIMED(prof, kIdImportNorm, st,
          hipLaunchKernelGGL(k_import_norm, dim3(grid_for(gu)), dim3(kWG), 0, st, a, batch));
    TIMED(prof, kIdImportBlocks, st,
          hipLaunchKernelGGL(k_import_blocks,
                             dim3(grid_for(a.geo.nblocks < 4096 ? a.geo.nblocks : 4096)),
                             dim3(kWG), 0, st, a));
    launch_reduce(r, st, prof);
}

void launch_export_headers(const PassArgs &a, uint64_t first, uint64_t count, uint8_t *out,
                           hipStream_t st)
{
    hipLaunchKernelGGL(k_export_headers, dim3(grid_for(count)), dim3(kWG), 0, st, a, first,
                       count, out);
}


// ------------------------------------------- allocation-free marginals ----
//
// sim_measure_probs_noalloc runs the probability kernels with their outcome
// bins and qubit list in this file-scope array instead of device memory
// allocated per call.  Each GPU holds its own copy until the process ends.
// In host code the array's name is only a stand-in: its device address on
// the current GPU comes from hipGetSymbolAddress, taken once per device and
// kept in g_noalloc_ptr; kernels, fills and copies use that address.  Every
// call on one GPU shares the array, so calls that overlap on one GPU race.
static __device__ __align__(256) uint8_t scratch[kNoAllocBytes];

namespace {
constexpr int kNoAllocDevices = 64;
std::mutex g_noalloc_mu;
void *g_noalloc_ptr[kNoAllocDevices] = {};
}  // namespace

std::mutex g_stage_mu;
uint8_t *g_stage_ptr[kNoAllocDevices] = {};

hipError_t slot_staging(int device, uint8_t **ptr)
{
    *ptr = nullptr;
    if (device < 0 || device >= kNoAllocDevices)
        return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_stage_mu);
    if (!g_stage_ptr[device]) {
        void *p = nullptr;
        const hipError_t e = hipMalloc(&p, kHwSlots * kScratchWave);
        if (e != hipSuccess)
            return e;
        g_stage_ptr[device] = (uint8_t *)p;
    }
    *ptr = g_stage_ptr[device];
    return hipSuccess;
}

hipError_t noalloc_scratch(int device, void **ptr)
{
    *ptr = nullptr;
    if (device < 0 || device >= kNoAllocDevices)
        return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_noalloc_mu);
    if (!g_noalloc_ptr[device]) {
        int cur = -1;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess)
            return e;
        if (cur != device)
            return hipErrorInvalidDevice;  // the caller makes `device` current
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess)
            return e;
        g_noalloc_ptr[device] = p;
    }
    *ptr = g_noalloc_ptr[device];
    return hipSuccess;
}

__global__ void k_zero_f64(double *p, uint64_t count)
{
    for (uint64_t k = blockIdx.x * (uint64_t)kWG + threadIdx.x; k < count;
         k += (uint64_t)gridDim.x * kWG)
        p[k] = 0.0;
}

void launch_zero_f64(double *p, uint64_t count, hipStream_t st)
{
    const uint64_t g = (count + kWG - 1) / kWG;
    hipLaunchKernelGGL(k_zero_f64, dim3(grid_for(g < 1024 ? g : 1024)), dim3(kWG), 0, st, p,
                       count);
}

}  // namespace aalc
