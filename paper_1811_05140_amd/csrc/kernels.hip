// kernels.hip -- gfx950 kernels of the compressed path.
//
// One pass of a gate runs Alg. 2 of the paper (decompress, normalise,
// gateComputation, compress at delta_0, delta_1, ... until the ratio reaches
// theta) for every stride, as these kernels on the sim stream:
//   k_pass<kFused>   per unit of two segments: decode + normalise + gate in
//                    LDS; the size of each plane record at the ladder levels
//                    the block can plausibly take (0 .. previous level + 1);
//                    encode at the block's previous level (the speculation),
//                    write the records, per-segment normsq
//   k_decide<false>  per block: the first computed level whose ratio reaches
//                    theta; a block whose choice differs from the speculation
//                    joins the replay list, one whose computed levels all
//                    miss theta joins the escalation list
//   k_pass<kEsc>     escalated blocks only: sizes of the remaining levels
//   k_decide<true>   escalated blocks: the choice among the remaining levels
//   k_pass<kReplay>  replayed blocks only: encode again at the chosen level
//   k_segtree        per block: pairwise normsq into the stream header
//   k_reduce         N^2 over blocks, s = 1/sqrt(N^2), statistics
// The level chosen is always exactly the one of Alg. 2 (the first level
// whose full-block ratio reaches theta, else the last); speculation only
// decides which records have to be written twice.  DIFFUSE adds a read-only
// mean pre-pass (k_mean + k_segtree + k_mean_final).
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

// Decode one plane record into dst[0 .. 2^s) (one wavefront, one chunk of
// 64 scalars per step), scaling each value by `scale` when do_scale
// (normalisation before the gate).  Lossy planes run the prefix sum in 32
// bits: within a chunk the partial sums are differences of two codes of
// magnitude below 2^30, so they are exact.
__device__ void decode_plane(const uint8_t *rec, int s, double delta,
                             double scale, bool do_scale, double *dst)
{
    const int lane = lane_id();
    const int C = 1 << (s - 6);
    const uint64_t anchor = *(const uint64_t *)rec;
    const uint32_t pw = *(const uint32_t *)(rec + 8);
    const uint32_t nout = *(const uint32_t *)(rec + 12);
    const uint8_t *widths = rec + kPlaneHdrBytes;
    const uint64_t *payload =
        (const uint64_t *)(rec + kPlaneHdrBytes + (pw ? pad8((uint32_t)C) : 0u));
    const double e = 2.0 * delta;
    uint64_t carry = anchor;
    uint32_t woff = 0;
    for (int c = 0; c < C; ++c) {
        const uint32_t w = pw ? (uint32_t)widths[c] : 0u;
        uint64_t z = 0;
        if (w) {
            const uint32_t bp = (uint32_t)lane * w;
            const uint32_t wi = bp >> 6, sh = bp & 63u;
            uint64_t v = payload[woff + wi] >> sh;
            if (sh + w > 64u)
                v |= payload[woff + wi + 1] << (64u - sh);
            if (w < 64u)
                v &= (1ull << w) - 1ull;
            z = v;
        }
        double x;
        if (delta == 0.0) {
            const uint64_t q = carry + wave_scan64(unzigzag64(z));
            carry = readlane64(q, 63);
            x = __longlong_as_double((long long)q);
        } else {
            const uint32_t z32 = (uint32_t)z;
            const uint32_t d = (z32 >> 1) ^ (0u - (z32 & 1u));
            const int32_t part = (int32_t)wave_scan32(d);
            const int64_t q = (int64_t)carry + (int64_t)part;
            carry = (uint64_t)(int64_t)__builtin_amdgcn_readlane((int)(int32_t)q, 63);
            x = (double)q * e;
        }
        if (do_scale)
            x = x * scale;
        dst[c * kChunk + lane] = x;
        woff += w;
    }
    const uint8_t *outl = (const uint8_t *)(payload + pw);
    for (uint32_t k = (uint32_t)lane; k < nout; k += 64u) {
        const uint32_t idx = *(const uint32_t *)(outl + (uint64_t)kOutlierBytes * k);
        double v = *(const double *)(outl + (uint64_t)kOutlierBytes * k + 8);
        if (do_scale)
            v = v * scale;
        dst[idx] = v;
    }
}

// Decode (or synthesise, for the basis-state source) the planes of a unit
// into LDS; wave w owns plane (w & 1) of segment (w >> 1).
__device__ void load_unit(const PassArgs &a, const Unit &uc, Planes &X,
                          double scale, bool do_scale)
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
            dst[o] = (p == 0 && ((g << s) | (uint64_t)o) == a.basis) ? 1.0 : 0.0;
        return;
    }
    const uint64_t j = g >> (a.geo.b - s);
    const double delta = *(const double *)(a.din.hdr + 32 * j + 16);
    decode_plane(a.arena_in + a.din.plane_off[2 * g + p], s, delta, scale, do_scale, dst);
}

__device__ void gate_unit(const GateArg &G, const Unit &uc, int s, Planes &X,
                          const double *tdiff)
{
    const int tid = threadIdx.x;
    if (G.kind == kNone)
        return;
    const uint64_t M = G.mask;
    const uint64_t Ms = M >> s;
    const uint32_t S = 1u << s;
    const uint32_t Ml = (uint32_t)(M & (S - 1));
    if (M == 0) {
        const uint32_t total = (uint32_t)uc.nsu << s;
        for (uint32_t t = tid; t < total; t += kWG) {
            const int us = (int)(t >> s);
            const uint32_t o = t & (S - 1);
            const uint64_t i = (uc.seg(us) << s) | o;
            double ar = X[us][0][o], ai = X[us][1][o];
            gate_diag(G, i, ar, ai, tdiff);
            X[us][0][o] = ar;
            X[us][1][o] = ai;
        }
    } else if (Ms) {
        for (uint32_t o = tid; o < S; o += kWG) {
            const uint32_t o2 = o ^ Ml;
            const uint64_t i = (uc.g[0] << s) | o;
            double ar = X[0][0][o], ai = X[0][1][o];
            double br = X[1][0][o2], bi = X[1][1][o2];
            gate_pair(G, i, ar, ai, br, bi);
            X[0][0][o] = ar;
            X[0][1][o] = ai;
            X[1][0][o2] = br;
            X[1][1][o2] = bi;
        }
    } else {
        const int hb = 31 - __builtin_clz(Ml);
        const uint32_t half = S >> 1;
        const uint32_t total = (uint32_t)uc.nsu * half;
        for (uint32_t t = tid; t < total; t += kWG) {
            const int us = (int)(t >> (s - 1));
            const uint32_t r = t & (half - 1);
            const uint32_t o = ((r >> hb) << (hb + 1)) | (r & ((1u << hb) - 1));
            const uint32_t o2 = o ^ Ml;
            const uint64_t i = (uc.seg(us) << s) | o;
            double ar = X[us][0][o], ai = X[us][1][o];
            double br = X[us][0][o2], bi = X[us][1][o2];
            gate_pair(G, i, ar, ai, br, bi);
            X[us][0][o] = ar;
            X[us][1][o] = ai;
            X[us][0][o2] = br;
            X[us][1][o2] = bi;
        }
    }
}

// Lossy code of one scalar at one level: q the int32 code, `out` the outlier
// flag, xh the value a decoder reconstructs (the scalar itself for outliers).
__device__ __forceinline__ void lossy_code(double x, double delta, double e, double r,
                                           int32_t &q, bool &out, double &xh)
{
    const double y = x * r;
    if (fabs(y) < kQMax) {
        const double qr = __builtin_rint(y);
        q = (int32_t)qr;
        xh = qr * e;
        out = !(fabs(x - xh) < delta);
        if (out)
            xh = x;
    } else {
        q = 0;
        out = true;
        xh = x;
    }
}

__device__ __forceinline__ uint32_t zigzag32(int32_t d)
{
    return ((uint32_t)d << 1) ^ (uint32_t)(d >> 31);
}

__device__ __forceinline__ uint32_t bitlen32(uint32_t z)
{
    return z ? 32u - (uint32_t)__builtin_clz(z) : 0u;
}

// Sizes of one plane at ladder levels k0 .. k1 (one wavefront; levels outer
// so that only one level's state is live).  Returns the (payload words,
// outliers) word of level `want` when it lies in the range.
__device__ uint32_t size_levels(const double *x, int s, const Ladder &lad, int k0, int k1,
                                int want, uint32_t *psz, uint64_t plane, uint64_t nplanes)
{
    const int lane = lane_id();
    const int C = 1 << (s - 6);
    uint32_t wanted = 0;
    for (int k = k0; k <= k1; ++k) {
        const double delta = lad.delta[k];
        uint32_t pw = 0, no = 0;
        if (delta == 0.0) {
            uint64_t carry = 0;
            for (int c = 0; c < C; ++c) {
                const uint64_t q = (uint64_t)__double_as_longlong(x[c * kChunk + lane]);
                const uint64_t prev = dpp64<kWaveShr1>(c == 0 ? q : carry, q);
                pw += wave_max32(bitlen64(zigzag64(q - prev)));
                carry = readlane64(q, 63);
            }
        } else {
            const double e = lad.e[k], r = lad.r[k];
            int32_t carry = 0;
            for (int c = 0; c < C; ++c) {
                int32_t q;
                bool out;
                double xh;
                lossy_code(x[c * kChunk + lane], delta, e, r, q, out, xh);
                const int32_t prev = (int32_t)dpp32<kWaveShr1>(
                    (uint32_t)(c == 0 ? q : carry), (uint32_t)q);
                pw += wave_max32(bitlen32(zigzag32(q - prev)));
                no += (uint32_t)__popcll(__ballot(out));
                carry = __builtin_amdgcn_readlane(q, 63);
            }
        }
        const uint32_t v = pw | (no << 16);
        if (lane == 0)
            psz[(uint64_t)k * nplanes + plane] = v;
        if (k == want)
            wanted = v;
    }
    return wanted;
}

// Scatter one chunk's fields (z of width w, lane l at bits [l w, l w + w))
// into w payload words through the wave's LDS word buffer.
__device__ __forceinline__ void pack_chunk(uint64_t z, uint32_t w, uint64_t *pb,
                                           uint64_t *dst)
{
    const int lane = lane_id();
    if (w == 64u) {
        dst[lane] = z;
        return;
    }
    if ((uint32_t)lane < w)
        pb[lane] = 0;
    __builtin_amdgcn_wave_barrier();
    const uint32_t bp = (uint32_t)lane * w;
    const uint32_t wi = bp >> 6, sh = bp & 63u;
    if (z) {
        atomicOr((unsigned long long *)&pb[wi], (unsigned long long)(z << sh));
        if (sh + w > 64u)
            atomicOr((unsigned long long *)&pb[wi + 1], (unsigned long long)(z >> (64u - sh)));
    }
    __builtin_amdgcn_wave_barrier();
    if ((uint32_t)lane < w)
        dst[lane] = pb[lane];
    __builtin_amdgcn_wave_barrier();
}

// Encode one plane at one level into its record (one wavefront).  x is
// overwritten with the decoded values x-hat for the normsq.
__device__ void encode_plane(double *x, int s, double delta, double e,
                             double r, uint32_t pszv, uint8_t *rec,
                             uint64_t *pb, uint32_t *err)
{
    const int lane = lane_id();
    const int C = 1 << (s - 6);
    const uint32_t pw_total = pszv & 0xFFFFu, nout_total = pszv >> 16;
    uint8_t *widths = rec + kPlaneHdrBytes;
    uint64_t *payload =
        (uint64_t *)(rec + kPlaneHdrBytes + (pw_total ? pad8((uint32_t)C) : 0u));
    uint8_t *outl = (uint8_t *)(payload + pw_total);
    const uint64_t lt_mask = (1ull << lane) - 1ull;
    uint32_t woff = 0, nout = 0;
    if (delta == 0.0) {
        uint64_t carry = 0;
        for (int c = 0; c < C; ++c) {
            const uint64_t q = (uint64_t)__double_as_longlong(x[c * kChunk + lane]);
            const uint64_t prev = dpp64<kWaveShr1>(c == 0 ? q : carry, q);
            const uint64_t z = zigzag64(q - prev);
            const uint32_t w = wave_max32(bitlen64(z));
            if (c == 0 && lane == 0) {
                *(uint64_t *)rec = q;
                *(uint32_t *)(rec + 8) = pw_total;
                *(uint32_t *)(rec + 12) = nout_total;
            }
            if (pw_total && lane == 0)
                widths[c] = (uint8_t)w;
            if (w && woff + w <= pw_total)
                pack_chunk(z, w, pb, payload + woff);
            carry = readlane64(q, 63);
            woff += w;
        }
    } else {
        int32_t carry = 0;
        for (int c = 0; c < C; ++c) {
            const double v = x[c * kChunk + lane];
            int32_t q;
            bool out;
            double xh;
            lossy_code(v, delta, e, r, q, out, xh);
            const int32_t prev =
                (int32_t)dpp32<kWaveShr1>((uint32_t)(c == 0 ? q : carry), (uint32_t)q);
            const uint32_t z = zigzag32(q - prev);
            const uint32_t w = wave_max32(bitlen32(z));
            if (c == 0 && lane == 0) {
                *(int64_t *)rec = (int64_t)q;
                *(uint32_t *)(rec + 8) = pw_total;
                *(uint32_t *)(rec + 12) = nout_total;
            }
            if (pw_total && lane == 0)
                widths[c] = (uint8_t)w;
            if (w && woff + w <= pw_total)
                pack_chunk((uint64_t)z, w, pb, payload + woff);
            const uint64_t bal = __ballot(out);
            if (out) {
                const uint32_t rank = nout + (uint32_t)__popcll(bal & lt_mask);
                if (rank < nout_total) {
                    uint8_t *ent = outl + (uint64_t)kOutlierBytes * rank;
                    *(uint32_t *)ent = (uint32_t)(c * kChunk + lane);
                    *(uint32_t *)(ent + 4) = 0u;
                    *(uint64_t *)(ent + 8) = (uint64_t)__double_as_longlong(v);
                }
            }
            nout += (uint32_t)__popcll(bal);
            x[c * kChunk + lane] = xh;
            carry = __builtin_amdgcn_readlane(q, 63);
            woff += w;
        }
    }
    if (pw_total && lane == 0)
        for (int i = C; i < (int)pad8((uint32_t)C); ++i)
            widths[i] = 0;
    if (lane == 0 && (woff != pw_total || nout != nout_total))
        atomicOr(err, kErrSize);
}

// Pairwise sums of a unit's segments: leaf(o) for the amplitudes of segment
// us, tree over o; the two waves of a segment each reduce one half.
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

template <int MODE>
__global__ __launch_bounds__(kWG) void k_pass(PassArgs a)
{
    if (a.dev->err)
        return;
    __shared__ Planes X;
    __shared__ uint64_t pack[4][64];
    __shared__ double red[8];
    __shared__ uint64_t rbytes[4];
    __shared__ uint64_t rbase;
    const int s = a.geo.s;
    const int wave = threadIdx.x >> 6, lane = lane_id();
    const int us = wave >> 1, p = wave & 1;
    const int L = a.lad.L;
    const double scale = a.dev->scale;
    const bool do_scale = !a.src_basis && scale != 1.0;
    const double *tdiff = a.dev->tdiff;
    const uint64_t Ms = a.gate.mask >> s;
    const uint64_t nplanes = 2 * a.geo.nseg;
    const int bs = a.geo.b - s;
    const uint64_t spb = 1ull << bs;
    const uint32_t padC = pad8(1u << (s - 6));
    uint64_t nitems;
    const uint32_t *list = nullptr;
    if (MODE == kFused) {
        nitems = a.geo.nunits;
    } else {
        const uint32_t cnt = MODE == kEsc ? a.dev->n_esc : a.dev->n_replay;
        list = MODE == kEsc ? a.esc_list : a.replay_list;
        nitems = (uint64_t)cnt << bs;
    }
    for (uint64_t it = blockIdx.x; it < nitems; it += gridDim.x) {
        Unit uc;
        uint64_t jsel = ~0ull;  // the block this item works for (kEsc, kReplay)
        if (MODE == kFused) {
            uc = unit_of(it, a.geo.nseg, Ms);
        } else {
            jsel = list[it >> bs];
            const uint64_t g = (jsel << bs) | (it & (spb - 1));
            uc = unit_of_seg(g, a.geo.nseg, Ms);
            // one item per (unit, block): skip when the unit's other segment
            // lies in the same block and comes first
            const uint64_t other = uc.nsu == 2 ? (uc.g[0] == g ? uc.g[1] : uc.g[0]) : g;
            if ((other >> bs) == jsel && other < g)
                continue;
        }
        load_unit(a, uc, X, scale, do_scale);
        __syncthreads();
        gate_unit(a.gate, uc, s, X, tdiff);
        __syncthreads();
        const bool active = us < uc.nsu;
        const uint64_t g = active ? uc.seg(us) : 0;
        const uint64_t j = g >> bs;
        const uint64_t plane = 2 * g + p;
        const bool mine = active && (MODE == kFused || j == jsel);
        int lev = 0;
        uint32_t pszv = 0;
        if (mine) {
            const int h = hint_level(a, j);
            const int cm = h + 1 < L ? h + 1 : L - 1;
            if (MODE == kFused) {
                lev = h;
                pszv = size_levels(&X[us][p][0], s, a.lad, 0, cm, h, a.psz, plane, nplanes);
            } else if (MODE == kEsc) {
                size_levels(&X[us][p][0], s, a.lad, cm + 1, L - 1, -1, a.psz, plane, nplanes);
            } else {
                lev = a.dout.blk_level[j];
                pszv = a.psz[(uint64_t)lev * nplanes + plane];
            }
        }
        if (MODE != kEsc) {
            // bump-allocate this unit's records in the output arena
            if (lane == 0)
                rbytes[wave] = mine ? rec_bytes(pszv, padC) : 0;
            __syncthreads();
            if (threadIdx.x == 0) {
                const uint64_t tot = rbytes[0] + rbytes[1] + rbytes[2] + rbytes[3];
                uint64_t base = 0;
                if (tot) {
                    base = atomicAdd((unsigned long long *)&a.dev->arena_used[a.out_arena],
                                     (unsigned long long)tot);
                    if (base + tot > a.arena_cap) {
                        if (atomicOr(&a.dev->err, kErrArena) == 0)
                            a.dev->err_pass = (uint32_t)a.pass;
                        base = ~0ull;
                    } else {
                        atomicMax((unsigned long long *)&a.dev->arena_peak,
                                  (unsigned long long)(base + tot));
                    }
                }
                rbase = base;
            }
            __syncthreads();
            if (mine && rbase != ~0ull) {
                uint64_t off = rbase;
                for (int w2 = 0; w2 < wave; ++w2)
                    off += rbytes[w2];
                if (lane == 0)
                    a.dout.plane_off[plane] = off;
                encode_plane(&X[us][p][0], s, a.lad.delta[lev], a.lad.e[lev], a.lad.r[lev],
                             pszv, a.arena_out + off, &pack[wave][0], &a.dev->err);
            }
            __syncthreads();
            const double ns = segment_tree(uc, s, red, [&](int su, int o) {
                const double re = X[su][0][o], im = X[su][1][o];
                const double rr = re * re;
                const double ii = im * im;
                return rr + ii;
            });
            if (threadIdx.x < (unsigned)uc.nsu) {
                const uint64_t gs = uc.seg((int)threadIdx.x);
                if (MODE == kFused || (gs >> bs) == jsel)
                    a.segnorm[gs] = ns;
            }
        }
        __syncthreads();
    }
}

// Read-only DIFFUSE pre-pass: per-segment pairwise sums of the normalised
// re and im parts.
__global__ __launch_bounds__(kWG) void k_mean(PassArgs a)
{
    if (a.dev->err)
        return;
    __shared__ Planes X;
    __shared__ double red[8];
    const int s = a.geo.s;
    const double scale = a.dev->scale;
    const bool do_scale = scale != 1.0;
    for (uint64_t u = blockIdx.x; u < a.geo.nunits; u += gridDim.x) {
        const Unit uc = unit_of(u, a.geo.nseg, 0);
        load_unit(a, uc, X, scale, do_scale);
        __syncthreads();
        for (int c = 0; c < 2; ++c) {
            const double sm = segment_tree(uc, s, red,
                                           [&](int su, int o) { return X[su][c][o]; });
            if (threadIdx.x < (unsigned)uc.nsu)
                a.segsum[(uint64_t)c * a.geo.nseg + uc.seg((int)threadIdx.x)] = sm;
        }
        __syncthreads();
    }
}

// ------------------------------------------------------ reductions --------

// Pairwise sum of m = 2^k values load(0..m) by one workgroup.
template <class Load>
__device__ double wg_tree(Load load, uint64_t m, double *lds)
{
    const int t = threadIdx.x;
    uint64_t nact;
    if (m >= kWG) {
        const uint64_t per = m / kWG;
        double stack[40];
        int sp = 0;
        for (uint64_t i = 0; i < per; ++i) {
            double v = load(t * per + i);
            for (uint64_t k = i; k & 1; k >>= 1)
                v = stack[--sp] + v;
            stack[sp++] = v;
        }
        lds[t] = stack[0];
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

__global__ __launch_bounds__(kWG) void k_mean_final(PassArgs a, double pow2)
{
    if (a.dev->err)
        return;
    __shared__ double lds[kWG];
    for (int c = 0; c < 2; ++c) {
        const double *p = a.blksum + (uint64_t)c * a.geo.nblocks;
        const double S = wg_tree([&](uint64_t i) { return p[i]; }, a.geo.nblocks, lds);
        if (threadIdx.x == 0)
            a.dev->tdiff[c] = S * pow2;
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
    if (!a.src_basis)
        atomicAdd((unsigned long long *)&a.dev->level_hist[d], 1ull);
}

// Alg. 2's choice for each block.  ESC = false: over the levels computed by
// the fused pass (0 .. previous level + 1).  ESC = true: over the remaining
// levels of escalated blocks.
template <bool ESC>
__global__ __launch_bounds__(kWG) void k_decide(PassArgs a)
{
    if (a.dev->err)
        return;
    __shared__ uint64_t red[kWG];
    __shared__ uint64_t tot[kMaxL];
    __shared__ uint64_t nout[kMaxL];
    const int L = a.lad.L;
    const double raw = (double)(16ull << a.geo.b);
    const uint64_t count = ESC ? a.dev->n_esc : a.geo.nblocks;
    for (uint64_t r = blockIdx.x; r < count; r += gridDim.x) {
        const uint64_t j = ESC ? a.esc_list[r] : r;
        const int h = hint_level(a, j);
        const int cm = h + 1 < L ? h + 1 : L - 1;
        const int k0 = ESC ? cm + 1 : 0;
        const int k1 = ESC ? L - 1 : cm;
        block_totals(a, j, k0, k1, red, tot, nout);
        if (threadIdx.x == 0) {
            int d = -1;
            for (int k = k0; k <= k1; ++k)
                if (raw >= a.lad.theta * (double)tot[k]) {
                    d = k;
                    break;
                }
            if (d < 0 && k1 == L - 1)
                d = L - 1;
            if (d < 0) {
                const uint32_t slot = atomicAdd(&a.dev->n_esc, 1u);
                a.esc_list[slot] = (uint32_t)j;
                atomicAdd((unsigned long long *)&a.dev->escalations, 1ull);
            } else {
                finalize_block(a, j, d, tot[d], nout[d]);
                if (d != h) {
                    const uint32_t slot = atomicAdd(&a.dev->n_replay, 1u);
                    a.replay_list[slot] = (uint32_t)j;
                    atomicAdd((unsigned long long *)&a.dev->replays, 1ull);
                }
            }
        }
        __syncthreads();
    }
}

// N^2, s, statistics; frees the input arena for the next pass.
__global__ __launch_bounds__(kWG) void k_reduce(PassArgs a)
{
    if (a.dev->err)
        return;
    __shared__ double lds[kWG];
    __shared__ uint64_t ures[kWG];
    const int t = threadIdx.x;
    const double N2 = wg_tree([&](uint64_t i) { return a.blknorm[i]; }, a.geo.nblocks, lds);
    uint64_t by = 0;
    for (uint64_t j = t; j < a.geo.nblocks; j += kWG)
        by += a.dout.blk_len[j];
    ures[t] = by;
    __syncthreads();
    for (int st = kWG / 2; st > 0; st >>= 1) {
        if (t < st)
            ures[t] += ures[t + st];
        __syncthreads();
    }
    if (t == 0) {
        DevState *d = a.dev;
        d->normsq = N2;
        if (N2 > 0.0 && __builtin_isfinite(N2)) {
            if (d->normalize)
                d->scale = inv_sqrt_exact(N2);
        } else {
            d->collapsed = 1;
            d->scale = 1.0;
        }
        const uint64_t res = ures[0];
        d->resident = res;
        if (res > d->peak_resident)
            d->peak_resident = res;
        const double ratio = (double)(16ull << a.geo.n) / (double)res;
        d->last_ratio = ratio;
        if (a.src_basis) {
            d->min_ratio = ratio;
        } else {
            d->passes += 1;
            if (ratio < d->min_ratio)
                d->min_ratio = ratio;
        }
        d->arena_used[a.in_arena] = 0;
        d->n_replay = 0;
        d->n_esc = 0;
    }
}

// ---------------------------------------------------- queries -------------

__global__ __launch_bounds__(kWG) void k_decode_range(PassArgs a, uint64_t u0,
                                                      uint64_t u1, uint64_t first,
                                                      uint64_t count, double *out)
{
    __shared__ Planes X;
    const int s = a.geo.s;
    const double scale = a.dev->scale;
    const bool do_scale = scale != 1.0;
    for (uint64_t u = u0 + blockIdx.x; u < u1; u += gridDim.x) {
        const Unit uc = unit_of(u, a.geo.nseg, 0);
        load_unit(a, uc, X, scale, do_scale);
        __syncthreads();
        for (int us = 0; us < uc.nsu; ++us)
            for (uint32_t o = threadIdx.x; o < (1u << s); o += kWG) {
                const uint64_t i = (uc.seg(us) << s) | o;
                if (i >= first && i < first + count) {
                    out[2 * (i - first)] = X[us][0][o];
                    out[2 * (i - first) + 1] = X[us][1][o];
                }
            }
        __syncthreads();
    }
}

__global__ __launch_bounds__(kWG) void k_probs(PassArgs a, const int *qubits, int nq,
                                               double *probs)
{
    __shared__ Planes X;
    __shared__ double bins[1024];
    const int s = a.geo.s;
    const double scale = a.dev->scale;
    const bool do_scale = scale != 1.0;
    const bool lds_bins = nq <= 10;
    const uint32_t nb = 1u << nq;
    if (lds_bins)
        for (uint32_t k = threadIdx.x; k < nb; k += kWG)
            bins[k] = 0.0;
    __syncthreads();
    for (uint64_t u = blockIdx.x; u < a.geo.nunits; u += gridDim.x) {
        const Unit uc = unit_of(u, a.geo.nseg, 0);
        load_unit(a, uc, X, scale, do_scale);
        __syncthreads();
        for (int us = 0; us < uc.nsu; ++us)
            for (uint32_t o = threadIdx.x; o < (1u << s); o += kWG) {
                const uint64_t i = (uc.seg(us) << s) | o;
                uint32_t oc = 0;
                for (int k = 0; k < nq; ++k)
                    oc |= (uint32_t)bit_of(i, qubits[k]) << k;
                const double re = X[us][0][o], im = X[us][1][o];
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
                           int S, double *dst, int p, double scale, bool do_scale)
{
    const int lane = lane_id();
    const int cnt = 1 << S;
    if (amp) {
        for (int o = lane; o < cnt; o += 64)
            dst[o] = amp[2 * (first + o) + p];
        return;
    }
    const int s = a.geo.s;
    for (int off = 0; off < cnt; off += (1 << s)) {
        const uint64_t g = (first + off) >> s;
        const uint64_t j = g >> (a.geo.b - s);
        const double delta = *(const double *)(a.din.hdr + 32 * j + 16);
        decode_plane(a.arena_in + a.din.plane_off[2 * g + p], s, delta, scale, do_scale,
                     dst + off);
    }
}

__global__ __launch_bounds__(kWG) void k_inner(PassArgs A, PassArgs B,
                                               const double *ampA,
                                               const double *ampB, int S,
                                               uint64_t nranges, double *part)
{
    __shared__ Planes X;
    __shared__ double lds[kWG];
    const int wave = threadIdx.x >> 6;
    const double sa = ampA ? 1.0 : A.dev->scale;
    const double sb = ampB ? 1.0 : B.dev->scale;
    for (uint64_t u = blockIdx.x; u < nranges; u += gridDim.x) {
        const uint64_t first = u << S;
        if (wave < 2)
            load_range(A, ampA, first, S, &X[0][wave][0], wave, sa, sa != 1.0);
        else
            load_range(B, ampB, first, S, &X[1][wave - 2][0], wave - 2, sb, sb != 1.0);
        __syncthreads();
        const uint64_t m = 1ull << S;
        for (int c = 0; c < 4; ++c) {
            const double v = wg_tree(
                [&](uint64_t o) {
                    const double ar = X[0][0][o], ai = X[0][1][o];
                    const double br = X[1][0][o], bi = X[1][1][o];
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

__global__ void k_rsqrt(const double *in, double *out, uint64_t count)
{
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < count;
         i += (uint64_t)gridDim.x * blockDim.x)
        out[i] = inv_sqrt_exact(in[i]);
}

// Canonical stream of block j (header + plane records in plane order) into
// `out` (one workgroup).
__global__ __launch_bounds__(kWG) void k_export(PassArgs a, uint64_t j, uint8_t *out)
{
    __shared__ uint64_t offs[2 << 10];  // planes per block: at most 2^(1 + 20 - 10)
    __shared__ uint64_t red[kWG];
    const int t = threadIdx.x;
    const int s = a.geo.s;
    const uint64_t npb = 2ull << (a.geo.b - s);
    const uint32_t padC = pad8(1u << (s - 6));
    const uint64_t base = j * npb;
    const uint64_t per = (npb + kWG - 1) / kWG;
    // sizes of this thread's planes, from their record headers
    uint64_t local = 0;
    for (uint64_t q = t * per; q < (t + 1) * per && q < npb; ++q) {
        const uint8_t *rec = a.arena_in + a.din.plane_off[base + q];
        const uint32_t pw = *(const uint32_t *)(rec + 8);
        const uint32_t no = *(const uint32_t *)(rec + 12);
        const uint64_t sz = kPlaneHdrBytes + (pw ? padC : 0u) + 8ull * pw +
                            (uint64_t)kOutlierBytes * no;
        offs[q] = sz;
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
    uint64_t run = kHdrBytes + red[t] - local;
    for (uint64_t q = t * per; q < (t + 1) * per && q < npb; ++q) {
        const uint64_t sz = offs[q];
        offs[q] = run;
        run += sz;
    }
    if (t < 4)
        ((uint64_t *)out)[t] = ((const uint64_t *)(a.din.hdr + 32 * j))[t];
    __syncthreads();
    // copy records: wave w takes planes w, w+4, ...
    const int wave = t >> 6, lane = lane_id();
    for (uint64_t q = wave; q < npb; q += 4) {
        const uint64_t *src = (const uint64_t *)(a.arena_in + a.din.plane_off[base + q]);
        const uint64_t end = (q + 1 < npb) ? offs[q + 1] : (uint64_t)a.din.blk_len[j];
        const uint64_t nw = (end - offs[q]) / 8;
        uint64_t *dst = (uint64_t *)(out + offs[q]);
        for (uint64_t k = lane; k < nw; k += 64)
            dst[k] = src[k];
    }
}

// ------------------------------------------------------- launchers --------

const char *const kKernelNames[kNumKernelIds] = {
    "pass", "decide", "esc_size", "esc_decide", "replay", "block_norm", "reduce",
    "mean", "mean_tree", "mean_final", "init_state", "sv_pair", "sv_diag",
    "sv_partial", "sv_final"};

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

__global__ void k_init_state(DevState *dev, int normalize)
{
    if (threadIdx.x == 0) {
        DevState d = {};
        d.scale = 1.0;
        d.normalize = normalize;
        *dev = d;
    }
}

void launch_init_state(DevState *dev, int normalize, hipStream_t st, Prof *prof)
{
    TIMED(prof, kIdInitState, st,
          hipLaunchKernelGGL(k_init_state, dim3(1), dim3(64), 0, st, dev, normalize));
}

void launch_mean(const PassArgs &a, hipStream_t st, Prof *prof)
{
    PassArgs m = a;
    TIMED(prof, kIdMean, st,
          hipLaunchKernelGGL(k_mean, dim3(grid_for(a.geo.nunits)), dim3(kWG), 0, st, m));
    const uint64_t spb = 1ull << (a.geo.b - a.geo.s);
    for (int c = 0; c < 2; ++c)
        TIMED(prof, kIdMeanTree, st,
              hipLaunchKernelGGL(k_segtree, dim3(grid_for(a.geo.nblocks)), dim3(kWG), 0,
                                 st, m,
                                 (const double *)(a.segsum + (uint64_t)c * a.geo.nseg),
                                 a.blksum + (uint64_t)c * a.geo.nblocks, spb,
                                 a.geo.nblocks, 0));
    TIMED(prof, kIdMeanFinal, st,
          hipLaunchKernelGGL(k_mean_final, dim3(1), dim3(kWG), 0, st, m,
                             ldexp(1.0, 1 - a.geo.n)));
}

void launch_pass(const PassArgs &a, hipStream_t st, Prof *prof)
{
    const unsigned gu = grid_for(a.geo.nunits), gb = grid_for(a.geo.nblocks);
    const unsigned gside = grid_for(a.geo.nunits < 2048 ? a.geo.nunits : 2048);
    const unsigned gdec = grid_for(a.geo.nblocks < 1024 ? a.geo.nblocks : 1024);
    const uint64_t spb = 1ull << (a.geo.b - a.geo.s);
    TIMED(prof, kIdPass, st,
          hipLaunchKernelGGL(k_pass<kFused>, dim3(gu), dim3(kWG), 0, st, a));
    TIMED(prof, kIdDecide, st,
          hipLaunchKernelGGL(k_decide<false>, dim3(gb), dim3(kWG), 0, st, a));
    if (a.lad.L > 1) {
        TIMED(prof, kIdEscSize, st,
              hipLaunchKernelGGL(k_pass<kEsc>, dim3(gside), dim3(kWG), 0, st, a));
        TIMED(prof, kIdEscDecide, st,
              hipLaunchKernelGGL(k_decide<true>, dim3(gdec), dim3(kWG), 0, st, a));
        TIMED(prof, kIdReplay, st,
              hipLaunchKernelGGL(k_pass<kReplay>, dim3(gside), dim3(kWG), 0, st, a));
    }
    TIMED(prof, kIdBlockNorm, st,
          hipLaunchKernelGGL(k_segtree, dim3(gb), dim3(kWG), 0, st, a,
                             (const double *)a.segnorm, a.blknorm, spb, a.geo.nblocks, 1));
    TIMED(prof, kIdReduce, st, hipLaunchKernelGGL(k_reduce, dim3(1), dim3(kWG), 0, st, a));
}

void launch_encode_basis(const PassArgs &a, hipStream_t st, Prof *prof)
{
    launch_pass(a, st, prof);
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

void launch_rsqrt(const double *in, double *out, uint64_t count, hipStream_t st)
{
    hipLaunchKernelGGL(k_rsqrt, dim3(grid_for((count + kWG - 1) / kWG)), dim3(kWG), 0, st,
                       in, out, count);
}

void launch_export(const PassArgs &a, uint64_t j, uint8_t *out, hipStream_t st)
{
    hipLaunchKernelGGL(k_export, dim3(1), dim3(kWG), 0, st, a, j, out);
}

}  // namespace aalc
