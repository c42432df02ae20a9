// entropy.hip -- the entropy stage of checkpoints on gfx950: block streams v1
// to block entropy streams v1 ("AAE1") and back.
//
// SZ follows its predictor and quantiser with an entropy coder and a
// dictionary coder (Sec. III names that pipeline).  The resident streams keep
// the fixed-width chunk packer, which the pass kernels decode a wavefront at a
// time; where streams leave the pass loop (checkpoints, eviction to the host)
// this stage re-codes them losslessly:
//
//  * plane runs: a plane record equal byte for byte to the record two planes
//    before it (the same component of the previous segment) is a repeat, and
//    each maximal run of repeats is one item with no body;
//  * chunk codes: each chunk's 64 zigzagged residuals go out in the shortest
//    of fixed width w (cost 64 w bits), Golomb-Rice with parameter k < w
//    (q = z >> k one-bits, a zero bit, the k low bits; cost 64 (k + 1) +
//    sum_l (z_l >> k), the smallest best k), or sparse (a 64-bit mask of the
//    nonzero fields, then those fields in w bits; cost 64 + nnz w); ties go to
//    fixed width, then Rice, then sparse.  Golomb codes are the optimal
//    prefix codes of geometrically distributed residuals (Gallager and van
//    Voorhis, 1975); the sparse code is the zero-run coder of chunks with a
//    few nonzero residuals;
//  * a plane whose coded body would not be shorter than its v1 record is
//    stored verbatim.
// The layout is given with sim_export_state_entropy in include/aalcsim.h.
//
// Work decomposition: one workgroup per block.  16-byte records (one value,
// no payload) are settled one per thread; every other plane goes to a
// wavefront, which compares it with the one two planes before it and codes
// it a chunk at a time with one residual per lane (costs by wavefront sums,
// bits OR-ed into a per-wave LDS buffer, then copied out).  Item tags and body
// offsets come from workgroup scans over the planes, so a block holds at most
// kEMaxPlanes planes (b - s <= 11; the library takes b <= 20, s = 10).
// Decoding runs the same way: every chunk code but Rice is decoded one
// residual per lane; a Rice chunk is walked by one lane (its fields have no
// fixed positions).  Every read of an entropy
// stream stays within it: item, body, code and outlier extents are checked
// against the stream's length before they are read, and any inconsistency
// sets kErrImport (the import kernels that follow then do nothing).
#pragma clang fp contract(off)

#include "device.h"

namespace aalc {

namespace {

constexpr uint32_t kEMagic = 0x31454141u;  // "AAE1"
constexpr uint32_t kERun = 0x80000000u;
constexpr uint32_t kEVerb = 0x40000000u;
constexpr uint32_t kESlow = 0xFFFFFFFFu;    // a plane left to the whole wave
constexpr int kMFixed = 128;               // fixed width w: mode 128 + w
constexpr int kMSparse = 63;               // sparse width w: mode 63 + w
constexpr int kEMaxPlanes = 4096;
constexpr int kEBodyHdr = 24;              // coded body header bytes (pw > 0)
constexpr int kEWords = 16 * 64;           // most payload words of a plane (s <= 10)

__device__ __forceinline__ int lane() { return threadIdx.x & 63; }

__device__ __forceinline__ uint32_t pad8u(uint32_t n) { return (n + 7u) & ~7u; }

__device__ __forceinline__ uint32_t wsum32(uint32_t v)
{
    for (int m = 32; m > 0; m >>= 1)
        v += (uint32_t)__shfl_xor((int)v, m);
    return v;
}

__device__ __forceinline__ uint64_t wmax64(uint64_t v)
{
    for (int m = 32; m > 0; m >>= 1) {
        const uint64_t o = (uint64_t)__shfl_xor((long long)v, m);
        v = o > v ? o : v;
    }
    return v;
}

// Exclusive prefix sum over the 64 lanes.
__device__ __forceinline__ uint32_t wscan_excl(uint32_t v)
{
    const int l = lane();
    uint32_t x = v;
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t o = (uint32_t)__shfl_up((int)x, d);
        if (l >= d)
            x += o;
    }
    return x - v;
}

__device__ __forceinline__ uint64_t lanemask_lt() { return (1ull << lane()) - 1ull; }

__device__ __forceinline__ int bitlen(uint64_t z) { return z ? 64 - __clzll((long long)z) : 0; }

// n <= 64 bits at bit offset o of little-endian words W[0 .. nw); bits at or
// past word nw read as 0 (callers check extents; this only keeps reads in
// bounds).
__device__ __forceinline__ uint64_t get_bits(const uint64_t *W, uint64_t nw, uint64_t o, int n)
{
    if (n == 0)
        return 0;
    const uint64_t i = o >> 6;
    const int sh = (int)(o & 63);
    uint64_t v = i < nw ? W[i] >> sh : 0ull;
    if (sh && sh + n > 64 && i + 1 < nw)
        v |= W[i + 1] << (64 - sh);
    return n == 64 ? v : v & ((1ull << n) - 1ull);
}

// OR n <= 64 bits of v into the LDS bit buffer B (dwords) at bit offset o.
__device__ __forceinline__ void put_bits(uint32_t *B, uint64_t o, uint64_t v, int n)
{
    if (n == 0)
        return;
    if (n < 64)
        v &= (1ull << n) - 1ull;
    if (v == 0)
        return;
    const uint32_t i = (uint32_t)(o >> 5), sh = (uint32_t)(o & 31);
    const uint64_t lo = v << sh;
    const uint32_t hi = sh ? (uint32_t)(v >> (64 - sh)) : 0u;
    if ((uint32_t)lo)
        atomicOr(&B[i], (uint32_t)lo);
    if ((uint32_t)(lo >> 32))
        atomicOr(&B[i + 1], (uint32_t)(lo >> 32));
    if (hi)
        atomicOr(&B[i + 2], hi);
}

// Set bits [o, o + q) of B.
__device__ __forceinline__ void put_ones(uint32_t *B, uint64_t o, uint32_t q)
{
    while (q) {
        const uint32_t i = (uint32_t)(o >> 5), sh = (uint32_t)(o & 31);
        const uint32_t take = min(q, 32u - sh);
        const uint32_t m = (take == 32u ? 0xFFFFFFFFu : ((1u << take) - 1u)) << sh;
        atomicOr(&B[i], m);
        o += take;
        q -= take;
    }
}

// Chunk code of one chunk: the lane's residual z, the chunk width w.
struct ChunkCode {
    int mode;       // fixed 128 + w, sparse 63 + w, Rice k
    uint32_t bits;  // coded length
    uint64_t mask;  // nonzero fields
};

__device__ ChunkCode choose_code(uint64_t z, int w)
{
    ChunkCode r;
    r.mask = __ballot(z != 0ull);
    if (w == 0) {
        r.mode = kMFixed;
        r.bits = 0;
        return r;
    }
    const uint32_t fixed = 64u * (uint32_t)w;
    // Rice: only k <= w - 2 can cost less than fixed width, and no k whose
    // 64 (k + 1) already reaches the best cost can do better; the largest z
    // (at least 2^(w-1)) alone adds 2^(w-1-k) >= 4096 >= 64 w for k <= w - 13,
    // so the search starts at w - 12; terms saturate at 2^20, where no sum
    // can win
    uint32_t best = fixed;
    int kbest = -1;
    for (int k = w > 12 ? w - 12 : 0; k + 2 <= w && 64u * (uint32_t)(k + 1) < best; ++k) {
        const uint64_t q = z >> k;
        const uint32_t t = q > (1ull << 20) ? (1u << 20) : (uint32_t)q;
        const uint32_t cost = 64u * (uint32_t)(k + 1) + wsum32(t);
        if (cost < best) {
            best = cost;
            kbest = k;
        }
    }
    const uint32_t sparse = 64u + (uint32_t)__popcll(r.mask) * (uint32_t)w;
    const uint32_t rice = kbest >= 0 ? best : 0xFFFFFFFFu;
    if (fixed <= rice && fixed <= sparse) {
        r.mode = kMFixed + w;
        r.bits = fixed;
    } else if (rice <= sparse) {
        r.mode = kbest;
        r.bits = rice;
    } else {
        r.mode = kMSparse + w;
        r.bits = sparse;
    }
    return r;
}

// Lane l's residual of chunk c of a v1 plane record (payload at word offset
// woff, width w).
__device__ __forceinline__ uint64_t chunk_field(const uint64_t *pay, uint32_t woff, int w)
{
    return get_bits(pay + woff, (uint64_t)w, (uint64_t)lane() * (uint64_t)w, w);
}

struct EncArgs {
    PassArgs a;
    uint64_t first, count;
    uint32_t *elen;        // [count] entropy stream bytes (size pass)
    const uint64_t *eoff;  // [count] output offsets (write pass)
    uint8_t *out;
};

__device__ __forceinline__ const uint8_t *plane_rec(const PassArgs &a, uint64_t plane)
{
    return a.arena_in + rec_at(a.din, plane);
}

__device__ __forceinline__ uint32_t rec_len(const uint8_t *rec, uint32_t padC)
{
    const uint32_t pw = *(const uint32_t *)(rec + 8), no = *(const uint32_t *)(rec + 12);
    return kPlaneHdrBytes + (pw ? padC : 0u) + 8u * pw + kOutlierBytes * no;
}

// The literal tag of a v1 record (coded body bytes, or kEVerb | its length);
// with WRITE, its body written at dst.  wb: this wave's zeroed LDS buffer.
template <bool WRITE>
__device__ uint32_t code_plane(const uint8_t *rec, int C, uint32_t *wb, uint8_t *dst)
{
    const int l = lane();
    const uint32_t padC = pad8u((uint32_t)C);
    const uint32_t pw = *(const uint32_t *)(rec + 8), nout = *(const uint32_t *)(rec + 12);
    const uint32_t vlen = kPlaneHdrBytes + (pw ? padC : 0u) + 8u * pw + kOutlierBytes * nout;
    if (pw == 0) {
        // the coded body of a plane without payload is its record
        if (WRITE) {
            const uint64_t *s = (const uint64_t *)rec;
            uint64_t *d = (uint64_t *)dst;
            for (uint32_t k = l; k < vlen / 8; k += 64)
                d[k] = s[k];
        }
        return kEVerb | vlen;
    }
    const uint8_t *wid = rec + kPlaneHdrBytes;
    const uint64_t *pay = (const uint64_t *)(rec + kPlaneHdrBytes + padC);
    const int wl = l < C ? wid[l] : 0;
    uint32_t woff = 0, cbits = 0, nlen = 0;
    int mode_l = 0;
    uint32_t len_l = 0;  // lane c < C: coded length of chunk c
    for (int c = 0; c < C; ++c) {
        const int w = __shfl(wl, c);
        const uint64_t z = chunk_field(pay, woff, w);
        const ChunkCode cc = choose_code(z, w);
        if (WRITE) {
            if (cc.mode >= kMFixed) {
                put_bits(wb, cbits + (uint64_t)l * (uint64_t)w, z, w);
            } else if (cc.mode > kMSparse) {
                if (l == 0)
                    put_bits(wb, cbits, cc.mask, 64);
                if (z) {
                    const uint32_t rank = (uint32_t)__popcll(cc.mask & lanemask_lt());
                    put_bits(wb, cbits + 64u + (uint64_t)rank * (uint64_t)w, z, w);
                }
            } else {
                const int k = cc.mode;
                const uint32_t q = (uint32_t)(z >> k);  // < 2^12 when Rice is taken
                const uint32_t o = cbits + wscan_excl(q + 1u + (uint32_t)k);
                put_ones(wb, o, q);
                put_bits(wb, (uint64_t)o + q + 1u, z, k);
            }
        }
        if (l == c) {
            mode_l = cc.mode;
            len_l = cc.bits;
        }
        nlen += cc.mode < kMFixed;
        cbits += cc.bits;
        woff += (uint32_t)w;
    }
    const uint32_t cw = (cbits + 63u) / 64u;
    const uint32_t body = (uint32_t)kEBodyHdr + padC + pad8u(2u * nlen) + 8u * cw +
                          kOutlierBytes * nout;
    if (body >= vlen) {
        if (WRITE) {
            const uint64_t *s = (const uint64_t *)rec;
            uint64_t *d = (uint64_t *)dst;
            for (uint32_t k = l; k < vlen / 8; k += 64)
                d[k] = s[k];
            for (uint32_t k = l; k < 2u * cw; k += 64)
                wb[k] = 0u;
        }
        return kEVerb | vlen;
    }
    if (WRITE) {
        if (l == 0) {
            *(uint64_t *)dst = *(const uint64_t *)rec;
            *(uint32_t *)(dst + 8) = pw;
            *(uint32_t *)(dst + 12) = nout;
            *(uint32_t *)(dst + 16) = cw;
            *(uint32_t *)(dst + 20) = 0u;
        }
        uint8_t *modes = dst + kEBodyHdr;
        if ((uint32_t)l < padC)
            modes[l] = l < C ? (uint8_t)mode_l : (uint8_t)0;
        // u16 lengths of the chunks that are not fixed width, in chunk order
        const bool nf = l < C && mode_l < kMFixed;
        const uint64_t nfm = __ballot(nf);
        uint16_t *lens = (uint16_t *)(modes + padC);
        if (nf)
            lens[__popcll(nfm & lanemask_lt())] = (uint16_t)len_l;
        const uint32_t lpad = pad8u(2u * nlen);
        if ((uint32_t)l < (lpad - 2u * nlen) / 2u)
            lens[nlen + l] = 0;
        uint64_t *code = (uint64_t *)(modes + padC + lpad);
        for (uint32_t k = l; k < cw; k += 64) {
            code[k] = (uint64_t)wb[2 * k] | ((uint64_t)wb[2 * k + 1] << 32);
            wb[2 * k] = 0u;
            wb[2 * k + 1] = 0u;
        }
        const uint64_t *os = pay + pw;
        uint64_t *od = code + cw;
        for (uint32_t k = l; k < 2u * nout; k += 64)
            od[k] = os[k];
    }
    return body;
}

// Workgroup-wide exclusive scan of one value per thread; returns the total.
__device__ uint32_t wg_scan(uint32_t v, uint32_t *red, uint32_t &excl)
{
    const int t = threadIdx.x;
    red[t] = v;
    __syncthreads();
    for (int d = 1; d < kWG; d <<= 1) {
        const uint32_t add = t >= d ? red[t - d] : 0u;
        __syncthreads();
        red[t] += add;
        __syncthreads();
    }
    excl = red[t] - v;
    const uint32_t tot = red[kWG - 1];
    __syncthreads();
    return tot;
}

__device__ uint64_t wg_scan64(uint64_t v, uint64_t *red, uint64_t &excl)
{
    const int t = threadIdx.x;
    red[t] = v;
    __syncthreads();
    for (int d = 1; d < kWG; d <<= 1) {
        const uint64_t add = t >= d ? red[t - d] : 0ull;
        __syncthreads();
        red[t] += add;
        __syncthreads();
    }
    excl = red[t] - v;
    const uint64_t tot = red[kWG - 1];
    __syncthreads();
    return tot;
}

// Pairwise sum of m = 2^k doubles from src (the perfect binary tree over
// index order), through the LDS array v (m doubles).
__device__ double wg_pairwise(const double *src, uint32_t m, double *v)
{
    const int t = threadIdx.x;
    for (uint32_t i = t; i < m; i += kWG)
        v[i] = src[i];
    __syncthreads();
    for (uint32_t h = m >> 1; h >= 1; h >>= 1) {
        double tmp[8];
        const uint32_t per = (h + kWG - 1) / kWG;
        for (uint32_t r = 0; r < per && r < 8; ++r) {
            const uint32_t i = t + r * kWG;
            tmp[r] = i < h ? v[2 * i] + v[2 * i + 1] : 0.0;
        }
        __syncthreads();
        for (uint32_t r = 0; r < per && r < 8; ++r) {
            const uint32_t i = t + r * kWG;
            if (i < h)
                v[i] = tmp[r];
        }
        __syncthreads();
    }
    const double s = v[0];
    __syncthreads();
    return s;
}

struct EncLds {
    uint32_t tag[kEMaxPlanes];   // per plane: kERun (repeat) or its literal tag
    uint32_t aux[kEMaxPlanes];   // item starts, then body offsets
    uint16_t lst[kEMaxPlanes];   // the planes left to the waves
    uint32_t wb[4][2 * kEWords];  // per wave: coded bits
    uint32_t red[kWG];
    uint32_t nlst;
};

template <bool WRITE>
__global__ __launch_bounds__(kWG) void k_ent_encode(EncArgs e)
{
    __shared__ EncLds S;
    const PassArgs &a = e.a;
    const int t = threadIdx.x, wave = t >> 6, l = lane();
    const int s = a.geo.s;
    const int C = 1 << (s - 6);
    const uint32_t padC = pad8u((uint32_t)C);
    const uint32_t P = 2u << (a.geo.b - s);
    for (int k = t; k < 4 * 2 * kEWords; k += kWG)
        (&S.wb[0][0])[k] = 0u;
    __syncthreads();
    for (uint64_t bi = blockIdx.x; bi < e.count; bi += gridDim.x) {
        const uint64_t j = e.first + bi;
        const uint64_t base = j * P;
        // per plane: repeat of the plane two before, else its literal tag.
        // First one plane per lane: a 16-byte record (one value, no payload,
        // no outliers) repeats the plane two before iff that record is 16
        // bytes with the same anchor, else it is stored verbatim; the other
        // planes are marked, then taken by the waves in turn, one plane per
        // wave.
        if (t == 0)
            S.nlst = 0u;
        __syncthreads();
        for (uint32_t q = (uint32_t)t; q < P; q += kWG) {
            const uint8_t *rec = plane_rec(a, base + q);
            uint32_t tg = kESlow;
            if (*(const uint64_t *)(rec + 8) == 0ull) {
                bool rep = false;
                if (q >= 2) {
                    const uint8_t *r2 = plane_rec(a, base + q - 2);
                    rep = *(const uint64_t *)(r2 + 8) == 0ull &&
                          *(const uint64_t *)r2 == *(const uint64_t *)rec;
                }
                tg = rep ? kERun : (kEVerb | kPlaneHdrBytes);
            } else {
                S.lst[atomicAdd(&S.nlst, 1u)] = (uint16_t)q;
            }
            S.tag[q] = tg;
        }
        __syncthreads();
        const uint32_t nlst = S.nlst;
        for (uint32_t i = wave; i < nlst; i += 4) {
            const uint32_t q = S.lst[i];
            const uint8_t *rec = plane_rec(a, base + q);
            const uint32_t len = rec_len(rec, padC);
            bool rep = false;
            if (q >= 2) {
                const uint8_t *r2 = plane_rec(a, base + q - 2);
                if (rec_len(r2, padC) == len) {
                    bool diff = false;
                    const uint64_t *x = (const uint64_t *)rec, *y = (const uint64_t *)r2;
                    for (uint32_t k = l; k < len / 8; k += 64)
                        diff |= x[k] != y[k];
                    rep = __ballot(diff) == 0ull;
                }
            }
            const uint32_t tg = rep ? kERun : code_plane<false>(rec, C, S.wb[wave], nullptr);
            if (l == 0)
                S.tag[q] = tg;
        }
        __syncthreads();
        // items: a literal plane, or a maximal run of repeats
        const uint32_t per = (P + kWG - 1) / kWG;
        const uint32_t q0 = min(P, t * per), q1 = min(P, q0 + per);
        uint32_t nit = 0, nby = 0;
        for (uint32_t q = q0; q < q1; ++q) {
            const bool rep = S.tag[q] == kERun;
            nit += !rep || (q > 0 && S.tag[q - 1] != kERun) || q == 0;
            nby += rep ? 0u : (S.tag[q] & ~kEVerb);
        }
        uint32_t it0, by0;
        const uint32_t nitems = wg_scan(nit, S.red, it0);
        const uint32_t nbody = wg_scan(nby, S.red, by0);
        const bool scaled = a.din.bscale[j] != 1.0;
        const uint32_t tagb = pad8u(4u * nitems);
        const uint32_t bstart = kHdrBytes + 8u + (scaled ? kScaleBytes : 0u) + tagb;
        const uint32_t elen = bstart + nbody;
        if (!WRITE) {
            if (t == 0)
                e.elen[bi] = elen;
            __syncthreads();
            continue;
        }
        uint8_t *out = e.out + e.eoff[bi];
        // item starts (aux by item index), then tags
        {
            uint32_t it = it0;
            for (uint32_t q = q0; q < q1; ++q) {
                const bool rep = S.tag[q] == kERun;
                if (!rep || q == 0 || S.tag[q - 1] != kERun)
                    S.aux[it++] = q;
            }
        }
        __syncthreads();
        uint32_t *tags = (uint32_t *)(out + kHdrBytes + 8u + (scaled ? kScaleBytes : 0u));
        for (uint32_t i = t; i < nitems; i += kWG) {
            const uint32_t q = S.aux[i];
            const uint32_t nx = i + 1 < nitems ? S.aux[i + 1] : P;
            tags[i] = S.tag[q] == kERun ? (kERun | (nx - q)) : S.tag[q];
        }
        if (t == 0 && (nitems & 1u))
            tags[nitems] = 0u;
        __syncthreads();
        // body offsets by plane
        {
            uint32_t off = by0;
            for (uint32_t q = q0; q < q1; ++q) {
                S.aux[q] = off;
                off += S.tag[q] == kERun ? 0u : (S.tag[q] & ~kEVerb);
            }
        }
        // header: the v1 header with the entropy magic and length; normsq
        // pairwise over the block's segment sums; v1 length, item count, scale
        const double ns = wg_pairwise(a.din.segnorm + j * (P / 2), P / 2,
                                      (double *)&S.wb[0][0]);
        if (t == 0) {
            const uint64_t *h = (const uint64_t *)(a.din.hdr + 32 * j);
            uint64_t *o = (uint64_t *)out;
            o[0] = (h[0] & ~0xFFFFFFFFull) | kEMagic;
            o[1] = (h[1] & 0xFFFFFFFFull) | ((uint64_t)elen << 32);
            o[2] = h[2];
            *(double *)(out + 24) = ns;
            *(uint32_t *)(out + 32) = a.din.blk_len[j];
            *(uint32_t *)(out + 36) = nitems;
            if (scaled)
                *(double *)(out + 40) = a.din.bscale[j];
        }
        // the LDS buffer doubled as the tree's storage: clear it again
        for (int k = t; k < 4 * 2 * kEWords; k += kWG)
            (&S.wb[0][0])[k] = 0u;
        __syncthreads();
        // 16-byte verbatim records one per lane, the other literals one per
        // wave
        for (uint32_t q = (uint32_t)t; q < P; q += kWG)
            if (S.tag[q] == (kEVerb | kPlaneHdrBytes)) {
                const uint64_t *src = (const uint64_t *)plane_rec(a, base + q);
                uint64_t *dst = (uint64_t *)(out + bstart + S.aux[q]);
                dst[0] = src[0];
                dst[1] = src[1];
            }
        for (uint32_t i = wave; i < nlst; i += 4) {
            const uint32_t q = S.lst[i];
            if (S.tag[q] != kERun)
                code_plane<true>(plane_rec(a, base + q), C, S.wb[wave],
                                 out + bstart + S.aux[q]);
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------ decode ------

struct DecArgs {
    PassArgs a;            // geo, dev (error bits)
    uint64_t count;        // blocks
    const uint8_t *src;    // streams as given (v1 or entropy), block k at src + soff[k]
    const uint64_t *soff;  // [count + 1]
    uint8_t *dst;          // v1 streams, block k at dst + doff[k]
    const uint64_t *doff;  // [count + 1]
};

__device__ __forceinline__ void fail(const DecArgs &d) { atomicOr(&d.a.dev->err, kErrImport); }

struct DecLds {
    uint32_t A[kEMaxPlanes];      // per item: planes covered; then per plane: item + 1 if literal
    uint32_t B[kEMaxPlanes];      // per item: first plane; then per plane: source plane + 1
    uint32_t Cb[kEMaxPlanes];     // per item: body offset
    uint32_t D[kEMaxPlanes];      // per plane: v1 record size, then offset
    uint32_t pk[4][2 * kEWords];  // per wave: packed v1 payload
    uint64_t zb[4][64];           // per wave: residuals of a Rice chunk
    uint16_t lst[kEMaxPlanes];    // the planes left to the waves
    uint32_t red[kWG];
    uint64_t red64[kWG];
    uint32_t nlst;
};

// One coded literal body B (tb bytes, within the stream) into the v1
// record D; false when malformed.
__device__ bool decode_coded(const uint8_t *B, uint32_t tb, int C, uint32_t *pk, uint64_t *zb,
                             uint8_t *D)
{
    const int l = lane();
    const uint32_t padC = pad8u((uint32_t)C);
    const uint32_t pw = *(const uint32_t *)(B + 8), nout = *(const uint32_t *)(B + 12);
    if (pw == 0) {
        if (tb != kPlaneHdrBytes + kOutlierBytes * nout)
            return false;
        for (uint32_t k = l; k < tb / 8; k += 64)
            ((uint64_t *)D)[k] = ((const uint64_t *)B)[k];
        return true;
    }
    if (tb < (uint32_t)kEBodyHdr + padC)
        return false;
    const uint32_t cw = *(const uint32_t *)(B + 16);
    if (*(const uint32_t *)(B + 20) != 0u)
        return false;
    const uint8_t *modes = B + kEBodyHdr;
    const int m_l = (uint32_t)l < padC ? modes[l] : 0;
    if (__ballot((uint32_t)l >= (uint32_t)C && (uint32_t)l < padC && m_l != 0))
        return false;
    const bool nf = l < C && m_l < kMFixed;
    const uint64_t nfm = __ballot(nf);
    const uint32_t nlen = (uint32_t)__popcll(nfm);
    const uint64_t need = (uint64_t)kEBodyHdr + padC + pad8u(2u * nlen) + 8ull * cw +
                          (uint64_t)kOutlierBytes * nout;
    if (need != tb)
        return false;
    const uint8_t *lb = modes + padC;
    const uint32_t lpad = pad8u(2u * nlen);
    if (__ballot((uint32_t)l >= 2u * nlen && (uint32_t)l < lpad && lb[l] != 0))
        return false;
    const uint64_t *code = (const uint64_t *)(lb + lpad);
    const uint64_t nbits = 64ull * cw;
    // chunk lengths and starts (lane c < C)
    bool badm = false;
    uint32_t len_l = 0;
    if (l < C) {
        if (m_l >= kMFixed) {
            badm = m_l > kMFixed + 64;
            len_l = 64u * (uint32_t)(m_l - kMFixed);
        } else {
            const uint32_t li = (uint32_t)__popcll(nfm & lanemask_lt());
            len_l = (uint32_t)lb[2 * li] | ((uint32_t)lb[2 * li + 1] << 8);
        }
    }
    if (__ballot(badm))
        return false;
    const uint32_t start_l = wscan_excl(len_l);
    const uint32_t total = wsum32(len_l);
    if ((uint64_t)total > nbits || (total + 63u) / 64u != cw)
        return false;
    // padding bits after the last code are zero
    if (total % 64u != 0u && (code[cw - 1] >> (total % 64u)) != 0ull)
        return false;
    uint32_t woff = 0;
    uint8_t w_l = 0;
    for (int c = 0; c < C; ++c) {
        const int m = __shfl(m_l, c);
        const uint64_t cb = (uint32_t)__shfl((int)start_l, c);
        const uint64_t end = cb + (uint32_t)__shfl((int)len_l, c);
        uint64_t z = 0;
        int w = 0;
        if (m >= kMFixed) {
            w = m - kMFixed;
            z = get_bits(code, cw, cb + (uint64_t)l * (uint64_t)w, w);
        } else if (m > kMSparse) {
            w = m - kMSparse;
            if (cb + 64 > end)
                return false;
            const uint64_t mask = get_bits(code, cw, cb, 64);
            if (64ull + (uint64_t)__popcll(mask) * (uint64_t)w != end - cb)
                return false;
            if ((mask >> l) & 1ull) {
                const uint32_t rank = (uint32_t)__popcll(mask & lanemask_lt());
                z = get_bits(code, cw, cb + 64u + (uint64_t)rank * (uint64_t)w, w);
            }
            if (__ballot(((mask >> l) & 1ull) && z == 0ull))
                return false;
        } else {
            // one lane walks the chunk's 64 fields
            const int k = m;
            int ok = 1;
            if (l == 0) {
                uint64_t pos = cb;
                for (int f = 0; f < 64 && ok; ++f) {
                    uint64_t q = 0;
                    for (;;) {
                        if (pos >= end) {
                            ok = 0;
                            break;
                        }
                        const int avail = (int)min((uint64_t)64, end - pos);
                        const uint64_t win = get_bits(code, cw, pos, avail);
                        const uint64_t inv = ~win & (avail == 64 ? ~0ull : ((1ull << avail) - 1ull));
                        if (inv) {
                            const int ones = __builtin_ctzll(inv);
                            q += (uint64_t)ones;
                            pos += (uint64_t)ones + 1;
                            break;
                        }
                        q += (uint64_t)avail;
                        pos += (uint64_t)avail;
                    }
                    if (!ok)
                        break;
                    if ((k > 0 && (q >> (64 - k)) != 0ull) || pos + (uint64_t)k > end) {
                        ok = 0;
                        break;
                    }
                    zb[f] = (q << k) | get_bits(code, cw, pos, k);
                    pos += (uint64_t)k;
                }
                if (ok && pos != end)
                    ok = 0;
            }
            if (!__shfl(ok, 0))
                return false;
            z = zb[l];
            w = bitlen(wmax64(z));
        }
        if (l == c)
            w_l = (uint8_t)w;
        put_bits(pk, (uint64_t)woff * 64u + (uint64_t)l * (uint64_t)w, z, w);
        woff += (uint32_t)w;
    }
    if (woff != pw) {
        for (uint32_t k = l; k < 2u * kEWords; k += 64)
            pk[k] = 0u;
        return false;
    }
    // the v1 record: header, widths, payload, outliers
    if (l == 0) {
        *(uint64_t *)D = *(const uint64_t *)B;
        *(uint32_t *)(D + 8) = pw;
        *(uint32_t *)(D + 12) = nout;
    }
    if ((uint32_t)l < padC)
        D[kPlaneHdrBytes + l] = l < C ? w_l : (uint8_t)0;
    uint64_t *pay = (uint64_t *)(D + kPlaneHdrBytes + padC);
    for (uint32_t k = l; k < pw; k += 64) {
        pay[k] = (uint64_t)pk[2 * k] | ((uint64_t)pk[2 * k + 1] << 32);
        pk[2 * k] = 0u;
        pk[2 * k + 1] = 0u;
    }
    const uint64_t *os = code + cw;
    for (uint32_t k = l; k < 2u * nout; k += 64)
        pay[pw + k] = os[k];
    return true;
}

// Inclusive max-scan of one value per thread over the workgroup.
__device__ uint32_t wg_max_scan(uint32_t v, uint32_t *red)
{
    const int t = threadIdx.x;
    red[t] = v;
    __syncthreads();
    for (int d = 1; d < kWG; d <<= 1) {
        const uint32_t o = t >= d ? red[t - d] : 0u;
        __syncthreads();
        red[t] = max(red[t], o);
        __syncthreads();
    }
    const uint32_t r = red[t];
    __syncthreads();
    return r;
}

__global__ __launch_bounds__(kWG) void k_ent_decode(DecArgs d)
{
    __shared__ DecLds S;
    const PassArgs &a = d.a;
    const int t = threadIdx.x, wave = t >> 6, l = lane();
    const int s = a.geo.s;
    const int C = 1 << (s - 6);
    const uint32_t padC = pad8u((uint32_t)C);
    const uint32_t P = 2u << (a.geo.b - s);
    for (int k = t; k < 4 * 2 * kEWords; k += kWG)
        (&S.pk[0][0])[k] = 0u;
    __syncthreads();
    for (uint64_t bi = blockIdx.x; bi < d.count; bi += gridDim.x) {
        if (a.dev->err)
            return;
        const uint8_t *E = d.src + d.soff[bi];
        const uint64_t len = d.soff[bi + 1] - d.soff[bi];
        uint8_t *V = d.dst + d.doff[bi];
        const uint64_t vlen = d.doff[bi + 1] - d.doff[bi];
        if (*(const uint32_t *)E != kEMagic) {
            // a v1 stream: copied as it is (its records are checked later)
            const uint64_t *x = (const uint64_t *)E;
            uint64_t *y = (uint64_t *)V;
            for (uint64_t k = t; k < len / 8; k += kWG)
                y[k] = x[k];
            continue;
        }
        // the host checked magic, geometry, flags, level, lengths and the
        // scale word; here: items, bodies and codes
        const bool scaled = (E[5] & kHdrScaled) != 0;
        const uint32_t ni = *(const uint32_t *)(E + 36);
        const uint32_t tpos = kHdrBytes + 8u + (scaled ? kScaleBytes : 0u);
        if (ni == 0 || ni > P || (uint64_t)tpos + pad8u(4u * ni) > len) {
            if (t == 0)
                fail(d);
            return;
        }
        const uint32_t *tags = (const uint32_t *)(E + tpos);
        const uint32_t bstart = tpos + pad8u(4u * ni);
        // items: planes covered and body bytes (thread t: items [i0, i1))
        const uint32_t per = (ni + kWG - 1) / kWG;
        const uint32_t i0 = min(ni, t * per), i1 = min(ni, i0 + per);
        uint32_t npl = 0;
        uint64_t nby = 0;
        bool bad = (ni & 1u) && t == 0 && tags[ni] != 0u;
        for (uint32_t i = i0; i < i1; ++i) {
            const uint32_t tg = tags[i];
            const uint32_t c = (tg & kERun) ? (tg & ~kERun) : 1u;
            const uint32_t by = (tg & kERun) ? 0u : (tg & ~kEVerb);
            bad |= c == 0u || c > P || by % 8u != 0u || by > len;
            S.A[i] = c;
            S.Cb[i] = by;
            npl += c;
            nby += by;
        }
        bad |= nby > len;
        if (__syncthreads_or(bad)) {
            if (t == 0)
                fail(d);
            return;
        }
        // planes: at most 4096 items of at most 4096 each; bytes in 64 bits
        uint32_t pl0;
        uint64_t by0;
        const uint32_t npt = wg_scan(npl, S.red, pl0);
        const uint64_t nbt = wg_scan64(nby, S.red64, by0);
        const bool fits = (uint64_t)bstart + nbt == len;
        for (uint32_t i = i0, p = pl0, o = (uint32_t)by0; i < i1; ++i) {
            const uint32_t c = S.A[i], by = S.Cb[i];
            S.B[i] = p;
            S.Cb[i] = o;
            bad |= (tags[i] & kERun) && p < 2u;
            p += c;
            o += by;
        }
        if (__syncthreads_or(bad || npt != P || !fits)) {
            if (t == 0)
                fail(d);
            return;
        }
        // per plane: A[q] = item + 1 when plane q is a literal, else 0
        uint32_t lit_of[16];
        for (uint32_t i = i0, r = 0; i < i1; ++i, ++r)
            lit_of[r & 15] = (tags[i] & kERun) ? 0xFFFFFFFFu : S.B[i];
        __syncthreads();
        for (uint32_t q = t; q < P; q += kWG)
            S.A[q] = 0u;
        __syncthreads();
        for (uint32_t i = i0, r = 0; i < i1; ++i, ++r)
            if (lit_of[r & 15] != 0xFFFFFFFFu)
                S.A[lit_of[r & 15]] = i + 1u;
        __syncthreads();
        // source plane of each plane: the last literal plane at or before it
        // with the same parity (a repeat copies the plane two before it)
        const uint32_t qp = (P + kWG - 1) / kWG;
        const uint32_t a0 = min(P, t * qp), a1 = min(P, a0 + qp);
        uint32_t m0 = 0, m1 = 0;
        for (uint32_t q = a0; q < a1; ++q)
            if (S.A[q]) {
                if (q & 1u)
                    m1 = q + 1u;
                else
                    m0 = q + 1u;
            }
        uint32_t c0 = wg_max_scan(m0, S.red);
        uint32_t c1 = wg_max_scan(m1, S.red);
        // exclusive: the previous thread's inclusive value
        S.red[t] = c0;
        __syncthreads();
        c0 = t ? S.red[t - 1] : 0u;
        __syncthreads();
        S.red[t] = c1;
        __syncthreads();
        c1 = t ? S.red[t - 1] : 0u;
        __syncthreads();
        // B[q] = source plane + 1; D[q] = v1 record size (from the source
        // literal's body: a verbatim record's own fields, or a coded body's)
        uint64_t nvs = 0;
        for (uint32_t q = a0; q < a1; ++q) {
            if (S.A[q]) {
                if (q & 1u)
                    c1 = q + 1u;
                else
                    c0 = q + 1u;
            }
            const uint32_t sp = (q & 1u) ? c1 : c0;
            S.B[q] = sp;
            uint32_t sz = 0;
            if (sp == 0u) {
                bad = true;
            } else {
                const uint32_t it = S.A[sp - 1u] - 1u;
                const uint32_t tg = tags[it];
                const uint32_t tb = tg & ~kEVerb;
                const uint8_t *Bd = E + bstart + S.Cb[it];
                if (tb < kPlaneHdrBytes) {
                    bad = true;
                } else {
                    const uint32_t pw = *(const uint32_t *)(Bd + 8);
                    const uint32_t no = *(const uint32_t *)(Bd + 12);
                    const uint64_t s64 = (uint64_t)kPlaneHdrBytes + (pw ? padC : 0u) +
                                         8ull * pw + (uint64_t)kOutlierBytes * no;
                    if (s64 > vlen || ((tg & kEVerb) && s64 != tb))
                        bad = true;
                    else
                        sz = (uint32_t)s64;
                }
            }
            S.D[q] = sz;
            nvs += sz;
        }
        uint64_t v0;
        const uint64_t vtot = wg_scan64(nvs, S.red64, v0);
        const uint32_t vstart = kHdrBytes + (scaled ? kScaleBytes : 0u);
        for (uint32_t q = a0, o = vstart + (uint32_t)v0; q < a1; ++q) {
            const uint32_t sz = S.D[q];
            S.D[q] = o;
            o += sz;
        }
        if (__syncthreads_or(bad || (uint64_t)vstart + vtot != vlen)) {
            if (t == 0)
                fail(d);
            return;
        }
        // the v1 header and scale word
        if (t < 4) {
            uint64_t v = ((const uint64_t *)E)[t];
            if (t == 0)
                v = (v & ~0xFFFFFFFFull) | kMagic;
            if (t == 1)
                v = (v & 0xFFFFFFFFull) | ((uint64_t)vlen << 32);
            ((uint64_t *)V)[t] = v;
        }
        if (t == 4 && scaled)
            ((uint64_t *)V)[4] = *(const uint64_t *)(E + 40);
        // the records: a wave takes 64 planes at a time, a plane whose
        // source is a 16-byte verbatim record copied by its lane, the others
        // decoded by the whole wave one by one
        bool ok = true;
        if (t == 0)
            S.nlst = 0u;
        __syncthreads();
        for (uint32_t q = (uint32_t)t; q < P; q += kWG) {
            const uint32_t it = S.A[S.B[q] - 1u] - 1u;
            if (tags[it] == (kEVerb | kPlaneHdrBytes)) {
                const uint64_t *src = (const uint64_t *)(E + bstart + S.Cb[it]);
                uint64_t *dst = (uint64_t *)(V + S.D[q]);
                dst[0] = src[0];
                dst[1] = src[1];
            } else {
                S.lst[atomicAdd(&S.nlst, 1u)] = (uint16_t)q;
            }
        }
        __syncthreads();
        const uint32_t nlst = S.nlst;
        for (uint32_t i = wave; i < nlst; i += 4) {
            const uint32_t q = S.lst[i];
            const uint32_t it = S.A[S.B[q] - 1u] - 1u;
            const uint32_t tg = tags[it];
            const uint32_t tb = tg & ~kEVerb;
            const uint8_t *Bd = E + bstart + S.Cb[it];
            uint8_t *Dd = V + S.D[q];
            if (tg & kEVerb) {
                for (uint32_t k = l; k < tb / 8; k += 64)
                    ((uint64_t *)Dd)[k] = ((const uint64_t *)Bd)[k];
            } else if (!decode_coded(Bd, tb, C, S.pk[wave], S.zb[wave], Dd)) {
                ok = false;
                break;
            }
        }
        if (__syncthreads_or(!ok)) {
            if (t == 0)
                fail(d);
            return;
        }
    }
}

}  // namespace

void launch_entropy_size(const PassArgs &a, uint64_t first, uint64_t count, uint32_t *elen,
                         hipStream_t st)
{
    EncArgs e{a, first, count, elen, nullptr, nullptr};
    const unsigned g = (unsigned)(count < 2048 ? count : 2048);
    hipLaunchKernelGGL(k_ent_encode<false>, dim3(g), dim3(kWG), 0, st, e);
}

void launch_entropy_write(const PassArgs &a, uint64_t first, uint64_t count,
                          const uint64_t *eoff, uint8_t *out, hipStream_t st)
{
    EncArgs e{a, first, count, nullptr, eoff, out};
    const unsigned g = (unsigned)(count < 2048 ? count : 2048);
    hipLaunchKernelGGL(k_ent_encode<true>, dim3(g), dim3(kWG), 0, st, e);
}

void launch_entropy_expand(const PassArgs &a, uint64_t count, const uint8_t *src,
                           const uint64_t *soff, uint8_t *dst, const uint64_t *doff,
                           hipStream_t st)
{
    DecArgs d{a, count, src, soff, dst, doff};
    const unsigned g = (unsigned)(count < 2048 ? count : 2048);
    hipLaunchKernelGGL(k_ent_decode, dim3(g), dim3(kWG), 0, st, d);
}

}  // namespace aalc
