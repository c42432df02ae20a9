/*
 * oracle.c -- plain FP64 CPU reference for amplitude-aware lossy compressed
 * state-vector simulation.
 *
 * TEST INFRASTRUCTURE ONLY (see oracle.h).  Written for obviousness, not for
 * speed: bits are packed one at a time, every ladder level is compressed in
 * full exactly as the AALC loop states, and sums follow the perfect binary
 * tree that defines them.
 *
 * Paper sections followed:
 *   Sec. II   amplitude vector, pair update of a single-qubit gate, controlled
 *             two-qubit gate, pure-state fidelity.
 *   Sec. III  stride partition (Alg. 1), error-bounded lossy compression with
 *             normalisation before the gate, lossless compression, AALC error
 *             bound ladder and ratio threshold (Alg. 2).
 * Where the paper leaves a choice open (codec internals, stride size,
 * gates spanning strides, normalisation scope, fidelity square) this file
 * follows the readings listed in the design notes of the repository and in
 * the block-stream format definition; each such place says which reading.
 *
 * Build: cc -O2 -std=c11 -ffp-contract=off -fno-fast-math -fopenmp -shared -fPIC
 * (OpenMP only spreads the independent block groups of a pass over threads;
 * every result is the same with one thread or many.)
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_MAGIC 0x31424141u /* "AAB1" little-endian */
#define HDR_BYTES 32u
#define PLANE_HDR_BYTES 16u
#define OUTLIER_BYTES 16u
#define CHUNK 64u
/* Bound on |y| for an in-range code: 2^30 - 1, so that every code lies in
 * [-(2^30 - 1), 2^30 - 1] and every Lorenzo residual of two codes fits in 32
 * signed bits (the lossy residual of the format is then the same whether it
 * is formed in 32- or 64-bit arithmetic). */
#define QMAX 1073741823.0

/* ------------------------------------------------------------------------ */
/* growable byte buffer                                                     */
/* ------------------------------------------------------------------------ */
typedef struct {
    uint8_t *p;
    size_t len, cap;
} obuf;

static int ob_put(obuf *o, const void *src, size_t n)
{
    if (o->len + n > o->cap) {
        size_t nc = o->cap ? o->cap : 256;
        while (nc < o->len + n)
            nc *= 2;
        uint8_t *np = (uint8_t *)realloc(o->p, nc);
        if (!np)
            return OR_ENOMEM;
        o->p = np;
        o->cap = nc;
    }
    memcpy(o->p + o->len, src, n);
    o->len += n;
    return OR_OK;
}
static int ob_u32(obuf *o, uint32_t v) { return ob_put(o, &v, 4); }
static int ob_u64(obuf *o, uint64_t v) { return ob_put(o, &v, 8); }
static int ob_zero(obuf *o, size_t n)
{
    static const uint8_t z[64] = {0};
    while (n) {
        size_t k = n < 64 ? n : 64;
        if (ob_put(o, z, k))
            return OR_ENOMEM;
        n -= k;
    }
    return OR_OK;
}

static uint64_t rd_u64(const uint8_t *p) { uint64_t v; memcpy(&v, p, 8); return v; }
static uint32_t rd_u32(const uint8_t *p) { uint32_t v; memcpy(&v, p, 4); return v; }
static double rd_f64(const uint8_t *p) { double v; memcpy(&v, p, 8); return v; }
static uint64_t dbits(double x) { uint64_t v; memcpy(&v, &x, 8); return v; }
static double bitsd(uint64_t v) { double x; memcpy(&x, &v, 8); return x; }

/* ------------------------------------------------------------------------ */
/* sums                                                                     */
/* ------------------------------------------------------------------------ */

/* Perfect binary tree: sum(v[0:m]) = sum(v[0:m/2]) + sum(v[m/2:m]).  This is
 * the summation order fixed for every norm, mean and inner product. */
double or_pairwise(const double *v, size_t m)
{
    if (m == 1)
        return v[0];
    return or_pairwise(v, m / 2) + or_pairwise(v + m / 2, m / 2);
}

/* ------------------------------------------------------------------------ */
/* codec: error-bounded quantiser, integer Lorenzo predictor, fixed-length  */
/* chunk packing (Sec. III: SZ-style prediction + quantisation under an     */
/* absolute bound delta; delta = 0 is the lossless level)                   */
/* ------------------------------------------------------------------------ */

static int bitlen64(uint64_t z)
{
    int n = 0;
    while (z) {
        n++;
        z >>= 1;
    }
    return n;
}

/* zigzag of a two's-complement 64-bit difference: 0,-1,1,-2,... -> 0,1,2,3 */
static uint64_t zigzag(uint64_t c)
{
    uint64_t sign = (c >> 63) ? ~(uint64_t)0 : 0;
    return (c << 1) ^ sign;
}
static uint64_t unzigzag(uint64_t z) { return (z >> 1) ^ (0 - (z & 1)); }

/* ---- pointwise-relative levels (the log transform of Sec. III's [xin2018]
 * reference, SZ's relative mode): a ladder entry delta < 0 is the relative
 * bound eps = -delta; a value x != 0 is coded through log2|x| quantised with
 * an absolute bound dL in the log domain, its sign in the code's low bit.
 * With dL = fl(1.4 eps) < log2(1 + eps) (for eps <= 0.05), a log-domain error
 * within dL keeps |x - xhat| below eps |x|; the check below is what bounds
 * every stored value, a value that fails it is an outlier.
 *
 * clog2 / cexp2 are this codec's logarithm and power of two, built from
 * IEEE additions, multiplications and one division, each one rounding, in
 * a fixed order (the GPU evaluates the same operations): accurate to a few
 * ulps, which only decides how rarely the check fails. */
#define REL_QOFF 268435456.0   /* 2^28: offset of log codes, so codes are >= 1 */
#define REL_QRANGE 268435455.0 /* |y| < 2^28 - 1: codes 2 (q + 2^28) + sign <= 2^30 - 1 */

/* log2 a for finite a > 0: a = m 2^k with m in [sqrt(1/2), sqrt(2)),
 * ln m = 2 atanh(t), t = (m - 1)/(m + 1), by its odd series to t^15. */
static double clog2(double a)
{
    uint64_t bits = dbits(a);
    int e = (int)((bits >> 52) & 0x7FF);
    if (e == 0) { /* subnormal: scale by 2^54 first (exact) */
        bits = dbits(a * 0x1p54);
        e = (int)((bits >> 52) & 0x7FF) - 54;
    }
    double m = bitsd((bits & 0x000FFFFFFFFFFFFFull) | 0x3FF0000000000000ull);
    int k = e - 1023;
    if (m > 0x1.6a09e667f3bcdp+0) { /* m > sqrt 2 */
        m = m * 0.5;
        k = k + 1;
    }
    double t = (m - 1.0) / (m + 1.0);
    double t2 = t * t;
    double p = 0x1.1111111111111p-4; /* 1/15 */
    p = p * t2 + 0x1.3b13b13b13b14p-4;   /* 1/13 */
    p = p * t2 + 0x1.745d1745d1746p-4;   /* 1/11 */
    p = p * t2 + 0x1.c71c71c71c71cp-4;   /* 1/9 */
    p = p * t2 + 0x1.2492492492492p-3;   /* 1/7 */
    p = p * t2 + 0x1.999999999999ap-3;   /* 1/5 */
    p = p * t2 + 0x1.5555555555555p-2;   /* 1/3 */
    p = p * t2 + 1.0;
    double lnm = (2.0 * t) * p;
    return (double)k + lnm * 0x1.71547652b82fep+0; /* 1/ln 2 */
}

/* 2^y for finite y: y = k + f, f in [-1/2, 1/2], 2^f = e^(f ln 2) by its
 * Taylor series to the 13th power, then scaled by 2^k (exactly, or with one
 * rounding into the subnormals). */
static double cexp2(double y)
{
    double k = floor(y);
    double f = y - k;
    if (f > 0.5) {
        f = f - 1.0;
        k = k + 1.0;
    }
    double z = f * 0x1.62e42fefa39efp-1; /* ln 2 */
    double p = 0x1.6124613a86d09p-33; /* 1/13! */
    p = p * z + 0x1.1eed8eff8d898p-29; /* 1/12! */
    p = p * z + 0x1.ae64567f544e4p-26; /* 1/11! */
    p = p * z + 0x1.27e4fb7789f5cp-22; /* 1/10! */
    p = p * z + 0x1.71de3a556c734p-19; /* 1/9! */
    p = p * z + 0x1.a01a01a01a01ap-16; /* 1/8! */
    p = p * z + 0x1.a01a01a01a01ap-13; /* 1/7! */
    p = p * z + 0x1.6c16c16c16c17p-10; /* 1/6! */
    p = p * z + 0x1.1111111111111p-7;  /* 1/5! */
    p = p * z + 0x1.5555555555555p-5;  /* 1/4! */
    p = p * z + 0x1.5555555555555p-3;  /* 1/3! */
    p = p * z + 0.5;
    p = p * z + 1.0;
    p = p * z + 1.0;
    if (k > 1023.0)
        return INFINITY;
    if (k < -1022.0) { /* two steps: the second rounds into the subnormals */
        if (k < -1100.0)
            return 0.0;
        double two = bitsd((uint64_t)((int)k + 600 + 1023) << 52);
        return (p * two) * 0x1p-600;
    }
    return p * bitsd((uint64_t)((int)k + 1023) << 52);
}

double or_codec_log2(double a) { return clog2(a); }
double or_codec_exp2(double y) { return cexp2(y); }

/* Log-domain step of the relative bound eps: eL = 2 fl(1.4 eps). */
static double rel_step(double eps)
{
    double dl = 1.4 * eps;
    return 2.0 * dl;
}

/* Value of relative-level code c (c = 0: +0; else sign in bit 0, log code
 * (c >> 1) - 2^28 in steps of eL). */
static double rel_value(int64_t c, double eL)
{
    if (c == 0)
        return 0.0;
    double qv = (double)((c >> 1) - (int64_t)REL_QOFF);
    double mag = cexp2(qv * eL);
    return (c & 1) ? -mag : mag;
}

/* Code, outlier flag and decoded value of x at relative bound eps. */
static void rel_quantize(double x, double eps, double eL, double rL, int64_t *code,
                         uint8_t *out)
{
    if (x == 0.0) { /* +0 and -0: code 0, decoded +0, error 0 */
        *code = 0;
        *out = 0;
        return;
    }
    if (!isfinite(x)) {
        *code = 0;
        *out = 1;
        return;
    }
    double a = fabs(x);
    double y = clog2(a) * rL;
    if (!(fabs(y) < REL_QRANGE)) {
        *code = 0;
        *out = 1;
        return;
    }
    double qr = nearbyint(y);
    int64_t c = 2 * ((int64_t)qr + (int64_t)REL_QOFF) + (x < 0.0 ? 1 : 0);
    double xh = rel_value(c, eL);
    *code = c;
    *out = !(fabs(x - xh) < eps * a);
}

/* A stream's error bound: 0 (lossless), an absolute bound > 0, or a
 * relative one -eps with eps in [2^-19, 0.05] (from 2^-19 on, the log codes
 * cover every finite nonzero double: 2^28 fl(2 fl(1.4 eps)) > 1075). */
static int delta_valid(double delta)
{
    if (delta >= 0.0)
        return isfinite(delta);
    return delta >= -0.05 && delta <= -0x1p-19;
}

/* Quantise one plane of m scalars at error bound delta.
 * Lossy (delta > 0), reading of Sec. III's bound D_i - delta <= D'_i <=
 * D_i + delta, applied per real component:
 *   e = 2 delta, r = fl(1/e), y = fl(x r)
 *   if |y| < 2^30 - 1:  q = round-half-even(y), xhat = fl(q e),
 *                   outlier iff not (|fl(x - xhat)| < delta)
 *   else (also NaN): q = 0, outlier.
 * Lossless (delta == 0, the zstd role of Sec. III): q = the 64 bits of x.
 * q is returned as a 64-bit two's-complement pattern. */
static void quantize_plane(const double *v, size_t m, double delta,
                           uint64_t *q, uint8_t *outl)
{
    if (delta < 0.0) { /* relative bound eps = -delta */
        double eps = -delta;
        double eL = rel_step(eps);
        double rL = 1.0 / eL;
        for (size_t i = 0; i < m; i++) {
            int64_t c;
            rel_quantize(v[i], eps, eL, rL, &c, &outl[i]);
            q[i] = (uint64_t)c;
        }
        return;
    }
    if (delta == 0.0) {
        for (size_t i = 0; i < m; i++) {
            q[i] = dbits(v[i]);
            outl[i] = 0;
        }
        return;
    }
    double e = 2.0 * delta;
    double r = 1.0 / e;
    for (size_t i = 0; i < m; i++) {
        double y = v[i] * r;
        if (fabs(y) < QMAX) {
            double qr = nearbyint(y); /* default mode: ties to even */
            int64_t qi = (int64_t)qr;
            double xh = (double)qi * e;
            q[i] = (uint64_t)qi;
            outl[i] = !(fabs(v[i] - xh) < delta);
        } else {
            q[i] = 0;
            outl[i] = 1;
        }
    }
}

/* Set bit `pos` of a little-endian word array. */
static void setbit(uint64_t *w, uint64_t pos) { w[pos >> 6] |= (uint64_t)1 << (pos & 63); }
static int getbit(const uint64_t *w, uint64_t pos) { return (int)((w[pos >> 6] >> (pos & 63)) & 1); }

/* Encode one plane (m = 2^s scalars) as a plane record of the block stream:
 *   i64 anchor (q_0) | u32 payload_words | u32 n_outliers |
 *   [width byte per chunk, zero-padded to 8 bytes, only if payload_words>0] |
 *   payload words | outliers (u32 index, u32 0, f64 value) ascending index. */
static int encode_plane(obuf *o, const double *v, size_t m, double delta,
                        uint32_t *nout_ret)
{
    size_t nch = m / CHUNK;
    uint64_t *q = (uint64_t *)malloc(m * 8);
    uint64_t *z = (uint64_t *)malloc(m * 8);
    uint8_t *outl = (uint8_t *)malloc(m);
    uint8_t *wid = (uint8_t *)malloc(nch);
    int rc = OR_ENOMEM;
    if (!q || !z || !outl || !wid)
        goto done;

    quantize_plane(v, m, delta, q, outl);

    /* Lorenzo on the integer codes: c_0 = 0, c_i = q_i - q_{i-1}. */
    z[0] = 0;
    for (size_t i = 1; i < m; i++)
        z[i] = zigzag(q[i] - q[i - 1]);

    uint32_t pw = 0, nout = 0;
    for (size_t c = 0; c < nch; c++) {
        int w = 0;
        for (size_t l = 0; l < CHUNK; l++) {
            int bl = bitlen64(z[c * CHUNK + l]);
            if (bl > w)
                w = bl;
        }
        wid[c] = (uint8_t)w;
        pw += (uint32_t)w;
    }
    for (size_t i = 0; i < m; i++)
        nout += outl[i];

    rc = OR_ENOMEM;
    if (ob_u64(o, q[0]) || ob_u32(o, pw) || ob_u32(o, nout))
        goto done;
    if (pw > 0) {
        size_t padded = (nch + 7) / 8 * 8;
        if (ob_put(o, wid, nch) || ob_zero(o, padded - nch))
            goto done;
    }
    for (size_t c = 0; c < nch; c++) {
        int w = wid[c];
        if (w == 0)
            continue;
        uint64_t words[64];
        memset(words, 0, sizeof words);
        /* field l occupies chunk-stream bits [l*w, l*w + w), LSB first */
        for (size_t l = 0; l < CHUNK; l++)
            for (int bit = 0; bit < w; bit++)
                if ((z[c * CHUNK + l] >> bit) & 1)
                    setbit(words, (uint64_t)l * (uint64_t)w + (uint64_t)bit);
        if (ob_put(o, words, (size_t)w * 8))
            goto done;
    }
    for (size_t i = 0; i < m; i++) {
        if (!outl[i])
            continue;
        if (ob_u32(o, (uint32_t)i) || ob_u32(o, 0) || ob_u64(o, dbits(v[i])))
            goto done;
    }
    *nout_ret = nout;
    rc = OR_OK;
done:
    free(q);
    free(z);
    free(outl);
    free(wid);
    return rc;
}

/* Decode one plane record starting at p (bounded by end).  Writes m values
 * to v with stride `stride` doubles.  Returns bytes consumed or 0 on error. */
static size_t decode_plane(const uint8_t *p, const uint8_t *end, size_t m,
                           double delta, double *v, size_t stride,
                           uint32_t *nout_ret)
{
    size_t nch = m / CHUNK;
    if ((size_t)(end - p) < PLANE_HDR_BYTES)
        return 0;
    uint64_t anchor = rd_u64(p);
    /* a lossy anchor is a code: a sign-extended value within +-(2^30 - 1) */
    if (delta != 0.0 && ((int64_t)anchor > (int64_t)QMAX || (int64_t)anchor < -(int64_t)QMAX))
        return 0;
    uint32_t pw = rd_u32(p + 8);
    uint32_t nout = rd_u32(p + 12);
    const uint8_t *cur = p + PLANE_HDR_BYTES;
    uint8_t wid[CHUNK * 4]; /* nch <= 2^(s-6) <= 256 for s <= 14 */
    if (nch > sizeof wid)
        return 0;
    memset(wid, 0, nch);
    if (pw > 0) {
        size_t padded = (nch + 7) / 8 * 8;
        if ((size_t)(end - cur) < padded)
            return 0;
        memcpy(wid, cur, nch);
        cur += padded;
        uint32_t sum = 0;
        /* a lossy residual fits 32 signed bits (codes are at most
         * 2^30 - 1 in magnitude), so its zigzag is at most 32 bits wide */
        int wmax = delta == 0.0 ? 64 : 32;
        for (size_t c = 0; c < nch; c++) {
            if (wid[c] > wmax)
                return 0;
            sum += wid[c];
        }
        if (sum != pw)
            return 0;
    }
    if ((size_t)(end - cur) < (size_t)pw * 8)
        return 0;
    const uint8_t *payload = cur;
    cur += (size_t)pw * 8;

    /* unpack + unzigzag + running sum from the anchor */
    uint64_t qprev = anchor;
    size_t woff = 0;
    for (size_t c = 0; c < nch; c++) {
        int w = wid[c];
        uint64_t words[64];
        memcpy(words, payload + woff * 8, (size_t)w * 8);
        for (size_t l = 0; l < CHUNK; l++) {
            size_t i = c * CHUNK + l;
            uint64_t zz = 0;
            for (int bit = 0; bit < w; bit++)
                if (getbit(words, (uint64_t)l * (uint64_t)w + (uint64_t)bit))
                    zz |= (uint64_t)1 << bit;
            if (i == 0 && zz != 0)
                return 0; /* c_0 is 0 by definition */
            uint64_t q = (i == 0) ? anchor : qprev + unzigzag(zz);
            qprev = q;
            if (delta == 0.0)
                v[i * stride] = bitsd(q);
            else if (delta < 0.0)
                v[i * stride] = rel_value((int64_t)q, rel_step(-delta));
            else
                v[i * stride] = (double)(int64_t)q * (2.0 * delta);
        }
        woff += (size_t)w;
    }
    /* outliers replace the dequantised value with the stored one */
    if ((size_t)(end - cur) < (size_t)nout * OUTLIER_BYTES)
        return 0;
    uint32_t last = 0;
    for (uint32_t k = 0; k < nout; k++) {
        uint32_t idx = rd_u32(cur);
        if (idx >= m || (k > 0 && idx <= last) || delta == 0.0)
            return 0;
        last = idx;
        v[idx * stride] = rd_f64(cur + 8);
        cur += OUTLIER_BYTES;
    }
    *nout_ret = nout;
    return (size_t)(cur - p);
}

/* Header byte 5 holds flags; bit 0 (OR_HDR_SCALED) says that the 8 bytes
 * after the header are the block's deferred scale c (an f64, finite, > 0
 * and not 1), counted in total_bytes.  The records follow; normsq is that
 * of the stored values x-hat, without c. */
#define OR_HDR_SCALED 1u

/* The deferred scale of a stream (1 when it has none); 0 when malformed. */
static double stream_scale(const uint8_t *stream, size_t len)
{
    if (!(stream[5] & OR_HDR_SCALED))
        return 1.0;
    if (len < HDR_BYTES + 8)
        return 0.0;
    const double c = rd_f64(stream + HDR_BYTES);
    return (isfinite(c) && c > 0.0 && c != 1.0) ? c : 0.0;
}

int or_decode_block(const uint8_t *stream, size_t len, double *x)
{
    if (len < HDR_BYTES || rd_u32(stream) != OR_MAGIC)
        return OR_EINVAL;
    int s = stream[6], b = stream[7];
    if (s < 6 || s > 14 || b < s || b > 40)
        return OR_EINVAL;
    if (rd_u32(stream + 12) != len)
        return OR_EINVAL;
    double delta = rd_f64(stream + 16);
    if (!delta_valid(delta))
        return OR_EINVAL;
    if ((stream[5] & ~OR_HDR_SCALED) || stream_scale(stream, len) == 0.0)
        return OR_EINVAL;
    const uint8_t *p = stream + HDR_BYTES + ((stream[5] & OR_HDR_SCALED) ? 8 : 0);
    const uint8_t *end = stream + len;
    size_t m = (size_t)1 << s;
    size_t nseg = (size_t)1 << (b - s);
    uint32_t nout = 0;
    for (size_t g = 0; g < nseg; g++) {
        for (int pl = 0; pl < 2; pl++) {
            uint32_t no = 0;
            size_t used = decode_plane(p, end, m, delta, x + 2 * g * m + pl, 2, &no);
            if (!used)
                return OR_EINVAL;
            nout += no;
            p += used;
        }
    }
    if (p != end || nout != rd_u32(stream + 8))
        return OR_EINVAL;
    return OR_OK;
}

/* normsq of the stored block: pairwise sum over amplitude index of
 * fl(fl(re*re) + fl(im*im)). */
static double block_normsq(const double *xh, size_t namp)
{
    double *leaf = (double *)malloc(namp * sizeof(double));
    if (!leaf)
        return NAN;
    for (size_t i = 0; i < namp; i++) {
        double rr = xh[2 * i] * xh[2 * i];
        double ii = xh[2 * i + 1] * xh[2 * i + 1];
        leaf[i] = rr + ii;
    }
    double r = or_pairwise(leaf, namp);
    free(leaf);
    return r;
}

/* Compress one stride at one error bound: the compress(delta_k, s_j) step of
 * Alg. 2.  Block stream v1:
 *   header 32 B: u32 magic | u8 level | u8 0 | u8 s | u8 b | u32 n_outliers |
 *                u32 total_bytes | f64 delta | f64 normsq
 *   then for each segment, re plane record then im plane record. */
static int encode_block_obuf(obuf *o, const double *x, int b, int s,
                             double delta, int level)
{
    size_t m = (size_t)1 << s;
    size_t nseg = (size_t)1 << (b - s);
    uint8_t hdr[HDR_BYTES];
    memset(hdr, 0, sizeof hdr);
    if (ob_put(o, hdr, HDR_BYTES))
        return OR_ENOMEM;
    double *v = (double *)malloc(m * sizeof(double));
    if (!v)
        return OR_ENOMEM;
    uint32_t nout_total = 0;
    for (size_t g = 0; g < nseg; g++) {
        for (int pl = 0; pl < 2; pl++) {
            for (size_t i = 0; i < m; i++)
                v[i] = x[2 * (g * m + i) + pl];
            uint32_t no = 0;
            if (encode_plane(o, v, m, delta, &no)) {
                free(v);
                return OR_ENOMEM;
            }
            nout_total += no;
        }
    }
    free(v);
    uint32_t magic = OR_MAGIC, total = (uint32_t)o->len;
    memcpy(hdr, &magic, 4);
    hdr[4] = (uint8_t)level;
    hdr[6] = (uint8_t)s;
    hdr[7] = (uint8_t)b;
    memcpy(hdr + 8, &nout_total, 4);
    memcpy(hdr + 12, &total, 4);
    memcpy(hdr + 16, &delta, 8);
    memcpy(o->p, hdr, HDR_BYTES);

    /* normsq from the values a decoder reconstructs from these bytes */
    size_t namp = (size_t)1 << b;
    double *xh = (double *)malloc(2 * namp * sizeof(double));
    if (!xh)
        return OR_ENOMEM;
    if (or_decode_block(o->p, o->len, xh)) {
        free(xh);
        return OR_EINVAL;
    }
    double ns = block_normsq(xh, namp);
    free(xh);
    memcpy(o->p + 24, &ns, 8);
    return OR_OK;
}

int or_encode_block(const double *x, int b, int s, double delta, int level,
                    uint8_t *out, size_t cap, size_t *len)
{
    if (s < 6 || b < s || b > 30 || !delta_valid(delta) || level < 0 || level > 255)
        return OR_EINVAL;
    obuf o = {0};
    int rc = encode_block_obuf(&o, x, b, s, delta, level);
    if (rc) {
        free(o.p);
        return rc;
    }
    *len = o.len;
    if (o.len > cap) {
        free(o.p);
        return OR_ENOMEM;
    }
    memcpy(out, o.p, o.len);
    free(o.p);
    return OR_OK;
}

/* Alg. 2, inner loop for one stride: for delta_k in delta_0..delta_n,
 * ratio = compress(delta_k, s_j); stop at the first ratio >= theta.  The
 * ratio is the raw stride size 16*2^b over the stream size, compared as
 * raw >= theta * size in FP64.  If no level qualifies the loop runs out and
 * the last level's stream is kept. */
static int aalc_encode_obuf(obuf *out, const double *x, int b, int s,
                            const double *ladder, int L, double theta,
                            uint64_t *sizes)
{
    double raw = (double)((uint64_t)16 << b);
    for (int k = 0; k < L; k++)
        if (sizes)
            sizes[k] = 0;
    for (int k = 0; k < L; k++) {
        obuf o = {0};
        int rc = encode_block_obuf(&o, x, b, s, ladder[k], k);
        if (rc) {
            free(o.p);
            return rc;
        }
        if (sizes)
            sizes[k] = o.len;
        if (raw >= theta * (double)o.len || k == L - 1) {
            *out = o;
            return k;
        }
        free(o.p);
    }
    return OR_EINVAL;
}

/* A ladder: optionally lossless first (0), then lossy levels of one kind,
 * absolute bounds (> 0, >= 2^-30) strictly increasing, or relative bounds
 * (entries -eps with eps in [2^-19, 0.05]) with eps strictly increasing. */
static int ladder_ok(const double *ladder, int L, double theta)
{
    if (L < 1 || L > 8 || !(theta >= 1.0) || !isfinite(theta))
        return 0;
    int kind = 0; /* 1 absolute, -1 relative */
    for (int k = 0; k < L; k++) {
        double d = ladder[k];
        if (!isfinite(d))
            return 0;
        if (d == 0.0) {
            if (k != 0)
                return 0;
            continue;
        }
        int kk = d > 0.0 ? 1 : -1;
        if (kind && kk != kind)
            return 0;
        kind = kk;
        double mag = fabs(d);
        if (mag < (kk < 0 ? 0x1p-19 : 0x1p-30) || (kk < 0 && mag > 0.05))
            return 0;
        if (k > 0 && ladder[k - 1] != 0.0 && !(mag > fabs(ladder[k - 1])))
            return 0;
    }
    return 1;
}

int or_aalc_encode(const double *x, int b, int s, const double *ladder, int L,
                   double theta, uint8_t *out, size_t cap, size_t *len,
                   uint64_t *sizes)
{
    if (s < 6 || b < s || b > 30 || !ladder_ok(ladder, L, theta))
        return OR_EINVAL;
    obuf o = {0};
    int k = aalc_encode_obuf(&o, x, b, s, ladder, L, theta, sizes);
    if (k < 0) {
        free(o.p);
        return k;
    }
    *len = o.len;
    if (o.len > cap) {
        free(o.p);
        return OR_ENOMEM;
    }
    memcpy(out, o.p, o.len);
    free(o.p);
    return k;
}

/* ------------------------------------------------------------------------ */
/* gates (Sec. II)                                                          */
/* ------------------------------------------------------------------------ */

/* complex product u*a with one rounding per operation:
 * re = fl(fl(ur ar) - fl(ui ai)), im = fl(fl(ur ai) + fl(ui ar)) */
static void cmul(const double *u, const double *a, double *out)
{
    double rr = u[0] * a[0];
    double ii = u[1] * a[1];
    double ri = u[0] * a[1];
    double ir = u[1] * a[0];
    out[0] = rr - ii;
    out[1] = ri + ir;
}

/* Coupling mask: amplitude i interacts with i ^ mask (0 = diagonal). */
static uint64_t gate_mask(const or_gate *g)
{
    switch (g->kind) {
    case OR_G_U:
    case OR_G_X:
        return (uint64_t)1 << g->q0;
    case OR_G_CU:
        return (uint64_t)1 << g->q1;
    case OR_G_SWAP:
        return ((uint64_t)1 << g->q0) | ((uint64_t)1 << g->q1);
    default:
        return 0;
    }
}

static int gate_valid(const or_gate *g, int n)
{
    switch (g->kind) {
    case OR_G_U:
    case OR_G_DIAG1:
    case OR_G_X:
        return g->q0 >= 0 && g->q0 < n;
    case OR_G_CU:
    case OR_G_CPHASE:
    case OR_G_CZ:
    case OR_G_SWAP:
        return g->q0 >= 0 && g->q0 < n && g->q1 >= 0 && g->q1 < n && g->q0 != g->q1;
    case OR_G_PHASE_FLIP:
        return g->index < ((uint64_t)1 << n);
    case OR_G_DIFFUSE:
        return 1;
    default:
        return 0;
    }
}

/* A view of up to two blocks of the state by global amplitude index. */
typedef struct {
    double *base[2];
    uint64_t blk[2];
    int nb;
    int b;
} gview;

static double *at(const gview *v, uint64_t i)
{
    uint64_t j = i >> v->b;
    int k = (v->nb == 2 && j == v->blk[1]) ? 1 : 0;
    return v->base[k] + 2 * (i & (((uint64_t)1 << v->b) - 1));
}

static int bit(uint64_t i, int q) { return (int)((i >> q) & 1); }

/* Apply gate g to every amplitude of the view.  Pair gates follow the
 * Sec. II update [a0'; a1'] = U [a0; a1] on indices that differ only in the
 * target bit; the controlled form acts where the control bit is 1. */
static void gate_apply(const or_gate *g, const gview *v, const double *tdiff)
{
    uint64_t mask = gate_mask(g);
    uint64_t per = (uint64_t)1 << v->b;
    const double *u00 = g->u, *u01 = g->u + 2, *u10 = g->u + 4, *u11 = g->u + 6;
    for (int k = 0; k < v->nb; k++) {
        for (uint64_t li = 0; li < per; li++) {
            uint64_t i = (v->blk[k] << v->b) | li;
            if (mask) {
                uint64_t j = i ^ mask;
                if (!(i < j))
                    continue;
                double *a = at(v, i), *bb = at(v, j);
                switch (g->kind) {
                case OR_G_CU: /* U on the control = 1 subspace */
                    if (!bit(i, g->q0))
                        break;
                    /* fall through */
                case OR_G_U: {
                    double p[2], q[2], r[2], t[2];
                    cmul(u00, a, p);
                    cmul(u01, bb, q);
                    cmul(u10, a, r);
                    cmul(u11, bb, t);
                    a[0] = p[0] + q[0];
                    a[1] = p[1] + q[1];
                    bb[0] = r[0] + t[0];
                    bb[1] = r[1] + t[1];
                    break;
                }
                case OR_G_X:
                case OR_G_SWAP:
                    if (g->kind == OR_G_SWAP && bit(i, g->q0) == bit(i, g->q1))
                        break;
                    {
                        double t0 = a[0], t1 = a[1];
                        a[0] = bb[0];
                        a[1] = bb[1];
                        bb[0] = t0;
                        bb[1] = t1;
                    }
                    break;
                default:
                    break;
                }
            } else {
                double *a = at(v, i);
                switch (g->kind) {
                case OR_G_DIAG1:
                    if (bit(i, g->q0)) {
                        double r[2];
                        cmul(u11, a, r);
                        a[0] = r[0];
                        a[1] = r[1];
                    }
                    break;
                case OR_G_CPHASE:
                    if (bit(i, g->q0) && bit(i, g->q1)) {
                        double r[2];
                        cmul(u11, a, r);
                        a[0] = r[0];
                        a[1] = r[1];
                    }
                    break;
                case OR_G_CZ:
                    if (bit(i, g->q0) && bit(i, g->q1)) {
                        a[0] = -a[0];
                        a[1] = -a[1];
                    }
                    break;
                case OR_G_PHASE_FLIP:
                    if (i == g->index) {
                        a[0] = -a[0];
                        a[1] = -a[1];
                    }
                    break;
                case OR_G_DIFFUSE:
                    /* (2|s><s| - I) psi = 2 mean(psi) - psi, per component */
                    a[0] = tdiff[0] - a[0];
                    a[1] = tdiff[1] - a[1];
                    break;
                default:
                    break;
                }
            }
        }
    }
}

/* Pairwise mean-doubling for DIFFUSE over a plain array:
 * t = 2 * (pairwise sum) / 2^n, the division being an exact power-of-two
 * scaling. */
static int diffuse_t_plain(const double *amp, int n, double *t)
{
    size_t N = (size_t)1 << n;
    double *tmp = (double *)malloc(N * sizeof(double));
    if (!tmp)
        return OR_ENOMEM;
    for (int c = 0; c < 2; c++) {
        for (size_t i = 0; i < N; i++)
            tmp[i] = amp[2 * i + c];
        t[c] = or_pairwise(tmp, N) * ldexp(1.0, 1 - n);
    }
    free(tmp);
    return OR_OK;
}

int or_sv_apply_gate(double *amp, int n, const or_gate *g)
{
    if (n < 1 || n > 34 || !g || !gate_valid(g, n))
        return OR_EINVAL;
    double t[2] = {0.0, 0.0};
    if (g->kind == OR_G_DIFFUSE && diffuse_t_plain(amp, n, t))
        return OR_ENOMEM;
    gview v = {{amp, amp}, {0, 0}, 1, n};
    gate_apply(g, &v, t);
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Alg. 2 driver                                                            */
/* ------------------------------------------------------------------------ */

struct or_sim {
    int n, b, s, L, normalize;
    int shortcut;        /* OR_SC_* flags (Sec. V); 0 = Alg. 2 as written */
    double ladder[8];
    double theta;
    uint64_t nblocks;
    uint8_t **streams;   /* plain block streams (header byte 5 is 0) */
    size_t *lens;
    double *bscale;      /* per-block deferred scale c_j (1.0 unless skipped) */
    double normsq, scale;
    int collapsed;
    double min_ratio, last_ratio;
    uint64_t passes;
    uint64_t level_hist[8];
};

static void normalize_block(double *x, size_t nscalar, double scale)
{
    if (scale == 1.0)
        return; /* multiplying by 1 is the identity; skipping keeps NaN bits */
    for (size_t i = 0; i < nscalar; i++)
        x[i] = x[i] * scale;
}

/* Encode one block at level `level` only (no other level tried). */
static int fixed_encode_obuf(obuf *out, const double *x, int b, int s,
                             const double *ladder, int level)
{
    return encode_block_obuf(out, x, b, s, ladder[level], level) ? OR_ENOMEM : level;
}

/* Decompress, normalise, gateComputation and AALC-compress one group: the
 * body of Alg. 2 for the stride(s) a gate touches together.  A gate whose
 * pairs span two strides processes both strides of each coupled pair as one
 * group (reading of Alg. 1 for high qubits).  fac[k] is the factor the
 * decoded values of block k are multiplied by (the normalisation s, times
 * the block's deferred scale when it has one); force[k] >= 0 encodes block k
 * at that level instead of running the ladder (permutation shortcut). */
static int group_run_f(int n, int b, int s, const double *ladder, int L,
                       double theta, const double *fac, const int *force,
                       const double *tdiff, const or_gate *g, uint64_t j0,
                       const uint8_t *const *in, const size_t *inlen, obuf *out,
                       int *levels)
{
    (void)n;
    uint64_t mb = gate_mask(g) >> b;
    int nb = mb ? 2 : 1;
    size_t namp = (size_t)1 << b;
    double *x[2] = {NULL, NULL};
    int rc = OR_OK;
    for (int k = 0; k < nb; k++) {
        x[k] = (double *)malloc(2 * namp * sizeof(double));
        if (!x[k]) {
            rc = OR_ENOMEM;
            goto done;
        }
        if (or_decode_block(in[k], inlen[k], x[k])) {
            rc = OR_EINVAL;
            goto done;
        }
        normalize_block(x[k], 2 * namp, fac[k]);
    }
    {
        gview v = {{x[0], x[1]}, {j0, j0 ^ mb}, nb, b};
        gate_apply(g, &v, tdiff);
    }
    for (int k = 0; k < nb; k++) {
        int lev = (force && force[k] >= 0)
                      ? fixed_encode_obuf(&out[k], x[k], b, s, ladder, force[k])
                      : aalc_encode_obuf(&out[k], x[k], b, s, ladder, L, theta, NULL);
        if (lev < 0) {
            rc = lev;
            goto done;
        }
        levels[k] = lev;
    }
done:
    free(x[0]);
    free(x[1]);
    return rc;
}

static int group_run(int n, int b, int s, const double *ladder, int L,
                     double theta, double scale, const double *tdiff,
                     const or_gate *g, uint64_t j0, const uint8_t *const *in,
                     const size_t *inlen, obuf *out, int *levels)
{
    const double fac[2] = {scale, scale};
    return group_run_f(n, b, s, ladder, L, theta, fac, NULL, tdiff, g, j0, in,
                       inlen, out, levels);
}

int or_process_group(int n, int b, int s, const double *ladder, int L,
                     double theta, double scale, const double *tdiff,
                     const or_gate *g, uint64_t j0, const uint8_t *in0,
                     size_t len0, const uint8_t *in1, size_t len1,
                     uint8_t *out0, size_t cap0, size_t *olen0, uint8_t *out1,
                     size_t cap1, size_t *olen1)
{
    if (s < 6 || b < s || b > n || n > 48 || !ladder_ok(ladder, L, theta) ||
        !g || !gate_valid(g, n) || j0 >= ((uint64_t)1 << (n - b)))
        return OR_EINVAL;
    uint64_t mb = gate_mask(g) >> b;
    if (mb && (j0 ^ mb) < j0)
        return OR_EINVAL; /* the group is named by its lower block */
    double t0[2] = {0.0, 0.0};
    const uint8_t *in[2] = {in0, in1};
    size_t inl[2] = {len0, len1};
    obuf out[2] = {{0}, {0}};
    int lev[2];
    int rc = group_run(n, b, s, ladder, L, theta, scale, tdiff ? tdiff : t0, g,
                       j0, in, inl, out, lev);
    if (rc == OR_OK) {
        *olen0 = out[0].len;
        if (out[0].len > cap0)
            rc = OR_ENOMEM;
        else
            memcpy(out0, out[0].p, out[0].len);
        if (mb) {
            *olen1 = out[1].len;
            if (out[1].len > cap1)
                rc = OR_ENOMEM;
            else
                memcpy(out1, out[1].p, out[1].len);
        }
    }
    free(out[0].p);
    free(out[1].p);
    return rc;
}

static double stream_normsq(const uint8_t *p) { return rd_f64(p + 24); }

/* N^2 = pairwise over blocks of the per-block normsq (the block sums are the
 * aligned subtrees of the tree over all 2^n amplitudes); s = 1/sqrt(N^2),
 * applied before the next gate (Sec. III: the state vector is normalised
 * before the gate computation). */
/* Bytes of block j as exported: its stream, plus the 8-byte deferred scale
 * when that is not 1. */
static size_t export_len(const or_sim *sim, uint64_t j)
{
    return sim->lens[j] + (sim->bscale[j] != 1.0 ? 8 : 0);
}

/* Weight of block j in N^2: its normsq, times fl(c_j^2) when the block
 * carries a deferred scale c_j != 1. */
static double block_weight(const or_sim *sim, uint64_t j)
{
    const double ns = stream_normsq(sim->streams[j]);
    const double c = sim->bscale[j];
    if (c == 1.0)
        return ns;
    const double c2 = c * c;
    return ns * c2;
}

/* Factor the decoded values of block j are multiplied by before the gate
 * (and in every read-out): fl(c_j * s); s itself when c_j is 1. */
static double block_factor(const or_sim *sim, uint64_t j)
{
    return sim->bscale[j] * sim->scale;
}

static void update_norm(or_sim *sim)
{
    double *v = (double *)malloc(sim->nblocks * sizeof(double));
    uint64_t total = 0;
    for (uint64_t j = 0; j < sim->nblocks; j++) {
        v[j] = block_weight(sim, j);
        total += export_len(sim, j);
    }
    sim->normsq = or_pairwise(v, sim->nblocks);
    free(v);
    double N2 = sim->normsq;
    if (N2 > 0.0 && isfinite(N2)) {
        if (sim->normalize)
            sim->scale = 1.0 / sqrt(N2);
    } else {
        sim->collapsed = 1;
        sim->scale = 1.0;
    }
    double raw = (double)((uint64_t)16 << sim->n);
    sim->last_ratio = raw / (double)total;
    if (sim->passes == 0 || sim->last_ratio < sim->min_ratio)
        sim->min_ratio = sim->last_ratio;
}

or_sim *or_create(int n, int b, int s, const double *ladder, int L,
                  double theta, int normalize)
{
    if (n < 6 || n > 40 || b < 6 || b > n || b > 30 || s < 6 || s > 14 || s > b ||
        !ladder_ok(ladder, L, theta))
        return NULL;
    or_sim *sim = (or_sim *)calloc(1, sizeof *sim);
    if (!sim)
        return NULL;
    sim->n = n;
    sim->b = b;
    sim->s = s;
    sim->L = L;
    sim->normalize = normalize ? 1 : 0;
    memcpy(sim->ladder, ladder, (size_t)L * sizeof(double));
    sim->theta = theta;
    sim->nblocks = (uint64_t)1 << (n - b);
    sim->streams = (uint8_t **)calloc(sim->nblocks, sizeof(uint8_t *));
    sim->lens = (size_t *)calloc(sim->nblocks, sizeof(size_t));
    sim->bscale = (double *)malloc(sim->nblocks * sizeof(double));
    if (!sim->streams || !sim->lens || !sim->bscale || or_set_basis(sim, 0)) {
        or_destroy(sim);
        return NULL;
    }
    return sim;
}

void or_destroy(or_sim *sim)
{
    if (!sim)
        return;
    if (sim->streams)
        for (uint64_t j = 0; j < sim->nblocks; j++)
            free(sim->streams[j]);
    free(sim->streams);
    free(sim->lens);
    free(sim->bscale);
    free(sim);
}

int or_set_basis(or_sim *sim, uint64_t x)
{
    if (!sim || x >= ((uint64_t)1 << sim->n))
        return OR_EINVAL;
    size_t namp = (size_t)1 << sim->b;
    double *blk = (double *)calloc(2 * namp, sizeof(double));
    if (!blk)
        return OR_ENOMEM;
    for (uint64_t j = 0; j < sim->nblocks; j++) {
        int has = (x >> sim->b) == j;
        if (has)
            blk[2 * (x & (namp - 1))] = 1.0;
        obuf o = {0};
        int lev = aalc_encode_obuf(&o, blk, sim->b, sim->s, sim->ladder, sim->L,
                                   sim->theta, NULL);
        if (has)
            blk[2 * (x & (namp - 1))] = 0.0;
        if (lev < 0) {
            free(blk);
            free(o.p);
            return lev;
        }
        free(sim->streams[j]);
        sim->streams[j] = o.p;
        sim->lens[j] = o.len;
        sim->bscale[j] = 1.0;
    }
    free(blk);
    sim->collapsed = 0;
    sim->scale = 1.0;
    sim->passes = 0;
    memset(sim->level_hist, 0, sizeof sim->level_hist);
    update_norm(sim);
    return OR_OK;
}

/* S = pairwise over all amplitudes of the normalised decoded values (per
 * component).  Block sums are aligned subtrees. */
int or_amplitude_sum(const or_sim *sim, double *S)
{
    size_t namp = (size_t)1 << sim->b;
    double *x = (double *)malloc(2 * namp * sizeof(double));
    double *tmp = (double *)malloc(namp * sizeof(double));
    double *bs[2];
    bs[0] = (double *)malloc(sim->nblocks * sizeof(double));
    bs[1] = (double *)malloc(sim->nblocks * sizeof(double));
    int rc = OR_ENOMEM;
    if (!x || !tmp || !bs[0] || !bs[1])
        goto done;
    for (uint64_t j = 0; j < sim->nblocks; j++) {
        rc = or_decode_block(sim->streams[j], sim->lens[j], x);
        if (rc)
            goto done;
        normalize_block(x, 2 * namp, block_factor(sim, j));
        for (int c = 0; c < 2; c++) {
            for (size_t i = 0; i < namp; i++)
                tmp[i] = x[2 * i + c];
            bs[c][j] = or_pairwise(tmp, namp);
        }
    }
    for (int c = 0; c < 2; c++)
        S[c] = or_pairwise(bs[c], sim->nblocks);
    rc = OR_OK;
done:
    free(x);
    free(tmp);
    free(bs[0]);
    free(bs[1]);
    return rc;
}

/* Whether the gate leaves amplitude i as it is, by the structure of the
 * gate alone (its kind and qubits, not its matrix entries): a diagonal or
 * controlled gate acts only where its qubits are 1, PHASE_FLIP only at its
 * index, SWAP only where its two bits differ. */
static int leaves_unchanged(const or_gate *g, uint64_t i)
{
    switch (g->kind) {
    case OR_G_DIAG1:
        return !bit(i, g->q0);
    case OR_G_CPHASE:
    case OR_G_CZ:
        return !(bit(i, g->q0) && bit(i, g->q1));
    case OR_G_CU:
        return !bit(i, g->q0);
    case OR_G_PHASE_FLIP:
        return i != g->index;
    case OR_G_SWAP:
        return bit(i, g->q0) == bit(i, g->q1);
    default:
        return 0;
    }
}

/* A stride none of whose amplitudes the gate changes (Sec. V: such strides
 * need not be compressed again). */
static int block_untouched(const or_gate *g, int b, uint64_t j)
{
    const uint64_t per = (uint64_t)1 << b;
    for (uint64_t li = 0; li < per; li++)
        if (!leaves_unchanged(g, (j << b) | li))
            return 0;
    return 1;
}

/* Gates that only reorder amplitudes (Sec. V: X, CNOT; SWAP likewise): X,
 * SWAP, and the controlled form of exactly [[0, 1], [1, 0]]. */
static int is_permutation(const or_gate *g)
{
    if (g->kind == OR_G_X || g->kind == OR_G_SWAP)
        return 1;
    if (g->kind != OR_G_CU)
        return 0;
    static const double X[8] = {0.0, 0.0, 1.0, 0.0, 1.0, 0.0, 0.0, 0.0};
    for (int k = 0; k < 8; k++)
        if (dbits(g->u[k]) != dbits(X[k]))
            return 0;
    return 1;
}

int or_set_shortcut(or_sim *sim, int flags)
{
    if (!sim || (flags & ~(OR_SC_PERMUTE | OR_SC_SKIP)))
        return OR_EINVAL;
    sim->shortcut = flags;
    return OR_OK;
}

/* Alg. 2: for each gate, for each stride (group): decompress, normalize,
 * gateComputation, AALC compress.  Every block is re-encoded on every gate,
 * including blocks the gate leaves unchanged, as Alg. 1 states -- unless a
 * shortcut of Sec. V is on:
 *   OR_SC_PERMUTE: under a gate that only reorders amplitudes (X, SWAP,
 *     CNOT) each block is compressed at the ladder level its own previous
 *     stream used, without trying other levels;
 *   OR_SC_SKIP: a block the gate leaves unchanged keeps its stream; its
 *     normalisation is deferred into the block's scale c_j <- fl(c_j s), and
 *     a block is decoded with the factor fl(c_j s) (c_j back to 1 once it is
 *     compressed again). */
int or_apply_gate(or_sim *sim, const or_gate *g)
{
    if (!sim || !g || !gate_valid(g, sim->n))
        return OR_EINVAL;
    double t[2] = {0.0, 0.0};
    if (g->kind == OR_G_DIFFUSE) {
        /* (2|s><s| - I): t = 2 * mean = S * 2^(1-n) per component */
        int rc = or_amplitude_sum(sim, t);
        if (rc)
            return rc;
        for (int c = 0; c < 2; c++)
            t[c] = t[c] * ldexp(1.0, 1 - sim->n);
    }
    const int perm = (sim->shortcut & OR_SC_PERMUTE) && is_permutation(g);
    const int skip = (sim->shortcut & OR_SC_SKIP) != 0;
    uint64_t mb = gate_mask(g) >> sim->b;
    uint8_t **ns = (uint8_t **)calloc(sim->nblocks, sizeof(uint8_t *));
    size_t *nl = (size_t *)calloc(sim->nblocks, sizeof(size_t));
    uint8_t *lv = (uint8_t *)calloc(sim->nblocks, 1);
    double *nc = (double *)malloc(sim->nblocks * sizeof(double));
    int rc = OR_OK;
    if (!ns || !nl || !lv || !nc) {
        rc = OR_ENOMEM;
        goto fail;
    }
    /* The groups are independent (each reads its own input streams and
     * writes its own output streams), so they may run on several threads;
     * the result does not depend on the order. */
#pragma omp parallel for schedule(dynamic, 1)
    for (uint64_t j = 0; j < sim->nblocks; j++) {
        if (mb && (j ^ mb) < j)
            continue;
        const int nbk = mb ? 2 : 1;
        const uint64_t jj[2] = {j, j ^ mb};
        int r = OR_OK;
        if (skip && block_untouched(g, sim->b, jj[0]) &&
            (nbk == 1 || block_untouched(g, sim->b, jj[1]))) {
            for (int k = 0; k < nbk && !r; k++) {
                const uint64_t q = jj[k];
                uint8_t *cp = (uint8_t *)malloc(sim->lens[q]);
                if (!cp) {
                    r = OR_ENOMEM;
                    break;
                }
                memcpy(cp, sim->streams[q], sim->lens[q]);
                ns[q] = cp;
                nl[q] = sim->lens[q];
                lv[q] = sim->streams[q][4];
                nc[q] = sim->bscale[q] * sim->scale;
            }
        } else {
            const uint8_t *in[2] = {sim->streams[j], mb ? sim->streams[j ^ mb] : NULL};
            size_t inl[2] = {sim->lens[j], mb ? sim->lens[j ^ mb] : 0};
            const double fac[2] = {block_factor(sim, j), mb ? block_factor(sim, j ^ mb) : 1.0};
            const int force[2] = {perm ? (int)sim->streams[j][4] : -1,
                                  perm && mb ? (int)sim->streams[j ^ mb][4] : -1};
            obuf out[2] = {{0}, {0}};
            int lev[2] = {0, 0};
            r = group_run_f(sim->n, sim->b, sim->s, sim->ladder, sim->L, sim->theta, fac,
                            force, t, g, j, in, inl, out, lev);
            if (r) {
                free(out[0].p);
                free(out[1].p);
            } else {
                for (int k = 0; k < nbk; k++) {
                    ns[jj[k]] = out[k].p;
                    nl[jj[k]] = out[k].len;
                    lv[jj[k]] = (uint8_t)lev[k];
                    nc[jj[k]] = 1.0;
                }
            }
        }
        if (r) {
#pragma omp critical(or_rc)
            rc = rc ? rc : r;
        }
    }
    if (rc)
        goto fail;
    uint64_t hist[8] = {0};
    for (uint64_t j = 0; j < sim->nblocks; j++)
        hist[lv[j]]++;
    for (uint64_t j = 0; j < sim->nblocks; j++) {
        free(sim->streams[j]);
        sim->streams[j] = ns[j];
        sim->lens[j] = nl[j];
    }
    memcpy(sim->bscale, nc, sim->nblocks * sizeof(double));
    free(ns);
    free(nl);
    free(lv);
    free(nc);
    for (int k = 0; k < 8; k++)
        sim->level_hist[k] += hist[k];
    sim->passes++;
    update_norm(sim);
    return sim->collapsed ? OR_ECOLLAPSED : OR_OK;
fail:
    if (ns)
        for (uint64_t j = 0; j < sim->nblocks; j++)
            free(ns[j]);
    free(ns);
    free(nl);
    free(lv);
    free(nc);
    return rc;
}

int or_set_threads(int nthreads)
{
#ifdef _OPENMP
    if (nthreads < 1)
        return OR_EINVAL;
    omp_set_num_threads(nthreads);
    return omp_get_max_threads();
#else
    (void)nthreads;
    return 1;
#endif
}

int or_get_amplitudes(const or_sim *sim, uint64_t first, uint64_t count,
                      double *out)
{
    if (!sim || first + count > ((uint64_t)1 << sim->n) || first + count < first)
        return OR_EINVAL;
    size_t namp = (size_t)1 << sim->b;
    double *x = (double *)malloc(2 * namp * sizeof(double));
    if (!x)
        return OR_ENOMEM;
    uint64_t cur = ~(uint64_t)0;
    for (uint64_t k = 0; k < count; k++) {
        uint64_t i = first + k, j = i >> sim->b;
        if (j != cur) {
            if (or_decode_block(sim->streams[j], sim->lens[j], x)) {
                free(x);
                return OR_EINVAL;
            }
            normalize_block(x, 2 * namp, block_factor(sim, j));
            cur = j;
        }
        out[2 * k] = x[2 * (i & (namp - 1))];
        out[2 * k + 1] = x[2 * (i & (namp - 1)) + 1];
    }
    free(x);
    return OR_OK;
}

int or_export_block(const or_sim *sim, uint64_t j, uint8_t *buf, size_t cap,
                    size_t *len)
{
    if (!sim || j >= sim->nblocks)
        return OR_EINVAL;
    const size_t L = export_len(sim, j);
    *len = L;
    if (cap < L)
        return OR_ENOMEM;
    if (L == sim->lens[j]) {
        memcpy(buf, sim->streams[j], L);
        return OR_OK;
    }
    /* a deferred scale: flag it in the header, place it after the header */
    memcpy(buf, sim->streams[j], HDR_BYTES);
    buf[5] |= OR_HDR_SCALED;
    const uint32_t total = (uint32_t)L;
    memcpy(buf + 12, &total, 4);
    memcpy(buf + HDR_BYTES, &sim->bscale[j], 8);
    memcpy(buf + HDR_BYTES + 8, sim->streams[j] + HDR_BYTES, sim->lens[j] - HDR_BYTES);
    return OR_OK;
}

/* Checkpoint resume: the state becomes the one whose block streams are
 * given, exactly as if those streams had just been written by a pass (the
 * per-block normsq fields give N^2 and the scale of the next gate, as after
 * every pass).  Each stream is checked before anything is replaced: header
 * fields against this simulator (magic, s, b, a ladder level whose bound
 * equals the header's delta bit for bit), the records as or_decode_block
 * checks them, and the header normsq against the normsq of the decoded
 * values.  On any failure the state is left unchanged. */
int or_import_state(or_sim *sim, const uint8_t *buf, size_t len)
{
    if (!sim || (!buf && len))
        return OR_EINVAL;
    size_t namp = (size_t)1 << sim->b;
    uint64_t nb = sim->nblocks;
    size_t *off = (size_t *)malloc(nb * sizeof(size_t));
    size_t *ln = (size_t *)malloc(nb * sizeof(size_t));
    double *x = (double *)malloc(2 * namp * sizeof(double));
    uint8_t **copies = (uint8_t **)calloc(nb, sizeof(uint8_t *));
    int rc = OR_ENOMEM;
    if (!off || !ln || !x || !copies)
        goto done;
    rc = OR_EINVAL;
    size_t pos = 0;
    for (uint64_t j = 0; j < nb; j++) {
        if (len - pos < HDR_BYTES)
            goto done;
        const uint8_t *h = buf + pos;
        uint32_t total = rd_u32(h + 12);
        int level = h[4];
        if (rd_u32(h) != OR_MAGIC || (h[5] & ~OR_HDR_SCALED) || h[6] != sim->s ||
            h[7] != sim->b || level >= sim->L ||
            dbits(rd_f64(h + 16)) != dbits(sim->ladder[level]) || total < HDR_BYTES ||
            total > len - pos)
            goto done;
        if (or_decode_block(h, total, x) != OR_OK)
            goto done;
        if (dbits(block_normsq(x, namp)) != dbits(rd_f64(h + 24)))
            goto done;
        off[j] = pos;
        ln[j] = total;
        pos += total;
    }
    if (pos != len)
        goto done;
    rc = OR_ENOMEM;
    /* stored as plain streams, the deferred scales beside them */
    for (uint64_t j = 0; j < nb; j++) {
        const uint8_t *h = buf + off[j];
        const size_t extra = (h[5] & OR_HDR_SCALED) ? 8 : 0;
        copies[j] = (uint8_t *)malloc(ln[j] - extra);
        if (!copies[j])
            goto done;
        memcpy(copies[j], h, HDR_BYTES);
        copies[j][5] = 0;
        const uint32_t plain = (uint32_t)(ln[j] - extra);
        memcpy(copies[j] + 12, &plain, 4);
        memcpy(copies[j] + HDR_BYTES, h + HDR_BYTES + extra, ln[j] - extra - HDR_BYTES);
    }
    for (uint64_t j = 0; j < nb; j++) {
        const uint8_t *h = buf + off[j];
        const size_t extra = (h[5] & OR_HDR_SCALED) ? 8 : 0;
        free(sim->streams[j]);
        sim->streams[j] = copies[j];
        sim->lens[j] = ln[j] - extra;
        sim->bscale[j] = stream_scale(h, ln[j]);
        copies[j] = NULL;
    }
    sim->collapsed = 0;
    sim->scale = 1.0;
    sim->passes = 0;
    memset(sim->level_hist, 0, sizeof sim->level_hist);
    update_norm(sim);
    rc = sim->collapsed ? OR_ECOLLAPSED : OR_OK;
done:
    if (copies)
        for (uint64_t j = 0; j < nb; j++)
            free(copies[j]);
    free(copies);
    free(x);
    free(ln);
    free(off);
    return rc;
}

int or_get_stats(const or_sim *sim, or_stats *st)
{
    if (!sim || !st)
        return OR_EINVAL;
    memset(st, 0, sizeof *st);
    st->normsq = sim->normsq;
    st->scale = sim->scale;
    st->collapsed = sim->collapsed;
    for (uint64_t j = 0; j < sim->nblocks; j++)
        st->resident_bytes += export_len(sim, j);
    st->min_ratio = sim->min_ratio;
    st->last_ratio = sim->last_ratio;
    st->passes = sim->passes;
    memcpy(st->level_hist, sim->level_hist, sizeof st->level_hist);
    return OR_OK;
}

/* Outcome probabilities of the listed qubits: P(o) = sum over indices whose
 * listed bits spell o of |a_i|^2, a = normalised amplitudes, ascending i. */
int or_measure_probs(const or_sim *sim, const int *qubits, int nq,
                     double *probs)
{
    if (!sim || nq < 1 || nq > 24)
        return OR_EINVAL;
    for (int k = 0; k < nq; k++) {
        if (qubits[k] < 0 || qubits[k] >= sim->n)
            return OR_EINVAL;
        for (int m = 0; m < k; m++)
            if (qubits[m] == qubits[k])
                return OR_EINVAL;
    }
    memset(probs, 0, ((size_t)1 << nq) * sizeof(double));
    size_t namp = (size_t)1 << sim->b;
    double *x = (double *)malloc(2 * namp * sizeof(double));
    if (!x)
        return OR_ENOMEM;
    for (uint64_t j = 0; j < sim->nblocks; j++) {
        if (or_decode_block(sim->streams[j], sim->lens[j], x)) {
            free(x);
            return OR_EINVAL;
        }
        normalize_block(x, 2 * namp, block_factor(sim, j));
        for (size_t li = 0; li < namp; li++) {
            uint64_t i = (j << sim->b) | li;
            uint64_t o = 0;
            for (int k = 0; k < nq; k++)
                o |= (uint64_t)bit(i, qubits[k]) << k;
            double rr = x[2 * li] * x[2 * li];
            double ii = x[2 * li + 1] * x[2 * li + 1];
            probs[o] += rr + ii;
        }
    }
    free(x);
    return OR_OK;
}

/* Pure-state fidelity (Sec. II) with the modulus squared and both norms
 * divided out, so that it lies in [0, 1] for any two non-zero vectors. */
double or_fidelity(const double *a, const double *b, int n)
{
    size_t N = (size_t)1 << n;
    double *re = (double *)malloc(N * sizeof(double));
    double *im = (double *)malloc(N * sizeof(double));
    double *na = (double *)malloc(N * sizeof(double));
    double *nb = (double *)malloc(N * sizeof(double));
    double F = NAN;
    if (re && im && na && nb) {
        for (size_t i = 0; i < N; i++) {
            double ar = a[2 * i], ai = a[2 * i + 1], br = b[2 * i], bi = b[2 * i + 1];
            double p1 = ar * br, p2 = ai * bi, p3 = ar * bi, p4 = ai * br;
            re[i] = p1 + p2; /* conj(a) b */
            im[i] = p3 - p4;
            double q1 = ar * ar, q2 = ai * ai, q3 = br * br, q4 = bi * bi;
            na[i] = q1 + q2;
            nb[i] = q3 + q4;
        }
        double R = or_pairwise(re, N), I = or_pairwise(im, N);
        double A = or_pairwise(na, N), B = or_pairwise(nb, N);
        double num = R * R + I * I;
        F = num / (A * B);
    }
    free(re);
    free(im);
    free(na);
    free(nb);
    return F;
}

/* ------------------------------------------------------------------------ */
/* entropy stage: block entropy stream v1                                   */
/* ------------------------------------------------------------------------ */
/* SZ follows its predictor and quantiser with an entropy coder and a
 * dictionary coder (Sec. III names SZ's pipeline).  This stage re-codes a
 * block stream v1 losslessly, at two levels:
 *
 *  * plane runs: a plane record equal byte for byte to the record two planes
 *    before it (the same component of the previous segment) is a repeat;
 *    each maximal run of consecutive repeats is one item with no body;
 *  * chunk codes: the 64 zigzagged residuals z_l of a chunk of width w > 0
 *    are written in the shortest of three codes -- fixed width w (as in
 *    v1), cost 64 w bits; Golomb-Rice with parameter k < w (q = z >> k
 *    one-bits, a zero bit, then the k low bits of z, least significant
 *    first), cost 64 (k + 1) + sum_l (z_l >> k), the smallest k of least
 *    cost taken; sparse, cost 64 + nnz w: a 64-bit mask whose bit l says
 *    z_l != 0, then each nonzero z_l (l ascending) in w bits.  Ties go to
 *    fixed width, then Rice, then sparse.  For geometrically distributed
 *    residuals the Golomb codes are the optimal prefix codes (Gallager and
 *    van Voorhis, 1975), i.e. the Huffman code; the sparse code is the
 *    zero-run coder of chunks that hold a few nonzero residuals.
 *
 * Layout (little-endian):
 *   header (32 B): the v1 header with magic 0x31454141 ("AAE1") and
 *                  total_bytes = the length of this stream
 *   u32 v1_bytes (length of the v1 stream) | u32 n_items
 *   [f64 scale]    iff header flag bit 0, as in v1
 *   n_items u32 tags, zero-padded to a multiple of 8 bytes
 *   item bodies in item order
 * A tag with bit 31 set is a run of (tag & 0x7FFFFFFF) >= 1 repeat planes
 * (never one of the first two planes); otherwise it is one literal plane:
 * with bit 30 set its body is the v1 record itself, of (tag & 0x3FFFFFFF)
 * bytes (taken when the coded body would not be shorter); else the tag is
 * the byte count of its coded body:
 *   i64 anchor | u32 payload_words (pw, v1's) | u32 n_outliers
 *   if pw > 0:
 *     u32 coded_words | u32 0
 *     C mode bytes, zero-padded to a multiple of 8
 *     u16 coded bit length of each chunk that is not fixed-width, in chunk
 *       order, zero-padded to a multiple of 8 bytes
 *     coded_words u64 words: the chunks' codes back to back in chunk order
 *       in one little-endian bit stream, zero-padded to a whole word
 *   outliers as in v1
 * Mode byte m: 128 + w (0 <= w <= 64) fixed width w; k < 64 Rice with
 * parameter k (the chunk's v1 width is the bit length of its largest z);
 * 63 + w (1 <= w <= 64) sparse with width w.  A chunk of width 0 is fixed
 * width 0 (no bits). */

#define OR_EMAGIC 0x31454141u /* "AAE1" little-endian */
#define E_RUN 0x80000000u
#define E_VERBATIM 0x40000000u
#define M_FIXED 128
#define M_SPARSE 63 /* sparse width w: mode M_SPARSE + w, 64 .. 127 */

typedef struct {
    const uint8_t *p;
    size_t len;
} or_rec;

typedef struct {
    uint64_t *w;
    size_t nbits, cap; /* cap in words */
} bitw;

static int bw_put(bitw *b, int bit)
{
    if ((b->nbits >> 6) >= b->cap) {
        size_t nc = b->cap ? 2 * b->cap : 64;
        uint64_t *nw = (uint64_t *)realloc(b->w, nc * 8);
        if (!nw)
            return OR_ENOMEM;
        memset(nw + b->cap, 0, (nc - b->cap) * 8);
        b->w = nw;
        b->cap = nc;
    }
    if (bit)
        setbit(b->w, b->nbits);
    b->nbits++;
    return OR_OK;
}

static int bw_bits(bitw *b, uint64_t v, int n)
{
    for (int i = 0; i < n; i++)
        if (bw_put(b, (int)((v >> i) & 1)))
            return OR_ENOMEM;
    return OR_OK;
}

static size_t pad8z(size_t n) { return (n + 7) / 8 * 8; }

/* The plane records of a v1 stream in order (lengths from their fields). */
static int v1_records(const uint8_t *v1, size_t len, size_t nplanes, size_t nch, or_rec *rec)
{
    const uint8_t *p = v1 + HDR_BYTES + ((v1[5] & OR_HDR_SCALED) ? 8 : 0);
    const uint8_t *end = v1 + len;
    for (size_t k = 0; k < nplanes; k++) {
        if (p > end || (size_t)(end - p) < PLANE_HDR_BYTES)
            return OR_EINVAL;
        const uint32_t pw = rd_u32(p + 8), no = rd_u32(p + 12);
        const size_t r = PLANE_HDR_BYTES + (pw ? pad8z(nch) : 0) + 8 * (size_t)pw +
                         OUTLIER_BYTES * (size_t)no;
        if ((size_t)(end - p) < r)
            return OR_EINVAL;
        rec[k].p = p;
        rec[k].len = r;
        p += r;
    }
    return p == end ? OR_OK : OR_EINVAL;
}

/* Mode byte and coded bits of a chunk of width w holding z[0..63]. */
static int chunk_mode(const uint64_t *z, int w, uint64_t *bits)
{
    *bits = 0;
    if (w == 0)
        return M_FIXED;
    const uint64_t fixed = 64u * (uint64_t)w;
    uint64_t rice = UINT64_MAX, nnz = 0;
    int kbest = 0;
    for (int k = 0; k < w; k++) {
        /* terms saturate at 2^20: a saturated sum exceeds every fixed-width
         * cost (at most 64 * 64), so it never wins; sums that can win are
         * exact */
        uint64_t cost = 64u * (uint64_t)(k + 1);
        for (int l = 0; l < (int)CHUNK; l++) {
            const uint64_t q = z[l] >> k;
            cost += q > (1u << 20) ? (1u << 20) : q;
        }
        if (cost < rice) {
            rice = cost;
            kbest = k;
        }
    }
    for (int l = 0; l < (int)CHUNK; l++)
        nnz += z[l] != 0;
    const uint64_t sparse = 64u + nnz * (uint64_t)w;
    if (fixed <= rice && fixed <= sparse) {
        *bits = fixed;
        return M_FIXED + w;
    }
    if (rice <= sparse) {
        *bits = rice;
        return kbest;
    }
    *bits = sparse;
    return M_SPARSE + w;
}

/* Literal body of one v1 plane record. */
static int encode_literal(obuf *o, const uint8_t *rec, size_t nch)
{
    const uint32_t pw = rd_u32(rec + 8), nout = rd_u32(rec + 12);
    const uint8_t *wid = rec + PLANE_HDR_BYTES;
    const uint8_t *payload = wid + (pw ? pad8z(nch) : 0);
    if (ob_put(o, rec, PLANE_HDR_BYTES))
        return OR_ENOMEM;
    if (pw == 0)
        return ob_put(o, payload, OUTLIER_BYTES * (size_t)nout) ? OR_ENOMEM : OR_OK;
    uint8_t mode[CHUNK * 4];
    uint16_t lens[CHUNK * 4];
    size_t nlen = 0;
    bitw bw = {0};
    int rc = OR_OK;
    if (nch > sizeof mode)
        return OR_EINVAL;
    size_t woff = 0;
    for (size_t c = 0; c < nch && rc == OR_OK; c++) {
        const int w = wid[c];
        uint64_t words[64], z[CHUNK], bits;
        memcpy(words, payload + 8 * woff, 8 * (size_t)w);
        for (size_t l = 0; l < CHUNK; l++) {
            z[l] = 0;
            for (int bit = 0; bit < w; bit++)
                if (getbit(words, (uint64_t)l * (uint64_t)w + (uint64_t)bit))
                    z[l] |= (uint64_t)1 << bit;
        }
        const int m = chunk_mode(z, w, &bits);
        const size_t start = bw.nbits;
        mode[c] = (uint8_t)m;
        if (m >= M_FIXED) {
            for (size_t l = 0; l < CHUNK && rc == OR_OK; l++)
                rc = bw_bits(&bw, z[l], w);
        } else if (m > M_SPARSE) {
            uint64_t mask = 0;
            for (size_t l = 0; l < CHUNK; l++)
                if (z[l])
                    mask |= (uint64_t)1 << l;
            rc = bw_bits(&bw, mask, 64);
            for (size_t l = 0; l < CHUNK && rc == OR_OK; l++)
                if (z[l])
                    rc = bw_bits(&bw, z[l], w);
        } else {
            for (size_t l = 0; l < CHUNK && rc == OR_OK; l++) {
                for (uint64_t q = z[l] >> m; q > 0 && rc == OR_OK; q--)
                    rc = bw_put(&bw, 1);
                if (rc == OR_OK)
                    rc = bw_put(&bw, 0);
                if (rc == OR_OK)
                    rc = bw_bits(&bw, z[l], m);
            }
        }
        if (rc == OR_OK && bw.nbits - start != bits)
            rc = OR_EINVAL; /* cannot happen: the cost is the code's length */
        if (m < M_FIXED)
            lens[nlen++] = (uint16_t)bits;
        woff += (size_t)w;
    }
    const uint32_t cw = (uint32_t)((bw.nbits + 63) / 64);
    if (rc == OR_OK &&
        (ob_u32(o, cw) || ob_u32(o, 0) || ob_put(o, mode, nch) || ob_zero(o, pad8z(nch) - nch) ||
         (nlen && ob_put(o, lens, 2 * nlen)) || ob_zero(o, pad8z(2 * nlen) - 2 * nlen) ||
         (cw && ob_put(o, bw.w, 8 * (size_t)cw)) ||
         ob_put(o, payload + 8 * (size_t)pw, OUTLIER_BYTES * (size_t)nout)))
        rc = OR_ENOMEM;
    free(bw.w);
    return rc;
}

int or_entropy_encode(const uint8_t *v1, size_t len, uint8_t *out, size_t cap,
                      size_t *olen)
{
    if (!v1 || !olen || len < HDR_BYTES || rd_u32(v1) != OR_MAGIC || rd_u32(v1 + 12) != len)
        return OR_EINVAL;
    const int s = v1[6], b = v1[7];
    if (s < 6 || s > 14 || b < s || b > 40 || (v1[5] & ~OR_HDR_SCALED))
        return OR_EINVAL;
    const size_t nch = (size_t)1 << (s - 6);
    const size_t np = (size_t)2 << (b - s);
    const size_t scaled = (v1[5] & OR_HDR_SCALED) ? 8 : 0;
    or_rec *rec = (or_rec *)malloc(np * sizeof(or_rec));
    uint32_t *tags = (uint32_t *)malloc(np * 4);
    obuf body = {0}, o = {0};
    int rc = OR_ENOMEM;
    if (!rec || !tags)
        goto done;
    rc = v1_records(v1, len, np, nch, rec);
    if (rc)
        goto done;
    size_t ni = 0;
    int prev_rep = 0;
    for (size_t k = 0; k < np; k++) {
        const int rep = k >= 2 && rec[k].len == rec[k - 2].len &&
                        memcmp(rec[k].p, rec[k - 2].p, rec[k].len) == 0;
        if (rep && prev_rep) {
            tags[ni - 1]++; /* extends the run of the previous plane */
        } else if (rep) {
            tags[ni++] = E_RUN | 1u;
        } else {
            const size_t before = body.len;
            rc = encode_literal(&body, rec[k].p, nch);
            if (rc)
                goto done;
            if (body.len - before >= rec[k].len) {
                body.len = before;
                rc = ob_put(&body, rec[k].p, rec[k].len) ? OR_ENOMEM : OR_OK;
                if (rc)
                    goto done;
                tags[ni++] = E_VERBATIM | (uint32_t)rec[k].len;
            } else {
                tags[ni++] = (uint32_t)(body.len - before);
            }
        }
        prev_rep = rep;
    }
    rc = OR_ENOMEM;
    if (ob_put(&o, v1, HDR_BYTES) || ob_u32(&o, (uint32_t)len) || ob_u32(&o, (uint32_t)ni) ||
        (scaled && ob_put(&o, v1 + HDR_BYTES, 8)) || ob_put(&o, tags, 4 * ni) ||
        ob_zero(&o, pad8z(4 * ni) - 4 * ni) || (body.len && ob_put(&o, body.p, body.len)))
        goto done;
    {
        const uint32_t magic = OR_EMAGIC, total = (uint32_t)o.len;
        memcpy(o.p, &magic, 4);
        memcpy(o.p + 12, &total, 4);
    }
    *olen = o.len;
    rc = OR_OK;
    if (!out || cap < o.len)
        rc = OR_ENOMEM;
    else
        memcpy(out, o.p, o.len);
done:
    free(o.p);
    free(body.p);
    free(tags);
    free(rec);
    return rc;
}

/* n bits (n <= 64) at *pos of a bit stream of nbits bits; -1 past its end. */
static int br_get(const uint8_t *bytes, size_t nbits, size_t *pos, int n, uint64_t *v)
{
    if (*pos + (size_t)n > nbits)
        return -1;
    uint64_t r = 0;
    for (int i = 0; i < n; i++) {
        const size_t p = *pos + (size_t)i;
        if ((bytes[p >> 3] >> (p & 7)) & 1)
            r |= (uint64_t)1 << i;
    }
    *pos += (size_t)n;
    *v = r;
    return 0;
}

/* The 64 fields of one chunk coded in mode m in bits [*pos, end) of code;
 * its v1 width into *w.  0, or -1 when malformed. */
static int decode_chunk(const uint8_t *code, size_t end, size_t *pos, int m, uint64_t *z, int *w)
{
    if (m >= M_FIXED && m <= M_FIXED + 64) {
        *w = m - M_FIXED;
        for (size_t l = 0; l < CHUNK; l++)
            if (br_get(code, end, pos, *w, &z[l]))
                return -1;
        return 0;
    }
    if (m > M_SPARSE && m < M_FIXED) {
        uint64_t mask;
        *w = m - M_SPARSE;
        if (br_get(code, end, pos, 64, &mask))
            return -1;
        for (size_t l = 0; l < CHUNK; l++) {
            z[l] = 0;
            if ((mask >> l) & 1) {
                if (br_get(code, end, pos, *w, &z[l]) || z[l] == 0)
                    return -1;
            }
        }
        return 0;
    }
    if (m <= M_SPARSE) {
        uint64_t zmax = 0;
        for (size_t l = 0; l < CHUNK; l++) {
            uint64_t q = 0, bit = 1, low = 0;
            for (;;) {
                if (br_get(code, end, pos, 1, &bit))
                    return -1;
                if (!bit)
                    break;
                q++;
            }
            if (m > 0 && (q >> (64 - m)) != 0)
                return -1;
            if (br_get(code, end, pos, m, &low))
                return -1;
            z[l] = (q << m) | low;
            if (z[l] > zmax)
                zmax = z[l];
        }
        *w = bitlen64(zmax);
        return 0;
    }
    return -1;
}

/* One literal body (tag bytes at p) appended to o as a v1 plane record. */
static int decode_literal(obuf *o, const uint8_t *p, size_t tag, size_t nch)
{
    if (tag < PLANE_HDR_BYTES)
        return OR_EINVAL;
    const uint32_t pw = rd_u32(p + 8), nout = rd_u32(p + 12);
    if (pw == 0) {
        if (tag != PLANE_HDR_BYTES + OUTLIER_BYTES * (size_t)nout)
            return OR_EINVAL;
        return ob_put(o, p, tag) ? OR_ENOMEM : OR_OK;
    }
    if (tag < PLANE_HDR_BYTES + 8 + pad8z(nch))
        return OR_EINVAL;
    const uint32_t cw = rd_u32(p + 16);
    if (rd_u32(p + 20) != 0)
        return OR_EINVAL;
    const uint8_t *mode = p + PLANE_HDR_BYTES + 8;
    size_t nlen = 0;
    for (size_t c = 0; c < nch; c++)
        nlen += mode[c] < M_FIXED;
    for (size_t c = nch; c < pad8z(nch); c++)
        if (mode[c])
            return OR_EINVAL;
    const size_t need = PLANE_HDR_BYTES + 8 + pad8z(nch) + pad8z(2 * nlen) + 8 * (size_t)cw +
                        OUTLIER_BYTES * (size_t)nout;
    if (need != tag)
        return OR_EINVAL;
    const uint8_t *lens = mode + pad8z(nch);
    for (size_t i = 2 * nlen; i < pad8z(2 * nlen); i++)
        if (lens[i])
            return OR_EINVAL;
    const uint8_t *code = lens + pad8z(2 * nlen);
    const size_t nbits = 64 * (size_t)cw;
    uint64_t(*zz)[CHUNK] = (uint64_t(*)[CHUNK])malloc(nch * sizeof *zz);
    uint8_t wid[CHUNK * 4];
    if (!zz)
        return OR_ENOMEM;
    int rc = OR_EINVAL;
    size_t pos = 0, li = 0;
    uint32_t sum = 0;
    for (size_t c = 0; c < nch; c++) {
        const int m = mode[c];
        size_t end = nbits;
        if (m < M_FIXED) {
            /* a coded length given for the chunk must be what it decodes to */
            end = pos + (size_t)(lens[2 * li] | (lens[2 * li + 1] << 8));
            if (end > nbits)
                goto done;
        }
        int w = 0;
        if (decode_chunk(code, end, &pos, m, zz[c], &w))
            goto done;
        if (m < M_FIXED && pos != end)
            goto done;
        li += m < M_FIXED;
        wid[c] = (uint8_t)w;
        sum += (uint32_t)w;
    }
    /* the codes end in the last word; its padding bits are zero */
    if ((pos + 63) / 64 != cw || sum != pw)
        goto done;
    for (size_t q = pos; q < nbits; q++)
        if ((code[q >> 3] >> (q & 7)) & 1)
            goto done;
    rc = OR_ENOMEM;
    if (ob_put(o, p, PLANE_HDR_BYTES) || ob_put(o, wid, nch) || ob_zero(o, pad8z(nch) - nch))
        goto done;
    for (size_t c = 0; c < nch; c++) {
        const int w = wid[c];
        uint64_t words[64];
        memset(words, 0, sizeof words);
        for (size_t l = 0; l < CHUNK; l++)
            for (int bit = 0; bit < w; bit++)
                if ((zz[c][l] >> bit) & 1)
                    setbit(words, (uint64_t)l * (uint64_t)w + (uint64_t)bit);
        if (ob_put(o, words, 8 * (size_t)w))
            goto done;
    }
    if (ob_put(o, code + 8 * (size_t)cw, OUTLIER_BYTES * (size_t)nout))
        goto done;
    rc = OR_OK;
done:
    free(zz);
    return rc;
}

int or_entropy_decode(const uint8_t *e, size_t len, uint8_t *out, size_t cap, size_t *olen)
{
    if (!e || !olen || len < HDR_BYTES + 8 || rd_u32(e) != OR_EMAGIC ||
        rd_u32(e + 12) != len || len % 8)
        return OR_EINVAL;
    const int s = e[6], b = e[7];
    if (s < 6 || s > 14 || b < s || b > 40 || (e[5] & ~OR_HDR_SCALED))
        return OR_EINVAL;
    const uint32_t v1len = rd_u32(e + HDR_BYTES), ni = rd_u32(e + HDR_BYTES + 4);
    const size_t scaled = (e[5] & OR_HDR_SCALED) ? 8 : 0;
    const size_t nch = (size_t)1 << (s - 6);
    const size_t np = (size_t)2 << (b - s);
    /* every v1 plane record takes at least 16 bytes */
    if ((uint64_t)v1len < HDR_BYTES + scaled + (uint64_t)PLANE_HDR_BYTES * np || v1len % 8 ||
        ni == 0 || ni > np)
        return OR_EINVAL;
    *olen = v1len;
    const size_t tpos = HDR_BYTES + 8 + scaled;
    if (len < tpos + pad8z(4 * (size_t)ni))
        return OR_EINVAL;
    const uint8_t *tags = e + tpos;
    for (size_t i = 4 * (size_t)ni; i < pad8z(4 * (size_t)ni); i++)
        if (tags[i])
            return OR_EINVAL;
    size_t bpos = tpos + pad8z(4 * (size_t)ni);
    size_t *roff = (size_t *)malloc(np * sizeof(size_t));
    size_t *rlen = (size_t *)malloc(np * sizeof(size_t));
    obuf o = {0};
    int rc = OR_ENOMEM;
    if (!roff || !rlen)
        goto done;
    if (ob_put(&o, e, HDR_BYTES) || (scaled && ob_put(&o, e + HDR_BYTES + 8, 8)))
        goto done;
    size_t k = 0;
    for (uint32_t i = 0; i < ni; i++) {
        const uint32_t t = rd_u32(tags + 4 * (size_t)i);
        rc = OR_EINVAL;
        if (t & E_RUN) {
            const uint32_t R = t & ~E_RUN;
            if (R == 0 || k < 2 || R > np - k)
                goto done;
            for (uint32_t r = 0; r < R; r++, k++) {
                roff[k] = o.len;
                rlen[k] = rlen[k - 2];
                rc = OR_ENOMEM;
                if (ob_zero(&o, rlen[k]))
                    goto done;
                memcpy(o.p + roff[k], o.p + roff[k - 2], rlen[k]);
            }
        } else {
            const size_t tb = t & ~E_VERBATIM;
            if (k >= np || tb % 8 || tb > len - bpos)
                goto done;
            roff[k] = o.len;
            if (t & E_VERBATIM) {
                /* a v1 record, its length from its own fields */
                rc = OR_EINVAL;
                if (tb < PLANE_HDR_BYTES)
                    goto done;
                const uint32_t pw = rd_u32(e + bpos + 8), no = rd_u32(e + bpos + 12);
                if (tb != PLANE_HDR_BYTES + (pw ? pad8z(nch) : 0) + 8 * (size_t)pw +
                              OUTLIER_BYTES * (size_t)no)
                    goto done;
                rc = ob_put(&o, e + bpos, tb) ? OR_ENOMEM : OR_OK;
            } else {
                rc = decode_literal(&o, e + bpos, tb, nch);
            }
            if (rc)
                goto done;
            rlen[k] = o.len - roff[k];
            bpos += tb;
            k++;
        }
    }
    rc = OR_EINVAL;
    if (k != np || bpos != len || o.len != v1len)
        goto done;
    {
        const uint32_t magic = OR_MAGIC;
        memcpy(o.p, &magic, 4);
        memcpy(o.p + 12, &v1len, 4);
    }
    rc = OR_OK;
    if (!out || cap < o.len)
        rc = OR_ENOMEM;
    else
        memcpy(out, o.p, o.len);
done:
    free(o.p);
    free(rlen);
    free(roff);
    return rc;
}
