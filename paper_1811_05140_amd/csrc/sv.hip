// sv.hip -- the uncompressed FP64 state-vector path: the "no compression"
// comparator of the paper's runtime and fidelity figures.  One complex128
// array of 2^n amplitudes in HBM; each gate streams it once (32 bytes per
// amplitude per gate), with the same gate arithmetic as the compressed path.
#pragma clang fp contract(off)

#include "device.h"
#include "gates.h"

namespace aalc {

namespace {

constexpr int kSvWG = 256;

unsigned sv_grid(uint64_t items)
{
    const uint64_t per = (items + kSvWG - 1) / kSvWG;
    const uint64_t cap = 1ull << 16;
    return (unsigned)(per < cap ? (per ? per : 1) : cap);
}

__global__ __launch_bounds__(kSvWG) void k_sv_basis(double *amp, uint64_t N, uint64_t x)
{
    for (uint64_t i = blockIdx.x * (uint64_t)kSvWG + threadIdx.x; i < N;
         i += (uint64_t)gridDim.x * kSvWG) {
        amp[2 * i] = (i == x) ? 1.0 : 0.0;
        amp[2 * i + 1] = 0.0;
    }
}

// Pairs (i, i ^ mask) with the top bit of mask clear in i.
__global__ __launch_bounds__(kSvWG) void k_sv_pair(double *amp, GateArg G,
                                                   uint64_t npairs)
{
    const int hb = 63 - __builtin_clzll(G.mask);
    const uint64_t lo = (1ull << hb) - 1;
    for (uint64_t p = blockIdx.x * (uint64_t)kSvWG + threadIdx.x; p < npairs;
         p += (uint64_t)gridDim.x * kSvWG) {
        const uint64_t i = ((p >> hb) << (hb + 1)) | (p & lo);
        const uint64_t j = i ^ G.mask;
        double2 a = *(const double2 *)(amp + 2 * i);
        double2 b = *(const double2 *)(amp + 2 * j);
        double ar = a.x, ai = a.y, br = b.x, bi = b.y;
        gate_pair(G, i, ar, ai, br, bi);
        *(double2 *)(amp + 2 * i) = make_double2(ar, ai);
        *(double2 *)(amp + 2 * j) = make_double2(br, bi);
    }
}

__global__ __launch_bounds__(kSvWG) void k_sv_diag(double *amp, GateArg G, uint64_t N,
                                                   const double *tdiff)
{
    for (uint64_t i = blockIdx.x * (uint64_t)kSvWG + threadIdx.x; i < N;
         i += (uint64_t)gridDim.x * kSvWG) {
        double2 a = *(const double2 *)(amp + 2 * i);
        double ar = a.x, ai = a.y;
        gate_diag(G, i, ar, ai, tdiff);
        *(double2 *)(amp + 2 * i) = make_double2(ar, ai);
    }
}

// Pairwise sum of 2^k leaves by one workgroup (perfect tree).
template <class Load>
__device__ double tree_wg(Load load, uint64_t m, double *lds)
{
    const int t = threadIdx.x;
    uint64_t nact;
    if (m >= kSvWG) {
        const uint64_t per = m / kSvWG;
        double stack[40];
        int sp = 0;
        for (uint64_t i = 0; i < per; ++i) {
            double v = load(t * per + i);
            for (uint64_t k = i; k & 1; k >>= 1)
                v = stack[--sp] + v;
            stack[sp++] = v;
        }
        lds[t] = stack[0];
        nact = kSvWG;
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

// part[c][r] = pairwise over range r (2^k amplitudes) of component c
// (c = 0, 1: re, im; c = 2: |a|^2).
__global__ __launch_bounds__(kSvWG) void k_sv_partial(const double *amp, uint64_t per,
                                                      uint64_t nr, int mode, double *part)
{
    __shared__ double lds[kSvWG];
    for (uint64_t r = blockIdx.x; r < nr; r += gridDim.x) {
        const double *p = amp + 2 * r * per;
        if (mode == 0) {
            for (int c = 0; c < 2; ++c) {
                const double v = tree_wg([&](uint64_t i) { return p[2 * i + c]; }, per, lds);
                if (threadIdx.x == 0)
                    part[(uint64_t)c * nr + r] = v;
            }
        } else {
            const double v = tree_wg(
                [&](uint64_t i) {
                    const double re = p[2 * i], im = p[2 * i + 1];
                    const double rr = re * re;
                    const double ii = im * im;
                    return rr + ii;
                },
                per, lds);
            if (threadIdx.x == 0)
                part[r] = v;
        }
    }
}

__global__ __launch_bounds__(kSvWG) void k_sv_final(const double *part, uint64_t nr,
                                                    int ncomp, double mul, double *out)
{
    __shared__ double lds[kSvWG];
    for (int c = 0; c < ncomp; ++c) {
        const double *p = part + (uint64_t)c * nr;
        const double v = tree_wg([&](uint64_t i) { return p[i]; }, nr, lds);
        if (threadIdx.x == 0)
            out[c] = v * mul;
    }
}

__global__ __launch_bounds__(kSvWG) void k_sv_probs(const double *amp, uint64_t N,
                                                    const int *qubits, int nq,
                                                    double *probs)
{
    __shared__ double bins[1024];
    const bool lds_bins = nq <= 10;
    const uint32_t nb = 1u << nq;
    if (lds_bins)
        for (uint32_t k = threadIdx.x; k < nb; k += kSvWG)
            bins[k] = 0.0;
    __syncthreads();
    for (uint64_t i = blockIdx.x * (uint64_t)kSvWG + threadIdx.x; i < N;
         i += (uint64_t)gridDim.x * kSvWG) {
        uint32_t oc = 0;
        for (int k = 0; k < nq; ++k)
            oc |= (uint32_t)bit_of(i, qubits[k]) << k;
        const double re = amp[2 * i], im = amp[2 * i + 1];
        const double rr = re * re;
        const double ii = im * im;
        const double pv = rr + ii;
        if (lds_bins)
            atomicAdd(&bins[oc], pv);
        else
            atomicAdd(&probs[oc], pv);
    }
    __syncthreads();
    if (lds_bins)
        for (uint32_t k = threadIdx.x; k < nb; k += kSvWG)
            if (bins[k] != 0.0)
                atomicAdd(&probs[k], bins[k]);
}

}  // namespace

void sv_set_basis(double *amp, int n, uint64_t x, hipStream_t st)
{
    const uint64_t N = 1ull << n;
    hipLaunchKernelGGL(k_sv_basis, dim3(sv_grid(N)), dim3(kSvWG), 0, st, amp, N, x);
}

// Range split for the pairwise reductions: ranges of 2^min(n, 16) leaves.
static void ranges_of(int n, uint64_t &per, uint64_t &nr)
{
    const int k = n < 16 ? n : 16;
    per = 1ull << k;
    nr = 1ull << (n - k);
}

#define TIMED(prof, id, st, launch)                                              \
    do {                                                                         \
        if (prof)                                                                \
            (prof)->begin((id), (st));                                           \
        launch;                                                                  \
        if (prof)                                                                \
            (prof)->end((id), (st));                                             \
    } while (0)

void sv_apply(double *amp, int n, const GateArg &g, double *scratch, double *tdiff_dev,
              hipStream_t st, Prof *prof)
{
    const uint64_t N = 1ull << n;
    if (g.kind == kDiffuse) {
        uint64_t per, nr;
        ranges_of(n, per, nr);
        TIMED(prof, kIdSvPartial, st,
              hipLaunchKernelGGL(k_sv_partial, dim3(sv_grid(nr * kSvWG)), dim3(kSvWG), 0, st,
                                 (const double *)amp, per, nr, 0, scratch));
        TIMED(prof, kIdSvFinal, st,
              hipLaunchKernelGGL(k_sv_final, dim3(1), dim3(kSvWG), 0, st,
                                 (const double *)scratch, nr, 2, ldexp(1.0, 1 - n),
                                 tdiff_dev));
    }
    if (g.mask) {
        TIMED(prof, kIdSvPair, st,
              hipLaunchKernelGGL(k_sv_pair, dim3(sv_grid(N / 2)), dim3(kSvWG), 0, st, amp, g,
                                 N / 2));
    } else {
        TIMED(prof, kIdSvDiag, st,
              hipLaunchKernelGGL(k_sv_diag, dim3(sv_grid(N)), dim3(kSvWG), 0, st, amp, g, N,
                                 (const double *)tdiff_dev));
    }
}

void sv_probs(const double *amp, int n, const int *qubits_dev, int nq, double *probs_dev,
              hipStream_t st)
{
    const uint64_t N = 1ull << n;
    hipLaunchKernelGGL(k_sv_probs, dim3(sv_grid(N)), dim3(kSvWG), 0, st, amp, N,
                       qubits_dev, nq, probs_dev);
}

void sv_normsq(const double *amp, int n, double *scratch, double *out_dev, hipStream_t st)
{
    uint64_t per, nr;
    ranges_of(n, per, nr);
    hipLaunchKernelGGL(k_sv_partial, dim3(sv_grid(nr * kSvWG)), dim3(kSvWG), 0, st, amp, per,
                       nr, 1, scratch);
    hipLaunchKernelGGL(k_sv_final, dim3(1), dim3(kSvWG), 0, st, (const double *)scratch, nr,
                       1, 1.0, out_dev);
}

// out[0..1] = pairwise sums of the re and im parts over all amplitudes.
void sv_sum(const double *amp, int n, double *scratch, double *out_dev, hipStream_t st)
{
    uint64_t per, nr;
    ranges_of(n, per, nr);
    hipLaunchKernelGGL(k_sv_partial, dim3(sv_grid(nr * kSvWG)), dim3(kSvWG), 0, st, amp, per,
                       nr, 0, scratch);
    hipLaunchKernelGGL(k_sv_final, dim3(1), dim3(kSvWG), 0, st, (const double *)scratch, nr,
                       2, 1.0, out_dev);
}

}  // namespace aalc
