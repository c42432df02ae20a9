// gates.h -- gate arithmetic shared by the compressed and uncompressed
// kernels: the pair update of a single-qubit gate and the controlled form
// (Sec. II of the paper), diagonal phases, swaps and the Grover operators.
// One IEEE binary64 rounding per multiply and add, no contraction.
#pragma once
#pragma clang fp contract(off)

#include "device.h"

namespace aalc {

// complex product u*a, one rounding per operation
__device__ __forceinline__ void cmul(double ur, double ui, double ar, double ai,
                                     double &o_r, double &o_i)
{
    double rr = ur * ar;
    double ii = ui * ai;
    double ri = ur * ai;
    double ir = ui * ar;
    o_r = rr - ii;
    o_i = ri + ir;
}

__device__ __forceinline__ int bit_of(uint64_t i, int q) { return (int)((i >> q) & 1u); }

// Pair update (Sec. II): a = amplitude i (target bit clear), b = i ^ mask.
__device__ __forceinline__ void gate_pair(const GateArg &G, uint64_t i,
                                          double &ar, double &ai, double &br,
                                          double &bi)
{
    switch (G.kind) {
    case kCU:
        if (!bit_of(i, G.q0))
            return;
        [[fallthrough]];
    case kU: {
        double pr, pi, qr, qi, rr, ri, tr, ti;
        cmul(G.u[0], G.u[1], ar, ai, pr, pi);
        cmul(G.u[2], G.u[3], br, bi, qr, qi);
        cmul(G.u[4], G.u[5], ar, ai, rr, ri);
        cmul(G.u[6], G.u[7], br, bi, tr, ti);
        ar = pr + qr;
        ai = pi + qi;
        br = rr + tr;
        bi = ri + ti;
        return;
    }
    case kSwap:
        if (bit_of(i, G.q0) == bit_of(i, G.q1))
            return;
        [[fallthrough]];
    case kX: {
        double t0 = ar, t1 = ai;
        ar = br;
        ai = bi;
        br = t0;
        bi = t1;
        return;
    }
    default:
        return;
    }
}

__device__ __forceinline__ void gate_diag(const GateArg &G, uint64_t i,
                                          double &ar, double &ai,
                                          const double *tdiff)
{
    switch (G.kind) {
    case kDiag1:
        if (bit_of(i, G.q0)) {
            double r, m;
            cmul(G.u[6], G.u[7], ar, ai, r, m);
            ar = r;
            ai = m;
        }
        return;
    case kCPhase:
        if (bit_of(i, G.q0) && bit_of(i, G.q1)) {
            double r, m;
            cmul(G.u[6], G.u[7], ar, ai, r, m);
            ar = r;
            ai = m;
        }
        return;
    case kCZ:
        if (bit_of(i, G.q0) && bit_of(i, G.q1)) {
            ar = -ar;
            ai = -ai;
        }
        return;
    case kPhaseFlip:
        if (i == G.index) {
            ar = -ar;
            ai = -ai;
        }
        return;
    case kDiffuse:
        ar = tdiff[0] - ar;
        ai = tdiff[1] - ai;
        return;
    default:
        return;
    }
}

}  // namespace aalc
