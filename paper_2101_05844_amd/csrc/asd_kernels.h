// Kernels of the Active Set dual iteration (gfx950).
//
// One iteration of Algorithm 1 (Sec. 4) is split into two passes over the
// layers:
//   backward pass (per neuron layer k = 0..n-1): the primal coefficients f_k of
//     eq:dual-active-set, which need W_{k+1}^T and the masked (W_{k+1} . I)^T
//     products, then the closed-form inner minimisation eq:as-primalk-min /
//     eq:as-primal0-min (x*_k, z*_k), and optionally the objective terms;
//   forward pass (per ReLU layer k = 1..n-1): W_k x*_{k-1} and the masked
//     (W_k . I) x*_{k-1} products, the supergradient eq:as-supergradient, the
//     projected Adam step, and the derived per-neuron sums the next backward
//     pass reads.
// Active-set extension (the separation oracle eq:oracle) runs between the two
// passes at addition iterations.
//
// Compact masks.  In Active Set the inner minimiser is integral: z*_k in
// {0,1} and every x*_{k-1}[j] is an end of its box.  Evaluating eq:oracle there
// gives, for neuron i: an all-ones row when z*_k[i] = 1; when z*_k[i] = 0,
// I[i,j] = 1 exactly where W[i,j] = 0, the box of j is a single point, or
// x*_{k-1}[j] sits at the end that minimises W[i,j] x (l for W > 0, u for
// W < 0).  A mask is therefore stored as the z*_k bits of layer k and the
// "x*_{k-1} = u" bits of layer k-1 at the time it was added, and
// (W . I) products split by weight sign:
//   (W . I) x [i]      = z_I[i] ? (W x)[i] : (W+ (eL . x) + W- (eH . x))[i]
//   (W . I)^T beta [j] = (W^T (z_I . beta))[j] + eL[j] (W+^T u)[j] + eH[j] (W-^T u)[j]
// with u = (1 - z_I) . beta, eL = "x_I = l" and eH = "x_I = u" (both set for a
// point box).  The general oracle for fractional z (asd_oracle) evaluates
// eq:oracle entry by entry.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>

#include <type_traits>

#include "asd_internal.h"

namespace asd {

constexpr int CB = 4;   // channels per thread (register blocking)
constexpr int KS = 4;   // waves splitting a reduction (one channel each in the epilogue)

__device__ __forceinline__ unsigned getbit(const uint32_t* bits, long bi) {
    return (bits[bi >> 5] >> (bi & 31)) & 1u;
}

// Writes the 64 predicate bits of one wavefront covering bit indices
// [base, base + 64) with base a multiple of 64.
__device__ __forceinline__ void put_wave_bits(uint32_t* bits, long base, bool pred, int lane) {
    unsigned long long m = __ballot(pred);
    if (lane == 0) {
        bits[(base >> 5)] = (uint32_t)(m & 0xffffffffull);
        bits[(base >> 5) + 1] = (uint32_t)(m >> 32);
    }
}

template <typename T> __device__ __forceinline__ T tmax0(T a) { return a > (T)0 ? a : (T)0; }
template <typename T> __device__ __forceinline__ T tmin0(T a) { return a < (T)0 ? a : (T)0; }
__device__ __forceinline__ float tsqrt(float a) { return sqrtf(a); }
__device__ __forceinline__ double tsqrt(double a) { return sqrt(a); }

// ---------------------------------------------------------------------------
// Tap enumeration of layer L's receptive field for output column (s, p).
// ---------------------------------------------------------------------------
struct FwdTap {
    long a;     // input neuron address in the internal layout, or -1 (padding)
    long bi;    // input bit index
};

// The taps t0, t0 + 1, ... of output column (s, p) in the order of
// fwd_tap, without a division per tap: (channel, kernel row, kernel column)
// of a convolution, (channel, position) of a dense layer's input, advanced
// one tap at a time.
struct TapWalk {
    int ci, ky, kx;  // dense: channel ci, input position ky
    int iy0, ix0;    // convolution: first input row and column of the field
};

__device__ __forceinline__ TapWalk tap_walk(const LayerGeo& g, int p, int t) {
    TapWalk w;
    if (g.kind == ASD_LAYER_DENSE) {
        w.ci = t / g.in.P;
        w.ky = t - w.ci * g.in.P;
        w.kx = 0;
        w.iy0 = w.ix0 = 0;
    } else {
        const int k2 = g.ksz * g.ksz;
        w.ci = t / k2;
        const int rem = t - w.ci * k2;
        w.ky = rem / g.ksz;
        w.kx = rem - w.ky * g.ksz;
        const int oy = p / g.out.W, ox = p - oy * g.out.W;
        w.iy0 = oy * g.stride - g.pad;
        w.ix0 = ox * g.stride - g.pad;
    }
    return w;
}

__device__ __forceinline__ FwdTap tap_at(const LayerGeo& g, int S, int s, const TapWalk& w) {
    FwdTap r;
    if (g.kind == ASD_LAYER_DENSE) {
        r.a = ((long)w.ci * S + s) * g.in.P + w.ky;
        r.bi = (long)w.ci * g.in.colpad + (long)s * g.in.P + w.ky;
    } else {
        const int iy = w.iy0 + w.ky, ix = w.ix0 + w.kx;
        if (iy < 0 || iy >= g.in.H || ix < 0 || ix >= g.in.W) {
            r.a = -1;
            r.bi = 0;
        } else {
            const int pin = iy * g.in.W + ix;
            r.a = ((long)w.ci * S + s) * g.in.P + pin;
            r.bi = (long)w.ci * g.in.colpad + (long)s * g.in.P + pin;
        }
    }
    return r;
}

__device__ __forceinline__ void tap_next(const LayerGeo& g, TapWalk& w) {
    if (g.kind == ASD_LAYER_DENSE) {
        if (++w.ky == g.in.P) {
            w.ky = 0;
            ++w.ci;
        }
    } else if (++w.kx == g.ksz) {
        w.kx = 0;
        if (++w.ky == g.ksz) {
            w.ky = 0;
            ++w.ci;
        }
    }
}

__device__ __forceinline__ FwdTap fwd_tap(const LayerGeo& g, int S, int s, int p, int t) {
    FwdTap r;
    if (g.kind == ASD_LAYER_DENSE) {
        const int Pin = g.in.P;
        const int cj = t / Pin, pj = t - cj * Pin;
        r.a = ((long)cj * S + s) * Pin + pj;
        r.bi = (long)cj * g.in.colpad + (long)s * Pin + pj;
    } else {
        const int k2 = g.ksz * g.ksz;
        const int ci = t / k2;
        const int rem = t - ci * k2;
        const int ky = rem / g.ksz, kx = rem - ky * g.ksz;
        const int oy = p / g.out.W, ox = p - oy * g.out.W;
        const int iy = oy * g.stride - g.pad + ky, ix = ox * g.stride - g.pad + kx;
        if (iy < 0 || iy >= g.in.H || ix < 0 || ix >= g.in.W) {
            r.a = -1;
            r.bi = 0;
        } else {
            const int pin = iy * g.in.W + ix;
            r.a = ((long)ci * S + s) * g.in.P + pin;
            r.bi = (long)ci * g.in.colpad + (long)s * g.in.P + pin;
        }
    }
    return r;
}

// ---------------------------------------------------------------------------
// Forward pass: products, supergradient, update (or export) for ReLU layer k.
// ---------------------------------------------------------------------------
template <typename T>
struct FwdArgs {
    LayerGeo g;                 // layer k
    int S;
    int nm;                     // active masks
    const T* xin;               // x*_{k-1}
    const uint32_t* deg_in;     // point boxes of layer k-1
    const T* xout;              // x*_k
    const uint32_t* zbits;      // z*_k
    ReluLayerT<T> R;            // layer k arrays
    StepArgsT<T> st;
    int mode;                   // 0 update, 1 export supergradient
    int freeze;                 // the slots' multipliers stay 0 (layer 1 of an l2-ball input domain)
    T* gout[3 + kMaxMasks];     // export targets, caller layout [S][n_k]
};

template <typename T>
__global__ void __launch_bounds__(kWave * KS) k_forward(FwdArgs<T> A) {
    extern __shared__ unsigned char red_raw[];
    T* red = reinterpret_cast<T*>(red_raw);  // [KS][CB][1 + nm][64]
    const LayerGeo& g = A.g;
    const int lane = threadIdx.x, wave = __builtin_amdgcn_readfirstlane(threadIdx.y);  // wave-uniform
    const long col = (long)blockIdx.x * kWave + lane;
    const int c0 = blockIdx.y * CB;
    const int S = A.S, nm = A.nm;
    const bool colok = col < g.out.cols;
    const int s = colok ? (int)(col / g.out.P) : 0;
    const int p = colok ? (int)(col - (long)s * g.out.P) : 0;

    T acc[CB];
    T accm[kMaxMasks][CB];
#pragma unroll
    for (int e = 0; e < CB; ++e) {
        acc[e] = 0;
#pragma unroll
        for (int q = 0; q < kMaxMasks; ++q) accm[q][e] = 0;
    }
    const int F = g.fan;
    const int t0 = (int)((long)F * wave / KS), t1 = (int)((long)F * (wave + 1) / KS);
    if (colok) {
        TapWalk tw = tap_walk(g, p, t0);
        for (int t = t0; t < t1; ++t, tap_next(g, tw)) {
            const FwdTap tp = tap_at(g, S, s, tw);
            const bool ok = tp.a >= 0;
            const T x = ok ? A.xin[tp.a] : (T)0;
            const unsigned dg = ok ? getbit(A.deg_in, tp.bi) : 0u;
            T w[CB];
#pragma unroll
            for (int e = 0; e < CB; ++e) {
                const int c = c0 + e;
                w[e] = c < g.out.C ? (T)g.W[(long)c * F + t] : (T)0;
                acc[e] += w[e] * x;
            }
#pragma unroll
            for (int q = 0; q < kMaxMasks; ++q) {
                if (q < nm) {
                    const unsigned xb = ok ? getbit(A.R.slot[q].xbits, tp.bi) : 0u;
                    const T aL = (!xb || dg) ? x : (T)0;
                    const T aH = (xb || dg) ? x : (T)0;
#pragma unroll
                    for (int e = 0; e < CB; ++e) accm[q][e] += tmax0(w[e]) * aL + tmin0(w[e]) * aH;
                }
            }
        }
    }
    const int ncomp = 1 + nm;
#pragma unroll
    for (int e = 0; e < CB; ++e) {
        red[((wave * CB + e) * ncomp + 0) * kWave + lane] = acc[e];
#pragma unroll
        for (int q = 0; q < kMaxMasks; ++q)
            if (q < nm) red[((wave * CB + e) * ncomp + 1 + q) * kWave + lane] = accm[q][e];
    }
    __syncthreads();
    // epilogue: wave e handles channel c0 + e (CB == KS)
    const int e = wave;
    const int c = c0 + e;
    if (!colok || c >= g.out.C) return;
    T yd = 0;
    T ym[kMaxMasks];
    for (int w = 0; w < KS; ++w) yd += red[((w * CB + e) * ncomp + 0) * kWave + lane];
#pragma unroll
    for (int q = 0; q < kMaxMasks; ++q) {
        ym[q] = 0;
        if (q < nm)
            for (int w = 0; w < KS; ++w) ym[q] += red[((w * CB + e) * ncomp + 1 + q) * kWave + lane];
    }
    const long idx = ((long)c * S + s) * g.out.P + p;
    const long bi = (long)c * g.out.colpad + col;
    const T bb = (T)g.b[c];
    const T xhat = yd + bb;
    const T x = A.xout[idx];
    const T z = (T)getbit(A.zbits, bi);
    const T lh = A.R.lhat[idx], uh = A.R.uhat[idx];
    const T ga = xhat - x;
    const T gb0 = x - z * uh;
    const T gb1 = x - xhat + ((T)1 - z) * lh;
    T gm[kMaxMasks];
    T zq[kMaxMasks];
#pragma unroll
    for (int q = 0; q < kMaxMasks; ++q) {
        gm[q] = 0;
        zq[q] = 0;
        if (q < nm) {
            const MaskSlotT<T>& M = A.R.slot[q];
            zq[q] = (T)getbit(M.zbits, bi);
            const T mq = zq[q] != (T)0 ? yd : ym[q];
            gm[q] = x - mq + M.LI[idx] * ((T)1 - z) - z * bb - M.UI[idx] * z;
        }
    }
    if (A.mode == 1) {
        const long ex = (long)s * g.out.N + (long)c * g.out.P + p;
        if (A.gout[0]) A.gout[0][ex] = ga;
        if (A.gout[1]) A.gout[1][ex] = gb0;
        if (A.gout[2]) A.gout[2][ex] = gb1;
#pragma unroll
        for (int q = 0; q < kMaxMasks; ++q)
            if (q < nm && A.gout[3 + q]) A.gout[3 + q][ex] = gm[q];
        return;
    }
    const StepArgsT<T>& st = A.st;
    const T lr_s = st.lrs ? st.lrs[s] : st.lr;
    auto step = [&](T th, T* m, T* v, T gr, int grp) -> T {
        if (st.rule == ASD_RULE_SUPERGRADIENT) return tmax0(th + lr_s * gr);
        const T mm = st.b1 * m[idx] + ((T)1 - st.b1) * gr;
        const T vv = st.b2 * v[idx] + ((T)1 - st.b2) * gr * gr;
        m[idx] = mm;
        v[idx] = vv;
        const T mh = mm / st.bc1[grp];
        const T vh = vv / st.bc2[grp];
        return tmax0(th + lr_s * mh / (tsqrt(vh) + st.eps));
    };
    const T al = step(A.R.alpha[idx], A.R.alpha_m, A.R.alpha_v, ga, 0);
    const T b0 = step(A.R.beta0[idx], A.R.beta0_m, A.R.beta0_v, gb0, 0);
    const T b1 = step(A.R.beta1[idx], A.R.beta1_m, A.R.beta1_v, gb1, 0);
    A.R.alpha[idx] = al;
    A.R.beta0[idx] = b0;
    A.R.beta1[idx] = b1;
    T own = al - b0 - b1;
    T gg = b0 * uh + b1 * lh;
    T vs = -al + b1;
#pragma unroll
    for (int q = 0; q < kMaxMasks; ++q) {
        if (q < nm) {
            const MaskSlotT<T>& M = A.R.slot[q];
            const T bq = A.freeze ? (T)0 : step(M.beta[idx], M.m, M.v, gm[q], 1 + q);
            M.beta[idx] = bq;
            own -= bq;
            gg += bq * (M.LI[idx] + M.UI[idx] + bb);
            vs += zq[q] != (T)0 ? bq : (T)0.5 * bq;
            M.u[idx] = zq[q] != (T)0 ? (T)0 : bq;
        }
    }
    A.R.own[idx] = own;
    A.R.g[idx] = gg;
    A.R.vs[idx] = vs;
}

// ---------------------------------------------------------------------------
// Backward pass: f_k, the inner minimisation, objective terms.
// Tc = compute type, Ts = state type, the same type: the iterations and the
// final bound of an FP64 plan.  (The FP64 final bound of an FP32 plan has
// kernels of its own, in sign classes.)
// ---------------------------------------------------------------------------
template <typename Ts>
struct BwdArgs {
    LayerGeo gn;                // layer k+1 (its input layout is layer k)
    int S;
    int k;                      // neuron layer (0 = input)
    int last;                   // k + 1 == n: backward operand is -c
    int nm_next;                // active masks of layer k+1 (0 if last)
    int nm_own;                 // active masks of layer k (k >= 1)
    const Ts* cvec;             // objective rows, layout of layer n
    ReluLayerT<Ts> Rn;          // layer k+1 arrays (if not last)
    ReluLayerT<Ts> Rk;          // layer k arrays (if k >= 1)
    NeuronArraysT<Ts> nk;       // layer k box, outputs
    const float* bk;            // bias of layer k (k >= 1), per channel
    int want_obj;
    double* fout;               // if set: f_k per neuron (internal layout)
    Ts* fext;                   // if set: f_k per neuron (caller layout [S][n_k])
};

template <typename Tc, typename Ts>
__device__ __forceinline__ Tc bwd_operand(const BwdArgs<Ts>& A, long a, long bi, Tc* uq) {
    // dense operand v and masked operands u_q at output neuron address a of
    // layer k+1, formed from the duals and the slots' z bits
    if (A.last) return -(Tc)A.cvec[a];
    Tc v = -(Tc)A.Rn.alpha[a] + (Tc)A.Rn.beta1[a];
#pragma unroll
    for (int q = 0; q < kMaxMasks; ++q) {
        if (q < A.nm_next) {
            const Tc bq = (Tc)A.Rn.slot[q].beta[a];
            const unsigned zb = getbit(A.Rn.slot[q].zbits, bi);
            if (zb) {
                v += bq;
                uq[q] = 0;
            } else {
                uq[q] = bq;
            }
        }
    }
    return v;
}

template <typename Tc, typename Ts>
__global__ void __launch_bounds__(kWave * KS) k_backward(BwdArgs<Ts> A) {
    extern __shared__ unsigned char red_raw[];
    Tc* red = reinterpret_cast<Tc*>(red_raw);  // [KS][CB][64]
    static_assert(sizeof(Tc) == sizeof(Ts), "one type for sums and state");
    const LayerGeo& g = A.gn;
    const NeuronLayout& L = g.in;   // layer k
    const NeuronLayout& O = g.out;  // layer k+1
    const int lane = threadIdx.x, wave = __builtin_amdgcn_readfirstlane(threadIdx.y);  // wave-uniform
    const long col = (long)blockIdx.x * kWave + lane;
    const int c0 = blockIdx.y * CB;
    const int S = A.S, nm = A.nm_next;
    const bool colok = col < L.cols;
    const int s = colok ? (int)(col / L.P) : 0;
    const int p = colok ? (int)(col - (long)s * L.P) : 0;

    // this neuron's point-box bits and the slots' x-bits (eL = !x or point,
    // eH = x or point per mask)
    unsigned dg4 = 0, xq4[kMaxMasks];
#pragma unroll
    for (int q = 0; q < kMaxMasks; ++q) xq4[q] = 0;
    if (colok) {
#pragma unroll
        for (int e = 0; e < CB; ++e) {
            if (c0 + e < L.C) {
                const long bie = (long)(c0 + e) * L.colpad + col;
                dg4 |= getbit(A.nk.deg, bie) << e;
#pragma unroll
                for (int q = 0; q < kMaxMasks; ++q)
                    if (q < nm) xq4[q] |= getbit(A.Rn.slot[q].xbits, bie) << e;
            }
        }
    }
    // W+^T u and W-^T u per mask, folded with the bits at the end
    Tc acc[CB];
    Tc accP[kMaxMasks][CB], accQ[kMaxMasks][CB];
#pragma unroll
    for (int e = 0; e < CB; ++e) {
        acc[e] = 0;
#pragma unroll
        for (int q = 0; q < kMaxMasks; ++q) accP[q][e] = accQ[q][e] = 0;
    }
    auto add = [&](int e, Tc w, Tc v, const Tc* uq) {
        acc[e] += w * v;
#pragma unroll
        for (int q = 0; q < kMaxMasks; ++q) {
            if (q < nm) {
                accP[q][e] += tmax0(w) * uq[q];
                accQ[q][e] += tmin0(w) * uq[q];
            }
        }
    };
    if (colok) {
        if (g.kind == ASD_LAYER_DENSE) {
            // reduction over the outputs i of the dense layer k+1
            const int n1 = O.C;
            const int i0 = (int)((long)n1 * wave / KS), i1 = (int)((long)n1 * (wave + 1) / KS);
            for (int i = i0; i < i1; ++i) {
                const long a = (long)i * S + s;  // dense output layout, P = 1
                const long bi = (long)i * O.colpad + s;
                Tc uq[kMaxMasks];
                const Tc v = bwd_operand<Tc, Ts>(A, a, bi, uq);
#pragma unroll
                for (int e = 0; e < CB; ++e) {
                    const int c = c0 + e;
                    const Tc w = c < L.C ? (Tc)g.W[(long)i * g.fan + (long)c * L.P + p] : (Tc)0;
                    add(e, w, v, uq);
                }
            }
        } else {
            // transposed convolution: input (c, y, x) receives output (co, oy, ox)
            // through tap (ky, kx) with oy * stride - pad + ky = y
            const int y = p / L.W, x = p - (p / L.W) * L.W;
            const int co0 = (int)((long)O.C * wave / KS), co1 = (int)((long)O.C * (wave + 1) / KS);
            const int ks = g.ksz, str = g.stride;
            const int ky0 = (y + g.pad) % str, kx0 = (x + g.pad) % str;
            // (y + pad - ky) is a multiple of the stride for every ky of the
            // loop: the output row falls by one per step of ky
            const int oyf = (y + g.pad - ky0) / str, oxf = (x + g.pad - kx0) / str;
            for (int co = co0; co < co1; ++co) {
                int oy = oyf;
                for (int ky = ky0; ky < ks; ky += str, --oy) {
                    if (oy < 0 || oy >= O.H) continue;
                    int ox = oxf;
                    for (int kx = kx0; kx < ks; kx += str, --ox) {
                        if (ox < 0 || ox >= O.W) continue;
                        const int op = oy * O.W + ox;
                        const long a = ((long)co * S + s) * O.P + op;
                        const long bi = (long)co * O.colpad + (long)s * O.P + op;
                        Tc uq[kMaxMasks];
                        const Tc v = bwd_operand<Tc, Ts>(A, a, bi, uq);
#pragma unroll
                        for (int e = 0; e < CB; ++e) {
                            const int c = c0 + e;
                            const Tc w = c < L.C ? (Tc)g.W[(((long)co * L.C + c) * ks + ky) * ks + kx] : (Tc)0;
                            add(e, w, v, uq);
                        }
                    }
                }
            }
        }
    }
    // fold the masked products with this neuron's e-bits before reducing
    // across waves: f gets eL (W+^T u) + eH (W-^T u) per mask
#pragma unroll
    for (int e = 0; e < CB; ++e) {
        Tc part = acc[e];
        const bool dg = (dg4 >> e) & 1u;
#pragma unroll
        for (int q = 0; q < kMaxMasks; ++q) {
            if (q < nm) {
                const bool xq = (xq4[q] >> e) & 1u;
                if (!xq || dg) part += accP[q][e];
                if (xq || dg) part += accQ[q][e];
            }
        }
        red[(wave * CB + e) * kWave + lane] = part;
    }
    __syncthreads();
    const int e = wave;
    const int c = c0 + e;
    if (c >= L.C) return;  // whole wave leaves together
    const long idx = ((long)c * S + s) * L.P + p;
    Tc f = 0;
    bool xb = false, zb = false;
    if (colok) {
        for (int w = 0; w < KS; ++w) f += red[(w * CB + e) * kWave + lane];
        const int nmo = A.nm_own;
        if (A.k >= 1) f += (Tc)A.Rk.own[idx];
        if (A.fout) A.fout[idx] = (double)f;
        if (A.fext) A.fext[(long)s * L.N + (long)c * L.P + p] = (Ts)f;
        // x-bit "x* = upper end"; a point box counts as both ends and keeps the bit set
        xb = f >= 0 || ((dg4 >> e) & 1u);
        const Tc xv = xb ? (Tc)A.nk.hi[idx] : (Tc)A.nk.lo[idx];
        A.nk.xstar[idx] = (Ts)xv;
        Tc term = -f * xv;
        if (A.k >= 1) {
            const Tc gk = (Tc)A.Rk.g[idx];
            zb = gk >= 0;
            term -= zb ? gk : (Tc)0;
            if (A.want_obj) {
                const Tc bb = (Tc)A.bk[c];
                Tc cst = bb * (Tc)A.Rk.alpha[idx] + (Tc)A.Rk.beta1[idx] * ((Tc)A.Rk.lhat[idx] - bb);
                for (int q = 0; q < nmo; ++q) cst += (Tc)A.Rk.slot[q].LI[idx] * (Tc)A.Rk.slot[q].beta[idx];
                term += cst;
            }
        }
        if (A.want_obj) A.nk.term[idx] = (double)term;
    }
    const long base = (long)c * L.colpad + (long)blockIdx.x * kWave;
    put_wave_bits(A.nk.xbits, base, colok && xb, lane);
    if (A.k >= 1) put_wave_bits(A.Rk.zbits, base, colok && zb, lane);
}

// ---------------------------------------------------------------------------
// Active-set extension: the constants LI, UI of slot q of ReLU layer k from
// the given compact mask bits (Tc == Ts), or, for the final bound of an FP32
// plan (Tc = double, Ts = float), every active slot's constants in FP64 and
// the FP64 per-neuron sums of the bound.
// ---------------------------------------------------------------------------
template <typename Ts>
struct MaskArgs {
    LayerGeo g;                 // layer k
    int S;
    int q;                      // slot to fill
    int nm;                     // active masks
    const Ts* lo_in; const Ts* hi_in;   // box of layer k-1
    const uint32_t* zsrc;       // z bits of layer k
    const uint32_t* xsrc;       // x*_{k-1} == hi bits of layer k-1
    int zero_state;             // also zero the slot's beta, moments, u
    const uint32_t* deg_in;
    ReluLayerT<Ts> R;
};

// One tap t of the mask constants of channels c0 .. c0 + CB - 1: the box
// ends lo, hi of the input, its point-box bit dg and the mask's x-bit xb.
template <typename Tc>
__device__ __forceinline__ void mask_tap(const LayerGeo& g, int t, int c0, int F, unsigned zmask, Tc lo, Tc hi,
                                         unsigned dg, unsigned xb, Tc (&LI)[CB], Tc (&UI)[CB]) {
    const bool eL = !xb || dg, eH = xb || dg;
#pragma unroll
    for (int e = 0; e < CB; ++e) {
        const int c = c0 + e;
        const Tc w = c < g.out.C ? (Tc)g.W[(long)c * F + t] : (Tc)0;
        const Tc wl = w >= 0 ? w * lo : w * hi;   // W . Lcheck
        const Tc wu = w >= 0 ? w * hi : w * lo;   // W . Ucheck
        const bool zi = (zmask >> e) & 1u;
        const bool bit = zi || (w > 0 ? eL : (w < 0 ? eH : true));
        // selects of values (a branch lets the compiler select the target
        // instead and index the accumulators dynamically, in scratch memory)
        LI[e] = bit ? LI[e] + wl : LI[e];
        UI[e] = bit ? UI[e] : UI[e] + wu;
    }
}

// NW: waves splitting the fan-in; DV: a dense layer over channels of 4k
// positions whose fan-in splits into multiples of 4 taps
template <typename Tc, typename Ts, int NW, bool DV>
__global__ void __launch_bounds__(kWave * NW) k_mask_consts(MaskArgs<Ts> A) {
    static_assert(NW >= CB, "one wave per channel finishes the sums");
    extern __shared__ unsigned char red_raw[];
    Tc* red = reinterpret_cast<Tc*>(red_raw);  // [NW][CB][2][64]
    static_assert(sizeof(Tc) == sizeof(Ts), "one type for sums and state");
    const LayerGeo& g = A.g;
    const int lane = threadIdx.x, wave = __builtin_amdgcn_readfirstlane(threadIdx.y);  // wave-uniform
    const long col = (long)blockIdx.x * kWave + lane;
    const int c0 = blockIdx.y * CB;
    const int S = A.S;
    const bool colok = col < g.out.cols;
    const int s = colok ? (int)(col / g.out.P) : 0;
    const int p = colok ? (int)(col - (long)s * g.out.P) : 0;
    const long bicol0 = (long)c0 * g.out.colpad + col;

    // the slot's LI and UI over this wave's taps
    Tc LI[CB], UI[CB];
#pragma unroll
    for (int e = 0; e < CB; ++e) LI[e] = UI[e] = 0;
    const int F = g.fan;
    const int t0 = (int)((long)F * wave / NW), t1 = (int)((long)F * (wave + 1) / NW);
    if (colok) {
        const uint32_t* zb = A.zsrc;
        const uint32_t* xbits = A.xsrc;
        unsigned zmask = 0;
#pragma unroll
        for (int e = 0; e < CB; ++e)
            if (c0 + e < g.out.C) zmask |= getbit(zb, bicol0 + (long)e * g.out.colpad) << e;
        if constexpr (DV) {
            // dense layer over channels of 4k positions: 4 consecutive taps
            // are consecutive positions of one channel (one vector load of
            // each box end; their bits share a word), same order of the sums
            for (int t = t0; t < t1; t += 4) {
                const int ci = t / g.in.P, pj = t - ci * g.in.P;
                const long a = ((long)ci * S + s) * g.in.P + pj;
                const long bi = (long)ci * g.in.colpad + (long)s * g.in.P + pj;
                const unsigned dw = A.deg_in[bi >> 5] >> (bi & 31), xw = xbits[bi >> 5] >> (bi & 31);
                Tc lo[4], hi[4];
                if constexpr (sizeof(Ts) == 4) {
                    const float4 l = *reinterpret_cast<const float4*>(A.lo_in + a);
                    const float4 h = *reinterpret_cast<const float4*>(A.hi_in + a);
                    lo[0] = (Tc)l.x, lo[1] = (Tc)l.y, lo[2] = (Tc)l.z, lo[3] = (Tc)l.w;
                    hi[0] = (Tc)h.x, hi[1] = (Tc)h.y, hi[2] = (Tc)h.z, hi[3] = (Tc)h.w;
                } else {
                    const double2 l0 = reinterpret_cast<const double2*>(A.lo_in + a)[0];
                    const double2 l1 = reinterpret_cast<const double2*>(A.lo_in + a)[1];
                    const double2 h0 = reinterpret_cast<const double2*>(A.hi_in + a)[0];
                    const double2 h1 = reinterpret_cast<const double2*>(A.hi_in + a)[1];
                    lo[0] = (Tc)l0.x, lo[1] = (Tc)l0.y, lo[2] = (Tc)l1.x, lo[3] = (Tc)l1.y;
                    hi[0] = (Tc)h0.x, hi[1] = (Tc)h0.y, hi[2] = (Tc)h1.x, hi[3] = (Tc)h1.y;
                }
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    mask_tap<Tc>(g, t + u, c0, F, zmask, lo[u], hi[u], (dw >> u) & 1u, (xw >> u) & 1u, LI, UI);
            }
        } else {
            TapWalk tw = tap_walk(g, p, t0);
#pragma unroll 4
            for (int t = t0; t < t1; ++t, tap_next(g, tw)) {
                const FwdTap tp = tap_at(g, S, s, tw);
                if (tp.a < 0) continue;
                mask_tap<Tc>(g, t, c0, F, zmask, (Tc)A.lo_in[tp.a], (Tc)A.hi_in[tp.a], getbit(A.deg_in, tp.bi),
                             getbit(xbits, tp.bi), LI, UI);
            }
        }
    }
#pragma unroll
    for (int e = 0; e < CB; ++e) {
        red[((wave * CB + e) * 2 + 0) * kWave + lane] = LI[e];
        red[((wave * CB + e) * 2 + 1) * kWave + lane] = UI[e];
    }
    __syncthreads();
    const int e = wave;
    if (e >= CB) return;
    const int c = c0 + e;
    if (!colok || c >= g.out.C) return;
    const long idx = ((long)c * S + s) * g.out.P + p;
    Tc r0 = 0, r1 = 0;
    for (int w = 0; w < NW; ++w) {
        r0 += red[((w * CB + e) * 2 + 0) * kWave + lane];
        r1 += red[((w * CB + e) * 2 + 1) * kWave + lane];
    }
    MaskSlotT<Ts> M = A.R.slot[A.q];
    M.LI[idx] = (Ts)r0;
    M.UI[idx] = (Ts)r1;
    if (A.zero_state) {
        M.beta[idx] = 0;
        M.m[idx] = 0;
        M.v[idx] = 0;
        M.u[idx] = 0;
    }
}

// Copies n 32-bit words.
static __global__ void k_copy_words(uint32_t* dst, const uint32_t* src, long n) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

// Fills n 32-bit words with zero (a kernel, so it can sit in a captured graph).
static __global__ void k_zero_words(uint32_t* dst, long n) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = 0u;
}

// Recomputes the derived per-neuron sums from the duals (after an import or
// at initialisation): own, g, vs and u_q.
template <typename T>
struct DeriveArgs {
    NeuronLayout nl;
    int S;
    int nm;
    const float* b;
    ReluLayerT<T> R;
};

template <typename T>
__global__ void k_derive(DeriveArgs<T> A) {
    const long col = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const int c = blockIdx.y;
    if (col >= A.nl.cols) return;
    const int s = (int)(col / A.nl.P), p = (int)(col - (long)s * A.nl.P);
    const long idx = ((long)c * A.S + s) * A.nl.P + p;
    const long bi = (long)c * A.nl.colpad + col;
    const T al = A.R.alpha[idx], b0 = A.R.beta0[idx], b1 = A.R.beta1[idx];
    const T bb = (T)A.b[c];
    T own = al - b0 - b1;
    T gg = b0 * A.R.uhat[idx] + b1 * A.R.lhat[idx];
    T vs = -al + b1;
    for (int q = 0; q < A.nm; ++q) {
        const MaskSlotT<T>& M = A.R.slot[q];
        const T bq = M.beta[idx];
        const bool zq = getbit(M.zbits, bi);
        own -= bq;
        gg += bq * (M.LI[idx] + M.UI[idx] + bb);
        vs += zq ? bq : (T)0.5 * bq;
        M.u[idx] = zq ? (T)0 : bq;
    }
    A.R.own[idx] = own;
    A.R.g[idx] = gg;
    A.R.vs[idx] = vs;
}

// ---------------------------------------------------------------------------
// Layout conversion between the caller's [S][N] arrays and the internal one.
// mode 0: int = ext; 1: int = max(ext, 0); 2: ext = int.
// ---------------------------------------------------------------------------
template <typename Ti, typename Te>
__global__ void k_layout(Ti* in_arr, Te* ex_arr, NeuronLayout nl, int S, int mode) {
    const long col = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const int c = blockIdx.y;
    if (col >= nl.cols) return;
    const int s = (int)(col / nl.P), p = (int)(col - (long)s * nl.P);
    const long in_ = ((long)c * S + s) * nl.P + p;
    const long ex = (long)s * nl.N + (long)c * nl.P + p;
    if (mode == 0) {
        in_arr[in_] = (Ti)ex_arr[ex];
    } else if (mode == 1) {
        in_arr[in_] = ex_arr[ex] > 0 ? (Ti)ex_arr[ex] : (Ti)0;
    } else {
        if constexpr (!std::is_const<Te>::value) ex_arr[ex] = (Te)in_arr[in_];
    }
}

// Bits of an internal bit array -> caller [S][N] values 0/1 (mode 0), or
// "value == hi" bits from caller values (mode 1), or "value >= 0.5" (mode 2),
// or point-box bits lo == hi from internal arrays (mode 3), or bits ->
// caller values hi / lo (mode 4).
template <typename T, typename Te>
struct BitArgs {
    NeuronLayout nl;
    int S;
    int mode;
    uint32_t* bits;
    Te* fext;
    const T* hi;   // internal (modes 1, 3, 4)
    const T* lo;   // internal (modes 3, 4)
};

template <typename T, typename Te>
__global__ void k_bits(BitArgs<T, Te> A) {
    const int lane = threadIdx.x & 63;
    const long col = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const int c = blockIdx.y;
    const bool ok = col < A.nl.cols;
    const int s = ok ? (int)(col / A.nl.P) : 0;
    const int p = ok ? (int)(col - (long)s * A.nl.P) : 0;
    const long in_ = ((long)c * A.S + s) * A.nl.P + p;
    const long ex = (long)s * A.nl.N + (long)c * A.nl.P + p;
    const long bi = (long)c * A.nl.colpad + col;
    if (A.mode == 0) {
        if (ok) A.fext[ex] = (Te)getbit(A.bits, bi);
        return;
    }
    if (A.mode == 4) {
        if (ok) A.fext[ex] = (Te)(getbit(A.bits, bi) ? A.hi[in_] : A.lo[in_]);
        return;
    }
    bool pred = false;
    if (ok) {
        if (A.mode == 1) pred = (T)A.fext[ex] == A.hi[in_];
        else if (A.mode == 2) pred = A.fext[ex] >= (Te)0.5;
        else pred = A.lo[in_] == A.hi[in_];
    }
    if (col - lane < A.nl.colpad) put_wave_bits(A.bits, (long)c * A.nl.colpad + (col - lane), pred, lane);
}

// Device copy of one layer's array table, passed by value as the kernel
// argument (no host buffer has to outlive the launch).  One thread.
template <typename T>
__global__ void k_store_layer(ReluLayerT<T>* dst, ReluLayerT<T> v) {
    *dst = v;
}

// Per-subproblem objective: sum of every neuron term (fixed order) plus b_n^T c.
template <typename T>
struct ReduceArgs {
    int S;
    int nlayers;                       // neuron layers 0..n-1
    NeuronLayout nl[kMaxLayers];
    const double* term[kMaxLayers];
    const T* cint;                     // objective rows, internal layout of layer n ([C][S][P])
    const float* bn;                   // bias of layer n, per channel
    int c_last, p_last;                // channels and positions of layer n
    double* out;
};

// Per-subproblem finiteness flags: bit 0 = the bound is not finite (first
// kernel, one thread per subproblem), bit 1 = some multiplier of the
// subproblem is not finite (second kernel, one thread per neuron of a ReLU
// layer, flags OR-ed in with vector atomics).
static __global__ void __launch_bounds__(256) k_flags_bound(const double* lb, const int32_t* inflags, int32_t* flags,
                                                            int S) {
    const int s = blockIdx.x * 256 + threadIdx.x;
    if (s < S) flags[s] = (isfinite(lb[s]) ? 0 : 1) | inflags[s];
}

// Intermediate bounds by the solver (App. E): the replicated batch of the
// sub-network's 2 n_k D subproblems, subproblem s = (2 d + h) n_k + j for box
// d, neuron j, h = 0 (lower bound, row e_j) or 1 (upper bound, row -e_j).
// Row r of dst [rows][n] = row r / per of src.
static __global__ void __launch_bounds__(256) k_bcast_rows(float* dst, const float* src, long rows, int n, int per) {
    const long i = (long)blockIdx.x * 256 + threadIdx.x;
    if (i >= rows * n) return;
    const long r = i / n;
    dst[i] = src[(r / per) * n + (i - r * n)];
}

static __global__ void __launch_bounds__(256) k_ib_objective(float* c, long S, int nk) {
    const long i = (long)blockIdx.x * 256 + threadIdx.x;
    if (i >= S * nk) return;
    const long s = i / nk;
    const int e = (int)(i - s * nk), j = (int)(s % nk);
    const bool up = (s / nk) % 2 == 1;
    c[i] = e == j ? (up ? -1.f : 1.f) : 0.f;
}

// lhat = max(lhat, d_lo), uhat = min(uhat, -d_hi), the dual bounds rounded
// outward to FP32; a bound that is not finite leaves the interval bound.
static __global__ void __launch_bounds__(256) k_ib_combine(float* lhat, float* uhat, const double* dB, int D, int nk) {
    const long i = (long)blockIdx.x * 256 + threadIdx.x;
    if (i >= (long)D * nk) return;
    const long d = i / nk;
    const int j = (int)(i - d * nk);
    const double lo = dB[(2 * d) * nk + j], hi = -dB[(2 * d + 1) * nk + j];
    if (isfinite(lo)) lhat[i] = fmaxf(lhat[i], __double2float_rd(lo));
    if (isfinite(hi)) uhat[i] = fminf(uhat[i], __double2float_ru(hi));
}

// l2-ball input domain (the input set C of Sec. 2): x*_0 maximises f_0^T x_0
// over ||x_0 - centre|| <= radius, i.e. x*_0 = centre + radius f_0 / ||f_0||
// (the centre where f_0 = 0); with term set, the objective terms -f_0 x*_0 of
// the final bound.  One block per subproblem; the norm is a fixed-order
// block sum in FP64.  f_0 in the caller's layout [S][n_0] (f_internal = 0)
// or the internal one; centre [S][n_0] and radius [S] as the caller gave
// them; x*_0 and the terms in the internal layout.
template <typename Ts, typename Tf>
__global__ void __launch_bounds__(256) k_l2_input(const Tf* f0, int f_internal, const float* centre,
                                                  const float* radius, Ts* xstar, double* term, NeuronLayout nl,
                                                  int S) {
    __shared__ double red[256];
    const int s = blockIdx.x;
    const long n = nl.N;
    auto internal = [&](long j) {
        const long c = j / nl.P;
        return ((long)c * S + s) * nl.P + (j - c * nl.P);
    };
    double acc = 0;
    for (long j = threadIdx.x; j < n; j += 256) {
        const double f = (double)f0[f_internal ? internal(j) : (long)s * n + j];
        acc += f * f;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    const double nrm = sqrt(red[0]);
    const double r = (double)radius[s];
    for (long j = threadIdx.x; j < n; j += 256) {
        const long ii = internal(j);
        const double f = (double)f0[f_internal ? ii : (long)s * n + j];
        const double x = (double)centre[(long)s * n + j] + (nrm > 0 ? r * f / nrm : 0.0);
        xstar[ii] = (Ts)x;
        if (term) term[ii] = -f * x;
    }
}

// dst = -src (n entries): the backward operand of a convolutional output
// layer, -c in its internal layout.
static __global__ void __launch_bounds__(256) k_negate(float* dst, const float* src, long n) {
    const long i = (long)blockIdx.x * 256 + threadIdx.x;
    if (i < n) dst[i] = -src[i];
}

// Input check of a batch (caller layout [S][n]): bit 2 of flags[s] is set
// where an entry of subproblem s is not finite or, with hi given, lo > hi
// (an empty interval: the subdomain is infeasible).  One thread per entry.
static __global__ void __launch_bounds__(256) k_flags_inputs(const float* lo, const float* hi, long n, int S,
                                                             int32_t* flags) {
    const long i = (long)blockIdx.x * 256 + threadIdx.x;
    if (i >= n * S) return;
    const float a = lo[i];
    bool bad = !isfinite(a);
    if (hi) {
        const float b = hi[i];
        bad = bad || !isfinite(b) || a > b;
    }
    if (bad) atomicOr(&flags[i / n], 4);
}

template <typename T>
__global__ void __launch_bounds__(256) k_flags_duals(ReluLayerT<T> R, NeuronLayout nl, int S, int nm, int32_t* flags) {
    const long col = (long)blockIdx.x * 256 + threadIdx.x;
    const int c = blockIdx.y;
    if (col >= nl.cols) return;
    const int s = (int)(col / nl.P);
    const long idx = (long)c * nl.cols + col;
    bool ok = isfinite(R.alpha[idx]) && isfinite(R.beta0[idx]) && isfinite(R.beta1[idx]);
    for (int q = 0; q < nm; ++q) ok = ok && isfinite(R.slot[q].beta[idx]);
    if (!ok) atomicOr(&flags[s], 2);
}

// Learning rate of Active Set iteration t for each updated subproblem on its
// own linear schedule over its budget (the same expression as the shared
// schedule, in FP64).
template <typename T>
__global__ void __launch_bounds__(256) k_lr_schedule(const int* budgets, int Sa, int t, double lr0, double lr1, T* lrs) {
    const int s = blockIdx.x * 256 + threadIdx.x;
    if (s >= Sa) return;
    const int Ts = budgets[s];
    lrs[s] = (T)(Ts <= 1 ? lr0 : lr0 + (lr1 - lr0) * (double)t / (double)(Ts - 1));
}

template <typename T>
__global__ void __launch_bounds__(256) k_reduce_obj(ReduceArgs<T> A) {
    __shared__ double part[256];
    const int s = blockIdx.x;
    double acc = 0;
    for (int k = 0; k < A.nlayers; ++k) {
        const NeuronLayout& nl = A.nl[k];
        for (long n = threadIdx.x; n < nl.N; n += blockDim.x) {
            const int c = (int)(n / nl.P), p = (int)(n - (long)c * nl.P);
            acc += A.term[k][((long)c * A.S + s) * nl.P + p];
        }
    }
    if (threadIdx.x == 0)
        for (int ch = 0; ch < A.c_last; ++ch)
            for (int p = 0; p < A.p_last; ++p)
                acc += (double)A.bn[ch] * (double)A.cint[((long)ch * A.S + s) * A.p_last + p];
    part[threadIdx.x] = acc;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) A.out[s] = part[0];
}

// ---------------------------------------------------------------------------
// General separation oracle (eq:oracle) at an arbitrary primal point, caller
// layout: x_prev [S][n_{k-1}], z [S][n_k]; bits [S][n_k][ceil(F/32)].
// ---------------------------------------------------------------------------
template <typename T>
struct OracleArgs {
    LayerGeo g;
    int S;
    const T* xprev;
    const T* z;
    const T* lo_in; const T* hi_in;  // internal layout, layer k-1
    uint32_t* bits;
    T* LI; T* UI;
};

template <typename T>
__global__ void k_oracle(OracleArgs<T> A) {
    const long gid = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const LayerGeo& g = A.g;
    if (gid >= (long)A.S * g.out.N) return;
    const int s = (int)(gid / g.out.N);
    const long i = gid - (long)s * g.out.N;
    const int c = (int)(i / g.out.P), p = (int)(i - (long)c * g.out.P);
    const T zi = A.z[gid];
    const int F = g.fan, nw = (F + 31) / 32;
    uint32_t word = 0;
    T LI = 0, UI = 0;
    for (int t = 0; t < F; ++t) {
        const FwdTap tp = fwd_tap(g, A.S, s, p, t);
        bool bit = false;
        if (tp.a >= 0) {
            // caller index of the input neuron
            const long ci = tp.a / ((long)A.S * g.in.P);
            const long pin = tp.a - (ci * A.S + s) * g.in.P;
            const T x = A.xprev[(long)s * g.in.N + ci * g.in.P + pin];
            const T lo = A.lo_in[tp.a], hi = A.hi_in[tp.a];
            const T w = (T)g.W[(long)c * F + t];
            const T Lc = w >= 0 ? lo : hi, Uc = w >= 0 ? hi : lo;
            const T d = ((T)1 - zi) * Lc + zi * Uc - x;
            // sign of d * w without forming the product (no underflow to 0)
            bit = (d == (T)0) || (w == (T)0) || ((d > (T)0) == (w > (T)0));
            if (bit) LI += w * Lc;
            else UI += w * Uc;
        }
        if (bit) word |= 1u << (t & 31);
        if ((t & 31) == 31 || t == F - 1) {
            A.bits[gid * nw + (t >> 5)] = word;
            word = 0;
        }
    }
    A.LI[gid] = LI;
    A.UI[gid] = UI;
}

// ---------------------------------------------------------------------------
// Interval propagation (App. E), FP64 sums, outward rounding to FP32.
// Caller layout; lo_in/hi_in are the previous layer's bounds (for layer 1 the
// input box; later layers read the pre-activation bounds of the previous
// layer and clamp at 0).
// ---------------------------------------------------------------------------
struct IbpArgs {
    LayerGeo g;
    int S;
    const float* lo_in; const float* hi_in;
    int clamp_in;
    float* lo_out; float* hi_out;
};

static __global__ void k_ibp(IbpArgs A) {
    const long gid = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const LayerGeo& g = A.g;
    if (gid >= (long)A.S * g.out.N) return;
    const int s = (int)(gid / g.out.N);
    const long i = gid - (long)s * g.out.N;
    const int c = (int)(i / g.out.P), p = (int)(i - (long)c * g.out.P);
    double lo = g.b[c], hi = g.b[c];
    const int F = g.fan;
    for (int t = 0; t < F; ++t) {
        long j;
        if (g.kind == ASD_LAYER_DENSE) {
            j = t;
        } else {
            const int k2 = g.ksz * g.ksz;
            const int ci = t / k2, rem = t - ci * k2;
            const int ky = rem / g.ksz, kx = rem - ky * g.ksz;
            const int oy = p / g.out.W, ox = p - oy * g.out.W;
            const int iy = oy * g.stride - g.pad + ky, ix = ox * g.stride - g.pad + kx;
            if (iy < 0 || iy >= g.in.H || ix < 0 || ix >= g.in.W) continue;
            j = (long)ci * g.in.P + iy * g.in.W + ix;
        }
        double l = A.lo_in[(long)s * g.in.N + j], u = A.hi_in[(long)s * g.in.N + j];
        if (A.clamp_in) {
            l = l > 0 ? l : 0;
            u = u > 0 ? u : 0;
        }
        const double w = g.W[(long)c * F + t];
        if (w >= 0) {
            lo += w * l;
            hi += w * u;
        } else {
            lo += w * u;
            hi += w * l;
        }
    }
    A.lo_out[gid] = __double2float_rd(lo);
    A.hi_out[gid] = __double2float_ru(hi);
}

}  // namespace asd
