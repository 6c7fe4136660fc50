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

// ---------------------------------------------------------------------------
// Tap enumeration of layer L's receptive field for output column (s, p).
// ---------------------------------------------------------------------------
struct FwdTap {
    long a;     // input neuron address in the internal layout, or -1 (padding)
    long bi;    // input bit index
};

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
struct FwdArgs {
    LayerGeo g;                 // layer k
    int S;
    int nm;                     // active masks
    const float* xin;           // x*_{k-1}
    const uint32_t* deg_in;     // point boxes of layer k-1
    const float* xout;          // x*_k
    const uint32_t* zbits;      // z*_k
    ReluLayer R;                // layer k arrays
    StepArgs st;
    int mode;                   // 0 update, 1 export supergradient
    float* gout[3 + kMaxMasks]; // export targets, caller layout [S][n_k]
};

__global__ void __launch_bounds__(kWave * KS) k_forward(FwdArgs A) {
    extern __shared__ float red[];  // [KS][CB][1 + nm][64]
    const LayerGeo& g = A.g;
    const int lane = threadIdx.x, wave = threadIdx.y;
    const long col = (long)blockIdx.x * kWave + lane;
    const int c0 = blockIdx.y * CB;
    const int S = A.S, nm = A.nm;
    const bool colok = col < g.out.cols;
    const int s = colok ? (int)(col / g.out.P) : 0;
    const int p = colok ? (int)(col - (long)s * g.out.P) : 0;

    float acc[CB];
    float accm[kMaxMasks][CB];
#pragma unroll
    for (int e = 0; e < CB; ++e) {
        acc[e] = 0.f;
#pragma unroll
        for (int q = 0; q < kMaxMasks; ++q) accm[q][e] = 0.f;
    }
    const int F = g.fan;
    const int t0 = (int)((long)F * wave / KS), t1 = (int)((long)F * (wave + 1) / KS);
    if (colok) {
        for (int t = t0; t < t1; ++t) {
            const FwdTap tp = fwd_tap(g, S, s, p, t);
            const bool ok = tp.a >= 0;
            const float x = ok ? A.xin[tp.a] : 0.f;
            const unsigned dg = ok ? getbit(A.deg_in, tp.bi) : 0u;
            float w[CB];
#pragma unroll
            for (int e = 0; e < CB; ++e) {
                const int c = c0 + e;
                w[e] = c < g.out.C ? g.W[(long)c * F + t] : 0.f;
                acc[e] = fmaf(w[e], x, acc[e]);
            }
#pragma unroll
            for (int q = 0; q < kMaxMasks; ++q) {
                if (q < nm) {
                    const unsigned xb = ok ? getbit(A.R.slot[q].xbits, tp.bi) : 0u;
                    const float aL = (!xb || dg) ? x : 0.f;
                    const float aH = (xb || dg) ? x : 0.f;
#pragma unroll
                    for (int e = 0; e < CB; ++e)
                        accm[q][e] = fmaf(fmaxf(w[e], 0.f), aL, fmaf(fminf(w[e], 0.f), aH, accm[q][e]));
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
    float yd = 0.f;
    float ym[kMaxMasks];
    for (int w = 0; w < KS; ++w) yd += red[((w * CB + e) * ncomp + 0) * kWave + lane];
#pragma unroll
    for (int q = 0; q < kMaxMasks; ++q) {
        ym[q] = 0.f;
        if (q < nm)
            for (int w = 0; w < KS; ++w) ym[q] += red[((w * CB + e) * ncomp + 1 + q) * kWave + lane];
    }
    const long idx = ((long)c * S + s) * g.out.P + p;
    const long bi = (long)c * g.out.colpad + col;
    const float bb = g.b[c];
    const float xhat = yd + bb;
    const float x = A.xout[idx];
    const float z = (float)getbit(A.zbits, bi);
    const float lh = A.R.lhat[idx], uh = A.R.uhat[idx];
    const float ga = xhat - x;
    const float gb0 = x - z * uh;
    const float gb1 = x - xhat + (1.f - z) * lh;
    float gm[kMaxMasks];
    float zq[kMaxMasks];
#pragma unroll
    for (int q = 0; q < kMaxMasks; ++q) {
        gm[q] = 0.f;
        zq[q] = 0.f;
        if (q < nm) {
            const MaskSlot& M = A.R.slot[q];
            zq[q] = (float)getbit(M.zbits, bi);
            const float mq = zq[q] != 0.f ? yd : ym[q];
            gm[q] = x - mq + M.LI[idx] * (1.f - z) - z * bb - M.UI[idx] * z;
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
    const StepArgs& st = A.st;
    auto step = [&](float th, float* m, float* v, float gr, int grp) -> float {
        if (st.rule == ASD_RULE_SUPERGRADIENT) return fmaxf(th + st.lr * gr, 0.f);
        float mm = st.b1 * m[idx] + (1.f - st.b1) * gr;
        float vv = st.b2 * v[idx] + (1.f - st.b2) * gr * gr;
        m[idx] = mm;
        v[idx] = vv;
        const float mh = mm / st.bc1[grp];
        const float vh = vv / st.bc2[grp];
        return fmaxf(th + st.lr * mh / (sqrtf(vh) + st.eps), 0.f);
    };
    const float al = step(A.R.alpha[idx], A.R.alpha_m, A.R.alpha_v, ga, 0);
    const float b0 = step(A.R.beta0[idx], A.R.beta0_m, A.R.beta0_v, gb0, 0);
    const float b1 = step(A.R.beta1[idx], A.R.beta1_m, A.R.beta1_v, gb1, 0);
    A.R.alpha[idx] = al;
    A.R.beta0[idx] = b0;
    A.R.beta1[idx] = b1;
    float own = al - b0 - b1;
    float gg = b0 * uh + b1 * lh;
    float vdn = -al + b1;
#pragma unroll
    for (int q = 0; q < kMaxMasks; ++q) {
        if (q < nm) {
            const MaskSlot& M = A.R.slot[q];
            const float bq = step(M.beta[idx], M.m, M.v, gm[q], 1 + q);
            M.beta[idx] = bq;
            own -= bq;
            gg += bq * (M.LI[idx] + M.UI[idx] + bb);
            vdn += zq[q] * bq;
            M.u[idx] = (1.f - zq[q]) * bq;
        }
    }
    A.R.own[idx] = own;
    A.R.g[idx] = gg;
    A.R.vdn[idx] = vdn;
}

// ---------------------------------------------------------------------------
// Backward pass: f_k, the inner minimisation, objective terms.
// Template T = float (iterations, fixed-dual evaluation) or double (final
// bound: every sum in FP64 from the FP32 duals and weights).
// ---------------------------------------------------------------------------
struct BwdArgs {
    LayerGeo gn;                // layer k+1 (its input layout is layer k)
    int S;
    int k;                      // neuron layer (0 = input)
    int last;                   // k + 1 == n: backward operand is -c
    int nm_next;                // active masks of layer k+1 (0 if last)
    int nm_own;                 // active masks of layer k (k >= 1)
    const float* cvec;          // objective rows, layout of layer n
    ReluLayer Rn;               // layer k+1 arrays (if not last)
    ReluLayer Rk;               // layer k arrays (if k >= 1)
    NeuronArrays nk;            // layer k box, outputs
    const float* bk;            // bias of layer k (k >= 1), per channel
    int want_obj;
};

template <typename T>
__device__ __forceinline__ T bwd_operand(const BwdArgs& A, long a, long bi, T* uq) {
    // dense operand v and masked operands u_q at output neuron address a of layer k+1
    if (A.last) return -(T)A.cvec[a];
    if (sizeof(T) == 4) {
#pragma unroll
        for (int q = 0; q < kMaxMasks; ++q)
            if (q < A.nm_next) uq[q] = (T)A.Rn.slot[q].u[a];
        return (T)A.Rn.vdn[a];
    }
    T v = -(T)A.Rn.alpha[a] + (T)A.Rn.beta1[a];
#pragma unroll
    for (int q = 0; q < kMaxMasks; ++q) {
        if (q < A.nm_next) {
            const T bq = (T)A.Rn.slot[q].beta[a];
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

template <typename T>
__global__ void __launch_bounds__(kWave * KS) k_backward(BwdArgs A) {
    extern __shared__ unsigned char red_raw[];
    T* red = reinterpret_cast<T*>(red_raw);  // [KS][CB][64]
    const LayerGeo& g = A.gn;
    const NeuronLayout& L = g.in;   // layer k
    const NeuronLayout& O = g.out;  // layer k+1
    const int lane = threadIdx.x, wave = threadIdx.y;
    const long col = (long)blockIdx.x * kWave + lane;
    const int c0 = blockIdx.y * CB;
    const int S = A.S, nm = A.nm_next;
    const bool colok = col < L.cols;
    const int s = colok ? (int)(col / L.P) : 0;
    const int p = colok ? (int)(col - (long)s * L.P) : 0;

    T acc[CB];
    T accP[kMaxMasks][CB], accQ[kMaxMasks][CB];
#pragma unroll
    for (int e = 0; e < CB; ++e) {
        acc[e] = 0;
#pragma unroll
        for (int q = 0; q < kMaxMasks; ++q) accP[q][e] = accQ[q][e] = 0;
    }
    if (colok) {
        if (g.kind == ASD_LAYER_DENSE) {
            // reduction over the outputs i of the dense layer k+1
            const int n1 = O.C;
            const int i0 = (int)((long)n1 * wave / KS), i1 = (int)((long)n1 * (wave + 1) / KS);
            for (int i = i0; i < i1; ++i) {
                const long a = (long)i * S + s;  // dense output layout, P = 1
                const long bi = (long)i * O.colpad + s;
                T uq[kMaxMasks];
                const T v = bwd_operand<T>(A, a, bi, uq);
#pragma unroll
                for (int e = 0; e < CB; ++e) {
                    const int c = c0 + e;
                    const T w = c < L.C ? (T)g.W[(long)i * g.fan + (long)c * L.P + p] : (T)0;
                    acc[e] += w * v;
#pragma unroll
                    for (int q = 0; q < kMaxMasks; ++q) {
                        if (q < nm) {
                            accP[q][e] += (w > 0 ? w : (T)0) * uq[q];
                            accQ[q][e] += (w < 0 ? w : (T)0) * uq[q];
                        }
                    }
                }
            }
        } else {
            // transposed convolution: input (c, y, x) receives output (co, oy, ox)
            // through tap (ky, kx) with oy * stride - pad + ky = y
            const int y = p / L.W, x = p - (p / L.W) * L.W;
            const int co0 = (int)((long)O.C * wave / KS), co1 = (int)((long)O.C * (wave + 1) / KS);
            const int ks = g.ksz, str = g.stride;
            const int ky0 = (y + g.pad) % str, kx0 = (x + g.pad) % str;
            for (int co = co0; co < co1; ++co) {
                for (int ky = ky0; ky < ks; ky += str) {
                    const int oy = (y + g.pad - ky) / str;
                    if (oy < 0 || oy >= O.H) continue;
                    for (int kx = kx0; kx < ks; kx += str) {
                        const int ox = (x + g.pad - kx) / str;
                        if (ox < 0 || ox >= O.W) continue;
                        const int op = oy * O.W + ox;
                        const long a = ((long)co * S + s) * O.P + op;
                        const long bi = (long)co * O.colpad + (long)s * O.P + op;
                        T uq[kMaxMasks];
                        const T v = bwd_operand<T>(A, a, bi, uq);
#pragma unroll
                        for (int e = 0; e < CB; ++e) {
                            const int c = c0 + e;
                            const T w = c < L.C ? (T)g.W[(((long)co * L.C + c) * ks + ky) * ks + kx] : (T)0;
                            acc[e] += w * v;
#pragma unroll
                            for (int q = 0; q < kMaxMasks; ++q) {
                                if (q < nm) {
                                    accP[q][e] += (w > 0 ? w : (T)0) * uq[q];
                                    accQ[q][e] += (w < 0 ? w : (T)0) * uq[q];
                                }
                            }
                        }
                    }
                }
            }
        }
    }
    // fold the masked products with this neuron's e-bits before reducing
    // across waves: f gets eL (W+^T u) + eH (W-^T u) per mask
    {
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
#pragma unroll
        for (int e = 0; e < CB; ++e) {
            T part = acc[e];
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
    }
    __syncthreads();
    const int e = wave;
    const int c = c0 + e;
    if (c >= L.C) return;  // whole wave leaves together
    const long idx = ((long)c * S + s) * L.P + p;
    T f = 0;
    bool xb = false, zb = false;
    if (colok) {
        for (int w = 0; w < KS; ++w) f += red[(w * CB + e) * kWave + lane];
        const int nmo = A.nm_own;
        if (A.k >= 1) {
            if (sizeof(T) == 4) {
                f += (T)A.Rk.own[idx];
            } else {
                f += (T)A.Rk.own64[idx];
            }
        }
        xb = f >= 0;
        const T xv = xb ? (T)A.nk.hi[idx] : (T)A.nk.lo[idx];
        A.nk.xstar[idx] = (float)xv;
        T term = -f * xv;
        if (A.k >= 1) {
            T gk;
            if (sizeof(T) == 4) gk = (T)A.Rk.g[idx];
            else gk = (T)A.Rk.g64[idx];
            zb = gk >= 0;
            term -= zb ? gk : (T)0;
            if (A.want_obj) {
                if (sizeof(T) == 4) {
                    const T bb = (T)A.bk[c];
                    T cst = bb * (T)A.Rk.alpha[idx] + (T)A.Rk.beta1[idx] * ((T)A.Rk.lhat[idx] - bb);
                    for (int q = 0; q < nmo; ++q) cst += (T)A.Rk.slot[q].LI[idx] * (T)A.Rk.slot[q].beta[idx];
                    term += cst;
                } else {
                    term += (T)A.Rk.const64[idx];
                }
            }
        }
        if (A.want_obj) A.nk.term[idx] = (double)term;
    }
    const long base = (long)c * L.colpad + (long)blockIdx.x * kWave;
    put_wave_bits(A.nk.xbits, base, colok && xb, lane);
    if (A.k >= 1) put_wave_bits(A.Rk.zbits, base, colok && zb, lane);
}

template __global__ void k_backward<float>(BwdArgs);
template __global__ void k_backward<double>(BwdArgs);

// ---------------------------------------------------------------------------
// Active-set extension: store the compact mask of slot q of ReLU layer k and
// its constants LI, UI (T = float), or recompute every active slot's
// constants in FP64 and the FP64 per-neuron sums of the final bound
// (T = double).
// ---------------------------------------------------------------------------
struct MaskArgs {
    LayerGeo g;                 // layer k
    int S;
    int q;                      // slot to fill (T = float)
    int nm;                     // active masks (T = double)
    const float* lo_in; const float* hi_in;   // box of layer k-1
    const uint32_t* zsrc;       // z bits of layer k (T = float)
    const uint32_t* xsrc;       // x*_{k-1} == hi bits of layer k-1 (T = float)
    int zero_state;             // T = float: also zero the slot's beta, moments, u
    const uint32_t* deg_in;
    ReluLayer R;
};

template <typename T>
__global__ void __launch_bounds__(kWave * KS) k_mask_consts(MaskArgs A) {
    extern __shared__ unsigned char red_raw[];
    T* red = reinterpret_cast<T*>(red_raw);  // [KS][CB][2][64]
    const LayerGeo& g = A.g;
    const int lane = threadIdx.x, wave = threadIdx.y;
    const long col = (long)blockIdx.x * kWave + lane;
    const int c0 = blockIdx.y * CB;
    const int S = A.S;
    const bool f64 = sizeof(T) == 8;
    const int q0 = f64 ? 0 : A.q;
    const int nsl = f64 ? A.nm : 1;
    const bool colok = col < g.out.cols;
    const int s = colok ? (int)(col / g.out.P) : 0;
    const int p = colok ? (int)(col - (long)s * g.out.P) : 0;
    const long bicol0 = (long)c0 * g.out.colpad + col;

    T LI[kMaxMasks][CB], UI[kMaxMasks][CB];
    unsigned zmask[kMaxMasks];
#pragma unroll
    for (int j = 0; j < kMaxMasks; ++j) {
        zmask[j] = 0;
#pragma unroll
        for (int e = 0; e < CB; ++e) LI[j][e] = UI[j][e] = 0;
    }
    if (colok && nsl > 0) {
#pragma unroll
        for (int j = 0; j < kMaxMasks; ++j) {
            if (j < nsl) {
                const uint32_t* zb = f64 ? A.R.slot[q0 + j].zbits : A.zsrc;
#pragma unroll
                for (int e = 0; e < CB; ++e)
                    if (c0 + e < g.out.C) zmask[j] |= getbit(zb, bicol0 + (long)e * g.out.colpad) << e;
            }
        }
        const int F = g.fan;
        const int t0 = (int)((long)F * wave / KS), t1 = (int)((long)F * (wave + 1) / KS);
        for (int t = t0; t < t1; ++t) {
            const FwdTap tp = fwd_tap(g, S, s, p, t);
            if (tp.a < 0) continue;
            const T lo = (T)A.lo_in[tp.a], hi = (T)A.hi_in[tp.a];
            const unsigned dg = getbit(A.deg_in, tp.bi);
#pragma unroll
            for (int j = 0; j < kMaxMasks; ++j) {
                if (j < nsl) {
                    const uint32_t* xbits = f64 ? A.R.slot[q0 + j].xbits : A.xsrc;
                    const unsigned xb = getbit(xbits, tp.bi);
                    const bool eL = !xb || dg, eH = xb || dg;
#pragma unroll
                    for (int e = 0; e < CB; ++e) {
                        const int c = c0 + e;
                        const T w = c < g.out.C ? (T)g.W[(long)c * F + t] : (T)0;
                        const T wl = w >= 0 ? w * lo : w * hi;   // W . Lcheck
                        const T wu = w >= 0 ? w * hi : w * lo;   // W . Ucheck
                        const bool zi = (zmask[j] >> e) & 1u;
                        const bool bit = zi || (w > 0 ? eL : (w < 0 ? eH : true));
                        if (bit) LI[j][e] += wl;
                        else UI[j][e] += wu;
                    }
                }
            }
        }
    }
    // FP32 (one slot): reduce LI and UI.  FP64 (every active slot): each wave
    // folds its partial LI/UI of all slots with the slot multipliers into the
    // two sums the final bound needs, sum_q beta_q (LI_q + UI_q) and
    // sum_q beta_q LI_q, then the waves' partials are reduced.
#pragma unroll
    for (int e = 0; e < CB; ++e) {
        T r0 = 0, r1 = 0;
        if (!f64) {
            r0 = LI[0][e];
            r1 = UI[0][e];
        } else if (colok && c0 + e < g.out.C) {
            const long idx_e = ((long)(c0 + e) * S + s) * g.out.P + p;
#pragma unroll
            for (int j = 0; j < kMaxMasks; ++j) {
                if (j < nsl) {
                    const T bq = (T)A.R.slot[j].beta[idx_e];
                    r0 += bq * (LI[j][e] + UI[j][e]);
                    r1 += bq * LI[j][e];
                }
            }
        }
        red[((wave * CB + e) * 2 + 0) * kWave + lane] = r0;
        red[((wave * CB + e) * 2 + 1) * kWave + lane] = r1;
    }
    __syncthreads();
    const int e = wave;
    const int c = c0 + e;
    if (!colok || c >= g.out.C) return;
    const long idx = ((long)c * S + s) * g.out.P + p;
    T r0 = 0, r1 = 0;
    for (int w = 0; w < KS; ++w) {
        r0 += red[((w * CB + e) * 2 + 0) * kWave + lane];
        r1 += red[((w * CB + e) * 2 + 1) * kWave + lane];
    }
    if (!f64) {
        MaskSlot M = A.R.slot[q0];
        M.LI[idx] = (float)r0;
        M.UI[idx] = (float)r1;
        if (A.zero_state) {
            M.beta[idx] = 0.f;
            M.m[idx] = 0.f;
            M.v[idx] = 0.f;
            M.u[idx] = 0.f;
        }
        return;
    }
    // FP64 sums of the final bound for neuron (c, s, p) of layer k:
    // own = alpha - beta0 - beta1 - sum beta_I,
    // g = beta0 uhat + beta1 lhat + sum beta_I (LI + UI + b),
    // const = b alpha + beta1 (lhat - b) + sum LI beta_I.
    const double bb = (double)g.b[c];
    const double al = A.R.alpha[idx], b0 = A.R.beta0[idx], b1 = A.R.beta1[idx];
    const double lh = A.R.lhat[idx], uh = A.R.uhat[idx];
    double sb = 0;
    for (int j = 0; j < nsl; ++j) sb += (double)A.R.slot[j].beta[idx];
    A.R.own64[idx] = al - b0 - b1 - sb;
    A.R.g64[idx] = b0 * uh + b1 * lh + (double)r0 + bb * sb;
    A.R.const64[idx] = bb * al + b1 * (lh - bb) + (double)r1;
}

template __global__ void k_mask_consts<float>(MaskArgs);
template __global__ void k_mask_consts<double>(MaskArgs);

// Copies n 32-bit words.
__global__ void k_copy_words(uint32_t* dst, const uint32_t* src, long n) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

// Fills n 32-bit words with zero (a kernel, so it can sit in a captured graph).
__global__ void k_zero_words(uint32_t* dst, long n) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = 0u;
}

// Recomputes the derived per-neuron sums from the duals (after an import or
// at initialisation): own, g, vdn and u_q (FP32).
struct DeriveArgs {
    NeuronLayout nl;
    int S;
    int nm;
    const float* b;
    ReluLayer R;
};

__global__ void k_derive(DeriveArgs A) {
    const long col = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const int c = blockIdx.y;
    if (col >= A.nl.cols) return;
    const int s = (int)(col / A.nl.P), p = (int)(col - (long)s * A.nl.P);
    const long idx = ((long)c * A.S + s) * A.nl.P + p;
    const long bi = (long)c * A.nl.colpad + col;
    const float al = A.R.alpha[idx], b0 = A.R.beta0[idx], b1 = A.R.beta1[idx];
    const float bb = A.b[c];
    float own = al - b0 - b1;
    float gg = b0 * A.R.uhat[idx] + b1 * A.R.lhat[idx];
    float vdn = -al + b1;
    for (int q = 0; q < A.nm; ++q) {
        const MaskSlot& M = A.R.slot[q];
        const float bq = M.beta[idx];
        const float zq = (float)getbit(M.zbits, bi);
        own -= bq;
        gg += bq * (M.LI[idx] + M.UI[idx] + bb);
        vdn += zq * bq;
        M.u[idx] = (1.f - zq) * bq;
    }
    A.R.own[idx] = own;
    A.R.g[idx] = gg;
    A.R.vdn[idx] = vdn;
}

// ---------------------------------------------------------------------------
// Layout conversion between the caller's [S][N] arrays and the internal one.
// ---------------------------------------------------------------------------
// mode 0: dst_int = src_ext; 1: dst_int = max(src_ext, 0); 2: dst_ext = src_int
__global__ void k_layout(float* dst, const float* src, NeuronLayout nl, int S, int mode) {
    const long col = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const int c = blockIdx.y;
    if (col >= nl.cols) return;
    const int s = (int)(col / nl.P), p = (int)(col - (long)s * nl.P);
    const long in_ = ((long)c * S + s) * nl.P + p;
    const long ex = (long)s * nl.N + (long)c * nl.P + p;
    if (mode == 0) dst[in_] = src[ex];
    else if (mode == 1) dst[in_] = fmaxf(src[ex], 0.f);
    else dst[ex] = src[in_];
}

// Bits of an internal bit array -> caller [S][N] floats (0/1, mode 0), or
// "value == hi" bits from caller floats (mode 1), or "value >= 0.5" (mode 2),
// or point-box bits lo == hi from internal arrays (mode 3), or bits ->
// caller values hi / lo (mode 4).
struct BitArgs {
    NeuronLayout nl;
    int S;
    int mode;
    uint32_t* bits;
    float* fext;
    const float* hi;   // internal (mode 1)
    const float* lo;   // internal (mode 3)
};

__global__ void k_bits(BitArgs A) {
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
        if (ok) A.fext[ex] = (float)getbit(A.bits, bi);
        return;
    }
    if (A.mode == 4) {
        if (ok) A.fext[ex] = getbit(A.bits, bi) ? A.hi[in_] : A.lo[in_];
        return;
    }
    bool pred = false;
    if (ok) {
        if (A.mode == 1) pred = A.fext[ex] == A.hi[in_];
        else if (A.mode == 2) pred = A.fext[ex] >= 0.5f;
        else pred = A.lo[in_] == A.hi[in_];
    }
    if (col - lane < A.nl.colpad) put_wave_bits(A.bits, (long)c * A.nl.colpad + (col - lane), pred, lane);
}

// Per-subproblem objective: sum of every neuron term (fixed order) plus b_n^T c.
struct ReduceArgs {
    int S;
    int nlayers;                       // neuron layers 0..n-1
    NeuronLayout nl[kMaxLayers];
    const double* term[kMaxLayers];
    const float* cint;                 // objective rows, internal layout [n_last][S]
    const float* bn;
    int n_last;
    double* out;
};

__global__ void __launch_bounds__(256) k_reduce_obj(ReduceArgs A) {
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
        for (int i = 0; i < A.n_last; ++i) acc += (double)A.bn[i] * (double)A.cint[(long)i * A.S + s];
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
struct OracleArgs {
    LayerGeo g;
    int S;
    const float* xprev;
    const float* z;
    const float* lo_in; const float* hi_in;  // internal layout, layer k-1
    uint32_t* bits;
    float* LI; float* UI;
};

__global__ void k_oracle(OracleArgs A) {
    const long gid = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const LayerGeo& g = A.g;
    if (gid >= (long)A.S * g.out.N) return;
    const int s = (int)(gid / g.out.N);
    const long i = gid - (long)s * g.out.N;
    const int c = (int)(i / g.out.P), p = (int)(i - (long)c * g.out.P);
    const float zi = A.z[gid];
    const int F = g.fan, nw = (F + 31) / 32;
    uint32_t word = 0;
    float LI = 0.f, UI = 0.f;
    for (int t = 0; t < F; ++t) {
        const FwdTap tp = fwd_tap(g, A.S, s, p, t);
        bool bit = false;
        if (tp.a >= 0) {
            // caller index of the input neuron
            const long ci = tp.a / ((long)A.S * g.in.P);
            const long pin = tp.a - (ci * A.S + s) * g.in.P;
            const float x = A.xprev[(long)s * g.in.N + ci * g.in.P + pin];
            const float lo = A.lo_in[tp.a], hi = A.hi_in[tp.a];
            const float w = g.W[(long)c * F + t];
            const float Lc = w >= 0 ? lo : hi, Uc = w >= 0 ? hi : lo;
            const float d = (1.f - zi) * Lc + zi * Uc - x;
            bit = (d == 0.f) || (w == 0.f) || ((d > 0.f) == (w > 0.f));
            if (bit) LI = fmaf(w, Lc, LI);
            else UI = fmaf(w, Uc, UI);
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
// Caller layout; lo_in/hi_in are the previous layer's post-activation box
// (for layer 1 the input box; later layers read the pre-activation bounds
// of the previous layer and clamp at 0).
// ---------------------------------------------------------------------------
struct IbpArgs {
    LayerGeo g;
    int S;
    const float* lo_in; const float* hi_in;
    int clamp_in;
    float* lo_out; float* hi_out;
};

__global__ void k_ibp(IbpArgs A) {
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
