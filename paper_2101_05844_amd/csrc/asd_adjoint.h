// Gradient of the dual bound with respect to the network and the input box.
//
// d_B is the minimum over the primal box of the Lagrangian of the relaxation
// in constraint form (App. D), which is linear in (x, z); at fixed duals and
// fixed active sets its minimiser (x*, z*) is a vertex, so (Danskin) the
// gradient of d_B is the Lagrangian's partial derivative at (x*, z*) wherever
// the minimiser is unique.  For ReLU layer k, weight entry (i, j), with
// Lchk = l[j], Uchk = u[j] where W[i,j] >= 0 (swapped where W < 0, Sec. 2.2):
//   dW[i,j] = x*[j] (alpha[i] - beta1[i] - sum_I I[i,j] beta_I[i])
//             + sum_I beta_I[i] ((1 - z*[i]) I[i,j] Lchk - z*[i] (1 - I[i,j]) Uchk)
//   db[i]   = alpha[i] - beta1[i] - z*[i] sum_I beta_I[i]
// and for the last layer dW = c x*^T, db = c.  The input box enters through
// x*_0 (the end chosen by the sign of f_0) and through the check entries of
// layer 1's masks.  The bounds of layers 1..n-1 are held fixed.
//
// Every sum runs in FP64 in a fixed order (the result does not depend on
// scheduling), weighted by the caller's per-subproblem factors g_s: the
// weight and bias gradients are sum_s g_s dd_s/dW, the box gradients g_s
// dd_s/dl0 per subproblem.  Mask entries I[i,j] come from the compact bits
// as in the iteration: I = 1 where z_I[i] = 1, W[i,j] = 0, the box of j is a
// point, or x_I[j] sits at the end minimising W[i,j] x.
#pragma once
#include <hip/hip_runtime.h>

#include "asd_fast.h"
#include "asd_internal.h"

namespace asd {

constexpr int kGradThreads = 256;

template <typename Ts>
struct GradArgs {
    LayerGeo g;                  // layer k (1-based)
    int S;
    int last;                    // k == n
    int nm;                      // active masks of layer k
    const double* gs;            // [S] per-subproblem factors
    const Ts* xin;               // x*_{k-1}, internal layout
    const Ts* lo_in; const Ts* hi_in;
    const uint32_t* deg_in;      // point boxes of layer k-1
    const Ts* cvec;              // last layer: objective rows, internal layout
    const ReluLayerT<Ts>* R;     // layer k arrays (device copy; not last)
    // two-stage reductions: stage one writes part[chunk * entries + e]
    long r_chunk;                // terms (subproblems, or subproblem-positions) per chunk
    long entries;
    double* part;
    // box gradients (layer 1's view of the input)
    const double* f0;            // f_0, internal layout
    double* dl0; double* du0;    // caller layout [S][n_0]
};

__device__ __forceinline__ unsigned gbit(const uint32_t* bits, long bi) {
    return (bits[bi >> 5] >> (bi & 31)) & 1u;
}
__device__ __forceinline__ unsigned gbit(const uint32_t* bits, int bi) {
    return (bits[(unsigned)bi >> 5] >> (bi & 31)) & 1u;
}

// Contribution of mask slot q to entry (i, j) at one term: beta' = g_s beta_I,
// x, the check ends Lc/Uc of j for the sign of W[i,j], z = z*_k[i].
__device__ __forceinline__ double slot_term(bool I, bool z, double bq, double x, double Lc, double Uc) {
    return I ? (z ? -bq * x : bq * (Lc - x)) : (z ? -bq * Uc : 0.0);
}

// Mask entry from the compact bits: z_I of the output, the slot's x bit and
// the point-box bit of the input, the sign of the weight.
__device__ __forceinline__ bool mask_entry(bool zq, float w, bool dg, bool xq) {
    return zq || w == 0.f || dg || (w > 0.f ? !xq : xq);
}

constexpr int kGdTO = 16;              // dense: outputs per block (registers per lane)
constexpr int kGcTO = 4, kGcTT = 4;    // convolution: output channels x taps per block
static_assert(kGcTO * kGcTT <= 32, "the weight-sign masks of a convolution tile are 32-bit");

// Dense layer, stage one.  Lanes run over the inputs j (coalesced reads of
// x*, l, u of layer k-1 and of the weights), each lane keeps kGdTO outputs i
// in registers, the block loops over one chunk of subproblems; the output-side
// values (duals, z bits) are uniform across the block.
template <typename Ts>
__global__ void __launch_bounds__(kGradThreads) k_gw_dense(GradArgs<Ts> A) {
    const cptr_t<ReluLayerT<Ts>> R = kconst_t(A.R);
    const LayerGeo& g = A.g;
    const NeuronLayout& L = g.in;
    const NeuronLayout& O = g.out;
    const int S = A.S;
    const int j = blockIdx.x * kGradThreads + threadIdx.x;
    const int i0 = blockIdx.y * kGdTO;
    const int s0 = (int)(blockIdx.z * A.r_chunk);
    const int s1 = min(S, (int)(s0 + A.r_chunk));
    const bool jok = j < g.fan;
    const int jj = jok ? j : 0;
    const int cj = jj / L.P, pj = jj - cj * L.P;
    const int nto = min(kGdTO, O.C - i0);
    double acc[kGdTO];
    float w[kGdTO];   // only the signs enter the gradient
#pragma unroll
    for (int to = 0; to < kGdTO; ++to) {
        acc[to] = 0;
        w[to] = to < nto ? g.W[(long)(i0 + to) * g.fan + jj] : 0.f;
    }
    for (int s = s0; s < s1; ++s) {
        const long a_in = ((long)cj * S + s) * L.P + pj;
        const double x = (double)A.xin[a_in];
        const double gsv = A.gs[s];
        if (A.last) {
#pragma unroll
            for (int to = 0; to < kGdTO; ++to)
                if (to < nto) acc[to] += gsv * (double)A.cvec[(long)(i0 + to) * S + s] * x;
            continue;
        }
        const long bi = (long)cj * L.colpad + (long)s * L.P + pj;
        const double lo = (double)A.lo_in[a_in], hi = (double)A.hi_in[a_in];
        const bool dg = gbit(A.deg_in, bi);
        unsigned xqb = 0;
        for (int q = 0; q < A.nm; ++q) xqb |= gbit(R->slot[q].xbits, bi) << q;
#pragma unroll
        for (int to = 0; to < kGdTO; ++to) {
            if (to < nto) {
                const long a_out = (long)(i0 + to) * S + s;
                const long bo = (long)(i0 + to) * O.colpad + s;
                const bool z = gbit(R->zbits, bo);
                double t = x * gsv * ((double)R->alpha[a_out] - (double)R->beta1[a_out]);
                const double Lc = w[to] >= 0.f ? lo : hi, Uc = w[to] >= 0.f ? hi : lo;
                for (int q = 0; q < A.nm; ++q) {
                    const double bq = gsv * (double)R->slot[q].beta[a_out];
                    const bool I = mask_entry(gbit(R->slot[q].zbits, bo), w[to], dg, (xqb >> q) & 1u);
                    t += slot_term(I, z, bq, x, Lc, Uc);
                }
                acc[to] += t;
            }
        }
    }
    if (jok)
#pragma unroll
        for (int to = 0; to < kGdTO; ++to)
            if (to < nto) A.part[(long)blockIdx.z * A.entries + (long)(i0 + to) * g.fan + j] = acc[to];
}

// Convolution, stage one.  Lanes run over the (subproblem, output position)
// terms of one chunk (coalesced reads of the output-side duals), each lane
// keeps a tile of kGcTO output channels x kGcTT taps (c_in, ky, kx) in
// registers; the block's partial sums are reduced across lanes (butterfly)
// and waves (fixed order).
template <typename Ts>
__global__ void __launch_bounds__(kGradThreads) k_gw_conv(GradArgs<Ts> A) {
    const cptr_t<ReluLayerT<Ts>> R = kconst_t(A.R);
    __shared__ double red[kGradThreads / 64][kGcTO * kGcTT];
    const LayerGeo& g = A.g;
    const NeuronLayout& L = g.in;
    const NeuronLayout& O = g.out;
    // every neuron and bit index of a layer fits in 31 bits (checked when the
    // workspace is sized), so the addressing below runs in 32-bit integers
    const int S = A.S;
    const int co0 = blockIdx.z * kGcTO;
    const int t0 = blockIdx.y * kGcTT;
    const int r0 = (int)(blockIdx.x * A.r_chunk);
    const int r1 = (int)min((long)S * O.P, (long)r0 + A.r_chunk);
    const int k2 = g.ksz * g.ksz;
    const int nto = min(kGcTO, O.C - co0);
    const int cstride = S * O.P;          // channel stride of the output layout
    const int ocp = (int)O.colpad, icp = (int)L.colpad;
    // only the signs of the tile's weights enter the gradient: bit to*kGcTT+tt
    uint32_t wpos = 0, wzero = 0, wnonneg = 0;
    int ci[kGcTT], dy[kGcTT], dx[kGcTT];
    bool tok[kGcTT];
#pragma unroll
    for (int tt = 0; tt < kGcTT; ++tt) {
        const int t = t0 + tt;
        tok[tt] = t < g.fan;
        const int tc = tok[tt] ? t : 0;
        ci[tt] = tc / k2;
        const int rem = tc - ci[tt] * k2;
        dy[tt] = rem / g.ksz - g.pad;
        dx[tt] = rem - (rem / g.ksz) * g.ksz - g.pad;
#pragma unroll
        for (int to = 0; to < kGcTO; ++to) {
            const float wv = (to < nto && tok[tt]) ? g.W[(co0 + to) * g.fan + tc] : 0.f;
            const uint32_t bit = 1u << (to * kGcTT + tt);
            if (wv > 0.f) wpos |= bit;
            if (wv == 0.f) wzero |= bit;
            if (wv >= 0.f) wnonneg |= bit;
        }
    }
    double acc[kGcTO][kGcTT];
#pragma unroll
    for (int to = 0; to < kGcTO; ++to)
#pragma unroll
        for (int tt = 0; tt < kGcTT; ++tt) acc[to][tt] = 0;
    for (int r = r0 + (int)threadIdx.x; r < r1; r += kGradThreads) {
        const int s = r / O.P, p = r - s * O.P;
        const int oy = p / O.W, ox = p - oy * O.W;
        const double gsv = A.gs[s];
        const int a0 = co0 * cstride + r;   // output (co0, s, p)
        const int b0 = co0 * ocp + r;
        double x[kGcTT], lo[kGcTT], hi[kGcTT];
        int ain[kGcTT], bin[kGcTT];
        unsigned okb = 0, dgb = 0;
#pragma unroll
        for (int tt = 0; tt < kGcTT; ++tt) {
            const int iy = oy * g.stride + dy[tt], ix = ox * g.stride + dx[tt];
            const bool ok = tok[tt] && iy >= 0 && iy < L.H && ix >= 0 && ix < L.W;
            const int pin = ok ? iy * L.W + ix : 0;
            ain[tt] = (ci[tt] * S + s) * L.P + pin;
            bin[tt] = ci[tt] * icp + s * L.P + pin;
            x[tt] = ok ? (double)A.xin[ain[tt]] : 0.0;
            lo[tt] = ok ? (double)A.lo_in[ain[tt]] : 0.0;
            hi[tt] = ok ? (double)A.hi_in[ain[tt]] : 0.0;
            okb |= (unsigned)ok << tt;
            if (ok) dgb |= gbit(A.deg_in, bin[tt]) << tt;
        }
        unsigned zb = 0;
#pragma unroll
        for (int to = 0; to < kGcTO; ++to) {
            if (to < nto) {
                const int a = a0 + to * cstride;
                zb |= gbit(R->zbits, b0 + to * ocp) << to;
                const double Av = gsv * ((double)R->alpha[a] - (double)R->beta1[a]);
#pragma unroll
                for (int tt = 0; tt < kGcTT; ++tt) acc[to][tt] += x[tt] * Av;
            }
        }
        for (int q = 0; q < A.nm; ++q) {
            const cptr_t<MaskSlotT<Ts>> M = &R->slot[q];
            const uint32_t* xbits = M->xbits;
            unsigned xqb = 0;
#pragma unroll
            for (int tt = 0; tt < kGcTT; ++tt)
                if ((okb >> tt) & 1u) xqb |= gbit(xbits, bin[tt]) << tt;
            const Ts* beta = M->beta;
            const uint32_t* zbits = M->zbits;
#pragma unroll
            for (int to = 0; to < kGcTO; ++to) {
                if (to < nto) {
                    const double bq = gsv * (double)beta[a0 + to * cstride];
                    const bool zq = gbit(zbits, b0 + to * ocp);
                    const bool z = (zb >> to) & 1u;
#pragma unroll
                    for (int tt = 0; tt < kGcTT; ++tt) {
                        const int e = to * kGcTT + tt;
                        const bool xq = (xqb >> tt) & 1u;
                        const bool I = zq || ((wzero >> e) & 1u) || ((dgb >> tt) & 1u) ||
                                       (((wpos >> e) & 1u) ? !xq : xq);
                        const bool nn = (wnonneg >> e) & 1u;
                        const double t = slot_term(I, z, bq, x[tt], nn ? lo[tt] : hi[tt], nn ? hi[tt] : lo[tt]);
                        if ((okb >> tt) & 1u) acc[to][tt] += t;
                    }
                }
            }
        }
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int to = 0; to < kGcTO; ++to)
#pragma unroll
        for (int tt = 0; tt < kGcTT; ++tt) {
            double v = acc[to][tt];
#pragma unroll
            for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
            if (lane == 0) red[wave][to * kGcTT + tt] = v;
        }
    __syncthreads();
    if ((int)threadIdx.x < kGcTO * kGcTT) {
        const int to = threadIdx.x / kGcTT, tt = threadIdx.x - to * kGcTT;
        double v = 0;
        for (int wv = 0; wv < kGradThreads / 64; ++wv) v += red[wv][threadIdx.x];
        if (to < nto && tok[tt]) A.part[(long)blockIdx.x * A.entries + (long)(co0 + to) * g.fan + t0 + tt] = v;
    }
}

// Bias, stage one: block (chunk, channel), fixed-order block sum.
template <typename Ts>
__global__ void __launch_bounds__(kGradThreads) k_gb_part(GradArgs<Ts> A) {
    const cptr_t<ReluLayerT<Ts>> R = kconst_t(A.R);
    __shared__ double red[kGradThreads];
    const NeuronLayout& O = A.g.out;
    const int co = blockIdx.y;
    const int S = A.S;
    const long r0 = (long)blockIdx.x * A.r_chunk;
    const long r1 = min((long)S * O.P, r0 + A.r_chunk);
    double acc = 0;
    for (long r = r0 + threadIdx.x; r < r1; r += kGradThreads) {
        const int s = (int)(r / O.P);
        const long a_out = (long)co * S * O.P + r;
        double t;
        if (A.last) {
            t = (double)A.cvec[a_out];
        } else {
            t = (double)R->alpha[a_out] - (double)R->beta1[a_out];
            if (gbit(R->zbits, (long)co * O.colpad + r))
                for (int q = 0; q < A.nm; ++q) t -= (double)R->slot[q].beta[a_out];
        }
        acc += A.gs[s] * t;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = kGradThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) A.part[(long)blockIdx.x * A.entries + co] = red[0];
}

// Stage two: out[e] = sum over chunks of part[chunk * entries + e], in chunk order.
static __global__ void __launch_bounds__(kGradThreads) k_gsum(const double* part, long entries, int chunks, double* out) {
    const long e = (long)blockIdx.x * kGradThreads + threadIdx.x;
    if (e >= entries) return;
    double v = 0;
    for (int c = 0; c < chunks; ++c) v += part[(long)c * entries + e];
    out[e] = v;
}

// One thread per input neuron and subproblem (internal layout of layer 0).
// A = layer 1's arguments (R, nm, g) with the box pointers of layer 0.
template <typename Ts>
__global__ void __launch_bounds__(kGradThreads) k_grad_box(GradArgs<Ts> A) {
    const cptr_t<ReluLayerT<Ts>> R = kconst_t(A.R);
    const LayerGeo& g = A.g;
    const NeuronLayout& L = g.in;
    const NeuronLayout& O = g.out;
    const int S = A.S;
    const long gid = (long)blockIdx.x * kGradThreads + threadIdx.x;
    if (gid >= (long)L.C * L.cols) return;
    const int c = (int)(gid / L.cols);
    const long col = gid - (long)c * L.cols;
    const int s = (int)(col / L.P), p = (int)(col - (long)s * L.P);
    const double f = A.f0[gid];
    double dl = f < 0 ? -f : 0.0;
    double du = f >= 0 ? -f : 0.0;
    if (!A.last && A.nm > 0) {
        const long bi = (long)c * L.colpad + col;
        const bool dg = gbit(A.deg_in, bi);
        // the x bits of every mask slot at this input (the same for all the
        // outputs that read it)
        static_assert(kMaxMasks <= 32, "x bits of the mask slots are kept in one word");
        unsigned xqb = 0;
        for (int q = 0; q < A.nm; ++q) xqb |= gbit(R->slot[q].xbits, bi) << q;
        // contribution of one layer-1 output (neuron address a_out, bit bo)
        // reading this input with weight w
        auto add = [&](double w, long a_out, long bo) {
            const bool z = gbit(R->zbits, bo);
            for (int q = 0; q < A.nm; ++q) {
                const double bq = (double)R->slot[q].beta[a_out];
                const bool zq = gbit(R->slot[q].zbits, bo);
                const bool xq = (xqb >> q) & 1u;
                const bool I = zq || w == 0 || dg || (w > 0 ? !xq : xq);
                // I: Lchk term (1 - z) w, on l where w >= 0 and on u where w < 0;
                // not I: Uchk term -z w, on u where w >= 0 and on l where w < 0
                if (I) {
                    if (!z) {
                        if (w >= 0) dl += bq * w;
                        else du += bq * w;
                    }
                } else if (z) {
                    if (w >= 0) du -= bq * w;
                    else dl -= bq * w;
                }
            }
        };
        if (g.kind == ASD_LAYER_DENSE) {
            const int j = c * L.P + p;
            for (int i = 0; i < O.C; ++i) add((double)g.W[(long)i * g.fan + j], (long)i * S + s, (long)i * O.colpad + s);
        } else {
            const int y = p / L.W, x = p - (p / L.W) * L.W;
            const int ks = g.ksz, str = g.stride;
            const int ky0 = (y + g.pad) % str, kx0 = (x + g.pad) % str;
            for (int co = 0; co < O.C; ++co)
                for (int ky = ky0; ky < ks; ky += str) {
                    const int oy = (y + g.pad - ky) / str;
                    if (oy < 0 || oy >= O.H) continue;
                    for (int kx = kx0; kx < ks; kx += str) {
                        const int ox = (x + g.pad - kx) / str;
                        if (ox < 0 || ox >= O.W) continue;
                        const int op = oy * O.W + ox;
                        add((double)g.W[(((long)co * L.C + c) * ks + ky) * ks + kx], ((long)co * S + s) * O.P + op,
                            (long)co * O.colpad + (long)s * O.P + op);
                    }
                }
        }
    }
    const double gsv = A.gs[s];
    const long ex = (long)s * L.N + (long)c * L.P + p;
    if (A.dl0) A.dl0[ex] = gsv * dl;
    if (A.du0) A.du0[ex] = gsv * du;
}

}  // namespace asd
