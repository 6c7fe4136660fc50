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
    ReluLayerT<Ts> R;            // layer k arrays (not last)
    double* out;                 // dW (flattened weight tensor) or db [C_out]
    // box gradients (layer 1's view of the input)
    const double* f0;            // f_0, internal layout
    double* dl0; double* du0;    // caller layout [S][n_0]
};

__device__ __forceinline__ unsigned gbit(const uint32_t* bits, long bi) {
    return (bits[bi >> 5] >> (bi & 31)) & 1u;
}

// Fixed-order block sum of one double per thread; the result is valid in
// thread 0.
__device__ __forceinline__ double block_sum(double v, double* red) {
    red[threadIdx.x] = v;
    __syncthreads();
    for (int w = kGradThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    return red[0];
}

// Per-term mask contribution of entry (i, j) at one subproblem: the part of
// dW[i,j] that involves beta_I, for every active slot.
template <typename Ts>
__device__ __forceinline__ double mask_terms(const ReluLayerT<Ts>& R, int nm, long a_out, long bo, long bi,
                                             double w, double x, double lo, double hi, bool z, bool dg) {
    const double Lchk = w >= 0 ? lo : hi, Uchk = w >= 0 ? hi : lo;
    double t = 0;
    for (int q = 0; q < nm; ++q) {
        const double bq = (double)R.slot[q].beta[a_out];
        const bool zq = gbit(R.slot[q].zbits, bo);
        const bool xq = gbit(R.slot[q].xbits, bi);
        const bool I = zq || w == 0 || dg || (w > 0 ? !xq : xq);
        if (I) t += bq * (z ? -x : Lchk - x);
        else if (z) t -= bq * Uchk;
    }
    return t;
}

// One block per weight entry; the threads stride over the (subproblem,
// output position) pairs the entry is used at.
template <typename Ts>
__global__ void __launch_bounds__(kGradThreads) k_grad_weight(GradArgs<Ts> A) {
    __shared__ double red[kGradThreads];
    const LayerGeo& g = A.g;
    const NeuronLayout& L = g.in;
    const NeuronLayout& O = g.out;
    const long e = blockIdx.x;
    const int S = A.S;
    int co, ci = 0, pj = 0, ky = 0, kx = 0;
    if (g.kind == ASD_LAYER_DENSE) {
        co = (int)(e / g.fan);
        const int j = (int)(e - (long)co * g.fan);
        ci = j / L.P;
        pj = j - ci * L.P;
    } else {
        const int k2 = g.ksz * g.ksz;
        co = (int)(e / ((long)L.C * k2));
        const int rem = (int)(e - (long)co * L.C * k2);
        ci = rem / k2;
        ky = (rem - ci * k2) / g.ksz;
        kx = rem - ci * k2 - ky * g.ksz;
    }
    const double w = (double)g.W[e];
    double acc = 0;
    const long R = (long)S * O.P;
    for (long r = threadIdx.x; r < R; r += kGradThreads) {
        const int s = (int)(r / O.P), p = (int)(r - (long)s * O.P);
        int pin;
        if (g.kind == ASD_LAYER_DENSE) {
            pin = pj;
        } else {
            const int oy = p / O.W, ox = p - oy * O.W;
            const int iy = oy * g.stride - g.pad + ky, ix = ox * g.stride - g.pad + kx;
            if (iy < 0 || iy >= L.H || ix < 0 || ix >= L.W) continue;  // padding tap: no entry
            pin = iy * L.W + ix;
        }
        const long a_in = ((long)ci * S + s) * L.P + pin;
        const long bi = (long)ci * L.colpad + (long)s * L.P + pin;
        const long a_out = ((long)co * S + s) * O.P + p;
        const double x = (double)A.xin[a_in];
        double t;
        if (A.last) {
            t = (double)A.cvec[a_out] * x;
        } else {
            const long bo = (long)co * O.colpad + r;
            t = x * ((double)A.R.alpha[a_out] - (double)A.R.beta1[a_out]);
            if (A.nm > 0)
                t += mask_terms(A.R, A.nm, a_out, bo, bi, w, x, (double)A.lo_in[a_in], (double)A.hi_in[a_in],
                                gbit(A.R.zbits, bo), gbit(A.deg_in, bi));
        }
        acc += A.gs[s] * t;
    }
    const double tot = block_sum(acc, red);
    if (threadIdx.x == 0) A.out[e] = tot;
}

// One block per output channel.
template <typename Ts>
__global__ void __launch_bounds__(kGradThreads) k_grad_bias(GradArgs<Ts> A) {
    __shared__ double red[kGradThreads];
    const NeuronLayout& O = A.g.out;
    const int co = blockIdx.x;
    const int S = A.S;
    double acc = 0;
    const long R = (long)S * O.P;
    for (long r = threadIdx.x; r < R; r += kGradThreads) {
        const int s = (int)(r / O.P);
        const long a_out = (long)co * S * O.P + r;
        double t;
        if (A.last) {
            t = (double)A.cvec[a_out];
        } else {
            t = (double)A.R.alpha[a_out] - (double)A.R.beta1[a_out];
            if (gbit(A.R.zbits, (long)co * O.colpad + r))
                for (int q = 0; q < A.nm; ++q) t -= (double)A.R.slot[q].beta[a_out];
        }
        acc += A.gs[s] * t;
    }
    const double tot = block_sum(acc, red);
    if (threadIdx.x == 0) A.out[co] = tot;
}

// One thread per input neuron and subproblem (internal layout of layer 0).
// A = layer 1's arguments (R, nm, g) with the box pointers of layer 0.
template <typename Ts>
__global__ void __launch_bounds__(kGradThreads) k_grad_box(GradArgs<Ts> A) {
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
        // contribution of one layer-1 output (neuron address a_out, bit bo)
        // reading this input with weight w
        auto add = [&](double w, long a_out, long bo) {
            const bool z = gbit(A.R.zbits, bo);
            for (int q = 0; q < A.nm; ++q) {
                const double bq = (double)A.R.slot[q].beta[a_out];
                const bool zq = gbit(A.R.slot[q].zbits, bo);
                const bool xq = gbit(A.R.slot[q].xbits, bi);
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
