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

constexpr int kGdTO = 16;              // last dense layer: outputs per block (registers per lane)

// Last (dense) layer, stage one: dW = sum_s g_s c_s x*_s^T.  Lanes run over
// the inputs j (coalesced reads of x*), each lane keeps kGdTO outputs i in
// registers, the block loops over one chunk of subproblems.
template <typename Ts>
__global__ void __launch_bounds__(kGradThreads) k_gw_last(GradArgs<Ts> A) {
    const LayerGeo& g = A.g;
    const NeuronLayout& L = g.in;
    const int S = A.S;
    const int j = blockIdx.x * kGradThreads + threadIdx.x;
    const int i0 = blockIdx.y * kGdTO;
    const int s0 = (int)(blockIdx.z * A.r_chunk);
    const int s1 = min(S, (int)(s0 + A.r_chunk));
    const bool jok = j < g.fan;
    const int jj = jok ? j : 0;
    const int cj = jj / L.P, pj = jj - cj * L.P;
    const int nto = min(kGdTO, g.out.C - i0);
    double acc[kGdTO];
#pragma unroll
    for (int to = 0; to < kGdTO; ++to) acc[to] = 0;
    for (int s = s0; s < s1; ++s) {
        const double x = (double)A.xin[((long)cj * S + s) * L.P + pj];
        const double gsv = A.gs[s];
#pragma unroll
        for (int to = 0; to < kGdTO; ++to)
            if (to < nto) acc[to] += gsv * (double)A.cvec[(long)(i0 + to) * S + s] * x;
    }
    if (jok)
#pragma unroll
        for (int to = 0; to < kGdTO; ++to)
            if (to < nto) A.part[(long)blockIdx.z * A.entries + (long)(i0 + to) * g.fan + j] = acc[to];
}

// ---------------------------------------------------------------------------
// Weight gradient of a ReLU layer k, in sign classes.
//
// Sum the slot terms of one (output o, input j) pair over the masks q, with
// b_q = g_s beta_q[o], I_q = z_q[o] | d_q[j] where d_q[j] = 1 on a point box
// of j, else the x bit test of the weight's sign class (w > 0: x not at the
// upper end; w < 0: x at the upper end; w = 0: always 1):
//   z[o] = 0:  sum_q = (Lc - x) PD          PD = sum_q I_q b_q
//   z[o] = 1:  sum_q = (Uc - x) PD - Uc B   B = sum_q b_q
// and with P = sum_{z_q} b_q, Q_q = (1 - z_q) b_q, X0 = sum_q xbit_q Q_q
// (x bits cleared on a point box):  PD = B - X0 (w > 0), P + X0 (w < 0, no
// point box), B (w = 0 or a point box).  Adding x (alpha - beta_1) g_s, the
// whole pair term is
//   x Ax + (c - x) (PD - [z] B),   Ax = g_s (alpha - beta_1) - [z] B,
// c = Lc (z = 0) or Uc (z = 1), where (Lc, Uc) = (l, u) for w >= 0 and (u, l)
// for w < 0.  Per pair that is one fused multiply-add per mask plus six, and
// the weight's class enters through two per-lane constants: the coefficient
// of X0 (-1, 0, +1) and 2 [w < 0] (which picks P over B, and c's end).
//
// Mapping: each lane owns TT taps (input positions of the receptive field,
// fan index t = block tap base + lane + 64 tt) of TO output channels; a wave
// walks the terms (subproblem, output position) of its share one at a time,
// so the output-side values of a term are the same for all its lanes.  They
// are formed once per (channel, term) by the block into LDS (records of
// Ax, [z ? 0 : B], P - B, [z ? -1 : 1], Q_q); the input side is one record
// per neuron (x, l, u, bits), gathered per lane.  Block partial sums are
// added across the waves in a fixed order and written per chunk of terms.

// Input-side record of one neuron of layer k-1 for the weight gradient of
// ReLU layer k: its value at the minimiser, its box, and bits (bit 0: point
// box; bit 1 + q: x bit of mask slot q of layer k, cleared on a point box).
template <typename Ts> struct GwIn;
template <> struct __align__(16) GwIn<float> { float x, l, u; uint32_t bits; };
template <> struct __align__(16) GwIn<double> { double x, l, u; uint32_t bits, pad; };

template <typename Ts>
__global__ void __launch_bounds__(kGradThreads) k_gw_in(GradArgs<Ts> A, GwIn<Ts>* out) {
    const cptr_t<ReluLayerT<Ts>> R = kconst_t(A.R);
    const NeuronLayout& L = A.g.in;
    const long gid = (long)blockIdx.x * kGradThreads + threadIdx.x;
    if (gid >= (long)L.C * L.cols) return;
    const int c = (int)(gid / L.cols);
    const long bi = (long)c * L.colpad + (gid - (long)c * L.cols);
    const unsigned dg = gbit(A.deg_in, bi);
    unsigned bits = dg;
    if (!dg)
        for (int q = 0; q < A.nm; ++q) bits |= gbit(R->slot[q].xbits, bi) << (1 + q);
    GwIn<Ts> r;
    r.x = A.xin[gid];
    r.l = A.lo_in[gid];
    r.u = A.hi_in[gid];
    r.bits = bits;
    out[gid] = r;
}

constexpr int kGwRB = 64;   // terms per LDS batch (16 per wave)

template <typename Ts>
struct GwArgs {
    int S, fan, kh, kw, stride, pad;
    int inH, inW, inP;           // layer k-1 spatial size
    int outC, outH, outW, outP;  // layer k
    long outcols, outcolpad;     // S * outP, and the bit stride of a channel
    const float* W;              // [outC][fan]
    const double* gs;            // [S]
    const GwIn<Ts>* in;          // records of layer k-1 (internal layout)
    const ReluLayerT<Ts>* R;     // layer k (device copy)
    long r_chunk;                // terms per block (a multiple of kGwRB)
    long entries;                // outC * fan
    double* part;                // [chunk][entries]
};

template <typename Ts, int NM, int TO, int TT>
__global__ void __launch_bounds__(kGradThreads) k_gw_relu(GwArgs<Ts> A) {
    constexpr int RL = 4 + NM;                 // Ax, Bz, P - B, zs, Q_0 .. Q_{NM-1}
    constexpr int RLP = (RL + 1) & ~1;         // 16-byte aligned records
    constexpr int SLOT = RLP > TT ? RLP : TT;
    __shared__ __align__(16) double lds[TO * kGwRB * SLOT];
    const cptr_t<ReluLayerT<Ts>> R = kconst_t(A.R);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int co0 = blockIdx.z * TO;
    const int tb = blockIdx.y * (64 * TT);
    const long nterms = (long)A.S * A.outP;
    const long r0 = (long)blockIdx.x * A.r_chunk;
    const long r1 = min(nterms, r0 + A.r_chunk);
    const int khw = A.kh * A.kw;
    // the lane's taps: input offsets (before the term's) and weight classes
    int off[TT], dy[TT], dx[TT];
    bool tok[TT];
    double sg[TT][TO], ng[TT][TO];
#pragma unroll
    for (int tt = 0; tt < TT; ++tt) {
        const int t = tb + lane + 64 * tt;
        tok[tt] = t < A.fan;
        const int tc = tok[tt] ? t : 0;
        const int ci = tc / khw, rem = tc - ci * khw;
        const int ky = rem / A.kw, kx = rem - (rem / A.kw) * A.kw;
        dy[tt] = ky - A.pad;
        dx[tt] = kx - A.pad;
        off[tt] = ci * A.S * A.inP + dy[tt] * A.inW + dx[tt];
#pragma unroll
        for (int to = 0; to < TO; ++to) {
            const float w = (tok[tt] && co0 + to < A.outC) ? A.W[(long)(co0 + to) * A.fan + tc] : 0.f;
            sg[tt][to] = w > 0.f ? -1.0 : (w < 0.f ? 1.0 : 0.0);
            ng[tt][to] = w < 0.f ? 2.0 : 0.0;
        }
    }
    double acc[TT][TO];
#pragma unroll
    for (int tt = 0; tt < TT; ++tt)
#pragma unroll
        for (int to = 0; to < TO; ++to) acc[tt][to] = 0;
    for (long rb = r0; rb < r1; rb += kGwRB) {
        __syncthreads();
        for (int e = threadIdx.x; e < TO * kGwRB; e += kGradThreads) {
            const int to = e / kGwRB, rl = e - (e / kGwRB) * kGwRB;
            const long r = rb + rl;
            const int co = co0 + to;
            double rec[RLP];
#pragma unroll
            for (int i = 0; i < RLP; ++i) rec[i] = 0;
            rec[3] = 1.0;
            if (r < r1 && co < A.outC) {
                const int s = (int)(r / A.outP);
                const long a = (long)co * A.outcols + r;
                const long bo = (long)co * A.outcolpad + r;
                const double gsv = A.gs[s];
                const bool z = gbit(R->zbits, bo);
                const double Av = gsv * ((double)R->alpha[a] - (double)R->beta1[a]);
                double B = 0, PmB = 0;
#pragma unroll
                for (int q = 0; q < NM; ++q) {
                    const double bq = gsv * (double)R->slot[q].beta[a];
                    B += bq;
                    if (!gbit(R->slot[q].zbits, bo)) {
                        rec[4 + q] = bq;
                        PmB -= bq;
                    }
                }
                rec[0] = z ? Av - B : Av;
                rec[1] = z ? 0.0 : B;
                rec[2] = PmB;
                rec[3] = z ? -1.0 : 1.0;
            }
            double* d = &lds[(to * kGwRB + rl) * RLP];
#pragma unroll
            for (int i = 0; i < RLP; ++i) d[i] = rec[i];
        }
        __syncthreads();
        const long rw = rb + wave * (kGwRB / 4);
        const long rwe = min(r1, rw + kGwRB / 4);
        if (rw >= rwe) continue;
        // the wave's terms in order: (s, oy, ox) stepped, the next term's input
        // records loaded while this one is processed
        int s = (int)(rw / A.outP);
        int oy, ox;
        {
            const int p = (int)(rw - (long)s * A.outP);
            oy = p / A.outW;
            ox = p - oy * A.outW;
        }
        GwIn<Ts> cur[TT];
        auto fetch = [&](int s_, int oy_, int ox_, GwIn<Ts>* v) {
            const int iy0 = oy_ * A.stride, ix0 = ox_ * A.stride;
            const int base = s_ * A.inP + iy0 * A.inW + ix0;
#pragma unroll
            for (int tt = 0; tt < TT; ++tt) {
                const int iy = iy0 + dy[tt], ix = ix0 + dx[tt];
                const bool ok = tok[tt] && (unsigned)iy < (unsigned)A.inH && (unsigned)ix < (unsigned)A.inW;
                if (ok) {
                    v[tt] = A.in[off[tt] + base];
                } else {
                    v[tt].x = v[tt].l = v[tt].u = 0;
                    v[tt].bits = 0;
                }
            }
        };
        fetch(s, oy, ox, cur);
        for (long r = rw; r < rwe; ++r) {
            int s2 = s, oy2 = oy, ox2 = ox + 1;
            if (ox2 == A.outW) {
                ox2 = 0;
                if (++oy2 == A.outH) {
                    oy2 = 0;
                    ++s2;
                }
            }
            GwIn<Ts> nxt[TT];
            if (r + 1 < rwe) {
                fetch(s2, oy2, ox2, nxt);
            } else {
#pragma unroll
                for (int tt = 0; tt < TT; ++tt) {
                    nxt[tt].x = nxt[tt].l = nxt[tt].u = 0;
                    nxt[tt].bits = 0;
                }
            }
            double xd[TT], mm[TT], hm[TT], hn[TT], dq[TT][NM > 0 ? NM : 1];
#pragma unroll
            for (int tt = 0; tt < TT; ++tt) {
                const GwIn<Ts>& v = cur[tt];
                const double x = (double)v.x, l = (double)v.l, u = (double)v.u;
                xd[tt] = x;
                mm[tt] = 0.5 * (l + u) - x;
                hm[tt] = 0.5 * (u - l);
                hn[tt] = (v.bits & 1u) ? 0.0 : 0.5;
#pragma unroll
                for (int q = 0; q < NM; ++q) dq[tt][q] = ((v.bits >> (1 + q)) & 1u) ? 1.0 : 0.0;
            }
            const int rl = (int)(r - rb);
#pragma unroll
            for (int to = 0; to < TO; ++to) {
                const double* d = &lds[(to * kGwRB + rl) * RLP];
                double rec[RLP];
#pragma unroll
                for (int i = 0; i < RLP; ++i) rec[i] = d[i];
#pragma unroll
                for (int tt = 0; tt < TT; ++tt) {
                    double X = 0;
                    if constexpr (NM > 0) {
                        X = dq[tt][0] * rec[4];
#pragma unroll
                        for (int q = 1; q < NM; ++q) X = fma(dq[tt][q], rec[4 + q], X);
                    }
                    const double bse = fma(ng[tt][to] * hn[tt], rec[2], rec[1]);
                    const double PD = fma(sg[tt][to], X, bse);
                    const double cmx = fma(fma(ng[tt][to], rec[3], -rec[3]), hm[tt], mm[tt]);
                    acc[tt][to] = fma(xd[tt], rec[0], acc[tt][to]);
                    acc[tt][to] = fma(cmx, PD, acc[tt][to]);
                }
            }
#pragma unroll
            for (int tt = 0; tt < TT; ++tt) cur[tt] = nxt[tt];
            s = s2;
            oy = oy2;
            ox = ox2;
        }
    }
    // waves 0 + 1 + 2 + 3, in that order
    for (int w = 1; w < 4; ++w) {
        __syncthreads();
        if (wave == w)
#pragma unroll
            for (int tt = 0; tt < TT; ++tt)
#pragma unroll
                for (int to = 0; to < TO; ++to) lds[(tt * TO + to) * 64 + lane] = acc[tt][to];
        __syncthreads();
        if (wave == 0)
#pragma unroll
            for (int tt = 0; tt < TT; ++tt)
#pragma unroll
                for (int to = 0; to < TO; ++to) acc[tt][to] += lds[(tt * TO + to) * 64 + lane];
    }
    if (wave == 0)
#pragma unroll
        for (int tt = 0; tt < TT; ++tt)
#pragma unroll
            for (int to = 0; to < TO; ++to)
                if (tok[tt] && co0 + to < A.outC)
                    A.part[(long)blockIdx.x * A.entries + (long)(co0 + to) * A.fan + tb + lane + 64 * tt] =
                        acc[tt][to];
}

// Box gradient through layer 1 in sign classes, one block per (chunk of
// kGbNI x 256 inputs, subproblem s).  Per (layer-1 output o, input j) with
// weight w and b_q = beta_q[o] (g_s applies at the end), the mask terms of
// k_grad_box (one per slot) add up to t = PD' w with PD' = PD - [z] B as in
// the weight gradient; t goes to dl[j] where (w >= 0) == (z = 0) and to
// du[j] otherwise (w = 0 gives t = 0).  Lanes keep dl + du and dl - du (the sign
// of a pair is [w >= 0 ? 1 : -1] [z ? -1 : 1]); the block stages the records
// (Bz, P - B, zs, Q_q) of a range of whole output channels of s in LDS, and
// the convolution's weights.
constexpr int kGbNI = 4;    // inputs per lane

template <typename Ts, int NM, bool DENSE>
__global__ void __launch_bounds__(kGradThreads) k_grad_box_sc(GradArgs<Ts> A, int NC) {
    constexpr int RL = 3 + NM;                 // Bz, P - B, zs, Q_0 .. Q_{NM-1}
    constexpr int RLP = (RL + 1) & ~1;
    // record stride: an odd number of 16-byte units, so that neighbouring
    // outputs read by one wave fall in different LDS banks
    constexpr int RLS = (RLP / 2) % 2 ? RLP : RLP + 2;
    extern __shared__ __align__(16) double lds_box[];
    const cptr_t<ReluLayerT<Ts>> R = kconst_t(A.R);
    const LayerGeo& g = A.g;
    const NeuronLayout& L = g.in;
    const NeuronLayout& O = g.out;
    const int S = A.S;
    const int s = blockIdx.y;
    const int jb = blockIdx.x * kGradThreads * kGbNI + threadIdx.x;
    double* rec = lds_box;
    float* wl = reinterpret_cast<float*>(lds_box + (size_t)NC * O.P * RLS);
    const int ks = g.ksz, str = g.stride;
    if (!DENSE) {
        for (int e = threadIdx.x; e < O.C * g.fan; e += kGradThreads) wl[e] = g.W[e];
    }
    double sacc[kGbNI], dacc[kGbNI];
    uint32_t xb[kGbNI];
#pragma unroll
    for (int i = 0; i < kGbNI; ++i) {
        sacc[i] = dacc[i] = 0;
        xb[i] = 0;
        const int j = jb + kGradThreads * i;
        if (j < L.N) {
            const int c = j / L.P, p = j - (j / L.P) * L.P;
            const long bi = (long)c * L.colpad + (long)s * L.P + p;
            const unsigned dg = gbit(A.deg_in, bi);
            unsigned b = dg;
            if (!dg)
#pragma unroll
                for (int q = 0; q < NM; ++q) b |= gbit(R->slot[q].xbits, bi) << (1 + q);
            xb[i] = b;
        }
    }
    for (int c0 = 0; c0 < O.C; c0 += NC) {
        const int nc = min(NC, O.C - c0);
        __syncthreads();
        for (int o = threadIdx.x; o < nc * O.P; o += kGradThreads) {
            const int co = c0 + o / O.P, op = o - (o / O.P) * O.P;
            const long a = ((long)co * S + s) * O.P + op;
            const long bo = (long)co * O.colpad + (long)s * O.P + op;
            const bool z = gbit(R->zbits, bo);
            double r[RLP];
#pragma unroll
            for (int i = 0; i < RLP; ++i) r[i] = 0;
            double B = 0, PmB = 0;
#pragma unroll
            for (int q = 0; q < NM; ++q) {
                const double bq = (double)R->slot[q].beta[a];
                B += bq;
                if (!gbit(R->slot[q].zbits, bo)) {
                    r[3 + q] = bq;
                    PmB -= bq;
                }
            }
            r[0] = z ? 0.0 : B;
            r[1] = PmB;
            r[2] = z ? -1.0 : 1.0;
#pragma unroll
            for (int i = 0; i < RLP; ++i) rec[(size_t)o * RLS + i] = r[i];
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < kGbNI; ++i) {
            const int j = jb + kGradThreads * i;
            if (j >= L.N) continue;
            double dq[NM > 0 ? NM : 1];
#pragma unroll
            for (int q = 0; q < NM; ++q) dq[q] = ((xb[i] >> (1 + q)) & 1u) ? 1.0 : 0.0;
            const double hn = (xb[i] & 1u) ? 0.0 : 0.5;
            // one (output record, weight) pair
            auto pair = [&](const double* r, float wf) {
                const double w = (double)wf;
                double X = 0;
                if constexpr (NM > 0) {
                    X = dq[0] * r[3];
#pragma unroll
                    for (int q = 1; q < NM; ++q) X = fma(dq[q], r[3 + q], X);
                }
                const double ng = wf < 0.f ? 2.0 : 0.0;
                const double sg = wf > 0.f ? -1.0 : (wf < 0.f ? 1.0 : 0.0);
                const double PD = fma(sg, X, fma(ng * hn, r[1], r[0]));
                const double t = PD * w;
                sacc[i] += t;
                dacc[i] = fma((1.0 - ng) * r[2], t, dacc[i]);
            };
            if (DENSE) {
                for (int co = c0; co < c0 + nc; ++co) pair(&rec[(size_t)(co - c0) * RLS], g.W[(long)co * g.fan + j]);
            } else {
                const int c = j / L.P, p = j - (j / L.P) * L.P;
                const int y = p / L.W, x = p - (p / L.W) * L.W;
                const int ky0 = (y + g.pad) % str, kx0 = (x + g.pad) % str;
                for (int co = c0; co < c0 + nc; ++co)
                    for (int ky = ky0; ky < ks; ky += str) {
                        const int oy = (y + g.pad - ky) / str;
                        if (oy < 0 || oy >= O.H) continue;
                        for (int kx = kx0; kx < ks; kx += str) {
                            const int ox = (x + g.pad - kx) / str;
                            if (ox < 0 || ox >= O.W) continue;
                            pair(&rec[((size_t)(co - c0) * O.P + oy * O.W + ox) * RLS],
                                 wl[((co * L.C + c) * ks + ky) * ks + kx]);
                        }
                    }
            }
        }
    }
    const double gsv = A.gs[s];
#pragma unroll
    for (int i = 0; i < kGbNI; ++i) {
        const int j = jb + kGradThreads * i;
        if (j >= L.N) continue;
        const int c = j / L.P, p = j - (j / L.P) * L.P;
        const double f = A.f0[((long)c * S + s) * L.P + p];
        const double dl = 0.5 * (sacc[i] + dacc[i]) + (f < 0 ? -f : 0.0);
        const double du = 0.5 * (sacc[i] - dacc[i]) + (f >= 0 ? -f : 0.0);
        const long ex = (long)s * L.N + j;
        if (A.dl0) A.dl0[ex] = gsv * dl;
        if (A.du0) A.du0[ex] = gsv * du;
    }
}

// LDS bytes of k_grad_box_sc for record ranges of NC output channels (0 when
// the sign-class box kernel does not apply: an output layer, or records or
// weights too large for LDS).
inline size_t grad_box_lds(const LayerGeo& g, int nm, int NC) {
    const size_t rlp = (size_t)((3 + nm + 1) & ~1);
    const size_t rls = (rlp / 2) % 2 ? rlp : rlp + 2;
    const size_t b = (size_t)NC * g.out.P * rls * 8 + (g.kind == ASD_LAYER_DENSE ? 0 : (size_t)g.out.C * g.fan * 4);
    return b;
}

// Taps per lane and output channels per block of the weight-gradient kernel
// for a fan-in (every configuration covers any fan-in; these balance lanes,
// registers and LDS reads).
inline void gw_config(int fan, int* TT, int* TO) {
    *TT = fan <= 64 ? 1 : (fan <= 128 ? 2 : 4);
    *TO = *TT == 1 ? 8 : 4;
}

// Weight gradient of ReLU layer k (k < n) with NM active masks into the
// plan's partial-sum buffer (chunk-major), from the input records at inrec;
// compiled per mask count (asd_grad.hip).
template <int NM>
asd_status grad_weight_nm(asd_plan* P, int k, const double* gs, const void* inrec, hipStream_t st);
// Box gradient through layer 1 with NM active masks (sign-class kernel);
// *done is left false where that kernel does not apply.
template <int NM>
asd_status grad_box_nm(asd_plan* P, const double* gs, double* dl0, double* du0, bool* done, hipStream_t st);

// FP64 per-neuron sums of the final bound of an FP32 plan for ReLU layer k
// with NM active masks (sign classes; asd_final.hip, compiled per mask
// count); inrec: room for the input records of layer k-1 (GwIn<float>).
template <int NM>
asd_status final_sums_nm(asd_plan* P, int k, void* inrec, hipStream_t st);
// FP64 backward pass of the final bound of an FP32 plan into neuron layer k,
// NM = active masks of layer k+1 (sign classes; asd_final.hip); orec: room
// for the output records of layer k+1 (bf_rec_units(NM) 16-byte units per
// neuron).
template <int NM>
asd_status backward_final_nm(const BwdArgs<float>& a, void* orec, hipStream_t st);
constexpr int bf_rec_units(int nm) { return (16 + 4 * nm + 15) / 16; }

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

// Stage two: out[e] = sum over chunks of part[chunk * entries + e].  A block
// takes 64 entries (lanes, coalesced) and kGsumW waves, wave w summing a
// contiguous range of chunks in order; the waves' sums are then added in
// wave order (a fixed order: the result does not depend on scheduling).
constexpr int kGsumW = 16;
static __global__ void __launch_bounds__(64 * kGsumW) k_gsum(const double* part, long entries, int chunks, double* out) {
    __shared__ double red[kGsumW][64];
    const int lane = threadIdx.x, w = threadIdx.y;
    const long e = (long)blockIdx.x * 64 + lane;
    const int c0 = (int)((long)chunks * w / kGsumW), c1 = (int)((long)chunks * (w + 1) / kGsumW);
    double v = 0;
    if (e < entries) {
#pragma unroll 8
        for (int c = c0; c < c1; ++c) v += part[(long)c * entries + e];
    }
    red[w][lane] = v;
    __syncthreads();
    if (w == 0 && e < entries) {
        double t = 0;
        for (int i = 0; i < kGsumW; ++i) t += red[i][lane];
        out[e] = t;
    }
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
