// Iteration kernels of the Active Set dual (Algorithm 1, Sec. 4) for gfx950.
//
// Masked products in (1 + K) form.  Every mask the separation oracle
// eq:oracle adds in Active Set comes from an integral primal point, so its
// row i is all ones when z_I[i] = 1 and otherwise, for input j,
//   I[i, j] = 1  iff  W[i, j] = 0, or the box of j is a point, or
//                     x_I[j] sits at the end minimising W[i, j] x.
// With sigma_I[j] = +1 when x_I[j] is the lower end and -1 when it is the
// upper end (a point box counts as the upper end), each non-point input j
// contributes W+ x or W- x, i.e. (W x + sigma |W| x) / 2.  Hence, with no
// point boxes away from zero among the inputs,
//   (W . I) x [i]      = z_I[i] ? (W x)[i] : ((W x)[i] + (|W| (sigma_I . x))[i]) / 2
// (a point box at x != 0 adds (W+ x_point)[i] to the second form), and
//   (W . I)^T beta [j] = (W^T (z_I beta + u/2))[j] + sigma_I[j] (|W|^T u)[j] / 2
// for non-point j, with u = (1 - z_I) . beta.  One iteration therefore needs
// one W product plus one |W| product per active mask in each direction, all
// dense contractions over the same operands; |W| is the absolute-value
// source modifier of the multiply-add, so no second weight array exists.
// Point boxes need no exact f in an iteration: their x* is the box value
// whatever the sign of f.
//
// Packed bits.  For each neuron of layer k one 16-bit word holds the x-bits
// of every slot of ReLU layer k+1 (bit q) and "point box away from zero"
// (bit 15); for each neuron of a ReLU layer one byte holds the slots' z
// bits.  A tap then costs one x load and one 16-bit load whatever K is.
//
// Mapping.  Convolutions (both directions) and dense backward passes into a
// narrow layer use the "column" mapping of the general kernels: 64 lanes =
// 64 consecutive columns (subproblem, position) of one channel group, the
// reduction split over the block's waves and combined through LDS.  Forward
// weights are read through the scalar unit from a transposed copy
// Wt[tap][channel] (wave-uniform addresses); backward convolution weights
// are staged in LDS per channel group.  Dense forward passes split the
// reduction over blocks, stage x tiles in LDS (lanes = subproblems) and
// write partial sums that a second kernel adds in a fixed order before the
// update.  Dense backward passes into a layer whose positions come in whole
// wavefronts put lanes on positions and give each thread several
// subproblems, whose operands are wave-uniform scalar loads.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "asd_kernels.h"

namespace asd {

typedef const __attribute__((address_space(4))) float* cfloat_p;
template <typename T>
using cptr_t = const __attribute__((address_space(4))) T*;

// Reads through the scalar data cache: only for arrays no kernel of the
// launch writes, at wave-uniform addresses (non-uniform addresses still work
// through vector loads).
__device__ __forceinline__ cfloat_p kconst(const float* p) { return (cfloat_p)p; }
template <typename T>
__device__ __forceinline__ cptr_t<T> kconst_t(const T* p) { return (cptr_t<T>)p; }

template <typename T> __device__ __forceinline__ T flip(T x, unsigned bit) { return bit ? -x : x; }

constexpr int kPointBit = 15;

// ---------------------------------------------------------------------------
// Shared forward update of one neuron (c, s, p) of ReLU layer k from its
// products: yd = (W x)[i], ym[q] = (|W| (sigma_q . x))[i] + 2 (W+ x_point)[i].
// Supergradient eq:as-supergradient, the projected step, and the derived
// sums own, g, vs, u_q.
// ---------------------------------------------------------------------------
template <typename T>
struct FastFwdArgs {
    LayerGeo g;                 // layer k
    int S;
    int nm;
    int Cpad;                   // channel stride of Wt
    int ksplit;                 // dense: blocks splitting the fan-in
    const float* Wt;            // [fan][Cpad] transposed weights (zero columns past C)
    const T* xin;               // x*_{k-1}
    const uint16_t* xpk;        // packed bits of layer k-1
    const int* pointflag;       // layer k-1 has point boxes away from zero
    const T* xout;              // x*_k
    const ReluLayerT<T>* R;     // layer k arrays, a copy in device memory (read
                                // in the update only, through the scalar cache)
    StepArgsT<T> st;
    T* part;                    // dense: partial products [ksplit][1 + nm][Cpad][S]
};

template <typename T, int NM>
__device__ __forceinline__ void fwd_update(const FastFwdArgs<T>& A, int c, long idx, long bi, T yd,
                                           const T* ym) {
    const cptr_t<ReluLayerT<T>> R = kconst_t(A.R);
    const T bb = (T)A.g.b[c];
    const T xhat = yd + bb;
    const T x = A.xout[idx];
    const T z = (T)getbit(R->zbits, bi);
    const T lh = R->lhat[idx], uh = R->uhat[idx];
    const T ga = xhat - x;
    const T gb0 = x - z * uh;
    const T gb1 = x - xhat + ((T)1 - z) * lh;
    const unsigned zq = NM > 0 ? (unsigned)R->zpk[idx] : 0u;
    T gm[NM > 0 ? NM : 1], LI[NM > 0 ? NM : 1], UI[NM > 0 ? NM : 1];
#pragma unroll
    for (int q = 0; q < NM; ++q) {
        LI[q] = R->slot[q].LI[idx];
        UI[q] = R->slot[q].UI[idx];
        const T mq = ((zq >> q) & 1u) ? yd : (T)0.5 * (yd + ym[q]);
        gm[q] = x - mq + LI[q] * ((T)1 - z) - z * bb - UI[q] * z;
    }
    const StepArgsT<T>& st = A.st;
    auto step = [&](T th, T* m, T* v, T gr, int grp) -> T {
        if (st.rule == ASD_RULE_SUPERGRADIENT) return tmax0(th + st.lr * gr);
        const T mm = st.b1 * m[idx] + ((T)1 - st.b1) * gr;
        const T vv = st.b2 * v[idx] + ((T)1 - st.b2) * gr * gr;
        m[idx] = mm;
        v[idx] = vv;
        const T mh = mm / st.bc1[grp];
        const T vh = vv / st.bc2[grp];
        return tmax0(th + st.lr * mh / (tsqrt(vh) + st.eps));
    };
    const T al = step(R->alpha[idx], R->alpha_m, R->alpha_v, ga, 0);
    const T b0 = step(R->beta0[idx], R->beta0_m, R->beta0_v, gb0, 0);
    const T b1 = step(R->beta1[idx], R->beta1_m, R->beta1_v, gb1, 0);
    R->alpha[idx] = al;
    R->beta0[idx] = b0;
    R->beta1[idx] = b1;
    T own = al - b0 - b1;
    T gg = b0 * uh + b1 * lh;
    T vs = -al + b1;
#pragma unroll
    for (int q = 0; q < NM; ++q) {
        const cptr_t<MaskSlotT<T>> M = &R->slot[q];
        const T bq = step(M->beta[idx], M->m, M->v, gm[q], 1 + q);
        M->beta[idx] = bq;
        own -= bq;
        gg += bq * (LI[q] + UI[q] + bb);
        const bool zb = (zq >> q) & 1u;
        vs += zb ? bq : (T)0.5 * bq;
        M->u[idx] = zb ? (T)0 : bq;
    }
    R->own[idx] = own;
    R->g[idx] = gg;
    R->vs[idx] = vs;
}

// ---------------------------------------------------------------------------
// Forward pass of a convolutional ReLU layer k (column mapping).
// Grid (colpad_k / 64, ceil(C_k / CB)), block (64, KS).
// ---------------------------------------------------------------------------
template <typename T, int NM, int CB, int KSZ>
__global__ void __launch_bounds__(kWave * KS) k_fwd_conv(FastFwdArgs<T> A) {
    static_assert(CB % KS == 0, "CB must be a multiple of KS");
    constexpr int EPW = CB / KS;  // epilogue channels per wave
    constexpr int NA = NM > 0 ? NM : 1;
    __shared__ T red[KS][CB][kWave];
    const LayerGeo& g = A.g;
    const int lane = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.y);  // wave-uniform
    const long col = (long)blockIdx.x * kWave + lane;
    const int c0 = blockIdx.y * CB;
    const int S = A.S;
    const bool colok = col < g.out.cols;
    const int s = colok ? (int)(col / g.out.P) : 0;
    const int p = colok ? (int)(col - (long)s * g.out.P) : 0;
    const int oy = p / g.out.W, ox = p - (p / g.out.W) * g.out.W;
    const int ks = KSZ > 0 ? KSZ : g.ksz;
    const int iy0 = oy * g.stride - g.pad, ix0 = ox * g.stride - g.pad;
    unsigned colmask = 0;
    for (int kx = 0; kx < ks; ++kx) {
        const int ix = ix0 + kx;
        if (ix >= 0 && ix < g.in.W) colmask |= 1u << kx;
    }
    T yd[CB], ym[NA][CB];
#pragma unroll
    for (int e = 0; e < CB; ++e) {
        yd[e] = 0;
#pragma unroll
        for (int q = 0; q < NA; ++q) ym[q][e] = 0;
    }
    const cfloat_p Wt = kconst(A.Wt);
    const int Cp = A.Cpad;
    const int R = g.in.C * ks;  // tap rows (ci, ky)
    const int r0 = R * wave / KS, r1 = R * (wave + 1) / KS;
    const bool pointin = NM > 0 && *kconst_t<int>(A.pointflag) != 0;
    // Taps of one row (ci, ky): loads are issued unconditionally from clamped
    // addresses and zeroed afterwards, so a row's loads overlap.
    constexpr int KX = KSZ > 0 ? KSZ : 1;
    auto row_taps = [&](int r, int ci, int ky, auto&& body) {
        const int iy = iy0 + ky;
        const bool rowok = iy >= 0 && iy < g.in.H;
        const long base = ((long)ci * S + s) * g.in.P + (long)iy * g.in.W + ix0;
        const long wrow = (long)r * ks * Cp + c0;
        for (int kx0 = 0; kx0 < ks; kx0 += KX) {
            T xv[KX];
            unsigned hv[KX];
#pragma unroll
            for (int u = 0; u < KX; ++u) {
                const int kx = kx0 + u;
                const bool ok = rowok && ((colmask >> kx) & 1u);
                const long a = ok ? base + kx : 0;
                const T xl = A.xin[a];
                const unsigned hl = NM > 0 ? (unsigned)A.xpk[a] : 0u;
                xv[u] = ok ? xl : (T)0;
                hv[u] = ok ? hl : 0u;
            }
#pragma unroll
            for (int u = 0; u < KX; ++u) {
                float w[CB];
#pragma unroll
                for (int e = 0; e < CB; ++e) w[e] = Wt[wrow + (long)(kx0 + u) * Cp + e];
                body(xv[u], hv[u], w);
            }
        }
    };
    auto rows = [&](auto&& body) {
        int ci = r0 / ks, ky = r0 - (r0 / ks) * ks;
        for (int r = r0; r < r1; ++r) {
            row_taps(r, ci, ky, body);
            if (++ky == ks) {
                ky = 0;
                ++ci;
            }
        }
    };
    if (colok) {
        rows([&](T x, unsigned h, const float* w) {
#pragma unroll
            for (int e = 0; e < CB; ++e) yd[e] += (T)w[e] * x;
#pragma unroll
            for (int q = 0; q < NM; ++q) {
                const T sx = flip(x, (h >> q) & 1u);
#pragma unroll
                for (int e = 0; e < CB; ++e) ym[q][e] += (T)fabsf(w[e]) * sx;
            }
        });
        if (pointin) {
            // point boxes away from zero: (W . I) x gains W+ x_point on z = 0 rows
            T yp[CB];
#pragma unroll
            for (int e = 0; e < CB; ++e) yp[e] = 0;
            rows([&](T x, unsigned h, const float* w) {
                const T xp = ((h >> kPointBit) & 1u) ? x : (T)0;
#pragma unroll
                for (int e = 0; e < CB; ++e) yp[e] += (T)fmaxf(w[e], 0.f) * xp;
            });
#pragma unroll
            for (int q = 0; q < NM; ++q)
#pragma unroll
                for (int e = 0; e < CB; ++e) ym[q][e] += (T)2 * yp[e];
        }
    }
    // reduce each component over the waves; wave w keeps channels w * EPW ..
    T tot[1 + NM][EPW];
#pragma unroll
    for (int r = 0; r <= NM; ++r) {
#pragma unroll
        for (int e = 0; e < CB; ++e) red[wave][e][lane] = r == 0 ? yd[e] : ym[r > 0 ? r - 1 : 0][e];
        __syncthreads();
#pragma unroll
        for (int j = 0; j < EPW; ++j) {
            T a = 0;
#pragma unroll
            for (int w = 0; w < KS; ++w) a += red[w][wave * EPW + j][lane];
            tot[r][j] = a;
        }
        __syncthreads();
    }
    if (!colok) return;
#pragma unroll
    for (int j = 0; j < EPW; ++j) {
        const int c = c0 + wave * EPW + j;
        if (c >= g.out.C) break;
        const long idx = ((long)c * S + s) * g.out.P + p;
        const long bi = (long)c * g.out.colpad + col;
        T ymj[NA];
#pragma unroll
        for (int q = 0; q < NM; ++q) ymj[q] = tot[1 + q][j];
        fwd_update<T, NM>(A, c, idx, bi, tot[0][j], ymj);
    }
}

// ---------------------------------------------------------------------------
// Forward pass of a dense ReLU layer k, split over the fan-in.
// Part kernel: grid (ceil(S / 64), ceil(C_k / (KS * CB)), ksplit), block
// (64, KS): lanes = subproblems, wave = CB output channels; x tiles of 64
// taps x 64 subproblems are staged in LDS.
// ---------------------------------------------------------------------------
constexpr int kDenseTile = 64;

template <typename T, int NM, int CB>
__global__ void __launch_bounds__(kWave * KS) k_fwd_dense_part(FastFwdArgs<T> A) {
    constexpr int NA = NM > 0 ? NM : 1;
    __shared__ T xs[kDenseTile][kWave + 1];
    __shared__ uint16_t hs[kDenseTile][kWave + 2];
    const LayerGeo& g = A.g;
    const int lane = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.y);  // wave-uniform
    const int tid = wave * kWave + lane;
    const int S = A.S;
    const int s0 = blockIdx.x * kWave;
    const int cb = (blockIdx.y * KS + wave) * CB;
    const int F = g.fan;
    const int Pin = g.in.P;
    const int t0 = (int)((long)F * blockIdx.z / A.ksplit), t1 = (int)((long)F * (blockIdx.z + 1) / A.ksplit);
    const cfloat_p Wt = kconst(A.Wt);
    const int Cp = A.Cpad;
    const bool pointin = NM > 0 && *kconst_t<int>(A.pointflag) != 0;
    T yd[CB], ym[NA][CB];
#pragma unroll
    for (int e = 0; e < CB; ++e) {
        yd[e] = 0;
#pragma unroll
        for (int q = 0; q < NA; ++q) ym[q][e] = 0;
    }
    for (int tc = t0; tc < t1; tc += kDenseTile) {
        const int nt = min(kDenseTile, t1 - tc);
        // stage: runs of consecutive positions of one subproblem when the
        // input has positions, runs of subproblems otherwise
        for (int e = tid; e < kDenseTile * kWave; e += kWave * KS) {
            const int sl = Pin > 1 ? e / kDenseTile : e % kWave;
            const int tl = Pin > 1 ? e % kDenseTile : e / kWave;
            const int s = s0 + sl;
            T v = 0;
            uint16_t h = 0;
            if (s < S && tl < nt) {
                const int t = tc + tl;
                const int ci = t / Pin, pp = t - (t / Pin) * Pin;
                const long a = ((long)ci * S + s) * Pin + pp;
                v = A.xin[a];
                if (NM > 0) h = A.xpk[a];
            }
            xs[tl][sl] = v;
            hs[tl][sl] = h;
        }
        __syncthreads();
        if (cb < g.out.C) {
#pragma unroll 4
            for (int tl = 0; tl < nt; ++tl) {
                const T x = xs[tl][lane];
                const unsigned h = NM > 0 ? (unsigned)hs[tl][lane] : 0u;
                float w[CB];
                const long wrow = (long)(tc + tl) * Cp + cb;
#pragma unroll
                for (int e = 0; e < CB; ++e) w[e] = Wt[wrow + e];
#pragma unroll
                for (int e = 0; e < CB; ++e) yd[e] += (T)w[e] * x;
#pragma unroll
                for (int q = 0; q < NM; ++q) {
                    const T sx = flip(x, (h >> q) & 1u);
#pragma unroll
                    for (int e = 0; e < CB; ++e) ym[q][e] += (T)fabsf(w[e]) * sx;
                }
            }
            if (pointin) {
                // point boxes away from zero: (W . I) x gains W+ x_point on z = 0 rows
                T yp[CB];
#pragma unroll
                for (int e = 0; e < CB; ++e) yp[e] = 0;
                for (int tl = 0; tl < nt; ++tl) {
                    const T xp = ((hs[tl][lane] >> kPointBit) & 1u) ? xs[tl][lane] : (T)0;
                    const long wrow = (long)(tc + tl) * Cp + cb;
#pragma unroll
                    for (int e = 0; e < CB; ++e) yp[e] += (T)fmaxf(Wt[wrow + e], 0.f) * xp;
                }
#pragma unroll
                for (int q = 0; q < NM; ++q)
#pragma unroll
                    for (int e = 0; e < CB; ++e) ym[q][e] += (T)2 * yp[e];
            }
        }
        __syncthreads();
    }
    const int s = s0 + lane;
    if (s >= S) return;
    const long zs = (long)blockIdx.z * (1 + NM);
#pragma unroll
    for (int e = 0; e < CB; ++e) {
        const int c = cb + e;
        if (c >= g.out.C) break;
        A.part[((zs + 0) * Cp + c) * S + s] = yd[e];
#pragma unroll
        for (int q = 0; q < NM; ++q) A.part[((zs + 1 + q) * Cp + c) * S + s] = ym[q][e];
    }
}

// Sums the partial products in a fixed order and updates.  Grid
// (ceil(S / 256), C_k), block 256.
template <typename T, int NM>
__global__ void __launch_bounds__(256) k_fwd_dense_epi(FastFwdArgs<T> A) {
    constexpr int NA = NM > 0 ? NM : 1;
    const int s = blockIdx.x * 256 + threadIdx.x;
    const int c = blockIdx.y;
    const int S = A.S;
    if (s >= S) return;
    const int Cp = A.Cpad;
    T yd = 0, ym[NA];
#pragma unroll
    for (int q = 0; q < NA; ++q) ym[q] = 0;
    for (int z = 0; z < A.ksplit; ++z) {
        const long zs = (long)z * (1 + NM);
        yd += A.part[((zs + 0) * Cp + c) * S + s];
#pragma unroll
        for (int q = 0; q < NM; ++q) ym[q] += A.part[((zs + 1 + q) * Cp + c) * S + s];
    }
    const long idx = (long)c * S + s;  // dense layout, P = 1
    const long bi = (long)c * A.g.out.colpad + s;
    fwd_update<T, NM>(A, c, idx, bi, yd, ym);
}

// ---------------------------------------------------------------------------
// Backward pass into neuron layer k: f_k from layer k+1's operands, then the
// inner minimisation (x*_k, z*_k bits).  Only the iteration needs these
// kernels, so f at point boxes is not formed exactly (x* does not depend on
// it) and no objective terms are written.
// ---------------------------------------------------------------------------
template <typename T>
struct FastBwdArgs {
    LayerGeo gn;                // layer k+1 (its input layout is layer k)
    int S;
    int k;
    int last;                   // layer k+1 is the output layer: operand -c
    int nm;                     // masks of layer k+1
    const float* Wr;            // dense: W rows padded to fanpad (zeros past layer k)
    int fanpad;
    const T* cvec;              // objective rows (layout of layer n)
    const T* vs;                // layer k+1 operand of the W^T product
    const T* u[kMaxMasks];      // layer k+1 operands of the |W|^T products
    const uint16_t* xpk;        // packed bits of layer k
    NeuronArraysT<T> nk;        // layer k box and outputs
    const T* own;               // layer k (k >= 1)
    const T* gk;
    uint32_t* zbits;            // layer k (k >= 1)
};

// Finishes neuron (c, col) of layer k from its f (without own): x*, bits.
// Every lane of the wave calls it (ballots).
template <typename T>
__device__ __forceinline__ void bwd_finish(const FastBwdArgs<T>& A, int c, long col, bool ok, long idx, T f,
                                           long wave_base, int lane) {
    bool xb = false, zb = false;
    if (ok) {
        const long bi = (long)c * A.gn.in.colpad + col;
        if (A.k >= 1) f += A.own[idx];
        xb = f >= (T)0 || getbit(A.nk.deg, bi);
        A.nk.xstar[idx] = xb ? A.nk.hi[idx] : A.nk.lo[idx];
        if (A.k >= 1) zb = A.gk[idx] >= (T)0;
    }
    put_wave_bits(A.nk.xbits, wave_base, xb, lane);
    if (A.k >= 1) put_wave_bits(A.zbits, wave_base, zb, lane);
}

// Transposed convolution (column mapping over layer k).  Grid
// (colpad_k / 64, ceil(C_k / CB)), block (64, KS); dynamic LDS holds the
// block's weights as [C_{k+1}][ks][ks][CB].  KSZ, STR > 0 fix the kernel
// size and stride (taps of one output channel unrolled), 0 = any.
template <typename T, int NM, int CB, int KSZ, int STR>
__global__ void __launch_bounds__(kWave * KS) k_bwd_conv(FastBwdArgs<T> A) {
    static_assert(CB % KS == 0, "CB must be a multiple of KS");
    constexpr int EPW = CB / KS;
    constexpr int NA = NM > 0 ? NM : 1;
    extern __shared__ float wl[];
    __shared__ T red[KS][CB][kWave];
    const LayerGeo& g = A.gn;
    const NeuronLayout& L = g.in;
    const NeuronLayout& O = g.out;
    const int lane = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.y);  // wave-uniform
    const int tid = wave * kWave + lane;
    const long col = (long)blockIdx.x * kWave + lane;
    const int c0 = blockIdx.y * CB;
    const int S = A.S;
    const int ks = g.ksz, st = g.stride;
    const int nw = O.C * ks * ks * CB;
    for (int i = tid; i < nw; i += kWave * KS) {
        const int e = i % CB;
        const int rest = i / CB;  // (co * ks + ky) * ks + kx
        const int co = rest / (ks * ks);
        const int kk = rest - co * ks * ks;
        const int c = c0 + e;
        wl[i] = c < L.C ? g.W[((long)co * L.C + c) * ks * ks + kk] : 0.f;
    }
    __syncthreads();
    const bool colok = col < L.cols;
    const int s = colok ? (int)(col / L.P) : 0;
    const int p = colok ? (int)(col - (long)s * L.P) : 0;
    const int y = p / L.W, x = p - (p / L.W) * L.W;
    const int ry = (y + g.pad) % st, qy = (y + g.pad) / st;
    const int rx = (x + g.pad) % st, qx = (x + g.pad) / st;
    T acc[CB], au[NA][CB];
#pragma unroll
    for (int e = 0; e < CB; ++e) {
        acc[e] = 0;
#pragma unroll
        for (int q = 0; q < NA; ++q) au[q][e] = 0;
    }
    const int co0 = O.C * wave / KS, co1 = O.C * (wave + 1) / KS;
    // taps per axis: ky = ry + st * jy receives output row qy - jy
    const int JT = (ks + st - 1) / st;
    constexpr int J = (KSZ > 0 && STR > 0) ? (KSZ + STR - 1) / STR : 1;
    if (colok) {
        for (int co = co0; co < co1; ++co) {
            const long obase = ((long)co * S + s) * O.P;
            const int wco = co * ks * ks;
            for (int jy0 = 0; jy0 < JT; jy0 += J) {
                for (int jx0 = 0; jx0 < JT; jx0 += J) {
                    T vv[J][J], uu[NA][J][J];
                    int kk[J][J];
#pragma unroll
                    for (int jy = 0; jy < J; ++jy) {
#pragma unroll
                        for (int jx = 0; jx < J; ++jx) {
                            const int ky = ry + st * (jy0 + jy), kx = rx + st * (jx0 + jx);
                            const int oy = qy - (jy0 + jy), ox = qx - (jx0 + jx);
                            const bool ok = ky < ks && kx < ks && oy >= 0 && oy < O.H && ox >= 0 && ox < O.W;
                            const long a = ok ? obase + (long)oy * O.W + ox : 0;
                            const T vl = A.vs[a];
                            vv[jy][jx] = ok ? vl : (T)0;
#pragma unroll
                            for (int q = 0; q < NM; ++q) {
                                const T ul = A.u[q][a];
                                uu[q][jy][jx] = ok ? ul : (T)0;
                            }
                            kk[jy][jx] = ok ? ky * ks + kx : 0;
                        }
                    }
#pragma unroll
                    for (int jy = 0; jy < J; ++jy) {
#pragma unroll
                        for (int jx = 0; jx < J; ++jx) {
                            const float* wp = &wl[(wco + kk[jy][jx]) * CB];
#pragma unroll
                            for (int e = 0; e < CB; ++e) {
                                acc[e] += (T)wp[e] * vv[jy][jx];
#pragma unroll
                                for (int q = 0; q < NM; ++q) au[q][e] += (T)fabsf(wp[e]) * uu[q][jy][jx];
                            }
                        }
                    }
                }
            }
        }
    }
    // fold sigma_q (this neuron's packed x-bits) before the cross-wave sum
#pragma unroll
    for (int e = 0; e < CB; ++e) {
        T part = acc[e];
        if (NM > 0 && colok && c0 + e < L.C) {
            const unsigned h = A.xpk[((long)(c0 + e) * S + s) * L.P + p];
#pragma unroll
            for (int q = 0; q < NM; ++q) part += (T)0.5 * flip(au[q][e], (h >> q) & 1u);
        }
        red[wave][e][lane] = part;
    }
    __syncthreads();
    const long wave_base = (long)blockIdx.x * kWave;
#pragma unroll
    for (int j = 0; j < EPW; ++j) {
        const int e = wave * EPW + j;
        const int c = c0 + e;
        if (c >= L.C) break;  // uniform
        T f = 0;
#pragma unroll
        for (int w = 0; w < KS; ++w) f += red[w][e][lane];
        const long idx = ((long)c * S + s) * L.P + p;
        bwd_finish<T>(A, c, col, colok, idx, f, (long)c * L.colpad + wave_base, lane);
    }
}

// Dense layer k+1 into layer k, column mapping (any P_k; P1 = (P_k == 1),
// when the weights are wave-uniform scalar loads).  Grid (colpad_k / 64,
// ceil(C_k / CB)), block (64, KS), the outputs of layer k+1 split over waves.
template <typename T, int NM, int CB, bool P1>
__global__ void __launch_bounds__(kWave * KS) k_bwd_dense(FastBwdArgs<T> A) {
    static_assert(CB % KS == 0, "CB must be a multiple of KS");
    constexpr int EPW = CB / KS;
    constexpr int NA = NM > 0 ? NM : 1;
    __shared__ T red[KS][CB][kWave];
    const LayerGeo& g = A.gn;
    const NeuronLayout& L = g.in;
    const int lane = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.y);  // wave-uniform
    const long col = (long)blockIdx.x * kWave + lane;
    const int c0 = blockIdx.y * CB;
    const int S = A.S;
    const bool colok = col < L.cols;
    const int s = colok ? (int)(col / L.P) : 0;
    const int p = colok ? (int)(col - (long)s * L.P) : 0;
    const int n1 = g.out.C;
    const int i0 = n1 * wave / KS, i1 = n1 * (wave + 1) / KS;
    const cfloat_p Wr = kconst(A.Wr);
    T acc[CB], au[NA][CB];
#pragma unroll
    for (int e = 0; e < CB; ++e) {
        acc[e] = 0;
#pragma unroll
        for (int q = 0; q < NA; ++q) au[q][e] = 0;
    }
    if (colok) {
#pragma unroll 4
        for (int i = i0; i < i1; ++i) {
            const long a = (long)i * S + s;
            const T v = A.last ? -A.cvec[a] : A.vs[a];
            T uq[NA];
#pragma unroll
            for (int q = 0; q < NM; ++q) uq[q] = A.u[q][a];
            const long wrow = P1 ? (long)i * A.fanpad + c0 : (long)i * A.fanpad + (long)c0 * L.P + p;
#pragma unroll
            for (int e = 0; e < CB; ++e) {
                const float wf = Wr[wrow + (P1 ? (long)e : (long)e * L.P)];
                acc[e] += (T)wf * v;
#pragma unroll
                for (int q = 0; q < NM; ++q) au[q][e] += (T)fabsf(wf) * uq[q];
            }
        }
    }
#pragma unroll
    for (int e = 0; e < CB; ++e) {
        T part = acc[e];
        if (NM > 0 && colok && c0 + e < L.C) {
            const unsigned h = A.xpk[((long)(c0 + e) * S + s) * L.P + p];
#pragma unroll
            for (int q = 0; q < NM; ++q) part += (T)0.5 * flip(au[q][e], (h >> q) & 1u);
        }
        red[wave][e][lane] = part;
    }
    __syncthreads();
    const long wave_base = (long)blockIdx.x * kWave;
#pragma unroll
    for (int j = 0; j < EPW; ++j) {
        const int e = wave * EPW + j;
        const int c = c0 + e;
        if (c >= L.C) break;
        T f = 0;
#pragma unroll
        for (int w = 0; w < KS; ++w) f += red[w][e][lane];
        const long idx = ((long)c * S + s) * L.P + p;
        bwd_finish<T>(A, c, col, colok, idx, f, (long)c * L.colpad + wave_base, lane);
    }
}

// Dense layer k+1 into a layer k whose positions come in whole wavefronts
// (P_k % 64 == 0): lanes = 64 positions of one channel, each thread SB
// consecutive subproblems whose operands are wave-uniform scalar loads (the
// last tile is shifted back to end at S, so S >= SB).  Grid
// (C_k * P_k / 64, ceil(S / SB)), block (64, KS), the outputs of layer k+1
// split over waves.
template <typename T, int NM, int SB>
__global__ void __launch_bounds__(kWave * KS) k_bwd_dense_pos(FastBwdArgs<T> A) {
    static_assert(SB % KS == 0, "SB must be a multiple of KS");
    constexpr int EPW = SB / KS;
    constexpr int NA = NM > 0 ? NM : 1;
    __shared__ T red[KS][SB][kWave];
    const LayerGeo& g = A.gn;
    const NeuronLayout& L = g.in;
    const int lane = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.y);  // wave-uniform
    const int S = A.S;
    const int tiles = L.P / kWave;
    const int c = blockIdx.x / tiles;
    const int p = (blockIdx.x - c * tiles) * kWave + lane;
    const int s0 = blockIdx.y * SB;
    const int sb = min(s0, S - SB);
    const int n1 = g.out.C;
    const int i0 = n1 * wave / KS, i1 = n1 * (wave + 1) / KS;
    const long F = g.fan;
    const cptr_t<T> vs = kconst_t<T>(A.last ? A.cvec : A.vs);
    const T vsign = A.last ? (T)-1 : (T)1;
    T acc[SB], au[NA][SB];
#pragma unroll
    for (int j = 0; j < SB; ++j) {
        acc[j] = 0;
#pragma unroll
        for (int q = 0; q < NA; ++q) au[q][j] = 0;
    }
#pragma unroll 2
    for (int i = i0; i < i1; ++i) {
        const float wf = g.W[(long)i * F + (long)c * L.P + p];
        const T w = (T)wf, wa = (T)fabsf(wf);
        const long a = (long)i * S + sb;
#pragma unroll
        for (int j = 0; j < SB; ++j) acc[j] += w * vs[a + j];
#pragma unroll
        for (int q = 0; q < NM; ++q) {
            const cptr_t<T> uq = kconst_t<T>(A.u[q]);
#pragma unroll
            for (int j = 0; j < SB; ++j) au[q][j] += wa * uq[a + j];
        }
    }
#pragma unroll
    for (int j = 0; j < SB; ++j) {
        T part = vsign * acc[j];
        if (NM > 0) {
            const unsigned h = A.xpk[((long)c * S + sb + j) * L.P + p];
#pragma unroll
            for (int q = 0; q < NM; ++q) part += (T)0.5 * flip(au[q][j], (h >> q) & 1u);
        }
        red[wave][j][lane] = part;
    }
    __syncthreads();
#pragma unroll
    for (int jj = 0; jj < EPW; ++jj) {
        const int j = wave * EPW + jj;
        const int s = sb + j;
        if (s < s0) continue;  // uniform: computed by the previous tile
        T f = 0;
#pragma unroll
        for (int w = 0; w < KS; ++w) f += red[w][j][lane];
        const long idx = ((long)c * S + s) * L.P + p;
        const long col = (long)s * L.P + p;
        bwd_finish<T>(A, c, col, true, idx, f, (long)c * L.colpad + (long)s * L.P + (p - lane), lane);
    }
}

// ---------------------------------------------------------------------------
// Packed bits.  Grid (ceil(cols / 256), C), block 256.
// x words of layer k from the x-bit arrays of the nm slots of ReLU layer k+1,
// the point-box bits of layer k and its lower ends; flags a point box away
// from zero in *pointflag.
// ---------------------------------------------------------------------------
template <typename T>
struct PackArgs {
    NeuronLayout nl;
    int S;
    int nm;
    const uint32_t* bits[kMaxMasks];
    const uint32_t* deg;        // x words only
    const T* lo;                // x words only
    uint16_t* xpk;              // x words, or
    uint8_t* zpk;               // z bytes
    int* pointflag;
};

template <typename T>
__global__ void __launch_bounds__(256) k_pack(PackArgs<T> A) {
    const long col = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const int c = blockIdx.y;
    bool point_nz = false;
    if (col < A.nl.cols) {
        const int s = (int)(col / A.nl.P), p = (int)(col - (long)s * A.nl.P);
        const long idx = ((long)c * A.S + s) * A.nl.P + p;
        const long bi = (long)c * A.nl.colpad + col;
        unsigned w = 0;
        const bool dg = A.xpk ? getbit(A.deg, bi) != 0u : false;
        for (int q = 0; q < A.nm; ++q) w |= (getbit(A.bits[q], bi) | (dg ? 1u : 0u)) << q;
        if (A.xpk) {
            point_nz = dg && A.lo[idx] != (T)0;
            if (point_nz) w |= 1u << kPointBit;
            A.xpk[idx] = (uint16_t)w;
        } else {
            A.zpk[idx] = (uint8_t)w;
        }
    }
    if (A.pointflag) {
        const unsigned long long m = __ballot(point_nz);
        if (m != 0ull && (threadIdx.x & 63) == 0) atomicOr(A.pointflag, 1);
    }
}

// Transposed forward weights Wt[t][c] = W[c][t], zero for c >= C.
// Grid (ceil(fan * Cpad / 256)), block 256.
__global__ void __launch_bounds__(256) k_transpose_w(const float* W, float* Wt, int C, int fan, int Cpad) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (long)fan * Cpad) return;
    const int t = (int)(i / Cpad), c = (int)(i - (long)t * Cpad);
    Wt[i] = c < C ? W[(long)c * fan + t] : 0.f;
}

// Dense weights with rows padded to fanpad: Wr[i][j] = W[i][j] for j < fan.
__global__ void __launch_bounds__(256) k_pad_rows(const float* W, float* Wr, int n_out, int fan, int fanpad) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (long)n_out * fanpad) return;
    const int r = (int)(i / fanpad), j = (int)(i - (long)r * fanpad);
    Wr[i] = j < fan ? W[(long)r * fan + j] : 0.f;
}

}  // namespace asd
