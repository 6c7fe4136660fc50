// Saddle Point (Sec. 5, Algorithm 2) and AS-SP on the plan's layers.
//
// The multipliers of the exponentially many Anderson constraints of ReLU
// layer k are kept only through the four per-neuron sums of eq:suff-stats
// (zeta1_k, zeta3_k, zeta4_k in layer k's layout, zeta2_k in layer k-1's),
// beside alpha_k and the SP-FW primal iterate (x_k, z_k) with values in the
// boxes.  One iteration:
//   * primal conditional gradient: the minimiser of the Lagrangian at the
//     current duals, from f_k = alpha_k - zeta1_k + zeta2_{k+1}
//     - W_{k+1}^T alpha_{k+1} and g_k = zeta3_k + zeta4_k + b_k zeta1_k (one
//     transposed product per layer: the statistics replace the masked ones);
//   * dual conditional gradient at the primal iterate: alpha goes to its cap
//     where the ReLU residual W x + b - x is >= 0 (eq:alphak-condg); per
//     neuron the most violated of beta_{k,0}, beta_{k,1} and the oracle's mask
//     at the fractional iterate (eq:oracle; eq:betak-condg and the
//     proposition after it) gets the beta cap when its violation is >= 0;
//   * convex combination of both iterates with gamma_t = 1 / (t + gamma0).
// The set-up converts the plan's duals (Big-M or Active Set with masks) into
// the statistics, sets the caps of eq:price-caps and runs the primal
// initialisation of App. C.2 (projected subgradient steps on the Big-M primal
// view).  Readings: the fourth statistic takes the complement mask with the
// U-check matrix (as the beta_{k,0} term and the constraint require); ties of
// the vertex choice go to beta_{k,0}, then beta_{k,1}, then the oracle's
// mask; the oracle's test per weight is (l - x) + z (u - l) >= 0 for W >= 0
// and (u - x) - z (u - l) <= 0 for W < 0, so that a point box ties exactly
// (bit 1).
//
// Layouts: every array is in the plan's internal neuron layout
// ((c S + s) P + p).  This unit is compiled without floating-point
// contraction: each product and sum rounds on its own, so that the decisions
// taken at exact ties of the iterates (a mask bit where x_j and z_i share
// their vertex history, a clipped primal entry) are taken identically by any
// implementation that evaluates the same expressions in the same precision.
#include <cmath>

#include "asd_plan.h"

using namespace asd;

namespace asd {

// Arrays per layer (the first ten in the order of asd_sp_field).
enum SpArr {
    SA_X = 0, SA_XBAR, SA_ALPHA, SA_Z1, SA_Z3, SA_Z4, SA_MUA, SA_MUB, SA_Z, SA_ZETA2,
    SA_ZBAR, SA_AROW, SA_BROW, SA_B0ROW, SA_COUNT
};
static_assert(SA_COUNT <= 16, "plan field sp_arr holds 16 arrays per layer");

}  // namespace asd

namespace {

constexpr int kSpBlock = 256;
constexpr int kSpLdsBlock = 1024;  // one block per subproblem: 16 waves

__device__ __forceinline__ void split_index(long idx, int S, const NeuronLayout& L, int& c, int& s, int& p) {
    const long sp = (long)S * L.P;
    c = (int)(idx / sp);
    const long r = idx - (long)c * sp;
    s = (int)(r / L.P);
    p = (int)(r - (long)s * L.P);
}

// Calls fn(w, a, bi) for every output neuron of layer L (geometry g) that
// reads input neuron (c, s, p) of layer L-1: w = W[i][j], a its address in
// layer L's internal layout, bi its bit index.
template <class Fn>
__device__ __forceinline__ void for_rows(const LayerGeo& g, int S, int c, int s, int p, Fn&& fn) {
    const NeuronLayout& L = g.in;
    const NeuronLayout& O = g.out;
    if (g.kind == ASD_LAYER_DENSE) {
        const long j = (long)c * L.P + p;
        for (int i = 0; i < O.C; ++i)
            fn(g.W[(long)i * g.fan + j], (long)i * S + s, (long)i * O.colpad + s);
    } else {
        const int y = p / L.W, x = p - (p / L.W) * L.W;
        const int ks = g.ksz, str = g.stride;
        const int ky0 = (y + g.pad) % str, kx0 = (x + g.pad) % str;
        const int oyf = (y + g.pad - ky0) / str, oxf = (x + g.pad - kx0) / str;
        for (int co = 0; co < O.C; ++co) {
            int oy = oyf;
            for (int ky = ky0; ky < ks; ky += str, --oy) {
                if (oy < 0 || oy >= O.H) continue;
                int ox = oxf;
                for (int kx = kx0; kx < ks; kx += str, --ox) {
                    if (ox < 0 || ox >= O.W) continue;
                    const int op = oy * O.W + ox;
                    fn(g.W[(((long)co * L.C + c) * ks + ky) * ks + kx], ((long)co * S + s) * O.P + op,
                       (long)co * O.colpad + (long)s * O.P + op);
                }
            }
        }
    }
}

template <typename T>
__device__ __forceinline__ T clip_to(T v, T lo, T hi) {
    return v < lo ? lo : (v > hi ? hi : v);
}

// Oracle mask bit of weight w between column value x in [l, u] and row z.
template <typename T>
__device__ __forceinline__ bool mask_bit(T w, T l, T u, T x, T z) {
    return w >= (T)0 ? (l - x) + z * (u - l) >= (T)0 : (u - x) - z * (u - l) <= (T)0;
}

// ---------------------------------------------------------------------------
// Set-up: statistics and caps of ReLU layer k from the plan's duals
// ---------------------------------------------------------------------------

template <typename T>
struct SpConvertArgs {
    long n;              // neurons of layer k times S
    int S;
    NeuronLayout L;      // layer k
    const float* b;      // bias per channel
    ReluLayerT<T> R;
    int nm;
    T* alpha; T* z1; T* z3; T* z4; T* mua; T* mub;
    T cap_a, cap_b;
};

template <typename T>
__global__ void __launch_bounds__(kSpBlock) k_sp_convert(SpConvertArgs<T> A) {
    const long idx = (long)blockIdx.x * kSpBlock + threadIdx.x;
    if (idx >= A.n) return;
    int c, s, p;
    split_index(idx, A.S, A.L, c, s, p);
    const T b = (T)A.b[c];
    const T al = A.R.alpha[idx], b0 = A.R.beta0[idx], b1 = A.R.beta1[idx];
    const T lh = A.R.lhat[idx], uh = A.R.uhat[idx];
    T s1 = b0 + b1;
    T s3 = b1 * (lh - b);
    T s4 = b0 * (uh - b);
    for (int q = 0; q < A.nm; ++q) {
        const MaskSlotT<T>& M = A.R.slot[q];
        const T bq = M.beta[idx];
        s1 = s1 + bq;
        s3 = s3 + M.LI[idx] * bq;
        s4 = s4 + M.UI[idx] * bq;
    }
    A.alpha[idx] = al;
    A.z1[idx] = s1;
    A.z3[idx] = s3;
    A.z4[idx] = s4;
    A.mua[idx] = al > (T)0 ? al : A.cap_a;
    A.mub[idx] = s1 > (T)0 ? s1 : A.cap_b;
}

// zeta2_k = W_k^T beta_{k,1} + sum_q (W_k . I_q)^T beta_{k,q}, per neuron of
// layer k-1; the masks of the slots are given by their stored z bits (rows)
// and x bits (columns; a point box counts as either end).
template <typename T>
struct SpZeta2MaskArgs {
    LayerGeo g;          // layer k
    int S, nm;
    ReluLayerT<T> R;     // layer k
    const uint32_t* deg; // layer k-1 point boxes
    T* zeta2;            // layer k-1 layout
};

template <typename T>
__global__ void __launch_bounds__(kSpBlock) k_sp_zeta2_masks(SpZeta2MaskArgs<T> A) {
    const NeuronLayout& L = A.g.in;
    const long idx = (long)blockIdx.x * kSpBlock + threadIdx.x;
    if (idx >= (long)L.C * A.S * L.P) return;
    int c, s, p;
    split_index(idx, A.S, L, c, s, p);
    const long bic = (long)c * L.colpad + (long)s * L.P + p;
    const bool dg = getbit(A.deg, bic) != 0u;
    unsigned xq = 0;
    for (int q = 0; q < A.nm; ++q) xq |= getbit(A.R.slot[q].xbits, bic) << q;
    T full = 0, masked = 0;
    for_rows(A.g, A.S, c, s, p, [&](float wf, long a, long bi) {
        const T w = (T)wf;
        full += w * A.R.beta1[a];
        for (int q = 0; q < A.nm; ++q) {
            const MaskSlotT<T>& M = A.R.slot[q];
            const bool zb = getbit(M.zbits, bi) != 0u;
            const bool xb = (xq >> q) & 1u;
            // z = 1: the full row; z = 0: W+ where x is at its lower end, W-
            // where it is at its upper end (both at a point box)
            const bool bit = zb || (w >= (T)0 ? (!xb || dg) : (xb || dg));
            if (bit) masked += w * M.beta[a];
        }
    });
    A.zeta2[idx] = full + masked;
}

// ---------------------------------------------------------------------------
// Products along the rows of ReLU layer k (one thread per neuron of layer k)
// ---------------------------------------------------------------------------

template <typename T>
struct SpFwdArgs {
    LayerGeo g;                                   // layer k
    int S;
    const T* xin; const T* loin; const T* hiin;   // layer k-1: primal iterate, box
    const T* x; const T* z;                       // layer k: primal iterate
    const T* lhat; const T* uhat;
    T* alpha; T* z1; T* z3; T* z4;                // iteration: combined in place
    const T* mua; const T* mub;
    T* arow; T* brow; T* b0row;
    T gam, omg;                                   // gamma_t and 1 - gamma_t
};

// MODE 0: inner maximiser of the Big-M primal view at (x, z): alpha* -> arow,
// beta*_1 -> brow, beta*_0 -> b0row.  MODE 1: dual conditional gradient and
// its convex combination into alpha, zeta1, zeta3, zeta4; the vertex's
// row weights of zeta2 -> arow (beta_{k,1}), brow (the oracle's mask).
// Per-row accumulation of one weight: the product and, in MODE 1, the
// oracle's mask sums (eq:oracle at the iterate) with their check constants.
template <typename T, int MODE>
__device__ __forceinline__ void fwd_tap(T w, T xj, T l, T u, T zi, T& yd, T& sI, T& LI, T& UI) {
    yd += w * xj;
    if constexpr (MODE == 1) {
        if (mask_bit(w, l, u, xj, zi)) {
            sI += w * xj;
            LI += w * (w >= (T)0 ? l : u);
        } else {
            UI += w * (w >= (T)0 ? u : l);
        }
    }
}

template <typename T, int MODE>
__device__ __forceinline__ void fwd_epilogue(const SpFwdArgs<T>& A, long idx, int c, T zi, T yd, T sI, T LI, T UI) {
    const T b = (T)A.g.b[c];
    const T x = A.x[idx];
    const T lh = A.lhat[idx], uh = A.uhat[idx];
    const T xh = yd + b;
    const T va = xh - x;
    const T v0 = x - zi * uh;
    const T v1 = x - xh + ((T)1 - zi) * lh;
    if constexpr (MODE == 0) {
        A.arow[idx] = va >= (T)0 ? A.mua[idx] : (T)0;
        const bool pick1 = v1 > v0;
        const bool on = (v0 > v1 ? v0 : v1) >= (T)0;
        A.brow[idx] = on && pick1 ? A.mub[idx] : (T)0;
        A.b0row[idx] = on && !pick1 ? A.mub[idx] : (T)0;
    } else {
        // grouped so that the exact ties come out exact: at z = 1 (full row,
        // UI = 0) as beta_{k,1}'s value, at z = 0 (columns at their check
        // corners: sI and LI the same sum) as beta_{k,0}'s
        const T vI = x - ((sI - LI * ((T)1 - zi)) + zi * (b + UI));
        T best = v0;
        int ch = 0;
        if (v1 > best) { best = v1; ch = 1; }
        if (vI > best) { best = vI; ch = 2; }
        const T w = best >= (T)0 ? A.mub[idx] : (T)0;
        const T w0 = w * (T)(ch == 0), w1 = w * (T)(ch == 1), w2 = w * (T)(ch == 2);
        const T ab = va >= (T)0 ? A.mua[idx] : (T)0;
        const T gm = A.gam, om = A.omg;
        A.alpha[idx] = om * A.alpha[idx] + gm * ab;
        A.z1[idx] = om * A.z1[idx] + gm * w;
        A.z3[idx] = om * A.z3[idx] + gm * (w1 * (lh - b) + w2 * LI);
        A.z4[idx] = om * A.z4[idx] + gm * (w0 * (uh - b) + w2 * UI);
        A.arow[idx] = w1;
        A.brow[idx] = w2;
    }
}

// One thread per neuron of layer k, inputs read from global memory (any
// size of layer k-1).
template <typename T, int MODE>
__global__ void __launch_bounds__(kSpBlock) k_sp_fwd(SpFwdArgs<T> A) {
    const LayerGeo& g = A.g;
    const long idx = (long)blockIdx.x * kSpBlock + threadIdx.x;
    if (idx >= (long)g.out.C * A.S * g.out.P) return;
    int c, s, p;
    split_index(idx, A.S, g.out, c, s, p);
    const T zi = A.z[idx];
    T yd = 0, sI = 0, LI = 0, UI = 0;
    const float* Wc = g.W + (long)c * g.fan;
    TapWalk tw = tap_walk(g, p, 0);
    for (int t = 0; t < g.fan; ++t, tap_next(g, tw)) {
        const FwdTap tp = tap_at(g, A.S, s, tw);
        if (tp.a < 0) continue;  // padding
        const T l = MODE == 1 ? A.loin[tp.a] : (T)0, u = MODE == 1 ? A.hiin[tp.a] : (T)0;
        fwd_tap<T, MODE>((T)Wc[t], A.xin[tp.a], l, u, zi, yd, sI, LI, UI);
    }
    fwd_epilogue<T, MODE>(A, idx, c, zi, yd, sI, LI, UI);
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// A column of layer k-1 as staged in LDS: iterate, box and box width (the
// width u - l rounds as in the test of the oracle's bit).
template <typename T>
struct alignas(4 * sizeof(T)) SpCol {
    T x, l, u, d;
};

// Per-row accumulation of one weight from a staged column (the arithmetic of
// fwd_tap with the stored width).
template <typename T, int MODE>
__device__ __forceinline__ void fwd_tap_col(T w, const SpCol<T>& q, T zi, T& yd, T& sI, T& LI, T& UI) {
    const T p = w * q.x;
    yd += p;
    if constexpr (MODE == 1) {
        const bool bit = w >= (T)0 ? (q.l - q.x) + zi * q.d >= (T)0 : (q.u - q.x) - zi * q.d <= (T)0;
        if (bit) {
            sI += p;
            LI += w * (w >= (T)0 ? q.l : q.u);
        } else {
            UI += w * (w >= (T)0 ? q.u : q.l);
        }
    }
}

// One block per subproblem: layer k-1's iterate and box staged in LDS
// (one SpCol per neuron), then a dense layer takes one row per wave (lanes
// split the fan-in, partial sums folded across the wave) and a convolution
// one output neuron per thread; CU: every wave's outputs share one channel
// (P_k a multiple of 64), so the weights are wave-uniform (scalar loads, a
// uniform branch on their sign).
template <typename T, int MODE, bool CU>
__global__ void __launch_bounds__(kSpLdsBlock) k_sp_fwd_lds(SpFwdArgs<T> A) {
    extern __shared__ unsigned char sp_lds_raw[];
    const LayerGeo& g = A.g;
    const NeuronLayout& Li = g.in;
    const NeuronLayout& Lo = g.out;
    const int s = blockIdx.x, S = A.S;
    const long Ni = Li.N;
    SpCol<T>* col = reinterpret_cast<SpCol<T>*>(sp_lds_raw);
    for (long j = threadIdx.x; j < Ni; j += kSpLdsBlock) {
        const int c = (int)(j / Li.P), p = (int)(j - (long)c * Li.P);
        const long a = ((long)c * S + s) * Li.P + p;
        SpCol<T> q;
        q.x = A.xin[a];
        if constexpr (MODE == 1) {
            q.l = A.loin[a];
            q.u = A.hiin[a];
            q.d = q.u - q.l;
        } else {
            q.l = q.u = q.d = (T)0;
        }
        col[j] = q;
    }
    __syncthreads();
    if (g.kind == ASD_LAYER_DENSE) {
        const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
        for (int i = wave; i < Lo.C; i += kSpLdsBlock / 64) {
            const long idx = (long)i * S + s;
            const T zi = A.z[idx];
            const float* Wi = g.W + (long)i * g.fan;
            T yd = 0, sI = 0, LI = 0, UI = 0;
#pragma unroll 4
            for (int j = lane; j < g.fan; j += 64) fwd_tap_col<T, MODE>((T)Wi[j], col[j], zi, yd, sI, LI, UI);
            yd = wave_sum(yd);
            if constexpr (MODE == 1) {
                sI = wave_sum(sI);
                LI = wave_sum(LI);
                UI = wave_sum(UI);
            }
            if (lane == 0) fwd_epilogue<T, MODE>(A, idx, i, zi, yd, sI, LI, UI);
        }
    } else {
        const int ks = g.ksz;
        for (long o = threadIdx.x; o < Lo.N; o += kSpLdsBlock) {
            int c = (int)(o / Lo.P);
            if constexpr (CU) c = __builtin_amdgcn_readfirstlane(c);
            const int p = (int)(o - (long)c * Lo.P);
            const long idx = ((long)c * S + s) * Lo.P + p;
            const T zi = A.z[idx];
            const int oy = p / Lo.W, ox = p - (p / Lo.W) * Lo.W;
            const int iy0 = oy * g.stride - g.pad, ix0 = ox * g.stride - g.pad;
            // wave-uniform weights are read through the scalar cache
            const cfloat_p Wc = kconst(g.W + (long)c * g.fan);
            T yd = 0, sI = 0, LI = 0, UI = 0;
            for (int ci = 0; ci < Li.C; ++ci) {
                for (int ky = 0; ky < ks; ++ky) {
                    const int iy = iy0 + ky;
                    if (iy < 0 || iy >= Li.H) continue;
                    for (int kx = 0; kx < ks; ++kx) {
                        const int ix = ix0 + kx;
                        if (ix < 0 || ix >= Li.W) continue;
                        fwd_tap_col<T, MODE>((T)Wc[(ci * ks + ky) * ks + kx], col[ci * Li.P + iy * Li.W + ix], zi,
                                             yd, sI, LI, UI);
                    }
                }
            }
            fwd_epilogue<T, MODE>(A, idx, c, zi, yd, sI, LI, UI);
        }
    }
}

// ---------------------------------------------------------------------------
// Products along the columns (one thread per neuron j of layer L-1, reading
// the rows of layer L that take it)
// ---------------------------------------------------------------------------

template <typename T, typename Tc>
struct SpTrArgs {
    LayerGeo g;          // layer L
    int S;
    int own;             // layer L-1 is a ReLU layer (L >= 2)
    int next;            // layer L is a ReLU layer (L <= n-1)
    const T* cvec;       // L = n: objective rows (layout of layer n)
    // rows (layer L)
    const T* ralpha;     // alpha_L (BWD), alpha*_L (INIT)
    const T* rbeta1;     // beta*_{L,1} (INIT)
    const T* rz;         // z_L (STEP)
    const T* rw1; const T* rw2;  // vertex row weights (STEP)
    // columns (layer L-1)
    const T* lo; const T* hi;
    T* x; T* z;          // primal iterate (INIT: stepped; STEP: combined)
    T* xbar; T* zbar;    // primal conditional gradient (BWD, STEP: written)
    const T* alpha; const T* z1; const T* z3; const T* z4;  // own statistics (BWD)
    const T* zeta2;      // zeta2_L (BWD: read; STEP: combined in place)
    T* zeta2w;
    const T* a0; const T* b0; const T* b1;  // own inner maximiser (INIT)
    const T* lhat; const T* uhat;           // own bounds (INIT)
    const float* bown;   // bias of layer L-1 per channel
    double* term;        // BWD with the bound: per-neuron objective terms
    T gam, omg, eta;
};

// MODE 0 (BWD): f_{L-1} and the minimiser (x_bar, z_bar) of the Lagrangian
// at the current duals; with `term` also the neuron's part of d (computed in
// Tc).  MODE 1 (INIT): a projected subgradient step of the Big-M primal view
// at its inner maximiser.  MODE 3 (STEP): see step_epilogue.
template <typename T, typename Tc, int MODE>
__device__ __forceinline__ void tr_epilogue(const SpTrArgs<T, Tc>& A, long idx, int c, Tc acc1, Tc acc2) {
    const Tc lo = (Tc)A.lo[idx], hi = (Tc)A.hi[idx];
    if constexpr (MODE == 0) {
        // f = -W^T alpha_L + zeta2_L + alpha - zeta1
        Tc f = -acc1;
        if (A.next) f = f + (Tc)A.zeta2[idx];
        Tc gv = 0, al = 0, z3 = 0, bb = 0;
        if (A.own) {
            al = (Tc)A.alpha[idx];
            const Tc z1 = (Tc)A.z1[idx];
            z3 = (Tc)A.z3[idx];
            bb = (Tc)A.bown[c];
            f = f + al - z1;
            gv = z3 + (Tc)A.z4[idx] + bb * z1;
        }
        const Tc xb = f >= (Tc)0 ? hi : lo;
        const Tc zb = gv >= (Tc)0 ? (Tc)1 : (Tc)0;
        if (A.term) {
            double t = -(double)f * (double)xb;
            if (A.own) t += (double)bb * (double)al + (double)z3 - (double)gv * (double)zb;
            A.term[idx] = t;
        } else {
            A.xbar[idx] = (T)xb;
            if (A.own) A.zbar[idx] = (T)zb;
        }
    } else {
        // Big-M f (reading R4) at (alpha*, beta*): -W^T alpha*_L + W^T beta*_{L,1}
        // + alpha* - beta*_0 - beta*_1, and g = beta*_0 uhat + beta*_1 lhat
        Tc f = -acc1;
        if (A.next) f = f + acc2;
        if (A.own) f = f + ((Tc)A.a0[idx] - (Tc)A.b0[idx] - (Tc)A.b1[idx]);
        const Tc eta = (Tc)A.eta;
        const Tc xn = (Tc)A.x[idx] + eta * f;
        A.x[idx] = (T)(xn < lo ? lo : (xn > hi ? hi : xn));
        if (A.own) {
            const Tc gv = (Tc)A.b0[idx] * (Tc)A.uhat[idx] + (Tc)A.b1[idx] * (Tc)A.lhat[idx];
            const Tc zn = (Tc)A.z[idx] + eta * gv;
            A.z[idx] = (T)(zn < (Tc)0 ? (Tc)0 : (zn > (Tc)1 ? (Tc)1 : zn));
        }
    }
}

// MODE 3 (STEP), the column side of one iteration after the rows' dual
// step: zeta2_L <- (1 - gamma) zeta2_L + gamma (W_L^T w1 + (W_L . I)^T w2)
// at the iterate (x^t, z^t); the primal combination of layer L-1 with its
// conditional gradient (clipped to the boxes, a no-op in exact arithmetic
// that keeps rounding from moving an entry one unit outside its box); and
// the next primal conditional gradient from the duals just formed
// (accB = W_L^T alpha_L, or W_n^T c).
template <typename T, typename Tc>
__device__ __forceinline__ void step_epilogue(const SpTrArgs<T, Tc>& A, long idx, int c, T l, T u, T xj, T accZ,
                                              T accB) {
    T z2 = 0;
    if (A.next) {
        z2 = A.omg * A.zeta2w[idx] + A.gam * accZ;
        A.zeta2w[idx] = z2;
    }
    A.x[idx] = clip_to(A.omg * xj + A.gam * A.xbar[idx], l, u);
    T f = -accB;
    if (A.next) f = f + z2;
    T gv = 0;
    if (A.own) {
        A.z[idx] = clip_to(A.omg * A.z[idx] + A.gam * A.zbar[idx], (T)0, (T)1);
        const T z1 = A.z1[idx];
        f = f + A.alpha[idx] - z1;
        gv = A.z3[idx] + A.z4[idx] + (T)A.bown[c] * z1;
        A.zbar[idx] = gv >= (T)0 ? (T)1 : (T)0;
    }
    A.xbar[idx] = f >= (T)0 ? u : l;
}

// One thread per neuron of layer L-1, row data read from global memory.
template <typename T, typename Tc, int MODE>
__global__ void __launch_bounds__(kSpBlock) k_sp_tr(SpTrArgs<T, Tc> A) {
    const LayerGeo& g = A.g;
    const NeuronLayout& L = g.in;
    const long idx = (long)blockIdx.x * kSpBlock + threadIdx.x;
    if (idx >= (long)L.C * A.S * L.P) return;
    int c, s, p;
    split_index(idx, A.S, L, c, s, p);
    if constexpr (MODE == 3) {
        const T l = A.lo[idx], u = A.hi[idx], xj = A.x[idx];
        T accZ = 0, accB = 0;
        if (A.next) {
            for_rows(g, A.S, c, s, p, [&](float wf, long a, long) {
                const T w = (T)wf;
                const T w2 = A.rw2[a];
                accZ += w * A.rw1[a];
                if (w2 != (T)0 && mask_bit(w, l, u, xj, A.rz[a])) accZ += w * w2;
                accB += w * A.ralpha[a];
            });
        } else {
            for_rows(g, A.S, c, s, p, [&](float wf, long a, long) { accB += (T)wf * A.cvec[a]; });
        }
        step_epilogue(A, idx, c, l, u, xj, accZ, accB);
        return;
    }
    Tc acc1 = 0, acc2 = 0;
    if (A.next) {
        for_rows(g, A.S, c, s, p, [&](float wf, long a, long) {
            const Tc w = (Tc)wf;
            acc1 += w * (Tc)A.ralpha[a];
            if constexpr (MODE == 1) acc2 += w * (Tc)A.rbeta1[a];
        });
    } else {
        for_rows(g, A.S, c, s, p, [&](float wf, long a, long) { acc1 += (Tc)wf * (Tc)A.cvec[a]; });
    }
    tr_epilogue<T, Tc, MODE>(A, idx, c, acc1, acc2);
}

// Calls fn(w, r) for every output neuron r (co P_L + op, the subproblem's
// own row index) of layer L that reads input neuron (c, p) of layer L-1.
template <class Fn>
__device__ __forceinline__ void for_rows_local(const LayerGeo& g, const float* Wsrc, int c, int p, Fn&& fn) {
    const NeuronLayout& L = g.in;
    const NeuronLayout& O = g.out;
    if (g.kind == ASD_LAYER_DENSE) {
        const long j = (long)c * L.P + p;
        for (int i = 0; i < O.C; ++i) fn(g.W[(long)i * g.fan + j], i);
    } else {
        const int y = p / L.W, x = p - (p / L.W) * L.W;
        const int ks = g.ksz, str = g.stride;
        const int ky0 = (y + g.pad) % str, kx0 = (x + g.pad) % str;
        const int oyf = (y + g.pad - ky0) / str, oxf = (x + g.pad - kx0) / str;
        for (int co = 0; co < O.C; ++co) {
            int oy = oyf;
            for (int ky = ky0; ky < ks; ky += str, --oy) {
                if (oy < 0 || oy >= O.H) continue;
                int ox = oxf;
                for (int kx = kx0; kx < ks; kx += str, --ox) {
                    if (ox < 0 || ox >= O.W) continue;
                    fn(Wsrc[(((long)co * L.C + c) * ks + ky) * ks + kx], co * O.P + oy * O.W + ox);
                }
            }
        }
    }
}

// for_rows_local for a convolution of kernel size KS and stride STR known at
// compile time: the taps of each output channel unrolled, an invalid tap
// (outside the output map, or past the kernel) called with weight 0 and row
// 0, which adds only signed zeros to the caller's sums.
template <int KS, int STR, class Fn>
__device__ __forceinline__ void for_rows_conv_fixed(const LayerGeo& g, const float* Wsrc, int c, int p, Fn&& fn) {
    const NeuronLayout& L = g.in;
    const NeuronLayout& O = g.out;
    constexpr int NT = (KS + STR - 1) / STR;
    const int y = p / L.W, x = p - (p / L.W) * L.W;
    const int ky0 = (y + g.pad) % STR, kx0 = (x + g.pad) % STR;
    const int oyf = (y + g.pad - ky0) / STR, oxf = (x + g.pad - kx0) / STR;
    for (int co = 0; co < O.C; ++co) {
        const float* Wco = Wsrc + ((long)co * L.C + c) * (KS * KS);
#pragma unroll
        for (int a = 0; a < NT; ++a) {
            const int ky = ky0 + a * STR, oy = oyf - a;
            const bool vy = ky < KS && oy >= 0 && oy < O.H;
#pragma unroll
            for (int b = 0; b < NT; ++b) {
                const int kx = kx0 + b * STR, ox = oxf - b;
                const bool v = vy && kx < KS && ox >= 0 && ox < O.W;
                const float wv = Wco[v ? ky * KS + kx : 0];
                fn(v ? wv : 0.f, v ? co * O.P + oy * O.W + ox : 0);
            }
        }
    }
}

// One block per subproblem: the rows of layer L it reads staged in LDS
// (up to 3 N_L values), then one thread per neuron of layer L-1.
template <typename T, typename Tc, int MODE, bool WL, int KS = 0, int STR = 0>
__global__ void __launch_bounds__(kSpLdsBlock) k_sp_tr_lds(SpTrArgs<T, Tc> A) {
    extern __shared__ unsigned char sp_lds_raw[];
    const LayerGeo& g = A.g;
    const NeuronLayout& L = g.in;
    const NeuronLayout& O = g.out;
    const int s = blockIdx.x, S = A.S;
    const long No = O.N;
    T* r0 = reinterpret_cast<T*>(sp_lds_raw);
    T* r1 = r0 + No;
    SpCol<T>* rq = reinterpret_cast<SpCol<T>*>(sp_lds_raw);  // STEP: {w1, w2, z, alpha} per row
    for (long i = threadIdx.x; i < No; i += kSpLdsBlock) {
        const int c = (int)(i / O.P), p = (int)(i - (long)c * O.P);
        const long a = ((long)c * S + s) * O.P + p;
        if constexpr (MODE == 3) {
            if (A.next) {
                SpCol<T> q;
                q.x = A.rw1[a];
                q.l = A.rw2[a];
                q.u = A.rz[a];
                q.d = A.ralpha[a];
                rq[i] = q;
            } else {
                r0[i] = A.cvec[a];
            }
        } else if (!A.next) {
            r0[i] = A.cvec[a];
        } else {
            r0[i] = A.ralpha[a];
            if constexpr (MODE == 1) r1[i] = A.rbeta1[a];
        }
    }
    // WL: a convolution's weights follow the rows (the transposed walk reads
    // them at lane-dependent taps)
    const float* Wsrc = g.W;
    if constexpr (WL) {
        const int nrow = MODE == 3 ? (A.next ? 4 : 1) : (MODE == 1 && A.next ? 2 : 1);
        float* wl = reinterpret_cast<float*>(sp_lds_raw + (size_t)nrow * No * sizeof(T));
        const long nw = (long)O.C * g.fan;
        for (long i = threadIdx.x; i < nw; i += kSpLdsBlock) wl[i] = g.W[i];
        Wsrc = wl;
    }
    __syncthreads();
    auto rows = [&](int c, int p, auto&& fn) {
        if constexpr (KS > 0) for_rows_conv_fixed<KS, STR>(g, Wsrc, c, p, fn);
        else for_rows_local(g, Wsrc, c, p, fn);
    };
    for (long jj = threadIdx.x; jj < L.N; jj += kSpLdsBlock) {
        const int c = (int)(jj / L.P), p = (int)(jj - (long)c * L.P);
        const long idx = ((long)c * S + s) * L.P + p;
        if constexpr (MODE == 3) {
            const T l = A.lo[idx], u = A.hi[idx], xj = A.x[idx];
            T accZ = 0, accB = 0;
            if (A.next) {
                rows(c, p, [&](float wf, int r) {
                    const T w = (T)wf;
                    const SpCol<T> q = rq[r];
                    accZ += w * q.x;
                    if (q.l != (T)0 && mask_bit(w, l, u, xj, q.u)) accZ += w * q.l;
                    accB += w * q.d;
                });
            } else {
                rows(c, p, [&](float wf, int r) { accB += (T)wf * r0[r]; });
            }
            step_epilogue(A, idx, c, l, u, xj, accZ, accB);
        } else {
            Tc acc1 = 0, acc2 = 0;
            rows(c, p, [&](float wf, int r) {
                const Tc w = (Tc)wf;
                acc1 += w * (Tc)r0[r];
                if constexpr (MODE == 1) {
                    if (A.next) acc2 += w * (Tc)r1[r];
                }
            });
            if (!A.next) acc2 = 0;
            tr_epilogue<T, Tc, MODE>(A, idx, c, acc1, acc2);
        }
    }
}

// x <- x_bar, z <- z_bar (the primal iterate's start).
template <typename T>
__global__ void __launch_bounds__(kSpBlock) k_sp_copy(T* x, const T* xb, T* z, const T* zb, long n) {
    const long i = (long)blockIdx.x * kSpBlock + threadIdx.x;
    if (i >= n) return;
    x[i] = xb[i];
    if (z) z[i] = zb[i];
}

struct SpReduceArgs {
    int n, S;
    NeuronLayout L[kMaxLayers + 1];
    const double* term[kMaxLayers];
    const void* cvec;    // layout of layer n
    int c64;
    const float* bn;     // bias of layer n
    double* out;
};

// d per subproblem: c^T b_n plus the per-neuron terms of every layer (one
// block per subproblem, FP64 sums).
__global__ void __launch_bounds__(kSpBlock) k_sp_reduce(SpReduceArgs A) {
    __shared__ double red[kSpBlock];
    const int s = blockIdx.x;
    double acc = 0;
    const NeuronLayout& Ln = A.L[A.n];
    for (long j = threadIdx.x; j < Ln.N; j += kSpBlock) {
        const int c = (int)(j / Ln.P), p = (int)(j - (long)c * Ln.P);
        const long a = ((long)c * A.S + s) * Ln.P + p;
        const double cv = A.c64 ? ((const double*)A.cvec)[a] : (double)((const float*)A.cvec)[a];
        acc += cv * (double)A.bn[c];
    }
    for (int k = 0; k < A.n; ++k) {
        const NeuronLayout& L = A.L[k];
        for (long j = threadIdx.x; j < L.N; j += kSpBlock) {
            const int c = (int)(j / L.P), p = (int)(j - (long)c * L.P);
            acc += A.term[k][((long)c * A.S + s) * L.P + p];
        }
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = kSpBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) A.out[s] = red[0];
}

// Internal layout -> caller layout [S][N].
template <typename T>
__global__ void __launch_bounds__(kSpBlock) k_sp_layout(const T* src, T* dst, NeuronLayout L, int S) {
    const long idx = (long)blockIdx.x * kSpBlock + threadIdx.x;
    if (idx >= L.N * S) return;
    int c, s, p;
    split_index(idx, S, L, c, s, p);
    dst[(long)s * L.N + (long)c * L.P + p] = src[idx];
}

inline unsigned blocks_of(long n) { return (unsigned)((n + kSpBlock - 1) / kSpBlock); }

double sp_linear_lr(double lr0, double lr1, int t, int T) {
    if (T <= 1) return lr0;
    return lr0 + (lr1 - lr0) * (double)t / (double)(T - 1);
}

template <typename T>
T* arr(asd_plan* P, int k, int a) {
    return reinterpret_cast<T*>(P->sp_arr[k][a]);
}

// Elements of array a of layer k.
long sp_count(const asd_plan* P, int k, int a) {
    if (a == SA_ZETA2) return P->nl[k - 1].N * P->S;
    return P->nl[k].N * P->S;
}

bool sp_has(const asd_plan* P, int k, int a) { return k >= 1 || a == SA_X || a == SA_XBAR; }

size_t sp_layout_bytes(const asd_plan* P) {
    const size_t es = is64(P) ? 8 : 4;
    auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
    size_t off = 0;
    for (int k = 0; k < P->n; ++k) {
        for (int a = 0; a < SA_COUNT; ++a)
            if (sp_has(P, k, a)) off += al((size_t)sp_count(P, k, a) * es);
        off += al((size_t)P->nl[k].N * P->S * 8);
    }
    return off;
}

void sp_carve(asd_plan* P, void* ws) {
    const size_t es = is64(P) ? 8 : 4;
    auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
    char* base = static_cast<char*>(ws);
    size_t off = 0;
    for (int k = 0; k < P->n; ++k) {
        for (int a = 0; a < 16; ++a) P->sp_arr[k][a] = nullptr;
        for (int a = 0; a < SA_COUNT; ++a) {
            if (!sp_has(P, k, a)) continue;
            P->sp_arr[k][a] = base + off;
            off += al((size_t)sp_count(P, k, a) * es);
        }
        P->sp_term[k] = reinterpret_cast<double*>(base + off);
        off += al((size_t)P->nl[k].N * P->S * 8);
    }
}

template <typename T>
const T* cvec_of(asd_plan* P);
template <>
const float* cvec_of<float>(asd_plan* P) { return P->cvecf; }
template <>
const double* cvec_of<double>(asd_plan* P) { return P->cvecd; }

// The transposed products into layer L-1 in mode MODE.
template <typename T, typename Tc, int MODE>
asd_status launch_tr(asd_plan* P, int L, double eta, double gam, bool bound, hipStream_t st) {
    SpTrArgs<T, Tc> A{};
    A.g = P->geo[L];
    A.S = P->S;
    A.own = L >= 2;
    A.next = L <= P->n - 1;
    A.cvec = cvec_of<T>(P);
    const int k = L - 1;
    NeuronArraysT<T>& na = NA<T>(P)[k];
    A.lo = na.lo;
    A.hi = na.hi;
    A.x = arr<T>(P, k, SA_X);
    A.xbar = arr<T>(P, k, SA_XBAR);
    if (A.next) {
        A.ralpha = MODE == 1 ? arr<T>(P, L, SA_AROW) : arr<T>(P, L, SA_ALPHA);
        A.rbeta1 = arr<T>(P, L, SA_BROW);
        A.rz = arr<T>(P, L, SA_Z);
        A.rw1 = arr<T>(P, L, SA_AROW);
        A.rw2 = arr<T>(P, L, SA_BROW);
        A.zeta2 = arr<T>(P, L, SA_ZETA2);
        A.zeta2w = arr<T>(P, L, SA_ZETA2);
    }
    if (A.own) {
        A.z = arr<T>(P, k, SA_Z);
        A.zbar = arr<T>(P, k, SA_ZBAR);
        A.alpha = arr<T>(P, k, SA_ALPHA);
        A.z1 = arr<T>(P, k, SA_Z1);
        A.z3 = arr<T>(P, k, SA_Z3);
        A.z4 = arr<T>(P, k, SA_Z4);
        A.a0 = arr<T>(P, k, SA_AROW);
        A.b0 = arr<T>(P, k, SA_B0ROW);
        A.b1 = arr<T>(P, k, SA_BROW);
        A.lhat = RL<T>(P)[k].lhat;
        A.uhat = RL<T>(P)[k].uhat;
        A.bown = P->geo[k].b;
    }
    A.term = bound ? P->sp_term[k] : nullptr;
    A.gam = (T)gam;
    A.omg = (T)(1.0 - gam);
    A.eta = (T)eta;
    // rows staged per subproblem where they fit in one block's LDS
    const int nrow = MODE == 3 ? (A.next ? 4 : 1) : (MODE == 1 && A.next ? 2 : 1);  // 4: one SpCol per row
    const size_t lds = (size_t)nrow * P->nl[L].N * sizeof(T);
    const size_t wl = A.g.kind == ASD_LAYER_CONV2D ? (size_t)P->nl[L].C * A.g.fan * sizeof(float) : 0;
    const int ks = A.g.ksz, sd = A.g.stride;
    const dim3 grid((unsigned)P->S), block(kSpLdsBlock);
    if (P->sp_prm.lds_staging && wl && lds + wl <= (size_t)std::min(P->lds_max, 80 * 1024)) {
        if (ks == 4 && sd == 2)
            hipLaunchKernelGGL((k_sp_tr_lds<T, Tc, MODE, true, 4, 2>), grid, block, lds + wl, st, A);
        else if (ks == 3 && sd == 1)
            hipLaunchKernelGGL((k_sp_tr_lds<T, Tc, MODE, true, 3, 1>), grid, block, lds + wl, st, A);
        else
            hipLaunchKernelGGL((k_sp_tr_lds<T, Tc, MODE, true>), grid, block, lds + wl, st, A);
    } else if (P->sp_prm.lds_staging && lds <= (size_t)P->lds_max)
        hipLaunchKernelGGL((k_sp_tr_lds<T, Tc, MODE, false>), dim3((unsigned)P->S), dim3(kSpLdsBlock), lds, st, A);
    else
        hipLaunchKernelGGL((k_sp_tr<T, Tc, MODE>), dim3(blocks_of(P->nl[k].N * P->S)), dim3(kSpBlock), 0, st, A);
    LAUNCH_CHECK();
    return ASD_OK;
}

template <typename T, int MODE>
asd_status launch_fwd(asd_plan* P, int k, double gam, hipStream_t st) {
    SpFwdArgs<T> A{};
    A.g = P->geo[k];
    A.S = P->S;
    A.xin = arr<T>(P, k - 1, SA_X);
    A.loin = NA<T>(P)[k - 1].lo;
    A.hiin = NA<T>(P)[k - 1].hi;
    A.x = arr<T>(P, k, SA_X);
    A.z = arr<T>(P, k, SA_Z);
    A.lhat = RL<T>(P)[k].lhat;
    A.uhat = RL<T>(P)[k].uhat;
    A.alpha = arr<T>(P, k, SA_ALPHA);
    A.z1 = arr<T>(P, k, SA_Z1);
    A.z3 = arr<T>(P, k, SA_Z3);
    A.z4 = arr<T>(P, k, SA_Z4);
    A.mua = arr<T>(P, k, SA_MUA);
    A.mub = arr<T>(P, k, SA_MUB);
    A.arow = arr<T>(P, k, SA_AROW);
    A.brow = arr<T>(P, k, SA_BROW);
    A.b0row = arr<T>(P, k, SA_B0ROW);
    A.gam = (T)gam;
    A.omg = (T)(1.0 - gam);
    // layer k-1 staged per subproblem where it fits in one block's LDS
    const size_t lds = (size_t)P->nl[k - 1].N * sizeof(SpCol<T>);
    const bool cu = A.g.kind == ASD_LAYER_CONV2D && P->nl[k].P % 64 == 0;
    const bool staged = P->sp_prm.lds_staging && lds <= (size_t)P->lds_max;
    const dim3 grid((unsigned)P->S), block(kSpLdsBlock);
    if (staged && cu)
        hipLaunchKernelGGL((k_sp_fwd_lds<T, MODE, true>), grid, block, lds, st, A);
    else if (staged)
        hipLaunchKernelGGL((k_sp_fwd_lds<T, MODE, false>), grid, block, lds, st, A);
    else
        hipLaunchKernelGGL((k_sp_fwd<T, MODE>), dim3(blocks_of(P->nl[k].N * P->S)), dim3(kSpBlock), 0, st, A);
    LAUNCH_CHECK();
    return ASD_OK;
}

template <typename T>
asd_status launch_copy(asd_plan* P, int k, hipStream_t st) {
    const long n = P->nl[k].N * P->S;
    T* z = k >= 1 ? arr<T>(P, k, SA_Z) : nullptr;
    const T* zb = k >= 1 ? arr<T>(P, k, SA_ZBAR) : nullptr;
    hipLaunchKernelGGL(k_sp_copy<T>, dim3(blocks_of(n)), dim3(kSpBlock), 0, st, arr<T>(P, k, SA_X),
                       (const T*)arr<T>(P, k, SA_XBAR), z, zb, n);
    LAUNCH_CHECK();
    return ASD_OK;
}

template <typename T>
asd_status sp_init_t(asd_plan* P, hipStream_t st) {
    const asd_sp_params& q = P->sp_prm;
    for (int k = 1; k < P->n; ++k) {
        SpConvertArgs<T> A{};
        A.n = P->nl[k].N * P->S;
        A.S = P->S;
        A.L = P->nl[k];
        A.b = P->geo[k].b;
        A.R = RL<T>(P)[k];
        A.nm = P->n_masks;
        A.alpha = arr<T>(P, k, SA_ALPHA);
        A.z1 = arr<T>(P, k, SA_Z1);
        A.z3 = arr<T>(P, k, SA_Z3);
        A.z4 = arr<T>(P, k, SA_Z4);
        A.mua = arr<T>(P, k, SA_MUA);
        A.mub = arr<T>(P, k, SA_MUB);
        A.cap_a = (T)q.cap_alpha;
        A.cap_b = (T)q.cap_beta;
        hipLaunchKernelGGL(k_sp_convert<T>, dim3(blocks_of(A.n)), dim3(kSpBlock), 0, st, A);
        LAUNCH_CHECK();
        SpZeta2MaskArgs<T> Z{};
        Z.g = P->geo[k];
        Z.S = P->S;
        Z.nm = P->n_masks;
        Z.R = RL<T>(P)[k];
        Z.deg = NA<T>(P)[k - 1].deg;
        Z.zeta2 = arr<T>(P, k, SA_ZETA2);
        hipLaunchKernelGGL(k_sp_zeta2_masks<T>, dim3(blocks_of(P->nl[k - 1].N * P->S)), dim3(kSpBlock), 0, st, Z);
        LAUNCH_CHECK();
    }
    // the primal iterate starts at the minimiser of the Lagrangian, which is
    // also the first iteration's primal conditional gradient (x_bar, z_bar)
    for (int L = 1; L <= P->n; ++L) TRY((launch_tr<T, T, 0>(P, L, 0.0, 0.0, false, st)));
    for (int k = 0; k < P->n; ++k) TRY(launch_copy<T>(P, k, st));
    // App. C.2: subgradient steps on the Big-M primal view
    for (int tau = 0; tau < q.init_steps; ++tau) {
        const double eta = sp_linear_lr(q.init_lr0, q.init_lr1, tau, q.init_steps);
        for (int k = 1; k < P->n; ++k) TRY((launch_fwd<T, 0>(P, k, 0.0, st)));
        for (int L = 1; L <= P->n; ++L) TRY((launch_tr<T, T, 1>(P, L, eta, 0.0, false, st)));
    }
    return ASD_OK;
}

template <typename T>
asd_status sp_run_t(asd_plan* P, int t_begin, int n_iters, hipStream_t st) {
    for (int t = t_begin; t < t_begin + n_iters; ++t) {
        // the primal conditional gradient of iteration t is in x_bar, z_bar
        // (formed at the set-up or by the previous iteration's column pass)
        const double gam = 1.0 / ((double)t + P->sp_prm.gamma0);
        for (int k = 1; k < P->n; ++k) TRY((launch_fwd<T, 1>(P, k, gam, st)));
        for (int L = 1; L <= P->n; ++L) TRY((launch_tr<T, T, 3>(P, L, 0.0, gam, false, st)));
    }
    return ASD_OK;
}

template <typename T>
asd_status sp_bound_t(asd_plan* P, double* out, hipStream_t st) {
    for (int L = 1; L <= P->n; ++L) TRY((launch_tr<T, double, 0>(P, L, 0.0, 0.0, true, st)));
    SpReduceArgs R{};
    R.n = P->n;
    R.S = P->S;
    for (int k = 0; k <= P->n; ++k) R.L[k] = P->nl[k];
    for (int k = 0; k < P->n; ++k) R.term[k] = P->sp_term[k];
    R.cvec = cvec_of<T>(P);
    R.c64 = sizeof(T) == 8;
    R.bn = P->geo[P->n].b;
    R.out = out;
    hipLaunchKernelGGL(k_sp_reduce, dim3((unsigned)P->S), dim3(kSpBlock), 0, st, R);
    LAUNCH_CHECK();
    return ASD_OK;
}

asd_status check_sp_params(const asd_sp_params* q) {
    if (!q) return fail(ASD_EINVAL, "NULL Saddle Point params");
    if (q->iters < 0 || q->init_steps < 0) return fail(ASD_EINVAL, "negative iteration count");
    if (!(q->gamma0 >= 1.0) || !std::isfinite(q->gamma0)) return fail(ASD_EINVAL, "gamma0 must be >= 1");
    if (!(q->cap_alpha > 0.0) || !(q->cap_beta > 0.0) || !std::isfinite(q->cap_alpha) ||
        !std::isfinite(q->cap_beta))
        return fail(ASD_EINVAL, "price caps must be positive and finite");
    if (!std::isfinite(q->init_lr0) || !std::isfinite(q->init_lr1) || q->init_lr0 < 0.0 || q->init_lr1 < 0.0)
        return fail(ASD_EINVAL, "primal step sizes must be finite and >= 0");
    if (q->lds_staging != 0 && q->lds_staging != 1) return fail(ASD_EINVAL, "lds_staging must be 0 or 1");
    return ASD_OK;
}

}  // namespace

extern "C" {

void asd_sp_params_default(asd_sp_params* p) {
    if (!p) return;
    p->iters = 100;
    p->gamma0 = 10.0;
    p->init_steps = 100;
    p->init_lr0 = 1e-2;
    p->init_lr1 = 1e-5;
    p->cap_alpha = 1e-3;
    p->cap_beta = 1e-3;
    p->lds_staging = 1;
}

asd_status asd_sp_workspace_size(const asd_plan* P, size_t* bytes) {
    if (!P || !bytes) return fail(ASD_EINVAL, "NULL argument");
    *bytes = sp_layout_bytes(P);
    return ASD_OK;
}

asd_status asd_sp_init(asd_plan* P, const asd_sp_params* params, void* ws, size_t bytes, hipStream_t st) {
    if (!P || !ws) return fail(ASD_EINVAL, "NULL argument");
    if (!P->loaded) return fail(ASD_EINVAL, "asd_init has not been called");
    if (P->domain != ASD_DOMAIN_BOX) return fail(ASD_EINVAL, "Saddle Point takes box input domains only");
    TRY(check_sp_params(params));
    if ((uintptr_t)ws % 256) return fail(ASD_EINVAL, "workspace must be 256-byte aligned");
    if (bytes < sp_layout_bytes(P)) return fail(ASD_ENOMEM, "Saddle Point workspace too small");
    P->sp_ready = false;
    P->sp_prm = *params;
    sp_carve(P, ws);
    TRY(is64(P) ? sp_init_t<double>(P, st) : sp_init_t<float>(P, st));
    P->sp_ready = true;
    return ASD_OK;
}

asd_status asd_sp_run(asd_plan* P, int32_t t_begin, int32_t n_iters, hipStream_t st) {
    if (!P) return fail(ASD_EINVAL, "NULL plan");
    if (!P->sp_ready) return fail(ASD_EINVAL, "asd_sp_init has not been called for the loaded batch");
    if (t_begin < 0 || n_iters < 0) return fail(ASD_EINVAL, "negative iteration index or count");
    return is64(P) ? sp_run_t<double>(P, t_begin, n_iters, st) : sp_run_t<float>(P, t_begin, n_iters, st);
}

asd_status asd_sp_bound(asd_plan* P, double* out_lb, hipStream_t st) {
    if (!P || !out_lb) return fail(ASD_EINVAL, "NULL argument");
    if (!P->sp_ready) return fail(ASD_EINVAL, "asd_sp_init has not been called for the loaded batch");
    return is64(P) ? sp_bound_t<double>(P, out_lb, st) : sp_bound_t<float>(P, out_lb, st);
}

asd_status asd_sp_solve(asd_plan* P, const asd_sp_params* params, void* ws, size_t bytes, double* out_lb,
                        hipStream_t st) {
    if (!out_lb) return fail(ASD_EINVAL, "NULL argument");
    TRY(asd_sp_init(P, params, ws, bytes, st));
    TRY(asd_sp_run(P, 0, params->iters, st));
    return asd_sp_bound(P, out_lb, st);
}

asd_status asd_sp_read(asd_plan* P, int32_t field, int32_t k, void* dst, hipStream_t st) {
    if (!P || !dst) return fail(ASD_EINVAL, "NULL argument");
    if (!P->sp_ready) return fail(ASD_EINVAL, "asd_sp_init has not been called for the loaded batch");
    if (field < ASD_SP_X || field > ASD_SP_ZETA2) return fail(ASD_EINVAL, "unknown field %d", field);
    const bool any = field == ASD_SP_X || field == ASD_SP_XBAR;
    if (k < (any ? 0 : 1) || k >= P->n) return fail(ASD_EINVAL, "layer %d out of range", k);
    const NeuronLayout L = field == ASD_SP_ZETA2 ? P->nl[k - 1] : P->nl[k];
    const unsigned nb = blocks_of(L.N * P->S);
    if (is64(P))
        hipLaunchKernelGGL(k_sp_layout<double>, dim3(nb), dim3(kSpBlock), 0, st,
                           (const double*)P->sp_arr[k][field], (double*)dst, L, P->S);
    else
        hipLaunchKernelGGL(k_sp_layout<float>, dim3(nb), dim3(kSpBlock), 0, st,
                           (const float*)P->sp_arr[k][field], (float*)dst, L, P->S);
    LAUNCH_CHECK();
    return ASD_OK;
}

}  // extern "C"
