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

// Streaming access to the per-neuron state of the update (read and written
// once per iteration), non-temporal where measured faster: the loads with
// active masks; the stores of multipliers and moments always, those of the
// backward operands (own, g, vs, u_q) in the Big-M iterations only.
template <bool NT, typename T>
__device__ __forceinline__ T ld_stream(const T* p) {
    if constexpr (NT) return __builtin_nontemporal_load(p);
    else return *p;
}
template <bool NT, typename T>
__device__ __forceinline__ void st_stream(T* p, T v) {
    if constexpr (NT) __builtin_nontemporal_store(v, p);
    else *p = v;
}

template <typename T> __device__ __forceinline__ T flip(T x, unsigned bit) { return bit ? -x : x; }

constexpr int kPointBit = 15;

// Workgroups go to the 8 XCDs round-robin by linear id, and each XCD has its
// own L2.  Column kernels renumber their workgroups so that every XCD gets one
// contiguous range of (column tile, channel group) pairs, all channel groups
// of a column tile next to each other: tiles that read the same inputs then
// share one L2.  Returns (column tile, channel group).
// Integer division n / d for 0 <= n < 2^22 by a divisor known only at run
// time: a float reciprocal estimate, corrected once.
struct FastDiv {
    int d;
    float rcp;
};
__device__ __forceinline__ int fdiv(int n, FastDiv f) {
    int q = (int)((float)n * f.rcp);
    const int r = n - q * f.d;
    q += (r >= f.d ? 1 : 0) - (r < 0 ? 1 : 0);
    return q;
}

// Subproblem and position of column col = s P + p, in 32-bit arithmetic
// (column counts fit 31 bits: checked when the workspace is sized)
__device__ __forceinline__ int col_sub(long col, int P) { return (int)((uint32_t)col / (uint32_t)P); }

// (tile, group) of block lin of a gx x gy grid, XCD-aware: the blocks the
// hardware sends to one XCD (lin % 8) take one contiguous range of tiles.
__device__ __forceinline__ void xcd_tile_of(unsigned lin, unsigned gx, unsigned gy, int& tile, int& group) {
    const unsigned n = gx * gy;
    const unsigned x = lin & 7u, q = n >> 3, r = n & 7u;
    const unsigned logical = (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + (lin >> 3);
    tile = (int)(logical / gy);
    group = (int)(logical - (logical / gy) * gy);
}

__device__ __forceinline__ void xcd_tile(int& tile, int& group) {
    xcd_tile_of(blockIdx.y * gridDim.x + blockIdx.x, gridDim.x, gridDim.y, tile, group);
}

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
    int Sa;                     // subproblems updated: s < Sa (the geometry's
                                // column counts cover the same prefix)
    T* part;                    // dense: partial products [ksplit][1 + nm][Cpad][S]
    int freeze;                 // the slots' multipliers stay 0 (layer 1 of an l2-ball input domain)
    // evaluation at fixed duals (st.rule == kRuleEval): the supergradient
    // entries of alpha, beta_0, beta_1 and each slot's beta, caller layout
    // [S][n_k] (null: not wanted); nothing of the state is written
    T* gout[3 + kMaxMasks];
};

// Update rule of an evaluation pass (not a public asd_rule): the update
// kernels write the supergradient to FastFwdArgs::gout instead of stepping.
constexpr int kRuleEval = 2;

// Element idx = (c S + s) P + p of a layer's internal layout at its place
// (s, c, p) in the caller's row-major [S][N] layout.
__device__ __forceinline__ long caller_index(uint32_t idx, int S, const NeuronLayout& L) {
    const uint32_t sp = (uint32_t)S * (uint32_t)L.P;
    const uint32_t c = idx / sp, r = idx - c * sp;
    const uint32_t s = r / (uint32_t)L.P, p = r - s * (uint32_t)L.P;
    return (long)s * L.N + (long)c * L.P + p;
}

// State of one neuron read by the update (loads only, so that the loads of
// several neurons can be in flight together: the compiler cannot move a
// neuron's loads above an earlier neuron's stores).
template <typename T, int NM>
struct FwdIn {
    T x, lh, uh, z, bb;
    T th[3], m[3], v[3];  // alpha, beta0, beta1 and their moments
    unsigned zq;
    T LI[NM > 0 ? NM : 1], UI[NM > 0 ? NM : 1], bq[NM > 0 ? NM : 1], mq[NM > 0 ? NM : 1], vq[NM > 0 ? NM : 1];
};

// Load of element idx (< 2^30, so that its byte offset is a 32-bit value)
// from a wave-uniform base: base register plus 32-bit offset addressing.
template <typename T>
__device__ __forceinline__ T ld32(const T* base, uint32_t idx) {
    const uint32_t off = idx * (uint32_t)sizeof(T);
    return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + off);
}
// The same, non-temporal: operands staged once per block and not read again.
template <typename T>
__device__ __forceinline__ T ld32_stream(const T* base, uint32_t idx) {
    const uint32_t off = idx * (uint32_t)sizeof(T);
    return __builtin_nontemporal_load(reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + off));
}

// BF16 storage of Adam moments: round to nearest even on the FP32 bits, and
// back by placing the 16 stored bits on top (moments are finite).
__device__ __forceinline__ uint16_t bf16_rne(float f) {
    const uint32_t u = __float_as_uint(f);
    return (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}
__device__ __forceinline__ float bf16_val(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// BF16 matrix-core operands (ASD_PREC_BF16): four values rounded to BF16
// (nearest even), the operand of one lane of a v_mfma_*bf16_1k instruction.
// Slot i of that operand takes the place of the lane's operand in the i-th
// of four consecutive FP32 instructions of the same shape (32x32x2 ->
// 32x32x8, 16x16x4 -> 16x16x16, 4x4x1 -> 4x4x4), so a kernel's tap order
// carries over unchanged.
typedef short shortx4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ shortx4 bf16x4(float a, float b, float c, float d) {
    shortx4 r;
    r[0] = (short)bf16_rne(a);
    r[1] = (short)bf16_rne(b);
    r[2] = (short)bf16_rne(c);
    r[3] = (short)bf16_rne(d);
    return r;
}
__device__ __forceinline__ shortx4 bf16x4(const float* v) { return bf16x4(v[0], v[1], v[2], v[3]); }
// |v| and -v slot by slot: the sign bit of each BF16 value
__device__ __forceinline__ shortx4 bf16_abs(shortx4 v) { return v & (short)0x7fff; }
__device__ __forceinline__ shortx4 bf16_flip(shortx4 v, unsigned b0, unsigned b1, unsigned b2, unsigned b3) {
    shortx4 m;
    m[0] = (short)(b0 << 15);
    m[1] = (short)(b1 << 15);
    m[2] = (short)(b2 << 15);
    m[3] = (short)(b3 << 15);
    return v ^ m;
}

// Mixed mode (MB): the two Adam moments of a multiplier share one 32-bit
// word of the m array, m in the high and v in the low 16 bits, each BF16;
// the v array is unused.
__device__ __forceinline__ void load_moments_bf16(const float* pm, uint32_t idx, float& m, float& v) {
    const uint32_t w = reinterpret_cast<const uint32_t*>(pm)[idx];
    m = __uint_as_float(w & 0xffff0000u);
    v = __uint_as_float(w << 16);
}
__device__ __forceinline__ void store_moments_bf16(float* pm, uint32_t idx, float m, float v) {
    reinterpret_cast<uint32_t*>(pm)[idx] = ((uint32_t)bf16_rne(m) << 16) | (uint32_t)bf16_rne(v);
}

// One moment of the mixed mode (the high half of each packed word for m,
// hi = 1; the low half for v) <-> caller [S][N] floats (mode 0: set, rounding
// to BF16 and keeping the other half; mode 2: get).
static __global__ void k_layout_bf16(uint32_t* in_arr, float* ex_arr, NeuronLayout nl, int S, int mode, int hi) {
    const long col = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const int c = blockIdx.y;
    if (col >= nl.cols) return;
    const int s = col_sub(col, nl.P), p = (int)col - s * nl.P;
    const long in_ = ((long)c * S + s) * nl.P + p;
    const long ex = (long)s * nl.N + (long)c * nl.P + p;
    const uint32_t w = in_arr[in_];
    if (mode == 0) {
        const uint32_t h = bf16_rne(ex_arr[ex]);
        in_arr[in_] = hi ? ((w & 0x0000ffffu) | (h << 16)) : ((w & 0xffff0000u) | h);
    } else {
        ex_arr[ex] = bf16_val((uint16_t)(hi ? (w >> 16) : (w & 0xffffu)));
    }
}

template <typename T, int NM, bool MB>
__device__ __forceinline__ void fwd_load(const FastFwdArgs<T>& A, int c, uint32_t idx, uint32_t bi, FwdIn<T, NM>& in) {
    static_assert(!MB || sizeof(T) == 4, "BF16 moments go with FP32 duals");
    __builtin_assume(idx < (1u << 30));  // byte offsets fit 32 bits (checked at plan creation)
    const cptr_t<ReluLayerT<T>> R = kconst_t(A.R);
    const bool adam = A.st.rule == ASD_RULE_ADAM;
    in.bb = (T)A.g.b[c];
    in.x = A.xout[idx];
    in.z = (T)getbit(R->zbits, bi);
    in.lh = ld_stream<(NM > 0)>(&R->lhat[idx]);
    in.uh = ld_stream<(NM > 0)>(&R->uhat[idx]);
    in.th[0] = ld_stream<(NM > 0)>(&R->alpha[idx]);
    in.th[1] = ld_stream<(NM > 0)>(&R->beta0[idx]);
    in.th[2] = ld_stream<(NM > 0)>(&R->beta1[idx]);
    for (int j = 0; j < 3; ++j) in.m[j] = in.v[j] = (T)0;
#pragma unroll
    for (int q = 0; q < (NM > 0 ? NM : 1); ++q) in.mq[q] = in.vq[q] = (T)0;
    if (adam) {
        if constexpr (MB) {
            load_moments_bf16(R->alpha_m, idx, in.m[0], in.v[0]);
            load_moments_bf16(R->beta0_m, idx, in.m[1], in.v[1]);
            load_moments_bf16(R->beta1_m, idx, in.m[2], in.v[2]);
        } else {
            in.m[0] = ld_stream<(NM > 0)>(&R->alpha_m[idx]);
            in.v[0] = ld_stream<(NM > 0)>(&R->alpha_v[idx]);
            in.m[1] = ld_stream<(NM > 0)>(&R->beta0_m[idx]);
            in.v[1] = ld_stream<(NM > 0)>(&R->beta0_v[idx]);
            in.m[2] = ld_stream<(NM > 0)>(&R->beta1_m[idx]);
            in.v[2] = ld_stream<(NM > 0)>(&R->beta1_v[idx]);
        }
    }
    in.zq = NM > 0 ? (unsigned)R->zpk[idx] : 0u;
#pragma unroll
    for (int q = 0; q < NM; ++q) {
        const cptr_t<MaskSlotT<T>> M = &R->slot[q];
        in.LI[q] = ld_stream<(NM > 0)>(&M->LI[idx]);
        in.UI[q] = ld_stream<(NM > 0)>(&M->UI[idx]);
        in.bq[q] = ld_stream<(NM > 0)>(&M->beta[idx]);
        if (adam) {
            if constexpr (MB) {
                load_moments_bf16(M->m, idx, in.mq[q], in.vq[q]);
            } else {
                in.mq[q] = ld_stream<(NM > 0)>(&M->m[idx]);
                in.vq[q] = ld_stream<(NM > 0)>(&M->v[idx]);
            }
        }
    }
}

// Supergradient eq:as-supergradient from the products yd = (W x)[i] and
// ym[q] = (|W| (sigma_q . x))[i] + 2 (W+ x_point)[i], the projected step, the
// derived sums own, g, vs, u_q; stores only.
template <typename T, int NM, bool MB>
__device__ __forceinline__ void fwd_store(const FastFwdArgs<T>& A, uint32_t idx, int s, const FwdIn<T, NM>& in, T yd,
                                          const T* ym) {
    __builtin_assume(idx < (1u << 30));
    const cptr_t<ReluLayerT<T>> R = kconst_t(A.R);
    const StepArgsT<T>& st = A.st;
    const bool adam = st.rule != ASD_RULE_SUPERGRADIENT;
    const T x = in.x, z = in.z, bb = in.bb, lh = in.lh, uh = in.uh;
    const T xhat = yd + bb;
    T gr[3];
    gr[0] = xhat - x;
    gr[1] = x - z * uh;
    gr[2] = x - xhat + ((T)1 - z) * lh;
    // supergradient of slot q's multiplier from the masked product
    // (W . I_q) x = z_q ? yd : (yd + ym[q]) / 2
    auto gmask = [&](int q) -> T {
        const bool zb = (in.zq >> q) & 1u;
        const T mq = zb ? yd : (T)0.5 * (yd + ym[q]);
        return x - mq + in.LI[q] * ((T)1 - z) - z * bb - in.UI[q] * z;
    };
    if (st.rule == kRuleEval) {
        const long ex = caller_index(idx, A.S, A.g.out);
#pragma unroll
        for (int j = 0; j < 3; ++j)
            if (A.gout[j]) A.gout[j][ex] = gr[j];
#pragma unroll
        for (int q = 0; q < NM; ++q)
            if (A.gout[3 + q]) A.gout[3 + q][ex] = gmask(q);
        return;
    }
    // Adam: theta + (lr / (1 - b1^t)) m / (sqrt(v / (1 - b2^t)) + eps), with
    // the hardware square root and reciprocal (a few ulps in FP32)
    const T lr_s = st.lrs ? st.lrs[s] : st.lr;
    auto step = [&](T th, T m, T v, T g, int grp, T* mo, T* vo) -> T {
        if (!adam) return tmax0(th + lr_s * g);
        const T c1 = st.lrs ? lr_s * st.ib1[grp] : st.c1[grp];
        const T mm = st.b1 * m + ((T)1 - st.b1) * g;
        const T vv = st.b2 * v + ((T)1 - st.b2) * g * g;
        if constexpr (MB) {
            store_moments_bf16(mo, idx, mm, vv);
        } else {
            st_stream<true>(&mo[idx], mm);
            st_stream<true>(&vo[idx], vv);
        }
        if constexpr (sizeof(T) == 4) {
            const float den = __builtin_amdgcn_sqrtf(vv * st.ib2[grp]) + st.eps;
            return tmax0(th + c1 * mm * __builtin_amdgcn_rcpf(den));
        } else {
            return tmax0(th + c1 * mm / (tsqrt(vv * st.ib2[grp]) + st.eps));
        }
    };
    const T al = step(in.th[0], in.m[0], in.v[0], gr[0], 0, R->alpha_m, R->alpha_v);
    const T b0 = step(in.th[1], in.m[1], in.v[1], gr[1], 0, R->beta0_m, R->beta0_v);
    const T b1 = step(in.th[2], in.m[2], in.v[2], gr[2], 0, R->beta1_m, R->beta1_v);
    st_stream<true>(&R->alpha[idx], al);
    st_stream<true>(&R->beta0[idx], b0);
    st_stream<true>(&R->beta1[idx], b1);
    T own = al - b0 - b1;
    T gg = b0 * uh + b1 * lh;
    T vs = -al + b1;
#pragma unroll
    for (int q = 0; q < NM; ++q) {
        const cptr_t<MaskSlotT<T>> M = &R->slot[q];
        const bool zb = (in.zq >> q) & 1u;
        const T bq = A.freeze ? (T)0 : step(in.bq[q], in.mq[q], in.vq[q], gmask(q), 1 + q, M->m, M->v);
        st_stream<true>(&M->beta[idx], bq);
        own -= bq;
        gg += bq * (in.LI[q] + in.UI[q] + bb);
        vs += zb ? bq : (T)0.5 * bq;
        st_stream<(NM == 0)>(&M->u[idx], zb ? (T)0 : bq);
    }
    st_stream<(NM == 0)>(&R->own[idx], own);
    st_stream<(NM == 0)>(&R->g[idx], gg);
    st_stream<(NM == 0)>(&R->vs[idx], vs);
}

template <typename T, int NM, bool MB>
__device__ __forceinline__ void fwd_update(const FastFwdArgs<T>& A, int c, uint32_t idx, int s, uint32_t bi, T yd,
                                           const T* ym) {
    FwdIn<T, NM> in;
    fwd_load<T, NM, MB>(A, c, idx, bi, in);
    fwd_store<T, NM, MB>(A, idx, s, in, yd, ym);
}

// ---------------------------------------------------------------------------
// Forward pass of a convolutional ReLU layer k (column mapping).
// Grid (colpad_k / 64, ceil(C_k / CB)), block (64, KS).
// ---------------------------------------------------------------------------
// wave: this wave's index among the KSP (wave-uniform); red: KSP x CB x 64.
template <typename T, int NM, int CB, int KSZ, bool MB, int KSP>  // KSP: waves splitting the taps
__device__ __forceinline__ void fwd_conv_block(const FastFwdArgs<T>& A, int tile, int group, int wave,
                                               T (*red)[CB][kWave]) {
    static_assert(CB % KSP == 0, "CB must be a multiple of KSP");
    constexpr int EPW = CB / KSP;  // epilogue channels per wave
    constexpr int NA = NM > 0 ? NM : 1;
    const LayerGeo& g = A.g;
    const int lane = threadIdx.x;
    const long col = (long)tile * kWave + lane;
    const int c0 = group * CB;
    const int S = A.S;
    const bool colok = col < g.out.cols;
    const int s = colok ? col_sub(col, g.out.P) : 0;
    const int p = colok ? (int)col - s * g.out.P : 0;
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
    const int r0 = R * wave / KSP, r1 = R * (wave + 1) / KSP;
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
            for (int w = 0; w < KSP; ++w) a += red[w][wave * EPW + j][lane];
            tot[r][j] = a;
        }
        __syncthreads();
    }
    if (!colok) return;
    FwdIn<T, NM> in[EPW];
#pragma unroll
    for (int j = 0; j < EPW; ++j) {  // loads of every neuron first
        const int c = min(c0 + wave * EPW + j, g.out.C - 1);
        fwd_load<T, NM, MB>(A, c, ((long)c * S + s) * g.out.P + p, (long)c * g.out.colpad + col, in[j]);
    }
#pragma unroll
    for (int j = 0; j < EPW; ++j) {
        const int c = c0 + wave * EPW + j;
        if (c >= g.out.C) break;
        T ymj[NA];
#pragma unroll
        for (int q = 0; q < NM; ++q) ymj[q] = tot[1 + q][j];
        fwd_store<T, NM, MB>(A, ((long)c * S + s) * g.out.P + p, s, in[j], tot[0][j], ymj);
    }
}

template <typename T, int NM, int CB, int KSZ, bool MB>
__global__ void __launch_bounds__(kWave * KS) k_fwd_conv(FastFwdArgs<T> A) {
    __shared__ T red[KS][CB][kWave];
    int tile, group;
    xcd_tile(tile, group);
    fwd_conv_block<T, NM, CB, KSZ, MB, KS>(A, tile, group, __builtin_amdgcn_readfirstlane(threadIdx.y), red);
}

// ---------------------------------------------------------------------------
// Forward pass of a dense ReLU layer k on the matrix cores, split over the
// fan-in: every product is a GEMM, (W | |W|)[C_k x fan] times the input
// columns [fan x S] (x*_{k-1} for W, sigma_q . x*_{k-1} for |W|), tiled
// 32 x 32 with v_mfma_f32_32x32x2f32.  Operand layout of that instruction
// (lane l of 64): A[l % 32][l / 32], B[l / 32][l % 32]; accumulator register
// r holds C[8 (r / 4) + 4 (l / 32) + r % 4][l % 32].
// Grid (ceil(S / 32), Cpad / 32, ksplit), block (64, KS): the block owns one
// 32 x 32 output tile and a ksplit-th of the fan-in, its waves split that
// range again and add their tiles through LDS in a fixed order.  Writes
// partial products [ksplit][1 + NM][Cpad][S] for k_fwd_dense_epi, or, with
// one split, updates the tile's neurons itself.
// ---------------------------------------------------------------------------
typedef float floatx16 __attribute__((ext_vector_type(16)));

// The products of one trip of 4 steps of the 32 x 32 forward tiles: step u
// takes the lane's weight w[u], input x[u] and packed bits h[u]; the W
// product into acc[0], the |W| product of mask q with x sign-flipped by the
// mask's bit into acc[1 + q], the W+ product of the inputs at point boxes
// away from zero into accp.  FP32: four v_mfma_f32_32x32x2f32 per product;
// BF16: one v_mfma_f32_32x32x8bf16_1k with the four steps in its slots.
template <int NM, bool BF>
__device__ __forceinline__ void mfma_trip_32(const float* w, const float* x, const unsigned* h, bool pointin,
                                             floatx16* acc, floatx16& accp) {
    constexpr int U = 4;
    if constexpr (BF) {
        const shortx4 wb = bf16x4(w), xb = bf16x4(x);
        acc[0] = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(wb, xb, acc[0], 0, 0, 0);
        const shortx4 wa = bf16_abs(wb);
#pragma unroll
        for (int q = 0; q < NM; ++q)
            acc[1 + q] = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(
                wa, bf16_flip(xb, (h[0] >> q) & 1u, (h[1] >> q) & 1u, (h[2] >> q) & 1u, (h[3] >> q) & 1u), acc[1 + q],
                0, 0, 0);
        if (pointin) {
            float wp[U], xp[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                wp[u] = fmaxf(w[u], 0.f);
                xp[u] = ((h[u] >> kPointBit) & 1u) ? x[u] : 0.f;
            }
            accp = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(bf16x4(wp), bf16x4(xp), accp, 0, 0, 0);
        }
    } else {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            acc[0] = __builtin_amdgcn_mfma_f32_32x32x2f32(w[u], x[u], acc[0], 0, 0, 0);
            const float wabs = fabsf(w[u]);
#pragma unroll
            for (int q = 0; q < NM; ++q)
                acc[1 + q] =
                    __builtin_amdgcn_mfma_f32_32x32x2f32(wabs, flip(x[u], (h[u] >> q) & 1u), acc[1 + q], 0, 0, 0);
        }
        if (pointin) {
            // point boxes away from zero: (W . I) x gains W+ x_point on z = 0 rows
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const float xp = ((h[u] >> kPointBit) & 1u) ? x[u] : 0.f;
                accp = __builtin_amdgcn_mfma_f32_32x32x2f32(fmaxf(w[u], 0.f), xp, accp, 0, 0, 0);
            }
        }
    }
}

// UPD (one split, ksplit == 1): the block holds the whole products of its
// tile and updates its neurons itself (no partial sums, no epilogue).
template <int NM, int KW, bool UPD = false, bool MB = false, bool BF = false>  // KW: waves splitting the block's fan-in range; BF: BF16 operands
__device__ __forceinline__ void fwd_dense_mfma_block(const FastFwdArgs<float>& A, int bx, int by, int bz,
                                                     float (*red)[16][kWave]) {
    constexpr int U = 4;  // steps of 2 taps per trip
    static_assert(U == 4, "a lane's 16-byte input load holds its 4 taps of a trip");
    const LayerGeo& g = A.g;
    const int lane = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.y);
    const int S = A.S;
    const int Cp = A.Cpad;
    const int m0 = by * 32;
    const int n0 = bx * 32;
    const int F = g.fan;
    const int Pin = g.in.P;
    // input channels of a multiple of 8 positions: a lane's 4 taps of a trip
    // are consecutive positions of one channel (one 16-byte load), the taps
    // of a wave's range whole groups of 8
    const bool vec = Pin % 8 == 0 && F % 8 == 0;
    const long zr = (long)bz * KW + wave, nz = (long)A.ksplit * KW;
    const int t0 = vec ? 8 * (int)((F / 8) * zr / nz) : (int)(F * zr / nz);
    const int t1 = vec ? 8 * (int)((F / 8) * (zr + 1) / nz) : (int)(F * (zr + 1) / nz);
    const int half = lane >> 5;          // k offset of this lane within a step
    const int col = lane & 31;           // A row / B column of this lane
    const int s = min(n0 + col, S - 1);  // clamped: columns past S are computed and dropped
    const bool pointin = NM > 0 && *kconst_t<int>(A.pointflag) != 0;
    floatx16 acc[1 + NM], accp;
#pragma unroll
    for (int r = 0; r <= NM; ++r)
#pragma unroll
        for (int i = 0; i < 16; ++i) acc[r][i] = 0.f;
#pragma unroll
    for (int i = 0; i < 16; ++i) accp[i] = 0.f;
    float wv[U], xv[U];
    unsigned hv[U];
    // loads of the trip starting at tap k (lanes past t1 read tap t0 and get
    // 0): step u takes tap k + 4 half + u (vec), else k + 2 u + half
    auto load = [&](int k) {
        if (vec) {
            const int tb = k + 4 * half;
            const int tt = tb < t1 ? tb : t0;
            const int ci = tt / Pin, pp = tt - (tt / Pin) * Pin;
            const long b_idx = ((long)ci * S + s) * Pin + pp;
            const float4 x4 = *reinterpret_cast<const float4*>(A.xin + b_idx);
            xv[0] = x4.x;
            xv[1] = x4.y;
            xv[2] = x4.z;
            xv[3] = x4.w;
            if (NM > 0) {
                const uint2 h4 = *reinterpret_cast<const uint2*>(A.xpk + b_idx);
                hv[0] = h4.x & 0xffffu;
                hv[1] = h4.x >> 16;
                hv[2] = h4.y & 0xffffu;
                hv[3] = h4.y >> 16;
            } else {
#pragma unroll
                for (int u = 0; u < U; ++u) hv[u] = 0u;
            }
#pragma unroll
            for (int u = 0; u < U; ++u) wv[u] = A.Wt[(long)(tt + u) * Cp + m0 + col];
            return;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int t = k + 2 * u + half;
            const int tt = t < t1 ? t : t0;
            const int ci = tt / Pin, pp = tt - (tt / Pin) * Pin;
            const long b_idx = ((long)ci * S + s) * Pin + pp;
            wv[u] = A.Wt[(long)tt * Cp + m0 + col];
            xv[u] = A.xin[b_idx];
            hv[u] = NM > 0 ? (unsigned)A.xpk[b_idx] : 0u;
        }
    };
    if (t0 < t1) load(t0);
    for (int k = t0; k < t1; k += 2 * U) {
        float w2[U], x2[U];
        unsigned h2[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            w2[u] = wv[u];
            x2[u] = xv[u];
            h2[u] = hv[u];
        }
        if (k + 2 * U < t1) load(k + 2 * U);  // next trip's loads in flight during this trip
        // taps past the range contribute nothing
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const bool tok = (vec ? k + 4 * half + u : k + 2 * u + half) < t1;
            w2[u] = tok ? w2[u] : 0.f;
            x2[u] = tok ? x2[u] : 0.f;
        }
        mfma_trip_32<NM, BF>(w2, x2, h2, pointin, acc, accp);
    }
    // add the waves' tiles (fixed order), one product at a time; wave w
    // finishes accumulator registers 4w .. 4w + 3
    const int sw = n0 + col;
    if constexpr (UPD) {
        // the sums an epilogue would read from one split, then the update of
        // register i's neuron (channel m0 + 8 (i / 4) + 4 half + i % 4,
        // subproblem sw) as the epilogue does it
        constexpr int NR = 16 / KW;
        float tot[1 + NM][NR];
#pragma unroll
        for (int r = 0; r <= NM; ++r) {
#pragma unroll
            for (int i = 0; i < 16; ++i) red[wave][i][lane] = r == 0 ? acc[0][i] : acc[r][i] + 2.f * accp[i];
            __syncthreads();
#pragma unroll
            for (int ii = 0; ii < NR; ++ii) {
                const int i = wave * NR + ii;
                float v = 0.f;
#pragma unroll
                for (int w = 0; w < KW; ++w) v += red[w][i][lane];
                tot[r][ii] = 0.f + v;
            }
            __syncthreads();
        }
        if (sw >= A.Sa) return;  // no barrier below
#pragma unroll
        for (int ii = 0; ii < NR; ++ii) {
            const int i = wave * NR + ii;
            const int c = m0 + 8 * (i / 4) + 4 * half + (i % 4);
            if (c >= g.out.C) continue;
            float ym[NM > 0 ? NM : 1];
#pragma unroll
            for (int q = 0; q < NM; ++q) ym[q] = 0.f + tot[1 + q][ii];
            const long idx = (long)c * S + sw;  // dense layout, P = 1
            FwdIn<float, NM> in;
            fwd_load<float, NM, MB>(A, c, (uint32_t)idx, (uint32_t)((long)c * g.out.colpad + sw), in);
            fwd_store<float, NM, MB>(A, idx, sw, in, tot[0][ii], ym);
        }
        return;
    }
    const long zs = (long)bz * (1 + NM);
#pragma unroll
    for (int r = 0; r <= NM; ++r) {
#pragma unroll
        for (int i = 0; i < 16; ++i) red[wave][i][lane] = r == 0 ? acc[0][i] : acc[r][i] + 2.f * accp[i];
        __syncthreads();
#pragma unroll
        for (int ii = 0; ii < 16 / KW; ++ii) {
            const int i = wave * (16 / KW) + ii;
            float v = 0.f;
#pragma unroll
            for (int w = 0; w < KW; ++w) v += red[w][i][lane];
            const int m = m0 + 8 * (i / 4) + 4 * half + (i % 4);
            if (sw < S && m < g.out.C) A.part[((zs + r) * Cp + m) * S + sw] = v;
        }
        __syncthreads();
    }
}

template <int NM, int KW, bool UPD, bool MB, bool BF>
__global__ void __launch_bounds__(kWave * KW) k_fwd_dense_mfma(FastFwdArgs<float> A) {
    __shared__ float red[KW][16][kWave];
    fwd_dense_mfma_block<NM, KW, UPD, MB, BF>(A, blockIdx.x, blockIdx.y, blockIdx.z, red);
}

// ---------------------------------------------------------------------------
// Forward pass of a convolutional ReLU layer k on the matrix cores (implicit
// GEMM, same instruction and operand layout as the dense kernel): output tile
// = 32 channels x 32 consecutive columns (subproblem, position); B gathers
// x*_{k-1} at each column's receptive field (zero outside the image).  With
// SPLITK the 4 waves of a block split the taps of one tile and add their
// tiles through LDS in a fixed order, then each updates 4 accumulator
// registers' neurons; without it each wave owns a tile.  The update
// (fwd_update) is fused: register r of lane l is neuron (channel
// m0 + 8 (r / 4) + 4 (l / 32) + r % 4, column n0 + l % 32), so every
// register's state access is two 128-byte runs.
// Grid (column tiles / (SPLITK ? 1 : KS), Cpad / 32), block (64, KS).
// ---------------------------------------------------------------------------
template <int NM, bool SPLITK, int KSZ, bool MB, int KW, bool BF = false>  // KW: waves per block; BF: BF16 operands
__device__ __forceinline__ void fwd_conv_mfma_block(const FastFwdArgs<float>& A, int tile, int group,
                                                    float (*red)[16][kWave]) {
    constexpr int U = 4;  // steps of 2 taps per trip
    const LayerGeo& g = A.g;
    const int lane = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.y);
    const long ntile = SPLITK ? tile : (long)tile * KW + wave;
    const int m0 = group * 32;
    const long n0 = ntile * 32;
    if (!SPLITK && n0 >= g.out.cols) return;  // whole wave, no barrier below
    const int S = A.S;
    const int Cp = A.Cpad;
    const int half = lane >> 5, cl = lane & 31;
    const long col = n0 + cl;
    const bool colok = col < g.out.cols;
    const long cc = colok ? col : g.out.cols - 1;  // clamped column for the gathers
    const int s = col_sub(cc, g.out.P);
    const int p = (int)cc - s * g.out.P;
    const int oy = p / g.out.W, ox = p - (p / g.out.W) * g.out.W;
    const int ks = KSZ > 0 ? KSZ : g.ksz;
    const int ks2 = ks * ks;
    const int iy0 = oy * g.stride - g.pad, ix0 = ox * g.stride - g.pad;
    const long xbase = (long)s * g.in.P;
    const long cstride = (long)S * g.in.P;
    const int F = g.fan;
    const int t0 = SPLITK ? F * wave / KW : 0, t1 = SPLITK ? F * (wave + 1) / KW : F;
    const bool pointin = NM > 0 && *kconst_t<int>(A.pointflag) != 0;
    floatx16 acc[1 + NM], accp;
#pragma unroll
    for (int r = 0; r <= NM; ++r)
#pragma unroll
        for (int i = 0; i < 16; ++i) acc[r][i] = 0.f;
#pragma unroll
    for (int i = 0; i < 16; ++i) accp[i] = 0.f;
    float wv[U], xv[U];
    unsigned hv[U];
    bool okv[U];
    auto load = [&](int k) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int t = k + 2 * u + half;
            const bool tok = t < t1;
            const int tt = tok ? t : t0;
            const int ci = tt / ks2, rr = tt - (tt / ks2) * ks2;
            const int ky = rr / ks, kx = rr - (rr / ks) * ks;
            const int iy = iy0 + ky, ix = ix0 + kx;
            const bool ok = tok && iy >= 0 && iy < g.in.H && ix >= 0 && ix < g.in.W;
            const long b_idx = ok ? (long)ci * cstride + xbase + (long)iy * g.in.W + ix : 0;
            wv[u] = A.Wt[(long)tt * Cp + m0 + cl];
            xv[u] = A.xin[b_idx];
            hv[u] = NM > 0 ? (unsigned)A.xpk[b_idx] : 0u;
            okv[u] = ok;
        }
    };
    if (t0 < t1) load(t0);
    for (int k = t0; k < t1; k += 2 * U) {
        float w2[U], x2[U];
        unsigned h2[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            w2[u] = k + 2 * u + half < t1 ? wv[u] : 0.f;
            x2[u] = okv[u] ? xv[u] : 0.f;
            h2[u] = okv[u] ? hv[u] : 0u;
        }
        if (k + 2 * U < t1) load(k + 2 * U);  // next trip's loads in flight during this trip
        mfma_trip_32<NM, BF>(w2, x2, h2, pointin, acc, accp);
    }
#pragma unroll
    for (int q = 0; q < NM; ++q)
#pragma unroll
        for (int i = 0; i < 16; ++i) acc[1 + q][i] += 2.f * accp[i];
    constexpr int NR = SPLITK ? 16 / KW : 16;  // accumulator registers this wave updates
    float tot[1 + NM][NR];
    if constexpr (SPLITK) {
#pragma unroll
        for (int r = 0; r <= NM; ++r) {
#pragma unroll
            for (int i = 0; i < 16; ++i) red[wave][i][lane] = acc[r][i];
            __syncthreads();
#pragma unroll
            for (int ii = 0; ii < NR; ++ii) {
                float v = 0.f;
#pragma unroll
                for (int w = 0; w < KW; ++w) v += red[w][wave * NR + ii][lane];
                tot[r][ii] = v;
            }
            __syncthreads();
        }
    } else {
#pragma unroll
        for (int r = 0; r <= NM; ++r)
#pragma unroll
            for (int i = 0; i < 16; ++i) tot[r][i] = acc[r][i];
    }
    if (!colok) return;
    // update neuron by neuron: batching the loads of several neurons costs
    // registers (two waves per SIMD instead of three) and measured slower
    constexpr int NB = 1;
    static_assert(NR % NB == 0, "batch size");
#pragma unroll
    for (int b0 = 0; b0 < NR; b0 += NB) {
        FwdIn<float, NM> in[NB];
#pragma unroll
        for (int jb = 0; jb < NB; ++jb) {
            const int ii = b0 + jb;
            const int i = SPLITK ? wave * NR + ii : ii;
            const int c = min(m0 + 8 * (i / 4) + 4 * half + (i % 4), g.out.C - 1);
            fwd_load<float, NM, MB>(A, c, (long)c * S * g.out.P + col, (long)c * g.out.colpad + col, in[jb]);
        }
#pragma unroll
        for (int jb = 0; jb < NB; ++jb) {
            const int ii = b0 + jb;
            const int i = SPLITK ? wave * NR + ii : ii;
            const int c = m0 + 8 * (i / 4) + 4 * half + (i % 4);
            if (c >= g.out.C) continue;
            float ym[NM > 0 ? NM : 1];
#pragma unroll
            for (int q = 0; q < NM; ++q) ym[q] = tot[1 + q][ii];
            fwd_store<float, NM, MB>(A, (long)c * S * g.out.P + col, s, in[jb], tot[0][ii], ym);
        }
    }
}

template <int NM, bool SPLITK, int KSZ, bool MB, int KW, bool BF>
__global__ void __launch_bounds__(kWave * KW) k_fwd_conv_mfma(FastFwdArgs<float> A) {
    __shared__ float red[SPLITK ? KW : 1][16][kWave];
    int tile, group;
    xcd_tile(tile, group);
    fwd_conv_mfma_block<NM, SPLITK, KSZ, MB, KW, BF>(A, tile, group, red);
}

// The products of a dense layer (k_fwd_dense_mfma, 8 waves per split) and
// the forward pass of a convolutional layer on the matrix cores
// (k_fwd_conv_mfma, 8 waves per tile) in one launch: the two are
// independent (each reads x* of its own layers and writes its own layer's
// state or partial products), so the dense blocks, first in the grid, run
// beside the convolution's instead of before or after them.  Grid
// (nd + cgx cgy): blocks [0, nd) are the dense grid (dgx x dgy x ksplit, x
// fastest), the rest the convolution's cgx x cgy grid.  Block (64, 8).
template <int NM, int KSZ, bool MB, bool DU, bool BF>  // DU: one split, the dense blocks update
__global__ void __launch_bounds__(kWave * 8) k_fwd_conv_dense(FastFwdArgs<float> Ac, FastFwdArgs<float> Ad, int nd,
                                                              int dgx, int dgy, int cgx, int cgy) {
    __shared__ float red[8][16][kWave];
    const int lin = blockIdx.x;
    if (lin < nd) {
        const int bx = lin % dgx, rest = lin / dgx;
        fwd_dense_mfma_block<NM, 8, DU, MB, BF>(Ad, bx, rest % dgy, rest / dgy, red);
    } else {
        int tile, group;
        xcd_tile_of((unsigned)(lin - nd), (unsigned)cgx, (unsigned)cgy, tile, group);
        fwd_conv_mfma_block<NM, true, KSZ, MB, 8, BF>(Ac, tile, group, red);
    }
}

// The whole forward pass of a net with one VALU-mapped convolution, one
// convolution on the matrix cores and one dense layer in one launch: the
// three are independent (each reads x* of its own two layers and writes its
// own layer's state or partial products).  Grid (nd + nc + (nv + 1) / 2):
// the dense products' blocks (dgx x dgy x ksplit) first, then the two
// convolutions' blocks interleaved, one matrix-core block every ip blocks
// while they last (ip = 1, all matrix-core blocks first, measured fastest).
// A VALU block of the launch runs two blocks of the
// column kernel side by side, waves 0-3 and 4-7 (each 4 waves splitting
// the taps as when launched alone, both through the same barriers; the
// second one past the grid when nv is odd computes nothing it stores).
// Block (64, 8).
template <int NM, int KSC, int KSV, bool MB, bool DU, bool BF>  // DU: one split, the dense blocks update
__global__ void __launch_bounds__(kWave * 8) k_fwd_trio(FastFwdArgs<float> Av, FastFwdArgs<float> Ac,
                                                        FastFwdArgs<float> Ad, int nd, int dgx, int dgy, int nc,
                                                        int cgx, int cgy, int vgx, int vgy, int ip) {
    __shared__ float red[8][16][kWave];
    const int lin = blockIdx.x;
    if (lin < nd) {
        const int bx = lin % dgx, rest = lin / dgx;
        fwd_dense_mfma_block<NM, 8, DU, MB, BF>(Ad, bx, rest % dgy, rest / dgy, red);
        return;
    }
    const int l = lin - nd;
    const int before = min(l / ip + 1, nc);  // matrix-core positions 0, ip, 2 ip, ... up to l
    int tile, group;
    if (l % ip == 0 && l / ip < nc) {
        xcd_tile_of((unsigned)(l / ip), (unsigned)cgx, (unsigned)cgy, tile, group);
        fwd_conv_mfma_block<NM, true, KSC, MB, 8, BF>(Ac, tile, group, red);
    } else {
        const int wave = __builtin_amdgcn_readfirstlane(threadIdx.y);
        const int half = wave >> 2;
        const int v = 2 * (l - before) + half;  // < nv except in a last, half-used block
        xcd_tile_of((unsigned)min(v, vgx * vgy - 1), (unsigned)vgx, (unsigned)vgy, tile, group);
        if (v >= vgx * vgy) tile = vgx;  // past the columns: stores nothing
        fwd_conv_block<float, NM, 8, KSV, MB, KS>(Av, tile, group, wave & 3,
                                                  reinterpret_cast<float (*)[8][kWave]>(&red[4 * half][0][0]));
    }
}

// Sums the partial products in a fixed order and updates.  Grid
// (ceil(S / 256), C_k), block 256.
template <typename T, int NM, bool MB>
__global__ void __launch_bounds__(256) k_fwd_dense_epi(FastFwdArgs<T> A) {
    constexpr int NA = NM > 0 ? NM : 1;
    const int s = blockIdx.x * 256 + threadIdx.x;
    const int c = blockIdx.y;
    const int S = A.S;
    if (s >= A.Sa) return;
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
    fwd_update<T, NM, MB>(A, c, idx, s, bi, yd, ym);
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
    const float* Wb;            // convolution: class weights [group][class][nkp][16]
    const float* Wl4;           // convolution: [group][C_{k+1} k k + 1][CB] (last row zero), CB = 4
    const float* Wl8;           // and CB = 8
    int nkp;                    // taps per class (C_{k+1} J^2) rounded up to 4
    const T* cvec;              // objective rows (layout of layer n)
    const T* vs;                // layer k+1 operand of the W^T product
    const T* u[kMaxMasks];      // layer k+1 operands of the |W|^T products
    const uint16_t* xpk;        // packed bits of layer k
    NeuronArraysT<T> nk;        // layer k box and outputs
    const T* own;               // layer k (k >= 1)
    const T* gk;
    uint32_t* zbits;            // layer k (k >= 1)
    T* fout;                    // evaluation at fixed duals: f_k, caller layout [S][n_k] (else null)
};

// Finishing a neuron of layer k from its f (without own): x*, bits, in
// loads and stores so that several neurons' loads can be in flight
// together; the stores' ballots need every lane of the wave.
template <typename T>
struct BwdIn {
    T own, g, lo, hi;  // compared only when stored: a load may stay in flight until then
};

template <typename T>
__device__ __forceinline__ void bwd_load(const FastBwdArgs<T>& A, int c, long col, bool ok, uint32_t idx,
                                         BwdIn<T>& in) {
    __builtin_assume(idx < (1u << 30));
    in.own = in.g = (T)0;
    in.lo = in.hi = (T)0;
    if (!ok) return;
    if (A.k >= 1) {
        in.own = A.own[idx];
        in.g = A.gk[idx];
    }
    in.lo = A.nk.lo[idx];
    in.hi = A.nk.hi[idx];
}

template <typename T>
__device__ __forceinline__ void bwd_store(const FastBwdArgs<T>& A, bool ok, uint32_t idx, T f, const BwdIn<T>& in,
                                          long wave_base, int lane) {
    __builtin_assume(idx < (1u << 30));
    bool xb = false, zb = false;
    if (ok) {
        if (A.k >= 1) f += in.own;
        if (A.fout) A.fout[caller_index(idx, A.S, A.gn.in)] = f;
        xb = f >= (T)0 || in.lo == in.hi;  // a point box takes its value
        A.nk.xstar[idx] = xb ? in.hi : in.lo;
        if (A.k >= 1) zb = in.g >= (T)0;
    }
    put_wave_bits(A.nk.xbits, wave_base, xb, lane);
    if (A.k >= 1) put_wave_bits(A.zbits, wave_base, zb, lane);
}

// Transposed convolution (column mapping over layer k).  Grid
// (colpad_k / 64, ceil(C_k / CB)), block (64, KS); dynamic LDS holds the
// block's weights as [C_{k+1}][ks][ks][CB].  KSZ, STR > 0 fix the kernel
// size and stride (taps of one output channel unrolled), 0 = any.
template <typename T, int NM, int CB, int KSZ, int STR, int KSP>
__global__ void __launch_bounds__(kWave * KSP) k_bwd_conv(FastBwdArgs<T> A) {
    constexpr int KS = KSP;  // waves splitting the reduction (1: a wave owns all taps of its columns)
    static_assert(CB % KS == 0, "CB must be a multiple of KS");
    constexpr int EPW = CB / KS;
    constexpr int NA = NM > 0 ? NM : 1;
    extern __shared__ __attribute__((aligned(16))) float wl[];
    __shared__ T red[KS][CB][kWave];
    const LayerGeo& g = A.gn;
    const NeuronLayout& L = g.in;
    const NeuronLayout& O = g.out;
    const int lane = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.y);  // wave-uniform
    const int tid = wave * kWave + lane;
    int tile, group;
    xcd_tile(tile, group);
    const long col = (long)tile * kWave + lane;
    const int c0 = group * CB;
    const int S = A.S;
    const int ks = KSZ > 0 ? KSZ : g.ksz, st = STR > 0 ? STR : g.stride;
    const int nrow = O.C * ks * ks;
    // weights [(co * ks + ky) * ks + kx][e] of this channel group, then one
    // zero row that taps outside the output map point at (their operands are
    // then read from a valid address and multiplied by zero); laid out once
    // per plan by k_col_weights, copied here in 16-byte pieces
    {
        const float4* src = reinterpret_cast<const float4*>((CB == 4 ? A.Wl4 : A.Wl8) + (long)group * (nrow + 1) * CB);
        float4* dst = reinterpret_cast<float4*>(wl);
        const int n4 = (nrow + 1) * CB / 4;
        for (int i = tid; i < n4; i += kWave * KS) dst[i] = src[i];
    }
    __syncthreads();
    const bool colok = col < L.cols;
    const int s = colok ? col_sub(col, L.P) : 0;
    const int p = colok ? (int)col - s * L.P : 0;
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
    // this lane's packed x-bits, loaded before the products
    unsigned hb[CB];
#pragma unroll
    for (int e = 0; e < CB; ++e)
        hb[e] = NM > 0 && colok ? (unsigned)A.xpk[((long)min(c0 + e, L.C - 1) * S + s) * L.P + p] : 0u;
    // taps per axis: ky = ry + st * jy receives output row qy - jy
    const int JT = (ks + st - 1) / st;
    constexpr int J = (KSZ > 0 && STR > 0) ? (KSZ + STR - 1) / STR : 1;
    // UC output channels per trip: all their gathers are issued before the
    // first product of the trip (1: larger trips cost occupancy, measured
    // slower on the benchmark shapes)
    constexpr int UC = 1;
    if (colok) {
        for (int cu = co0; cu < co1; cu += UC) {
            for (int jy0 = 0; jy0 < JT; jy0 += J) {
                for (int jx0 = 0; jx0 < JT; jx0 += J) {
                    T vv[UC][J][J], uu[UC][NA][J][J];
                    int kk[UC][J][J];
#pragma unroll
                    for (int uc = 0; uc < UC; ++uc) {
                        const int co = min(cu + uc, co1 - 1);
                        // neuron indices fit 31 bits (checked when the
                        // workspace is sized): 32-bit offsets from the bases
                        const uint32_t obase = ((uint32_t)co * (uint32_t)S + (uint32_t)s) * (uint32_t)O.P;
#pragma unroll
                        for (int jy = 0; jy < J; ++jy) {
#pragma unroll
                            for (int jx = 0; jx < J; ++jx) {
                                const int ky = ry + st * (jy0 + jy), kx = rx + st * (jx0 + jx);
                                const int oy = qy - (jy0 + jy), ox = qx - (jx0 + jx);
                                const bool ok = cu + uc < co1 && ky < ks && kx < ks && oy >= 0 && oy < O.H &&
                                                ox >= 0 && ox < O.W;
                                const uint32_t a = ok ? obase + (uint32_t)(oy * O.W + ox) : 0u;
                                vv[uc][jy][jx] = ld32(A.vs, a);
#pragma unroll
                                for (int q = 0; q < NM; ++q) uu[uc][q][jy][jx] = ld32(A.u[q], a);
                                kk[uc][jy][jx] = ok ? (co * ks + ky) * ks + kx : nrow;  // zero row
                            }
                        }
                    }
#pragma unroll
                    for (int uc = 0; uc < UC; ++uc) {
#pragma unroll
                        for (int jy = 0; jy < J; ++jy) {
#pragma unroll
                            for (int jx = 0; jx < J; ++jx) {
                                const T v = vv[uc][jy][jx];
                                const float* wp = &wl[kk[uc][jy][jx] * CB];
#pragma unroll
                                for (int e = 0; e < CB; ++e) {
                                    acc[e] += (T)wp[e] * v;
#pragma unroll
                                    for (int q = 0; q < NM; ++q) au[q][e] += (T)fabsf(wp[e]) * uu[uc][q][jy][jx];
                                }
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
#pragma unroll
        for (int q = 0; q < NM; ++q) part += (T)0.5 * flip(au[q][e], (hb[e] >> q) & 1u);
        red[wave][e][lane] = part;
    }
    __syncthreads();
    const long wave_base = (long)tile * kWave;
    BwdIn<T> in[EPW];
#pragma unroll
    for (int j = 0; j < EPW; ++j) {  // loads of every neuron first
        const int c = min(c0 + wave * EPW + j, L.C - 1);
        bwd_load<T>(A, c, col, colok, ((long)c * S + s) * L.P + p, in[j]);
    }
#pragma unroll
    for (int j = 0; j < EPW; ++j) {
        const int e = wave * EPW + j;
        const int c = c0 + e;
        if (c >= L.C) break;  // uniform
        T f = 0;
#pragma unroll
        for (int w = 0; w < KS; ++w) f += red[w][e][lane];
        bwd_store<T>(A, colok, ((long)c * S + s) * L.P + p, f, in[j], (long)c * L.colpad + wave_base, lane);
    }
}

// Transposed convolution on the matrix cores (v_mfma_f32_16x16x4f32: lane l
// holds A[l % 16][l / 16] and B[l / 16][l % 16]; accumulator register r is
// C[4 (l / 16) + r][l % 16]).  The positions (y, x) of layer k fall into
// stride^2 parity classes ((y + pad) % st, (x + pad) % st); within a class
// every position receives output (qy - jy, qx - jx) of layer k+1 through tap
// (ry + st jy, rx + st jx), (qy, qx) = ((y + pad) / st, (x + pad) / st), so
// f over a class is a dense GEMM: A = the class's weights (16 channels x
// C_{k+1} J^2 taps, J = ceil(ks / st), zero where a tap falls outside the
// kernel), B = the operands of layer k+1 at those outputs (zero outside it).
// Grid (S, ceil(C_k / 16)), block (64, NW): a block owns one subproblem and
// 16 channels.  Work items are (class, 16 NT positions of the class), one
// per wave (NW = items, at most 8).  The operand images
// of the subproblem (v and every u_q, with a zero border of J - 1 outputs)
// are staged in LDS in chunks of CC output channels, so the B gathers are LDS
// reads; product r's images start at float r * RS (RS fixed per mask count,
// so the 1 + NM reads of one tap differ only in their immediate offsets).
// Partial f (sigma_q folded) is then parked in natural position order in a
// region of its own (float fboff on), and the waves finish 64-position runs
// (P_k % 64 == 0).
struct BwdConvShape {
    int J, off, Hp, Wp;   // taps per axis, border, staged image size
    int CC;               // output channels per staged chunk
    int items, NW;        // work items, waves per block
    int fboff;            // LDS float offset of the parked f
    FastDiv dimg, dWp;    // divisions by Hp Wp and by Wp
    FastDiv dOP, dOW;     // divisions by P_{k+1} and by W_{k+1}
};

// LDS floats reserved per product for the staged images (48 KB over the
// 1 + NM products)
template <int NM>
__host__ __device__ constexpr int bwd_mfma_rs() {
    return (12288 / (1 + NM)) & ~3;
}

// k_bwd_conv_m4 with the LDS share of two blocks per CU (78 KB): 70 KB of
// staged images over the 1 + NM products, at most 8 KB of weights after them
template <int NM>
__host__ __device__ constexpr int bwd_m4_rs_big() {
    return (17920 / (1 + NM)) & ~3;
}
constexpr int kM4BigWeightFloats = 2048;

// Stages the operand images of one subproblem for output channels
// [cb, cb + cc) of layer k+1 (v and every u_q) into the interiors of the
// images at opnd + r RS (the borders were zeroed once); UL elements per
// thread, the loads of every product in flight before the LDS stores.
template <int NM>
__device__ __forceinline__ void stage_operands(const FastBwdArgs<float>& A, const BwdConvShape& B, float* opnd,
                                               int cb, int cc, uint32_t obase, uint32_t ostride, int tid, int nthr,
                                               int RS) {
    constexpr int UL = 4;
    const NeuronLayout& O = A.gn.out;
    const int img = B.Hp * B.Wp, Wp = B.Wp, off = B.off;
    const int total = cc * O.P;
    for (int e0 = tid; e0 < total; e0 += UL * nthr) {
        uint32_t src[UL];
        int dst[UL];
#pragma unroll
        for (int u = 0; u < UL; ++u) {
            const int e = e0 + u * nthr;
            const int ee = e < total ? e : 0;
            const int col = fdiv(ee, B.dOP);
            const int pix = ee - col * O.P;
            const int oy = fdiv(pix, B.dOW), ox = pix - oy * O.W;
            // neuron indices fit 31 bits (checked when the workspace is sized)
            src[u] = (uint32_t)(cb + col) * ostride + obase + (uint32_t)pix;
            dst[u] = e < total ? col * img + (oy + off) * Wp + ox + off : -1;
        }
        float v[1 + NM][UL];
#pragma unroll
        for (int r = 0; r <= NM; ++r) {
            const float* base = r == 0 ? A.vs : A.u[r > 0 ? r - 1 : 0];
#pragma unroll
            for (int u = 0; u < UL; ++u) v[r][u] = ld32_stream(base, src[u]);
        }
#pragma unroll
        for (int u = 0; u < UL; ++u) {
            if (dst[u] < 0) continue;
#pragma unroll
            for (int r = 0; r <= NM; ++r) opnd[r * RS + dst[u]] = v[r][u];
        }
    }
}

// Transposed convolution of stride 2 into a layer of at most 4 channels on
// the matrix cores (v_mfma_f32_4x4x1_16b_f32: in each block b of 4 lanes,
// lane 4b + i supplies row i of A, lane 4b + j column j of B, and register
// r of lane 4b + j receives D[r][j]).  A = the 4 channels' weights at one
// tap, B = the operand of each lane's position at that tap, so register e
// of a lane accumulates channel e of its own position.  The lanes of a
// block must share the tap, hence the parity class: within each run of
// SW = min(W_k, 64) positions of a row the lanes take the even columns
// first, then the odd ones (W_k % 8 == 0, W_k divides 64 or 64 divides W_k).
// Grid (S), block (64, P_k / 64): a block owns one subproblem, wave w its
// positions [64 w, 64 w + 64).  The operand images of the subproblem are
// staged in LDS as for k_bwd_conv_mfma (zero borders, chunks of CC output
// channels, product r at float r RS: with BIG the LDS share of two blocks
// per CU, which holds all channels of small layers at few masks), the weights
// [C_{k+1}][ks][ks][4] (then one zero row) after them at float fboff; the
// sums go back to natural order through lane shuffles before the finishing
// stores.
template <int NM, int KSZ, bool BF = false, bool BIG = false>  // BF (4 x 4 kernels, stride 2): the 4 taps of a channel in one bf16 instruction
__global__ void __launch_bounds__(kWave * 16) k_bwd_conv_m4(FastBwdArgs<float> A, BwdConvShape B) {
    typedef float floatx4 __attribute__((ext_vector_type(4)));
    constexpr int CB = 4;
    constexpr int NA = NM > 0 ? NM : 1;
    constexpr int st = 2;
    constexpr int RS = BIG ? bwd_m4_rs_big<NM>() : bwd_mfma_rs<NM>();
    extern __shared__ __attribute__((aligned(16))) float lds[];
    const LayerGeo& g = A.gn;
    const NeuronLayout& L = g.in;
    const NeuronLayout& O = g.out;
    const int lane = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.y);
    const int nw = L.P / kWave;
    const int tid = wave * kWave + lane, nthr = kWave * nw;
    const int s = blockIdx.x;
    const int S = A.S;
    const int ks = KSZ > 0 ? KSZ : g.ksz;
    const int nrow = O.C * ks * ks;
    const int CC = B.CC, off = B.off, Wp = B.Wp, img = B.Hp * B.Wp;
    float* opnd = lds;
    float* wl = lds + B.fboff;
    // finishing inputs of this lane's natural position p2 (layer k is the
    // input: its box only), loaded right after the first chunk is staged
    // where registers allow two blocks per CU, so their latency overlaps the
    // products (which read LDS only)
    constexpr bool PRE = !BF && NM <= 2;
    const int p2 = wave * kWave + lane;
    const long ncol = (long)s * L.P + p2;
    BwdIn<float> in[CB];
    auto load_box = [&]() {
#pragma unroll
        for (int e = 0; e < CB; ++e) {
            const uint32_t idx = (uint32_t)(((long)min(e, L.C - 1) * S + s) * L.P + p2);
            in[e].own = in[e].g = 0.f;
            // the input box, read once (non-temporal: measured faster)
            in[e].lo = ld_stream<true>(&A.nk.lo[idx]);
            in[e].hi = ld_stream<true>(&A.nk.hi[idx]);
        }
    };
    {
        const float4* src = reinterpret_cast<const float4*>(A.Wl4);
        float4* dst = reinterpret_cast<float4*>(wl);
        const int n4 = (nrow + 1) * CB / 4;
        for (int i = tid; i < n4; i += nthr) dst[i] = src[i];
    }
    // zero borders: the interiors are overwritten by every chunk
#pragma unroll
    for (int r = 0; r <= NM; ++r)
        for (int i = tid; i < CC * img; i += nthr) opnd[r * RS + i] = 0.f;
    // this lane's position
    const int SW = min(L.W, kWave), half = SW >> 1;
    const int seg = lane / SW, li = lane - seg * SW;
    const int p = wave * kWave + seg * SW + (li < half ? 2 * li : 2 * (li - half) + 1);
    const int y = p / L.W, x = p - (p / L.W) * L.W;
    const int ry = (y + g.pad) % st, qy = (y + g.pad) / st;
    const int rx = (x + g.pad) % st, qx = (x + g.pad) / st;
    const int lb = (qy + off) * Wp + qx + off;  // staged image offset of tap (0, 0)
    floatx4 acc = {0.f, 0.f, 0.f, 0.f};
    floatx4 au[NA];
#pragma unroll
    for (int q = 0; q < NA; ++q) au[q] = floatx4{0.f, 0.f, 0.f, 0.f};
    // this lane's packed x-bits (channels past C_k read channel C_k - 1)
    const uint32_t nidx = (uint32_t)s * (uint32_t)L.P + (uint32_t)p, cstride = (uint32_t)S * (uint32_t)L.P;
    unsigned hb[CB];
#pragma unroll
    for (int e = 0; e < CB; ++e)
        hb[e] = NM > 0 ? (unsigned)ld32(A.xpk, (uint32_t)min(e, L.C - 1) * cstride + nidx) : 0u;
    constexpr int JC = KSZ > 0 ? (KSZ + st - 1) / st : 0;
    const int J = JC > 0 ? JC : (ks + st - 1) / st;
    auto stage = [&](int cb) {
        __syncthreads();  // the previous chunk's reads are done (and the borders zeroed)
        stage_operands<NM>(A, B, opnd, cb, min(CC, O.C - cb), (uint32_t)s * (uint32_t)O.P,
                           (uint32_t)S * (uint32_t)O.P, tid, nthr, RS);
        __syncthreads();
    };
    auto products = [&](int cb) {
        const int cc = min(CC, O.C - cb);
        for (int c = 0; c < cc; ++c) {
            const int co = cb + c;
            if constexpr (BF && JC == 2) {
                // the channel's 2 x 2 taps (jy, jx) in slots 2 jy + jx of one
                // v_mfma_f32_4x4x4bf16_1k per product
                float w4[4], o4[1 + NM][4];
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const int ty = t >> 1, tx = t & 1;
                    const int ky = ry + st * ty, kx = rx + st * tx;
                    const bool tap = ky < ks && kx < ks;
                    const int kk = tap ? (co * ks + ky) * ks + kx : nrow;  // zero row
                    w4[t] = wl[kk * CB + (lane & 3)];
                    const float* o = opnd + c * img + lb - ty * Wp - tx;
#pragma unroll
                    for (int r = 0; r <= NM; ++r) o4[r][t] = o[r * RS];
                }
                const shortx4 wb = bf16x4(w4);
                acc = __builtin_amdgcn_mfma_f32_4x4x4bf16_1k(wb, bf16x4(o4[0]), acc, 0, 0, 0);
                const shortx4 wa = bf16_abs(wb);
#pragma unroll
                for (int q = 0; q < NM; ++q)
                    au[q] = __builtin_amdgcn_mfma_f32_4x4x4bf16_1k(wa, bf16x4(o4[1 + q]), au[q], 0, 0, 0);
                continue;
            }
#pragma unroll
            for (int jy = 0; jy < (JC > 0 ? JC : 1); ++jy) {
#pragma unroll
                for (int jx = 0; jx < (JC > 0 ? JC : 1); ++jx) {
                    // fixed kernel size: the J x J taps unrolled; any size: one
                    // tap per trip of the loops below
                    for (int jy2 = 0; jy2 < (JC > 0 ? 1 : J); ++jy2) {
                        for (int jx2 = 0; jx2 < (JC > 0 ? 1 : J); ++jx2) {
                            const int ty = jy + jy2, tx = jx + jx2;
                            const int ky = ry + st * ty, kx = rx + st * tx;
                            const bool tap = ky < ks && kx < ks;  // shared by the lanes of a block
                            const int kk = tap ? (co * ks + ky) * ks + kx : nrow;  // zero row
                            const float w = wl[kk * CB + (lane & 3)];
                            const float wabs = fabsf(w);
                            const float* o = opnd + c * img + lb - ty * Wp - tx;
                            acc = __builtin_amdgcn_mfma_f32_4x4x1f32(w, o[0], acc, 0, 0, 0);
#pragma unroll
                            for (int q = 0; q < NM; ++q)
                                au[q] = __builtin_amdgcn_mfma_f32_4x4x1f32(wabs, o[(1 + q) * RS], au[q], 0, 0, 0);
                        }
                    }
                }
            }
        }
        };
    stage(0);
    if constexpr (PRE) load_box();
    products(0);
    for (int cb = CC; cb < O.C; cb += CC) {
        stage(cb);
        products(cb);
    }
    // fold sigma_q (this lane's packed x-bits), then fetch each channel's
    // sum from the lane that computed the natural position of this lane
    const int ns = lane / SW, ni = lane - ns * SW;
    const int from = ns * SW + ((ni & 1) ? half + (ni >> 1) : (ni >> 1));
    float f[CB];
#pragma unroll
    for (int e = 0; e < CB; ++e) {
        float part = acc[e];
#pragma unroll
        for (int q = 0; q < NM; ++q) part += 0.5f * flip(au[q][e], (hb[e] >> q) & 1u);
        f[e] = __shfl(part, from);
    }
    if constexpr (!PRE) load_box();
#pragma unroll
    for (int e = 0; e < CB; ++e) {
        if (e >= L.C) break;  // uniform
        bwd_store<float>(A, true, ((long)e * S + s) * L.P + p2, f[e], in[e], (long)e * L.colpad + ncol - lane, lane);
    }
}

// Finishing of rows x P_k neurons of subproblem s, channels c0 .. c0 + rows
// - 1, from f parked in fbuf [rows][P_k] (natural order), in 64-position
// runs (P_k % 64 == 0): wave w takes batches of NB runs starting at run
// NB (w + nw i), their loads in flight together.  finish_prefetch loads
// the inputs of the first PF runs of a wave's first batch before the
// products, so their latency overlaps them (PF as registers allow).
constexpr int kFinishNB = 8;

// The loads carry no branch, so a batch issues back to back: into the
// input layer (no own duals, no z) the own and g loads read the box instead,
// and bwd_store ignores them there.
template <int PF>
__device__ __forceinline__ void finish_load(const FastBwdArgs<float>& A, int s, int c0, int nrun, int ch0, int lane,
                                            BwdIn<float>* in) {
    const NeuronLayout& L = A.gn.in;
    const int runs = L.P / kWave;
    const float* po = A.k >= 1 ? A.own : A.nk.lo;
    const float* pg = A.k >= 1 ? A.gk : A.nk.lo;
#pragma unroll
    for (int b = 0; b < PF; ++b) {
        const int ch = min(ch0 + b, nrun - 1);
        const int c = ch / runs;
        const int p = (ch - c * runs) * kWave + lane;
        const uint32_t idx = (uint32_t)(((long)(c0 + c) * A.S + s) * L.P + p);
        in[b].own = po[idx];
        in[b].g = pg[idx];
        in[b].lo = A.nk.lo[idx];
        in[b].hi = A.nk.hi[idx];
    }
}

template <int PF>
__device__ __forceinline__ void finish_prefetch(const FastBwdArgs<float>& A, int s, int c0, int rows, int wave,
                                                int lane, BwdIn<float> (&pre)[PF > 0 ? PF : 1]) {
    const int nrun = rows * (A.gn.in.P / kWave);
    if constexpr (PF > 0) finish_load<PF>(A, s, c0, nrun, min(wave * kFinishNB, nrun - 1), lane, pre);
}

template <int PF>
__device__ __forceinline__ void finish_runs(const FastBwdArgs<float>& A, const float* fbuf, int s, int c0, int rows,
                                            int wave, int nw, int lane, const BwdIn<float> (&pre)[PF > 0 ? PF : 1]) {
    static_assert(PF <= kFinishNB, "at most one batch is prefetched");
    const NeuronLayout& L = A.gn.in;
    const int S = A.S;
    const int runs = L.P / kWave;
    const int nrun = rows * runs;
    for (int ch0 = wave * kFinishNB; ch0 < nrun; ch0 += nw * kFinishNB) {
        BwdIn<float> in[kFinishNB];
        if (ch0 == wave * kFinishNB) {
#pragma unroll
            for (int b = 0; b < PF; ++b) in[b] = pre[b];
            finish_load<kFinishNB - PF>(A, s, c0, nrun, ch0 + PF, lane, in + PF);
        } else {
            finish_load<kFinishNB>(A, s, c0, nrun, ch0, lane, in);
        }
#pragma unroll
        for (int b = 0; b < kFinishNB; ++b) {
            const int ch = ch0 + b;
            if (ch >= nrun) break;  // uniform
            const int c = ch / runs;
            const int p = (ch - c * runs) * kWave + lane;
            const long col = (long)s * L.P + p;
            bwd_store<float>(A, true, ((long)(c0 + c) * S + s) * L.P + p, fbuf[c * L.P + p], in[b],
                             (long)(c0 + c) * L.colpad + col - lane, lane);
        }
    }
}

// WL (one round of items, all output channels in one chunk): the block's
// class weights are staged in LDS too (at float fboff) and f is parked over
// the staged images, so the products read LDS only; the finishing inputs
// of each wave's first runs are loaded right after the staging, and their
// latency overlaps the products (a wait for a later vector load would wait
// for them as well).
template <int NM, int KSZ, int STR, int NT, bool BF = false, bool WL = false>  // NT: column tiles of 16 per item; BF: BF16 operands
__global__ void __launch_bounds__(kWave * 8) k_bwd_conv_mfma(FastBwdArgs<float> A, BwdConvShape B) {
    typedef float floatx4 __attribute__((ext_vector_type(4)));
    extern __shared__ __attribute__((aligned(16))) float lds[];
    const LayerGeo& g = A.gn;
    const NeuronLayout& L = g.in;
    const NeuronLayout& O = g.out;
    const int lane = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.y);
    const int NW = B.NW;
    const int tid = wave * kWave + lane;
    const int S = A.S;
    const int s = blockIdx.x;
    const int grp = blockIdx.y;
    const int c0 = grp * 16;
    const int rows = min(16, L.C - c0);
    const int ks = KSZ > 0 ? KSZ : g.ksz;
    const int st = STR > 0 ? STR : g.stride;
    const int pd = g.pad;
    constexpr int JC = (KSZ > 0 && STR > 0) ? (KSZ + STR - 1) / STR : 0;  // taps per axis if fixed
    const int J = JC > 0 ? JC : B.J, J2 = J * J, off = B.off, Wp = B.Wp, img = B.Hp * B.Wp;
    const int nkp = A.nkp;
    const int r4 = lane >> 4, cl = lane & 15;
    const int CC = B.CC;
    constexpr int RS = bwd_mfma_rs<NM>();
    float* opnd = lds;                       // product r: [CC][Hp][Wp] at float r RS
    float* fbuf = WL ? lds : lds + B.fboff;  // [rows][P_k]
    const float* wlds = lds + B.fboff;       // WL: class weights [class][nkp][16]
    const uint32_t obase = (uint32_t)s * (uint32_t)O.P;
    const uint32_t ostride = (uint32_t)S * (uint32_t)O.P;
    if constexpr (WL) {
        const float4* src = reinterpret_cast<const float4*>(A.Wb + (long)grp * st * st * nkp * 16);
        float4* dst = reinterpret_cast<float4*>(lds + B.fboff);
        const int n4 = st * st * nkp * 4;
        for (int i = tid; i < n4; i += kWave * NW) dst[i] = src[i];
    }
    // zero borders: the interiors are overwritten by every chunk
#pragma unroll
    for (int r = 0; r <= NM; ++r)
        for (int i = tid; i < CC * img; i += kWave * NW) opnd[r * RS + i] = 0.f;
    // WL (all output channels in one chunk): stage once, then load the
    // finishing inputs of the first runs, as many as leave 4 waves per SIMD
    constexpr int PF = WL ? (NT == 2 ? (NM <= 2 ? 8 : NM == 3 ? 4 : 0) : 0) : 0;
    BwdIn<float> pre[PF > 0 ? PF : 1];
    if constexpr (WL) {
        __syncthreads();
        stage_operands<NM>(A, B, opnd, 0, O.C, obase, ostride, tid, kWave * NW, RS);
        __syncthreads();
        finish_prefetch<PF>(A, s, c0, rows, wave, lane, pre);
    }
    {
        // find this wave's item (the host launches one wave per item): class
        // cls, first position n0 within the class
        const int item = wave;
        int cls = -1, n0 = 0, cnt = 0, yf = 0, xf = 0, nx = 1;
        {
            int idx = 0;
            for (int c = 0; c < st * st && cls < 0; ++c) {
                const int ry = c / st, rx = c - (c / st) * st;
                const int yf_ = ((ry - pd) % st + st) % st, xf_ = ((rx - pd) % st + st) % st;
                const int ny_ = yf_ < L.H ? (L.H - 1 - yf_) / st + 1 : 0;
                const int nx_ = xf_ < L.W ? (L.W - 1 - xf_) / st + 1 : 0;
                const int cnt_ = ny_ * nx_;
                const int groups = (cnt_ + NT * 16 - 1) / (NT * 16);
                if (item < idx + groups) {
                    cls = c;
                    n0 = (item - idx) * NT * 16;
                    cnt = cnt_;
                    yf = yf_;
                    xf = xf_;
                    nx = nx_;
                }
                idx += groups;
            }
        }
        const bool has = cls >= 0;  // uniform
        int qy[NT], qx[NT], pos[NT];
        bool nok[NT];
#pragma unroll
        for (int j = 0; j < NT; ++j) {
            const int n = n0 + j * 16 + cl;
            nok[j] = has && n < cnt;
            const int nn = nok[j] ? n : 0;
            const int iy = nn / nx, ix = nn - (nn / nx) * nx;
            const int y = yf + st * iy, x = xf + st * ix;
            qy[j] = (y + pd) / st + off;  // staged-image coordinates of tap jy = 0
            qx[j] = (x + pd) / st + off;
            pos[j] = y * L.W + x;
        }
        floatx4 acc[NT][1 + NM];
#pragma unroll
        for (int j = 0; j < NT; ++j)
#pragma unroll
            for (int r = 0; r <= NM; ++r) acc[j][r] = floatx4{0.f, 0.f, 0.f, 0.f};
        // the packed x-bits of this lane's neurons, loaded now so their latency
        // overlaps the products
        unsigned hb[NT][4];
#pragma unroll
        for (int j = 0; j < NT; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int c = min(4 * r4 + r, rows - 1);
                hb[j][r] = NM > 0 ? (unsigned)A.xpk[((long)(c0 + c) * S + s) * L.P + pos[j]] : 0u;
            }
        const float* Wc = WL ? wlds + (long)(has ? cls : 0) * nkp * 16
                             : A.Wb + ((long)grp * st * st + (has ? cls : 0)) * nkp * 16;
        for (int cb = 0; cb < O.C; cb += CC) {
            const int cc = min(CC, O.C - cb);
            if constexpr (!WL) {
                __syncthreads();  // the previous chunk's reads are done
                stage_operands<NM>(A, B, opnd, cb, cc, obase, ostride, tid, kWave * NW, RS);
                __syncthreads();
            }
            if (!has) continue;
            if constexpr (JC == 2) {
                // J = 2: a step of 4 taps is one output channel; lane r4
                // takes tap (jy, jx) = (r4 / 2, r4 % 2) of every channel, so
                // its B reads sit at a fixed offset from the channel's image
                int lb[NT];
#pragma unroll
                for (int j = 0; j < NT; ++j) lb[j] = (qy[j] - (r4 >> 1)) * Wp + qx[j] - (r4 & 1);
                const float* wp = Wc + ((long)cb * 4 + r4) * 16 + cl;  // + 64 per output channel
                constexpr int U = BF ? 8 : (WL || NM >= 4) ? 4 : 6;  // channels whose weights are loaded ahead
                float wq[U];
                auto wload = [&](int c) {
#pragma unroll
                    for (int u = 0; u < U; ++u) wq[u] = wp[(long)min(c + u, cc - 1) * 64];
                };
                wload(0);
                for (int c = 0; c < cc; c += U) {
                    float w2[U];
#pragma unroll
                    for (int u = 0; u < U; ++u) w2[u] = wq[u];
                    if (c + U < cc) wload(c + U);
                    if constexpr (BF) {
                        // channels c + u0 .. c + u0 + 3 in the slots of one
                        // v_mfma_f32_16x16x16bf16_1k (channels past cc: zero
                        // weight, a staged channel's operand)
#pragma unroll
                        for (int u0 = 0; u0 < U; u0 += 4) {
                            if (c + u0 >= cc) break;  // uniform
                            float w4[4];
                            int cofs[4];
#pragma unroll
                            for (int jj = 0; jj < 4; ++jj) {
                                const bool cok = c + u0 + jj < cc;
                                w4[jj] = cok ? w2[u0 + jj] : 0.f;
                                cofs[jj] = min(c + u0 + jj, cc - 1) * img;
                            }
                            const shortx4 wb = bf16x4(w4);
                            const shortx4 wa = bf16_abs(wb);
#pragma unroll
                            for (int j = 0; j < NT; ++j) {
                                const float* o = opnd + lb[j];
                                acc[j][0] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(
                                    wb, bf16x4(o[cofs[0]], o[cofs[1]], o[cofs[2]], o[cofs[3]]), acc[j][0], 0, 0, 0);
#pragma unroll
                                for (int q = 0; q < NM; ++q) {
                                    const float* oq = o + (1 + q) * RS;
                                    acc[j][1 + q] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(
                                        wa, bf16x4(oq[cofs[0]], oq[cofs[1]], oq[cofs[2]], oq[cofs[3]]), acc[j][1 + q],
                                        0, 0, 0);
                                }
                            }
                        }
                        continue;
                    }
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        if (c + u >= cc) break;  // uniform
                        const float wa = w2[u];
                        const float wabs = fabsf(wa);
                        const int cofs = (c + u) * img;
#pragma unroll
                        for (int j = 0; j < NT; ++j) {
                            const float* o = opnd + lb[j] + cofs;
                            acc[j][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(wa, o[0], acc[j][0], 0, 0, 0);
#pragma unroll
                            for (int q = 0; q < NM; ++q)
                                acc[j][1 + q] = __builtin_amdgcn_mfma_f32_16x16x4f32(wabs, o[(1 + q) * RS],
                                                                                     acc[j][1 + q], 0, 0, 0);
                        }
                    }
                }
                continue;
            }
            // any J: steps of 4 taps; the weights of the next U steps are
            // loaded while this trip's products run
            const int kbeg = cb * J2, kend = (cb + cc) * J2;
            constexpr int U = 8;
            float wq[U];
            auto wload = [&](int kt) {
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int k = kt + 4 * u + r4;
                    wq[u] = Wc[(long)(k < kend ? k : kbeg) * 16 + cl];
                }
            };
            wload(kbeg);
            for (int kt = kbeg; kt < kend; kt += 4 * U) {
                float w2[U];
#pragma unroll
                for (int u = 0; u < U; ++u) w2[u] = kt + 4 * u + r4 < kend ? wq[u] : 0.f;
                if (kt + 4 * U < kend) wload(kt + 4 * U);
                if constexpr (BF) {
                    // steps u0 .. u0 + 3 in the slots of one bf16 instruction
                    // (steps past kend: zero weight, the first tap's operand)
#pragma unroll
                    for (int u0 = 0; u0 < U; u0 += 4) {
                        if (kt + 4 * u0 >= kend) break;  // uniform
                        int li[NT][4];
#pragma unroll
                        for (int jj = 0; jj < 4; ++jj) {
                            const int k = kt + 4 * (u0 + jj) + r4;
                            const int kk = k < kend ? k : kbeg;
                            const int col = kk / J2 - cb, rem = kk - (kk / J2) * J2;
                            const int jy = rem / J, jx = rem - (rem / J) * J;
                            const int ib = col * img - jy * Wp - jx;
#pragma unroll
                            for (int j = 0; j < NT; ++j) li[j][jj] = ib + qy[j] * Wp + qx[j];
                        }
                        const shortx4 wb = bf16x4(&w2[u0]);
                        const shortx4 wa = bf16_abs(wb);
#pragma unroll
                        for (int j = 0; j < NT; ++j) {
                            acc[j][0] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(
                                wb, bf16x4(opnd[li[j][0]], opnd[li[j][1]], opnd[li[j][2]], opnd[li[j][3]]), acc[j][0],
                                0, 0, 0);
#pragma unroll
                            for (int q = 0; q < NM; ++q) {
                                const float* oq = opnd + (1 + q) * RS;
                                acc[j][1 + q] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(
                                    wa, bf16x4(oq[li[j][0]], oq[li[j][1]], oq[li[j][2]], oq[li[j][3]]), acc[j][1 + q],
                                    0, 0, 0);
                            }
                        }
                    }
                    continue;
                }
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    if (kt + 4 * u >= kend) break;  // uniform
                    const int k = kt + 4 * u + r4;
                    const int kk = k < kend ? k : kbeg;
                    const int col = kk / J2 - cb, rem = kk - (kk / J2) * J2;
                    const int jy = rem / J, jx = rem - (rem / J) * J;
                    const float wa = w2[u];
                    const float wabs = fabsf(wa);
                    const int ib = col * img - jy * Wp - jx;
#pragma unroll
                    for (int j = 0; j < NT; ++j) {
                        const int li = ib + qy[j] * Wp + qx[j];
                        acc[j][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(wa, opnd[li], acc[j][0], 0, 0, 0);
#pragma unroll
                        for (int q = 0; q < NM; ++q)
                            acc[j][1 + q] = __builtin_amdgcn_mfma_f32_16x16x4f32(wabs, opnd[(1 + q) * RS + li],
                                                                                 acc[j][1 + q], 0, 0, 0);
                    }
                }
            }
        }
        // fold sigma_q of each neuron and park f in natural order (WL: over
        // the staged images, once every wave's products are done)
        if constexpr (WL) __syncthreads();
        if (has) {
#pragma unroll
            for (int j = 0; j < NT; ++j) {
                if (!nok[j]) continue;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int c = 4 * r4 + r;
                    if (c >= rows) continue;
                    float f = acc[j][0][r];
#pragma unroll
                    for (int q = 0; q < NM; ++q) f += 0.5f * flip(acc[j][1 + q][r], (hb[j][r] >> q) & 1u);
                    fbuf[c * L.P + pos[j]] = f;
                }
            }
        }
    }
    __syncthreads();
    finish_runs<PF>(A, fbuf, s, c0, rows, wave, NW, lane, pre);
}

// Class weights for k_bwd_conv_mfma: Wb[grp][cls][k][c] = W[co][16 grp + c][ky][kx]
// with k = (co J + jy) J + jx, ky = ry + st jy, kx = rx + st jx, zero past
// the kernel, past C_k or past C_{k+1} J^2.
// Weights of a convolution in the column transposed kernel's LDS layout:
// Wl[group][(co * k + ky) * k + kx][e] = W[co][group * cb + e][ky][kx] (zero
// past C_in), then one zero row per group.
static __global__ void __launch_bounds__(256) k_col_weights(const float* W, float* Wl, int Cin, int Cout, int kk2, int cb,
                                                     long n) {
    const long i = (long)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const int rows = Cout * kk2 + 1;
    const int e = (int)(i % cb);
    const long rest = i / cb;
    const int grp = (int)(rest / rows), row = (int)(rest - (long)grp * rows);
    const int c = grp * cb + e;
    const int co = row / kk2, kk = row - co * kk2;
    Wl[i] = (row < rows - 1 && c < Cin) ? W[((long)co * Cin + c) * kk2 + kk] : 0.f;
}

static __global__ void __launch_bounds__(256) k_class_weights(const float* W, float* Wb, int Ck, int C1, int ks, int st,
                                                       int nkp, long n) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int c = (int)(i % 16);
    const long r1 = i / 16;
    const int k = (int)(r1 % nkp);
    const long r2 = r1 / nkp;
    const int cls = (int)(r2 % (st * st));
    const int grp = (int)(r2 / (st * st));
    const int J = (ks + st - 1) / st;
    const int ry = cls / st, rx = cls % st;
    const int co = k / (J * J), jy = (k / J) % J, jx = k % J;
    const int ky = ry + st * jy, kx = rx + st * jx;
    const int cc = grp * 16 + c;
    float v = 0.f;
    if (co < C1 && ky < ks && kx < ks && cc < Ck) v = W[(((long)co * Ck + cc) * ks + ky) * ks + kx];
    Wb[i] = v;
}

// Dense layer k+1 into layer k, column mapping (any P_k; P1 = (P_k == 1),
// when the weights are wave-uniform scalar loads).  Grid (colpad_k / 64,
// ceil(C_k / CB)), block (64, KS), the outputs of layer k+1 split over waves.
template <typename T, int NM, int CB, bool P1>
__device__ __forceinline__ void bwd_dense_block(const FastBwdArgs<T>& A, int tile, int group, T (*red)[CB][kWave]) {
    static_assert(CB % KS == 0, "CB must be a multiple of KS");
    constexpr int EPW = CB / KS;
    constexpr int NA = NM > 0 ? NM : 1;
    const LayerGeo& g = A.gn;
    const NeuronLayout& L = g.in;
    const int lane = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.y);  // wave-uniform
    const long col = (long)tile * kWave + lane;
    const int c0 = group * CB;
    const int S = A.S;
    const bool colok = col < L.cols;
    const int s = colok ? col_sub(col, L.P) : 0;
    const int p = colok ? (int)col - s * L.P : 0;
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
    const long wave_base = (long)tile * kWave;
    BwdIn<T> in[EPW];
#pragma unroll
    for (int j = 0; j < EPW; ++j) {  // loads of every neuron first
        const int c = min(c0 + wave * EPW + j, L.C - 1);
        bwd_load<T>(A, c, col, colok, ((long)c * S + s) * L.P + p, in[j]);
    }
#pragma unroll
    for (int j = 0; j < EPW; ++j) {
        const int e = wave * EPW + j;
        const int c = c0 + e;
        if (c >= L.C) break;  // uniform
        T f = 0;
#pragma unroll
        for (int w = 0; w < KS; ++w) f += red[w][e][lane];
        bwd_store<T>(A, colok, ((long)c * S + s) * L.P + p, f, in[j], (long)c * L.colpad + wave_base, lane);
    }
}

template <typename T, int NM, int CB, bool P1>
__global__ void __launch_bounds__(kWave * KS) k_bwd_dense(FastBwdArgs<T> A) {
    __shared__ T red[KS][CB][kWave];
    int tile, group;
    xcd_tile(tile, group);
    bwd_dense_block<T, NM, CB, P1>(A, tile, group, red);
}

// Dense layer k+1 into a layer k whose positions come in whole wavefronts
// (P_k % 64 == 0): lanes = 64 positions of one channel, each thread SB
// consecutive subproblems whose operands are wave-uniform scalar loads (the
// last tile is shifted back to end at S, so S >= SB).  Grid
// (C_k * P_k / 64, ceil(S / SB)), block (64, KS), the outputs of layer k+1
// split over waves.
template <typename T, int NM, int SB, int KW>  // KW: waves splitting the outputs of layer k+1
__global__ void __launch_bounds__(kWave * KW) k_bwd_dense_pos(FastBwdArgs<T> A) {
    static_assert(SB % KW == 0, "SB must be a multiple of KW");
    constexpr int EPW = SB / KW;
    constexpr int NA = NM > 0 ? NM : 1;
    __shared__ T red[KW][SB][kWave];
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
    const int i0 = n1 * wave / KW, i1 = n1 * (wave + 1) / KW;
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
    BwdIn<T> in[EPW];
#pragma unroll
    for (int jj = 0; jj < EPW; ++jj) {  // loads of every neuron first
        const int s = sb + wave * EPW + jj;
        bwd_load<T>(A, c, (long)s * L.P + p, true, ((long)c * S + s) * L.P + p, in[jj]);
    }
#pragma unroll
    for (int jj = 0; jj < EPW; ++jj) {
        const int j = wave * EPW + jj;
        const int s = sb + j;
        if (s < s0) continue;  // uniform: computed by the previous tile
        T f = 0;
#pragma unroll
        for (int w = 0; w < KW; ++w) f += red[w][j][lane];
        const long idx = ((long)c * S + s) * L.P + p;
        bwd_store<T>(A, true, idx, f, in[jj], (long)c * L.colpad + (long)s * L.P + (p - lane), lane);
    }
}

// Dense layer k+1 into a layer k whose positions come in runs of 64 (P_k %
// 64 == 0) on the matrix cores (v_mfma_f32_16x16x4f32: lane l holds
// A[l % 16][l / 16] and B[l / 16][l % 16]; register r is
// C[4 (l / 16) + r][l % 16]).  A wave owns C = f over 16 subproblems (rows)
// x 16 positions of one channel (columns) and the whole contraction over
// the outputs of layer k+1: A = the operands of layer k+1 (v, or -c into
// the output layer's inputs, and every u_q) at those subproblems, B = W
// (|W| for the u_q) at those positions.  The four waves of a block share
// the subproblems, so the block stages their operands in LDS, KC outputs
// of layer k+1 at a time ([1 + NM][KC][16], zero past the last output),
// with every load of a chunk in flight together; the weights of the next
// trip of U steps are loaded during the current one.  The x-bits and the
// finishing inputs of the wave's neurons are loaded before the products, so
// their latency overlaps them; rows past the active subproblems are
// computed on clamped operands and dropped.  The bits of one register's 16
// positions of one subproblem are one 16-bit piece of the bit array.  Grid
// (ceil(Sa / 16), C_k P_k / 64), block (64, 4): wave w takes positions
// [16 w, 16 w + 16) of the block's 64.
template <int NM>
__host__ __device__ constexpr int bwd_dense_kc() {
    return NM <= 2 ? 128 : 64;
}
template <int NM>
__host__ __device__ constexpr int bwd_dense_lds_floats() {
    return (1 + NM) * bwd_dense_kc<NM>() * 16;
}

template <int NM, bool BF = false>  // BF: BF16 operands (v_mfma_f32_16x16x16bf16_1k, 4 steps per instruction)
__device__ __forceinline__ void bwd_dense_mfma_block(const FastBwdArgs<float>& A, int bx, int by, float* alds) {
    typedef float floatx4 __attribute__((ext_vector_type(4)));
    constexpr int NA = NM > 0 ? NM : 1;
    constexpr int KC = bwd_dense_kc<NM>();
    constexpr int U = 8;  // steps of 4 outputs per trip
    static_assert(KC % (4 * U) == 0, "trips must not straddle a staged chunk");
    const LayerGeo& g = A.gn;
    const NeuronLayout& L = g.in;
    const int lane = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.y);
    const int tid = wave * kWave + lane;
    const int S = A.S;
    const int Sa = (int)(L.cols / L.P);
    const int tiles = L.P / kWave;
    const int c = by / tiles;
    const int p0 = (by - c * tiles) * kWave + wave * 16;
    const int s0 = bx * 16;
    const int kq = lane >> 4, cl = lane & 15;
    const int p = p0 + cl;                // C column of this lane
    const int n1 = g.out.C;
    const long F = g.fan;
    const float* vsrc = A.last ? A.cvec : A.vs;
    const float vsign = A.last ? -1.f : 1.f;
    // weights of one trip: output i + 4 u + kq at this lane's position
    const float* wcol = g.W + (long)c * L.P + p;
    float wv[U];
    auto wload = [&](int i) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int ii = i + 4 * u + kq;
            wv[u] = wcol[(long)(ii < n1 ? ii : 0) * F];
        }
    };
    wload(0);
    // this lane's neurons: rows 4 kq + r, column cl
    unsigned hb[4];
    BwdIn<float> in[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int sc = min(s0 + 4 * kq + r, Sa - 1);
        const long idx = ((long)c * S + sc) * L.P + p;
        hb[r] = NM > 0 ? (unsigned)A.xpk[idx] : 0u;
        bwd_load<float>(A, c, (long)sc * L.P + p, true, idx, in[r]);
    }
    floatx4 acc = {0.f, 0.f, 0.f, 0.f};
    floatx4 au[NA];
#pragma unroll
    for (int q = 0; q < NA; ++q) au[q] = floatx4{0.f, 0.f, 0.f, 0.f};
    for (int i = 0; i < n1; i += 4 * U) {
        if (i % KC == 0) {
            // stage outputs [i, i + KC) of every operand
            __syncthreads();  // the previous chunk's reads are done
            constexpr int PER = KC * 16 / (4 * kWave);  // elements per thread and operand
            float v[1 + NM][PER];
#pragma unroll
            for (int r = 0; r <= NM; ++r) {
                const float* src = r == 0 ? vsrc : A.u[r > 0 ? r - 1 : 0];
#pragma unroll
                for (int j = 0; j < PER; ++j) {
                    const int e = tid + j * 4 * kWave;
                    const int ii = i + (e >> 4);
                    v[r][j] = ii < n1 ? src[(long)ii * S + min(s0 + (e & 15), Sa - 1)] : 0.f;
                }
            }
#pragma unroll
            for (int r = 0; r <= NM; ++r)
#pragma unroll
                for (int j = 0; j < PER; ++j) alds[r * KC * 16 + tid + j * 4 * kWave] = v[r][j];
            __syncthreads();
        }
        float w2[U];
#pragma unroll
        for (int u = 0; u < U; ++u) w2[u] = wv[u];
        if (i + 4 * U < n1) wload(i + 4 * U);
        const float* ab = alds + ((i % KC) + kq) * 16 + cl;  // + 64 per step, + 16 KC per operand
        if constexpr (BF) {
            // 4 steps in the slots of one instruction (outputs past n1:
            // zero operands)
#pragma unroll
            for (int u0 = 0; u0 < U; u0 += 4) {
                if (i + 4 * u0 >= n1) break;  // uniform
                const shortx4 wb = bf16x4(&w2[u0]);
                acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(
                    bf16x4(ab[(u0 + 0) * 64], ab[(u0 + 1) * 64], ab[(u0 + 2) * 64], ab[(u0 + 3) * 64]), wb, acc, 0,
                    0, 0);
                const shortx4 wa = bf16_abs(wb);
#pragma unroll
                for (int q = 0; q < NM; ++q) {
                    const float* aq = ab + (1 + q) * KC * 16;
                    au[q] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(
                        bf16x4(aq[(u0 + 0) * 64], aq[(u0 + 1) * 64], aq[(u0 + 2) * 64], aq[(u0 + 3) * 64]), wa,
                        au[q], 0, 0, 0);
                }
            }
        } else {
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (i + 4 * u >= n1) break;  // uniform
                acc = __builtin_amdgcn_mfma_f32_16x16x4f32(ab[u * 64], w2[u], acc, 0, 0, 0);
                const float wa = fabsf(w2[u]);
#pragma unroll
                for (int q = 0; q < NM; ++q)
                    au[q] = __builtin_amdgcn_mfma_f32_16x16x4f32(ab[(1 + q) * KC * 16 + u * 64], wa, au[q], 0, 0, 0);
            }
        }
    }
    uint16_t* xb16 = reinterpret_cast<uint16_t*>(A.nk.xbits);
    uint16_t* zb16 = reinterpret_cast<uint16_t*>(A.zbits);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int s = s0 + 4 * kq + r;
        const bool ok = s < Sa;  // uniform over each group of 16 lanes
        float f = vsign * acc[r];
#pragma unroll
        for (int q = 0; q < NM; ++q) f += 0.5f * flip(au[q][r], (hb[r] >> q) & 1u);
        bool xb = false, zb = false;
        if (ok) {
            if (A.k >= 1) f += in[r].own;
            const long idx = ((long)c * S + s) * L.P + p;
            if (A.fout) A.fout[caller_index((uint32_t)idx, S, L)] = f;
            xb = f >= 0.f || in[r].lo == in[r].hi;
            A.nk.xstar[idx] = xb ? in[r].hi : in[r].lo;
            if (A.k >= 1) zb = in[r].g >= 0.f;
        }
        const unsigned long long mx = __ballot(xb);
        const unsigned long long mz = __ballot(zb);
        if (ok && cl == 0) {
            const long piece = ((long)c * L.colpad + (long)s * L.P + p0) >> 4;
            xb16[piece] = (uint16_t)(mx >> (16 * kq));
            if (A.k >= 1) zb16[piece] = (uint16_t)(mz >> (16 * kq));
        }
    }
}

template <int NM, bool BF>
__global__ void __launch_bounds__(kWave * 4) k_bwd_dense_mfma(FastBwdArgs<float> A) {
    __shared__ float alds[bwd_dense_lds_floats<NM>()];
    bwd_dense_mfma_block<NM, BF>(A, blockIdx.x, blockIdx.y, alds);
}

// The column-mapped dense backward into the last ReLU layer (k_bwd_dense
// with one position per channel, the output layer's objective rows as
// operand) and the matrix-core dense backward into the layer below it
// (k_bwd_dense_mfma) in one launch: the two are independent (each reads the
// operands of its own layer k+1 and writes its own layer k), and the small
// one, first in the grid, runs beside the other instead of on its own.
// Grid (na + mgx mgy): blocks [0, na) are the column kernel's agx x agy grid,
// the rest the matrix-core kernel's mgx x mgy grid (x fastest).  Block
// (64, 4).
template <int NMB, bool BF>
__global__ void __launch_bounds__(kWave * 4) k_bwd_dense_pair(FastBwdArgs<float> Aa, FastBwdArgs<float> Ab, int na,
                                                              int agx, int agy, int mgx) {
    static_assert(KS == 4, "both kernels run 4 waves per block");
    // one LDS buffer for either role: the column kernel's partial sums or
    // the staged operands
    constexpr int kRed = KS * 8 * kWave;
    constexpr int kLds = kRed > bwd_dense_lds_floats<NMB>() ? kRed : bwd_dense_lds_floats<NMB>();
    __shared__ __attribute__((aligned(16))) float smem[kLds];
    const int lin = blockIdx.x;
    if (lin < na) {
        int tile, group;
        xcd_tile_of((unsigned)lin, (unsigned)agx, (unsigned)agy, tile, group);
        bwd_dense_block<float, 0, 8, true>(Aa, tile, group, reinterpret_cast<float (*)[8][kWave]>(smem));
    } else {
        const int l2 = lin - na;
        bwd_dense_mfma_block<NMB, BF>(Ab, l2 % mgx, l2 / mgx, smem);
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
        const int s = col_sub(col, A.nl.P), p = (int)col - s * A.nl.P;
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
static __global__ void __launch_bounds__(256) k_transpose_w(const float* W, float* Wt, int C, int fan, int Cpad) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (long)fan * Cpad) return;
    const int t = (int)(i / Cpad), c = (int)(i - (long)t * Cpad);
    Wt[i] = c < C ? W[(long)c * fan + t] : 0.f;
}

// Dense weights with rows padded to fanpad: Wr[i][j] = W[i][j] for j < fan.
static __global__ void __launch_bounds__(256) k_pad_rows(const float* W, float* Wr, int n_out, int fan, int fanpad) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (long)n_out * fanpad) return;
    const int r = (int)(i / fanpad), j = (int)(i - (long)r * fanpad);
    Wr[i] = j < fan ? W[(long)r * fan + j] : 0.f;
}

}  // namespace asd
