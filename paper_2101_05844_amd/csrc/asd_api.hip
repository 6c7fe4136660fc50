// Host side of libasdual: validation, workspace layout, and the iteration
// driver of Algorithm 1 / Algorithm 3.  Iterations run the kernels of
// asd_fast.h; evaluation at fixed duals, the final bound and the oracle run
// the general kernels of asd_kernels.h.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <new>
#include <string>
#include <type_traits>
#include <vector>

#include "asd_adjoint.h"
#include "asd_plan.h"

using namespace asd;

namespace {

thread_local std::string g_err = "no error";

}  // namespace

asd_status asd::fail(asd_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

namespace {

NeuronLayout make_layout(int C, int H, int W, int S) {
    NeuronLayout nl;
    nl.C = C;
    nl.H = H;
    nl.W = W;
    nl.P = H * W;
    nl.N = (long)C * nl.P;
    nl.cols = (long)S * nl.P;
    nl.colpad = (nl.cols + 63) / 64 * 64;
    nl.words = (long)C * nl.colpad / 32;
    return nl;
}

// ---------------------------------------------------------------------------
// Workspace carving (two passes: measure, then assign).
// ---------------------------------------------------------------------------
constexpr int kMaxKsplit = 8;  // dense forward partial sums per output (the partial-sum buffer's size)

struct Carver {
    char* base;
    size_t off;
    template <typename T>
    T* take(size_t count) {
        off = (off + 255) / 256 * 256;
        T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
        off += count * sizeof(T);
        return p;
    }
};

// Doubles after the gradient's partial sums that hold the input records of
// a ReLU layer's weight gradient and of the FP64 final sums (the largest
// input layer of a ReLU layer), or the output records of the FP64 final
// backward (the largest ReLU layer).
size_t grad_inrec_doubles(const asd_plan* P) {
    const size_t rec = is64(P) ? sizeof(GwIn<double>) : sizeof(GwIn<float>);
    size_t bytes = 0;
    for (int k = 1; k < P->n; ++k) bytes = std::max(bytes, (size_t)P->geo[k].in.C * P->geo[k].in.cols * rec);
    // FP32 plans: also the output records of the FP64 final backward (the
    // neurons of a ReLU layer, at the largest mask count)
    if (!is64(P))
        for (int k = 1; k < P->n; ++k)
            bytes = std::max(bytes, (size_t)P->geo[k].out.C * P->geo[k].out.cols * 16 *
                                        (size_t)bf_rec_units(P->prm.max_masks));
    return (bytes + 15) / 16 * 2 + 2;  // and up to 8 bytes to reach 16-byte alignment
}

// Input records of the weight gradient: after the partial sums, 16-byte aligned.
void* grad_inrec(asd_plan* P) { return P->gpart + ((P->gpart_w + P->gpart_b + 1) & ~(size_t)1); }

template <typename T>
void carve_t(asd_plan* P, Carver& cv) {
    const int S = P->S;
    for (int k = 0; k < P->n; ++k) {
        const NeuronLayout& nl = P->nl[k];
        const size_t ns = (size_t)nl.N * S;
        NeuronArraysT<T>& a = NA<T>(P)[k];
        a.lo = cv.take<T>(ns);
        a.hi = cv.take<T>(ns);
        a.xstar = cv.take<T>(ns);
        a.xbits = cv.take<uint32_t>(nl.words);
        a.deg = cv.take<uint32_t>(nl.words);
        a.term = cv.take<double>(ns);
        a.xpk = k + 1 < P->n ? cv.take<uint16_t>(ns) : nullptr;
    }
    for (int k = 1; k < P->n; ++k) {
        const NeuronLayout& nl = P->nl[k];
        const size_t ns = (size_t)nl.N * S;
        ReluLayerT<T>& r = RL<T>(P)[k];
        memset(&r, 0, sizeof(r));
        r.lhat = cv.take<T>(ns);
        r.uhat = cv.take<T>(ns);
        r.alpha = cv.take<T>(ns);
        r.beta0 = cv.take<T>(ns);
        r.beta1 = cv.take<T>(ns);
        r.alpha_m = cv.take<T>(ns);
        r.alpha_v = cv.take<T>(ns);
        r.beta0_m = cv.take<T>(ns);
        r.beta0_v = cv.take<T>(ns);
        r.beta1_m = cv.take<T>(ns);
        r.beta1_v = cv.take<T>(ns);
        r.own = cv.take<T>(ns);
        r.g = cv.take<T>(ns);
        r.vs = cv.take<T>(ns);
        r.zbits = cv.take<uint32_t>(nl.words);
        r.zpk = cv.take<uint8_t>(ns);
        if (sizeof(T) == 4) {
            r.own64 = cv.take<double>(ns);
            r.g64 = cv.take<double>(ns);
            r.const64 = cv.take<double>(ns);
        }
        for (int q = 0; q < P->prm.max_masks; ++q) {
            MaskSlotT<T>& m = r.slot[q];
            m.beta = cv.take<T>(ns);
            m.m = cv.take<T>(ns);
            m.v = cv.take<T>(ns);
            m.LI = cv.take<T>(ns);
            m.UI = cv.take<T>(ns);
            m.u = cv.take<T>(ns);
            m.zbits = cv.take<uint32_t>(nl.words);
            m.xbits = cv.take<uint32_t>(P->nl[k - 1].words);
        }
    }
    T* cv_arr = cv.take<T>((size_t)P->nl[P->n].N * S);
    if (sizeof(T) == 4) P->cvecf = reinterpret_cast<float*>(cv_arr);
    else P->cvecd = reinterpret_cast<double*>(cv_arr);
    // a convolutional output layer: -c as the operand of the iteration
    // kernels' transposed convolution into the last ReLU layer
    P->negc = (sizeof(T) == 4 && P->geo[P->n].kind == ASD_LAYER_CONV2D) ? cv.take<float>((size_t)P->nl[P->n].N * S)
                                                                        : nullptr;
    P->ball_c = cv.take<float>((size_t)P->nl[0].N * S);
    P->ball_r = cv.take<float>(S);
    P->f0f = sizeof(T) == 4 ? cv.take<float>((size_t)P->nl[0].N * S) : nullptr;
    size_t part = 0;
    for (int L = 1; L <= P->n; ++L) {
        const LayerGeo& g = P->geo[L];
        if (L < P->n) P->Wt[L] = cv.take<float>((size_t)g.fan * P->Cpad[L]);
        if (g.kind == ASD_LAYER_CONV2D)
        {
            P->Wb[L] = cv.take<float>((size_t)((g.in.C + 15) / 16) * g.stride * g.stride * P->nkp[L] * 16);
            const size_t rows = (size_t)g.out.C * g.ksz * g.ksz + 1;
            P->Wl4[L] = cv.take<float>((size_t)((g.in.C + 3) / 4) * rows * 4);
            P->Wl8[L] = cv.take<float>((size_t)((g.in.C + 7) / 8) * rows * 8);
        }
        if (g.kind == ASD_LAYER_DENSE) {
            P->Wr[L] = cv.take<float>((size_t)g.out.C * P->fanpad[L]);
            if (L < P->n)
                part = std::max(part, (size_t)kMaxKsplit * (1 + P->prm.max_masks) * P->Cpad[L] * S);
        }
    }
    P->part = cv.take<T>(part);
    P->pointflag = cv.take<int>(kMaxLayers);
    P->f0 = cv.take<double>((size_t)P->nl[0].N * S);
    P->gpart = cv.take<double>(P->gpart_w + P->gpart_b + grad_inrec_doubles(P));
    P->budgets_dev = cv.take<int>(S);
    P->inflags = cv.take<int32_t>(S);
    P->lrs = cv.take<T>(S);
    P->Rdev = cv.take<ReluLayerT<T>>(kMaxLayers);
}

void carve(asd_plan* P, Carver& cv) {
    if (is64(P)) carve_t<double>(P, cv);
    else carve_t<float>(P, cv);
}

asd_status check_params(const asd_params* p) {
    if (!p) return fail(ASD_EINVAL, "params is NULL");
    if (p->bigm_iters < 0 || p->as_iters < 0) return fail(ASD_EINVAL, "negative iteration count");
    if (p->add_every < 1) return fail(ASD_EINVAL, "add_every must be >= 1");
    if (p->add_count < 0) return fail(ASD_EINVAL, "add_count must be >= 0");
    if (p->max_masks < 0 || p->max_masks > ASD_MAX_MASKS)
        return fail(ASD_EINVAL, "max_masks must be in [0, %d]", ASD_MAX_MASKS);
    if (p->rule != ASD_RULE_ADAM && p->rule != ASD_RULE_SUPERGRADIENT) return fail(ASD_EINVAL, "unknown rule");
    if (p->precision != ASD_PREC_FP32 && p->precision != ASD_PREC_FP64 && p->precision != ASD_PREC_MIXED &&
        p->precision != ASD_PREC_BF16 && p->precision != ASD_PREC_BF16_ALL)
        return fail(ASD_EINVAL, "unknown precision %d", p->precision);
    if (!(p->adam_beta1 >= 0.0 && p->adam_beta1 < 1.0 && p->adam_beta2 >= 0.0 && p->adam_beta2 < 1.0))
        return fail(ASD_EINVAL, "Adam betas must be in [0, 1)");
    if (!(p->adam_eps > 0.0)) return fail(ASD_EINVAL, "Adam eps must be > 0");
    return ASD_OK;
}

void setup_plan_geometry(asd_plan* P) {
    const asd_net* net = P->net;
    const int S = P->S;
    P->gpart_w = P->gpart_b = 0;
    const asd_layer_desc& d0 = net->L[0];
    P->nl[0] = make_layout(d0.in_c, d0.kind == ASD_LAYER_DENSE ? 1 : d0.in_h,
                           d0.kind == ASD_LAYER_DENSE ? 1 : d0.in_w, S);
    for (int L = 1; L <= P->n; ++L) {
        const asd_layer_desc& d = net->L[L - 1];
        LayerGeo& g = P->geo[L];
        g.kind = d.kind;
        g.W = d.W;
        g.b = d.b;
        g.in = P->nl[L - 1];
        if (d.kind == ASD_LAYER_DENSE) {
            P->nl[L] = make_layout(d.out_c, 1, 1, S);
            g.ksz = 1;
            g.stride = 1;
            g.pad = 0;
            g.fan = (int)g.in.N;
        } else {
            P->nl[L] = make_layout(d.out_c, d.out_h, d.out_w, S);
            g.ksz = d.kernel;
            g.stride = d.stride;
            g.pad = d.pad;
            g.fan = d.in_c * d.kernel * d.kernel;
        }
        g.out = P->nl[L];
        P->Cpad[L] = (g.out.C + 31) / 32 * 32;
        {
            const int J = (g.ksz + g.stride - 1) / g.stride;
            P->nkp[L] = (g.out.C * J * J + 3) / 4 * 4;
        }
        P->fanpad[L] = (g.in.C + 7) / 8 * 8 * g.in.P;
        {
            // bound gradient: about 2048 blocks for the weights and 1024 for
            // the biases, at most 64 chunks, at least 16 subproblems (dense)
            // or 2048 terms (convolution, biases) per chunk
            auto split = [](long groups, long terms, long want_blocks, long min_terms, int* chunks, long* rchunk) {
                long c = (want_blocks + groups - 1) / groups;
                c = std::max(1L, std::min(c, std::min(64L, std::max(1L, terms / min_terms))));
                *rchunk = (terms + c - 1) / c;
                *chunks = (int)((terms + *rchunk - 1) / *rchunk);
            };
            const long entries = (long)g.out.C * g.fan;
            if (L == net->n) {
                split((long)((g.fan + kGradThreads - 1) / kGradThreads) * ((g.out.C + kGdTO - 1) / kGdTO), S, 2048,
                      16, &P->gw_chunks[L], &P->gw_rchunk[L]);
            } else {
                // ReLU layer: about 1024 blocks, chunks of whole LDS batches
                int TT, TO;
                gw_config(g.fan, &TT, &TO);
                const long groups = (long)((g.fan + 64 * TT - 1) / (64 * TT)) * ((g.out.C + TO - 1) / TO);
                const long terms = (long)S * g.out.P;
                const long batches = (terms + kGwRB - 1) / kGwRB;
                const long c = std::max(1L, std::min((1024 + groups - 1) / groups, std::min(512L, batches)));
                P->gw_rchunk[L] = (batches + c - 1) / c * kGwRB;
                P->gw_chunks[L] = (int)((terms + P->gw_rchunk[L] - 1) / P->gw_rchunk[L]);
            }
            split(g.out.C, (long)S * g.out.P, 1024, 2048, &P->gb_chunks[L], &P->gb_rchunk[L]);
            P->gpart_w = std::max(P->gpart_w, (size_t)P->gw_chunks[L] * entries);
            P->gpart_b = std::max(P->gpart_b, (size_t)P->gb_chunks[L] * g.out.C);
        }
        P->ksplit[L] = 1;
        P->fwd_mfma[L] = d.kind == ASD_LAYER_CONV2D && d.out_c >= 32;
        P->bwd_cb[L - 1] = 0;
        P->bwd_pos[L - 1] = 2;
        P->bwd_nt[L - 1] = 0;
        P->fwd_kw[L] = 8;
        P->bwd_kw[L - 1] = 8;
        if (d.kind == ASD_LAYER_DENSE) {
            // about two waves per SIMD (2048 waves of KS per 32 x 32 tile), at
            // least 32 taps per wave, at most 8 partial sums per output
            const long tiles = (long)((S + 31) / 32) * (P->Cpad[L] / 32);
            const long want = (2048 / KS + tiles - 1) / tiles;
            const long cap = std::max(1L, std::min(8L, (long)(g.fan / (32 * KS))));
            P->ksplit[L] = (int)std::max(1L, std::min(std::min(want, cap), (long)kMaxKsplit));
        }
    }
}


asd_status zero_words(void* p, long n, hipStream_t st) {
    if (n == 0) return ASD_OK;
    hipLaunchKernelGGL(k_zero_words, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st,
                       reinterpret_cast<uint32_t*>(p), n);
    LAUNCH_CHECK();
    return ASD_OK;
}

template <typename T>
asd_status zero_arr(T* p, size_t n, hipStream_t st) {
    return zero_words(p, (long)(n * sizeof(T) / 4), st);
}

asd_status copy_words(uint32_t* dst, const uint32_t* src, long n, hipStream_t st) {
    hipLaunchKernelGGL(k_copy_words, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, dst, src, n);
    LAUNCH_CHECK();
    return ASD_OK;
}

template <typename Ti, typename Te>
asd_status launch_layout(Ti* in_arr, Te* ex_arr, const NeuronLayout& nl, int S, int mode, hipStream_t st) {
    dim3 grid((unsigned)((nl.cols + 255) / 256), (unsigned)nl.C);
    hipLaunchKernelGGL((k_layout<Ti, Te>), grid, dim3(256), 0, st, in_arr, ex_arr, nl, S, mode);
    LAUNCH_CHECK();
    return ASD_OK;
}

template <typename T, typename Te>
asd_status launch_bits(const NeuronLayout& nl, int S, int mode, uint32_t* bits, Te* fext, const T* lo,
                       const T* hi, hipStream_t st) {
    BitArgs<T, Te> a;
    a.nl = nl;
    a.S = S;
    a.mode = mode;
    a.bits = bits;
    a.fext = fext;
    a.lo = lo;
    a.hi = hi;
    dim3 grid((unsigned)(nl.colpad / 256 + 1), (unsigned)nl.C);
    hipLaunchKernelGGL((k_bits<T, Te>), grid, dim3(256), 0, st, a);
    LAUNCH_CHECK();
    return ASD_OK;
}

template <typename T>
asd_status derive_layer(asd_plan* P, int k, hipStream_t st) {
    DeriveArgs<T> a;
    a.nl = P->nl[k];
    a.S = P->S;
    a.nm = P->n_masks;
    a.b = P->geo[k].b;
    a.R = RL<T>(P)[k];
    dim3 grid((unsigned)((a.nl.cols + 255) / 256), (unsigned)a.nl.C);
    hipLaunchKernelGGL(k_derive<T>, grid, dim3(256), 0, st, a);
    LAUNCH_CHECK();
    return ASD_OK;
}

// Packed x words of layer k (for the slots of ReLU layer k+1) and, with
// with_flag, the flag of point boxes away from zero.
template <typename T>
asd_status pack_layer_x(asd_plan* P, int k, int with_flag, hipStream_t st) {
    PackArgs<T> a;
    memset(&a, 0, sizeof(a));
    a.nl = P->nl[k];
    a.S = P->S;
    a.nm = P->n_masks;
    const ReluLayerT<T>& rn = RL<T>(P)[k + 1];
    for (int q = 0; q < a.nm; ++q) a.bits[q] = rn.slot[q].xbits;
    a.deg = NA<T>(P)[k].deg;
    a.lo = NA<T>(P)[k].lo;
    a.xpk = NA<T>(P)[k].xpk;
    a.pointflag = with_flag ? P->pointflag + k : nullptr;
    dim3 grid((unsigned)((a.nl.cols + 255) / 256), (unsigned)a.nl.C);
    hipLaunchKernelGGL(k_pack<T>, grid, dim3(256), 0, st, a);
    LAUNCH_CHECK();
    return ASD_OK;
}

// Packed z bytes of ReLU layer k.
template <typename T>
asd_status pack_layer_z(asd_plan* P, int k, hipStream_t st) {
    PackArgs<T> a;
    memset(&a, 0, sizeof(a));
    a.nl = P->nl[k];
    a.S = P->S;
    a.nm = P->n_masks;
    const ReluLayerT<T>& r = RL<T>(P)[k];
    for (int q = 0; q < a.nm; ++q) a.bits[q] = r.slot[q].zbits;
    a.zpk = r.zpk;
    dim3 grid((unsigned)((a.nl.cols + 255) / 256), (unsigned)a.nl.C);
    hipLaunchKernelGGL(k_pack<T>, grid, dim3(256), 0, st, a);
    LAUNCH_CHECK();
    return ASD_OK;
}

template <typename T>
asd_status pack_all(asd_plan* P, int with_flag, hipStream_t st) {
    for (int k = 0; k + 1 < P->n; ++k) TRY(pack_layer_x<T>(P, k, with_flag, st));
    for (int k = 1; k < P->n; ++k) TRY(pack_layer_z<T>(P, k, st));
    return ASD_OK;
}

// Weight copies of the iteration kernels (transposed forward weights, padded
// dense rows).
asd_status prepare_weights(asd_plan* P, hipStream_t st) {
    for (int L = 1; L <= P->n; ++L) {
        const LayerGeo& g = P->geo[L];
        if (L < P->n) {
            const long n = (long)g.fan * P->Cpad[L];
            hipLaunchKernelGGL(k_transpose_w, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, g.W, P->Wt[L],
                               g.out.C, g.fan, P->Cpad[L]);
            LAUNCH_CHECK();
        }
        if (g.kind == ASD_LAYER_CONV2D) {
            const long n = (long)((g.in.C + 15) / 16) * g.stride * g.stride * P->nkp[L] * 16;
            hipLaunchKernelGGL(k_class_weights, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, g.W, P->Wb[L],
                               g.in.C, g.out.C, g.ksz, g.stride, P->nkp[L], n);
            LAUNCH_CHECK();
            for (int cb = 4; cb <= 8; cb += 4) {
                const long rows = (long)g.out.C * g.ksz * g.ksz + 1;
                const long nl = (long)((g.in.C + cb - 1) / cb) * rows * cb;
                hipLaunchKernelGGL(k_col_weights, dim3((unsigned)((nl + 255) / 256)), dim3(256), 0, st, g.W,
                                   cb == 4 ? P->Wl4[L] : P->Wl8[L], g.in.C, g.out.C, g.ksz * g.ksz, cb, nl);
                LAUNCH_CHECK();
            }
        }
        if (g.kind == ASD_LAYER_DENSE) {
            const long n = (long)g.out.C * P->fanpad[L];
            hipLaunchKernelGGL(k_pad_rows, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, g.W, P->Wr[L],
                               g.out.C, g.fan, P->fanpad[L]);
            LAUNCH_CHECK();
        }
    }
    return ASD_OK;
}

asd_status fwd_fast(asd_plan* P, int k, const StepArgsT<float>& sa, hipStream_t st) {
    const bool mb = bf16_moments(P);
#define ASD_FWD_CALL(N) return fwd_fast_nm<N>(P, k, sa, mb, st)
    ASD_NM_DISPATCH(P->n_masks, ASD_FWD_CALL)
#undef ASD_FWD_CALL
}

asd_status fwd_trio(asd_plan* P, int kv, int kc, int kd, const StepArgsT<float>& sa, hipStream_t st) {
    const bool mb = bf16_moments(P);
#define ASD_TRIO_CALL(N) return fwd_trio_nm<N>(P, kv, kc, kd, sa, mb, st)
    ASD_NM_DISPATCH(P->n_masks, ASD_TRIO_CALL)
#undef ASD_TRIO_CALL
}

asd_status fwd_fused(asd_plan* P, int kc, int kd, const StepArgsT<float>& sa, hipStream_t st) {
    const bool mb = bf16_moments(P);
#define ASD_FUSED_CALL(N) return fwd_fused_nm<N>(P, kc, kd, sa, mb, st)
    ASD_NM_DISPATCH(P->n_masks, ASD_FUSED_CALL)
#undef ASD_FUSED_CALL
}

template <typename Tc, typename Ts>
asd_status launch_backward(asd_plan* P, int k, int want_obj, int role, hipStream_t st, double* fout = nullptr,
                           void* fext = nullptr);


// The backward passes into the last ReLU layer (dense, one position per
// channel: k_bwd_dense) and into the layer below (dense into 64-position
// channels on the matrix cores: k_bwd_dense_mfma) can share a launch
// (k_bwd_dense_pair); returns that lower layer, or -1.
int bwd_pair_layer(const asd_plan* P) {
    const int ka = P->n - 1, kb = P->n - 2;
    if (kb < 0 || P->prof == ASD_PROFILE_KERNELS) return -1;
    const LayerGeo& ga = P->geo[ka + 1];
    const LayerGeo& gb = P->geo[kb + 1];
    if (ga.kind != ASD_LAYER_DENSE || ga.in.P != 1) return -1;
    if (gb.kind != ASD_LAYER_DENSE || gb.in.P % kWave != 0 || P->bwd_pos[kb] != 2) return -1;
    return kb;
}

asd_status bwd_pair(asd_plan* P, hipStream_t st) {
#define ASD_PAIR_CALL(N) return bwd_pair_nm<N>(P, st)
    ASD_NM_DISPATCH(P->n_masks, ASD_PAIR_CALL)
#undef ASD_PAIR_CALL
}

asd_status bwd_fast(asd_plan* P, int k, hipStream_t st) {
    const int nm = (k + 1 == P->n) ? 0 : P->n_masks;
#define ASD_BWD_CALL(N) return bwd_fast_nm<N>(P, k, st)
    ASD_NM_DISPATCH(nm, ASD_BWD_CALL)
#undef ASD_BWD_CALL
}


// The l2-ball input domain's x*_0 (and, with term, the final bound's
// objective terms of layer 0) from f_0 of the backward pass just run.
template <typename Ts, typename Tf>
asd_status l2_input(asd_plan* P, const Tf* f0, int f_internal, double* term, hipStream_t st) {
    hipLaunchKernelGGL((k_l2_input<Ts, Tf>), dim3((unsigned)P->Sa), dim3(256), 0, st, f0, f_internal,
                       (const float*)P->ball_c, (const float*)P->ball_r, NA<Ts>(P)[0].xstar, term, P->nl[0], P->S);
    LAUNCH_CHECK();
    return ASD_OK;
}

// Backward pass for neuron layer k (f_k, inner minimisation, terms).
template <typename Tc, typename Ts>
asd_status launch_backward(asd_plan* P, int k, int want_obj, int role, hipStream_t st, double* fout, void* fext) {
    BwdArgs<Ts> a;
    memset(&a, 0, sizeof(a));
    a.gn = gview(P, k + 1);
    a.S = P->S;
    a.k = k;
    a.last = (k + 1 == P->n);
    a.nm_next = a.last ? 0 : P->n_masks;
    a.nm_own = k >= 1 ? P->n_masks : 0;
    a.cvec = CV<Ts>(P);
    if (!a.last) a.Rn = RL<Ts>(P)[k + 1];
    if (k >= 1) {
        a.Rk = RL<Ts>(P)[k];
        a.bk = P->geo[k].b;
    }
    a.nk = NA<Ts>(P)[k];
    a.want_obj = want_obj;
    a.fout = fout;
    a.fext = reinterpret_cast<Ts*>(fext);
    ProfScope ps(P, st, role, k);
    if constexpr (sizeof(Tc) > sizeof(Ts)) {
        // FP64 final bound of an FP32 plan: the sign-class kernel
#define ASD_BF_CALL(N) return backward_final_nm<N>(a, grad_inrec(P), st)
        ASD_NM_DISPATCH(a.nm_next, ASD_BF_CALL)
#undef ASD_BF_CALL
    } else {
        const size_t lds = (size_t)KS * CB * kWave * sizeof(Tc);
        hipLaunchKernelGGL((k_backward<Tc, Ts>), grid_cols(a.gn.in, CB), dim3(kWave, KS), lds, st, a);
        LAUNCH_CHECK();
        return ASD_OK;
    }
}

template <typename T>
asd_status launch_forward(asd_plan* P, int k, const StepArgsT<T>& sa, int mode, void* const* gout,
                          hipStream_t st) {
    FwdArgs<T> a;
    memset(&a, 0, sizeof(a));
    a.g = gview(P, k);
    a.S = P->S;
    a.nm = P->n_masks;
    a.xin = NA<T>(P)[k - 1].xstar;
    a.deg_in = NA<T>(P)[k - 1].deg;
    a.xout = NA<T>(P)[k].xstar;
    a.zbits = RL<T>(P)[k].zbits;
    a.R = RL<T>(P)[k];
    a.st = sa;
    a.mode = mode;
    a.freeze = P->domain == ASD_DOMAIN_L2 && k == 1;
    if (gout)
        for (int i = 0; i < 3 + kMaxMasks; ++i) a.gout[i] = reinterpret_cast<T*>(gout[i]);
    const size_t lds = (size_t)KS * CB * (1 + a.nm) * kWave * sizeof(T);
    ProfScope ps(P, st, mode == 0 ? ASD_K_FORWARD : ASD_K_OTHER, k);
    hipLaunchKernelGGL(k_forward<T>, grid_cols(a.g.out, CB), dim3(kWave, KS), lds, st, a);
    LAUNCH_CHECK();
    return ASD_OK;
}

// Mask constants of slot q of layer k from the given bit sources.
// k_mask_consts may read 4 taps at a time: a dense layer over channels of
// 4k positions whose fan-in splits over nw waves into multiples of 4.
bool mask_dv(const LayerGeo& g, int nw) {
    return g.kind == ASD_LAYER_DENSE && g.in.P % 4 == 0 && g.fan % (4 * nw) == 0;
}

template <typename T>
asd_status launch_mask_consts(asd_plan* P, int k, int q, const uint32_t* zsrc, const uint32_t* xsrc,
                              int zero_state, hipStream_t st) {
    MaskArgs<T> a;
    memset(&a, 0, sizeof(a));
    a.g = P->geo[k];
    a.S = P->S;
    a.q = q;
    a.nm = 1;
    a.lo_in = NA<T>(P)[k - 1].lo;
    a.hi_in = NA<T>(P)[k - 1].hi;
    a.zsrc = zsrc;
    a.xsrc = xsrc;
    a.zero_state = zero_state;
    a.deg_in = NA<T>(P)[k - 1].deg;
    a.R = RL<T>(P)[k];
    ProfScope ps(P, st, ASD_K_MASK, k);
    if (sizeof(T) == 4 && a.g.fan >= 1024) {
        // wide fan-in (few columns, long tap loops): 16 waves split it (FP64
        // plans keep the 4 partial sums of their tested arithmetic order)
        const size_t lds = (size_t)16 * CB * 2 * kWave * sizeof(T);
        if (mask_dv(a.g, 16))
            hipLaunchKernelGGL((k_mask_consts<T, T, 16, true>), grid_cols(P->nl[k], CB), dim3(kWave, 16), lds, st, a);
        else
            hipLaunchKernelGGL((k_mask_consts<T, T, 16, false>), grid_cols(P->nl[k], CB), dim3(kWave, 16), lds, st, a);
    } else {
        const size_t lds = (size_t)KS * CB * 2 * kWave * sizeof(T);
        if (mask_dv(a.g, KS))
            hipLaunchKernelGGL((k_mask_consts<T, T, KS, true>), grid_cols(P->nl[k], CB), dim3(kWave, KS), lds, st, a);
        else
            hipLaunchKernelGGL((k_mask_consts<T, T, KS, false>), grid_cols(P->nl[k], CB), dim3(kWave, KS), lds, st, a);
    }
    LAUNCH_CHECK();
    return ASD_OK;
}

asd_status launch_final_sums(asd_plan* P, int k, hipStream_t st) {
    ProfScope ps(P, st, ASD_K_FINAL, k);
#define ASD_FS_CALL(N) return final_sums_nm<N>(P, k, grad_inrec(P), st)
    ASD_NM_DISPATCH(P->n_masks, ASD_FS_CALL)
#undef ASD_FS_CALL
}

template <typename T>
asd_status reduce_objective(asd_plan* P, double* out, hipStream_t st) {
    ReduceArgs<T> a;
    memset(&a, 0, sizeof(a));
    a.S = P->S;
    a.nlayers = P->n;
    for (int k = 0; k < P->n; ++k) {
        a.nl[k] = P->nl[k];
        a.term[k] = NA<T>(P)[k].term;
    }
    // b_n^T c_s from the internal copy of c (layout of layer n)
    a.cint = CV<T>(P);
    a.bn = P->geo[P->n].b;
    a.c_last = P->nl[P->n].C;
    a.p_last = P->nl[P->n].P;
    a.out = out;
    hipLaunchKernelGGL(k_reduce_obj<T>, dim3((unsigned)P->S), dim3(256), 0, st, a);
    LAUNCH_CHECK();
    return ASD_OK;
}

double linear_lr(double lr0, double lr1, int t, int T) {
    if (T <= 1) return lr0;
    return lr0 + (lr1 - lr0) * (double)t / (double)(T - 1);
}

template <typename T>
StepArgsT<T> make_step_args(const asd_plan* P, double lr) {
    StepArgsT<T> sa;
    memset(&sa, 0, sizeof(sa));
    sa.rule = P->prm.rule;
    sa.lr = (T)lr;
    sa.b1 = (T)P->prm.adam_beta1;
    sa.b2 = (T)P->prm.adam_beta2;
    sa.eps = (T)P->prm.adam_eps;
    auto bc = [&](int step, T* c1, T* c2) {
        const int s = step > 0 ? step : 1;
        *c1 = (T)(1.0 - pow(P->prm.adam_beta1, (double)s));
        *c2 = (T)(1.0 - pow(P->prm.adam_beta2, (double)s));
    };
    bc(P->step, &sa.bc1[0], &sa.bc2[0]);
    for (int q = 0; q < kMaxMasks; ++q) bc(q < P->n_masks ? P->mask_step[q] : 1, &sa.bc1[1 + q], &sa.bc2[1 + q]);
    for (int g = 0; g < 1 + kMaxMasks; ++g) {
        const int stp = g == 0 ? P->step : (g - 1 < P->n_masks ? P->mask_step[g - 1] : 1);
        const int s1 = stp > 0 ? stp : 1;
        sa.c1[g] = (T)(lr / (1.0 - pow(P->prm.adam_beta1, (double)s1)));
        sa.ib2[g] = (T)(1.0 / (1.0 - pow(P->prm.adam_beta2, (double)s1)));
    }
    return sa;
}

template <typename T>
asd_status reset_group_moments(asd_plan* P, hipStream_t st) {
    for (int k = 1; k < P->n; ++k) {
        const size_t ns = (size_t)P->nl[k].N * P->S;
        ReluLayerT<T>& r = RL<T>(P)[k];
        T* arrs[6] = {r.alpha_m, r.alpha_v, r.beta0_m, r.beta0_v, r.beta1_m, r.beta1_v};
        for (T* a : arrs) TRY(zero_arr(a, ns, st));
    }
    P->step = 0;
    return ASD_OK;
}

// One iteration: backward pass, optional active-set extension, forward pass.
// FP32 plans run the (1 + K) kernels of asd_fast.h.  FP64 plans run the
// general kernels, whose masked products add the same terms as the mask
// constants (term by term, same order), so a supergradient entry that is
// exactly zero in exact arithmetic (for instance a fresh mask's row at the
// point it was added from, x = 0) is exactly zero here as in the FP64
// reference, and primal ties are broken the same way; the (1 + K) form
// reaches such entries through a cancellation that leaves a rounding residue.
// FP32-duals plans: one convolutional layer on the matrix cores and one
// dense layer (8 waves per tile and per split) share the forward launch,
// unless kernels are being timed one by one, and one VALU-mapped
// convolutional layer joins them where there is one.  -1 where there is no
// such layer.
void shared_forward_layers(const asd_plan* P, int& fc, int& fd, int& fv) {
    fc = fd = fv = -1;
    for (int k = 1; k < P->n && P->prof != ASD_PROFILE_KERNELS; ++k) {
        const LayerGeo& g = P->geo[k];
        if (fc < 0 && g.kind == ASD_LAYER_CONV2D && P->fwd_mfma[k] && P->fwd_kw[k] == 8) fc = k;
        if (fv < 0 && g.kind == ASD_LAYER_CONV2D && !P->fwd_mfma[k]) fv = k;
        if (fd < 0 && g.kind == ASD_LAYER_DENSE && P->fwd_kw[k] == 8) fd = k;
    }
    if (fc < 0 || fd < 0) fc = fd = fv = -1;
}

// The forward pass of an FP32-duals iteration (every ReLU layer's update).
template <typename T>
asd_status forward_pass(asd_plan* P, const StepArgsT<T>& sa, hipStream_t st) {
    int fc, fd, fv;
    shared_forward_layers(P, fc, fd, fv);
    for (int k = 1; k < P->n; ++k) {
        if (k == fc || k == fv) continue;
        if (k == fd) TRY(fv >= 0 ? fwd_trio(P, fv, fc, fd, sa, st) : fwd_fused(P, fc, fd, sa, st));
        else TRY(fwd_fast(P, k, sa, st));
    }
    return ASD_OK;
}

template <typename T>
asd_status iteration(asd_plan* P, bool as_phase, int t, double lr, hipStream_t st) {
    constexpr bool kGeneral = sizeof(T) == 8;
    // per-subproblem budgets: the subproblems whose budget exceeds t (a
    // prefix, budgets being non-increasing) are updated, each with the
    // learning rate of its own schedule
    const bool rag = as_phase && P->ragged;
    if (rag) {
        int sa = 0;
        while (sa < P->S && P->budgets[sa] > t) ++sa;
        P->Sa = sa;
        hipLaunchKernelGGL(k_lr_schedule<T>, dim3((unsigned)((sa + 255) / 256)), dim3(256), 0, st,
                           (const int*)P->budgets_dev, sa, t, P->prm.as_lr0, P->prm.as_lr1,
                           reinterpret_cast<T*>(P->lrs));
        LAUNCH_CHECK();
    }
    struct RestoreSa {
        asd_plan* P;
        ~RestoreSa() { P->Sa = P->S; }
    } restore{P};
    // FP32 plans: the backward launches into the last two layers can share
    // one (unless kernels are being timed one by one)
    int kpair = -1;
    if constexpr (!kGeneral) kpair = bwd_pair_layer(P);
    const bool l2 = P->domain == ASD_DOMAIN_L2;
    for (int k = P->n - 1; k >= 0; --k) {
        if constexpr (kGeneral) {
            TRY((launch_backward<T, T>(P, k, 0, ASD_K_BACKWARD, st, k == 0 && l2 ? P->f0 : nullptr)));
        } else {
            if (k == kpair) continue;
            if (kpair >= 0 && k == P->n - 1) TRY(bwd_pair(P, st));
            else TRY(bwd_fast(P, k, st));
        }
    }
    if (l2) {
        if constexpr (kGeneral) TRY((l2_input<T, double>(P, P->f0, 1, nullptr, st)));
        else TRY((l2_input<T, float>(P, P->f0f, 0, nullptr, st)));
    }
    if (as_phase && P->n >= 2 && (t % P->prm.add_every) < P->prm.add_count &&
        P->n_masks < P->prm.max_masks) {
        const int q = P->n_masks;
        for (int k = 1; k < P->n; ++k) {
            ReluLayerT<T>& r = RL<T>(P)[k];
            TRY(copy_words(r.slot[q].zbits, r.zbits, P->nl[k].words, st));
            TRY(copy_words(r.slot[q].xbits, NA<T>(P)[k - 1].xbits, P->nl[k - 1].words, st));
            TRY(launch_mask_consts<T>(P, k, q, r.zbits, NA<T>(P)[k - 1].xbits, 1, st));
        }
        P->mask_step[q] = 0;
        P->n_masks = q + 1;
        TRY(pack_all<T>(P, 0, st));
    }
    if (P->prm.rule == ASD_RULE_ADAM) {
        P->step += 1;
        for (int q = 0; q < P->n_masks; ++q) P->mask_step[q] += 1;
    }
    StepArgsT<T> sa = make_step_args<T>(P, lr);
    if (rag) {
        sa.lrs = reinterpret_cast<const T*>(P->lrs);
        for (int g = 0; g < 1 + kMaxMasks; ++g) {
            const int stp = g == 0 ? P->step : (g - 1 < P->n_masks ? P->mask_step[g - 1] : 1);
            sa.ib1[g] = (T)(1.0 / (1.0 - pow(P->prm.adam_beta1, (double)(stp > 0 ? stp : 1))));
        }
    }
    if constexpr (kGeneral) {
        for (int k = 1; k < P->n; ++k) TRY(launch_forward<T>(P, k, sa, 0, nullptr, st));
        return ASD_OK;
    } else {
        return forward_pass<T>(P, sa, st);
    }
}

// Bit 2 of the plan's input flags for every subproblem whose box, bounds
// or objective row hold a non-finite value or an empty interval.
asd_status check_inputs(asd_plan* P, const asd_batch* b, hipStream_t st) {
    const int S = P->S;
    TRY(zero_words(P->inflags, S, st));
    auto launch = [&](const float* lo, const float* hi, long n) -> asd_status {
        const long tot = n * S;
        hipLaunchKernelGGL(k_flags_inputs, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, lo, hi, n, S,
                           P->inflags);
        LAUNCH_CHECK();
        return ASD_OK;
    };
    TRY(launch(b->l0, b->u0, P->nl[0].N));
    for (int k = 1; k < P->n; ++k) TRY(launch(b->lhat[k - 1], b->uhat[k - 1], P->nl[k].N));
    return launch(b->c, nullptr, P->nl[P->n].N);
}

template <typename T>
asd_status init_t(asd_plan* P, const asd_batch* b, hipStream_t st) {
    const int S = P->S;
    NeuronArraysT<T>* na = NA<T>(P);
    TRY(check_inputs(P, b, st));
    TRY((launch_layout<T, const float>(na[0].lo, b->l0, P->nl[0], S, 0, st)));
    TRY((launch_layout<T, const float>(na[0].hi, b->u0, P->nl[0], S, 0, st)));
    for (int k = 1; k < P->n; ++k) {
        ReluLayerT<T>& r = RL<T>(P)[k];
        TRY((launch_layout<T, const float>(r.lhat, b->lhat[k - 1], P->nl[k], S, 0, st)));
        TRY((launch_layout<T, const float>(r.uhat, b->uhat[k - 1], P->nl[k], S, 0, st)));
        TRY((launch_layout<T, const float>(na[k].lo, b->lhat[k - 1], P->nl[k], S, 1, st)));
        TRY((launch_layout<T, const float>(na[k].hi, b->uhat[k - 1], P->nl[k], S, 1, st)));
    }
    for (int k = 0; k < P->n; ++k)
        TRY((launch_bits<T, T>(P->nl[k], S, 3, na[k].deg, nullptr, na[k].lo, na[k].hi, st)));
    TRY((launch_layout<T, const float>(CV<T>(P), b->c, P->nl[P->n], S, 0, st)));
    if (P->negc) {
        const long n = (long)P->nl[P->n].N * S;
        hipLaunchKernelGGL(k_negate, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, P->negc,
                           reinterpret_cast<const float*>(CV<T>(P)), n);
        LAUNCH_CHECK();
    }
    for (int k = 1; k < P->n; ++k) {
        const size_t ns = (size_t)P->nl[k].N * S;
        ReluLayerT<T>& r = RL<T>(P)[k];
        T* arrs[12] = {r.alpha, r.beta0, r.beta1, r.alpha_m, r.alpha_v, r.beta0_m,
                       r.beta0_v, r.beta1_m, r.beta1_v, r.own, r.g, r.vs};
        for (T* a : arrs) TRY(zero_arr(a, ns, st));
        for (int q = 0; q < P->prm.max_masks; ++q) {
            MaskSlotT<T>& m = r.slot[q];
            T* sarr[6] = {m.beta, m.m, m.v, m.LI, m.UI, m.u};
            for (T* a : sarr) TRY(zero_arr(a, ns, st));
            TRY(zero_words(m.zbits, P->nl[k].words, st));
            TRY(zero_words(m.xbits, P->nl[k - 1].words, st));
        }
    }
    TRY(prepare_weights(P, st));
    TRY(zero_words(P->pointflag, kMaxLayers, st));
    // the update kernels read the layer arrays from a device copy, written by
    // a kernel that takes each table as its argument (stream-ordered, and no
    // host memory is read after the launch)
    for (int k = 1; k < P->n; ++k) {
        hipLaunchKernelGGL(k_store_layer<T>, dim3(1), dim3(1), 0, st, RdevT<T>(P) + k, RL<T>(P)[k]);
        LAUNCH_CHECK();
    }
    return pack_all<T>(P, 1, st);
}

template <typename T>
asd_status run_t(asd_plan* P, bool as, int t_begin, int n_iters, int T_, hipStream_t st) {
    if (as && t_begin == 0 && n_iters > 0 && P->prm.rule == ASD_RULE_ADAM) TRY(reset_group_moments<T>(P, st));
    for (int t = t_begin; t < t_begin + n_iters; ++t) {
        const double lr = as ? linear_lr(P->prm.as_lr0, P->prm.as_lr1, t, T_)
                             : linear_lr(P->prm.bigm_lr0, P->prm.bigm_lr1, t, T_);
        TRY(iteration<T>(P, as, t, lr, st));
    }
    return ASD_OK;
}

asd_status bound_f32(asd_plan* P, double* out_lb, float* x0, hipStream_t st) {
    P->min_valid = false;
    for (int k = 1; k < P->n; ++k) TRY(launch_final_sums(P, k, st));
    for (int k = P->n - 1; k >= 0; --k)
        TRY((launch_backward<double, float>(P, k, 1, ASD_K_FINAL, st, k == 0 ? P->f0 : nullptr)));
    if (P->domain == ASD_DOMAIN_L2) TRY((l2_input<float, double>(P, P->f0, 1, P->naf[0].term, st)));
    TRY(reduce_objective<float>(P, out_lb, st));
    if (x0) TRY((launch_layout<float, float>(P->naf[0].xstar, x0, P->nl[0], P->S, 2, st)));
    P->min_valid = true;
    return ASD_OK;
}

asd_status bound_f64(asd_plan* P, double* out_lb, float* x0, hipStream_t st) {
    P->min_valid = false;
    for (int k = P->n - 1; k >= 0; --k)
        TRY((launch_backward<double, double>(P, k, 1, ASD_K_FINAL, st, k == 0 ? P->f0 : nullptr)));
    if (P->domain == ASD_DOMAIN_L2) TRY((l2_input<double, double>(P, P->f0, 1, P->nad[0].term, st)));
    TRY(reduce_objective<double>(P, out_lb, st));
    if (x0) TRY((launch_layout<double, float>(P->nad[0].xstar, x0, P->nl[0], P->S, 2, st)));
    P->min_valid = true;
    return ASD_OK;
}

// Gradient of sum_s g_s d_B(s) at the current duals and active sets.  The
// minimiser is recomputed exactly as asd_bound evaluates it (FP64 sums; for an
// FP32 plan from the FP32 duals), then each gradient is a fixed-order FP64
// reduction over the subproblems.
template <typename Ts>
asd_status bound_grad_t(asd_plan* P, const double* gs, double* const* dW, double* const* db, double* dl0,
                        double* du0, int reuse, hipStream_t st) {
    if (!(reuse && P->min_valid)) {
        P->min_valid = false;
        if constexpr (sizeof(Ts) == 4)
            for (int k = 1; k < P->n; ++k) TRY(launch_final_sums(P, k, st));
        for (int k = P->n - 1; k >= 0; --k)
            TRY((launch_backward<double, Ts>(P, k, 0, ASD_K_FINAL, st, k == 0 ? P->f0 : nullptr)));
        P->min_valid = true;
    }
    auto base_args = [&](int k) {
        GradArgs<Ts> a;
        memset(&a, 0, sizeof(a));
        a.g = P->geo[k];
        a.S = P->S;
        a.last = (k == P->n);
        a.nm = a.last ? 0 : P->n_masks;
        a.gs = gs;
        a.xin = NA<Ts>(P)[k - 1].xstar;
        a.lo_in = NA<Ts>(P)[k - 1].lo;
        a.hi_in = NA<Ts>(P)[k - 1].hi;
        a.deg_in = NA<Ts>(P)[k - 1].deg;
        a.cvec = CV<Ts>(P);
        a.R = a.last ? nullptr : RdevT<Ts>(P) + k;
        return a;
    };
    for (int k = 1; k <= P->n; ++k) {
        const LayerGeo& g = P->geo[k];
        if (dW && dW[k - 1]) {
            GradArgs<Ts> a = base_args(k);
            a.r_chunk = P->gw_rchunk[k];
            a.entries = (long)g.out.C * g.fan;
            a.part = P->gpart;
            {
                ProfScope ps(P, st, ASD_K_GRAD_WEIGHT, k);
                if (a.last) {
                    hipLaunchKernelGGL(k_gw_last<Ts>,
                                       dim3((unsigned)((g.fan + kGradThreads - 1) / kGradThreads),
                                            (unsigned)((g.out.C + kGdTO - 1) / kGdTO), (unsigned)P->gw_chunks[k]),
                                       dim3(kGradThreads), 0, st, a);
                    LAUNCH_CHECK();
                } else {
                    // input records of layer k-1, after the partial sums
                    GwIn<Ts>* rec = static_cast<GwIn<Ts>*>(grad_inrec(P));
                    const long nin = (long)g.in.C * g.in.cols;
                    hipLaunchKernelGGL(k_gw_in<Ts>, dim3((unsigned)((nin + kGradThreads - 1) / kGradThreads)),
                                       dim3(kGradThreads), 0, st, a, rec);
                    LAUNCH_CHECK();
#define ASD_GW_CALL(N)                                  \
    TRY(grad_weight_nm<N>(P, k, gs, rec, st)); \
    break;
                    ASD_NM_DISPATCH(a.nm, ASD_GW_CALL)
#undef ASD_GW_CALL
                }
                hipLaunchKernelGGL(k_gsum, dim3((unsigned)((a.entries + 63) / 64)), dim3(64, kGsumW), 0, st,
                                   (const double*)P->gpart, a.entries, P->gw_chunks[k], dW[k - 1]);
                LAUNCH_CHECK();
            }
        }
        if (db && db[k - 1]) {
            GradArgs<Ts> a = base_args(k);
            a.r_chunk = P->gb_rchunk[k];
            a.entries = g.out.C;
            a.part = P->gpart + P->gpart_w;
            ProfScope ps(P, st, ASD_K_GRAD_BIAS, k);
            hipLaunchKernelGGL(k_gb_part<Ts>, dim3((unsigned)P->gb_chunks[k], (unsigned)g.out.C), dim3(kGradThreads), 0,
                               st, a);
            LAUNCH_CHECK();
            hipLaunchKernelGGL(k_gsum, dim3((unsigned)((g.out.C + 63) / 64)), dim3(64, kGsumW), 0, st,
                               (const double*)a.part, (long)g.out.C, P->gb_chunks[k], db[k - 1]);
            LAUNCH_CHECK();
        }
    }
    if (dl0 || du0) {
        GradArgs<Ts> a = base_args(1);
        a.f0 = P->f0;
        a.dl0 = dl0;
        a.du0 = du0;
        const long n = (long)P->nl[0].C * P->nl[0].cols;
        ProfScope ps(P, st, ASD_K_GRAD_BOX, 0);
        bool done = false;
        if (!a.last) {
#define ASD_GB_CALL(N)                                        \
    TRY(grad_box_nm<N>(P, gs, dl0, du0, &done, st)); \
    break;
            ASD_NM_DISPATCH(a.nm, ASD_GB_CALL)
#undef ASD_GB_CALL
        }
        if (!done) {
            hipLaunchKernelGGL(k_grad_box<Ts>, dim3((unsigned)((n + kGradThreads - 1) / kGradThreads)),
                               dim3(kGradThreads), 0, st, a);
            LAUNCH_CHECK();
        }
    }
    return ASD_OK;
}

template <typename T>
T* field_ptr(asd_plan* P, int field, int k, int q) {
    ReluLayerT<T>& r = RL<T>(P)[k];
    switch (field) {
        case ASD_F_ALPHA: return r.alpha;
        case ASD_F_BETA0: return r.beta0;
        case ASD_F_BETA1: return r.beta1;
        case ASD_F_ALPHA_M: return r.alpha_m;
        case ASD_F_ALPHA_V: return r.alpha_v;
        case ASD_F_BETA0_M: return r.beta0_m;
        case ASD_F_BETA0_V: return r.beta0_v;
        case ASD_F_BETA1_M: return r.beta1_m;
        case ASD_F_BETA1_V: return r.beta1_v;
        case ASD_F_MASK_BETA: return r.slot[q].beta;
        case ASD_F_MASK_M: return r.slot[q].m;
        case ASD_F_MASK_V: return r.slot[q].v;
        case ASD_F_MASK_LI: return r.slot[q].LI;
        case ASD_F_MASK_UI: return r.slot[q].UI;
        default: return nullptr;
    }
}

asd_status check_field(asd_plan* P, int field, int k, int q) {
    if (!P) return fail(ASD_EINVAL, "NULL plan");
    if (!P->loaded) return fail(ASD_EINVAL, "asd_init has not been called");
    if (k < 1 || k >= P->n) return fail(ASD_EINVAL, "layer %d outside [1, %d]", k, P->n - 1);
    if (field < ASD_F_ALPHA || field > ASD_F_MASK_XPREV) return fail(ASD_EINVAL, "unknown field %d", field);
    if (field >= ASD_F_MASK_BETA && (q < 0 || q >= P->prm.max_masks))
        return fail(ASD_EINVAL, "slot %d outside [0, %d)", q, P->prm.max_masks);
    return ASD_OK;
}

bool is_moment(int field) {
    return field == ASD_F_ALPHA_M || field == ASD_F_ALPHA_V || field == ASD_F_BETA0_M || field == ASD_F_BETA0_V ||
           field == ASD_F_BETA1_M || field == ASD_F_BETA1_V || field == ASD_F_MASK_M || field == ASD_F_MASK_V;
}

// Moment fields of a mixed-mode plan: BF16 in the plan, float for the caller.
asd_status moment_bf16(asd_plan* P, int field, int k, int q, float* ext, int mode, hipStream_t st) {
    // both moments live in the m array: m in the high half, v in the low half
    int mfield = field, hi = 1;
    switch (field) {
        case ASD_F_ALPHA_V: mfield = ASD_F_ALPHA_M; hi = 0; break;
        case ASD_F_BETA0_V: mfield = ASD_F_BETA0_M; hi = 0; break;
        case ASD_F_BETA1_V: mfield = ASD_F_BETA1_M; hi = 0; break;
        case ASD_F_MASK_V: mfield = ASD_F_MASK_M; hi = 0; break;
        default: break;
    }
    uint32_t* arr = reinterpret_cast<uint32_t*>(field_ptr<float>(P, mfield, k, q));
    const NeuronLayout& nl = P->nl[k];
    dim3 grid((unsigned)((nl.cols + 255) / 256), (unsigned)nl.C);
    hipLaunchKernelGGL(k_layout_bf16, grid, dim3(256), 0, st, arr, ext, nl, P->S, mode, hi);
    LAUNCH_CHECK();
    return ASD_OK;
}

template <typename T>
asd_status state_get_t(asd_plan* P, int field, int k, int q, T* dst, hipStream_t st) {
    ReluLayerT<T>& r = RL<T>(P)[k];
    if constexpr (sizeof(T) == 4)
        if (bf16_moments(P) && is_moment(field)) return moment_bf16(P, field, k, q, dst, 2, st);
    if (field == ASD_F_MASK_Z)
        return launch_bits<T, T>(P->nl[k], P->S, 0, r.slot[q].zbits, dst, nullptr, nullptr, st);
    if (field == ASD_F_MASK_XPREV)
        return launch_bits<T, T>(P->nl[k - 1], P->S, 4, r.slot[q].xbits, dst, NA<T>(P)[k - 1].lo,
                                 NA<T>(P)[k - 1].hi, st);
    return launch_layout<T, T>(field_ptr<T>(P, field, k, q), dst, P->nl[k], P->S, 2, st);
}

template <typename T>
asd_status state_set_t(asd_plan* P, int field, int k, int q, const T* src, hipStream_t st) {
    ReluLayerT<T>& r = RL<T>(P)[k];
    T* s = const_cast<T*>(src);
    if constexpr (sizeof(T) == 4)
        if (bf16_moments(P) && is_moment(field)) return moment_bf16(P, field, k, q, s, 0, st);
    if (field == ASD_F_MASK_Z) {
        TRY((launch_bits<T, T>(P->nl[k], P->S, 2, r.slot[q].zbits, s, nullptr, nullptr, st)));
    } else if (field == ASD_F_MASK_XPREV) {
        TRY((launch_bits<T, T>(P->nl[k - 1], P->S, 1, r.slot[q].xbits, s, NA<T>(P)[k - 1].lo,
                               NA<T>(P)[k - 1].hi, st)));
    } else {
        TRY((launch_layout<T, T>(field_ptr<T>(P, field, k, q), s, P->nl[k], P->S, 0, st)));
    }
    if (field == ASD_F_MASK_Z || field == ASD_F_MASK_XPREV) TRY(pack_all<T>(P, 0, st));
    return derive_layer<T>(P, k, st);
}

template <typename T>
asd_status set_counts_t(asd_plan* P, int recompute, hipStream_t st) {
    if (recompute) {
        for (int k = 1; k < P->n; ++k)
            for (int q = 0; q < P->n_masks; ++q) {
                ReluLayerT<T>& r = RL<T>(P)[k];
                TRY(launch_mask_consts<T>(P, k, q, r.slot[q].zbits, r.slot[q].xbits, 0, st));
            }
    }
    for (int k = 1; k < P->n; ++k) TRY(derive_layer<T>(P, k, st));
    return pack_all<T>(P, 0, st);
}

// Minimiser, f, g of every layer and the supergradient at the current duals.
// General path: the term-wise kernels.  Iteration path (FP32-duals plans):
// the backward and forward launches of iteration() with the plan's kernel
// choices, the update replaced by writing the supergradient (kRuleEval).
template <typename T>
asd_status eval_t(asd_plan* P, const asd_eval_out* out, hipStream_t st) {
    constexpr bool kGeneral = sizeof(T) == 8;
    const bool iter = !kGeneral && out->path == ASD_EVAL_ITERATION;
    if (iter) {
        if (out->obj) return fail(ASD_EINVAL, "the iteration kernels do not form the objective (obj must be NULL)");
        struct Clear {
            asd_plan* P;
            ~Clear() {
                memset(P->ev_f, 0, sizeof(P->ev_f));
                memset(P->ev_g, 0, sizeof(P->ev_g));
            }
        } clear{P};
        for (int k = 0; k < P->n; ++k) P->ev_f[k] = out->f[k];
        const int kpair = bwd_pair_layer(P);
        for (int k = P->n - 1; k >= 0; --k) {
            if (k == kpair) continue;
            if (kpair >= 0 && k == P->n - 1) TRY(bwd_pair(P, st));
            else TRY(bwd_fast(P, k, st));
        }
        if (P->domain == ASD_DOMAIN_L2) {
            const float* f0 = out->f[0] ? reinterpret_cast<const float*>(out->f[0]) : P->f0f;
            TRY((l2_input<T, float>(P, f0, 0, nullptr, st)));
        }
        memset(P->ev_f, 0, sizeof(P->ev_f));
    } else {
        const bool l2 = P->domain == ASD_DOMAIN_L2;
        for (int k = P->n - 1; k >= 0; --k)
            TRY((launch_backward<T, T>(P, k, 1, ASD_K_OTHER, st, k == 0 && l2 ? P->f0 : nullptr, out->f[k])));
        if (l2) TRY((l2_input<T, double>(P, P->f0, 1, NA<T>(P)[0].term, st)));
        if (out->obj) TRY(reduce_objective<T>(P, out->obj, st));
    }
    for (int k = 0; k < P->n; ++k) {
        if (out->xstar[k])
            TRY((launch_layout<T, T>(NA<T>(P)[k].xstar, reinterpret_cast<T*>(out->xstar[k]), P->nl[k], P->S, 2,
                                     st)));
        if (k >= 1 && out->zstar[k])
            TRY((launch_bits<T, T>(P->nl[k], P->S, 0, RL<T>(P)[k].zbits, reinterpret_cast<T*>(out->zstar[k]),
                                   nullptr, nullptr, st)));
        if (k >= 1 && out->g[k])
            TRY((launch_layout<T, T>(RL<T>(P)[k].g, reinterpret_cast<T*>(out->g[k]), P->nl[k], P->S, 2, st)));
    }
    StepArgsT<T> sa = make_step_args<T>(P, 0.0);
    if (iter) {
        sa.rule = kRuleEval;
        bool any = false;
        for (int k = 1; k < P->n; ++k) {
            void* gk[3] = {out->grad_alpha[k], out->grad_beta0[k], out->grad_beta1[k]};
            for (int i = 0; i < 3; ++i) P->ev_g[k][i] = gk[i];
            for (int q = 0; q < kMaxMasks; ++q) P->ev_g[k][3 + q] = q < P->n_masks ? out->grad_mask[k][q] : nullptr;
            for (int i = 0; i < 3 + kMaxMasks; ++i) any = any || P->ev_g[k][i];
        }
        asd_status r = ASD_OK;
        if (any) {
            if constexpr (!kGeneral) r = forward_pass<T>(P, sa, st);
        }
        memset(P->ev_g, 0, sizeof(P->ev_g));
        return r;
    }
    for (int k = 1; k < P->n; ++k) {
        void* gout[3 + kMaxMasks] = {out->grad_alpha[k], out->grad_beta0[k], out->grad_beta1[k]};
        bool any = gout[0] || gout[1] || gout[2];
        for (int q = 0; q < kMaxMasks; ++q) {
            gout[3 + q] = out->grad_mask[k][q];
            any = any || gout[3 + q];
        }
        if (any) TRY(launch_forward<T>(P, k, sa, 1, gout, st));
    }
    return ASD_OK;
}

template <typename T>
asd_status oracle_t(asd_plan* P, int k, const T* x_prev, const T* z, uint32_t* bits, T* LI, T* UI,
                    hipStream_t st) {
    OracleArgs<T> a;
    a.g = P->geo[k];
    a.S = P->S;
    a.xprev = x_prev;
    a.z = z;
    a.lo_in = NA<T>(P)[k - 1].lo;
    a.hi_in = NA<T>(P)[k - 1].hi;
    a.bits = bits;
    a.LI = LI;
    a.UI = UI;
    const long n = (long)P->S * a.g.out.N;
    hipLaunchKernelGGL(k_oracle<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, a);
    LAUNCH_CHECK();
    return ASD_OK;
}

// Autotuning: each kernel choice of the FP32 iteration is timed alone on the
// loaded batch, with the plain rule at step size 0 so that no dual or moment
// changes (the backward kernels rewrite x* and its bits, which every
// iteration recomputes), and with `ktune` empty mask slots active (their
// multipliers are zero, so the products are those of K masks).
template <typename T>
asd_status autotune_t(asd_plan* P, int ktune, int reps, hipStream_t st) {
    const int nm0 = P->n_masks;
    const int rule0 = P->prm.rule;
    P->n_masks = ktune;
    P->prm.rule = ASD_RULE_SUPERGRADIENT;
    StepArgsT<T> sa = make_step_args<T>(P, 0.0);
    struct Restore {
        asd_plan* P;
        int nm, rule;
        ~Restore() {
            P->n_masks = nm;
            P->prm.rule = rule;
        }
    } restore{P, nm0, rule0};
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    asd_status err = ASD_OK;
    auto timed = [&](auto&& launch) -> float {
        if (err != ASD_OK) return 1e30f;
        asd_status r = launch();  // warm
        for (int i = 0; i < reps && r == ASD_OK; ++i) {
            if (i == 0 && hipEventRecord(e0, st) != hipSuccess) r = fail(ASD_EDEVICE, "hipEventRecord failed");
            if (r == ASD_OK) r = launch();
        }
        float ms = 1e30f;
        if (r == ASD_OK && (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                            hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
            r = fail(ASD_EDEVICE, "event timing failed");
        if (r != ASD_OK) err = r;
        return ms;
    };
    // every iterate's x* must exist before the forward kernels run
    for (int k = P->n - 1; k >= 0 && err == ASD_OK; --k) err = bwd_fast(P, k, st);
    for (int L = 1; L <= P->n && err == ASD_OK; ++L) {
        const LayerGeo& g = P->geo[L];
        if (L < P->n && g.kind == ASD_LAYER_DENSE) {
            const long cap = std::max(1L, std::min((long)kMaxKsplit, (long)(g.fan / (32 * KS))));
            int best = P->ksplit[L], bestkw = P->fwd_kw[L];
            float tbest = 1e30f;
            for (int kw = 4; kw <= 8; kw += 4)
                for (int ks = 1; ks <= cap; ks *= 2) {
                    P->ksplit[L] = ks;
                    P->fwd_kw[L] = kw;
                    const float t = timed([&] { return fwd_fast(P, L, sa, st); });
                    if (t < tbest) tbest = t, best = ks, bestkw = kw;
                }
            P->ksplit[L] = best;
            P->fwd_kw[L] = bestkw;
        }
        if (L < P->n && g.kind == ASD_LAYER_CONV2D) {
            // VALU column kernel, or the matrix cores with 4 or 8 waves per tile
            float tb[3];
            const int mf[3] = {0, 1, 1}, kw[3] = {8, 4, 8};
            for (int m = 0; m < 3; ++m) {
                P->fwd_mfma[L] = mf[m];
                P->fwd_kw[L] = kw[m];
                tb[m] = timed([&] { return fwd_fast(P, L, sa, st); });
            }
            const int b = tb[0] < tb[1] ? (tb[0] < tb[2] ? 0 : 2) : (tb[1] < tb[2] ? 1 : 2);
            P->fwd_mfma[L] = mf[b];
            P->fwd_kw[L] = kw[b];
        }
        const int k = L - 1;  // backward into neuron layer k through layer L
        const NeuronLayout& In = g.in;
        if (bwd_m4_fits(P, k)) {
            // matrix-core 4-channel kernel (0) or the VALU column kernel (4)
            float tb[2];
            const int cand[2] = {0, 4};
            for (int m = 0; m < 2; ++m) {
                P->bwd_cb[k] = cand[m];
                tb[m] = timed([&] { return bwd_fast(P, k, st); });
            }
            P->bwd_cb[k] = tb[0] <= tb[1] ? 0 : 4;
        }
        if (g.kind == ASD_LAYER_CONV2D && !(In.P % kWave == 0 && In.C >= 16) && In.C > 4) {
            float tb[2];
            const int cand[2] = {4, 8};
            for (int m = 0; m < 2; ++m) {
                P->bwd_cb[k] = cand[m];
                tb[m] = timed([&] { return bwd_fast(P, k, st); });
            }
            P->bwd_cb[k] = tb[0] < tb[1] ? 4 : 8;
        }
        if (g.kind == ASD_LAYER_CONV2D && In.P % kWave == 0 && In.C >= 16) {
            float tb[2];
            const int cand[2] = {2, 4};
            for (int m = 0; m < 2; ++m) {
                P->bwd_nt[k] = cand[m];
                tb[m] = timed([&] { return bwd_fast(P, k, st); });
            }
            P->bwd_nt[k] = tb[0] <= tb[1] ? 2 : 4;
        }
        if (g.kind == ASD_LAYER_DENSE && In.P % kWave == 0 && P->S >= 8) {
            // column kernel, positions on lanes with 4 or 8 waves, or the
            // matrix cores
            float tb[4];
            const int pos[4] = {0, 1, 1, 2}, kw[4] = {8, 4, 8, 4};
            int b = 0;
            for (int m = 0; m < 4; ++m) {
                P->bwd_pos[k] = pos[m];
                P->bwd_kw[k] = kw[m];
                tb[m] = timed([&] { return bwd_fast(P, k, st); });
                if (tb[m] < tb[b]) b = m;
            }
            P->bwd_pos[k] = pos[b];
            P->bwd_kw[k] = kw[b];
        }
    }
    // dense layers whose products can share the forward launch (with 8 waves
    // per split, beside a matrix-core convolution): waves and split count
    // timed with the whole forward pass (alone, more splits hide latency;
    // beside the convolutions, fewer blocks and no partial sums measure
    // faster), which also decides whether the layer shares the launch
    bool conv_mfma = false;
    for (int L = 1; L < P->n; ++L)
        conv_mfma |= P->geo[L].kind == ASD_LAYER_CONV2D && P->fwd_mfma[L] && P->fwd_kw[L] == 8;
    for (int L = 1; L < P->n && conv_mfma && P->prof != ASD_PROFILE_KERNELS && err == ASD_OK; ++L) {
        if (P->geo[L].kind != ASD_LAYER_DENSE) continue;
        const long cap = std::max(1L, std::min((long)kMaxKsplit, (long)(P->geo[L].fan / (32 * KS))));
        int best = P->ksplit[L], bestkw = P->fwd_kw[L];
        float tbest = 1e30f;
        for (int kw = 4; kw <= 8; kw += 4)
            for (int ks = 1; ks <= cap; ks *= 2) {
                P->ksplit[L] = ks;
                P->fwd_kw[L] = kw;
                const float t = timed([&] { return forward_pass<T>(P, sa, st); });
                if (t < tbest) tbest = t, best = ks, bestkw = kw;
            }
        P->ksplit[L] = best;
        P->fwd_kw[L] = bestkw;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return err;
}

template <typename T>
asd_status check_finite_t(asd_plan* P, int32_t* flags, hipStream_t st) {
    for (int k = 1; k < P->n; ++k) {
        const NeuronLayout& nl = P->nl[k];
        hipLaunchKernelGGL(k_flags_duals<T>, dim3((unsigned)((nl.cols + 255) / 256), (unsigned)nl.C), dim3(256), 0,
                           st, RL<T>(P)[k], nl, P->S, P->n_masks, flags);
        LAUNCH_CHECK();
    }
    return ASD_OK;
}

void invalidate_graph(asd_plan* P) {
    if (P->graph_valid) (void)hipGraphExecDestroy(P->graph_exec);
    P->graph_valid = false;
}

// Active Set iterations of the plan: the largest budget, or the schedule's T.
int as_iters_of(const asd_plan* P) { return P->ragged ? P->budgets[0] : P->prm.as_iters; }

}  // namespace

// Plan fields of a fresh plan over a workspace.
static void bind_plan(asd_plan* P, const asd_net* net, int S, const asd_params* params, void* workspace) {
    P->net = net;
    P->S = S;
    P->n = net->n;
    P->prm = *params;
    P->prof = ASD_PROFILE_OFF;
    P->prof_used = 0;
    setup_plan_geometry(P);
    Carver cv{reinterpret_cast<char*>(workspace), 0};
    carve(P, cv);
    P->Sa = S;
    P->ragged = false;
    P->min_valid = false;
    P->domain = ASD_DOMAIN_BOX;
    // LDS a block may use on the current device (64 KB where it cannot be read)
    int dev = 0, lds = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) {
        (void)hipGetLastError();  // no error left for the next launch check
        lds = 65536;
    }
    lds = std::max(lds, 65536);
    P->lds_max = lds;
}

// Workspace of asd_solve_static: one array per GPU the library runs on,
// kept until the process ends.  Host code reaches it only through the
// address hipGetSymbolAddress returns for the current device (the array's
// own name is a host-side stand-in).  Every call on a GPU reuses that GPU's
// array: asd_init clears all state a solve reads before writing it, and
// calls that overlap on one GPU race.
constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices];

}  // namespace

static asd_status scratch_of_current_device(void** out) {
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(ASD_EDEVICE, "device index %d outside [0, %d)", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(ASD_EDEVICE, "hipGetSymbolAddress of the static workspace failed: %s", hipGetErrorString(e));
        if ((uintptr_t)p % 256) return fail(ASD_EDEVICE, "static workspace is not 256-byte aligned");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return ASD_OK;
}

asd_status asd::launch_backward_iter(asd_plan* P, int k, hipStream_t st) {
    return launch_backward<float, float>(P, k, 0, ASD_K_BACKWARD, st);
}

// ===========================================================================
// Public API
// ===========================================================================
extern "C" {

const char* asd_last_error(void) { return g_err.c_str(); }
int32_t asd_abi_version(void) { return ASD_ABI_VERSION; }

void asd_params_default(asd_params* p) {
    if (!p) return;
    p->bigm_iters = 180;
    p->as_iters = 500;
    p->add_every = 450;
    p->add_count = 2;
    p->max_masks = 7;
    p->rule = ASD_RULE_ADAM;
    p->bigm_lr0 = 1e-2;
    p->bigm_lr1 = 1e-4;
    p->as_lr0 = 1e-3;
    p->as_lr1 = 1e-6;
    p->adam_beta1 = 0.9;
    p->adam_beta2 = 0.999;
    p->adam_eps = 1e-8;
    p->precision = ASD_PREC_FP32;
}

asd_status asd_net_create(const asd_layer_desc* layers, int32_t n_layers, asd_net** out) {
    if (!layers || !out) return fail(ASD_EINVAL, "NULL argument");
    if (n_layers < 2 || n_layers > ASD_MAX_LAYERS)
        return fail(ASD_EINVAL, "n_layers must be in [2, %d]", ASD_MAX_LAYERS);
    for (int i = 0; i < n_layers; ++i) {
        const asd_layer_desc& d = layers[i];
        if (!d.W || !d.b) return fail(ASD_EINVAL, "layer %d: NULL weight or bias", i + 1);
        if (d.kind == ASD_LAYER_DENSE) {
            if (d.in_c < 1 || d.out_c < 1) return fail(ASD_EINVAL, "layer %d: non-positive size", i + 1);
        } else if (d.kind == ASD_LAYER_CONV2D) {
            if (d.in_c < 1 || d.in_h < 1 || d.in_w < 1 || d.out_c < 1 || d.kernel < 1 || d.stride < 1 ||
                d.pad < 0)
                return fail(ASD_EINVAL, "layer %d: invalid convolution parameters", i + 1);
            if (d.kernel > 32) return fail(ASD_EINVAL, "layer %d: kernel size %d above 32", i + 1, d.kernel);
            const int oh = (d.in_h + 2 * d.pad - d.kernel) / d.stride + 1;
            const int ow = (d.in_w + 2 * d.pad - d.kernel) / d.stride + 1;
            if (oh < 1 || ow < 1 || oh != d.out_h || ow != d.out_w)
                return fail(ASD_EINVAL, "layer %d: output size %dx%d does not match (%dx%d)", i + 1, d.out_h,
                            d.out_w, oh, ow);
        } else {
            return fail(ASD_EINVAL, "layer %d: unknown kind %d", i + 1, d.kind);
        }
        if (i > 0) {
            const asd_layer_desc& p = layers[i - 1];
            const long prev_n = (long)p.out_c * (p.kind == ASD_LAYER_DENSE ? 1 : (long)p.out_h * p.out_w);
            if (d.kind == ASD_LAYER_DENSE) {
                if ((long)d.in_c != prev_n)
                    return fail(ASD_EINVAL, "layer %d: %d inputs but the previous layer has %ld outputs", i + 1,
                                d.in_c, prev_n);
            } else {
                if (p.kind != ASD_LAYER_CONV2D || d.in_c != p.out_c || d.in_h != p.out_h || d.in_w != p.out_w)
                    return fail(ASD_EINVAL, "layer %d: convolution input shape does not match layer %d", i + 1, i);
            }
        }
    }
    asd_net* net = new (std::nothrow) asd_net;
    if (!net) return fail(ASD_EINVAL, "host allocation failed");
    net->n = n_layers;
    net->L.assign(layers, layers + n_layers);
    *out = net;
    return ASD_OK;
}

void asd_net_destroy(asd_net* net) { delete net; }

asd_status asd_plan_workspace_size(const asd_net* net, int32_t S, const asd_params* params, size_t* bytes) {
    if (!net || !bytes) return fail(ASD_EINVAL, "NULL argument");
    if (S < 1) return fail(ASD_EINVAL, "S must be >= 1");
    TRY(check_params(params));
    asd_plan tmp{};
    tmp.net = net;
    tmp.S = S;
    tmp.n = net->n;
    tmp.prm = *params;
    setup_plan_geometry(&tmp);
    for (int k = 0; k <= tmp.n; ++k)
        if ((long)tmp.nl[k].C * tmp.nl[k].colpad >= (1L << 31))
            return fail(ASD_EINVAL, "layer %d holds %ld neurons over the batch; at most 2^31 are supported", k,
                        (long)tmp.nl[k].C * tmp.nl[k].colpad);
    Carver cv{nullptr, 0};
    carve(&tmp, cv);
    *bytes = cv.off + 256;
    return ASD_OK;
}

asd_status asd_plan_create(const asd_net* net, int32_t S, const asd_params* params, void* workspace,
                           size_t bytes, hipStream_t stream, asd_plan** out) {
    (void)stream;
    if (!net || !out || !workspace) return fail(ASD_EINVAL, "NULL argument");
    size_t need = 0;
    TRY(asd_plan_workspace_size(net, S, params, &need));
    if (bytes < need) return fail(ASD_ENOMEM, "workspace has %zu bytes, needs %zu", bytes, need);
    if ((uintptr_t)workspace % 256) return fail(ASD_EINVAL, "workspace must be 256-byte aligned");
    asd_plan* P = new (std::nothrow) asd_plan();  // value-initialised
    if (!P) return fail(ASD_EINVAL, "host allocation failed");
    bind_plan(P, net, S, params, workspace);
    *out = P;
    return ASD_OK;
}

asd_status asd_solve_static(const asd_net* net, const asd_params* params, const asd_batch* b, double* out_lb,
                            float* x0, hipStream_t st) {
    if (!net || !params || !b || !out_lb) return fail(ASD_EINVAL, "NULL argument");
    size_t need = 0;
    TRY(asd_plan_workspace_size(net, b->S, params, &need));
    if (need > kScratchBytes)
        return fail(ASD_EINVAL,
                    "S = %d needs %zu bytes of workspace; the static workspace of asd_solve_static holds %zu "
                    "(solve larger batches through a plan with a workspace of the caller's)",
                    b->S, need, kScratchBytes);
    void* ws = nullptr;
    TRY(scratch_of_current_device(&ws));
    // the plan lives on this stack frame: every launch below takes what it
    // needs as kernel arguments, so nothing host-side has to outlive the call
    asd_plan P{};
    bind_plan(&P, net, b->S, params, ws);
    return asd_solve(&P, b, out_lb, x0, st);
}

void asd_plan_destroy(asd_plan* plan) {
    if (!plan) return;
    invalidate_graph(plan);
    for (hipEvent_t e : plan->prof_pool) (void)hipEventDestroy(e);
    delete plan;
}

asd_status asd_plan_autotune(asd_plan* P, int32_t ktune, int32_t reps, hipStream_t st) {
    if (!P) return fail(ASD_EINVAL, "NULL plan");
    if (!P->loaded) return fail(ASD_EINVAL, "asd_init has not been called");
    if (ktune < 0 || ktune > P->prm.max_masks) return fail(ASD_EINVAL, "ktune %d outside [0, %d]", ktune, P->prm.max_masks);
    if (reps < 1) return fail(ASD_EINVAL, "reps must be >= 1");
    if (is64(P)) return ASD_OK;  // FP64 plans run the general kernels only
    if (P->n_masks > ktune) return fail(ASD_EINVAL, "the plan already has %d masks (> ktune)", P->n_masks);
    invalidate_graph(P);
    P->min_valid = false;
    return autotune_t<float>(P, ktune, reps, st);
}

asd_status asd_plan_get_tuning(const asd_plan* P, asd_tuning* out) {
    if (!P || !out) return fail(ASD_EINVAL, "NULL argument");
    memset(out, 0, sizeof(*out));
    for (int L = 1; L <= P->n; ++L) {
        out->ksplit[L - 1] = P->ksplit[L];
        out->fwd_mfma[L - 1] = P->fwd_mfma[L];
        out->bwd_cb[L - 1] = P->bwd_cb[L - 1];
        out->bwd_pos[L - 1] = P->bwd_pos[L - 1];
        out->bwd_nt[L - 1] = P->bwd_nt[L - 1];
        out->fwd_kw[L - 1] = P->fwd_kw[L];
        out->bwd_kw[L - 1] = P->bwd_kw[L - 1];
    }
    return ASD_OK;
}

asd_status asd_plan_set_tuning(asd_plan* P, const asd_tuning* in) {
    if (!P || !in) return fail(ASD_EINVAL, "NULL argument");
    for (int L = 1; L <= P->n; ++L) {
        if (in->ksplit[L - 1] < 1 || in->ksplit[L - 1] > kMaxKsplit)
            return fail(ASD_EINVAL, "ksplit of layer %d is %d, outside [1, %d]", L, in->ksplit[L - 1], kMaxKsplit);
        if (in->fwd_mfma[L - 1] != 0 && in->fwd_mfma[L - 1] != 1) return fail(ASD_EINVAL, "fwd_mfma must be 0 or 1");
        const int cb = in->bwd_cb[L - 1];
        if (cb != 0 && cb != 4 && cb != 8) return fail(ASD_EINVAL, "bwd_cb must be 0, 4 or 8");
        if (in->bwd_pos[L - 1] < 0 || in->bwd_pos[L - 1] > 2) return fail(ASD_EINVAL, "bwd_pos must be 0, 1 or 2");
        const int nt = in->bwd_nt[L - 1];
        if (nt != 0 && nt != 2 && nt != 4) return fail(ASD_EINVAL, "bwd_nt must be 0, 2 or 4");
        if (in->fwd_kw[L - 1] != 4 && in->fwd_kw[L - 1] != 8) return fail(ASD_EINVAL, "fwd_kw must be 4 or 8");
        if (in->bwd_kw[L - 1] != 4 && in->bwd_kw[L - 1] != 8) return fail(ASD_EINVAL, "bwd_kw must be 4 or 8");
    }
    invalidate_graph(P);
    for (int L = 1; L <= P->n; ++L) {
        P->ksplit[L] = in->ksplit[L - 1];
        P->fwd_mfma[L] = in->fwd_mfma[L - 1];
        P->bwd_cb[L - 1] = in->bwd_cb[L - 1];
        P->bwd_pos[L - 1] = in->bwd_pos[L - 1];
        P->bwd_nt[L - 1] = in->bwd_nt[L - 1];
        P->fwd_kw[L] = in->fwd_kw[L - 1];
        P->bwd_kw[L - 1] = in->bwd_kw[L - 1];
    }
    return ASD_OK;
}

asd_status asd_profile_enable(asd_plan* P, int32_t mode) {
    if (!P) return fail(ASD_EINVAL, "NULL plan");
    if (mode != ASD_PROFILE_OFF && mode != ASD_PROFILE_LAUNCHES && mode != ASD_PROFILE_KERNELS)
        return fail(ASD_EINVAL, "unknown profiling mode %d", mode);
    P->prof = mode;
    if (P->prof) {
        P->prof_recs.clear();
        P->prof_used = 0;
    }
    return ASD_OK;
}

asd_status asd_profile_read(asd_plan* P, asd_kernel_time* out, int32_t cap, int32_t* count) {
    if (!P || !count || (cap > 0 && !out)) return fail(ASD_EINVAL, "NULL argument");
    std::vector<asd_kernel_time> agg;
    for (const ProfRec& r : P->prof_recs) {
        HIP_TRY(hipEventSynchronize(r.b));
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, r.a, r.b));
        bool found = false;
        for (asd_kernel_time& t : agg)
            if (t.role == r.role && t.layer == r.layer) {
                t.launches += 1;
                t.total_ms += ms;
                found = true;
                break;
            }
        if (!found) agg.push_back(asd_kernel_time{r.role, r.layer, 1, (double)ms});
    }
    *count = (int32_t)agg.size();
    for (int i = 0; i < (int)agg.size() && i < cap; ++i) out[i] = agg[i];
    return ASD_OK;
}

asd_status asd_init(asd_plan* P, const asd_batch* b, hipStream_t st) {
    if (!P || !b) return fail(ASD_EINVAL, "NULL argument");
    P->min_valid = false;
    if (b->S != P->S) return fail(ASD_EINVAL, "batch has S = %d, plan has %d", b->S, P->S);
    if (!b->l0 || !b->u0 || !b->c) return fail(ASD_EINVAL, "NULL l0/u0/c");
    if (P->n > 1 && (!b->lhat || !b->uhat)) return fail(ASD_EINVAL, "NULL lhat/uhat");
    for (int k = 1; k < P->n; ++k)
        if (!b->lhat[k - 1] || !b->uhat[k - 1]) return fail(ASD_EINVAL, "NULL bound of layer %d", k);
    P->n_masks = 0;
    P->step = 0;
    for (int q = 0; q < kMaxMasks; ++q) P->mask_step[q] = 0;
    if (is64(P)) TRY(init_t<double>(P, b, st));
    else TRY(init_t<float>(P, b, st));
    P->loaded = true;
    P->sp_ready = false;  // the Saddle Point state belongs to the previous batch
    return ASD_OK;
}

asd_status asd_run(asd_plan* P, int32_t phase, int32_t t_begin, int32_t n_iters, hipStream_t st) {
    if (!P) return fail(ASD_EINVAL, "NULL plan");
    P->min_valid = false;
    if (!P->loaded) return fail(ASD_EINVAL, "asd_init has not been called");
    if (phase != ASD_PHASE_BIGM && phase != ASD_PHASE_AS) return fail(ASD_EINVAL, "unknown phase");
    const int T = phase == ASD_PHASE_BIGM ? P->prm.bigm_iters : as_iters_of(P);
    if (t_begin < 0 || n_iters < 0 || t_begin + n_iters > T)
        return fail(ASD_EINVAL, "iterations [%d, %d) outside [0, %d)", t_begin, t_begin + n_iters, T);
    const bool as = phase == ASD_PHASE_AS;
    if (is64(P)) return run_t<double>(P, as, t_begin, n_iters, T, st);
    return run_t<float>(P, as, t_begin, n_iters, T, st);
}

asd_status asd_bound(asd_plan* P, double* out_lb, float* x0, hipStream_t st) {
    if (!P || !out_lb) return fail(ASD_EINVAL, "NULL argument");
    if (!P->loaded) return fail(ASD_EINVAL, "asd_init has not been called");
    return is64(P) ? bound_f64(P, out_lb, x0, st) : bound_f32(P, out_lb, x0, st);
}

asd_status asd_bound_grad(asd_plan* P, const double* gs, double* const* dW, double* const* db, double* dl0,
                          double* du0, int32_t reuse, hipStream_t st) {
    if (!P || !gs) return fail(ASD_EINVAL, "NULL argument");
    if (!P->loaded) return fail(ASD_EINVAL, "asd_init has not been called");
    if (P->geo[P->n].kind != ASD_LAYER_DENSE)
        return fail(ASD_EINVAL, "the bound gradient needs a dense output layer");
    if (P->domain != ASD_DOMAIN_BOX) return fail(ASD_EINVAL, "the bound gradient is defined for box input domains");
    return is64(P) ? bound_grad_t<double>(P, gs, dW, db, dl0, du0, reuse, st)
                   : bound_grad_t<float>(P, gs, dW, db, dl0, du0, reuse, st);
}

asd_status asd_set_input_domain(asd_plan* P, int32_t domain, const float* centre, const float* radius,
                                hipStream_t st) {
    if (!P) return fail(ASD_EINVAL, "NULL plan");
    if (domain == ASD_DOMAIN_BOX) {
        invalidate_graph(P);
        P->domain = ASD_DOMAIN_BOX;
        return ASD_OK;
    }
    if (domain != ASD_DOMAIN_L2) return fail(ASD_EINVAL, "unknown input domain %d", domain);
    if (!centre || !radius) return fail(ASD_EINVAL, "NULL centre or radius");
    invalidate_graph(P);
    HIP_TRY(hipMemcpyAsync(P->ball_c, centre, sizeof(float) * P->nl[0].N * P->S, hipMemcpyDeviceToDevice, st));
    HIP_TRY(hipMemcpyAsync(P->ball_r, radius, sizeof(float) * P->S, hipMemcpyDeviceToDevice, st));
    P->domain = ASD_DOMAIN_L2;
    return ASD_OK;
}

asd_status asd_set_budgets(asd_plan* P, const int32_t* budgets, hipStream_t st) {
    if (!P) return fail(ASD_EINVAL, "NULL plan");
    if (!budgets) {
        invalidate_graph(P);
        P->ragged = false;
        P->budgets.clear();
        return ASD_OK;
    }
    for (int s = 0; s < P->S; ++s) {
        if (budgets[s] < 1) return fail(ASD_EINVAL, "budget of subproblem %d is %d; budgets must be >= 1", s, budgets[s]);
        if (s > 0 && budgets[s] > budgets[s - 1])
            return fail(ASD_EINVAL, "budgets must be non-increasing (subproblem %d: %d after %d)", s, budgets[s],
                        budgets[s - 1]);
    }
    invalidate_graph(P);
    P->budgets.assign(budgets, budgets + P->S);
    HIP_TRY(hipMemcpyAsync(P->budgets_dev, P->budgets.data(), sizeof(int) * P->S, hipMemcpyHostToDevice, st));
    // a later call may replace the host copy: finish this one first
    HIP_TRY(hipStreamSynchronize(st));
    P->ragged = true;
    return ASD_OK;
}

asd_status asd_solve(asd_plan* P, const asd_batch* b, double* out_lb, float* x0, hipStream_t st) {
    TRY(asd_init(P, b, st));
    TRY(asd_run(P, ASD_PHASE_BIGM, 0, P->prm.bigm_iters, st));
    TRY(asd_run(P, ASD_PHASE_AS, 0, as_iters_of(P), st));
    return asd_bound(P, out_lb, x0, st);
}

asd_status asd_check_finite(asd_plan* P, const double* lb, int32_t* flags, hipStream_t st) {
    if (!P || !lb || !flags) return fail(ASD_EINVAL, "NULL argument");
    if (!P->loaded) return fail(ASD_EINVAL, "asd_init has not been called");
    hipLaunchKernelGGL(k_flags_bound, dim3((unsigned)((P->S + 255) / 256)), dim3(256), 0, st, lb,
                       (const int32_t*)P->inflags, flags, P->S);
    LAUNCH_CHECK();
    return is64(P) ? check_finite_t<double>(P, flags, st) : check_finite_t<float>(P, flags, st);
}

asd_status asd_solve_graph(asd_plan* P, const asd_batch* b, double* out_lb, hipStream_t st) {
    if (!P || !b || !out_lb) return fail(ASD_EINVAL, "NULL argument");
    if (P->prof) return fail(ASD_EINVAL, "kernel profiling is on; it cannot run inside a captured graph");
    TRY(asd_init(P, b, st));
    if (!P->graph_valid) {
        // capture the iterations (kernels only: fills and copies inside them
        // are kernels too); the host state advances as the capture proceeds
        HIP_TRY(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
        asd_status r = asd_run(P, ASD_PHASE_BIGM, 0, P->prm.bigm_iters, st);
        if (r == ASD_OK) r = asd_run(P, ASD_PHASE_AS, 0, as_iters_of(P), st);
        hipGraph_t graph = nullptr;
        const hipError_t e = hipStreamEndCapture(st, &graph);
        if (r != ASD_OK) {
            if (graph) (void)hipGraphDestroy(graph);
            return r;
        }
        if (e != hipSuccess) return fail(ASD_EDEVICE, "hipStreamEndCapture failed: %s", hipGetErrorString(e));
        const hipError_t ei = hipGraphInstantiate(&P->graph_exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (ei != hipSuccess) return fail(ASD_EDEVICE, "hipGraphInstantiate failed: %s", hipGetErrorString(ei));
        P->graph_valid = true;
        P->graph_end_masks = P->n_masks;
        P->graph_end_step = P->step;
        for (int q = 0; q < kMaxMasks; ++q) P->graph_end_mask_step[q] = P->mask_step[q];
    }
    HIP_TRY(hipGraphLaunch(P->graph_exec, st));
    P->n_masks = P->graph_end_masks;
    P->step = P->graph_end_step;
    for (int q = 0; q < kMaxMasks; ++q) P->mask_step[q] = P->graph_end_mask_step[q];
    return asd_bound(P, out_lb, nullptr, st);
}

asd_status asd_solve_group(asd_plan* const* plans, const asd_batch* const* batches, double* const* out_lb,
                           int32_t n_plans, const hipStream_t* streams) {
    if (!plans || !batches || !out_lb || !streams || n_plans < 1) return fail(ASD_EINVAL, "NULL argument");
    for (int i = 0; i < n_plans; ++i) {
        if (!plans[i] || !batches[i] || !out_lb[i]) return fail(ASD_EINVAL, "NULL entry %d", i);
        for (int j = 0; j < i; ++j)
            if (plans[j] == plans[i]) return fail(ASD_EINVAL, "plan %d appears twice", i);
    }
    int tm = 0, ta = 0;
    for (int i = 0; i < n_plans; ++i) {
        TRY(asd_init(plans[i], batches[i], streams[i]));
        tm = std::max(tm, plans[i]->prm.bigm_iters);
        ta = std::max(ta, as_iters_of(plans[i]));
    }
    // one iteration of every plan in turn, each on its own stream, so the
    // kernels of different plans overlap on the device
    for (int t = 0; t < tm; ++t)
        for (int i = 0; i < n_plans; ++i)
            if (t < plans[i]->prm.bigm_iters) TRY(asd_run(plans[i], ASD_PHASE_BIGM, t, 1, streams[i]));
    for (int t = 0; t < ta; ++t)
        for (int i = 0; i < n_plans; ++i)
            if (t < as_iters_of(plans[i])) TRY(asd_run(plans[i], ASD_PHASE_AS, t, 1, streams[i]));
    for (int i = 0; i < n_plans; ++i) TRY(asd_bound(plans[i], out_lb[i], nullptr, streams[i]));
    return ASD_OK;
}

asd_status asd_state_get(asd_plan* P, int32_t field, int32_t k, int32_t q, void* dst, hipStream_t st) {
    TRY(check_field(P, field, k, q));
    if (!dst) return fail(ASD_EINVAL, "NULL destination");
    if (is64(P)) return state_get_t<double>(P, field, k, q, reinterpret_cast<double*>(dst), st);
    return state_get_t<float>(P, field, k, q, reinterpret_cast<float*>(dst), st);
}

asd_status asd_state_set(asd_plan* P, int32_t field, int32_t k, int32_t q, const void* src, hipStream_t st) {
    TRY(check_field(P, field, k, q));
    P->min_valid = false;
    if (!src) return fail(ASD_EINVAL, "NULL source");
    if (is64(P)) return state_set_t<double>(P, field, k, q, reinterpret_cast<const double*>(src), st);
    return state_set_t<float>(P, field, k, q, reinterpret_cast<const float*>(src), st);
}

asd_status asd_state_get_counts(const asd_plan* P, asd_counts* out) {
    if (!P || !out) return fail(ASD_EINVAL, "NULL argument");
    memset(out, 0, sizeof(*out));
    out->n_masks = P->n_masks;
    out->step = P->step;
    for (int q = 0; q < kMaxMasks; ++q) out->mask_step[q] = P->mask_step[q];
    return ASD_OK;
}

asd_status asd_state_set_counts(asd_plan* P, const asd_counts* in, int32_t recompute, hipStream_t st) {
    if (!P || !in) return fail(ASD_EINVAL, "NULL argument");
    P->min_valid = false;
    if (!P->loaded) return fail(ASD_EINVAL, "asd_init has not been called");
    if (in->n_masks < 0 || in->n_masks > P->prm.max_masks)
        return fail(ASD_EINVAL, "n_masks %d outside [0, %d]", in->n_masks, P->prm.max_masks);
    if (in->step < 0) return fail(ASD_EINVAL, "negative step");
    for (int q = 0; q < in->n_masks; ++q)
        if (in->mask_step[q] < 0) return fail(ASD_EINVAL, "negative mask step");
    P->n_masks = in->n_masks;
    P->step = in->step;
    for (int q = 0; q < kMaxMasks; ++q) P->mask_step[q] = q < in->n_masks ? in->mask_step[q] : 0;
    return is64(P) ? set_counts_t<double>(P, recompute, st) : set_counts_t<float>(P, recompute, st);
}

asd_status asd_eval(asd_plan* P, const asd_eval_out* out, hipStream_t st) {
    if (!P || !out) return fail(ASD_EINVAL, "NULL argument");
    P->min_valid = false;
    if (!P->loaded) return fail(ASD_EINVAL, "asd_init has not been called");
    if (out->path != ASD_EVAL_GENERAL && out->path != ASD_EVAL_ITERATION)
        return fail(ASD_EINVAL, "unknown evaluation path %d", out->path);
    return is64(P) ? eval_t<double>(P, out, st) : eval_t<float>(P, out, st);
}

asd_status asd_oracle(asd_plan* P, int32_t k, const void* x_prev, const void* z, uint32_t* mask_bits, void* LI,
                      void* UI, hipStream_t st) {
    if (!P || !x_prev || !z || !mask_bits || !LI || !UI) return fail(ASD_EINVAL, "NULL argument");
    if (!P->loaded) return fail(ASD_EINVAL, "asd_init has not been called");
    if (k < 1 || k >= P->n) return fail(ASD_EINVAL, "layer %d outside [1, %d]", k, P->n - 1);
    if (is64(P))
        return oracle_t<double>(P, k, reinterpret_cast<const double*>(x_prev), reinterpret_cast<const double*>(z),
                                mask_bits, reinterpret_cast<double*>(LI), reinterpret_cast<double*>(UI), st);
    return oracle_t<float>(P, k, reinterpret_cast<const float*>(x_prev), reinterpret_cast<const float*>(z),
                           mask_bits, reinterpret_cast<float*>(LI), reinterpret_cast<float*>(UI), st);
}

namespace {

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Workspace of asd_intermediate_bounds for ReLU layer k >= 2: the
// replicated batch of the sub-network of layers 1..k (2 n_k D subproblems),
// their bounds, and the sub-network's plan.
struct IbLayout {
    int S;
    size_t l0, u0, lh[kMaxLayers], uh[kMaxLayers], c, d, plan, total;
};

asd_status ib_layout(const asd_net& sub, const asd_plan& full, int D, const asd_params* prm, IbLayout& lay) {
    const int k = sub.n;
    const long S = 2L * full.nl[k].N * D;
    if (S > (1L << 30)) return fail(ASD_EINVAL, "layer %d: %ld subproblems", k, S);
    lay.S = (int)S;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off = align256(off + bytes);
        return at;
    };
    lay.l0 = take(sizeof(float) * S * full.nl[0].N);
    lay.u0 = take(sizeof(float) * S * full.nl[0].N);
    for (int i = 1; i < k; ++i) {
        lay.lh[i] = take(sizeof(float) * S * full.nl[i].N);
        lay.uh[i] = take(sizeof(float) * S * full.nl[i].N);
    }
    lay.c = take(sizeof(float) * S * full.nl[k].N);
    lay.d = take(sizeof(double) * S);
    size_t pb = 0;
    TRY(asd_plan_workspace_size(&sub, lay.S, prm, &pb));
    lay.plan = take(pb);
    lay.total = off;
    return ASD_OK;
}

asd_status launch_ibp(const LayerGeo& g, int S, const float* lo, const float* hi, bool clamp, float* lo_out,
                      float* hi_out, hipStream_t st) {
    IbpArgs a;
    a.g = g;
    a.S = S;
    a.lo_in = lo;
    a.hi_in = hi;
    a.clamp_in = clamp;
    a.lo_out = lo_out;
    a.hi_out = hi_out;
    const long n = (long)S * g.out.N;
    hipLaunchKernelGGL(k_ibp, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, a);
    LAUNCH_CHECK();
    return ASD_OK;
}

asd_status launch_rows(float* dst, const float* src, long rows, long n, int per, hipStream_t st) {
    const long tot = rows * n;
    hipLaunchKernelGGL(k_bcast_rows, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, dst, src, rows, (int)n,
                       per);
    LAUNCH_CHECK();
    return ASD_OK;
}

}  // namespace

asd_status asd_intermediate_workspace_size(const asd_net* net, int32_t D, const asd_params* params, size_t* bytes) {
    if (!net || !params || !bytes) return fail(ASD_EINVAL, "NULL argument");
    if (D < 1) return fail(ASD_EINVAL, "D must be >= 1");
    TRY(check_params(params));
    asd_plan full{};
    full.net = net;
    full.S = D;
    full.n = net->n;
    setup_plan_geometry(&full);
    size_t need = 256;
    for (int k = 2; k < net->n; ++k) {
        asd_net sub;
        sub.n = k;
        sub.L.assign(net->L.begin(), net->L.begin() + k);
        IbLayout lay;
        TRY(ib_layout(sub, full, D, params, lay));
        need = std::max(need, lay.total + 256);
    }
    *bytes = need;
    return ASD_OK;
}

asd_status asd_intermediate_bounds(const asd_net* net, int32_t D, const asd_params* params, const float* l0,
                                   const float* u0, float* const* lhat, float* const* uhat, void* workspace,
                                   size_t bytes, hipStream_t st) {
    if (!net || !params || !l0 || !u0 || !lhat || !uhat) return fail(ASD_EINVAL, "NULL argument");
    if (D < 1) return fail(ASD_EINVAL, "D must be >= 1");
    for (int k = 1; k < net->n; ++k)
        if (!lhat[k - 1] || !uhat[k - 1]) return fail(ASD_EINVAL, "NULL output of layer %d", k);
    size_t need = 0;
    TRY(asd_intermediate_workspace_size(net, D, params, &need));
    if (net->n > 2 && (!workspace || bytes < need))
        return fail(ASD_EINVAL, "workspace of %zu bytes; asd_intermediate_workspace_size asks %zu", bytes, need);
    asd_plan full{};
    full.net = net;
    full.S = D;
    full.n = net->n;
    setup_plan_geometry(&full);
    char* base = reinterpret_cast<char*>(align256(reinterpret_cast<size_t>(workspace)));
    for (int k = 1; k < net->n; ++k) {
        // interval propagation from the bounds found for layer k-1
        TRY(launch_ibp(full.geo[k], D, k == 1 ? l0 : lhat[k - 2], k == 1 ? u0 : uhat[k - 2], k > 1, lhat[k - 1],
                       uhat[k - 1], st));
        if (k == 1) continue;  // the box-constrained LP: interval propagation is exact
        asd_net sub;
        sub.n = k;
        sub.L.assign(net->L.begin(), net->L.begin() + k);
        IbLayout lay;
        TRY(ib_layout(sub, full, D, params, lay));
        const int nk = (int)full.nl[k].N;
        const int per = 2 * nk;
        float* l0s = reinterpret_cast<float*>(base + lay.l0);
        float* u0s = reinterpret_cast<float*>(base + lay.u0);
        TRY(launch_rows(l0s, l0, lay.S, full.nl[0].N, per, st));
        TRY(launch_rows(u0s, u0, lay.S, full.nl[0].N, per, st));
        const float* lhp[kMaxLayers] = {};
        const float* uhp[kMaxLayers] = {};
        for (int i = 1; i < k; ++i) {
            float* a = reinterpret_cast<float*>(base + lay.lh[i]);
            float* b = reinterpret_cast<float*>(base + lay.uh[i]);
            TRY(launch_rows(a, lhat[i - 1], lay.S, full.nl[i].N, per, st));
            TRY(launch_rows(b, uhat[i - 1], lay.S, full.nl[i].N, per, st));
            lhp[i - 1] = a;
            uhp[i - 1] = b;
        }
        float* c = reinterpret_cast<float*>(base + lay.c);
        const long nc = (long)lay.S * nk;
        hipLaunchKernelGGL(k_ib_objective, dim3((unsigned)((nc + 255) / 256)), dim3(256), 0, st, c, (long)lay.S, nk);
        LAUNCH_CHECK();
        double* dB = reinterpret_cast<double*>(base + lay.d);
        // the sub-network's solve on a plan held by this frame (every launch
        // takes what it needs as kernel arguments)
        asd_plan P{};
        bind_plan(&P, &sub, lay.S, params, base + lay.plan);
        const asd_batch b{lay.S, l0s, u0s, lhp, uhp, c};
        TRY(asd_solve(&P, &b, dB, nullptr, st));
        hipLaunchKernelGGL(k_ib_combine, dim3((unsigned)(((long)D * nk + 255) / 256)), dim3(256), 0, st,
                           lhat[k - 1], uhat[k - 1], (const double*)dB, D, nk);
        LAUNCH_CHECK();
    }
    return ASD_OK;
}

asd_status asd_interval_bounds(const asd_net* net, int32_t S, const float* l0, const float* u0,
                               float* const* lhat, float* const* uhat, hipStream_t st) {
    if (!net || !l0 || !u0 || !lhat || !uhat) return fail(ASD_EINVAL, "NULL argument");
    if (S < 1) return fail(ASD_EINVAL, "S must be >= 1");
    asd_plan tmp{};
    tmp.net = net;
    tmp.S = S;
    tmp.n = net->n;
    setup_plan_geometry(&tmp);
    const float* lo = l0;
    const float* hi = u0;
    for (int L = 1; L <= net->n; ++L) {
        if (!lhat[L - 1] || !uhat[L - 1]) return fail(ASD_EINVAL, "NULL output of layer %d", L);
        IbpArgs a;
        a.g = tmp.geo[L];
        a.S = S;
        a.lo_in = lo;
        a.hi_in = hi;
        a.clamp_in = L > 1;
        a.lo_out = lhat[L - 1];
        a.hi_out = uhat[L - 1];
        const long n = (long)S * a.g.out.N;
        hipLaunchKernelGGL(k_ibp, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, a);
        LAUNCH_CHECK();
        lo = lhat[L - 1];
        hi = uhat[L - 1];
    }
    return ASD_OK;
}

}  // extern "C"
