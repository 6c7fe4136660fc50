// Plan object of libasdual and the launch helpers shared by its translation
// units: asd_api.hip (host driver, general kernels, bound gradient) and
// asd_iter.hip, built once per active-mask count, which launches the
// iteration kernels of asd_fast.h for that count.
#pragma once
#include <hip/hip_runtime.h>

#include <stdarg.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "asd_fast.h"

namespace asd {

// Records the message of the calling thread's last error; returns st.
asd_status fail(asd_status st, const char* fmt, ...);

struct ProfRec {
    int role, layer;
    hipEvent_t a, b;
};

}  // namespace asd

#define HIP_TRY(expr)                                                                 \
    do {                                                                              \
        hipError_t e_ = (expr);                                                       \
        if (e_ != hipSuccess)                                                         \
            return fail(ASD_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

#define LAUNCH_CHECK()                                                                \
    do {                                                                              \
        hipError_t e_ = hipGetLastError();                                            \
        if (e_ != hipSuccess)                                                         \
            return fail(ASD_EDEVICE, "kernel launch failed: %s", hipGetErrorString(e_)); \
    } while (0)

#define TRY(expr)                      \
    do {                               \
        asd_status s_ = (expr);        \
        if (s_ != ASD_OK) return s_;   \
    } while (0)

struct asd_net {
    int n;  // layers
    std::vector<asd_layer_desc> L;
};

struct asd_plan {
    const asd_net* net;
    int S;
    int n;
    asd_params prm;
    asd::NeuronLayout nl[asd::kMaxLayers + 1];  // 0..n
    asd::LayerGeo geo[asd::kMaxLayers + 1];     // 1..n
    // typed views of the workspace; only those of the plan's precision are set
    asd::NeuronArraysT<float> naf[asd::kMaxLayers];
    asd::NeuronArraysT<double> nad[asd::kMaxLayers];
    asd::ReluLayerT<float> Rf[asd::kMaxLayers];
    asd::ReluLayerT<double> Rd[asd::kMaxLayers];
    float* cvecf;
    double* cvecd;
    // weight copies made at asd_init and iteration buffers
    float* Wt[asd::kMaxLayers + 1];        // [fan][Cpad] (ReLU layers)
    int Cpad[asd::kMaxLayers + 1];
    float* Wr[asd::kMaxLayers + 1];        // [n_out][fanpad] (dense layers)
    int fanpad[asd::kMaxLayers + 1];
    int ksplit[asd::kMaxLayers + 1];       // dense forward: blocks over the fan-in
    // kernel choices per layer (heuristic defaults, or asd_plan_autotune)
    int fwd_mfma[asd::kMaxLayers + 1];     // convolution forward on the matrix cores (else the VALU column kernel)
    int bwd_cb[asd::kMaxLayers + 1];       // column transposed convolution into layer k: channels per thread
    int bwd_pos[asd::kMaxLayers + 1];      // dense backward into layer k: positions on lanes
    int bwd_kw[asd::kMaxLayers + 1];       // dense backward with positions on lanes: waves per block (4 or 8)
    int fwd_kw[asd::kMaxLayers + 1];       // matrix-core convolution forward: waves per block (4 or 8)
    int bwd_nt[asd::kMaxLayers + 1];       // matrix-core transposed convolution into layer k: tiles per item (0 = 2 where it fits)
    float* Wb[asd::kMaxLayers + 1];        // convolution: class weights of the transposed product
    float* Wl4[asd::kMaxLayers + 1];       // convolution: weights in the column kernel's LDS layout, 4 and
    float* Wl8[asd::kMaxLayers + 1];       // 8 channels per group (k_col_weights)
    int nkp[asd::kMaxLayers + 1];
    void* part;                       // dense forward partial products
    int* pointflag;                   // [asd::kMaxLayers]: point box away from zero in layer k
    void* Rdev;                       // device copy of the asd::ReluLayerT array (update kernels)
    double* f0;                       // f_0 of the last bound evaluation
    bool min_valid;                   // x*, z* bits and f0 are those of the current state, in FP64
    // bound gradient: chunks of the two-stage reductions per layer and the
    // partial sums they write
    int gw_chunks[asd::kMaxLayers + 1];
    long gw_rchunk[asd::kMaxLayers + 1];
    int gb_chunks[asd::kMaxLayers + 1];
    long gb_rchunk[asd::kMaxLayers + 1];
    size_t gpart_w, gpart_b;          // doubles
    double* gpart;
    // per-subproblem Active Set budgets (non-increasing in s), or none
    bool ragged;
    std::vector<int> budgets;
    int* budgets_dev;                 // [S]
    int32_t* inflags;                 // [S] input check of the loaded batch (bit 2: invalid inputs)
    void* lrs;                        // [S] learning rates of the current iteration (T)
    int Sa;                           // subproblems the current iteration updates (a prefix)
    int lds_max;                      // LDS bytes one block may use on the plan's device
    float* negc;                      // convolutional output layer (FP32 duals): -c, layout of layer n
    // input domain (asd_set_input_domain): l2 ball centres [S][n_0], radii [S]
    // and, for FP32 iterations, f_0 [S][n_0] from the backward pass
    int domain;
    float* ball_c;
    float* ball_r;
    float* f0f;
    // Saddle Point state (asd_sp_init): arrays carved from the caller's SP
    // workspace, per layer and field (asd::SpArr), FP64 objective terms per
    // layer, and the step parameters; sp_ready until the next asd_init
    bool sp_ready;
    asd_sp_params sp_prm;
    void* sp_arr[asd::kMaxLayers][16];
    double* sp_term[asd::kMaxLayers];
    // captured iteration schedule (asd_solve_graph) and the host state it ends in
    hipGraphExec_t graph_exec;
    bool graph_valid;
    int graph_end_masks, graph_end_step, graph_end_mask_step[asd::kMaxMasks];
    // scalar state
    int n_masks;
    int step;
    int mask_step[asd::kMaxMasks];
    bool loaded;
    // evaluation at fixed duals through the iteration kernels (asd_eval):
    // caller arrays for f_k and the supergradient of layer k, null otherwise
    void* ev_f[asd::kMaxLayers];
    void* ev_g[asd::kMaxLayers][3 + asd::kMaxMasks];
    // kernel timing (asd_profile_mode)
    int prof;
    std::vector<asd::ProfRec> prof_recs;
    std::vector<hipEvent_t> prof_pool;
    size_t prof_used;
};

namespace asd {

template <typename T> NeuronArraysT<T>* NA(asd_plan* P);
template <> inline NeuronArraysT<float>* NA<float>(asd_plan* P) { return P->naf; }
template <> inline NeuronArraysT<double>* NA<double>(asd_plan* P) { return P->nad; }
template <typename T> ReluLayerT<T>* RL(asd_plan* P);
template <> inline ReluLayerT<float>* RL<float>(asd_plan* P) { return P->Rf; }
template <> inline ReluLayerT<double>* RL<double>(asd_plan* P) { return P->Rd; }
template <typename T> inline ReluLayerT<T>* RdevT(asd_plan* P) { return reinterpret_cast<ReluLayerT<T>*>(P->Rdev); }
template <typename T> T* CV(asd_plan* P);
template <> inline float* CV<float>(asd_plan* P) { return P->cvecf; }
template <> inline double* CV<double>(asd_plan* P) { return P->cvecd; }

inline bool is64(const asd_plan* P) { return P->prm.precision == ASD_PREC_FP64; }
// Adam moments stored as BF16 pairs (the mixed and the BF16 modes)
inline bool bf16_moments(const asd_plan* P) {
    return P->prm.precision == ASD_PREC_MIXED || P->prm.precision == ASD_PREC_BF16 ||
           P->prm.precision == ASD_PREC_BF16_ALL;
}
// BF16 operands in the forward matrix-core products (the supergradient's
// W x* and |W| (sigma . x*)), and in the transposed ones (f, which decides
// the minimiser)
inline bool bf16_forward(const asd_plan* P) {
    return P->prm.precision == ASD_PREC_BF16 || P->prm.precision == ASD_PREC_BF16_ALL;
}
inline bool bf16_backward(const asd_plan* P) { return P->prm.precision == ASD_PREC_BF16_ALL; }

// Event pair around one launch when profiling is on.
struct ProfScope {
    asd_plan* P;
    hipStream_t st;
    int idx;
    ProfScope(asd_plan* P_, hipStream_t st_, int role, int layer) : P(P_), st(st_), idx(-1) {
        if (!P || !P->prof) return;
        if (P->prof_used + 2 > P->prof_pool.size()) {
            for (int i = 0; i < 256; ++i) {
                hipEvent_t e;
                if (hipEventCreate(&e) != hipSuccess) return;
                P->prof_pool.push_back(e);
            }
        }
        ProfRec r{role, layer, P->prof_pool[P->prof_used], P->prof_pool[P->prof_used + 1]};
        P->prof_used += 2;
        if (hipEventRecord(r.a, st) != hipSuccess) return;
        idx = (int)P->prof_recs.size();
        P->prof_recs.push_back(r);
    }
    ~ProfScope() {
        if (idx >= 0) (void)hipEventRecord(P->prof_recs[idx].b, st);
    }
};

inline dim3 grid_cols(const NeuronLayout& nl, int chan_per_block) {
    return dim3((unsigned)((nl.cols + 63) / 64), (unsigned)((nl.C + chan_per_block - 1) / chan_per_block));
}

// Geometry of layer L restricted to the subproblems the current iteration
// updates (s < Sa): column counts cover that prefix; strides, bit strides and
// arrays are unchanged.
inline LayerGeo gview(const asd_plan* P, int L) {
    LayerGeo g = P->geo[L];
    g.in.cols = (long)P->Sa * g.in.P;
    g.out.cols = (long)P->Sa * g.out.P;
    return g;
}

#define ASD_NM_DISPATCH(nm, CALL)                                          \
    switch (nm) {                                                          \
        case 0: CALL(0);                                                   \
        case 1: CALL(1);                                                   \
        case 2: CALL(2);                                                   \
        case 3: CALL(3);                                                   \
        case 4: CALL(4);                                                   \
        case 5: CALL(5);                                                   \
        case 6: CALL(6);                                                   \
        case 7: CALL(7);                                                   \
        case 8: CALL(8);                                                   \
        default: return fail(ASD_EINVAL, "mask count %d outside [0, 8]", (int)(nm)); \
    }

template <typename T>
FastFwdArgs<T> fwd_args(asd_plan* P, int k, int nm, const StepArgsT<T>& sa) {
    FastFwdArgs<T> a;
    memset(&a, 0, sizeof(a));
    a.g = gview(P, k);
    a.S = P->S;
    a.Sa = P->Sa;
    a.nm = nm;
    a.Cpad = P->Cpad[k];
    a.ksplit = P->ksplit[k];
    a.Wt = P->Wt[k];
    a.xin = NA<T>(P)[k - 1].xstar;
    a.xpk = NA<T>(P)[k - 1].xpk;
    a.pointflag = P->pointflag + (k - 1);
    a.xout = NA<T>(P)[k].xstar;
    a.R = RdevT<T>(P) + k;
    a.st = sa;
    a.part = reinterpret_cast<T*>(P->part);
    a.freeze = P->domain == ASD_DOMAIN_L2 && k == 1;
    if (sa.rule == kRuleEval)
        for (int i = 0; i < 3 + kMaxMasks; ++i) a.gout[i] = reinterpret_cast<T*>(P->ev_g[k][i]);
    return a;
}

// Staged operand images of the transposed convolution through layer k+1
// (k_bwd_conv_mfma, k_bwd_conv_m4): taps per axis, zero border, image size.
inline BwdConvShape conv_shape(const LayerGeo& g) {
    BwdConvShape sh;
    memset(&sh, 0, sizeof(sh));
    const int st_ = g.stride, pd = g.pad;
    sh.J = (g.ksz + st_ - 1) / st_;
    sh.off = sh.J - 1;
    const int qymax = (g.in.H - 1 + pd) / st_, qxmax = (g.in.W - 1 + pd) / st_;
    sh.Hp = std::max(g.out.H, qymax + 1) + sh.off;
    sh.Wp = std::max(g.out.W, qxmax + 1) + sh.off;
    sh.dimg = FastDiv{sh.Hp * sh.Wp, 1.0f / (float)(sh.Hp * sh.Wp)};
    sh.dWp = FastDiv{sh.Wp, 1.0f / (float)sh.Wp};
    sh.dOP = FastDiv{g.out.P, 1.0f / (float)g.out.P};
    sh.dOW = FastDiv{g.out.W, 1.0f / (float)g.out.W};
    return sh;
}

// The transposed convolution into layer k fits k_bwd_conv_m4: layer k is the
// input, stride 2, at most 4 channels, every 64-position run whole rows of layer k or part of
// one with an even number of columns per parity, at most 16 such runs per
// subproblem, and the staged images of one output channel within the LDS
// share of a product at any mask count.
inline bool bwd_m4_fits(const asd_plan* P, int k) {
    const LayerGeo& g = P->geo[k + 1];
    const NeuronLayout& L = g.in;
    if (k != 0 || g.kind != ASD_LAYER_CONV2D || g.stride != 2 || L.C > 4 || k + 1 == P->n) return false;
    if (L.P % kWave != 0 || L.P > 16 * kWave || L.W % 8 != 0 || !(L.W % kWave == 0 || kWave % L.W == 0))
        return false;
    const BwdConvShape sh = conv_shape(g);
    return sh.Hp * sh.Wp <= bwd_mfma_rs<kMaxMasks>();
}

template <typename T>
FastBwdArgs<T> bwd_args(asd_plan* P, int k, int nm) {
    FastBwdArgs<T> a;
    memset(&a, 0, sizeof(a));
    a.gn = gview(P, k + 1);
    a.S = P->S;
    a.k = k;
    a.last = (k + 1 == P->n);
    a.nm = nm;
    a.Wr = P->Wr[k + 1];
    a.fanpad = P->fanpad[k + 1];
    a.cvec = CV<T>(P);
    if (!a.last) {
        const ReluLayerT<T>& rn = RL<T>(P)[k + 1];
        a.vs = rn.vs;
        for (int q = 0; q < nm; ++q) a.u[q] = rn.slot[q].u;
    } else {
        a.vs = reinterpret_cast<const T*>(P->negc);  // a convolutional output layer's operand
    }
    a.xpk = NA<T>(P)[k].xpk;
    a.nk = NA<T>(P)[k];
    if (k >= 1) {
        const ReluLayerT<T>& r = RL<T>(P)[k];
        a.own = r.own;
        a.gk = r.g;
        a.zbits = r.zbits;
    }
    a.Wb = P->Wb[k + 1];
    a.Wl4 = P->Wl4[k + 1];
    a.Wl8 = P->Wl8[k + 1];
    a.nkp = P->nkp[k + 1];
    a.fout = reinterpret_cast<T*>(P->ev_f[k]);
    if (k == 0 && P->domain == ASD_DOMAIN_L2 && !a.fout) a.fout = reinterpret_cast<T*>(P->f0f);
    return a;
}

// Launches of the iteration kernels for NM active masks (asd_iter.hip, one
// translation unit per NM; mb: BF16-stored moments).
template <int NM>
asd_status fwd_fast_nm(asd_plan* P, int k, const StepArgsT<float>& sa, bool mb, hipStream_t st);
template <int NM>
asd_status fwd_fused_nm(asd_plan* P, int kc, int kd, const StepArgsT<float>& sa, bool mb, hipStream_t st);
template <int NM>
asd_status fwd_trio_nm(asd_plan* P, int kv, int kc, int kd, const StepArgsT<float>& sa, bool mb, hipStream_t st);
template <int NM>
asd_status bwd_pair_nm(asd_plan* P, hipStream_t st);
template <int NM>
asd_status bwd_fast_nm(asd_plan* P, int k, hipStream_t st);

// The general backward kernel as an iteration step (shapes the column
// transposed convolution cannot hold in LDS); asd_api.hip.
asd_status launch_backward_iter(asd_plan* P, int k, hipStream_t st);

}  // namespace asd
