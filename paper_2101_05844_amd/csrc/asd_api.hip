// Host side of libasdual: validation, workspace layout, and the iteration
// driver of Algorithm 1 / Algorithm 3 (kernels in asd_kernels.h).
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <new>
#include <string>
#include <vector>

#include "asd_kernels.h"

using namespace asd;

namespace {

thread_local std::string g_err = "no error";

asd_status fail(asd_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

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

}  // namespace

struct asd_net {
    int n;  // layers
    std::vector<asd_layer_desc> L;
};

struct ProfRec {
    int role, layer;
    hipEvent_t a, b;
};

struct asd_plan {
    const asd_net* net;
    int S;
    int n;
    asd_params prm;
    NeuronLayout nl[kMaxLayers + 1];  // 0..n
    LayerGeo geo[kMaxLayers + 1];     // 1..n
    NeuronArrays na[kMaxLayers];      // 0..n-1
    ReluLayer R[kMaxLayers];          // 1..n-1
    float* cvec;                      // objective rows, layout n
    // scalar state
    int n_masks;
    int step;
    int mask_step[kMaxMasks];
    bool loaded;
    // kernel timing
    bool prof;
    std::vector<ProfRec> prof_recs;
    std::vector<hipEvent_t> prof_pool;
    size_t prof_used;
};

namespace {

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

}  // namespace

// ---------------------------------------------------------------------------
// Workspace carving (two passes: measure, then assign).
// ---------------------------------------------------------------------------
namespace {

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

void carve(asd_plan* P, Carver& cv) {
    const int S = P->S;
    for (int k = 0; k < P->n; ++k) {
        const NeuronLayout& nl = P->nl[k];
        const size_t ns = (size_t)nl.N * S;
        NeuronArrays& a = P->na[k];
        a.lo = cv.take<float>(ns);
        a.hi = cv.take<float>(ns);
        a.xstar = cv.take<float>(ns);
        a.xbits = cv.take<uint32_t>(nl.words);
        a.deg = cv.take<uint32_t>(nl.words);
        a.term = cv.take<double>(ns);
    }
    for (int k = 1; k < P->n; ++k) {
        const NeuronLayout& nl = P->nl[k];
        const size_t ns = (size_t)nl.N * S;
        ReluLayer& r = P->R[k];
        memset(&r, 0, sizeof(r));
        r.lhat = cv.take<float>(ns);
        r.uhat = cv.take<float>(ns);
        r.alpha = cv.take<float>(ns);
        r.beta0 = cv.take<float>(ns);
        r.beta1 = cv.take<float>(ns);
        r.alpha_m = cv.take<float>(ns);
        r.alpha_v = cv.take<float>(ns);
        r.beta0_m = cv.take<float>(ns);
        r.beta0_v = cv.take<float>(ns);
        r.beta1_m = cv.take<float>(ns);
        r.beta1_v = cv.take<float>(ns);
        r.own = cv.take<float>(ns);
        r.g = cv.take<float>(ns);
        r.vdn = cv.take<float>(ns);
        r.zbits = cv.take<uint32_t>(nl.words);
        r.own64 = cv.take<double>(ns);
        r.g64 = cv.take<double>(ns);
        r.const64 = cv.take<double>(ns);
        for (int q = 0; q < P->prm.max_masks; ++q) {
            MaskSlot& m = r.slot[q];
            m.beta = cv.take<float>(ns);
            m.m = cv.take<float>(ns);
            m.v = cv.take<float>(ns);
            m.LI = cv.take<float>(ns);
            m.UI = cv.take<float>(ns);
            m.u = cv.take<float>(ns);
            m.zbits = cv.take<uint32_t>(nl.words);
            m.xbits = cv.take<uint32_t>(P->nl[k - 1].words);
        }
    }
    P->cvec = cv.take<float>((size_t)P->nl[P->n].N * S);
}

asd_status check_params(const asd_params* p) {
    if (!p) return fail(ASD_EINVAL, "params is NULL");
    if (p->bigm_iters < 0 || p->as_iters < 0) return fail(ASD_EINVAL, "negative iteration count");
    if (p->add_every < 1) return fail(ASD_EINVAL, "add_every must be >= 1");
    if (p->add_count < 0) return fail(ASD_EINVAL, "add_count must be >= 0");
    if (p->max_masks < 0 || p->max_masks > ASD_MAX_MASKS)
        return fail(ASD_EINVAL, "max_masks must be in [0, %d]", ASD_MAX_MASKS);
    if (p->rule != ASD_RULE_ADAM && p->rule != ASD_RULE_SUPERGRADIENT) return fail(ASD_EINVAL, "unknown rule");
    if (!(p->adam_beta1 >= 0.f && p->adam_beta1 < 1.f && p->adam_beta2 >= 0.f && p->adam_beta2 < 1.f))
        return fail(ASD_EINVAL, "Adam betas must be in [0, 1)");
    if (!(p->adam_eps > 0.f)) return fail(ASD_EINVAL, "Adam eps must be > 0");
    return ASD_OK;
}

asd_status setup_plan_geometry(asd_plan* P) {
    const asd_net* net = P->net;
    const int S = P->S;
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
    }
    return ASD_OK;
}

inline dim3 grid_cols(const NeuronLayout& nl, int chan_per_block) {
    return dim3((unsigned)(nl.colpad / 64), (unsigned)((nl.C + chan_per_block - 1) / chan_per_block));
}

asd_status zero_floats(float* p, size_t n, hipStream_t st) {
    if (n == 0) return ASD_OK;
    const long words = (long)n;
    hipLaunchKernelGGL(k_zero_words, dim3((unsigned)((words + 255) / 256)), dim3(256), 0, st,
                       reinterpret_cast<uint32_t*>(p), words);
    LAUNCH_CHECK();
    return ASD_OK;
}

asd_status zero_words(uint32_t* p, long n, hipStream_t st) {
    if (n == 0) return ASD_OK;
    hipLaunchKernelGGL(k_zero_words, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, n);
    LAUNCH_CHECK();
    return ASD_OK;
}

asd_status copy_words(uint32_t* dst, const uint32_t* src, long n, hipStream_t st) {
    hipLaunchKernelGGL(k_copy_words, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, dst, src, n);
    LAUNCH_CHECK();
    return ASD_OK;
}

asd_status launch_layout(float* dst, const float* src, const NeuronLayout& nl, int S, int mode,
                         hipStream_t st) {
    dim3 grid((unsigned)((nl.cols + 255) / 256), (unsigned)nl.C);
    hipLaunchKernelGGL(k_layout, grid, dim3(256), 0, st, dst, src, nl, S, mode);
    LAUNCH_CHECK();
    return ASD_OK;
}

asd_status launch_bits(const NeuronLayout& nl, int S, int mode, uint32_t* bits, float* fext,
                       const float* lo, const float* hi, hipStream_t st) {
    BitArgs a;
    a.nl = nl;
    a.S = S;
    a.mode = mode;
    a.bits = bits;
    a.fext = fext;
    a.lo = lo;
    a.hi = hi;
    dim3 grid((unsigned)(nl.colpad / 256 + 1), (unsigned)nl.C);
    hipLaunchKernelGGL(k_bits, grid, dim3(256), 0, st, a);
    LAUNCH_CHECK();
    return ASD_OK;
}

asd_status derive_layer(asd_plan* P, int k, hipStream_t st) {
    DeriveArgs a;
    a.nl = P->nl[k];
    a.S = P->S;
    a.nm = P->n_masks;
    a.b = P->geo[k].b;
    a.R = P->R[k];
    dim3 grid((unsigned)((a.nl.cols + 255) / 256), (unsigned)a.nl.C);
    hipLaunchKernelGGL(k_derive, grid, dim3(256), 0, st, a);
    LAUNCH_CHECK();
    return ASD_OK;
}

// Backward pass for neuron layer k (f_k, inner minimisation, terms).
template <typename T>
asd_status launch_backward(asd_plan* P, int k, int want_obj, hipStream_t st) {
    BwdArgs a;
    memset(&a, 0, sizeof(a));
    a.gn = P->geo[k + 1];
    a.S = P->S;
    a.k = k;
    a.last = (k + 1 == P->n);
    a.nm_next = a.last ? 0 : P->n_masks;
    a.nm_own = k >= 1 ? P->n_masks : 0;
    a.cvec = P->cvec;
    if (!a.last) a.Rn = P->R[k + 1];
    if (k >= 1) {
        a.Rk = P->R[k];
        a.bk = P->geo[k].b;
    }
    a.nk = P->na[k];
    a.want_obj = want_obj;
    const size_t lds = (size_t)KS * CB * kWave * sizeof(T);
    ProfScope ps(P, st, sizeof(T) == 8 ? ASD_K_FINAL : ASD_K_BACKWARD, k);
    hipLaunchKernelGGL(k_backward<T>, grid_cols(P->nl[k], CB), dim3(kWave, KS), lds, st, a);
    LAUNCH_CHECK();
    return ASD_OK;
}

asd_status launch_forward(asd_plan* P, int k, const StepArgs& sa, int mode, float* const* gout,
                          hipStream_t st) {
    FwdArgs a;
    memset(&a, 0, sizeof(a));
    a.g = P->geo[k];
    a.S = P->S;
    a.nm = P->n_masks;
    a.xin = P->na[k - 1].xstar;
    a.deg_in = P->na[k - 1].deg;
    a.xout = P->na[k].xstar;
    a.zbits = P->R[k].zbits;
    a.R = P->R[k];
    a.st = sa;
    a.mode = mode;
    if (gout)
        for (int i = 0; i < 3 + kMaxMasks; ++i) a.gout[i] = gout[i];
    const size_t lds = (size_t)KS * CB * (1 + a.nm) * kWave * sizeof(float);
    ProfScope ps(P, st, mode == 0 ? ASD_K_FORWARD : ASD_K_OTHER, k);
    hipLaunchKernelGGL(k_forward, grid_cols(P->nl[k], CB), dim3(kWave, KS), lds, st, a);
    LAUNCH_CHECK();
    return ASD_OK;
}

// Mask constants of slot q of layer k from the given bit sources (FP32).
asd_status launch_mask_consts(asd_plan* P, int k, int q, const uint32_t* zsrc, const uint32_t* xsrc,
                              int zero_state, hipStream_t st) {
    MaskArgs a;
    memset(&a, 0, sizeof(a));
    a.g = P->geo[k];
    a.S = P->S;
    a.q = q;
    a.nm = 1;
    a.lo_in = P->na[k - 1].lo;
    a.hi_in = P->na[k - 1].hi;
    a.zsrc = zsrc;
    a.xsrc = xsrc;
    a.zero_state = zero_state;
    a.deg_in = P->na[k - 1].deg;
    a.R = P->R[k];
    const size_t lds = (size_t)KS * CB * 2 * kWave * sizeof(float);
    ProfScope ps(P, st, ASD_K_MASK, k);
    hipLaunchKernelGGL(k_mask_consts<float>, grid_cols(P->nl[k], CB), dim3(kWave, KS), lds, st, a);
    LAUNCH_CHECK();
    return ASD_OK;
}

asd_status launch_final_sums(asd_plan* P, int k, hipStream_t st) {
    MaskArgs a;
    memset(&a, 0, sizeof(a));
    a.g = P->geo[k];
    a.S = P->S;
    a.q = 0;
    a.nm = P->n_masks;
    a.lo_in = P->na[k - 1].lo;
    a.hi_in = P->na[k - 1].hi;
    a.deg_in = P->na[k - 1].deg;
    a.R = P->R[k];
    const size_t lds = (size_t)KS * CB * 2 * kWave * sizeof(double);
    ProfScope ps(P, st, ASD_K_FINAL, k);
    hipLaunchKernelGGL(k_mask_consts<double>, grid_cols(P->nl[k], CB), dim3(kWave, KS), lds, st, a);
    LAUNCH_CHECK();
    return ASD_OK;
}

asd_status reduce_objective(asd_plan* P, double* out, hipStream_t st) {
    ReduceArgs a;
    memset(&a, 0, sizeof(a));
    a.S = P->S;
    a.nlayers = P->n;
    for (int k = 0; k < P->n; ++k) {
        a.nl[k] = P->nl[k];
        a.term[k] = P->na[k].term;
    }
    // b_n^T c_s from the internal copy of c (layout n: [n_last][S])
    a.cint = P->cvec;
    a.bn = P->geo[P->n].b;
    a.n_last = P->nl[P->n].C;
    a.out = out;
    hipLaunchKernelGGL(k_reduce_obj, dim3((unsigned)P->S), dim3(256), 0, st, a);
    LAUNCH_CHECK();
    return ASD_OK;
}

float linear_lr(float lr0, float lr1, int t, int T) {
    if (T <= 1) return lr0;
    return (float)((double)lr0 + ((double)lr1 - (double)lr0) * (double)t / (double)(T - 1));
}

StepArgs make_step_args(const asd_plan* P, float lr) {
    StepArgs sa;
    memset(&sa, 0, sizeof(sa));
    sa.rule = P->prm.rule;
    sa.lr = lr;
    sa.b1 = P->prm.adam_beta1;
    sa.b2 = P->prm.adam_beta2;
    sa.eps = P->prm.adam_eps;
    auto bc = [&](int step, float* c1, float* c2) {
        const int s = step > 0 ? step : 1;
        *c1 = (float)(1.0 - pow((double)P->prm.adam_beta1, (double)s));
        *c2 = (float)(1.0 - pow((double)P->prm.adam_beta2, (double)s));
    };
    bc(P->step, &sa.bc1[0], &sa.bc2[0]);
    for (int q = 0; q < kMaxMasks; ++q) bc(q < P->n_masks ? P->mask_step[q] : 1, &sa.bc1[1 + q], &sa.bc2[1 + q]);
    return sa;
}

asd_status reset_group_moments(asd_plan* P, hipStream_t st) {
    for (int k = 1; k < P->n; ++k) {
        const size_t ns = (size_t)P->nl[k].N * P->S;
        ReluLayer& r = P->R[k];
        float* arrs[6] = {r.alpha_m, r.alpha_v, r.beta0_m, r.beta0_v, r.beta1_m, r.beta1_v};
        for (float* a : arrs) {
            asd_status s = zero_floats(a, ns, st);
            if (s) return s;
        }
    }
    P->step = 0;
    return ASD_OK;
}

// One iteration: backward pass, optional active-set extension, forward pass.
asd_status iteration(asd_plan* P, bool as_phase, int t, float lr, hipStream_t st) {
    asd_status s;
    for (int k = P->n - 1; k >= 0; --k)
        if ((s = launch_backward<float>(P, k, 0, st))) return s;
    if (as_phase && P->n >= 2 && (t % P->prm.add_every) < P->prm.add_count &&
        P->n_masks < P->prm.max_masks) {
        const int q = P->n_masks;
        for (int k = 1; k < P->n; ++k) {
            if ((s = copy_words(P->R[k].slot[q].zbits, P->R[k].zbits, P->nl[k].words, st))) return s;
            if ((s = copy_words(P->R[k].slot[q].xbits, P->na[k - 1].xbits, P->nl[k - 1].words, st))) return s;
            if ((s = launch_mask_consts(P, k, q, P->R[k].zbits, P->na[k - 1].xbits, 1, st))) return s;
        }
        P->mask_step[q] = 0;
        P->n_masks = q + 1;
    }
    if (P->prm.rule == ASD_RULE_ADAM) {
        P->step += 1;
        for (int q = 0; q < P->n_masks; ++q) P->mask_step[q] += 1;
    }
    const StepArgs sa = make_step_args(P, lr);
    for (int k = 1; k < P->n; ++k)
        if ((s = launch_forward(P, k, sa, 0, nullptr, st))) return s;
    return ASD_OK;
}

}  // namespace

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
    p->bigm_lr0 = 1e-2f;
    p->bigm_lr1 = 1e-4f;
    p->as_lr0 = 1e-3f;
    p->as_lr1 = 1e-6f;
    p->adam_beta1 = 0.9f;
    p->adam_beta2 = 0.999f;
    p->adam_eps = 1e-8f;
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
    if (layers[n_layers - 1].kind != ASD_LAYER_DENSE)
        return fail(ASD_EINVAL, "the last layer must be dense");
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
    asd_status s = check_params(params);
    if (s) return s;
    asd_plan tmp{};
    tmp.net = net;
    tmp.S = S;
    tmp.n = net->n;
    tmp.prm = *params;
    setup_plan_geometry(&tmp);
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
    asd_status s = asd_plan_workspace_size(net, S, params, &need);
    if (s) return s;
    if (bytes < need) return fail(ASD_ENOMEM, "workspace has %zu bytes, needs %zu", bytes, need);
    if ((uintptr_t)workspace % 256) return fail(ASD_EINVAL, "workspace must be 256-byte aligned");
    asd_plan* P = new (std::nothrow) asd_plan();  // value-initialised
    if (!P) return fail(ASD_EINVAL, "host allocation failed");
    P->net = net;
    P->S = S;
    P->n = net->n;
    P->prm = *params;
    P->prof = false;
    P->prof_used = 0;
    setup_plan_geometry(P);
    Carver cv{reinterpret_cast<char*>(workspace), 0};
    carve(P, cv);
    *out = P;
    return ASD_OK;
}

void asd_plan_destroy(asd_plan* plan) {
    if (!plan) return;
    for (hipEvent_t e : plan->prof_pool) (void)hipEventDestroy(e);
    delete plan;
}

asd_status asd_profile_enable(asd_plan* P, int32_t enable) {
    if (!P) return fail(ASD_EINVAL, "NULL plan");
    P->prof = enable != 0;
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
    if (b->S != P->S) return fail(ASD_EINVAL, "batch has S = %d, plan has %d", b->S, P->S);
    if (!b->l0 || !b->u0 || !b->c) return fail(ASD_EINVAL, "NULL l0/u0/c");
    if (P->n > 1 && (!b->lhat || !b->uhat)) return fail(ASD_EINVAL, "NULL lhat/uhat");
    for (int k = 1; k < P->n; ++k)
        if (!b->lhat[k - 1] || !b->uhat[k - 1]) return fail(ASD_EINVAL, "NULL bound of layer %d", k);
    asd_status s;
    const int S = P->S;
    if ((s = launch_layout(P->na[0].lo, b->l0, P->nl[0], S, 0, st))) return s;
    if ((s = launch_layout(P->na[0].hi, b->u0, P->nl[0], S, 0, st))) return s;
    for (int k = 1; k < P->n; ++k) {
        ReluLayer& r = P->R[k];
        if ((s = launch_layout(r.lhat, b->lhat[k - 1], P->nl[k], S, 0, st))) return s;
        if ((s = launch_layout(r.uhat, b->uhat[k - 1], P->nl[k], S, 0, st))) return s;
        if ((s = launch_layout(P->na[k].lo, b->lhat[k - 1], P->nl[k], S, 1, st))) return s;
        if ((s = launch_layout(P->na[k].hi, b->uhat[k - 1], P->nl[k], S, 1, st))) return s;
    }
    for (int k = 0; k < P->n; ++k)
        if ((s = launch_bits(P->nl[k], S, 3, P->na[k].deg, nullptr, P->na[k].lo, P->na[k].hi, st))) return s;
    if ((s = launch_layout(P->cvec, b->c, P->nl[P->n], S, 0, st))) return s;
    for (int k = 1; k < P->n; ++k) {
        const size_t ns = (size_t)P->nl[k].N * S;
        ReluLayer& r = P->R[k];
        float* arrs[12] = {r.alpha, r.beta0, r.beta1, r.alpha_m, r.alpha_v, r.beta0_m,
                           r.beta0_v, r.beta1_m, r.beta1_v, r.own, r.g, r.vdn};
        for (float* a : arrs)
            if ((s = zero_floats(a, ns, st))) return s;
        for (int q = 0; q < P->prm.max_masks; ++q) {
            MaskSlot& m = r.slot[q];
            float* sarr[6] = {m.beta, m.m, m.v, m.LI, m.UI, m.u};
            for (float* a : sarr)
                if ((s = zero_floats(a, ns, st))) return s;
            if ((s = zero_words(m.zbits, P->nl[k].words, st))) return s;
            if ((s = zero_words(m.xbits, P->nl[k - 1].words, st))) return s;
        }
    }
    P->n_masks = 0;
    P->step = 0;
    for (int q = 0; q < kMaxMasks; ++q) P->mask_step[q] = 0;
    P->loaded = true;
    return ASD_OK;
}

asd_status asd_run(asd_plan* P, int32_t phase, int32_t t_begin, int32_t n_iters, hipStream_t st) {
    if (!P) return fail(ASD_EINVAL, "NULL plan");
    if (!P->loaded) return fail(ASD_EINVAL, "asd_init has not been called");
    if (phase != ASD_PHASE_BIGM && phase != ASD_PHASE_AS) return fail(ASD_EINVAL, "unknown phase");
    const int T = phase == ASD_PHASE_BIGM ? P->prm.bigm_iters : P->prm.as_iters;
    if (t_begin < 0 || n_iters < 0 || t_begin + n_iters > T)
        return fail(ASD_EINVAL, "iterations [%d, %d) outside [0, %d)", t_begin, t_begin + n_iters, T);
    asd_status s;
    const bool as = phase == ASD_PHASE_AS;
    if (as && t_begin == 0 && n_iters > 0 && P->prm.rule == ASD_RULE_ADAM)
        if ((s = reset_group_moments(P, st))) return s;
    for (int t = t_begin; t < t_begin + n_iters; ++t) {
        const float lr = as ? linear_lr(P->prm.as_lr0, P->prm.as_lr1, t, T)
                            : linear_lr(P->prm.bigm_lr0, P->prm.bigm_lr1, t, T);
        if ((s = iteration(P, as, t, lr, st))) return s;
    }
    return ASD_OK;
}

asd_status asd_bound(asd_plan* P, double* out_lb, float* x0, hipStream_t st) {
    if (!P || !out_lb) return fail(ASD_EINVAL, "NULL argument");
    if (!P->loaded) return fail(ASD_EINVAL, "asd_init has not been called");
    asd_status s;
    for (int k = 1; k < P->n; ++k)
        if ((s = launch_final_sums(P, k, st))) return s;
    for (int k = P->n - 1; k >= 0; --k)
        if ((s = launch_backward<double>(P, k, 1, st))) return s;
    if ((s = reduce_objective(P, out_lb, st))) return s;
    if (x0 && (s = launch_layout(x0, P->na[0].xstar, P->nl[0], P->S, 2, st))) return s;
    return ASD_OK;
}

asd_status asd_solve(asd_plan* P, const asd_batch* b, double* out_lb, float* x0, hipStream_t st) {
    asd_status s;
    if ((s = asd_init(P, b, st))) return s;
    if ((s = asd_run(P, ASD_PHASE_BIGM, 0, P->prm.bigm_iters, st))) return s;
    if ((s = asd_run(P, ASD_PHASE_AS, 0, P->prm.as_iters, st))) return s;
    return asd_bound(P, out_lb, x0, st);
}

static float* field_ptr(asd_plan* P, int field, int k, int q) {
    ReluLayer& r = P->R[k];
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

static asd_status check_field(asd_plan* P, int field, int k, int q) {
    if (!P) return fail(ASD_EINVAL, "NULL plan");
    if (!P->loaded) return fail(ASD_EINVAL, "asd_init has not been called");
    if (k < 1 || k >= P->n) return fail(ASD_EINVAL, "layer %d outside [1, %d]", k, P->n - 1);
    if (field < ASD_F_ALPHA || field > ASD_F_MASK_XPREV) return fail(ASD_EINVAL, "unknown field %d", field);
    if (field >= ASD_F_MASK_BETA && (q < 0 || q >= P->prm.max_masks))
        return fail(ASD_EINVAL, "slot %d outside [0, %d)", q, P->prm.max_masks);
    return ASD_OK;
}

asd_status asd_state_get(asd_plan* P, int32_t field, int32_t k, int32_t q, float* dst, hipStream_t st) {
    asd_status s = check_field(P, field, k, q);
    if (s) return s;
    if (!dst) return fail(ASD_EINVAL, "NULL destination");
    if (field == ASD_F_MASK_Z)
        return launch_bits(P->nl[k], P->S, 0, P->R[k].slot[q].zbits, dst, nullptr, nullptr, st);
    if (field == ASD_F_MASK_XPREV)
        return launch_bits(P->nl[k - 1], P->S, 4, P->R[k].slot[q].xbits, dst, P->na[k - 1].lo,
                           P->na[k - 1].hi, st);
    return launch_layout(dst, field_ptr(P, field, k, q), P->nl[k], P->S, 2, st);
}

asd_status asd_state_set(asd_plan* P, int32_t field, int32_t k, int32_t q, const float* src, hipStream_t st) {
    asd_status s = check_field(P, field, k, q);
    if (s) return s;
    if (!src) return fail(ASD_EINVAL, "NULL source");
    if (field == ASD_F_MASK_Z) {
        s = launch_bits(P->nl[k], P->S, 2, P->R[k].slot[q].zbits, const_cast<float*>(src), nullptr, nullptr, st);
    } else if (field == ASD_F_MASK_XPREV) {
        s = launch_bits(P->nl[k - 1], P->S, 1, P->R[k].slot[q].xbits, const_cast<float*>(src),
                        P->na[k - 1].lo, P->na[k - 1].hi, st);
    } else {
        s = launch_layout(field_ptr(P, field, k, q), src, P->nl[k], P->S, 0, st);
    }
    if (s) return s;
    return derive_layer(P, k, st);
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
    if (!P->loaded) return fail(ASD_EINVAL, "asd_init has not been called");
    if (in->n_masks < 0 || in->n_masks > P->prm.max_masks)
        return fail(ASD_EINVAL, "n_masks %d outside [0, %d]", in->n_masks, P->prm.max_masks);
    if (in->step < 0) return fail(ASD_EINVAL, "negative step");
    for (int q = 0; q < in->n_masks; ++q)
        if (in->mask_step[q] < 0) return fail(ASD_EINVAL, "negative mask step");
    P->n_masks = in->n_masks;
    P->step = in->step;
    for (int q = 0; q < kMaxMasks; ++q) P->mask_step[q] = q < in->n_masks ? in->mask_step[q] : 0;
    asd_status s;
    if (recompute) {
        for (int k = 1; k < P->n; ++k)
            for (int q = 0; q < P->n_masks; ++q)
                if ((s = launch_mask_consts(P, k, q, P->R[k].slot[q].zbits, P->R[k].slot[q].xbits, 0, st)))
                    return s;
    }
    for (int k = 1; k < P->n; ++k)
        if ((s = derive_layer(P, k, st))) return s;
    return ASD_OK;
}

asd_status asd_eval(asd_plan* P, const asd_eval_out* out, hipStream_t st) {
    if (!P || !out) return fail(ASD_EINVAL, "NULL argument");
    if (!P->loaded) return fail(ASD_EINVAL, "asd_init has not been called");
    asd_status s;
    for (int k = P->n - 1; k >= 0; --k)
        if ((s = launch_backward<float>(P, k, 1, st))) return s;
    if (out->obj && (s = reduce_objective(P, out->obj, st))) return s;
    for (int k = 0; k < P->n; ++k) {
        if (out->xstar[k] && (s = launch_layout(out->xstar[k], P->na[k].xstar, P->nl[k], P->S, 2, st))) return s;
        if (k >= 1 && out->zstar[k] &&
            (s = launch_bits(P->nl[k], P->S, 0, P->R[k].zbits, out->zstar[k], nullptr, nullptr, st)))
            return s;
    }
    const StepArgs sa = make_step_args(P, 0.f);
    for (int k = 1; k < P->n; ++k) {
        float* gout[3 + kMaxMasks] = {out->grad_alpha[k], out->grad_beta0[k], out->grad_beta1[k]};
        bool any = gout[0] || gout[1] || gout[2];
        for (int q = 0; q < kMaxMasks; ++q) {
            gout[3 + q] = out->grad_mask[k][q];
            any = any || gout[3 + q];
        }
        if (any && (s = launch_forward(P, k, sa, 1, gout, st))) return s;
    }
    return ASD_OK;
}

asd_status asd_oracle(asd_plan* P, int32_t k, const float* x_prev, const float* z, uint32_t* mask_bits,
                      float* LI, float* UI, hipStream_t st) {
    if (!P || !x_prev || !z || !mask_bits || !LI || !UI) return fail(ASD_EINVAL, "NULL argument");
    if (!P->loaded) return fail(ASD_EINVAL, "asd_init has not been called");
    if (k < 1 || k >= P->n) return fail(ASD_EINVAL, "layer %d outside [1, %d]", k, P->n - 1);
    OracleArgs a;
    a.g = P->geo[k];
    a.S = P->S;
    a.xprev = x_prev;
    a.z = z;
    a.lo_in = P->na[k - 1].lo;
    a.hi_in = P->na[k - 1].hi;
    a.bits = mask_bits;
    a.LI = LI;
    a.UI = UI;
    const long n = (long)P->S * a.g.out.N;
    hipLaunchKernelGGL(k_oracle, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, a);
    LAUNCH_CHECK();
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
