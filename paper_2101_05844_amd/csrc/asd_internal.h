// Internal definitions shared by the kernels and the host side of libasdual.
//
// Data layout.  Every per-neuron array of a layer with C channels and P
// positions per channel (dense layers: C = neurons, P = 1) is stored
// channel-major over the batch: element (c, s, p) lives at (c * S + s) * P + p.
// A wavefront covers 64 consecutive "columns" col = s * P + p of one channel,
// so per-neuron state is read and written in contiguous 256-byte runs while
// the weights a thread needs are uniform across the wavefront.
//
// Bit arrays (primal choices, compact masks, degenerate boxes) use bit index
// c * colpad + col with colpad = S * P rounded up to a multiple of 64, so one
// wavefront's 64 bits are two whole 32-bit words written by a ballot.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/asdual.h"

namespace asd {

constexpr int kWave = 64;
constexpr int kMaxMasks = ASD_MAX_MASKS;
constexpr int kMaxLayers = ASD_MAX_LAYERS;

// Shape of the neurons of one layer output (k = 0 is the network input).
struct NeuronLayout {
    int C, H, W;   // channels and spatial size (dense: C = n, H = W = 1)
    int P;         // H * W
    long N;        // C * P neurons per subproblem
    long cols;     // S * P columns per channel
    long colpad;   // cols rounded up to a multiple of 64
    long words;    // 32-bit words of one bit array: C * colpad / 32
};

// Geometry of layer L (1-based) mapping neuron layout L-1 to neuron layout L.
struct LayerGeo {
    int kind;      // ASD_LAYER_DENSE or ASD_LAYER_CONV2D
    int ksz, stride, pad;
    int fan;       // fan-in per output neuron (dense: n_in; conv: c_in * k * k)
    NeuronLayout in, out;
    const float* W;
    const float* b;
};

__host__ __device__ inline long nidx(const NeuronLayout& nl, int S, int c, int s, int p) {
    return ((long)c * S + s) * nl.P + p;
}
__host__ __device__ inline long bidx(const NeuronLayout& nl, int c, long col) {
    return (long)c * nl.colpad + col;
}

// Per-ReLU-layer device arrays inside the workspace.
struct MaskSlot {
    float* beta;   // beta_{k,I} >= 0
    float* m;      // Adam moments
    float* v;
    float* LI;     // (W . I . Lcheck) row sums
    float* UI;     // (W . (1 - I) . Ucheck) row sums
    float* u;      // derived: (1 - z_I) * beta_{k,I}
    uint32_t* zbits;  // z*_k at addition (layout of layer k)
    uint32_t* xbits;  // x*_{k-1} == upper end at addition (layout of layer k-1)
};

struct ReluLayer {
    float* lhat; float* uhat;             // pre-activation bounds
    float* alpha; float* beta0; float* beta1;
    float* alpha_m; float* alpha_v;
    float* beta0_m; float* beta0_v;
    float* beta1_m; float* beta1_v;
    float* own;   // derived: alpha - beta0 - beta1 - sum_I beta_I
    float* g;     // derived: g_k (eq:dual-anderson-functions)
    float* vdn;   // derived: -alpha + beta1 + sum_I z_I beta_I (dense backward operand)
    uint32_t* zbits;  // z*_k at the current iterate
    MaskSlot slot[kMaxMasks];
    // FP64 final evaluation scratch
    double* own64; double* g64; double* const64;
};

struct NeuronArrays {
    float* lo; float* hi;      // post-activation box (k = 0: input box)
    float* xstar;              // current minimiser x*_k
    uint32_t* xbits;           // x*_k == hi
    uint32_t* deg;             // lo == hi
    double* term;              // objective terms per neuron
};

// Adam / step arguments of one iteration.
struct StepArgs {
    int rule;          // asd_rule
    float lr;
    float b1, b2, eps;
    float bc1[1 + kMaxMasks];   // 1 - b1^step for the alpha/beta group and each slot
    float bc2[1 + kMaxMasks];
};

}  // namespace asd
