// Internal definitions shared by the kernels and the host side of libasdual.
//
// Data layout.  Every per-neuron array of a layer with C channels and P
// positions per channel (dense layers: C = neurons, P = 1) is stored
// channel-major over the batch: element (c, s, p) lives at (c * S + s) * P + p.
// A wavefront covers 64 consecutive "columns" col = s * P + p of one channel,
// so per-neuron state is read and written in contiguous 256-byte runs while
// the weights a thread needs are uniform across the wavefront.
//
// Bit arrays (primal choices, compact masks, point boxes) use bit index
// c * colpad + col with colpad = S * P rounded up to a multiple of 64, so one
// wavefront's 64 bits are two whole 32-bit words written by a ballot.
//
// Precision.  A plan keeps its duals, moments, bounds and every intermediate
// in T = float (the production form) or T = double (used to check whole runs
// against the FP64 reference); network weights and caller inputs are FP32.
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

// Arrays of one active-set slot of a ReLU layer.
template <typename T>
struct MaskSlotT {
    T* beta;   // beta_{k,I} >= 0
    T* m;      // Adam moments
    T* v;
    T* LI;     // (W . I . Lcheck) row sums
    T* UI;     // (W . (1 - I) . Ucheck) row sums
    T* u;      // derived: (1 - z_I) * beta_{k,I} (operand of the |W|^T product of the slot)
    uint32_t* zbits;  // z*_k at addition (layout of layer k)
    uint32_t* xbits;  // x*_{k-1} == upper end at addition (layout of layer k-1)
};

// Arrays of one ReLU layer.
template <typename T>
struct ReluLayerT {
    T* lhat; T* uhat;             // pre-activation bounds
    T* alpha; T* beta0; T* beta1;
    T* alpha_m; T* alpha_v;       // Adam moments (mixed mode: both as BF16 in one word of the m array)
    T* beta0_m; T* beta0_v;
    T* beta1_m; T* beta1_v;
    T* own;   // derived: alpha - beta0 - beta1 - sum_I beta_I
    T* g;     // derived: g_k (eq:dual-anderson-functions)
    T* vs;    // derived: -alpha + beta1 + sum_I (1 + z_I) beta_I / 2 (operand of the W^T product)
    uint32_t* zbits;  // z*_k at the current iterate
    uint8_t* zpk;     // per neuron: bit q = z bit of slot q
    MaskSlotT<T> slot[kMaxMasks];
    // FP64 sums for the final bound of an FP32 plan
    double* own64; double* g64; double* const64;
};

template <typename T>
struct NeuronArraysT {
    T* lo; T* hi;              // post-activation box (k = 0: input box)
    T* xstar;                  // current minimiser x*_k
    uint32_t* xbits;           // x*_k == hi
    uint32_t* deg;             // lo == hi
    double* term;              // objective terms per neuron
    // per neuron, for the masks of the next ReLU layer: bit q (q < 8) = x-bit
    // of slot q OR point box; bit 15 = point box away from zero
    uint16_t* xpk;
};

// Adam / step arguments of one iteration.
template <typename T>
struct StepArgsT {
    int rule;          // asd_rule
    T lr;
    T b1, b2, eps;
    T bc1[1 + kMaxMasks];   // 1 - b1^step for the alpha/beta group and each slot
    T bc2[1 + kMaxMasks];
    T c1[1 + kMaxMasks];    // lr / (1 - b1^step)  (rounded once, on the host)
    T ib2[1 + kMaxMasks];   // 1 / (1 - b2^step)
    // per-subproblem learning rates (subproblems with their own iteration
    // budget, each on its own schedule), or null: then lr / c1 apply to all
    const T* lrs;
    T ib1[1 + kMaxMasks];   // 1 / (1 - b1^step), with lrs
};

}  // namespace asd
