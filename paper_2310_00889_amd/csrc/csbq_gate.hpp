// csbq_gate.hpp -- learned correction-tier gate: shapes and launchers.
//
// The gate maps a feature vector of a (target, element) pair to the
// correction tier (skip, the three upsampled whole-panel rules, the special
// quadrature).  The network is a three-hidden-layer perceptron with GATE_H
// ReLU units per layer and GATE_NO ordinal outputs: output k estimates
// P(tier > k) through a logistic function, so the predicted tier is the
// number of leading outputs above one half and the probability that the
// truth lies above the prediction is read off the next output.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "csbq_common.hpp"

namespace csbq {

constexpr int GATE_NF = 16;    // features (12 used, zero padded to one MFMA k-block)
constexpr int GATE_NU = 12;    // features in use
constexpr int GATE_H = 64;     // hidden units per layer
constexpr int GATE_NO = 4;     // ordinal outputs: P(tier > k), k = 0..3

// parameter layout (FP32): W1[NF][H] b1[H] W2[H][H] b2[H] W3[H][H] b3[H] W4[H][NO] b4[NO]
constexpr int GW1 = 0;
constexpr int GB1 = GW1 + GATE_NF * GATE_H;
constexpr int GW2 = GB1 + GATE_H;
constexpr int GB2 = GW2 + GATE_H * GATE_H;
constexpr int GW3 = GB2 + GATE_H;
constexpr int GB3 = GW3 + GATE_H * GATE_H;
constexpr int GW4 = GB3 + GATE_H;
constexpr int GB4 = GW4 + GATE_H * GATE_NO;
constexpr int GATE_NW = GB4 + GATE_NO;

// inference weights: bf16 MFMA fragments (see k_gate_mlp) and FP32 biases
constexpr int GATE_FRAG_W1 = 1 * 4;      // k-blocks x n-blocks of 16x16
constexpr int GATE_FRAG_W2 = 4 * 4;
constexpr int GATE_FRAG_W4 = 4 * 1;
constexpr int GATE_NFRAG = GATE_FRAG_W1 + 2 * GATE_FRAG_W2 + GATE_FRAG_W4;   // 40 fragments
constexpr int GATE_FRAG_ELEMS = 64 * 4;  // bf16 per fragment (4 per lane)
constexpr int GATE_NBIAS = 3 * GATE_H + 16;

// order (if not null): the pairs in the order the threads take them (the
// element-major order, so a wavefront's lanes share the element's circles);
// feat is indexed by pair either way
int launch_gate_features(hipStream_t st, int64_t P, const int* order, const int* pe, const int* pt, const double* xt,
                         int64_t T, const int64_t* tnode, const double* circ, const ElemInfo* info, const int* band,
                         float ltol, float* feat);
int launch_gate_mlp(hipStream_t st, int64_t P, const float* feat, const uint16_t* wfrag, const float* bias,
                    float tau_esc, int8_t* tier, uint8_t* esc, float* logits);
int launch_gate_train_step(hipStream_t st, int nblk, int spb, int64_t off, int64_t n, const int64_t* perm,
                           const float* feat, const int8_t* label, const float* W, const float* posw, float* partial);
int launch_gate_reduce(hipStream_t st, int nblk, const float* partial, float scale, float* grad);
int launch_gate_adam(hipStream_t st, float* W, const float* grad, float* m, float* v, float lr, float b1, float b2,
                     float eps, int step);
int launch_gate_labels(hipStream_t st, int64_t P, const double* c_up1, const double* c_up2, const double* c_up3,
                       const double* c_full, double thr_s, double thr_d, int8_t* label);
// predicted tier of every confident pair (a predicted tier 1 on an element
// closed at its ends, whose far-field rule is tier 1's rule, becomes tier 2);
// flag[i] = 1 for the pairs left to the criterion
int launch_gate_select(hipStream_t st, int64_t P, const int* perm, const int* pe, const ElemInfo* info,
                       const uint8_t* esc, const int8_t* tier_mlp, int8_t* tier, uint8_t* flag);

}  // namespace csbq
