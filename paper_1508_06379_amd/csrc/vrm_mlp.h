// Warm-start network shapes, parameter layout and device state (internal).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cstring>

namespace vrm {

constexpr int kMlpSlots = 32;    // LP columns seen by the network
constexpr int kMlpIn = 128;      // 2 * 32 offsets, 32 masks, q - 2, padding
constexpr int kMlpHid = 128;
constexpr int kMlpOut = 64;      // 32 basis logits, 32 fractions
// FP32 parameter vector: W1[in][hid], b1, W2[hid][hid], b2, W3[hid][out], b3
constexpr int kOffW1 = 0;
constexpr int kOffB1 = kOffW1 + kMlpIn * kMlpHid;
constexpr int kOffW2 = kOffB1 + kMlpHid;
constexpr int kOffB2 = kOffW2 + kMlpHid * kMlpHid;
constexpr int kOffW3 = kOffB2 + kMlpHid;
constexpr int kOffB3 = kOffW3 + kMlpHid * kMlpOut;
constexpr int kMlpParams = kOffB3 + kMlpOut;

constexpr int kEpiAcc = 0, kEpiBias = 1, kEpiBiasGelu = 2, kEpiGeluBwd = 3;

struct MlpState {
    int max_rows;
    int loaded;
    int step;
    float* w;        // FP32 master parameters
    float* g;        // gradients
    float* am;       // AdamW moments
    float* av;
    uint16_t* wbf;   // BF16 copy of w
    uint16_t* wt;    // BF16 weights transposed to [n][k] (inference)
    float* z1;       // pre-activations (rows x hid)
    float* z2;
    uint16_t* h1;    // activations, BF16
    uint16_t* h2;
    float* y;        // outputs (rows x out)
    uint16_t* dy;
    float* dyf;
    float* dz;
    uint16_t* dzb;
    uint16_t* dzb2;
    double* loss;
};

}  // namespace vrm
