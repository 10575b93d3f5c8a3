// Shapes and flat parameter layout of the lambda_0 set encoder, shared by the
// kernels and the host entry points.
#pragma once

namespace pbit {

constexpr int kNetF = 16;    // input features per element (five used)
constexpr int kNetCtx = 16;  // context values per set as stored (nine used)
constexpr int kNetH = 128;   // hidden width
constexpr int kNetZ = 144;   // head input: pooled (128) + context (16)

// parameter offsets (elements): W1[128][16] b1 W2[128][128] b2 W3[128][144] b3 w4[128] b4
constexpr int kOffW1 = 0;
constexpr int kOffB1 = kOffW1 + kNetH * kNetF;
constexpr int kOffW2 = kOffB1 + kNetH;
constexpr int kOffB2 = kOffW2 + kNetH * kNetH;
constexpr int kOffW3 = kOffB2 + kNetH;
constexpr int kOffB3 = kOffW3 + kNetH * kNetZ;
constexpr int kOffW4 = kOffB3 + kNetH;
constexpr int kOffB4 = kOffW4 + kNetH;
constexpr int kNetParams = kOffB4 + 1;
constexpr int kNetPhiParams = kOffW3;  // W1, b1, W2, b2

static_assert(kOffW2 % 8 == 0 && kOffW3 % 8 == 0, "16-byte aligned weight blocks");
static_assert(kNetH * kNetZ % 256 == 0, "head gradient split over 256 threads");

}  // namespace pbit
