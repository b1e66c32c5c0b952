// Learned slice planner: feature and network sizes, device helpers.
#pragma once
#include "fb_internal.h"

namespace fb {

constexpr int kPlanK = 16;         // Chebyshev moments mu_1 .. mu_16
constexpr int kPlanP = 20;         // Rademacher probes
constexpr int kPlanFeatures = 80;  // network input
constexpr int kPlanOutputs = 64;   // normalised counts n_-(s_k)/n
constexpr int kH0 = 80, kH1 = 256, kH2 = 256, kH3 = 64;
constexpr int kNetParams = kH0 * kH1 + kH1 + kH1 * kH2 + kH2 + kH2 * kH3 + kH3;

// features of an ingested band (host result, kPlanFeatures doubles)
int band_features_dev(const Band& bd, uint64_t seed, Arena& ar, double* feat, hipStream_t st);
// network forward for a batch (device arrays; H1, H2 scratch batch x 256)
int net_forward(const float* w, int batch, const float* X, float* Y, float* H1, float* H2,
                hipStream_t st);

}  // namespace fb
