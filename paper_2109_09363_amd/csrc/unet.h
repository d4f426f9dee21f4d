// Shape of the paper's Unet (Sec. 3.1, Fig. 4) shared by its forward and
// backward passes: widths per scale, the concatenation buffers, and the
// FP32 activations a training forward keeps for the backward pass.
#pragma once
#include <stddef.h>

namespace hyp {

constexpr int kUnetLevels = 5;
constexpr int kUnetLayers = 4 * kUnetLevels - 1;  // 10 encoder, 8 decoder, 1 output
constexpr int kUnetW[kUnetLevels] = {16, 16, 64, 64, 64};

// Concatenation buffer of Unet scale l (0..3): (ny >> l) x (nx >> l) pixels of
// kUnetW[l] skip channels then kUnetW[l + 1] upsampled ones; element offsets.
inline size_t unet_cat_offset(int nx, int ny, int l) {
  size_t o = 0;
  for (int k = 0; k < l; ++k) o += (size_t)(nx >> k) * (ny >> k) * (kUnetW[k] + kUnetW[k + 1]);
  return o;
}

// Element offsets (FP32) of what a training forward keeps besides the
// concatenation buffers: per scale l the first encoder output c1[l], the
// bottom encoder output c2 of the last scale, the pooled maps pool[l] (the
// input of scale l + 1), the decoder outputs d1[l], d2[l]; and, for the
// backward pass, one gradient map per scale for the skip channels.
struct UnetSave {
  size_t c1[kUnetLevels], c2_bottom, pool[kUnetLevels - 1], d1[kUnetLevels - 1],
      d2[kUnetLevels - 1], skip_grad[kUnetLevels - 1];
  size_t total;
};

inline UnetSave unet_save_layout(int nx, int ny) {
  UnetSave S{};
  size_t o = 0;
  auto px = [&](int l) { return (size_t)(nx >> l) * (ny >> l); };
  for (int l = 0; l < kUnetLevels; ++l) { S.c1[l] = o; o += px(l) * kUnetW[l]; }
  S.c2_bottom = o;
  o += px(kUnetLevels - 1) * kUnetW[kUnetLevels - 1];
  for (int l = 0; l + 1 < kUnetLevels; ++l) { S.pool[l] = o; o += px(l + 1) * kUnetW[l]; }
  for (int l = 0; l + 1 < kUnetLevels; ++l) { S.d1[l] = o; o += px(l) * kUnetW[l]; }
  for (int l = 0; l + 1 < kUnetLevels; ++l) { S.d2[l] = o; o += px(l) * kUnetW[l]; }
  for (int l = 0; l + 1 < kUnetLevels; ++l) { S.skip_grad[l] = o; o += px(l) * kUnetW[l]; }
  S.total = o;
  return S;
}

}  // namespace hyp
