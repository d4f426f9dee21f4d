// Shape of the paper's cascaded MultiScale / SmallScale networks (Sec. 3.1,
// Fig. 3) shared by their training forward and backward passes: the layers
// of each branch and the FP32 activations a training forward keeps.
#pragma once
#include <stddef.h>

#include "../../include/hyproj.h"

namespace hyp {

struct PnLayer {
  int ks, cin, cout;
  bool relu;
};

constexpr int kPnBranches = 3;
constexpr int kPnMaxLayers = 7;

// Layers of branch b (0 = coarsest, n/4 a side); returns the layer count.
// Every branch opens with a 5x5 convolution, has 3x3 ones in between and
// ends with a 1x1 to one channel; ReLU after all but the last two.
inline int pn_branch(int arch, int b, PnLayer* out) {
  const int a = arch == HYP_ARCH_MULTISCALE ? 64 : 32;
  const int mid = 32;
  if (b == 0) {
    const PnLayer L[5] = {{5, 2, a, true}, {3, a, a, true}, {3, a, a, true}, {3, a, a, false},
                          {1, a, 1, false}};
    for (int i = 0; i < 5; ++i) out[i] = L[i];
    return 5;
  }
  const PnLayer L[7] = {{5, 3, a, true}, {3, a, a, true},  {3, a, mid, true}, {3, mid, a, true},
                        {3, a, a, true}, {3, a, a, false}, {1, a, 1, false}};
  for (int i = 0; i < 7; ++i) out[i] = L[i];
  return 7;
}

// Element offsets (FP32) of what a training forward keeps: per branch b its
// input (2 or 3 channels at (n >> (2 - b))^2 pixels) and the output of every
// layer but the 1x1 head.
struct PnSave {
  size_t in[kPnBranches], out[kPnBranches][kPnMaxLayers];
  size_t total;
};

inline PnSave pn_save_layout(int arch, int nx, int ny) {
  PnSave S{};
  size_t o = 0;
  for (int b = 0; b < kPnBranches; ++b) {
    const size_t px = (size_t)(nx >> (2 - b)) * (ny >> (2 - b));
    PnLayer L[kPnMaxLayers];
    const int nl = pn_branch(arch, b, L);
    S.in[b] = o;
    o += px * L[0].cin;
    for (int i = 0; i + 1 < nl; ++i) {
      S.out[b][i] = o;
      o += px * L[i].cout;
    }
  }
  S.total = o;
  return S;
}

}  // namespace hyp
