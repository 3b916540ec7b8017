// Tap tables shared by the weight packer and the convolution launcher.
#pragma once

#include <hip/hip_runtime.h>

namespace rte {

// 3-tap-per-axis cross-correlation with padding 1: tap t (x fastest) reads
// input offset (kx - 1, ky - 1, kz - 1) relative to stride * output index.
__host__ __device__ inline void conv3_tap(int dim, int t, int k[3], int off[3]) {
  k[0] = t % 3;
  k[1] = (t / 3) % 3;
  k[2] = dim == 3 ? t / 9 : 0;
  for (int a = 0; a < 3; ++a) off[a] = (a < dim) ? k[a] - 1 : 0;
}

// Transposed convolution, kernel 4, stride 2, padding 1.  Fine index o and
// coarse index i are linked by o = 2 i - 1 + k.  For output parity p
// (o = 2 I + p) exactly two taps contribute per axis:
//   p = 0: k = 1 (i = I), k = 3 (i = I - 1);   p = 1: k = 0 (i = I + 1), k = 2 (i = I).
// Class index cls = px + 2 py + 4 pz; tap index t = tx + 2 ty + 4 tz selects
// one of the two taps per axis.
__host__ __device__ inline void convT4_tap(int dim, int cls, int t, int k[3], int off[3]) {
  for (int a = 0; a < 3; ++a) {
    if (a >= dim) {
      k[a] = 0;
      off[a] = 0;
      continue;
    }
    int p = (cls >> a) & 1;
    int ta = (t >> a) & 1;
    k[a] = (p == 0) ? (ta == 0 ? 1 : 3) : (ta == 0 ? 0 : 2);
    off[a] = (p + 1 - k[a]) / 2;
  }
}

}  // namespace rte
