// Tile shapes and coarse-kernel sizes: compile-time tables shared by the kernels (which are
// instantiated for them) and the host planner (which tiles level blocks with them).
#pragma once

#include "internal.h"

namespace es {

struct Shape3 {
  int a, b, c;
};
constexpr Shape3 shape_of(int K, int D, int V, int L) {
  // V: 0 wide, 1 narrow, 2 medium
  if (K == K_LP_UP2) return V == 0 ? Shape3{1, 64, 128} : (V == 1 ? Shape3{1, 32, 64} : Shape3{1, 32, 128});
  if (K == K_LP_DOWN_S && D == 3) return V == 0 ? Shape3{16, 8, 32} : (V == 1 ? Shape3{8, 8, 16} : Shape3{8, 8, 32});
  if (K == K_LP_DOWN_S) return V == 0 ? Shape3{1, 64, 64} : (V == 1 ? Shape3{1, 16, 64} : Shape3{1, 32, 64});
  if (K == K_LP_UP_S) return V == 0 ? Shape3{16, 16, 32} : (V == 1 ? Shape3{8, 8, 32} : Shape3{8, 16, 32});
  if (K == K_FB_DOWN_S) return V == 0 ? Shape3{16, 8, 32} : (V == 1 ? Shape3{8, 8, 16} : Shape3{8, 8, 32});
  if (K == K_FB_UP_S) return V == 0 ? Shape3{16, 16, 32} : (V == 1 ? Shape3{8, 8, 32} : Shape3{8, 16, 32});
  if (D == 1) {
    const bool an = (K == K_LP_DOWN || K == K_FB_DOWN);
    return an ? (V == 0 ? Shape3{1, 1, 256} : (V == 1 ? Shape3{1, 1, 64} : Shape3{1, 1, 128}))
              : (V == 0 ? Shape3{1, 1, 512} : (V == 1 ? Shape3{1, 1, 128} : Shape3{1, 1, 256}));
  }
  if (D == 2) {
    switch (K) {
      case K_LP_DOWN: return V == 0 ? Shape3{1, 32, 64} : (V == 1 ? Shape3{1, 8, 16} : Shape3{1, 16, 64});
      case K_LP_UP: return V == 0 ? Shape3{1, 64, 128} : (V == 1 ? Shape3{1, 16, 32} : Shape3{1, 32, 128});
      case K_FB_DOWN: return V == 0 ? Shape3{1, 16, 32} : (V == 1 ? Shape3{1, 8, 16} : Shape3{1, 16, 64});
      default: return V == 0 ? Shape3{1, 32, 64} : (V == 1 ? Shape3{1, 16, 32} : Shape3{1, 32, 128});
    }
  }
  switch (K) {
    case K_LP_DOWN:
      return V == 0 ? (L <= 8 ? Shape3{4, 8, 16} : Shape3{2, 4, 16})
                    : (V == 1 ? Shape3{2, 4, 8} : (L <= 8 ? Shape3{2, 8, 16} : Shape3{2, 4, 8}));
    case K_LP_UP: return V == 0 ? Shape3{4, 16, 32} : (V == 1 ? Shape3{4, 8, 16} : Shape3{4, 8, 32});
    case K_FB_DOWN:
      return V == 0 ? (L <= 8 ? Shape3{2, 8, 16} : Shape3{2, 4, 8}) : (V == 1 ? Shape3{2, 4, 8} : Shape3{2, 4, 16});
    default:
      return V == 0 ? (L <= 8 ? Shape3{4, 16, 16} : Shape3{4, 8, 16})
                    : (V == 1 ? Shape3{4, 8, 16} : (L <= 8 ? Shape3{4, 8, 32} : Shape3{4, 8, 16}));
  }
}
constexpr int kThreads = 256;       // threads of every level-kernel work-group

// Output rows per chunk of the streamed 2-D low-pass analysis kernel (measured on 64 x 1024^2 and
// 64 x 512^2 db8 levels against 4 and 16, with strips of 64, 128 and 256 columns).
constexpr int kStreamRows = 8;
constexpr int kCoarseThreads = 1024;    // low-pass coarse kernel
constexpr int kFbCoarseThreads = 1024;  // full-bank coarse kernels

// LDS of a block of at most CMAX floats: the pyramid (< 2B in 1-D, < 4B/3 in 2-D, < 8B/7 in 3-D)
// plus the temporaries (1-D: none; 2-D: B/2; 3-D: B/2 + B/2, the second synthesis pass writes a
// half block) stay below 9B/4.
constexpr int coarse_lds_floats(int cmax) { return cmax / 4 * 9; }

inline TileShape tile_shape(int kind, int ndim, int variant, int taps) {
  const Shape3 sh = shape_of(kind, ndim, variant, taps);
  TileShape t;
  t.t[0] = sh.a;
  t.t[1] = sh.b;
  t.t[2] = sh.c;
  return t;
}
inline int tile_threads(int, int, int) { return kThreads; }
inline int tail_threads() { return kFbCoarseThreads; }

// LDS the low-pass coarse kernel needs for a block (static arrays in two sizes, chosen at launch
// from this value); the full-bank coarse kernels use one fixed size.
inline size_t tail_lds_bytes(int kind, int, const int b[3], int) {
  if (kind != 3) return 0;
  return sizeof(float) * (size_t)coarse_lds_floats(b[0] * b[1] * b[2]);
}

}  // namespace es
