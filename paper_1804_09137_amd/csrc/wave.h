// Wave64 reductions on gfx950 without LDS round trips.
//
// Lanes are exchanged by DPP within 16-lane rows (quad_perm, row_mirror,
// row_half_mirror: VALU operations) and by v_permlane16_swap /
// v_permlane32_swap across rows and half-waves.  A `ds_bpermute` shuffle goes
// through the LDS crossbar with tens of cycles of latency; chains of them
// dominated the per-step time of the small QR kernels.
//
// Pairings used: xor 1 and xor 2 (quad_perm), i <-> 7 - i within 8 lanes
// (row_half_mirror: flips bit 2, and bits 0-1), i <-> 15 - i within 16 lanes
// (row_mirror: flips bit 3, and bits 0-2), and the row / half-wave swaps
// (flip bit 4 / bit 5).  Together they generate every lane permutation a
// reduction needs; each step of a butterfly pairs lanes that differ in the
// bit that selects what they keep.
#pragma once
#include <hip/hip_runtime.h>

namespace tlrk {
namespace wave {

constexpr int kXor1 = 0xB1;        // quad_perm [1, 0, 3, 2]
constexpr int kXor2 = 0x4E;        // quad_perm [2, 3, 0, 1]
constexpr int kHalfMirror = 0x141; // i <-> 7 - i in each group of 8
constexpr int kMirror = 0x140;     // i <-> 15 - i in each row of 16

__device__ inline int lo32(double v) { return (int)(__double_as_longlong(v) & 0xffffffffll); }
__device__ inline int hi32(double v) { return (int)(__double_as_longlong(v) >> 32); }
__device__ inline double mk(int lo, int hi) {
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

template <int CTRL>
__device__ inline double dpp(double v) {
  return mk(__builtin_amdgcn_update_dpp(0, lo32(v), CTRL, 0xF, 0xF, false),
            __builtin_amdgcn_update_dpp(0, hi32(v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ inline int dpp(int v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, false);
}

// OFF = 32: x <- [x lanes 0-31, y lanes 0-31], y <- [x lanes 32-63, y lanes 32-63].
// OFF = 16: x <- rows [x0, y0, x2, y2],  y <- rows [x1, y1, x3, y3].
template <int OFF>
__device__ inline void swap(double& x, double& y) {
  static_assert(OFF == 16 || OFF == 32, "swap: OFF must be 16 or 32");
  if (OFF == 32) {
    const auto l = __builtin_amdgcn_permlane32_swap((unsigned)lo32(x), (unsigned)lo32(y), false, false);
    const auto h = __builtin_amdgcn_permlane32_swap((unsigned)hi32(x), (unsigned)hi32(y), false, false);
    x = mk((int)l[0], (int)h[0]);
    y = mk((int)l[1], (int)h[1]);
  } else {
    const auto l = __builtin_amdgcn_permlane16_swap((unsigned)lo32(x), (unsigned)lo32(y), false, false);
    const auto h = __builtin_amdgcn_permlane16_swap((unsigned)hi32(x), (unsigned)hi32(y), false, false);
    x = mk((int)l[0], (int)h[0]);
    y = mk((int)l[1], (int)h[1]);
  }
}
template <int OFF>
__device__ inline void swap(int& x, int& y) {
  if (OFF == 32) {
    const auto r = __builtin_amdgcn_permlane32_swap((unsigned)x, (unsigned)y, false, false);
    x = (int)r[0];
    y = (int)r[1];
  } else {
    const auto r = __builtin_amdgcn_permlane16_swap((unsigned)x, (unsigned)y, false, false);
    x = (int)r[0];
    y = (int)r[1];
  }
}

// The value held by the lane that differs in bit log2(OFF) (OFF = 16, 32).
template <int OFF, class T>
__device__ inline T partner(T v, int lane) {
  T a = v, b = v;
  swap<OFF>(a, b);
  return (lane & OFF) ? a : b;
}

// Sum over the 64 lanes, returned to every lane.
__device__ inline double sum(double v) {
  v += dpp<kXor1>(v);
  v += dpp<kXor2>(v);
  v += dpp<kHalfMirror>(v);
  v += dpp<kMirror>(v);
  double a = v, b = v;
  swap<16>(a, b);
  v = a + b;
  a = v;
  b = v;
  swap<32>(a, b);
  return a + b;
}

// One transposed-butterfly step on the first 2H entries: a lane whose
// selecting bit is set keeps entries [H, 2H), the others [0, H); each adds
// the partner's copy of what it keeps.
template <int H, int CTRL, int BIT>
__device__ inline void bstep_dpp(double* v, int lane) {
  const bool hi = (lane & BIT) != 0;
#pragma unroll
  for (int i = 0; i < H; ++i) {
    const double keep = hi ? v[i + H] : v[i];
    const double send = hi ? v[i] : v[i + H];
    v[i] = keep + dpp<CTRL>(send);
  }
}
template <int H, int OFF>
__device__ inline void bstep_swap(double* v) {
#pragma unroll
  for (int i = 0; i < H; ++i) {
    double x = v[i], y = v[i + H];
    swap<OFF>(x, y);
    v[i] = x + y;
  }
}

// Reduces N (16 or 32) per-lane partial sums over the wave; lane l ends with
// the total of entry (l >> (6 - log2 N)) & (N - 1).  Far fewer exchanges than
// N separate reductions.  v is used as scratch.
template <int N>
__device__ inline double bfly(double (&v)[N], int lane) {
  static_assert(N == 16 || N == 32, "bfly: N must be 16 or 32");
  bstep_swap<N / 2, 32>(v);
  bstep_swap<N / 4, 16>(v);
  bstep_dpp<N / 8, kMirror, 8>(v, lane);
  bstep_dpp<N / 16, kHalfMirror, 4>(v, lane);
  double r = v[0];
  if (N == 32) {
    bstep_dpp<1, kXor2, 2>(v, lane);   // N = 32: entries [0, 2) left after the bit-2 step
    r = v[0];
    r += dpp<kXor1>(r);
  } else {
    r += dpp<kXor2>(r);
    r += dpp<kXor1>(r);
  }
  return r;
}

// Maximum of v over the wave (ties: the smaller idx), with its idx, and the
// sum of s, returned to every lane.
__device__ inline void max_sum(double& v, int& idx, double& s, int lane) {
#define TLRK_MAXSTEP(OV, OI)                                            \
  do {                                                                  \
    const double ov = (OV);                                             \
    const int oi = (OI);                                                \
    if (ov > v || (ov == v && oi < idx)) { v = ov; idx = oi; }          \
  } while (0)
  TLRK_MAXSTEP(dpp<kXor1>(v), dpp<kXor1>(idx));
  s += dpp<kXor1>(s);
  TLRK_MAXSTEP(dpp<kXor2>(v), dpp<kXor2>(idx));
  s += dpp<kXor2>(s);
  TLRK_MAXSTEP(dpp<kHalfMirror>(v), dpp<kHalfMirror>(idx));
  s += dpp<kHalfMirror>(s);
  TLRK_MAXSTEP(dpp<kMirror>(v), dpp<kMirror>(idx));
  s += dpp<kMirror>(s);
  TLRK_MAXSTEP(partner<16>(v, lane), partner<16>(idx, lane));
  s += partner<16>(s, lane);
  TLRK_MAXSTEP(partner<32>(v, lane), partner<32>(idx, lane));
  s += partner<32>(s, lane);
#undef TLRK_MAXSTEP
}

// The value of lane l (uniform l), returned to every lane.
__device__ inline double read(double v, int l) {
  return mk(__builtin_amdgcn_readlane(lo32(v), l), __builtin_amdgcn_readlane(hi32(v), l));
}

}  // namespace wave
}  // namespace tlrk
