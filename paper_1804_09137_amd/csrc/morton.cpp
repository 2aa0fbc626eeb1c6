// Host helper: Morton (Z-order) ordering of 2-D locations.  The paper does not
// state a point ordering; the build orders points along the Z-curve so that
// tiles hold spatially compact clusters (which keeps off-diagonal ranks low).
#include "tlr.h"

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <numeric>
#include <vector>

namespace {

// floor(((c - lo) / w) * 65535) with each operation rounded separately
std::vector<uint32_t> quantise(int64_t n, const double* c) {
  double lo = c[0], hi = c[0];
  for (int64_t i = 1; i < n; ++i) {
    lo = std::min(lo, c[i]);
    hi = std::max(hi, c[i]);
  }
  std::vector<uint32_t> q((size_t)n, 0u);
  const double w = hi - lo;
  if (w == 0.0) return q;
  for (int64_t i = 0; i < n; ++i) {
    volatile double t = (c[i] - lo) / w;
    volatile double u = t * 65535.0;
    q[(size_t)i] = (uint32_t)std::floor(u);
  }
  return q;
}

uint32_t spread16(uint32_t v) {  // bit b -> bit 2b
  v &= 0xFFFFu;
  v = (v | (v << 8)) & 0x00FF00FFu;
  v = (v | (v << 4)) & 0x0F0F0F0Fu;
  v = (v | (v << 2)) & 0x33333333u;
  v = (v | (v << 1)) & 0x55555555u;
  return v;
}

}  // namespace

extern "C" tlr_status tlr_morton_order(int64_t n, const double* x, const double* y, int64_t* perm) {
  if (n < 0 || (n > 0 && (!x || !y || !perm))) return TLR_EINVAL;
  if (n == 0) return TLR_OK;
  for (int64_t i = 0; i < n; ++i)
    if (!std::isfinite(x[i]) || !std::isfinite(y[i])) return TLR_EINVAL;
  const std::vector<uint32_t> qx = quantise(n, x), qy = quantise(n, y);
  std::vector<uint32_t> key((size_t)n);
  for (int64_t i = 0; i < n; ++i) key[(size_t)i] = spread16(qx[(size_t)i]) | (spread16(qy[(size_t)i]) << 1);
  std::vector<int64_t> p((size_t)n);
  std::iota(p.begin(), p.end(), (int64_t)0);
  std::stable_sort(p.begin(), p.end(), [&](int64_t a, int64_t b) { return key[(size_t)a] < key[(size_t)b]; });
  std::copy(p.begin(), p.end(), perm);
  return TLR_OK;
}
