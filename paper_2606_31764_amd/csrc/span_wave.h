// Knot-span search for a wavefront whose 64 lanes all evaluate one curve
// (sample emission and the sample adjoints): a 64-ary search over the knot
// vector, each lane reading one knot per round, finds the spans of the
// wavefront's lowest and highest parameter in two rounds for up to 4096
// knots, where a per-lane binary search is a chain of about a dozen
// dependent loads.  Included after nsplat_internal.h (find_span).
#pragma once

namespace nsp {

// find_span for a wavefront-uniform x (the largest i in [p, m-p-1] with
// U[i] <= x, the right-end and left-end rules as find_span's).
__device__ inline int span_uniform(const double* U, int p, int m, double x) {
  const int lo = p, hi = m - p - 1;
  if (x >= U[hi + 1] || !(U[lo] <= x)) return find_span(U, p, m, x);
  const int lane = __lane_id();
  int a = lo, n = hi - lo + 1;  // U[a] <= x; the answer lies in [a, a + n)
  while (n > 1) {
    const int step = (n + 63) >> 6;
    const int idx = a + lane * step;
    const bool ok = idx < a + n && U[idx] <= x;  // a prefix of the lanes (U ascending), lane 0 always
    const int k = 63 - __builtin_clzll(__ballot(ok));
    const int end = a + n;
    a += k * step;
    n = min(step, end - a);
  }
  return a;
}

// find_span(U, p, m, u) of every lane, all 64 lanes active and on one curve:
// the spans of the wavefront's lowest and highest u bound every lane's
// (find_span is monotone in u), and each lane takes the largest span start
// at or below its u in that window (the lowest span when none is).
__device__ inline int span_wave(const double* U, int p, int m, double u) {
  double umin = u, umax = u;
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    umin = fmin(umin, __shfl_xor(umin, off));
    umax = fmax(umax, __shfl_xor(umax, off));
  }
  int a = __builtin_amdgcn_readfirstlane(span_uniform(U, p, m, umin));
  int b = __builtin_amdgcn_readfirstlane(span_uniform(U, p, m, umax));
  while (a < b) {
    const int mid = (a + b + 1) >> 1;
    if (U[mid] <= u) a = mid;
    else b = mid - 1;
  }
  return a;
}

}  // namespace nsp
