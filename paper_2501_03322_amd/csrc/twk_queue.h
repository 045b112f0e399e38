// twk_queue.h -- the arithmetic of the contour queue's dispersed order.
//
// The persistent contour kernel takes its queue in a dispersed order:
// queue position p runs group (p * g) mod N of the N groups of tasks (a
// limb-darkened epoch's annulus contours form one group), with g coprime
// to N and close to N / phi (golden ratio), so that any run of consecutive
// positions samples the whole queue evenly.  The learned placement gives
// the row of class rank r the dispersed rank r * ginv mod N (ginv = g^-1
// mod N), so that dispersed rank p holds class rank p * g mod N, and then
// merges the two classes (merged_place_*).
#ifndef TWK_QUEUE_H
#define TWK_QUEUE_H

#include <hip/hip_runtime.h>

#include <cstdint>

namespace twk {

__host__ __device__ inline long long gcd64(long long a, long long b) {
  while (b) {
    const long long t = a % b;
    a = b;
    b = t;
  }
  return a;
}

// g coprime to N near N / phi and its inverse mod N (g = ginv = 1 for
// N <= 2 and, as a fallback, when no coprime g is found near N / phi).
__host__ __device__ inline void golden_stride(long long N, long long* g, long long* ginv) {
  *g = 1;
  *ginv = 1;
  if (N <= 2) return;
  long long s = (long long)((double)N * 0.6180339887498949);
  for (int k = 0; k < 4096 && gcd64(s, N) != 1; ++k) s = s + 1 < N ? s + 1 : 1;
  if (gcd64(s, N) != 1) return;
  // inverse by the extended Euclidean algorithm: x s = 1 (mod N)
  long long r0 = N, r1 = s, x0 = 0, x1 = 1;
  while (r1) {
    const long long qt = r0 / r1, r2 = r0 - qt * r1, x2 = x0 - qt * x1;
    r0 = r1;
    r1 = r2;
    x0 = x1;
    x1 = x2;
  }
  *g = s;
  *ginv = x0 < 0 ? x0 + N : x0;
}

// Task run at queue position p of n tasks in groups of grp (ng = n / grp
// groups, stride g): the same task of group (p / grp) * g mod ng.
__host__ __device__ inline long long dispersed_task(long long p, unsigned long long g, long long grp,
                                                    long long ng) {
  const long long gp = p / grp;
  return (long long)(((unsigned long long)gp * g) % (unsigned long long)ng) * grp + (p - gp * grp);
}

// The learned order merges the two dispersed classes: the n1 predicted-
// long rows are spread evenly over the first 1/F of the queue and the n0
// others fill the rest.  Long row q (its dispersed rank in its class) has
// the key (2q+1) / (2 F n1), other row b the key (2b+1) / (2 n0); a row's
// place is its rank in its class plus the number of rows of the other
// class before it (long first on equal keys), so the places are a
// permutation of 0 .. n0+n1-1.  Exact integer arithmetic: the counts are
// below 2^59 for up to 2^28 rows.
constexpr long long LONG_SPREAD = 2;  // F: the long rows lie in the first half

__host__ __device__ inline long long merged_place_long(long long q, long long n0, long long n1) {
  if (n0 <= 0) return q;
  // other rows b with (2b+1) F n1 < (2q+1) n0
  const long long m = ((2 * q + 1) * n0 - 1) / (LONG_SPREAD * n1);
  const long long c = (m + 1) / 2;
  return q + (c < 0 ? 0 : (c > n0 ? n0 : c));
}

__host__ __device__ inline long long merged_place_other(long long b, long long n0, long long n1) {
  if (n1 <= 0) return b;
  // long rows q with (2q+1) n0 <= (2b+1) F n1
  const long long m = (LONG_SPREAD * n1 * (2 * b + 1)) / n0;
  const long long c = (m + 1) / 2;
  return b + (c < 0 ? 0 : (c > n1 ? n1 : c));
}

}  // namespace twk

#endif  // TWK_QUEUE_H
