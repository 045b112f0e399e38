// twk_queue.h -- the arithmetic of the contour queue's dispersed order.
//
// The persistent contour kernel takes its queue in a dispersed order:
// queue position p runs group (p * g) mod N of the N groups of tasks (a
// limb-darkened epoch's annulus contours form one group), with g coprime
// to N and close to N / phi (golden ratio), so that any run of consecutive
// positions samples the whole queue evenly.  The learned placement writes
// the row of class rank r to position r * ginv mod N (ginv = g^-1 mod N),
// so that position p again holds rank p * g mod N.
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

}  // namespace twk

#endif  // TWK_QUEUE_H
