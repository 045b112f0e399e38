// twk_fs.h -- finite-source contour integration, one wavefront per source.
//
// Paper: Wang, Wang & Dong, arXiv 2501.03322, Secs. 2.3 (image construction
// and Stokes area), 2.4 (ghost detectors), 2.5 (error estimate and adaptive
// sampling) and 3 (iteration structure: 64 new limb samples per round, only
// new samples are solved, neighbouring links and areas are updated).
//
// MI355X mapping.  One 64-lane wavefront owns one extended source.  Each
// round, lane j solves one new limb point (coefficients, roots, residual
// classification, limb derivatives) in registers and writes the sample
// record to the wave's slice of a global scratch buffer (SoA, one slot per
// sample, slots in creation order).  The sorted order of the limb angles
// lives in LDS: th[] (angle), sl[] (slot) and wc[] (cumulative adaptive
// weight).  Totals, prefix sums and the quantile inversion are wave-wide
// shuffle scans over 64-wide strips of the sorted arrays; the merge of the
// 64 new samples into the sorted arrays is an in-place descending-strip
// move.  Only intervals that touch a new sample are relinked.
#pragma once

#include "twk_device.h"

namespace twk {

constexpr int WAVE = 64;
constexpr int NNEW = 64;        // new limb samples per round (Sec. 3)
constexpr int METHOD_CAP = 4096; // samples per source (Sec. 3)
constexpr double TWO_PI = 6.283185307179586;
constexpr double PI_64 = 3.141592653589793;

// A finite-source task: everything a wave needs, resolved by the pass that
// queued it.  roots: the five roots at the source centre (lens-2 frame),
// used to warm-start the first limb samples.
struct Task {
  int64_t out;  // index into the output arrays
  double s, q, rho, zx, zy;
  c64 roots[5];
};

// Per-wave slice of the sample scratch: SoA over slots [0, cap).
struct WaveMem {
  c64* root;       // [5][cap] real images first, ghost pair last
  c64* dz;         // [5][cap] z' of the real images
  double* w;       // [5][cap] z' ^ z''
  uint32_t* meta;  // [cap] n | par << 3 | flags << 8
  double* dA;      // [cap] area of the interval starting at this slot
  double* E;       // [cap] error of that interval
  uint32_t* ifl;   // [cap] interval flags
  int cap;
};

constexpr size_t kSlotBytes = 5 * 16 + 5 * 16 + 5 * 8 + 4 + 8 + 8 + 4;

__device__ __forceinline__ WaveMem wave_mem(char* base, int wave, int cap) {
  char* p = base + (size_t)wave * (size_t)cap * kSlotBytes;
  WaveMem m;
  m.cap = cap;
  m.root = (c64*)p;
  p += (size_t)5 * cap * 16;
  m.dz = (c64*)p;
  p += (size_t)5 * cap * 16;
  m.w = (double*)p;
  p += (size_t)5 * cap * 8;
  m.dA = (double*)p;
  p += (size_t)cap * 8;
  m.E = (double*)p;
  p += (size_t)cap * 8;
  m.meta = (uint32_t*)p;
  p += (size_t)cap * 4;
  m.ifl = (uint32_t*)p;
  return m;
}

// Interval flag bits
enum : uint32_t { IF_CROSS = 1u, IF_ANOMALY = 2u, IF_COUNT = 4u };

// ---------------------------------------------------------------- sample
struct Sample {
  Images im;
  c64 dz[5];
  double w[5];
};

// Returns the root sweeps spent: low 16 bits FP64, high 16 bits FP32.
template <bool MIXED>
__device__ inline uint32_t solve_sample(const Lens& L, c64 yc, double rho, double theta, c64 r[5],
                                        Sample& sm) {
  double sn, cs;
  sincos(theta, &sn, &cs);
  const c64 e = cz(cs, sn);
  const c64 y = yc + rho * e;
  c64 c[6];
  coefficients(L, y, c);
  int it, s32 = 0, s64;
  if (MIXED) {
    s32 = aberth32(c, r, 30);
    it = aberth64(c, r, 12);
    s64 = it;
    if (it > 12) {
      it = aberth64(c, r, 40);
      s64 += it;
    }
  } else {
    it = aberth64(c, r, 40);
    s64 = it;
  }
  if (it > 40) {
    cold_start(c, r);
    s64 += aberth64(c, r, 200);
  }
  finish_images(L, y, r, sm.im);
  const c64 zp1 = cz(-rho * sn, rho * cs);  // zeta' = i rho e^{i theta}
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    if (k < sm.im.n) {
      limb_derivs(L, sm.im.z[k], sm.im.J[k], zp1, rho, sm.dz[k], sm.w[k]);
    } else {
      sm.dz[k] = cz(0.0, 0.0);
      sm.w[k] = 0.0;
    }
  }
  return (uint32_t)s64 | ((uint32_t)s32 << 16);
}

__device__ __forceinline__ void store_sample(const WaveMem& m, int slot, const Sample& sm) {
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    m.root[k * m.cap + slot] = sm.im.z[k];
    m.dz[k * m.cap + slot] = sm.dz[k];
    m.w[k * m.cap + slot] = sm.w[k];
  }
  m.meta[slot] = (uint32_t)sm.im.n | (sm.im.par << 3) | (sm.im.flags << 8);
}

// ---------------------------------------------------------------- linking
struct Rec {
  c64 z[5];
  c64 dz[5];
  double w[5];
  int n;
  uint32_t par;
};

__device__ __forceinline__ void load_rec(const WaveMem& m, int slot, Rec& r) {
  uint32_t meta = m.meta[slot];
  r.n = meta & 7u;
  r.par = (meta >> 3) & 31u;
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    r.z[k] = m.root[k * m.cap + slot];
    r.dz[k] = m.dz[k * m.cap + slot];
    r.w[k] = m.w[k * m.cap + slot];
  }
}

// Least total distance injection of list A (ka entries) into list B
// (kb >= ka entries), ka, kb <= 3 (Sec. 2.3: "the way to minimize the sum
// of all distances is selected").  mB[i] receives the B position for A[i].
__device__ inline void inject(const c64* zA, const int* iA, int ka, const c64* zB, const int* iB,
                              int kb, int* mB) {
  double d[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      d[i][j] = (i < ka && j < kb) ? cabs64(zA[iA[i]] - zB[iB[j]]) : 0.0;
  double best = 1e308;
  int b0 = 0, b1 = 1, b2 = 2;
  for (int p0 = 0; p0 < kb; ++p0) {
    if (ka == 1) {
      if (d[0][p0] < best) { best = d[0][p0]; b0 = p0; }
      continue;
    }
    for (int p1 = 0; p1 < kb; ++p1) {
      if (p1 == p0) continue;
      if (ka == 2) {
        double t = d[0][p0] + d[1][p1];
        if (t < best) { best = t; b0 = p0; b1 = p1; }
        continue;
      }
      for (int p2 = 0; p2 < kb; ++p2) {
        if (p2 == p0 || p2 == p1) continue;
        double t = d[0][p0] + d[1][p1] + d[2][p2];
        if (t < best) { best = t; b0 = p0; b1 = p1; b2 = p2; }
      }
    }
  }
  mB[0] = b0;
  mB[1] = b1;
  mB[2] = b2;
}

struct Piece {
  double dA, E;
  uint32_t fl;
};

// Area and error of the interval between samples a and b (Sec. 2.3 area
// pieces; Sec. 2.5 errors).  Linked images of parity p contribute
// p [z_a ^ z_b / 2 + (dA_p1 + dA_p2)/2] with
//   dA_p1 = (w_a + w_b) dth^3 / 24,  dA_p2 = (z_b - z_a) ^ (z'_b - z'_a) dth / 12,
// errors E1 = |w_a - w_b| dth^3/48, E2 = 1.5 |dA_p (|dz|^2/(dth^2 |z'_a.z'_b|) - 1)|,
// E3 = |dA_p| dth^2 / 10, E4 = |dA_p1 - dA_p2|.  A pair created (destroyed)
// on the critical curve adds the chord from its - to + image (+ to -) and
// the cross-caustic correction (w_+ - w_-) dtt^3 / 24 with the effective
// step dtt = |z_+ - z_-| / sqrt|z'_+ . z'_-|; its errors are
// E1 = |w_+ + w_-| dtt^3/48, E2 = 1.5 |(z_+ - z_-).(z'_+ - z'_-) -+ 2 |z_+ - z_-|
// sqrt|z'_+.z'_-|| dtt ("-" for creation along +theta), E3 = |dA_p| dth^2/10.
__device__ inline Piece interval_piece(const Rec& a, const Rec& b, double dth) {
  int pa[5], ma[5], pb[5], mb[5];
  int npa = 0, nma = 0, npb = 0, nmb = 0;
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    if (k < a.n) {
      if ((a.par >> k) & 1u) pa[npa++] = k; else ma[nma++] = k;
    }
    if (k < b.n) {
      if ((b.par >> k) & 1u) pb[npb++] = k; else mb[nmb++] = k;
    }
  }
  Piece out{0.0, 0.0, (a.n != b.n) ? (uint32_t)IF_COUNT : 0u};
  const double dth2 = dth * dth, dth3 = dth2 * dth;
  uint32_t usedA = 0, usedB = 0;  // bit k: image k of a (b) linked
  // two parity classes, each linked by the least-distance injection
#pragma unroll
  for (int cls = 0; cls < 2; ++cls) {
    const int* la = cls == 0 ? pa : ma;
    const int* lb = cls == 0 ? pb : mb;
    const int na = cls == 0 ? npa : nma;
    const int nb = cls == 0 ? npb : nmb;
    const double par = cls == 0 ? 1.0 : -1.0;
    if (na == 0 || nb == 0 || na > 3 || nb > 3) {
      if (na + nb > 0 && (na > 3 || nb > 3)) out.fl |= IF_ANOMALY;
      continue;
    }
    int m[3];
    const bool swap = na > nb;
    if (!swap) inject(a.z, la, na, b.z, lb, nb, m);
    else inject(b.z, lb, nb, a.z, la, na, m);
    const int nl = swap ? nb : na;
    for (int t = 0; t < nl; ++t) {
      const int i = swap ? la[m[t]] : la[t];
      const int j = swap ? lb[t] : lb[m[t]];
      usedA |= 1u << i;
      usedB |= 1u << j;
      const c64 za = a.z[i], zb = b.z[j], da = a.dz[i], db = b.dz[j];
      const double wa = a.w[i], wb = b.w[j];
      const double dAt = 0.5 * cwedge(za, zb);
      const double dAp1 = (wa + wb) * dth3 * (1.0 / 24.0);
      const double dAp2 = cwedge(zb - za, db - da) * dth * (1.0 / 12.0);
      const double dAp = 0.5 * (dAp1 + dAp2);
      out.dA += par * (dAt + dAp);
      const double E1 = fabs(wa - wb) * dth3 * (1.0 / 48.0);
      const double ch2 = cnorm(za - zb);
      const double E2 = 1.5 * fabs(dAp * (ch2 / (dth2 * fabs(cdot(da, db))) - 1.0));
      const double E3 = 0.1 * fabs(dAp) * dth2;
      const double E4 = fabs(dAp1 - dAp2);
      out.E += E1 + E2 + E3 + E4;
    }
  }
  // left-over images: a created (at b) or destroyed (at a) pair
  int lpa = -1, lna = -1, lpb = -1, lnb = -1, ca = 0, cb = 0;
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    if (k < a.n && !((usedA >> k) & 1u)) {
      ++ca;
      if ((a.par >> k) & 1u) lpa = k; else lna = k;
    }
    if (k < b.n && !((usedB >> k) & 1u)) {
      ++cb;
      if ((b.par >> k) & 1u) lpb = k; else lnb = k;
    }
  }
  int kind = 0;
  if (ca == 0 && cb == 2 && lpb >= 0 && lnb >= 0) kind = 1;
  else if (cb == 0 && ca == 2 && lpa >= 0 && lna >= 0) kind = -1;
  else if (ca + cb > 0) out.fl |= IF_ANOMALY;
  if (kind != 0) {
    const Rec& c = kind > 0 ? b : a;
    const int ip = kind > 0 ? lpb : lpa, in = kind > 0 ? lnb : lna;
    const c64 zp = c.z[ip], zm = c.z[in], dp = c.dz[ip], dm = c.dz[in];
    const double wp = c.w[ip], wm = c.w[in];
    const double dd = sqrt(fabs(cdot(dp, dm)));
    const double sep = cabs64(zp - zm);
    const double dtt = sep / dd;
    const double dtt3 = dtt * dtt * dtt;
    const double dAp = (wp - wm) * dtt3 * (1.0 / 24.0);
    const double chord = kind > 0 ? 0.5 * cwedge(zm, zp) : 0.5 * cwedge(zp, zm);
    out.dA += chord + dAp;
    const double E1 = fabs(wp + wm) * dtt3 * (1.0 / 48.0);
    const double sgn = kind > 0 ? 1.0 : -1.0;
    const double E2 = 1.5 * fabs(cdot(zp - zm, dp - dm) - sgn * 2.0 * sep * dd) * dtt;
    const double E3 = 0.1 * fabs(dAp) * dth2;
    out.E += E1 + E2 + E3;
    out.fl |= IF_CROSS;
  }
  return out;
}

// ---------------------------------------------------------------- wave ops
__device__ __forceinline__ double wave_incl_scan(double v, int lane) {
#pragma unroll
  for (int o = 1; o < WAVE; o <<= 1) {
    double t = __shfl_up(v, o);
    if (lane >= o) v += t;
  }
  return v;
}

// Error-free transformation a + b = s + e (Knuth's TwoSum).
__device__ __forceinline__ void two_sum(double a, double b, double& s, double& e) {
  s = a + b;
  double bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}

// Wave-wide compensated sum of per-lane (hi, lo) partials; every lane gets
// the same bits (the butterfly combines commutatively).
__device__ __forceinline__ double wave_sum_comp(double hi, double lo) {
#pragma unroll
  for (int o = 1; o < WAVE; o <<= 1) {
    double h2 = __shfl_xor(hi, o), l2 = __shfl_xor(lo, o);
    double s, e;
    two_sum(hi, h2, s, e);
    hi = s;
    lo = lo + l2 + e;
  }
  return hi + lo;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 1; o < WAVE; o <<= 1) v += __shfl_xor(v, o);
  return v;
}

__device__ __forceinline__ uint32_t wave_or(uint32_t v) {
#pragma unroll
  for (int o = 1; o < WAVE; o <<= 1) v |= __shfl_xor(v, o);
  return v;
}

// ---------------------------------------------------------------- engine
template <int CAP>
struct FsLds {
  double th[CAP];      // sorted limb angles
  double wc[CAP + 1];  // interval errors, then their cumulative weights
  uint16_t sl[CAP];    // slot of each sorted position
  int ivl[NNEW];       // old interval index of each accepted new sample
};

struct FsOut {
  double mag, err;
  int n;
  uint32_t flags;
  bool overflow;
  // work counters of this source (wave totals)
  double sweeps32, sweeps64, intervals;
};

// Relink the interval starting at sorted position p (of N) and store its
// area, error and flags under the slot of its left sample.
template <int CAP>
__device__ __forceinline__ uint32_t relink(const WaveMem& m, const FsLds<CAP>& L, int p, int N) {
  const int q = p + 1 < N ? p + 1 : 0;
  const int sa = L.sl[p], sb = L.sl[q];
  const double dth = (p + 1 < N ? L.th[q] : L.th[q] + TWO_PI) - L.th[p];
  Rec a, b;
  load_rec(m, sa, a);
  load_rec(m, sb, b);
  Piece pc = interval_piece(a, b, dth);
  m.dA[sa] = pc.dA;
  m.E[sa] = pc.E;
  m.ifl[sa] = pc.fl;
  return pc.fl;
}

// Number of accepted new samples whose old interval index is < p.
__device__ __forceinline__ int count_before(const int* ivl, int m, int p) {
  int lo = 0, hi = m;  // first r with ivl[r] >= p
  while (lo < hi) {
    int mid = (lo + hi) >> 1;
    if (ivl[mid] < p) lo = mid + 1; else hi = mid;
  }
  return lo;
}

template <int CAP, bool MIXED>
__device__ FsOut fs_source(const Task& T, double tol, const WaveMem& m, FsLds<CAP>& L, int lane) {
  const Lens lens = make_lens(T.s, T.q);
  const c64 yc = cz(T.zx - lens.z2, T.zy);
  const double rho = T.rho;
  uint32_t fl = 0;
  uint32_t sw32 = 0, sw64 = 0, nint = 0;  // this lane's work
  int N = NNEW;
  // Initial samples: theta_j = 2 pi j / 64, warm-started from the roots at
  // the source centre.
  {
    const double th = TWO_PI * lane / (double)NNEW;
    c64 r[5];
#pragma unroll
    for (int k = 0; k < 5; ++k) r[k] = T.roots[k];
    Sample sm;
    const uint32_t sw = solve_sample<MIXED>(lens, yc, rho, th, r, sm);
    sw64 += sw & 0xffffu;
    sw32 += sw >> 16;
    store_sample(m, lane, sm);
    fl |= sm.im.flags & (F_ANOMALY | F_NEARDEGEN);
    L.th[lane] = th;
    L.sl[lane] = (uint16_t)lane;
  }
  __syncthreads();
  {
    uint32_t f = relink(m, L, lane, N);
    ++nint;
    if (f & IF_ANOMALY) fl |= F_ANOMALY;
  }
  __syncthreads();
  double A = 0.0, E = 0.0;
  bool overflow = false;
  for (;;) {
    // totals: compensated area, plain error; errors staged in wc[p+1]
    double hi = 0.0, lo = 0.0, es = 0.0;
    for (int p = lane; p < N; p += WAVE) {
      const int sa = L.sl[p];
      const double a = m.dA[sa], e = m.E[sa];
      double s, t;
      two_sum(hi, a, s, t);
      hi = s;
      lo += t;
      es += e;
      L.wc[p + 1] = e;
    }
    A = wave_sum_comp(hi, lo);
    E = wave_sum(es);
    if (E <= tol * fabs(A)) break;
    int nnew = NNEW;
    if (N + nnew > CAP) {
      if (CAP < METHOD_CAP) { overflow = true; break; }
      nnew = CAP - N;
      if (nnew <= 0) { fl |= F_CAP; break; }
    }
    // tolerance-subtracted weights, cumulative over sorted positions
    const double avg = tol * fabs(A) / N;
    __syncthreads();
    double carry = 0.0;
    for (int base = 0; base < N; base += WAVE) {
      const int p = base + lane;
      double w = 0.0;
      if (p < N) w = fmax(L.wc[p + 1] - avg, 0.0);
      double inc = wave_incl_scan(w, lane);
      if (p < N) L.wc[p + 1] = carry + inc;
      carry += __shfl(inc, WAVE - 1);
    }
    if (lane == 0) L.wc[0] = 0.0;
    __syncthreads();
    const double W = L.wc[N];
    if (!(W > 0.0)) break;
    // inverse transform: quantile (j + 1/2)/nnew of the cumulative weight
    bool valid = false;
    int iv = 0;
    double thn = 0.0;
    if (lane < nnew) {
      const double u = (lane + 0.5) / nnew * W;
      int lo2 = 1, hi2 = N;  // first p in [1, N] with wc[p] > u
      while (lo2 < hi2) {
        int mid = (lo2 + hi2) >> 1;
        if (L.wc[mid] > u) hi2 = mid; else lo2 = mid + 1;
      }
      iv = lo2 - 1;
      const double w0 = L.wc[iv], wi = L.wc[iv + 1] - w0;
      const double ta = L.th[iv];
      const double tb = iv + 1 < N ? L.th[iv + 1] : TWO_PI;
      thn = ta + (u - w0) / wi * (tb - ta);
      valid = wi > 0.0 && thn > ta && thn < tb;
    }
    const int piv = __shfl_up(iv, 1);
    const double pth = __shfl_up(thn, 1);
    if (lane > 0 && valid && piv == iv && !(thn > pth)) valid = false;
    const uint64_t mask = __ballot(valid);
    const int mcount = __popcll(mask);
    if (mcount == 0) { fl |= F_CAP; break; }
    const int rank = __popcll(mask & ((1ull << lane) - 1ull));
    if (valid) L.ivl[rank] = iv;
    // solve the new samples, warm-started from the left neighbour's roots
    if (valid) {
      const int nb = L.sl[iv];
      c64 r[5];
#pragma unroll
      for (int k = 0; k < 5; ++k) r[k] = m.root[k * m.cap + nb];
      Sample sm;
      const uint32_t sw = solve_sample<MIXED>(lens, yc, rho, thn, r, sm);
      sw64 += sw & 0xffffu;
      sw32 += sw >> 16;
      store_sample(m, N + rank, sm);
      fl |= sm.im.flags & (F_ANOMALY | F_NEARDEGEN);
    }
    __syncthreads();
    // merge: old position p moves to p + #(new samples in intervals < p),
    // strips from the top so that no unread entry is overwritten
    for (int base = ((N - 1) / WAVE) * WAVE; base >= 0; base -= WAVE) {
      const int p = base + lane;
      double vt = 0.0;
      uint16_t vs = 0;
      int sh = 0;
      if (p < N) {
        vt = L.th[p];
        vs = L.sl[p];
        sh = count_before(L.ivl, mcount, p);
      }
      __syncthreads();
      if (p < N) {
        L.th[p + sh] = vt;
        L.sl[p + sh] = vs;
      }
      __syncthreads();
    }
    int P = 0;
    if (valid) {
      P = iv + 1 + rank;
      L.th[P] = thn;
      L.sl[P] = (uint16_t)(N + rank);
    }
    N += mcount;
    __syncthreads();
    // relink the intervals touching new samples
    if (valid) {
      uint32_t f = relink(m, L, P, N);
      ++nint;
      if (rank == 0 || L.ivl[rank - 1] != iv) {
        f |= relink(m, L, P - 1, N);
        ++nint;
      }
      if (f & IF_ANOMALY) fl |= F_ANOMALY;
    }
    __syncthreads();
  }
  FsOut o;
  const double area = PI_64 * rho * rho;
  o.mag = A / area;
  o.err = E / area;
  o.n = N;
  o.flags = wave_or(fl);
  o.overflow = overflow;
  o.sweeps32 = wave_sum((double)sw32);
  o.sweeps64 = wave_sum((double)sw64);
  o.intervals = wave_sum((double)nint);
  return o;
}

}  // namespace twk
