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
// record (SoA, one slot per sample, slots in creation order) and its place
// in the sorted order of the limb angles (th[] angle, E[] error of the
// interval that starts there, sl[] slot) into the wave's LDS block.  A
// source that would outgrow the block has both copied to the wave's slice
// of global memory and continues there.  The area total is kept
// incrementally (compensated) from the intervals that change; the error
// total, the tolerance-subtracted weights, their prefix sum and the
// quantile inversion are one pass of wave-wide DPP scans over 64-wide
// strips of the sorted arrays.  The 64 new samples are merged into the
// sorted arrays by an in-place descending-strip move.  Only intervals that
// touch a new sample are relinked.
#pragma once
#include <type_traits>

#include "twk_device.h"

// Address spaces of the engine's pointers: records and sorted arrays in LDS,
// or (sources that outgrew LDS) in global memory.  Typed pointers let the compiler
// emit global and LDS instructions instead of generic (flat) ones, which
// wait on both memory counters and route LDS traffic through the vector
// memory pipeline.  (A CPU emulation build defines both as nothing.)
#ifndef TWK_GLOBAL_AS
#define TWK_GLOBAL_AS __attribute__((address_space(1)))
#endif
#ifndef TWK_LDS_AS
#define TWK_LDS_AS __attribute__((address_space(3)))
#endif

namespace twk {

constexpr int WAVE = 64;
constexpr int NNEW = 64;          // new limb samples per round (Sec. 3)
constexpr int METHOD_CAP = 4096;  // samples per source (Sec. 3)
constexpr double TWO_PI = 6.283185307179586;
constexpr double PI_64 = 3.141592653589793;

// A finite-source task: everything a wave needs, resolved by the pass that
// queued it.  roots: the five roots at the source centre (lens-2 frame),
// used to warm-start the first limb samples; tol: the relative tolerance
// this contour must meet.
struct Task {
  int64_t out;  // index into the output arrays
  double s, q, rho, zx, zy, tol;
  c64 roots[5];
};

typedef TWK_GLOBAL_AS double gdouble;
typedef TWK_GLOBAL_AS uint16_t guint16;
typedef TWK_LDS_AS double ldouble;
typedef TWK_LDS_AS uint16_t luint16;
typedef TWK_GLOBAL_AS float gfloat;
typedef TWK_LDS_AS float lfloat;

// Record fields that only enter correction terms, error estimates and warm
// starts (z', z' ^ z'', interval errors) are stored in FP32 on the mixed
// path (clamped to FP32's finite range) and in FP64 on the FP64 path; roots,
// angles and interval areas are FP64 on both.  The smaller records let more
// samples of a source stay in LDS.
template <bool MIXED>
using corr_t = typename std::conditional<MIXED, float, double>::type;
template <bool MIXED>
using lcorr_t = typename std::conditional<MIXED, lfloat, ldouble>::type;
template <bool MIXED>
using gcorr_t = typename std::conditional<MIXED, gfloat, gdouble>::type;
template <class T>
__device__ __forceinline__ void put(T& d, double v) {
  if constexpr (sizeof(T) == 4) d = (float)fmin(fmax(v, -3.0e38), 3.0e38);
  else d = v;
}

// Sample records, SoA over slots (slot = creation order): five roots
// (positive, negative real images, ghost pair) as (re, im), five z' as
// (re, im), five z' ^ z'', the area of the interval starting at the slot,
// and the meta word.  A record view addresses them either in LDS (RecL: the
// wave's LDS copy, for sources that fit) or in the wave's slice of global
// memory (RecG: sources that outgrew LDS); every function on records is a
// template on the view, so LDS-resident sources use LDS instructions only.
// One exception: on the mixed path the interval areas of an LDS-resident
// source stay in the wave's global slice (A = gdouble).  Without them the
// wave's LDS block at capacity 128 is 20 KiB, and eight waves fit a CU's
// 160 KiB instead of seven: 6 % faster on the limb-darkened batch, against
// a few global accesses per sample.
template <class D, class F, class U, class A = D>
struct RecView {
  D* root;  // [5][cap][2]
  F* dz;    // [5][cap][2]
  F* w;     // [5][cap]
  A* dA;    // [cap]
  U* meta;  // [cap]
  int cap;
};
typedef TWK_LDS_AS uint32_t luint32;
typedef TWK_GLOBAL_AS uint32_t guint32;
template <bool MIXED>
using larea_t = typename std::conditional<MIXED, gdouble, ldouble>::type;
template <bool MIXED>
using RecL = RecView<ldouble, lcorr_t<MIXED>, luint32, larea_t<MIXED>>;
template <bool MIXED>
using RecG = RecView<gdouble, gcorr_t<MIXED>, guint32>;

// Bytes per slot: records (212 on the FP64 path, 152 mixed) plus the
// sorted arrays (angle, interval error, slot).
__host__ __device__ constexpr size_t slot_bytes(bool mixed) {
  return mixed ? 5 * 16 + 5 * 8 + 5 * 4 + 8 + 4 + 8 + 4 + 2 : 5 * 16 + 5 * 16 + 5 * 8 + 8 + 4 + 8 + 8 + 2;
}
constexpr size_t kSlotBytesMax = slot_bytes(false);

// The wave's slice of global scratch: records of every slot plus the
// sorted-array spill copies (slices are kSlotBytesMax * METHOD_CAP apart).
template <bool MIXED>
struct WaveMem {
  RecG<MIXED> G;
  gdouble* sth;         // sorted angles (spill copy)
  gcorr_t<MIXED>* sE;   // sorted interval errors (spill copy)
  guint16* ssl;         // sorted slots (spill copy)
};

template <bool MIXED>
__device__ __forceinline__ WaveMem<MIXED> wave_mem(char* base, int wave) {
  constexpr size_t c = sizeof(corr_t<MIXED>);
  char* p = base + (size_t)wave * (size_t)METHOD_CAP * kSlotBytesMax;
  WaveMem<MIXED> m;
  m.G.cap = METHOD_CAP;
  m.G.root = (gdouble*)p;
  p += (size_t)5 * METHOD_CAP * 16;
  m.G.dz = (gcorr_t<MIXED>*)p;
  p += (size_t)5 * METHOD_CAP * 2 * c;
  m.G.w = (gcorr_t<MIXED>*)p;
  p += (size_t)5 * METHOD_CAP * c;
  m.G.dA = (gdouble*)p;
  p += (size_t)METHOD_CAP * 8;
  m.G.meta = (guint32*)p;
  p += (size_t)METHOD_CAP * 4;
  m.sth = (gdouble*)p;
  p += (size_t)METHOD_CAP * 8;
  m.sE = (gcorr_t<MIXED>*)p;
  p += (size_t)METHOD_CAP * c;
  m.ssl = (guint16*)p;
  return m;
}

template <class R>
__device__ __forceinline__ c64 ld_root(const R& m, int k, int slot) {
  return cz(m.root[2 * (k * m.cap + slot)], m.root[2 * (k * m.cap + slot) + 1]);
}
template <class R>
__device__ __forceinline__ c64 ld_dz(const R& m, int k, int slot) {
  return cz((double)m.dz[2 * (k * m.cap + slot)], (double)m.dz[2 * (k * m.cap + slot) + 1]);
}
template <class R>
__device__ __forceinline__ void st_root(const R& m, int k, int slot, c64 v) {
  m.root[2 * (k * m.cap + slot)] = v.x;
  m.root[2 * (k * m.cap + slot) + 1] = v.y;
}
template <class R>
__device__ __forceinline__ void st_dz(const R& m, int k, int slot, c64 v) {
  put(m.dz[2 * (k * m.cap + slot)], v.x);
  put(m.dz[2 * (k * m.cap + slot) + 1], v.y);
}
template <class R>
__device__ __forceinline__ auto& w_at(const R& m, int k, int slot) { return m.w[k * m.cap + slot]; }
template <class R>
__device__ __forceinline__ auto& dA_at(const R& m, int slot) { return m.dA[slot]; }
template <class R>
__device__ __forceinline__ auto& meta_at(const R& m, int slot) { return m.meta[slot]; }

// Interval flag bits
enum : uint32_t { IF_CROSS = 1u, IF_ANOMALY = 2u, IF_COUNT = 4u };

// Sample meta word: n (bits 0-2) | parity mask (3-7) | sample flags (8-15) |
// demoted (16) | demoted + image (17-19) | demoted - image (20-22) |
// suspect (23).
enum : uint32_t { M_DEMOTED = 1u << 16, M_SUSPECT = 1u << 23 };
// Image count of a solved sample, reported by solve_store beside its flags
// (not stored in the meta word).
enum : uint32_t { M_SEEN3 = 1u << 24, M_SEEN5 = 1u << 25 };

// Slope detector (Sec. 2.4.2).  A five-image sample whose ghost-pair
// margin is above SUSPECT (yet below the residual detector's gap) may hold
// a ghost pair taken for real; only such samples are examined, and a pair
// whose difference is shorter than PAIR_FLOOR (1 + |z|) is below the
// resolution of the test and counts as a genuine crossing.
constexpr double SUSPECT = 8.0;
constexpr double PAIR_FLOOR = 1e-7;

// ---------------------------------------------------------------- sample
// Solve the limb point at theta from the start r[] (warm: a neighbouring
// sample's roots advanced along their derivative; or the centre roots) and
// write its record to `slot`.  Returns the root sweeps spent (low 16 bits
// FP64, high 16 bits FP32) and the sample flags in *fl.
// CONV: the comparator (conventional coefficients, the legacy absolute-
// threshold classification).
template <bool MIXED, class R, bool CONV = false>
__device__ inline uint32_t solve_store(const Lens& L, c64 yc, double rho, double theta, c64 r[5],
                                       const R& m, int slot, uint32_t* fl) {
  double sn, cs;
  limb_sincos(theta, &sn, &cs);
  const c64 y = yc + rho * cz(cs, sn);
  c64 c[6];
  if constexpr (CONV) coefficients_conventional(L, y, c);
  else coefficients(L, y, c);
  int it, s32 = 0, s64;
  if (MIXED) s32 = aberth32(c, r, 12);
  it = aberth64(c, r, 40);
  s64 = it;
  if (it > 40) {
    cold_start(c, r);
    s64 += aberth64(c, r, 200);
  }
  Images im;
  if constexpr (CONV) finish_images_legacy(L, y, r, im);
  else finish_images(L, y, r, im);
  const c64 zp1 = cz(-rho * sn, rho * cs);  // zeta' = i rho e^{i theta}
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    c64 dz = cz(0.0, 0.0);
    double w = 0.0;
    if (k < im.n) limb_derivs(L, im.z[k], im.J[k], zp1, rho, dz, w);
    st_root(m, k, slot, im.z[k]);
    st_dz(m, k, slot, dz);
    put(w_at(m, k, slot), w);
  }
  const bool suspect = im.n == 5 && im.par == 3u && im.margin > SUSPECT;
  meta_at(m, slot) = (uint32_t)im.n | (im.par << 3) | (im.flags << 8) | (suspect ? M_SUSPECT : 0u);
  *fl = im.flags | (suspect ? M_SUSPECT : 0u) | (im.n == 5 ? M_SEEN5 : M_SEEN3);
  return (uint32_t)s64 | ((uint32_t)s32 << 16);
}

// Warm start for a new sample at theta between the stored samples sa (at
// ta) and sb (at tb): the real images of the nearer one advanced by their
// z'; the ghost pair, when both neighbours have three images, interpolated
// linearly between the neighbours' ghost pairs (paired by least total
// distance), else copied from the nearer one.
template <class R>
__device__ __forceinline__ void warm_start(const R& m, int sa, int sb, double ta, double tb,
                                           double theta, c64 r[5]) {
  const bool left = theta - ta <= tb - theta;
  const int sn = left ? sa : sb;
  const double dt = left ? theta - ta : theta - tb;
  const int n = meta_at(m, sn) & 7u;
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    r[k] = ld_root(m, k, sn);
    if (k < n) r[k] = r[k] + dt * ld_dz(m, k, sn);
  }
  if (n == 3 && (meta_at(m, left ? sb : sa) & 7u) == 3u) {
    const c64 a3 = ld_root(m, 3, sa), a4 = ld_root(m, 4, sa);
    c64 b3 = ld_root(m, 3, sb), b4 = ld_root(m, 4, sb);
    if (cnorm(a3 - b4) + cnorm(a4 - b3) < cnorm(a3 - b3) + cnorm(a4 - b4)) {
      const c64 x = b3;
      b3 = b4;
      b4 = x;
    }
    const double f = (theta - ta) / (tb - ta);
    r[3] = a3 + f * (b3 - a3);
    r[4] = a4 + f * (b4 - a4);
  }
}


// ---------------------------------------------------------------- linking
// Sample records keep their real images ordered by parity: positive ones
// first (one of three, two of five), then negative ones, then the ghost
// pair.  Linking (Sec. 2.3) pairs same-parity images of adjacent samples by
// the assignment whose summed image-to-image distance is smallest, tried
// over every permutation; when the counts differ, the left-over + and
// - images at the sample with five images are the pair created (or
// destroyed) on the critical curve.

// Least total distance injection of KA points into KB points (KA <= KB <= 3)
// for static list positions; returns the map packed two bits per entry.
template <int KA, int KB>
__device__ __forceinline__ uint32_t inject_static(const c64* za, const c64* zb) {
  double d[KA][KB];
#pragma unroll
  for (int i = 0; i < KA; ++i)
#pragma unroll
    for (int j = 0; j < KB; ++j) d[i][j] = cabs_fast(za[i] - zb[j]);
  double best = 1e308;
  uint32_t code = 0;
#pragma unroll
  for (int j0 = 0; j0 < KB; ++j0) {
    if (KA == 1) {
      if (d[0][j0] < best) { best = d[0][j0]; code = (uint32_t)j0; }
      continue;
    }
#pragma unroll
    for (int j1 = 0; j1 < KB; ++j1) {
      if (j1 == j0) continue;
      if (KA == 2) {
        const double t = d[0][j0] + d[1 % KA][j1];
        if (t < best) { best = t; code = (uint32_t)(j0 | j1 << 2); }
        continue;
      }
#pragma unroll
      for (int j2 = 0; j2 < KB; ++j2) {
        if (j2 == j0 || j2 == j1) continue;
        const double t = d[0][j0] + d[1 % KA][j1] + d[2 % KA][j2];
        if (t < best) { best = t; code = (uint32_t)(j0 | j1 << 2 | j2 << 4); }
      }
    }
  }
  return code;
}

// General least total distance injection (any counts up to 3 per parity
// class), for image sets whose parity counts are not the binary-lens ones.
__device__ inline void inject_any(const c64* zA, const int* iA, int ka, const c64* zB, const int* iB,
                                  int kb, int* mB) {
  double best = 1e308;
  int b0 = 0, b1 = 1, b2 = 2;
  for (int p0 = 0; p0 < kb; ++p0) {
    if (ka == 1) {
      const double t = cabs64(zA[iA[0]] - zB[iB[p0]]);
      if (t < best) { best = t; b0 = p0; }
      continue;
    }
    for (int p1 = 0; p1 < kb; ++p1) {
      if (p1 == p0) continue;
      const double t2 = cabs64(zA[iA[0]] - zB[iB[p0]]) + cabs64(zA[iA[1]] - zB[iB[p1]]);
      if (ka == 2) {
        if (t2 < best) { best = t2; b0 = p0; b1 = p1; }
        continue;
      }
      for (int p2 = 0; p2 < kb; ++p2) {
        if (p2 == p0 || p2 == p1) continue;
        const double t = t2 + cabs64(zA[iA[2]] - zB[iB[p2]]);
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

// Area and error contributions (Sec. 2.3 area pieces; Sec. 2.5 errors).
// A linked pair of parity p adds p [z_a ^ z_b / 2 + (dA_p1 + dA_p2)/2] with
//   dA_p1 = (w_a + w_b) dth^3 / 24,  dA_p2 = (z_b - z_a) ^ (z'_b - z'_a) dth / 12,
// errors E1 = |w_a - w_b| dth^3/48, E2 = 1.5 |dA_p (|dz|^2/(dth^2 |z'_a.z'_b|) - 1)|,
// E3 = |dA_p| dth^2 / 10, E4 = |dA_p1 - dA_p2|.
template <class R>
__device__ __forceinline__ void add_link(const R& m, int sa, int ia, int sb, int ib,
                                         double par, double dth, Piece& out) {
  const c64 za = ld_root(m, ia, sa), zb = ld_root(m, ib, sb);
  const c64 da = ld_dz(m, ia, sa), db = ld_dz(m, ib, sb);
  const double wa = w_at(m, ia, sa), wb = w_at(m, ib, sb);
  const double dth2 = dth * dth, dth3 = dth2 * dth;
  const double dAt = 0.5 * cwedge(za, zb);
  const double dAp1 = (wa + wb) * dth3 * (1.0 / 24.0);
  const double dAp2 = cwedge(zb - za, db - da) * dth * (1.0 / 12.0);
  const double dAp = 0.5 * (dAp1 + dAp2);
  out.dA += par * (dAt + dAp);
  const double E1 = fabs(wa - wb) * dth3 * (1.0 / 48.0);
  const double ch2 = cnorm(za - zb);
  const double E2 = 1.5 * fabs(dAp * (ch2 * rcp64(dth2 * fabs(cdot(da, db))) - 1.0));
  const double E3 = 0.1 * fabs(dAp) * dth2;
  const double E4 = fabs(dAp1 - dAp2);
  out.E += E1 + E2 + E3 + E4;
}

// A pair created (kind +1, at the later sample) or destroyed (kind -1, at
// the earlier sample) on the critical curve: the boundary runs from its -
// to its + image (creation) or + to - (destruction); chord plus the
// cross-caustic correction (w_+ - w_-) dtt^3 / 24 with the effective step
// dtt = |z_+ - z_-| / sqrt|z'_+ . z'_-|; errors E1 = |w_+ + w_-| dtt^3/48,
// E2 = 1.5 |(z_+ - z_-).(z'_+ - z'_-) -+ 2 |z_+ - z_-| sqrt|z'_+.z'_-|| dtt ("-"
// for creation along +theta), E3 = |dA_p| dth^2 / 10.
template <class R>
__device__ __forceinline__ void add_cross(const R& m, int sc, int ip, int in, int kind,
                                          double dth, Piece& out) {
  const c64 zp = ld_root(m, ip, sc), zm = ld_root(m, in, sc);
  const c64 dp = ld_dz(m, ip, sc), dm = ld_dz(m, in, sc);
  const double wp = w_at(m, ip, sc), wm = w_at(m, in, sc);
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
  const double E3 = 0.1 * fabs(dAp) * dth * dth;
  out.E += E1 + E2 + E3;
  out.fl |= IF_CROSS;
}

// Image sets whose parity counts are not 1+2 or 2+3: general linking of
// whatever same-parity images there are.
template <class R>
__device__ __attribute__((noinline)) Piece interval_piece_any(const R& m, int sa, int sb,
                                                              double dth) {
  c64 za[5], zb[5];
  const uint32_t ma_ = meta_at(m, sa), mb_ = meta_at(m, sb);
  const int na_ = ma_ & 7u, nb_ = mb_ & 7u;
  const uint32_t para = (ma_ >> 3) & 31u, parb = (mb_ >> 3) & 31u;
  for (int k = 0; k < 5; ++k) {
    za[k] = ld_root(m, k, sa);
    zb[k] = ld_root(m, k, sb);
  }
  int pa[5], ma[5], pb[5], mb[5];
  int npa = 0, nma = 0, npb = 0, nmb = 0;
  for (int k = 0; k < 5; ++k) {
    if (k < na_) {
      if ((para >> k) & 1u) pa[npa++] = k; else ma[nma++] = k;
    }
    if (k < nb_) {
      if ((parb >> k) & 1u) pb[npb++] = k; else mb[nmb++] = k;
    }
  }
  Piece out{0.0, 0.0, IF_ANOMALY | ((na_ != nb_) ? (uint32_t)IF_COUNT : 0u)};
  if (npa > 3 || nma > 3 || npb > 3 || nmb > 3) return out;
  uint32_t usedA = 0, usedB = 0;
  for (int cls = 0; cls < 2; ++cls) {
    const int* la = cls == 0 ? pa : ma;
    const int* lb = cls == 0 ? pb : mb;
    const int na = cls == 0 ? npa : nma;
    const int nb = cls == 0 ? npb : nmb;
    if (na == 0 || nb == 0) continue;
    int mt[3];
    const bool swap = na > nb;
    if (!swap) inject_any(za, la, na, zb, lb, nb, mt);
    else inject_any(zb, lb, nb, za, la, na, mt);
    const int nl = swap ? nb : na;
    for (int t = 0; t < nl; ++t) {
      const int i = swap ? la[mt[t]] : la[t];
      const int j = swap ? lb[t] : lb[mt[t]];
      usedA |= 1u << i;
      usedB |= 1u << j;
      add_link(m, sa, i, sb, j, cls == 0 ? 1.0 : -1.0, dth, out);
    }
  }
  int lpa = -1, lna = -1, lpb = -1, lnb = -1, ca = 0, cb = 0;
  for (int k = 0; k < 5; ++k) {
    if (k < na_ && !((usedA >> k) & 1u)) {
      ++ca;
      if ((para >> k) & 1u) lpa = k; else lna = k;
    }
    if (k < nb_ && !((usedB >> k) & 1u)) {
      ++cb;
      if ((parb >> k) & 1u) lpb = k; else lnb = k;
    }
  }
  if (ca == 0 && cb == 2 && lpb >= 0 && lnb >= 0) add_cross(m, sb, lpb, lnb, 1, dth, out);
  else if (cb == 0 && ca == 2 && lpa >= 0 && lna >= 0) add_cross(m, sa, lpa, lna, -1, dth, out);
  return out;
}

// Area and error of the interval between the samples in slots sa and sb,
// dth apart.  The four count patterns of a binary lens (3-3, 5-5, 3-5, 5-3)
// are linked with static list positions; image data are read from the
// (cached) sample records with computed offsets.
// Count pattern of an interval: 0 = 3-3, 1 = 5-5, 2 = 3-5 or 5-3 (all with
// the standard image order), 3 = anything else.
__device__ __forceinline__ int link_pattern(uint32_t ma, uint32_t mb) {
  const int na = ma & 7u, nb = mb & 7u;
  const uint32_t para = (ma >> 3) & 31u, parb = (mb >> 3) & 31u;
  const bool stda = (na == 3 && para == 1u) || (na == 5 && para == 3u);
  const bool stdb = (nb == 3 && parb == 1u) || (nb == 5 && parb == 3u);
  if (!stda || !stdb) return 3;
  return na == nb ? (na == 5 ? 1 : 0) : 2;
}

// Distance of a pair of the padded lists in the unified linking below
// (0 unless both entries are present).
__device__ __forceinline__ double pair_dist(c64 a, bool pa, c64 b, bool pb) {
  return (pa && pb) ? cabs_fast(a - b) : 0.0;
}

// Area and error of the interval between slots sa and sb, dth apart.
// path (the same for every active lane of the wave) selects the code:
// 0 = every interval of the wave is 3-3, 1 = every one is 5-5, 2 = mixed
// patterns.  Path 2 links every count pattern with the same instructions:
// the positive lists are padded to two entries and the negative lists to
// three with absent entries; among the permutations of each padded pair of
// lists that pair as few absent entries with present ones as possible, the
// one of least total distance over present pairs is the least-total-distance
// injection of the shorter list into the longer (first minimum in
// lexicographic order, like the static code); present-present pairs are
// links, and the two images
// left over at the five-image sample are the pair created (or destroyed) on
// the critical curve.  Patterns other than the binary-lens ones take the
// general (out-of-line) code.
template <class R>
__device__ inline Piece interval_piece(const R& m, int sa, int sb, double dth, int path) {
  const uint32_t ma_ = meta_at(m, sa), mb_ = meta_at(m, sb);
  const int na = ma_ & 7u, nb = mb_ & 7u;
  if (link_pattern(ma_, mb_) == 3) return interval_piece_any(m, sa, sb, dth);
  c64 za[5], zb[5];
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    za[k] = ld_root(m, k, sa);
    zb[k] = ld_root(m, k, sb);
  }
  Piece out{0.0, 0.0, na != nb ? (uint32_t)IF_COUNT : 0u};
  if (path == 0) {
    add_link(m, sa, 0, sb, 0, 1.0, dth, out);
    const uint32_t c = inject_static<2, 2>(za + 1, zb + 1);
    add_link(m, sa, 1, sb, 1 + (c & 3u), -1.0, dth, out);
    add_link(m, sa, 2, sb, 1 + ((c >> 2) & 3u), -1.0, dth, out);
    return out;
  }
  if (path == 1) {
    const uint32_t cp = inject_static<2, 2>(za, zb);
    add_link(m, sa, 0, sb, cp & 3u, 1.0, dth, out);
    add_link(m, sa, 1, sb, (cp >> 2) & 3u, 1.0, dth, out);
    const uint32_t cn = inject_static<3, 3>(za + 2, zb + 2);
    add_link(m, sa, 2, sb, 2 + (cn & 3u), -1.0, dth, out);
    add_link(m, sa, 3, sb, 2 + ((cn >> 2) & 3u), -1.0, dth, out);
    add_link(m, sa, 4, sb, 2 + ((cn >> 4) & 3u), -1.0, dth, out);
    return out;
  }
  // padded lists: record positions and presence
  const bool a5 = na == 5, b5 = nb == 5;
  const int pia[2] = {0, 1}, pib[2] = {0, 1};
  const bool ppa[2] = {true, a5}, ppb[2] = {true, b5};
  const int nia[3] = {a5 ? 2 : 1, a5 ? 3 : 2, 4}, nib[3] = {b5 ? 2 : 1, b5 ? 3 : 2, 4};
  const bool npa[3] = {true, true, a5}, npb[3] = {true, true, b5};
  c64 pza[2], pzb[2], nza[3], nzb[3];
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    pza[i] = za[pia[i]];
    pzb[i] = zb[pib[i]];
  }
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    nza[i] = a5 ? za[2 + i] : za[i < 2 ? 1 + i : 0];
    nzb[i] = b5 ? zb[2 + i] : zb[i < 2 ? 1 + i : 0];
  }
  // positives: identity or swap
  const int mid = (ppa[0] != ppb[0]) + (ppa[1] != ppb[1]);
  const int msw = (ppa[0] != ppb[1]) + (ppa[1] != ppb[0]);
  const double pid = pair_dist(pza[0], ppa[0], pzb[0], ppb[0]) + pair_dist(pza[1], ppa[1], pzb[1], ppb[1]);
  const double psw = pair_dist(pza[0], ppa[0], pzb[1], ppb[1]) + pair_dist(pza[1], ppa[1], pzb[0], ppb[0]);
  const bool swp = msw < mid || (msw == mid && psw < pid);
  // negatives: the six permutations in lexicographic order
  double nc[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) nc[i][j] = pair_dist(nza[i], npa[i], nzb[j], npb[j]);
  const int perms[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
  double best = 0.0;
  int bp = -1, bm = 4;
#pragma unroll
  for (int q = 0; q < 6; ++q) {
    const int mis = (npa[0] != npb[perms[q][0]]) + (npa[1] != npb[perms[q][1]]) +
                    (npa[2] != npb[perms[q][2]]);
    const double t = nc[0][perms[q][0]] + nc[1][perms[q][1]] + nc[2][perms[q][2]];
    if (mis < bm || (mis == bm && t < best)) {
      bm = mis;
      best = t;
      bp = q;
    }
  }
  // links (the absent ones contribute nothing) and the left-over pair
  int lpos = 0, lneg = 0;
  bool lp_at_b = false;
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const int j = swp ? 1 - i : i;
    if (ppa[i] && ppb[j]) add_link(m, sa, pia[i], sb, pib[j], 1.0, dth, out);
    else if (ppb[j]) { lpos = pib[j]; lp_at_b = true; }
    else if (ppa[i]) lpos = pia[i];
  }
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    int j = perms[0][i];
#pragma unroll
    for (int q = 1; q < 6; ++q)
      if (bp == q) j = perms[q][i];
    if (npa[i] && npb[j]) add_link(m, sa, nia[i], sb, nib[j], -1.0, dth, out);
    else if (npb[j]) lneg = nib[j];
    else if (npa[i]) lneg = nia[i];
  }
  // 3 -> 5: the pair is created at b; 5 -> 3: destroyed after a
  if (na != nb) add_cross(m, lp_at_b ? sb : sa, lpos, lneg, lp_at_b ? 1 : -1, dth, out);
  return out;
}

// Path of interval_piece for the wave: every lane calls it (inactive lanes
// with act = false); the ballots make the choice uniform.
__device__ __forceinline__ int link_path(bool act, int pattern) {
  const uint64_t b33 = __ballot(act && pattern == 0);
  const uint64_t b55 = __ballot(act && pattern == 1);
  const uint64_t bmx = __ballot(act && pattern == 2);
  if (bmx || (b33 && b55)) return 2;
  return b55 ? 1 : 0;
}

// ---------------------------------------------------------------- wave ops
// Cross-lane steps use DPP lane moves (row shifts and row broadcasts
// inside the VALU) rather than LDS-routed permutes: a 64-lane scan is four
// row_shr steps (1, 2, 4, 8: Hillis-Steele inside each 16-lane row) and two
// row broadcasts (lane 15 of a row into the next row, lane 31 into rows 2
// and 3).  Doubles move as two 32-bit halves.
template <int CTRL, int ROWS, bool ZERO>
__device__ __forceinline__ double dpp_f64(double v) {
  const uint64_t b = __builtin_bit_cast(uint64_t, v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)b, CTRL, ROWS, 0xF, ZERO);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(b >> 32), CTRL, ROWS, 0xF, ZERO);
  return __builtin_bit_cast(double, ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

template <int CTRL, int ROWS, bool ZERO>
__device__ __forceinline__ uint32_t dpp_u32(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, ROWS, 0xF, ZERO);
}

__device__ __forceinline__ double readlane_f64(double v, int lane) {
  const uint64_t b = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, lane);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), lane);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// Value of the previous lane (lane 0 gets 0).
__device__ __forceinline__ double prev_lane(double v) { return dpp_f64<0x138, 0xF, true>(v); }
__device__ __forceinline__ int prev_lane(int v) {
  return (int)dpp_u32<0x138, 0xF, true>((uint32_t)v);
}

__device__ __forceinline__ double wave_incl_scan(double v, int) {
  v += dpp_f64<0x111, 0xF, true>(v);
  v += dpp_f64<0x112, 0xF, true>(v);
  v += dpp_f64<0x114, 0xF, true>(v);
  v += dpp_f64<0x118, 0xF, true>(v);
  v += dpp_f64<0x142, 0xA, false>(v);
  v += dpp_f64<0x143, 0xC, false>(v);
  return v;
}

// Error-free transformation a + b = s + e (Knuth's TwoSum).
__device__ __forceinline__ void two_sum(double a, double b, double& s, double& e) {
  s = a + b;
  const double bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}

template <int CTRL, int ROWS, bool ZERO>
__device__ __forceinline__ void comp_step(double& hi, double& lo) {
  const double h2 = dpp_f64<CTRL, ROWS, ZERO>(hi), l2 = dpp_f64<CTRL, ROWS, ZERO>(lo);
  double s, e;
  two_sum(hi, h2, s, e);
  hi = s;
  lo = lo + l2 + e;
}

// Wave-wide compensated sum of per-lane (hi, lo) partials by a compensated
// scan; every lane receives the last lane's totals.
__device__ __forceinline__ void wave_sum_comp(double& hi, double& lo) {
  comp_step<0x111, 0xF, true>(hi, lo);
  comp_step<0x112, 0xF, true>(hi, lo);
  comp_step<0x114, 0xF, true>(hi, lo);
  comp_step<0x118, 0xF, true>(hi, lo);
  comp_step<0x142, 0xA, false>(hi, lo);
  comp_step<0x143, 0xC, false>(hi, lo);
  hi = readlane_f64(hi, WAVE - 1);
  lo = readlane_f64(lo, WAVE - 1);
}

__device__ __forceinline__ double wave_sum(double v) {
  return readlane_f64(wave_incl_scan(v, 0), WAVE - 1);
}

__device__ __forceinline__ uint32_t wave_or(uint32_t v) {
  v |= dpp_u32<0x111, 0xF, true>(v);
  v |= dpp_u32<0x112, 0xF, true>(v);
  v |= dpp_u32<0x114, 0xF, true>(v);
  v |= dpp_u32<0x118, 0xF, true>(v);
  v |= dpp_u32<0x142, 0xA, false>(v);
  v |= dpp_u32<0x143, 0xC, false>(v);
  return (uint32_t)__builtin_amdgcn_readlane((int)v, WAVE - 1);
}

// ---------------------------------------------------------------- engine
// LDS of one wave: sample records and sorted arrays for sources of up to
// LCAP samples (correction-term inputs in FP32 on the mixed path, whose
// interval areas stay in global memory: see RecView).
template <int LCAP, bool MIXED>
struct FsLdsArea {
  double dA[LCAP];
};
template <int LCAP>
struct FsLdsArea<LCAP, true> {};
template <int LCAP, bool MIXED>
struct FsLds : FsLdsArea<LCAP, MIXED> {
  double root[5 * LCAP * 2];  // records of the first LCAP slots (see RecView)
  corr_t<MIXED> dz[5 * LCAP * 2];
  corr_t<MIXED> w[5 * LCAP];
  uint32_t meta[LCAP];
  double th[LCAP];          // sorted limb angles
  corr_t<MIXED> E[LCAP];    // error of the interval starting at each sorted position
  uint16_t sl[LCAP];  // slot of each sorted position
  int ivl[NNEW];      // old interval index of each accepted new sample
};

// The sorted arrays in use: the LDS copy (ldouble/lcorr_t/luint16), or,
// once a source outgrows it, the spill copy in the wave's global slice
// (gdouble/gcorr_t/guint16).
template <class D, class F, class U, bool LDS>
struct SortedT {
  static constexpr bool kLds = LDS;
  D* th;
  F* E;
  U* sl;
  int cap;
};
template <bool MIXED>
using SortedL = SortedT<ldouble, lcorr_t<MIXED>, luint16, true>;
template <bool MIXED>
using SortedG = SortedT<gdouble, gcorr_t<MIXED>, guint16, false>;

// Synchronisation of the lanes of the source's wave (a workgroup is one
// wave).  While the source's arrays are in LDS only the compiler must not
// move LDS accesses across the point: one wave's LDS operations are executed
// in issue order.  Once they are in global memory a full workgroup barrier
// (which waits for every outstanding memory operation) orders them.
template <class Sorted>
__device__ __forceinline__ void lane_sync() {
  if constexpr (Sorted::kLds) __builtin_amdgcn_wave_barrier();
  else __syncthreads();
}

struct FsOut {
  double mag, err;
  int n;
  uint32_t flags;
  bool spilled;                          // outgrew the LDS copy
  double sweeps32, sweeps64, intervals;  // work of this source (wave totals)
};

// Relink the interval starting at sorted position p (of N): area to the
// global record of its left slot, error to the sorted arrays.
// Count pattern of the interval starting at sorted position p (of N).
template <class Sorted, class R>
__device__ __forceinline__ int relink_pattern(const R& m, const Sorted& S, int p, int N) {
  const int q = p + 1 < N ? p + 1 : 0;
  return link_pattern(meta_at(m, (int)S.sl[p]), meta_at(m, (int)S.sl[q]));
}

template <class Sorted, class R>
__device__ __forceinline__ Piece relink(const R& m, const Sorted& S, int p, int N, int path) {
  const int q = p + 1 < N ? p + 1 : 0;
  const int sa = S.sl[p], sb = S.sl[q];
  const double dth = (p + 1 < N ? S.th[q] : S.th[q] + TWO_PI) - S.th[p];
  const Piece pc = interval_piece(m, sa, sb, dth, path);
  dA_at(m, sa) = pc.dA;
  put(S.E[p], pc.E);
  return pc;
}

// ---------------------------------------------------------------- slope detector
// Demotion rewrites a five-image record (+ + - - -) as a three-image one
// whose ghost slots hold the demoted pair: [other +, remaining - (in order),
// demoted +, demoted -], remembering the pair so that the rewrite can be
// undone (records are re-examined from scratch every round, as the samples
// around a crossing change).
template <class R>
__device__ inline void permute_record(const R& m, int slot, const int* from) {
  c64 z[5], d[5];
  double w[5];
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    z[k] = ld_root(m, k, slot);
    d[k] = ld_dz(m, k, slot);
    w[k] = w_at(m, k, slot);
  }
  for (int k = 0; k < 5; ++k) {
    st_root(m, k, slot, z[from[k]]);
    st_dz(m, k, slot, d[from[k]]);
    put(w_at(m, k, slot), w[from[k]]);
  }
}

template <class R>
__device__ inline void demote(const R& m, int slot, int cp, int cn) {
  int from[5] = {1 - cp, 0, 0, cp, cn};
  int t = 1;
  for (int k = 2; k < 5; ++k)
    if (k != cn) from[t++] = k;
  permute_record(m, slot, from);
  const uint32_t mt = meta_at(m, slot);
  meta_at(m, slot) = 3u | (1u << 3) | (mt & 0xFF00u) | M_DEMOTED | ((uint32_t)cp << 17) |
                 ((uint32_t)cn << 20) | (mt & M_SUSPECT);
}

template <class R>
__device__ inline void undo_demotion(const R& m, int slot) {
  const uint32_t mt = meta_at(m, slot);
  if (!(mt & M_DEMOTED)) return;
  const int cp = (mt >> 17) & 7u, cn = (mt >> 20) & 7u;
  // current position of each original image
  int from[5];
  from[1 - cp] = 0;
  from[cp] = 3;
  from[cn] = 4;
  int t = 1;
  for (int k = 2; k < 5; ++k)
    if (k != cn) from[k] = t++;
  permute_record(m, slot, from);
  meta_at(m, slot) = 5u | (3u << 3) | (mt & 0xFF00u) | (mt & M_SUSPECT);
}

__device__ __forceinline__ bool standard5(uint32_t mt) {
  return (mt & 7u) == 5u && ((mt >> 3) & 31u) == 3u;
}
__device__ __forceinline__ bool standard3(uint32_t mt) {
  return (mt & 7u) == 3u && ((mt >> 3) & 31u) == 1u;
}

// Count change between adjacent samples a -> b: +1 if a pair is created at
// b (3 -> 5), -1 if destroyed after a (5 -> 3), 0 otherwise; (cp, cn) are the
// record positions of the unmatched + and - images at the five-image
// sample, by the same least-distance linking as the area pieces.
template <class R>
__device__ inline int pair_link(const R& m, int sa, int sb, int& cp, int& cn) {
  const uint32_t ma = meta_at(m, sa), mb = meta_at(m, sb);
  c64 za[5], zb[5];
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    za[k] = ld_root(m, k, sa);
    zb[k] = ld_root(m, k, sb);
  }
  if (standard3(ma) && standard5(mb)) {
    const uint32_t p = inject_static<1, 2>(za, zb);
    const uint32_t n = inject_static<2, 3>(za + 1, zb + 2);
    cp = 1 - (int)(p & 3u);
    cn = 2 + (3 - (int)(n & 3u) - (int)((n >> 2) & 3u));
    return 1;
  }
  if (standard5(ma) && standard3(mb)) {
    const uint32_t p = inject_static<1, 2>(zb, za);
    const uint32_t n = inject_static<2, 3>(zb + 1, za + 2);
    cp = 1 - (int)(p & 3u);
    cn = 2 + (3 - (int)(n & 3u) - (int)((n >> 2) & 3u));
    return -1;
  }
  return 0;
}

// Follow the pair (cp, cn) of five-image sample s0 to five-image sample s1.
template <class R>
__device__ inline bool follow_pair(const R& m, int s0, int s1, int& cp, int& cn) {
  if (!standard5(meta_at(m, s0)) || !standard5(meta_at(m, s1))) return false;
  c64 z0[5], z1[5];
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    z0[k] = ld_root(m, k, s0);
    z1[k] = ld_root(m, k, s1);
  }
  const uint32_t p = inject_static<2, 2>(z0, z1);
  const uint32_t n = inject_static<3, 3>(z0 + 2, z1 + 2);
  cp = (int)((p >> (2 * cp)) & 3u);
  cn = 2 + (int)((n >> (2 * (cn - 2))) & 3u);
  return true;
}

// Genuine crossing test: the new pair's difference D and the ghost pair's
// difference G at the neighbouring three-image sample are close to
// perpendicular, |D . G| <= cos(pi/4) |D| |G|.
__device__ inline bool perp_enough(c64 D, c64 G, c64 zref) {
  const double fl = PAIR_FLOOR * (1.0 + cabs64(zref));
  const double a = cabs64(D), b = cabs64(G);
  if (a < fl || b < fl) return true;
  return fabs(cdot(D, G)) <= 0.70710678118654752 * a * b;
}

template <class R>
__device__ __forceinline__ c64 root_at(const R& m, int slot, int k) {
  return ld_root(m, k, slot);
}

// From the three-image sample at sorted position kb, test the crossing into
// the run of len five-image samples starting at sorted position `first`
// (entered at its start or its end); if the pair is not perpendicular
// enough, walk into the run demoting suspect samples until consecutive
// pair differences turn perpendicular (or the whole run is walked: the
// piece is deleted).  Returns the number of samples demoted.
template <class Sorted, class R>
__device__ inline int walk_run(const R& m, const Sorted& S, int N, int kb, int first, int len,
                               bool from_start) {
  const int j0 = from_start ? 0 : len - 1, dj = from_start ? 1 : -1;
  const int sb = S.sl[kb];
  const int sc = S.sl[(first + j0) % N];
  const uint32_t mc = meta_at(m, sc);
  if (!(mc & M_SUSPECT) || (mc & M_DEMOTED)) return 0;
  int cp = 0, cn = 2;
  const int kind = from_start ? pair_link(m, sb, sc, cp, cn) : pair_link(m, sc, sb, cp, cn);
  if (kind != (from_start ? 1 : -1)) return 0;
  if (perp_enough(root_at(m, sc, cp) - root_at(m, sc, cn), root_at(m, sb, 3) - root_at(m, sb, 4),
                  root_at(m, sc, cp)))
    return 0;
  int demoted = 0;
  for (int j = j0; j >= 0 && j < len; j += dj) {
    const int sj = S.sl[(first + j) % N];
    if (meta_at(m, sj) & M_DEMOTED) break;
    bool more = false;
    int np = cp, nn = cn;
    const int jn = j + dj;
    if (jn >= 0 && jn < len) {
      const int sn = S.sl[(first + jn) % N];
      const uint32_t mn = meta_at(m, sn);
      if ((mn & M_SUSPECT) && !(mn & M_DEMOTED) && follow_pair(m, sj, sn, np, nn))
        more = !perp_enough(root_at(m, sj, cp) - root_at(m, sj, cn),
                            root_at(m, sn, np) - root_at(m, sn, nn), root_at(m, sj, cp));
    }
    demote(m, sj, cp, cn);
    ++demoted;
    if (!more) break;
    cp = np;
    cn = nn;
  }
  return demoted;
}

__device__ __forceinline__ int orig_n(uint32_t mt) { return (mt & M_DEMOTED) ? 5 : (int)(mt & 7u); }

// Runs of five-image samples between three-image ones, each examined from
// both ends (serial; sources with suspect samples are rare).
template <class Sorted, class R>
__device__ inline int detect_runs(const R& m, const Sorted& S, int N) {
  int anchor = -1;
  for (int i = 0; i < N; ++i)
    if (orig_n(meta_at(m, S.sl[i])) == 3) { anchor = i; break; }
  if (anchor < 0) return 0;
  int changed = 0;
  int i = 0;
  while (i < N) {
    if (orig_n(meta_at(m, S.sl[(anchor + i) % N])) != 5) { ++i; continue; }
    const int start = i;
    int len = 0;
    while (i < N && orig_n(meta_at(m, S.sl[(anchor + i) % N])) == 5) { ++len; ++i; }
    const int first = (anchor + start) % N;
    changed += walk_run(m, S, N, (anchor + start - 1 + N) % N, first, len, true);
    changed += walk_run(m, S, N, (anchor + start + len) % N, first, len, false);
  }
  return changed;
}

// Full slope-detector pass of one source: undo last round's demotions,
// re-examine every run, relink every interval and recompute the area total
// (compensated).  Returns true if any sample is demoted.
template <class Sorted, class R>
__device__ __forceinline__ bool slope_pass(const R& m, const Sorted& S, int N, int lane,
                                          double* Ahi, double* Alo, uint32_t* nint) {
  for (int p = lane; p < N; p += WAVE) undo_demotion(m, p);
  lane_sync<Sorted>();
  int changed = 0;
  if (lane == 0) changed = detect_runs(m, S, N);
  changed = __builtin_amdgcn_readlane(changed, 0);
  lane_sync<Sorted>();
  double h = 0.0, l = 0.0;
  for (int base = 0; base < N; base += WAVE) {
    const int p = base + lane;
    const bool act = p < N;
    const int path = link_path(act, act ? relink_pattern(m, S, p, N) : -1);
    if (!act) continue;
    const Piece pc = relink(m, S, p, N, path);
    double s1, e1;
    two_sum(h, pc.dA, s1, e1);
    h = s1;
    l += e1;
    ++*nint;
  }
  wave_sum_comp(h, l);
  *Ahi = h;
  *Alo = l;
  lane_sync<Sorted>();
  return changed > 0;
}

// Relative tolerance targeted by the stop test of a contour that crosses a
// caustic (some samples with three images, some with five): half the stated
// one.  Across a crossing the error estimate of Sec. 2.5 can fall short of
// the true error by up to about a factor 2 (the cross-caustic interval),
// measured against the tight oracle.  A contour that crosses no caustic
// stops at the stated tolerance: there the estimate exceeds the true error
// by a large factor (more than 4 even just outside a caustic).
constexpr double TOL_SAFETY = 0.5;

// Running state of one source's contour integration: wave-uniform totals
// and per-lane work counters.
struct FsState {
  int N;
  double Ahi, Alo, A, E;
  uint32_t fl, sw32, sw64, nint;
  bool suspects;  // some sample may hold a misjudged ghost pair
  uint32_t seen;  // bit 0: a three-image sample seen; bit 1: a five-image one
};
__device__ __forceinline__ FsState fs_fresh() {
  return FsState{0, 0.0, 0.0, 0.0, 0.0, 0u, 0u, 0u, 0u, false, 0u};
}

typedef TWK_LDS_AS int lint;

// Narrowest interval of limb angle that is refined further.  Near the limb
// angle where an image pair merges on the critical curve, the pair's
// separation falls as the square root of the angular distance; below about
// 1e-9 rad it is under the rounding of the near-double roots in binary64,
// so the classification and the pieces there are noise, and sampling into
// them only adds noise.
constexpr double THETA_FLOOR = 1e-9;

// Tolerance-subtracted weight of the interval starting at sorted position
// p of N (error e): zero for intervals narrower than THETA_FLOOR.
template <class Sorted>
__device__ __forceinline__ double interval_weight(const Sorted& S, int p, int N, double e,
                                                  double avg) {
  const double w = (p + 1 < N ? S.th[p + 1] : S.th[0] + TWO_PI) - S.th[p];
  return w > THETA_FLOOR ? fmax(e - avg, 0.0) : 0.0;
}

// How fs_rounds returned: the source is finished (stop test met, cap or no
// placeable sample); the next round would outgrow the LDS copy of the
// sorted arrays (the caller moves them to the wave's global slice and
// continues there); or the round limit was reached (round-by-round
// dispatch: the state is saved and the source continues in a later launch).
enum { FS_DONE = 0, FS_OUTGROWN = 1, FS_PAUSED = 2 };

// Rounds of the contour integration on the sorted arrays S, at most
// max_rounds of them (negative: no limit).  ivl: the wave's LDS array of
// NNEW interval indices of the round's new samples.
template <bool MIXED, class Sorted, class R, bool CONV = false>
__device__ __forceinline__ int fs_rounds(const Task& T, const Lens& lens, c64 yc, double tol,
                                         const R& m, lint* ivl, const Sorted& S, int lane,
                                         int n0, FsState& st, int max_rounds = -1) {
  const double rho = T.rho;
  // state in locals (written back once) so that it stays in registers
  int N = st.N;
  double Ahi = st.Ahi, Alo = st.Alo, A = st.A, E = st.E;
  uint32_t fl = st.fl, sw32 = st.sw32, sw64 = st.sw64, nint = st.nint;
  bool suspects = st.suspects;
  uint32_t seen = st.seen;
  bool outgrown = false, paused = false;
  if (N == 0) {
    // the first round starts from the roots at the source centre, parked in
    // the record slot each lane's first sample will take (slot = lane), so
    // that the round loop reads starts from records only
#pragma unroll
    for (int k = 0; k < 5; ++k) st_root(m, k, lane, T.roots[k]);
  }
  // One round per iteration.  The first n0 samples form the uniform grid
  // theta = 2 pi i / n0, laid down 64 at a time: round r adds the phase
  // offset r / (n0 / 64) of the base grid theta_j = 2 pi j / 64 (whose
  // first round starts from the roots at the source centre) and is not
  // followed by a stop test.  Later rounds place 64 samples by inverse
  // transform sampling.  Solving, merging and relinking have one call site
  // each, which keeps the kernel small.
  for (;;) {
    bool valid;
    uint32_t sf = 0u;  // flags and image count of this lane's new sample
    int iv = -1, rank, mcount;
    double thn;
    if (N < n0) {
      const int r = N / NNEW, m = n0 / NNEW;
      valid = true;
      thn = TWO_PI * (lane + (double)r / m) / NNEW;
      rank = lane;
      mcount = NNEW;
      if (N > 0) {
        // the new sample follows the r samples of base interval j
        iv = lane * r + r - 1;
        ivl[rank] = iv;
      }
    } else {
      // error total and total tolerance-subtracted weight (intervals
      // narrower than THETA_FLOOR weigh nothing)
      A = Ahi + Alo;
      const double tol_r = seen == 3u ? TOL_SAFETY * tol : tol;
      const double avg = tol_r * fabs(A) / N;
      double es = 0.0, ws = 0.0;
      for (int p = lane; p < N; p += WAVE) {
        const double e = S.E[p];
        es += e;
        ws += interval_weight(S, p, N, e, avg);
      }
      E = wave_sum(es);
      if (E <= tol_r * fabs(A)) break;
      // outgrowing the LDS copy: the caller continues in global memory
      if (N + NNEW > S.cap && S.cap < METHOD_CAP) {
        outgrown = true;
        break;
      }
      const int nnew = N + NNEW <= S.cap ? NNEW : S.cap - N;
      if (nnew <= 0) { fl |= F_CAP; break; }
      const double W = wave_sum(ws);
      if (!(W > 0.0)) break;
      // inverse transform sampling: lane j takes quantile (j + 1/2)/nnew of
      // the cumulative weight, located during one strip-wise scan
      const double u = (lane + 0.5) / nnew * W;
      bool found = false;
      double w0 = 0.0, wi = 0.0;
      double carry = 0.0;
      for (int base = 0; base < N; base += WAVE) {
        const int p = base + lane;
        const double w = p < N ? interval_weight(S, p, N, (double)S.E[p], avg) : 0.0;
        const double inc = wave_incl_scan(w, lane);
        const double tot = readlane_f64(inc, WAVE - 1);
        const bool mine = !found && lane < nnew && u < carry + tot;
        if (__ballot(mine)) {
          int lo = 0;  // first strip position whose inclusive sum exceeds u
#pragma unroll
          for (int step = 32; step >= 1; step >>= 1) {
            const double v = carry + __shfl(inc, lo + step - 1);
            if (!(v > u)) lo += step;
          }
          const int lq = lo < WAVE ? lo : WAVE - 1;
          const double wl = __shfl(w, lq), il = __shfl(inc, lq);
          if (mine) {
            found = true;
            iv = base + lq;
            wi = wl;
            w0 = carry + il - wl;
          }
        }
        carry += tot;
      }
      valid = false;
      thn = 0.0;
      if (found && iv < N) {
        const double ta = S.th[iv];
        const double tb = iv + 1 < N ? S.th[iv + 1] : TWO_PI;
        thn = ta + (u - w0) / wi * (tb - ta);
        valid = wi > 0.0 && thn > ta && thn < tb;
      }
      const int piv = prev_lane(iv);
      const double pth = prev_lane(thn);
      if (lane > 0 && valid && piv == iv && !(thn > pth)) valid = false;
      const uint64_t mask = __ballot(valid);
      mcount = __popcll(mask);
      if (mcount == 0) { fl |= F_CAP; break; }
      rank = __popcll(mask & ((1ull << lane) - 1ull));
      if (valid) ivl[rank] = iv;
    }
    // solve the new samples: the centre roots start the first round, later
    // samples start from the nearer neighbour's roots advanced along z'
    if (valid) {
      c64 r[5];
      if (N == 0) {
#pragma unroll
        for (int k = 0; k < 5; ++k) r[k] = ld_root(m, k, lane);
      } else {
        const double ta = S.th[iv];
        const int ivb = iv + 1 < N ? iv + 1 : 0;
        const double tb = iv + 1 < N ? S.th[ivb] : S.th[ivb] + TWO_PI;
        warm_start(m, (int)S.sl[iv], (int)S.sl[ivb], ta, tb, thn, r);
      }
      const uint32_t sw = solve_store<MIXED, R, CONV>(lens, yc, rho, thn, r, m, N + rank, &sf);
      sw64 += sw & 0xffffu;
      sw32 += sw >> 16;
      fl |= sf & (F_ANOMALY | F_NEARDEGEN);
      if (sf & M_SUSPECT) suspects = true;
    }
    suspects = __ballot(suspects) != 0;
    seen |= (__ballot((sf & M_SEEN3) != 0u) ? 1u : 0u) | (__ballot((sf & M_SEEN5) != 0u) ? 2u : 0u);
    lane_sync<Sorted>();
    // merge: old position p moves up by #(new samples in intervals < p);
    // strips from the top so that no unread entry is overwritten
    if (N > 0) {
      const int myivl = lane < mcount ? ivl[lane] : 0x7fffffff;
      for (int base = ((N - 1) / WAVE) * WAVE; base >= 0; base -= WAVE) {
        const int p = base + lane;
        int sh = 0;  // number of r with ivl[r] < p (ivl ascending), 0..64
#pragma unroll
        for (int step = 32; step >= 1; step >>= 1) {
          const int v = __shfl(myivl, sh + step - 1);
          if (v < p) sh += step;
        }
        if (__builtin_amdgcn_readlane(myivl, WAVE - 1) < p) sh = WAVE;  // lifting alone stops at 63
        double vt = 0.0, ve = 0.0;
        uint16_t vs = 0;
        if (p < N) {
          vt = S.th[p];
          ve = S.E[p];
          vs = S.sl[p];
        }
        lane_sync<Sorted>();
        if (p < N && sh > 0) {
          S.th[p + sh] = vt;
          put(S.E[p + sh], ve);
          S.sl[p + sh] = vs;
        }
        lane_sync<Sorted>();
      }
    }
    int P = 0;
    bool first = false;
    double dAold = 0.0;
    if (valid) {
      P = N == 0 ? lane : iv + 1 + rank;
      first = N > 0 && (rank == 0 || ivl[rank - 1] != iv);
      if (first) {
        // mixed path, LDS phase: the areas are in global memory, where the
        // wave barriers do not order other lanes' earlier stores
        if constexpr (Sorted::kLds && MIXED) __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
        dAold = dA_at(m, S.sl[P - 1]);
      }
    }
    lane_sync<Sorted>();
    if (valid) {
      S.th[P] = thn;
      S.sl[P] = (uint16_t)(N + rank);
    }
    N += mcount;
    lane_sync<Sorted>();
    // relink the intervals touching new samples: the one starting at the
    // new sample, and for the first new sample of a split interval the one
    // ending there; the area total changes by the new pieces minus the
    // replaced one (compensated)
    double dh = 0.0, dl = 0.0;
#pragma unroll 1
    for (int j = 0; j < 2; ++j) {
      const bool act = valid && (j == 0 || first);
      const int pp = j == 0 ? P : P - 1;
      const int path = link_path(act, act ? relink_pattern(m, S, pp, N) : -1);
      if (act) {
        const Piece pc = relink(m, S, pp, N, path);
        ++nint;
        double s1, e1;
        two_sum(dh, pc.dA, s1, e1);
        dh = s1;
        dl += e1;
        if (pc.fl & IF_ANOMALY) fl |= F_ANOMALY;
      }
    }
    if (first) {
      double s1, e1;
      two_sum(dh, -dAold, s1, e1);
      dh = s1;
      dl += e1;
    }
    wave_sum_comp(dh, dl);
    {
      double s1, e1;
      two_sum(Ahi, dh, s1, e1);
      Ahi = s1;
      Alo += dl + e1;
    }
    lane_sync<Sorted>();
    if (suspects && slope_pass(m, S, N, lane, &Ahi, &Alo, &nint)) fl |= F_SLOPE;
    if (--max_rounds == 0) {
      paused = true;
      break;
    }
  }
  st = FsState{N, Ahi, Alo, A, E, fl, sw32, sw64, nint, suspects, seen};
  return outgrown ? FS_OUTGROWN : (paused ? FS_PAUSED : FS_DONE);
}

// Output of a finished source from its final state.
__device__ __forceinline__ FsOut fs_output(const Task& T, const FsState& st, bool spilled) {
  FsOut o;
  const double area = PI_64 * T.rho * T.rho;
  o.mag = st.A / area;
  o.err = st.E / area;
  o.n = st.N;
  o.flags = wave_or(st.fl);
  o.spilled = spilled;
  o.sweeps32 = wave_sum((double)st.sw32);
  o.sweeps64 = wave_sum((double)st.sw64);
  o.intervals = wave_sum((double)st.nint);
  return o;
}

// The rounds of one source on the LDS copies of its records and sorted
// arrays (st: fresh state on entry, final or outgrown state on return).
// Returns true if the source outgrew the LDS copy: its records and sorted
// arrays are then copied to the wave's global slice, where
// fs_source_global continues it.
template <int LCAP, bool MIXED>
__device__ __forceinline__ bool fs_source_lds(const Task& T, double tol, const WaveMem<MIXED>& gm,
                                              FsLds<LCAP, MIXED>& L, int lane, int n0,
                                              FsState& st) {
  const Lens lens = make_lens(T.s, T.q);
  const c64 yc = cz(T.zx - lens.z2, T.zy);
  const SortedL<MIXED> S{(ldouble*)L.th, (lcorr_t<MIXED>*)L.E, (luint16*)L.sl, LCAP};
  larea_t<MIXED>* area;
  if constexpr (MIXED) area = gm.G.dA;
  else area = (ldouble*)L.dA;
  const RecL<MIXED> R{(ldouble*)L.root, (lcorr_t<MIXED>*)L.dz, (lcorr_t<MIXED>*)L.w, area,
               (luint32*)L.meta, LCAP};
  if (fs_rounds<MIXED>(T, lens, yc, tol, R, (lint*)L.ivl, S, lane, n0, st) != FS_OUTGROWN)
    return false;
  for (int p = lane; p < st.N; p += WAVE) {
    gm.sth[p] = S.th[p];
    gm.sE[p] = S.E[p];
    gm.ssl[p] = S.sl[p];
    // slot p's record (slots are 0 .. N-1)
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      st_root(gm.G, k, p, ld_root(R, k, p));
      st_dz(gm.G, k, p, ld_dz(R, k, p));
      w_at(gm.G, k, p) = w_at(R, k, p);
    }
    if constexpr (!MIXED) dA_at(gm.G, p) = dA_at(R, p);  // mixed: already there
    meta_at(gm.G, p) = meta_at(R, p);
  }
  __syncthreads();
  return true;
}

// The remaining rounds of a source that outgrew its LDS copy, on the
// records and sorted arrays in the wave's global slice.
template <bool MIXED>
__device__ __forceinline__ void fs_source_global(const Task& T, double tol, const WaveMem<MIXED>& gm,
                                                 lint* ivl, int lane, FsState& st) {
  const Lens lens = make_lens(T.s, T.q);
  const c64 yc = cz(T.zx - lens.z2, T.zy);
  const SortedG<MIXED> S{gm.sth, gm.sE, gm.ssl, METHOD_CAP};
  fs_rounds<MIXED>(T, lens, yc, tol, gm.G, ivl, S, lane, 0, st);
}

// One source from start to finish (both parts in sequence).  The
// persistent kernel instead runs the LDS part of many sources in one loop
// and the global part of an outgrown source after leaving it, so that the
// two parts' registers never meet in one loop and no call is made.
template <int LCAP, bool MIXED>
__device__ FsOut fs_source(const Task& T, double tol_stated, const WaveMem<MIXED>& gm,
                           FsLds<LCAP, MIXED>& L,
                           int lane, int n0) {
  FsState st = fs_fresh();
  const bool spilled = fs_source_lds<LCAP, MIXED>(T, tol_stated, gm, L, lane, n0, st);
  if (spilled) fs_source_global<MIXED>(T, tol_stated, gm, (lint*)L.ivl, lane, st);
  return fs_output(T, st, spilled);
}

// ------------------------------------------------------- round-by-round dispatch
// The paper's dispatch (Secs. 3, 4.1): one kernel launch per refinement
// round, over the list of sources not yet finished; a source's records and
// sorted arrays live in its global slice, and its running totals here,
// between launches.
struct RoundState {
  double Ahi, Alo, A, E;
  double sw32, sw64, nint;  // work of the rounds so far (wave totals)
  int N;
  uint32_t fl;              // OR of the lanes' flags so far
  int suspects;
  uint32_t seen;            // image counts seen so far (FsState::seen)
  int done;
};

// One round of one source.  fresh: the source starts (its first round lays
// down the first 64 samples of the uniform grid of n0).  Returns true when
// the source is finished, with its output in *o; otherwise its state is
// saved in *rs for the next launch.
template <bool MIXED, bool CONV = false>
__device__ bool fs_round_step(const Task& T, double tol_stated, const WaveMem<MIXED>& gm,
                              lint* ivl, int lane, int n0, RoundState* rs, bool fresh, FsOut* o) {
  const double tol = tol_stated;
  const Lens lens = make_lens(T.s, T.q);
  const c64 yc = cz(T.zx - lens.z2, T.zy);
  FsState st{0, 0.0, 0.0, 0.0, 0.0, 0u, 0u, 0u, 0u, false, 0u};
  double base32 = 0.0, base64 = 0.0, baseint = 0.0;
  if (!fresh) {
    const RoundState r = *rs;
    st = FsState{r.N, r.Ahi, r.Alo, r.A, r.E, r.fl, 0u, 0u, 0u, r.suspects != 0, r.seen};
    base32 = r.sw32;
    base64 = r.sw64;
    baseint = r.nint;
  }
  const SortedG<MIXED> S{gm.sth, gm.sE, gm.ssl, METHOD_CAP};
  const int how = fs_rounds<MIXED, SortedG<MIXED>, RecG<MIXED>, CONV>(T, lens, yc, tol, gm.G, ivl, S,
                                                                     lane, n0, st, 1);
  FsOut out = fs_output(T, st, true);
  out.sweeps32 += base32;
  out.sweeps64 += base64;
  out.intervals += baseint;
  if (lane == 0) {
    RoundState r;
    r.Ahi = st.Ahi;
    r.Alo = st.Alo;
    r.A = st.A;
    r.E = st.E;
    r.sw32 = out.sweeps32;
    r.sw64 = out.sweeps64;
    r.nint = out.intervals;
    r.N = st.N;
    r.fl = out.flags;
    r.suspects = st.suspects ? 1 : 0;
    r.seen = st.seen;
    r.done = how != FS_PAUSED;
    *rs = r;
  }
  *o = out;
  return how != FS_PAUSED;
}

}  // namespace twk
