// twk_cpu.cpp -- multi-core CPU backend of the finite-source binary-lens
// magnification method (the CPU version of the paper's Sec. 4.5).
//
// Paper: Wang, Wang & Dong, arXiv 2501.03322.  Declarations and argument
// contracts are in include/twk_cpu.h.  Plain C++17, std::complex<double>,
// one source per worker thread at a time.  Frame: the lens-2 frame of
// Sec. 2.2 (eta = z - z2, y = zeta - z2), in which lens 1 sits at -s and
// lens 2 at 0.
#include "../../include/twk_cpu.h"

#include <algorithm>
#include <atomic>
#include <cmath>
#include <complex>
#include <cstdint>
#include <thread>
#include <vector>

namespace {

using cd = std::complex<double>;

constexpr double TWO_PI = 6.283185307179586476925286766559;
constexpr double EPS = 2.220446049250313e-16;
constexpr int NNEW = 64;          // samples per round (Sec. 3)
constexpr int CAP = 4096;         // samples per source (Sec. 3)
constexpr double GAP = 100.0;     // ghost pair: second-largest residual over the noise
constexpr double FLOOR = 1e-9;    // narrowest interval refined (rad)
constexpr double SAFETY = 0.5;    // tolerance factor once the limb crosses a caustic
constexpr double CQ = 20.0;       // point-source test: quadrupole factor
constexpr double CG = 8.0;        // point-source test: ghost distance in units of rho
constexpr uint32_t F_POINT = 1u, F_CAP = 2u, F_NONFINITE = 16u, F_NEAR = 32u;

double wedge(cd a, cd b) { return (std::conj(a) * b).imag(); }
double dot(cd a, cd b) { return (std::conj(a) * b).real(); }

struct Lens {
  double s, m1, m2, z2;
};

Lens make_lens(double s, double q) { return {s, 1.0 / (1.0 + q), q / (1.0 + q), s / (1.0 + q)}; }

// Sec. 2.2, Eq. method-transformed: the coefficients c0..c5 of the quintic
// in the lens-2 frame, each a sum of terms of one order in q (no
// cancellation), with v_c = conj(y) + s and v_p = 1 + s conj(y); "Im(y) i"
// is i Im(y) and Re() takes the real parts of v_p, v_c and 1 - s y.
void quintic(const Lens& L, cd y, cd c[6]) {
  const double s = L.s, m2 = L.m2, ms = m2 * s;
  const cd yb = std::conj(y), iy(0.0, y.imag());
  const cd vc = yb + s, vp = 1.0 + s * yb;
  const double rvp = 1.0 + s * y.real(), rvc = y.real() + s, r1 = 1.0 - s * y.real();
  c[5] = -yb * vc;
  c[4] = (yb * y - 1.0 - 2.0 * s * yb) * vc + ms;
  c[3] = (2.0 * y - s) * (vp * vc + 2.0 * iy - ms) + 4.0 * (ms - y) * iy;
  c[2] = cd(rvp * rvp * rvc, y.imag() * rvp * r1) + s * y.imag() * y.imag() * (2.0 + s * vc) +
         ms * (2.0 * yb * (y - s) - (1.0 - s * y));
  c[1] = ms * ((s + 2.0 * y) * vp + s * (2.0 * s * iy - m2));
  c[0] = s * s * m2 * m2 * y;
}

// All five roots by simultaneous Aberth-Ehrlich correction from the start
// r[]: each root moves by p/p' deflated against the others.  Stops when the
// largest relative step is below 1e-14; returns false if it never does.
bool aberth(const cd c[6], cd r[5], int maxit) {
  for (int it = 0; it < maxit; ++it) {
    double worst = 0.0;
    for (int k = 0; k < 5; ++k) {
      cd p = c[5], d = 0.0;
      for (int j = 4; j >= 0; --j) {
        d = d * r[k] + p;
        p = p * r[k] + c[j];
      }
      if (p == 0.0 || d == 0.0) continue;
      cd inv = 0.0;
      for (int j = 0; j < 5; ++j)
        if (j != k) inv += 1.0 / (r[k] - r[j]);
      const cd ratio = p / d;
      const cd step = ratio / (1.0 - ratio * inv);
      r[k] -= step;
      worst = std::max(worst, std::abs(step) / std::max(std::abs(r[k]), 1e-300));
    }
    if (worst < 1e-14) return true;
  }
  return false;
}

void circle_start(const cd c[6], cd r[5]) {
  double rad = std::pow(std::abs(c[0]) / std::abs(c[5]), 0.2);
  if (!(rad > 0.0 && rad < 1e30)) rad = 1.0;
  for (int k = 0; k < 5; ++k) r[k] = std::polar(rad, 0.4 + TWO_PI * k / 5.0);
}

struct LensAt {
  cd R, fp;   // lens-equation residual, f'
  double J;   // 1 - |f'|^2
};

// Residual of the lens equation (Sec. 2.4.1) and the Jacobian at eta.
LensAt lens_at(const Lens& L, cd y, cd e) {
  const cd a = 1.0 / (e + L.s), b = 1.0 / e;
  LensAt o;
  o.R = y - e + L.m1 * std::conj(a) + L.m2 * std::conj(b);
  o.fp = L.m1 * a * a + L.m2 * b * b;
  o.J = 1.0 - std::norm(o.fp);
  return o;
}

cd fsecond(const Lens& L, cd e) {
  const cd a = 1.0 / (e + L.s), b = 1.0 / e;
  return -2.0 * (L.m1 * a * a * a + L.m2 * b * b * b);
}

// Images of the source point y: z[] positive-parity real images first, then
// negative ones, then the ghost pair; n = 3 or 5.
struct Images {
  cd z[5];
  double J[5];
  int n, npos;
  uint32_t flags;
};

// Roots r[] of y's quintic -> polished, classified images.
void classify(const Lens& L, cd y, cd r[5], Images& im) {
  LensAt at[5];
  for (int k = 0; k < 5; ++k) {
    // one Newton step on the lens equation, kept only when tiny against the
    // distance to the nearer lens and when it at least halves |R|: real
    // images near the critical curve recover the precision the polynomial
    // solve loses there; ghosts have no nearby solution
    at[k] = lens_at(L, y, r[k]);
    const cd dz = (at[k].R - std::conj(at[k].fp) * std::conj(at[k].R)) / at[k].J;
    const double scale = std::min(std::norm(r[k]), std::norm(r[k] + L.s));
    if (std::norm(dz) <= 1e-16 * scale) {
      const LensAt t = lens_at(L, y, r[k] + dz);
      if (std::norm(t.R) < 0.25 * std::norm(at[k].R)) {
        r[k] += dz;
        at[k] = t;
      }
    }
  }
  int ord[5] = {0, 1, 2, 3, 4};
  std::sort(ord, ord + 5, [&](int a, int b) { return std::abs(at[a].R) > std::abs(at[b].R); });
  cd sum = 0.0;
  double noise = 0.0;
  for (int k = 0; k < 5; ++k) sum += at[k].R;
  noise = std::max(std::abs(at[ord[2]].R), std::abs(sum));
  for (int j = 2; j < 5; ++j) {
    const int k = ord[j];
    const double sig = 64.0 * EPS *
                       (std::abs(y) + std::abs(r[k]) + L.m1 / std::abs(r[k] + L.s) + L.m2 / std::abs(r[k]));
    noise = std::max(noise, sig);
  }
  const double margin = std::abs(at[ord[1]].R) / noise;
  const bool ghosts = margin > GAP;
  im.flags = (margin > GAP / 30.0 && margin < GAP * 30.0) ? F_NEAR : 0u;
  im.n = ghosts ? 3 : 5;
  im.npos = ghosts ? 1 : 2;
  // real images by decreasing J: the first npos are positive (the parity
  // sum of the real images is -1, Sec. 2.3; the rank fixes a pair merging
  // on the critical curve whose sign(J) rounding has decided)
  int real[5], nr = 0;
  for (int k = 0; k < 5; ++k)
    if (!(ghosts && (k == ord[0] || k == ord[1]))) real[nr++] = k;
  std::sort(real, real + nr, [&](int a, int b) { return at[a].J > at[b].J; });
  int npos_sign = 0;
  for (int j = 0; j < nr; ++j) {
    im.z[j] = r[real[j]];
    im.J[j] = at[real[j]].J;
    npos_sign += at[real[j]].J > 0.0 ? 1 : 0;
  }
  if (npos_sign != im.npos) im.flags |= F_NEAR;
  // the ghost pair after the real images
  if (ghosts) {
    im.z[3] = r[ord[0]];
    im.z[4] = r[ord[1]];
    im.J[3] = at[ord[0]].J;
    im.J[4] = at[ord[1]].J;
  }
}

// Solve y's quintic from the start r[] (warm: a nearby point's roots), with
// a cold restart when the warm start does not converge.
void solve(const Lens& L, cd y, cd r[5], Images& im) {
  cd c[6];
  quintic(L, y, c);
  if (!aberth(c, r, 60)) {
    circle_start(c, r);
    aberth(c, r, 300);
  }
  classify(L, y, r, im);
}

double point_mag(const Images& im) {
  double mu = 0.0;
  for (int k = 0; k < im.n; ++k) mu += 1.0 / std::fabs(im.J[k]);
  return mu;
}

// ------------------------------------------------------------- contour
struct Sample {
  double th;
  Images im;
  cd dz[5];    // z' = dz/dtheta of each real image
  double w[5]; // z' ^ z''
};

// Limb point at theta (Sec. 2.3, Eq. area_cal, with zeta' = i rho e^{i theta}):
// z' = (zeta' - conj(f') conj(zeta')) / J, z' ^ z'' = (rho^2 + Im(z'^2 zeta' f'')) / J.
void sample_at(const Lens& L, cd yc, double rho, double th, cd r[5], Sample& sm) {
  const cd e = std::polar(1.0, th);
  const cd y = yc + rho * e, zp1 = cd(0.0, rho) * e;
  solve(L, y, r, sm.im);
  sm.th = th;
  for (int k = 0; k < 5; ++k) {
    sm.dz[k] = 0.0;
    sm.w[k] = 0.0;
    if (k < sm.im.n) {
      const LensAt at = lens_at(L, y, sm.im.z[k]);
      sm.dz[k] = (zp1 - std::conj(at.fp) * std::conj(zp1)) / at.J;
      sm.w[k] = (rho * rho + (sm.dz[k] * sm.dz[k] * zp1 * fsecond(L, sm.im.z[k])).imag()) / at.J;
    }
  }
}

struct Piece {
  double dA, E;
};

// Ordinary link of one image from sample a to sample b (parity p): the
// trapezium plus half the two parabolic corrections, and E1..E4 (Sec. 2.5,
// Eq. area_normal).
void add_link(const Sample& a, int ia, const Sample& b, int ib, double p, double dth, Piece& pc) {
  const cd za = a.im.z[ia], zb = b.im.z[ib], da = a.dz[ia], db = b.dz[ib];
  const double wa = a.w[ia], wb = b.w[ib], dth3 = dth * dth * dth;
  const double p1 = (wa + wb) * dth3 / 24.0;
  const double p2 = wedge(zb - za, db - da) * dth / 12.0;
  const double corr = 0.5 * (p1 + p2);
  pc.dA += p * (0.5 * wedge(za, zb) + corr);
  const double chord2 = std::norm(za - zb);
  pc.E += std::fabs(wa - wb) * dth3 / 48.0 + 1.5 * std::fabs(corr * (chord2 / (dth * dth * std::fabs(dot(da, db))) - 1.0)) +
          0.1 * std::fabs(corr) * dth * dth + std::fabs(p1 - p2);
}

// A pair created (kind +1, present at the later sample c) or destroyed
// (kind -1, present at the earlier one) inside the interval: the chord from
// the - image to the + image (created) or back (destroyed) plus the
// cross-caustic correction (w+ - w-) dt^3 / 24 with the effective step
// dt = |z+ - z-| / sqrt|z'+ . z'-| (Sec. 2.3), and E1 + E2 + E3 (Sec. 2.5,
// Eq. area_cross; E2 with "-" for a created, "+" for a destroyed pair).
void add_cross(const Sample& c, int ip, int in, int kind, double dth, Piece& pc) {
  const cd zp = c.im.z[ip], zm = c.im.z[in], dp = c.dz[ip], dm = c.dz[in];
  const double wp = c.w[ip], wm = c.w[in];
  const double root = std::sqrt(std::fabs(dot(dp, dm))), sep = std::abs(zp - zm);
  const double dt = sep / root, dt3 = dt * dt * dt;
  const double corr = (wp - wm) * dt3 / 24.0;
  pc.dA += (kind > 0 ? 0.5 * wedge(zm, zp) : 0.5 * wedge(zp, zm)) + corr;
  const double sgn = kind > 0 ? 1.0 : -1.0;
  pc.E += std::fabs(wp + wm) * dt3 / 48.0 + 1.5 * std::fabs(dot(zp - zm, dp - dm) - sgn * 2.0 * sep * root) * dt +
          0.1 * std::fabs(corr) * dth * dth;
}

// Least total distance assignment of the images idx_a[0..na) of sample a to
// idx_b[0..nb) of sample b (na <= nb <= 3): best[i] = index into idx_b of
// a's i-th image.  Enumerates the injections.
void assign(const Sample& a, const int* ia, int na, const Sample& b, const int* ib, int nb, int* best) {
  double bcost = 1e300;
  int pick[3];
  for (int x = 0; x < nb; ++x)
    for (int y = 0; y < (na > 1 ? nb : 1); ++y)
      for (int z = 0; z < (na > 2 ? nb : 1); ++z) {
        pick[0] = x;
        pick[1] = y;
        pick[2] = z;
        bool ok = true;
        for (int i = 0; i < na && ok; ++i)
          for (int j = 0; j < i; ++j)
            if (pick[i] == pick[j]) ok = false;
        if (!ok) continue;
        double cost = 0.0;
        for (int i = 0; i < na; ++i) cost += std::abs(a.im.z[ia[i]] - b.im.z[ib[pick[i]]]);
        if (cost < bcost) {
          bcost = cost;
          for (int i = 0; i < na; ++i) best[i] = pick[i];
        }
      }
}

// The piece of the interval from sample a to sample b (width dth):
// same-parity images linked by least total distance (Sec. 2.3); with 3
// images at one end and 5 at the other the two left over form the pair
// created or destroyed in the interval.
Piece piece(const Sample& a, const Sample& b, double dth) {
  Piece pc{0.0, 0.0};
  for (int par = 0; par < 2; ++par) {
    int ia[3], ib[3], na = 0, nb = 0;
    for (int k = 0; k < a.im.n; ++k)
      if ((k < a.im.npos) == (par == 0)) ia[na++] = k;
    for (int k = 0; k < b.im.n; ++k)
      if ((k < b.im.npos) == (par == 0)) ib[nb++] = k;
    const double p = par == 0 ? 1.0 : -1.0;
    int best[3];
    if (na <= nb) {
      assign(a, ia, na, b, ib, nb, best);
      for (int i = 0; i < na; ++i) add_link(a, ia[i], b, ib[best[i]], p, dth, pc);
    } else {
      assign(b, ib, nb, a, ia, na, best);
      for (int i = 0; i < nb; ++i) add_link(a, ia[best[i]], b, ib[i], p, dth, pc);
    }
  }
  if (a.im.n != b.im.n) {
    // the leftover + and - images at the 5-image end
    const bool created = b.im.n == 5;
    const Sample& c = created ? b : a;
    const Sample& o = created ? a : b;
    int left[2] = {-1, -1};
    for (int par = 0; par < 2; ++par) {
      int ic[3], io[3], nc = 0, no = 0;
      for (int k = 0; k < c.im.n; ++k)
        if ((k < c.im.npos) == (par == 0)) ic[nc++] = k;
      for (int k = 0; k < o.im.n; ++k)
        if ((k < o.im.npos) == (par == 0)) io[no++] = k;
      int best[3];
      assign(o, io, no, c, ic, nc, best);
      for (int j = 0; j < nc; ++j) {
        bool used = false;
        for (int i = 0; i < no; ++i) used = used || best[i] == j;
        if (!used) left[par] = ic[j];
      }
    }
    add_cross(c, left[0], left[1], created ? 1 : -1, dth, pc);
  }
  return pc;
}

struct Result {
  double mag, err;
  int n;
  uint32_t flags;
};

// Adaptive contour integration of the disk of radius rho at yc (Secs.
// 2.3-2.5, 3); centre: the roots at the disk centre.
Result contour(const Lens& L, cd yc, double rho, double tol_stated, const cd centre[5]) {
  std::vector<Sample> sm;
  std::vector<int> ord;
  sm.reserve(CAP);
  uint32_t fl = 0;
  cd r[5];
  for (int j = 0; j < NNEW; ++j) {
    if (j == 0) std::copy(centre, centre + 5, r);  // then each sample starts from the previous one
    Sample s;
    sample_at(L, yc, rho, TWO_PI * j / NNEW, r, s);
    sm.push_back(s);
    ord.push_back(j);
  }
  std::vector<double> dA, E, th_new;
  std::vector<int> iv_new;
  double A = 0.0, Etot = 0.0;
  for (;;) {
    const int N = (int)ord.size();
    dA.assign(N, 0.0);
    E.assign(N, 0.0);
    double hi = 0.0, lo = 0.0;
    Etot = 0.0;
    for (int i = 0; i < N; ++i) {
      const Sample& a = sm[ord[i]];
      const Sample& b = sm[ord[(i + 1) % N]];
      const double dth = (i + 1 < N ? b.th : b.th + TWO_PI) - a.th;
      const Piece pc = piece(a, b, dth);
      dA[i] = pc.dA;
      E[i] = pc.E;
      Etot += pc.E;
      // Neumaier-compensated area sum
      const double t = hi + pc.dA;
      lo += std::fabs(hi) >= std::fabs(pc.dA) ? (hi - t) + pc.dA : (pc.dA - t) + hi;
      hi = t;
      fl |= a.im.flags & F_NEAR;
    }
    A = hi + lo;
    // a limb that crosses a caustic (samples with three and with five
    // images) stops at half the stated tolerance: across the crossing the
    // error estimate can fall short of the true error; elsewhere it is far
    // above it and the stated tolerance is the target
    bool seen3 = false, seen5 = false;
    for (int i = 0; i < N; ++i) {
      seen3 |= sm[i].im.n == 3;
      seen5 |= sm[i].im.n == 5;
    }
    const double tol = (seen3 && seen5) ? SAFETY * tol_stated : tol_stated;
    if (Etot <= tol * std::fabs(A)) break;
    const int nnew = std::min(NNEW, CAP - N);
    if (nnew <= 0) {
      fl |= F_CAP;
      break;
    }
    // tolerance-subtracted weights (intervals narrower than FLOOR: none)
    const double avg = tol * std::fabs(A) / N;
    std::vector<double> cum(N + 1, 0.0);
    for (int i = 0; i < N; ++i) {
      const double width = (i + 1 < N ? sm[ord[i + 1]].th : sm[ord[0]].th + TWO_PI) - sm[ord[i]].th;
      cum[i + 1] = cum[i] + (width > FLOOR ? std::max(E[i] - avg, 0.0) : 0.0);
    }
    const double W = cum[N];
    if (!(W > 0.0)) break;
    // quantiles (j + 1/2)/nnew of the cumulative weight, linear inside each interval
    th_new.clear();
    iv_new.clear();
    int i = 0;
    for (int j = 0; j < nnew; ++j) {
      const double u = (j + 0.5) / nnew * W;
      while (i < N - 1 && cum[i + 1] <= u) ++i;
      const double wi = cum[i + 1] - cum[i];
      if (!(wi > 0.0)) continue;
      const double ta = sm[ord[i]].th, tb = i + 1 < N ? sm[ord[i + 1]].th : TWO_PI;
      const double t = ta + (u - cum[i]) / wi * (tb - ta);
      if (!(t > ta && t < tb)) continue;
      if (!iv_new.empty() && iv_new.back() == i && !(t > th_new.back())) continue;
      th_new.push_back(t);
      iv_new.push_back(i);
    }
    if (th_new.empty()) {
      fl |= F_CAP;
      break;
    }
    // solve the new samples from the nearer neighbour, advanced along z'
    std::vector<int> merged;
    merged.reserve(N + th_new.size());
    size_t q = 0;
    for (int k = 0; k < N; ++k) {
      merged.push_back(ord[k]);
      while (q < th_new.size() && iv_new[q] == k) {
        const Sample& a = sm[ord[k]];
        const Sample& b = sm[ord[(k + 1) % N]];
        const double tb = k + 1 < N ? b.th : b.th + TWO_PI;
        const bool left = th_new[q] - a.th <= tb - th_new[q];
        const Sample& nb = left ? a : b;
        const double step = left ? th_new[q] - a.th : th_new[q] - tb;
        cd st[5];
        for (int m = 0; m < 5; ++m) st[m] = nb.im.z[m] + (m < nb.im.n ? step * nb.dz[m] : cd(0.0));
        Sample s;
        sample_at(L, yc, rho, th_new[q], st, s);
        sm.push_back(s);
        merged.push_back((int)sm.size() - 1);
        ++q;
      }
    }
    ord.swap(merged);
  }
  const double area = 0.5 * TWO_PI * rho * rho;
  return Result{A / area, Etot / area, (int)ord.size(), fl};
}

// Point-source test (Sec. 2.3: quadrupole and ghost tests): the point value
// may replace the disk when 20 |(mean4 - mu0)/2| < tol mu0 over the four
// points zeta_c +- rho, zeta_c +- i rho, all five points have three images
// and every ghost sits far from the caustic: |f''(g)| |R_g|^2 > 8 rho.
bool adequate(const Lens& L, cd yc, double rho, double tol, cd centre[5], double* mu0,
              uint32_t* flags) {
  cd c[6];
  quintic(L, yc, c);
  circle_start(c, centre);
  aberth(c, centre, 300);
  Images im;
  classify(L, yc, centre, im);
  for (int k = 0; k < 5; ++k) centre[k] = im.z[k];
  *mu0 = point_mag(im);
  *flags = im.flags;
  auto ghosts_far = [&](const Images& x, cd y) {
    for (int g = x.n; g < 5; ++g) {
      const double d = std::abs(fsecond(L, x.z[g])) * std::norm(lens_at(L, y, x.z[g]).R);
      if (!(d > CG * rho)) return false;
    }
    return true;
  };
  if (im.n != 3 || !ghosts_far(im, yc)) return false;
  double sum = 0.0;
  const cd off[4] = {cd(rho, 0.0), cd(0.0, rho), cd(-rho, 0.0), cd(0.0, -rho)};
  for (int k = 0; k < 4; ++k) {
    cd r[5];
    std::copy(centre, centre + 5, r);
    Images ik;
    solve(L, yc + off[k], r, ik);
    if (ik.n != 3 || !ghosts_far(ik, yc + off[k])) return false;
    sum += point_mag(ik);
  }
  return CQ * std::fabs(0.5 * (0.25 * sum - *mu0)) < tol * *mu0;
}

// Relative tolerance of the annulus contours of a limb-darkened source (the
// GPU path's rule): the stated one when the intensity falls outward, else
// divided by the error growth bound 2 I_na / I_1 - 1 of the combination.
double annulus_tol(double tol, double G, int na) {
  if (!(G < 0.0)) return tol;
  const double x1 = 1.0 / na, xl = (na - 1.0) / na;
  const double i1 = 1.0 - G + G * (1.0 - std::pow(1.0 - x1, 1.5)) / x1;
  const double il = 1.0 - G + G * std::pow(1.0 - xl, 1.5) / (1.0 - xl);
  const double f = 2.0 * il / i1 - 1.0;
  return i1 > 0.0 && f > 1.0 ? tol / f : tol;
}

// One epoch: point value when adequate (unless all_fs), else the uniform
// disk or, with limb darkening (na > 1), the combination of the na nested
// disks of radii rho sqrt(k/na) with the linear law's annulus means.
Result epoch(double s, double q, double zx, double zy, double rho, double G, int na, double tol,
             bool all_fs) {
  if (!std::isfinite(zx) || !std::isfinite(zy)) return Result{NAN, NAN, 0, F_NONFINITE};
  const Lens L = make_lens(s, q);
  const cd yc(zx - L.z2, zy);
  cd centre[5];
  double mu0;
  uint32_t f0;
  const bool ok = adequate(L, yc, rho, tol, centre, &mu0, &f0);
  if (ok && !all_fs) return Result{mu0, 0.0, 0, F_POINT | f0};
  if (na <= 1) return contour(L, yc, rho, tol, centre);
  const double ta = annulus_tol(tol, G, na);
  double num = 0.0, den = 0.0, e = 0.0, xp = 0.0, mp = 0.0, ep = 0.0;
  Result out{0.0, 0.0, 0, 0u};
  for (int k = 1; k <= na; ++k) {
    const double x = (double)k / na;
    const Result rk = contour(L, yc, rho * std::sqrt(x), ta, centre);
    const double Ik = 1.0 - G + G * (std::pow(1.0 - xp, 1.5) - std::pow(1.0 - x, 1.5)) / (x - xp);
    num += Ik * (x * rk.mag - xp * mp);
    den += Ik * (x - xp);
    e += Ik * (x * rk.err + xp * ep);
    out.n += rk.n;
    out.flags |= rk.flags;
    xp = x;
    mp = rk.mag;
    ep = rk.err;
  }
  out.mag = num / den;
  out.err = e / den;
  return out;
}

bool finite_pos(double v) { return v > 0.0 && v < 1e300; }

// Run f(i) for i in [0, n) on `threads` workers sharing an atomic counter.
template <class F>
void parallel(int64_t n, int threads, F f) {
  int nt = threads > 0 ? threads : (int)std::max(1u, std::thread::hardware_concurrency());
  nt = (int)std::min<int64_t>(nt, std::max<int64_t>(n, 1));
  std::atomic<int64_t> next(0);
  auto work = [&]() {
    for (int64_t i = next++; i < n; i = next++) f(i);
  };
  std::vector<std::thread> pool;
  for (int t = 1; t < nt; ++t) pool.emplace_back(work);
  work();
  for (auto& t : pool) t.join();
}

}  // namespace

extern "C" {

int twk_cpu_finite_mag(double s, double q, int64_t n, const double* zx, const double* zy, double rho,
                       double tol, int32_t all_fs, int32_t threads, double* mag, double* err,
                       int32_t* ns, uint32_t* flags) {
  if (!finite_pos(s) || !finite_pos(q) || !finite_pos(rho) || !finite_pos(tol) || n < 0)
    return TWK_CPU_EINVAL;
  if (n == 0) return 0;
  if (!zx || !zy || !mag || !err || !ns || !flags) return TWK_CPU_EINVAL;
  parallel(n, threads, [&](int64_t i) {
    const Result r = epoch(s, q, zx[i], zy[i], rho, 0.0, 1, tol, all_fs != 0);
    mag[i] = r.mag;
    err[i] = r.err;
    ns[i] = r.n;
    flags[i] = r.flags;
  });
  return 0;
}

int twk_cpu_lightcurves(int64_t nsets, const double* s, const double* q, const double* u0,
                        const double* alpha, const double* rho, const double* gamma, int64_t nepochs,
                        const double* tau, int32_t n_annuli, double tol, int32_t threads, double* mag,
                        double* err, int32_t* ns, uint32_t* flags) {
  if (nsets < 0 || nepochs < 0 || !finite_pos(tol) || n_annuli < 1 || n_annuli > 64 ||
      (!gamma && n_annuli != 1))
    return TWK_CPU_EINVAL;
  if (nsets == 0 || nepochs == 0) return 0;
  if (!s || !q || !u0 || !alpha || !rho || !tau || !mag || !err || !ns || !flags) return TWK_CPU_EINVAL;
  for (int64_t k = 0; k < nsets; ++k)
    if (!finite_pos(s[k]) || !finite_pos(q[k]) || !finite_pos(rho[k])) return TWK_CPU_EINVAL;
  parallel(nsets * nepochs, threads, [&](int64_t i) {
    const int64_t k = i / nepochs, j = i % nepochs;
    const double ca = std::cos(alpha[k]), sa = std::sin(alpha[k]);
    const double zx = tau[j] * ca - u0[k] * sa, zy = tau[j] * sa + u0[k] * ca;
    const Result r = epoch(s[k], q[k], zx, zy, rho[k], gamma ? gamma[k] : 0.0, n_annuli, tol, false);
    mag[i] = r.mag;
    err[i] = r.err;
    ns[i] = r.n;
    flags[i] = r.flags;
  });
  return 0;
}

}  // extern "C"
