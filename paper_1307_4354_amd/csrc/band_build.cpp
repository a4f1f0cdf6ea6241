// Host construction of the computational band and its addressing (Sec. 3.1, Sec. 4.3).
//
// Compiled without floating-point contraction: every closest point, distance and stencil
// fraction is the IEEE double result of the operations below, in this order.  This fixed
// order is the convention that makes band membership and stencil bases reproducible
// bit for bit by any independent implementation that follows it.
//
// Band of level l (spacing h): nodes x = h * i with dist(x, S)^2 <= lam2 * (h * h),
// lam2 = 13 (2-D) or 17 (3-D) by default, i.e. radius sqrt(13) h / sqrt(17) h, wide enough
// to contain B_interp and B_edge of the cubic scheme.  Nodes are sorted x fastest.
#include <algorithm>
#include <cmath>
#include <limits>
#include <climits>
#include <cstdlib>
#include <cstring>
#include <omp.h>
#include <sstream>

#include "cpm_internal.h"

namespace cpm {
namespace {

// Closest point and squared distance (Sec. 2.1) for the analytic surfaces.  Ties resolve
// onto the surface: centre -> direction +x; torus axis -> radial direction +x; torus
// tube-centre circle -> outward radial direction.
// ---- level set: Dziuk's surface (y1 - y3^2)^2 + y2^2 + y3^2 = 1 -------------------------
// Closest point by Newton's method on the stationarity conditions of |y - x|^2 under
// phi(y) = 0 (the level-set example, Sec. 4.6.5, minimises the squared distance with
// Newton's method), F = (y - x + mu grad(phi), phi), J = [[I + mu Hess(phi), g], [g^T, 0]];
// the 3x3 block couples y1 and y3 only, so a step is solved in closed form.  The start is
// the nearest of 6 K^2 surface samples (a global start: the coarse bands reach beyond the
// surface's reach, where a local start can end at a stationary point that is not the
// closest point and leave holes in the band).  A node that provably has no surface point
// within the band radius is skipped (Lipschitz bound of phi on the ball); a node whose
// iteration does not converge, or ends farther than its start, keeps the start sample.
// Plain IEEE double operations in exactly this order (no contraction): the band is then
// identical to the one the float64 reference computes.
constexpr int kDziukK = 16;
constexpr int kDziukNewton = 25;

const std::vector<double>& dziuk_samples() {
  static const std::vector<double> S = [] {
    std::vector<double> out;
    out.reserve((size_t)6 * kDziukK * kDziukK * 3);
    double t[kDziukK];
    for (int i = 0; i < kDziukK; ++i) t[i] = (2.0 * (double)i + 1.0) / (double)kDziukK - 1.0;
    for (int face = 0; face < 6; ++face)
      for (int i = 0; i < kDziukK; ++i)
        for (int j = 0; j < kDziukK; ++j) {
          const double u = t[i], v = t[j];
          double P[3];
          switch (face) {
            case 0: P[0] = 1.0; P[1] = u; P[2] = v; break;
            case 1: P[0] = -1.0; P[1] = u; P[2] = v; break;
            case 2: P[0] = u; P[1] = 1.0; P[2] = v; break;
            case 3: P[0] = u; P[1] = -1.0; P[2] = v; break;
            case 4: P[0] = u; P[1] = v; P[2] = 1.0; break;
            default: P[0] = u; P[1] = v; P[2] = -1.0; break;
          }
          const double r = std::sqrt((P[0] * P[0] + P[1] * P[1]) + P[2] * P[2]);
          const double q0 = P[0] / r, q1 = P[1] / r, q2 = P[2] / r;
          out.push_back(q0 + q2 * q2);
          out.push_back(q1);
          out.push_back(q2);
        }
    return out;
  }();
  return S;
}

// x relative to the surface centre; returns false when x is provably farther than sqrt(thr)
bool dziuk_closest(const double* x, double thr, double* cp, double* dist2) {
  const double x1 = x[0], x2 = x[1], x3 = x[2];
  const double p0 = x1 - x3 * x3;
  const double ph0 = (p0 * p0 + x2 * x2) + (x3 * x3 - 1.0);
  const double r = std::sqrt(thr);
  const double ax3 = std::fabs(x3);
  const double P = ((std::fabs(p0) + r) + (2.0 * ax3) * r) + r * r;
  const double Y2 = std::fabs(x2) + r;
  const double Y3 = ax3 + r;
  const double q = 2.0 + 4.0 * P;
  const double G2 = (4.0 * (P * P) + 4.0 * (Y2 * Y2)) + (Y3 * Y3) * (q * q);
  if (!(ph0 * ph0 <= G2 * thr)) return false;
  const std::vector<double>& S = dziuk_samples();
  const size_t M = S.size() / 3;
  size_t best = 0;
  double bd = 0.0;
  for (size_t k = 0; k < M; ++k) {
    const double d0 = S[3 * k] - x1, d1 = S[3 * k + 1] - x2, d2 = S[3 * k + 2] - x3;
    const double d = (d0 * d0 + d1 * d1) + d2 * d2;
    if (k == 0 || d < bd) {
      bd = d;
      best = k;
    }
  }
  const double s1 = S[3 * best], s2 = S[3 * best + 1], s3 = S[3 * best + 2];
  double y1 = s1, y2 = s2, y3 = s3;
  double p = y1 - y3 * y3;
  double g1 = 2.0 * p, g2 = 2.0 * y2, g3 = 2.0 * y3 - 4.0 * y3 * p;
  double gg = (g1 * g1 + g2 * g2) + g3 * g3;
  double mu = (((x1 - y1) * g1 + (x2 - y2) * g2) + (x3 - y3) * g3) / gg;
  for (int it = 0; it < kDziukNewton; ++it) {
    p = y1 - y3 * y3;
    g1 = 2.0 * p;
    g2 = 2.0 * y2;
    g3 = 2.0 * y3 - 4.0 * y3 * p;
    const double ph = (p * p + y2 * y2) + (y3 * y3 - 1.0);
    const double F1 = (y1 - x1) + mu * g1;
    const double F2 = (y2 - x2) + mu * g2;
    const double F3 = (y3 - x3) + mu * g3;
    const double h33 = (2.0 - 4.0 * p) + 8.0 * (y3 * y3);
    const double a = 1.0 + 2.0 * mu;
    const double b = (-4.0 * mu) * y3;
    const double d = 1.0 + mu * h33;
    const double det = a * d - b * b;
    const double kf1 = (d * F1 - b * F3) / det;
    const double kf3 = (a * F3 - b * F1) / det;
    const double kf2 = F2 / a;
    const double kg1 = (d * g1 - b * g3) / det;
    const double kg3 = (a * g3 - b * g1) / det;
    const double kg2 = g2 / a;
    const double gkf = (g1 * kf1 + g2 * kf2) + g3 * kf3;
    const double gkg = (g1 * kg1 + g2 * kg2) + g3 * kg3;
    const double dmu = (ph - gkf) / gkg;
    y1 = y1 - (kf1 + kg1 * dmu);
    y2 = y2 - (kf2 + kg2 * dmu);
    y3 = y3 - (kf3 + kg3 * dmu);
    mu = mu + dmu;
  }
  p = y1 - y3 * y3;
  const double ph = (p * p + y2 * y2) + (y3 * y3 - 1.0);
  const double r1 = (y1 - x1) + mu * (2.0 * p);
  const double r2 = (y2 - x2) + mu * (2.0 * y2);
  const double r3 = (y3 - x3) + mu * (2.0 * y3 - 4.0 * y3 * p);
  const double e1 = y1 - x1, e2 = y2 - x2, e3 = y3 - x3;
  const double dn = (e1 * e1 + e2 * e2) + e3 * e3;
  const bool conv = std::fabs(ph) <= 1e-12 && std::fabs(r1) <= 1e-12 && std::fabs(r2) <= 1e-12 &&
                    std::fabs(r3) <= 1e-12;
  const double f1 = s1 - x1, f2 = s2 - x2, f3 = s3 - x3;
  const double ds = (f1 * f1 + f2 * f2) + f3 * f3;
  if (conv && dn <= ds) {
    cp[0] = y1;
    cp[1] = y2;
    cp[2] = y3;
    *dist2 = dn;
  } else {
    cp[0] = s1;
    cp[1] = s2;
    cp[2] = s3;
    *dist2 = ds;
  }
  return true;
}

// thr: squared band radius (used by the level set to skip far points and as the Newton
// filter; the analytic surfaces ignore it)
inline void closest_point(const cpm_surface& s, int dim, const double* x, double* cp,
                          double* dist2, double thr) {
  const double* c = s.center;
  if (s.kind == CPM_DZIUK) {
    const double xr[3] = {x[0] - c[0], x[1] - c[1], x[2] - c[2]};
    double y[3];
    if (!dziuk_closest(xr, thr, y, dist2)) {
      *dist2 = std::numeric_limits<double>::infinity();
      cp[0] = x[0];
      cp[1] = x[1];
      cp[2] = x[2];
      return;
    }
    cp[0] = y[0] + c[0];
    cp[1] = y[1] + c[1];
    cp[2] = y[2] + c[2];
    return;
  }
  if (s.kind == CPM_CIRCLE || s.kind == CPM_SPHERE) {
    double dx = x[0] - c[0];
    double dy = x[1] - c[1];
    double dz = dim == 3 ? x[2] - c[2] : 0.0;
    double rho2;
    if (dim == 2) {
      double a = dx * dx;
      double b = dy * dy;
      rho2 = a + b;
    } else {
      double a = dx * dx;
      double b = dy * dy;
      double ab = a + b;
      double cz = dz * dz;
      rho2 = ab + cz;
    }
    double rho = std::sqrt(rho2);
    double nx, ny, nz;
    if (rho == 0.0) {
      nx = 1.0;
      ny = 0.0;
      nz = 0.0;
    } else {
      nx = dx / rho;
      ny = dy / rho;
      nz = dz / rho;
    }
    double t;
    t = s.R * nx;
    cp[0] = c[0] + t;
    t = s.R * ny;
    cp[1] = c[1] + t;
    if (dim == 3) {
      t = s.R * nz;
      cp[2] = c[2] + t;
    }
    double d = rho - s.R;
    *dist2 = d * d;
    return;
  }
  // torus, axis along z
  double dx = x[0] - c[0];
  double dy = x[1] - c[1];
  double dz = x[2] - c[2];
  double a2 = dx * dx;
  double b2 = dy * dy;
  double rho = std::sqrt(a2 + b2);
  double ex, ey;
  if (rho == 0.0) {
    ex = 1.0;
    ey = 0.0;
  } else {
    ex = dx / rho;
    ey = dy / rho;
  }
  double a = rho - s.R;
  double b = dz;
  double aa = a * a;
  double bb = b * b;
  double t = std::sqrt(aa + bb);
  double na, nb;
  if (t == 0.0) {
    na = 1.0;
    nb = 0.0;
  } else {
    na = a / t;
    nb = b / t;
  }
  double rna = s.r * na;
  double rad = s.R + rna;
  double px = rad * ex;
  double py = rad * ey;
  double pz = s.r * nb;
  cp[0] = c[0] + px;
  cp[1] = c[1] + py;
  cp[2] = c[2] + pz;
  double d = t - s.r;
  *dist2 = d * d;
}

void bounding_box(const cpm_surface& s, int dim, double lo[3], double hi[3]) {
  if (s.kind == CPM_DZIUK) {
    // x1 = x3^2 +- sqrt(1 - x2^2 - x3^2) lies in [-1, 5/4]; |x2|, |x3| <= 1
    const double l[3] = {-1.0, -1.0, -1.0}, u[3] = {1.25, 1.0, 1.0};
    for (int a = 0; a < 3; ++a) {
      lo[a] = s.center[a] + l[a];
      hi[a] = s.center[a] + u[a];
    }
    return;
  }
  double ext[3];
  if (s.kind == CPM_TORUS) {
    ext[0] = ext[1] = s.R + s.r;
    ext[2] = s.r;
  } else {
    ext[0] = ext[1] = ext[2] = s.R;
  }
  for (int a = 0; a < dim; ++a) {
    lo[a] = s.center[a] - ext[a];
    hi[a] = s.center[a] + ext[a];
  }
}

inline int64_t box_key(const HostLevel& L, int64_t x, int64_t y, int64_t z) {
  int64_t rx = x - L.lo[0], ry = y - L.lo[1], rz = z - L.lo[2];
  if (rx < 0 || ry < 0 || rz < 0 || rx >= L.ext[0] || ry >= L.ext[1] || rz >= L.ext[2]) return -1;
  return (rz * L.ext[1] + ry) * L.ext[0] + rx;
}

inline int32_t lookup(const HostLevel& L, int64_t x, int64_t y, int64_t z) {
  int64_t k = box_key(L, x, y, z);
  return k < 0 ? -1 : L.map[k];
}

// Enumerate the band of one level; nodes come out sorted (z, y, x with x fastest).
cpm_status enumerate_level(const cpm_surface& s, int dim, double h, double lam2, HostLevel& L,
                           std::string& err) {
  L.dim = dim;
  L.h = h;
  L.lam2 = lam2;
  double lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
  bounding_box(s, dim, lo, hi);
  double lam = std::sqrt(lam2);
  for (int a = 0; a < 3; ++a) {
    if (a < dim) {
      L.lo[a] = (int64_t)std::floor((lo[a] - lam * h) / h) - 2;
      int64_t ihi = (int64_t)std::ceil((hi[a] + lam * h) / h) + 2;
      L.ext[a] = ihi - L.lo[a] + 1;
    } else {
      L.lo[a] = 0;
      L.ext[a] = 1;
    }
  }
  double box = (double)L.ext[0] * (double)L.ext[1] * (double)L.ext[2];
  if (box > 2.0e9) {
    err = "index box too large for the dense lookup map";
    return CPM_E_INVALID;
  }
  const double thr = lam2 * (h * h);
  const int64_t nz = L.ext[2];
  std::vector<std::vector<int32_t>> planes((size_t)nz);
  std::vector<std::vector<double>> pcp((size_t)nz);
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t kz = 0; kz < nz; ++kz) {
    int64_t z = L.lo[2] + kz;
    std::vector<int32_t>& P = planes[(size_t)kz];
    std::vector<double>& C = pcp[(size_t)kz];
    double x[3], cp[3], d2;
    for (int64_t y = L.lo[1]; y < L.lo[1] + L.ext[1]; ++y) {
      for (int64_t xi = L.lo[0]; xi < L.lo[0] + L.ext[0]; ++xi) {
        x[0] = (double)xi * h;
        x[1] = (double)y * h;
        x[2] = (double)z * h;
        closest_point(s, dim, x, cp, &d2, thr);
        if (d2 <= thr) {
          P.push_back((int32_t)xi);
          P.push_back((int32_t)y);
          if (dim == 3) P.push_back((int32_t)z);
          for (int a = 0; a < dim; ++a) C.push_back(cp[a]);
        }
      }
    }
  }
  int64_t n = 0;
  for (auto& P : planes) n += (int64_t)P.size() / dim;
  if (n <= 0 || n > INT32_MAX / 2) {
    err = n <= 0 ? "empty band" : "band too large for 32-bit indices";
    return CPM_E_INVALID;
  }
  L.n = n;
  L.idx.resize((size_t)(n * dim));
  L.cp.resize((size_t)(n * dim));
  size_t off = 0;
  for (int64_t kz = 0; kz < nz; ++kz) {
    auto& P = planes[(size_t)kz];
    auto& C = pcp[(size_t)kz];
    if (!P.empty()) {
      std::memcpy(&L.idx[off], P.data(), P.size() * sizeof(int32_t));
      std::memcpy(&L.cp[off], C.data(), C.size() * sizeof(double));
      off += P.size();
    }
    std::vector<int32_t>().swap(P);
    std::vector<double>().swap(C);
  }
  L.map.assign((size_t)(L.ext[0] * L.ext[1] * L.ext[2]), -1);
#pragma omp parallel for
  for (int64_t i = 0; i < n; ++i) {
    const int32_t* m = &L.idx[(size_t)(i * dim)];
    int64_t k = box_key(L, m[0], m[1], dim == 3 ? m[2] : 0);
    L.map[(size_t)k] = (int32_t)i;
  }
  return CPM_OK;
}

// Stencil of a point y on a grid of spacing h, degree p in {1, 3}: per axis
// t = y / h, base = floor(t) - (p - 1) / 2, frac = t - floor(t).
inline void stencil_base(const double* y, int dim, double h, int p, int64_t* base, double* frac) {
  for (int a = 0; a < dim; ++a) {
    double t = y[a] / h;
    double fl = std::floor(t);
    frac[a] = t - fl;
    base[a] = (int64_t)fl - (p - 1) / 2;
  }
}

// Fill x-run starts of a (p+1)^dim stencil of each node's closest point in `target`.
// runs[(b + (p+1) c) * n + i] = band index of node (bx, by + b, bz + c) of target, and the
// p following nodes along x must be the next band entries.
bool stencil_runs(const HostLevel& src, const HostLevel& target, int p, std::vector<int32_t>& runs,
                  std::vector<double>& frac, int64_t* bad_node) {
  const int dim = src.dim;
  const int64_t n = src.n;
  const int q = p + 1;
  const int nruns = dim == 2 ? q : q * q;
  runs.assign((size_t)(nruns * n), -1);
  frac.assign((size_t)(dim * n), 0.0);
  int64_t bad = -1;
#pragma omp parallel for
  for (int64_t i = 0; i < n; ++i) {
    int64_t base[3] = {0, 0, 0};
    double fr[3] = {0, 0, 0};
    stencil_base(&src.cp[(size_t)(i * dim)], dim, target.h, p, base, fr);
    for (int a = 0; a < dim; ++a) frac[(size_t)(a * n + i)] = fr[a];
    bool ok = true;
    for (int r = 0; r < nruns && ok; ++r) {
      int b = r % q, c = r / q;
      int64_t y = base[1] + b;
      int64_t z = dim == 3 ? base[2] + c : 0;
      int32_t j = lookup(target, base[0], y, z);
      if (j < 0) {
        ok = false;
        break;
      }
      for (int a = 1; a <= p; ++a) {
        if (lookup(target, base[0] + a, y, z) != j + a) {
          ok = false;
          break;
        }
      }
      runs[(size_t)(r * n + i)] = j;
    }
    if (!ok) {
#pragma omp critical
      if (bad < 0 || i < bad) bad = i;
    }
  }
  *bad_node = bad;
  return bad < 0;
}

// One workgroup's staged set: the [start, end) intervals of band indices that its rows read,
// merged into segments laid out one after another in LDS.  lds_of(x) is the LDS offset of
// band index x, which must lie in one of the intervals.
struct StageSet {
  std::vector<int32_t> seg_g, seg_e, seg_l;
  int32_t size = 0;
  void build(std::vector<std::pair<int32_t, int32_t>>& iv) {
    std::sort(iv.begin(), iv.end());
    seg_g.clear();
    seg_e.clear();
    seg_l.clear();
    size = 0;
    for (auto& v : iv) {
      if (!seg_g.empty() && v.first <= seg_e.back()) {
        if (v.second > seg_e.back()) {
          size += v.second - seg_e.back();
          seg_e.back() = v.second;
        }
      } else {
        seg_g.push_back(v.first);
        seg_e.push_back(v.second);
        seg_l.push_back(size);
        size += v.second - v.first;
      }
    }
  }
  void append_indices(std::vector<int32_t>& gidx) const {
    for (size_t j = 0; j < seg_g.size(); ++j)
      for (int32_t x = seg_g[j]; x < seg_e[j]; ++x) gidx.push_back(x);
  }
  // LDS offset that band index o maps to, o + lo being a staged index (segments are sorted
  // and disjoint)
  int32_t lds_of(int32_t o, int32_t lo) const {
    const size_t j = (size_t)(std::upper_bound(seg_g.begin(), seg_g.end(), o + lo) - seg_g.begin()) - 1;
    return seg_l[j] + (o - seg_g[j]);
  }
};

// LDS staging tables of the extension over a list of ns stencil slots (packed per slot,
// the level's group origins), for workgroups of kExtBlock * npt consecutive slots: the staged
// band indices and, per local group, the LDS offset of each x-run for x-offset 0 (the
// extension part of build_lds_tables, on an arbitrary slot list).
static void stage_slot_list(int64_t ns, const std::vector<int32_t>& packed, const std::vector<int32_t>& origin,
                            int S, int npt, std::vector<int32_t>& blkE, std::vector<int32_t>& gidx,
                            std::vector<int32_t>& blkG, std::vector<int32_t>& lorg, std::vector<int32_t>& packedL,
                            int32_t& maxE, int32_t& maxG);

// LDS staging tables of the extension (see HostLevel): for every workgroup of kExtBlock *
// extNpt consecutive stencil slots, merge the x-runs its nodes read into segments of consecutive
// band indices, lay the segments out one after another in LDS and record, per local group
// (a group cut at the workgroup boundary), where each x-run starts in LDS.  Levels with the
// fused-sweep addressing also get the fused sweep's tables on the same workgroups: rows
// widened by one node on each side in x, plus the cross rows.
void build_lds_tables(HostLevel& Lv, int S, int SX) {
  const int64_t n = Lv.n;
  bool sweep = Lv.fusedOK && !Lv.originX.empty();
  // slots per workgroup: 2 per thread on the largest levels (where the fused sweep, which
  // keeps one per thread, has no tables); CPM_EXT_NPT = 1, 2 or 4 overrides, and a value above
  // 1 drops the fused sweep's LDS tables (that pass then takes its gather form)
  int npt = !sweep && n >= kExtNptMinNodes ? 2 : 1;
  if (const char* e = std::getenv("CPM_EXT_NPT")) {
    const int v = std::atoi(e);
    if (v == 1 || v == 2 || v == 4) npt = v;
    if (npt > 1) sweep = false;
  }
  Lv.extNpt = npt;
  const int64_t wg = (int64_t)kExtBlock * npt;
  const int64_t nb = (n + wg - 1) / wg;
  const int32_t xmask = (1 << kXoffBits) - 1;
  Lv.blkE.assign((size_t)nb + 1, 0);
  Lv.blkG.assign((size_t)nb + 1, 0);
  Lv.gidx.clear();
  Lv.lorg.clear();
  Lv.packedL.assign((size_t)n, 0);
  Lv.maxE = 0;
  Lv.maxG = 0;
  Lv.blkE2.assign(sweep ? (size_t)nb + 1 : 0, 0);
  Lv.gidx2.clear();
  Lv.lorg2.clear();
  Lv.maxE2 = 0;
  std::vector<std::pair<int32_t, int32_t>> iv;  // [start, end) intervals of band indices
  StageSet set2;
  for (int64_t b = 0; b < nb; ++b) {
    const int64_t k0 = b * wg, k1 = std::min<int64_t>(n, k0 + wg);
    // local groups: runs of equal global group id
    std::vector<int64_t> lg_first;
    std::vector<int32_t> lg_gid, lg_xmin, lg_xmax;
    for (int64_t k = k0; k < k1; ++k) {
      const int32_t gid = Lv.packed[(size_t)k] >> kXoffBits, xo = Lv.packed[(size_t)k] & xmask;
      if (lg_gid.empty() || lg_gid.back() != gid) {
        lg_first.push_back(k);
        lg_gid.push_back(gid);
        lg_xmin.push_back(xo);
        lg_xmax.push_back(xo);
      } else {
        lg_xmin.back() = std::min(lg_xmin.back(), xo);
        lg_xmax.back() = std::max(lg_xmax.back(), xo);
      }
      Lv.packedL[(size_t)k] = (int32_t)(((lg_gid.size() - 1) << kXoffBits) | (size_t)xo);
    }
    iv.clear();
    for (size_t q = 0; q < lg_gid.size(); ++q)
      for (int s = 0; s < S; ++s) {
        const int32_t o = Lv.origin[(size_t)lg_gid[q] * S + s];
        iv.emplace_back(o + lg_xmin[q], o + lg_xmax[q] + 4);
      }
    std::sort(iv.begin(), iv.end());
    // merge into segments; seg_g[j], seg_l[j] = band start and LDS offset of segment j
    std::vector<int32_t> seg_g, seg_e, seg_l;
    int32_t off = 0;
    for (auto& v : iv) {
      if (!seg_g.empty() && v.first <= seg_e.back()) {
        if (v.second > seg_e.back()) {
          off += v.second - seg_e.back();
          seg_e.back() = v.second;
        }
      } else {
        seg_g.push_back(v.first);
        seg_e.push_back(v.second);
        seg_l.push_back(off);
        off += v.second - v.first;
      }
    }
    for (size_t j = 0; j < seg_g.size(); ++j)
      for (int32_t x = seg_g[j]; x < seg_e[j]; ++x) Lv.gidx.push_back(x);
    for (size_t q = 0; q < lg_gid.size(); ++q)
      for (int s = 0; s < S; ++s) {
        const int32_t o = Lv.origin[(size_t)lg_gid[q] * S + s];
        const int32_t start = o + lg_xmin[q];
        // segment containing start (segments are sorted and disjoint)
        size_t j = (size_t)(std::upper_bound(seg_g.begin(), seg_g.end(), start) - seg_g.begin()) - 1;
        Lv.lorg.push_back(seg_l[j] + (o - seg_g[j]));
      }
    Lv.blkE[(size_t)b + 1] = Lv.blkE[(size_t)b] + off;
    Lv.blkG[(size_t)b + 1] = Lv.blkG[(size_t)b] + (int32_t)lg_gid.size();
    Lv.maxE = std::max(Lv.maxE, off);
    Lv.maxG = std::max(Lv.maxG, (int32_t)lg_gid.size());
    if (!sweep) continue;
    // fused sweep: rows x0-1 .. x0+4 of every node, cross rows x0 .. x0+3
    iv.clear();
    for (size_t q = 0; q < lg_gid.size(); ++q) {
      for (int s = 0; s < S; ++s) {
        const int32_t o = Lv.origin[(size_t)lg_gid[q] * S + s];
        iv.emplace_back(o + lg_xmin[q] - 1, o + lg_xmax[q] + 5);
      }
      for (int s = 0; s < SX; ++s) {
        const int32_t o = Lv.originX[(size_t)lg_gid[q] * SX + s];
        iv.emplace_back(o + lg_xmin[q], o + lg_xmax[q] + 4);
      }
    }
    set2.build(iv);
    set2.append_indices(Lv.gidx2);
    for (size_t q = 0; q < lg_gid.size(); ++q) {
      for (int s = 0; s < S; ++s)
        Lv.lorg2.push_back(set2.lds_of(Lv.origin[(size_t)lg_gid[q] * S + s], lg_xmin[q] - 1));
      for (int s = 0; s < SX; ++s) Lv.lorg2.push_back(set2.lds_of(Lv.originX[(size_t)lg_gid[q] * SX + s], lg_xmin[q]));
    }
    Lv.blkE2[(size_t)b + 1] = Lv.blkE2[(size_t)b] + set2.size;
    Lv.maxE2 = std::max(Lv.maxE2, set2.size);
  }
}

static void stage_slot_list(int64_t ns, const std::vector<int32_t>& packed, const std::vector<int32_t>& origin,
                            int S, int npt, std::vector<int32_t>& blkE, std::vector<int32_t>& gidx,
                            std::vector<int32_t>& blkG, std::vector<int32_t>& lorg, std::vector<int32_t>& packedL,
                            int32_t& maxE, int32_t& maxG) {
  const int64_t wg = (int64_t)kExtBlock * npt, nb = (ns + wg - 1) / wg;
  const int32_t xmask = (1 << kXoffBits) - 1;
  blkE.assign((size_t)nb + 1, 0);
  blkG.assign((size_t)nb + 1, 0);
  gidx.clear();
  lorg.clear();
  packedL.assign((size_t)ns, 0);
  maxE = 0;
  maxG = 0;
  std::vector<std::pair<int32_t, int32_t>> iv;
  std::vector<int32_t> lg_gid, lg_xmin, lg_xmax;
  StageSet set;
  for (int64_t b = 0; b < nb; ++b) {
    const int64_t k0 = b * wg, k1 = std::min<int64_t>(ns, k0 + wg);
    lg_gid.clear();
    lg_xmin.clear();
    lg_xmax.clear();
    for (int64_t k = k0; k < k1; ++k) {
      const int32_t gid = packed[(size_t)k] >> kXoffBits, xo = packed[(size_t)k] & xmask;
      if (lg_gid.empty() || lg_gid.back() != gid) {
        lg_gid.push_back(gid);
        lg_xmin.push_back(xo);
        lg_xmax.push_back(xo);
      } else {
        lg_xmin.back() = std::min(lg_xmin.back(), xo);
        lg_xmax.back() = std::max(lg_xmax.back(), xo);
      }
      packedL[(size_t)k] = (int32_t)(((lg_gid.size() - 1) << kXoffBits) | (size_t)xo);
    }
    iv.clear();
    for (size_t q = 0; q < lg_gid.size(); ++q)
      for (int s = 0; s < S; ++s) {
        const int32_t o = origin[(size_t)lg_gid[q] * S + s];
        iv.emplace_back(o + lg_xmin[q], o + lg_xmax[q] + 4);
      }
    set.build(iv);
    set.append_indices(gidx);
    for (size_t q = 0; q < lg_gid.size(); ++q)
      for (int s = 0; s < S; ++s) lorg.push_back(set.lds_of(origin[(size_t)lg_gid[q] * S + s], lg_xmin[q]));
    blkE[(size_t)b + 1] = blkE[(size_t)b] + set.size;
    blkG[(size_t)b + 1] = blkG[(size_t)b] + (int32_t)lg_gid.size();
    maxE = std::max(maxE, set.size);
    maxG = std::max(maxG, (int32_t)lg_gid.size());
  }
}

// The residual-for-restriction subset of fine level F (see HostLevel::rsN): the fine nodes that
// the linear restriction stencils of coarse level C read, in F's stencil order, with F's
// groups, and their staging tables.  CPM_RESID_SUBSET=0 leaves it empty.
static void build_resid_subset(HostLevel& F, const HostLevel& C) {
  F.rsN = 0;
  std::vector<int32_t>().swap(F.rsPerm);
  std::vector<int32_t>().swap(F.rsPackedL);
  std::vector<double>().swap(F.rsFrac);
  if (const char* e = std::getenv("CPM_RESID_SUBSET"))
    if (std::strcmp(e, "0") == 0) return;
  if (F.blkE.empty() || F.perm.empty()) return;
  const int dim = F.dim, S = dim == 2 ? 4 : 16, nr = 1 << (dim - 1);
  const int64_t n = F.n, nc = C.n;
  std::vector<uint8_t> need((size_t)n, 0);
  for (int r = 0; r < nr; ++r)
    for (int64_t j = 0; j < nc; ++j) {
      const int32_t a = C.runR[(size_t)(r * nc + j)];
      need[(size_t)a] = 1;
      need[(size_t)a + 1] = 1;
    }
  std::vector<int32_t> packed;
  for (int64_t k = 0; k < n; ++k) {
    const int32_t i = F.perm[(size_t)k];
    if (!need[(size_t)i]) continue;
    F.rsPerm.push_back(i);
    packed.push_back(F.packed[(size_t)k]);
  }
  const int64_t ns = (int64_t)F.rsPerm.size();
  F.rsFrac.assign((size_t)(dim * ns), 0.0);
  for (int64_t k = 0; k < ns; ++k)
    for (int a = 0; a < dim; ++a) F.rsFrac[(size_t)(a * ns + k)] = F.fracE[(size_t)(a * n + F.rsPerm[(size_t)k])];
  F.rsNpt = ns >= kExtNptMinNodes ? 2 : 1;
  if (const char* e = std::getenv("CPM_RESID_NPT")) {  // slots per lane of its staging workgroups
    const int v = std::atoi(e);
    if (v == 1 || v == 2 || v == 4) F.rsNpt = v;
  }
  stage_slot_list(ns, packed, F.origin, S, F.rsNpt, F.rsBlkE, F.rsGidx, F.rsBlkG, F.rsLorg, F.rsPackedL, F.rsMaxE,
                  F.rsMaxG);
  F.rsN = ns;
}

// Stencil-ordered extension addressing and the B_interp neighbour lists of one level.
cpm_status build_stencil_order(HostLevel& Lv, int level, std::string& err) {
  const int dim = Lv.dim;
  const int64_t n = Lv.n;
  const int S = dim == 2 ? 4 : 16;
  // stencil base of every node (x of the base = x of the first run node)
  std::vector<int32_t> bx((size_t)n), by((size_t)n), bz((size_t)n, 0);
  for (int64_t i = 0; i < n; ++i) {
    const int32_t j = Lv.runE[(size_t)i];  // run (0, 0): node (bx, by, bz)
    bx[(size_t)i] = Lv.idx[(size_t)(j * dim)];
    by[(size_t)i] = Lv.idx[(size_t)(j * dim + 1)];
    if (dim == 3) bz[(size_t)i] = Lv.idx[(size_t)(j * dim + 2)];
  }
  // Visit order: stencil bases grouped into blocks of 16^dim cells ordered along a Morton
  // curve, (z, y, x) inside a block.  A workgroup's slots then hold a compact patch of the
  // surface rather than a strip along y, so the union of their stencils (the values it
  // stages) is about half as large, and consecutive workgroups touch neighbouring regions
  // whose rows stay in L2.  Blocks of 8^dim cells stage 7 % fewer values per node, but the
  // larger blocks keep more of the consecutive workgroups' rows in the caches (measured:
  // the FP64 cycle on the torus at h = 1/256 1.2 % faster).  CPM_MORTON_BITS sets log2 of
  // the block edge; a negative value gives the plain (z, y, x) order.
  int block_bits = 4;
  if (const char* e = std::getenv("CPM_MORTON_BITS")) block_bits = std::atoi(e);
  int32_t mn[3] = {INT32_MAX, INT32_MAX, INT32_MAX};
  for (int64_t i = 0; i < n; ++i) {
    mn[0] = std::min(mn[0], bx[(size_t)i]);
    mn[1] = std::min(mn[1], by[(size_t)i]);
    mn[2] = std::min(mn[2], bz[(size_t)i]);
  }
  std::vector<uint64_t> key((size_t)n, 0);
  if (block_bits >= 0) {
    for (int64_t i = 0; i < n; ++i) {
      const uint32_t c[3] = {(uint32_t)(bx[(size_t)i] - mn[0]) >> block_bits,
                             (uint32_t)(by[(size_t)i] - mn[1]) >> block_bits,
                             (uint32_t)(bz[(size_t)i] - mn[2]) >> block_bits};
      uint64_t m = 0;
      for (int bit = 0; bit < 20; ++bit)
        for (int a = 0; a < 3; ++a) m |= (uint64_t)((c[a] >> bit) & 1u) << (3 * bit + a);
      key[(size_t)i] = m;
    }
  }
  std::vector<int32_t> order((size_t)n);
  for (int64_t i = 0; i < n; ++i) order[(size_t)i] = (int32_t)i;
  std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
    if (key[(size_t)a] != key[(size_t)b]) return key[(size_t)a] < key[(size_t)b];
    if (bz[(size_t)a] != bz[(size_t)b]) return bz[(size_t)a] < bz[(size_t)b];
    if (by[(size_t)a] != by[(size_t)b]) return by[(size_t)a] < by[(size_t)b];
    return bx[(size_t)a] < bx[(size_t)b];
  });
  Lv.perm = order;
  Lv.packed.assign((size_t)n, 0);
  Lv.fracK.assign((size_t)(dim * n), 0.0);
  Lv.origin.clear();
  // cross rows of the widened stencil (fused sweep): first node of each row, which must be
  // followed by the 3 other nodes of the row in consecutive band entries.  Only levels up to
  // kFusedMaxNodes get them: the fused pass reads 2.5x the values of the extension, which pays
  // where launches and load latency dominate, not on large levels.
  const int SX = dim == 2 ? 2 : 16;
  bool xok = n <= kFusedMaxNodes;
  const int64_t nx = xok ? n : 0;
  std::vector<int32_t> runX((size_t)SX * (size_t)nx, -1);
#pragma omp parallel for reduction(&& : xok)
  for (int64_t i = 0; i < nx; ++i) {
    for (int s = 0; s < SX; ++s) {
      int64_t yy, zz;
      if (dim == 2) {
        yy = s == 0 ? -1 : 4;
        zz = 0;
      } else if (s < 8) {
        yy = s < 4 ? -1 : 4;
        zz = s & 3;
      } else {
        yy = s & 3;
        zz = s < 12 ? -1 : 4;
      }
      const int64_t x = bx[(size_t)i], y = by[(size_t)i] + yy, z = dim == 3 ? bz[(size_t)i] + zz : 0;
      const int32_t j = lookup(Lv, x, y, z);
      bool ok = j >= 0;
      for (int a = 1; ok && a < 4; ++a) ok = lookup(Lv, x + a, y, z) == j + a;
      if (!ok) xok = false;
      runX[(size_t)(s * n + i)] = j;
    }
  }
  Lv.fusedOK = xok;
  Lv.originX.clear();
  int64_t g = -1;
  int32_t gx0 = 0, gy = 0, gz = 0;
  std::vector<int32_t> org(S), orgX(SX);
  for (int64_t k = 0; k < n; ++k) {
    const int32_t i = order[(size_t)k];
    const int32_t dx = bx[(size_t)i] - gx0;
    bool fresh = g < 0 || by[(size_t)i] != gy || bz[(size_t)i] != gz || dx < 0 || dx >= (1 << kXoffBits);
    if (!fresh) {
      for (int s = 0; s < S; ++s)
        if (Lv.runE[(size_t)(s * n + i)] - dx != org[(size_t)s]) {
          fresh = true;
          break;
        }
    }
    if (!fresh && xok) {
      for (int s = 0; s < SX; ++s)
        if (runX[(size_t)(s * n + i)] - dx != orgX[(size_t)s]) {
          fresh = true;
          break;
        }
    }
    if (fresh) {
      ++g;
      gx0 = bx[(size_t)i];
      gy = by[(size_t)i];
      gz = bz[(size_t)i];
      for (int s = 0; s < S; ++s) {
        org[(size_t)s] = Lv.runE[(size_t)(s * n + i)];
        Lv.origin.push_back(org[(size_t)s]);
      }
      if (xok)
        for (int s = 0; s < SX; ++s) {
          orgX[(size_t)s] = runX[(size_t)(s * n + i)];
          Lv.originX.push_back(orgX[(size_t)s]);
        }
    }
    if (g >= kMaxGroups) {
      std::ostringstream os;
      os << "too many stencil groups on level " << level;
      err = os.str();
      return CPM_E_INVALID;
    }
    Lv.packed[(size_t)k] = (int32_t)((g << kXoffBits) | (bx[(size_t)i] - gx0));
    for (int a = 0; a < dim; ++a) Lv.fracK[(size_t)(a * n + k)] = Lv.fracE[(size_t)(a * n + i)];
  }
  Lv.ngroups = g + 1;
  build_lds_tables(Lv, S, SX);
  Lv.packedB.assign((size_t)n, 0);
  for (int64_t k = 0; k < n; ++k) Lv.packedB[(size_t)order[(size_t)k]] = Lv.packed[(size_t)k];
  // B_interp (every node of some cubic stencil) with its +-y, +-z neighbours
  std::vector<uint8_t> used((size_t)n, 0);
  for (int s = 0; s < S; ++s)
    for (int64_t i = 0; i < n; ++i) {
      const int32_t j = Lv.runE[(size_t)(s * n + i)];
      for (int a = 0; a < 4; ++a) used[(size_t)(j + a)] = 1;
    }
  Lv.ilist.clear();
  for (int64_t j = 0; j < n; ++j)
    if (used[(size_t)j]) Lv.ilist.push_back((int32_t)j);
  const int64_t m = (int64_t)Lv.ilist.size();
  const int nq = 2 * dim - 2;
  Lv.nbrI.assign((size_t)(nq * m), -1);
  for (int64_t k = 0; k < m; ++k) {
    const int32_t j = Lv.ilist[(size_t)k];
    for (int q = 0; q < nq; ++q) Lv.nbrI[(size_t)(q * m + k)] = Lv.nbr[(size_t)((q + 2) * n + j)];
    // the +-x neighbours are the adjacent band entries
    if (Lv.nbr[(size_t)j] != j - 1 || Lv.nbr[(size_t)(n + j)] != j + 1) {
      err = "internal: x neighbours of a stencil node are not adjacent";
      return CPM_E_BAND;
    }
  }
  // segments: consecutive list positions whose band indices and every neighbour index
  // advance by one together (every list node has all its axis neighbours in the band)
  Lv.nsSeg.clear();
  Lv.nsChunkSeg.clear();
  Lv.nsSegOff.assign((size_t)m, 0);
  int64_t seg = -1;
  for (int64_t k = 0; k < m; ++k) {
    const int32_t j = Lv.ilist[(size_t)k];
    bool fresh = k == 0 || j != Lv.ilist[(size_t)(k - 1)] + 1;
    for (int q = 0; q < nq && !fresh; ++q)
      fresh = Lv.nbrI[(size_t)(q * m + k)] != Lv.nbrI[(size_t)(q * m + k - 1)] + 1;
    if (fresh) {
      ++seg;
      Lv.nsSeg.push_back((int32_t)k);
      Lv.nsSeg.push_back(j);
      for (int q = 0; q < kNsumSegWords - 2; ++q)
        Lv.nsSeg.push_back(q < nq ? Lv.nbrI[(size_t)(q * m + k)] : -1);
    }
    if ((k & (kNsumChunk - 1)) == 0) Lv.nsChunkSeg.push_back((int32_t)seg);
    Lv.nsSegOff[(size_t)k] = (uint8_t)(seg - Lv.nsChunkSeg.back());  // < kNsumChunk segments per chunk
  }
  return CPM_OK;
}

// 3^dim patch addressing for the learned smoother, in band order.  Row (dy, dz) of node i
// is addressed by one reference index ref: the present node at x offset dx (-1, 0, 1) sits at
// ref + (dx + 1), except in a row whose middle node is absent while both outer ones are
// present, where the +1 node follows the -1 node directly (ref + 1): band order is x fastest,
// so the present nodes of one grid row are consecutive band entries.  The kernels read that
// case from the presence mask.
cpm_status build_patches(HostLevel& Lv, int level, std::string& err) {
  const int dim = Lv.dim;
  const int64_t n = Lv.n;
  const int rows = dim == 2 ? 3 : 9;
  Lv.patchRow.assign((size_t)(rows * n), 0);
  Lv.patchMask.assign((size_t)n, 0u);
  bool bad = false;
#pragma omp parallel for reduction(|| : bad)
  for (int64_t i = 0; i < n; ++i) {  // band order: the network visits nodes as stored
    const int32_t* m = &Lv.idx[(size_t)(i * dim)];
    uint32_t mask = 0;
    for (int r = 0; r < rows; ++r) {
      const int dy = r % 3 - 1, dz = dim == 3 ? r / 3 - 1 : 0;
      int32_t j3[3];
      uint32_t rm = 0;
      for (int dx = -1; dx <= 1; ++dx) {
        j3[dx + 1] = lookup(Lv, (int64_t)m[0] + dx, (int64_t)m[1] + dy, dim == 3 ? (int64_t)m[2] + dz : 0);
        if (j3[dx + 1] >= 0) rm |= 1u << (dx + 1);
      }
      int32_t ref = 0;
      for (int q = 0; q < 3; ++q)
        if (rm & (1u << q)) {
          ref = j3[q] - q;
          break;
        }
      const bool gap = rm == 5u;
      for (int q = 0; q < 3; ++q)
        if ((rm & (1u << q)) && j3[q] != ref + q - (gap && q == 2 ? 1 : 0)) bad = true;
      mask |= rm << (3 * r);
      Lv.patchRow[(size_t)(r * n + i)] = ref;
    }
    Lv.patchMask[(size_t)i] = mask;
  }
  if (bad) {
    std::ostringstream os;
    os << "internal: learned-smoother patch rows of level " << level << " are not consecutive band entries";
    err = os.str();
    return CPM_E_BAND;
  }
  Lv.patchOK = true;
  // Group consecutive nodes whose present rows all continue the group's rows (row r of node
  // t of the group = base_r + t).  A row with no present node is loaded but masked out, so
  // its base is free: it is fixed by the first node of the group that has the row.
  std::vector<int32_t> bases;  // groups x rows
  std::vector<int32_t> base((size_t)rows, 0);
  std::vector<char> fixed((size_t)rows, 0);
  Lv.patchPk.assign((size_t)n, 0);
  int64_t g = -1;
  int t = 0;
  auto flush = [&]() {
    for (int r = 0; r < rows; ++r) bases.push_back(fixed[(size_t)r] ? base[(size_t)r] : 0);
  };
  for (int64_t i = 0; i < n; ++i) {
    const uint32_t mask = Lv.patchMask[(size_t)i];
    bool fresh = g < 0 || t + 1 >= kPatchRun;
    for (int r = 0; r < rows && !fresh; ++r)
      if (((mask >> (3 * r)) & 7u) && fixed[(size_t)r] && Lv.patchRow[(size_t)(r * n + i)] != base[(size_t)r] + t + 1)
        fresh = true;
    if (fresh) {
      if (g >= 0) flush();
      ++g;
      t = 0;
      std::fill(fixed.begin(), fixed.end(), 0);
    } else {
      ++t;
    }
    for (int r = 0; r < rows; ++r)
      if (((mask >> (3 * r)) & 7u) && !fixed[(size_t)r]) {
        base[(size_t)r] = Lv.patchRow[(size_t)(r * n + i)] - t;
        fixed[(size_t)r] = 1;
      }
    Lv.patchPk[(size_t)i] = (int32_t)((g << kPatchBits) | t);
  }
  if (g >= 0) flush();
  const int64_t G = g + 1;
  if (G >= ((int64_t)1 << (31 - kPatchBits))) {
    // too many groups to pack: the level has no learned-smoother addressing, and a learned
    // solve on this band is refused (cpm_solve reports it)
    Lv.patchOK = false;
    std::vector<int32_t>().swap(Lv.patchRow);
    std::vector<uint32_t>().swap(Lv.patchMask);
    std::vector<int32_t>().swap(Lv.patchPk);
    return CPM_OK;
  }
  Lv.patchGroups = G;
  Lv.patchBase.assign((size_t)(rows * G), 0);
  for (int64_t q = 0; q < G; ++q)
    for (int r = 0; r < rows; ++r) Lv.patchBase[(size_t)(r * G + q)] = bases[(size_t)(q * rows + r)];
  return CPM_OK;
}

// Lagrange basis of the cubic stencil (nodes 0..3) at s = 1 + a, a in [0, 1).
inline void cubic_basis(double a, double w[4]) {
  const double am1 = a - 1.0, am2 = a - 2.0, ap1 = a + 1.0;
  w[0] = -(a * am1 * am2) * (1.0 / 6.0);
  w[1] = (ap1 * am1 * am2) * 0.5;
  w[2] = -(ap1 * a * am2) * 0.5;
  w[3] = (ap1 * a * am1) * (1.0 / 6.0);
}

// (E N)_ii for every node: the weights of node i's own cubic stencil at the stencil nodes
// that are axis neighbours of node i, summed and divided by h^2.  diag(A) = delta - (E N)_ii
// is the divisor of the standard Jacobi relaxation (Sec. 4.1, Sec. 4.5).  Also the same
// quantity for Remark 3.2's operator A = delta I - E_1 N + gamma (E_1 - E_3):
// q1 = (E_1 N)_ii - gamma (E_1)_ii + gamma (E_3)_ii, so that diag(A) = delta - q1.
void build_en_diagonal(HostLevel& Lv) {
  const int dim = Lv.dim;
  const int64_t n = Lv.n;
  const double ih2 = 1.0 / (Lv.h * Lv.h);
  const double gamma = 2.0 * dim * ih2;
  Lv.qdiag.assign((size_t)n, 0.0);
  Lv.q1diag.assign((size_t)n, 0.0);
#pragma omp parallel for
  for (int64_t i = 0; i < n; ++i) {
    const int32_t j0 = Lv.runE[(size_t)i];  // run (0, 0) starts at the stencil base
    int32_t base[3] = {0, 0, 0}, me[3] = {0, 0, 0};
    double w[3][4] = {{1.0, 0.0, 0.0, 0.0}, {1.0, 0.0, 0.0, 0.0}, {1.0, 0.0, 0.0, 0.0}};
    // linear weights on the same 4 positions: (0, 1 - a, a, 0) (its base is the cubic's + 1)
    double w1[3][4] = {{1.0, 0.0, 0.0, 0.0}, {1.0, 0.0, 0.0, 0.0}, {1.0, 0.0, 0.0, 0.0}};
    for (int a = 0; a < dim; ++a) {
      base[a] = Lv.idx[(size_t)(j0 * dim + a)];
      me[a] = Lv.idx[(size_t)(i * dim + a)];
      const double fr = Lv.fracE[(size_t)(a * n + i)];
      cubic_basis(fr, w[a]);
      w1[a][0] = 0.0;
      w1[a][1] = 1.0 - fr;
      w1[a][2] = fr;
      w1[a][3] = 0.0;
    }
    // weight of the grid node at offset off from node i in the stencil with 1-D weights ww
    auto weight = [&](const double (*ww)[4], const int* off) {
      double prod = 1.0;
      for (int b = 0; b < dim; ++b) {
        const int rel = me[b] + off[b] - base[b];
        if (rel < 0 || rel > 3) return 0.0;
        prod *= ww[b][rel];
      }
      return prod;
    };
    double q = 0.0, q1n = 0.0;
    for (int a = 0; a < dim; ++a)
      for (int sg = -1; sg <= 1; sg += 2) {
        int off[3] = {0, 0, 0};
        off[a] = sg;
        q += weight(w, off);
        q1n += weight(w1, off);
      }
    const int zero[3] = {0, 0, 0};
    Lv.qdiag[(size_t)i] = q * ih2;
    Lv.q1diag[(size_t)i] = (q1n * ih2 - gamma * weight(w1, zero)) + gamma * weight(w, zero);
  }
}

// Tiled-sweep tables (HostLevel::tileSlot ...).  A box row is stored as the band index of its
// first in-band node and the presence mask of its cells: the in-band nodes of one grid row are
// consecutive band entries (x fastest), so the node at box x is at
// first + popcount(mask & ((1 << x) - 1)), also where the row crosses the band twice.
void build_tiles(HostLevel& Lv) {
  Lv.ntiles = 0;
  std::vector<int32_t>().swap(Lv.tileSlot);
  std::vector<int32_t>().swap(Lv.tileOrg);
  std::vector<int32_t>().swap(Lv.tileRow);
  std::vector<int32_t>().swap(Lv.tperm);
  std::vector<int32_t>().swap(Lv.tloc);
  std::vector<double>().swap(Lv.fracT);
  int64_t min_nodes = kTileMinNodes;  // CPM_TILE_MIN_NODES lowers it (tests on small bands)
  if (const char* e = std::getenv("CPM_TILE_MIN_NODES")) min_nodes = std::atoll(e);
  if (Lv.dim != 3 || Lv.n < min_nodes) return;
  const int64_t n = Lv.n;
  auto fdiv = [](int32_t a, int32_t b) { return a >= 0 ? a / b : -((-a + b - 1) / b); };
  std::vector<int32_t> tc((size_t)(3 * n));
  int32_t mn[3] = {INT32_MAX, INT32_MAX, INT32_MAX};
  const int32_t T[3] = {kTileX, kTileY, kTileZ};
  for (int64_t i = 0; i < n; ++i) {
    const int32_t j = Lv.runE[(size_t)i];  // run (0, 0) starts at the stencil base
    for (int a = 0; a < 3; ++a) {
      const int32_t t = fdiv(Lv.idx[(size_t)(j * 3 + a)], T[a]);
      tc[(size_t)(3 * i + a)] = t;
      mn[a] = std::min(mn[a], t);
    }
  }
  // tiles in Morton order of their coordinates, so that consecutive workgroups (one per tile)
  // stage overlapping boxes while the shared rows are still in L2
  std::vector<std::pair<uint64_t, int32_t>> key((size_t)n);
#pragma omp parallel for
  for (int64_t i = 0; i < n; ++i) {
    uint64_t k = 0;
    for (int bit = 0; bit < 21; ++bit)
      for (int a = 0; a < 3; ++a)
        k |= (uint64_t)(((uint32_t)(tc[(size_t)(3 * i + a)] - mn[a]) >> bit) & 1u) << (3 * bit + a);
    key[(size_t)i] = {k, (int32_t)i};
  }
  std::sort(key.begin(), key.end());
  std::vector<int64_t> first;  // first slot of every tile
  for (int64_t k = 0; k < n; ++k)
    if (k == 0 || key[(size_t)k].first != key[(size_t)(k - 1)].first) first.push_back(k);
  const int64_t nt = (int64_t)first.size();
  first.push_back(n);
  Lv.tileSlot.resize((size_t)nt + 1);
  Lv.tileOrg.resize((size_t)(3 * nt));
  Lv.tileRow.assign((size_t)(2 * kBoxRows * nt), 0);
  Lv.tperm.resize((size_t)n);
  Lv.tloc.resize((size_t)n);
  Lv.fracT.resize((size_t)(3 * n));
  bool ok = true;
#pragma omp parallel for schedule(dynamic, 64) reduction(&& : ok)
  for (int64_t t = 0; t < nt; ++t) {
    const int64_t k0 = first[(size_t)t], k1 = first[(size_t)t + 1];
    const int32_t i0 = key[(size_t)k0].second;
    int32_t o[3];
    for (int a = 0; a < 3; ++a) o[a] = tc[(size_t)(3 * i0 + a)] * T[a] - 1;
    Lv.tileSlot[(size_t)t] = (int32_t)k0;
    for (int a = 0; a < 3; ++a) Lv.tileOrg[(size_t)(3 * t + a)] = o[a];
    for (int r = 0; r < kBoxRows; ++r) {
      const int64_t y = (int64_t)o[1] + r % kBoxY, z = (int64_t)o[2] + r / kBoxY;
      int32_t first = -1, prev = -1;
      uint32_t mask = 0;
      for (int x = 0; x < kBoxX; ++x) {
        const int32_t j = lookup(Lv, (int64_t)o[0] + x, y, z);
        if (j < 0) continue;
        if (first < 0) first = j;
        else if (j != prev + 1) ok = false;  // in-band nodes of a grid row are consecutive entries
        prev = j;
        mask |= 1u << x;
      }
      int32_t* row = &Lv.tileRow[(size_t)(2 * (t * kBoxRows + r))];
      row[0] = first < 0 ? 0 : first;
      row[1] = (int32_t)mask;
    }
    for (int64_t k = k0; k < k1; ++k) {
      const int32_t i = key[(size_t)k].second;
      const int32_t jb = Lv.runE[(size_t)i];
      int32_t loc = 0;
      bool inbox = true;
      for (int a = 0; a < 3; ++a) {
        const int32_t lb = Lv.idx[(size_t)(jb * 3 + a)] - (o[a] + 1);  // base within the tile
        const int32_t c = Lv.idx[(size_t)(i * 3 + a)] - o[a];       // own cell in the box
        const int32_t ext = a == 0 ? kBoxX : (a == 1 ? kBoxY : kBoxZ);
        if (lb < 0 || lb >= T[a]) ok = false;
        inbox = inbox && c >= 0 && c < ext;
        loc |= (lb & 31) << (5 * a);
        loc |= (inbox ? (c & 31) : 0) << (15 + 5 * a);
      }
      if (!inbox) loc &= (1 << 15) - 1;
      if (inbox) loc |= 1 << 30;
      Lv.tperm[(size_t)k] = i;
      Lv.tloc[(size_t)k] = loc;
      for (int a = 0; a < 3; ++a) Lv.fracT[(size_t)(a * n + k)] = Lv.fracE[(size_t)(a * n + i)];
    }
  }
  Lv.tileSlot[(size_t)nt] = (int32_t)n;
  if (!ok) {
    std::vector<int32_t>().swap(Lv.tileSlot);
    std::vector<int32_t>().swap(Lv.tileOrg);
    std::vector<int32_t>().swap(Lv.tileRow);
    std::vector<int32_t>().swap(Lv.tperm);
    std::vector<int32_t>().swap(Lv.tloc);
    std::vector<double>().swap(Lv.fracT);
    return;
  }
  Lv.ntiles = nt;
}

}  // namespace

// Reach of the surface (Sec. 2.1: the closest point is unique within it): the radius for a
// circle or sphere, min(r, R - r) for a torus (tube-centre circle and axis); for Dziuk's
// surface the smallest radius of curvature over the fixed surface samples, 1 / max |kappa|
// with the principal curvatures of the level set phi from its Hessian projected on the
// tangent plane (a local bound: the reach is no larger).
double surface_reach(const cpm_surface& s) {
  if (s.kind == CPM_CIRCLE || s.kind == CPM_SPHERE) return s.R;
  if (s.kind == CPM_TORUS) return std::min(s.r, s.R - s.r);
  const std::vector<double>& S = dziuk_samples();
  double kmax = 0.0;
  for (size_t k = 0; k < S.size() / 3; ++k) {
    const double x1 = S[3 * k], x2 = S[3 * k + 1], x3 = S[3 * k + 2];
    const double p = x1 - x3 * x3;
    const double g[3] = {2.0 * p, 2.0 * x2, 2.0 * x3 - 4.0 * x3 * p};
    const double H[3][3] = {{2.0, 0.0, -4.0 * x3}, {0.0, 2.0, 0.0}, {-4.0 * x3, 0.0, (2.0 - 4.0 * p) + 8.0 * x3 * x3}};
    const double gn = std::sqrt((g[0] * g[0] + g[1] * g[1]) + g[2] * g[2]);
    const double n[3] = {g[0] / gn, g[1] / gn, g[2] / gn};
    // shape operator P H P / |grad phi|, P = I - n n^T; its eigenvalues are 0 (along n) and
    // the two principal curvatures
    double P[3][3], PH[3][3], W[3][3];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) P[i][j] = (i == j ? 1.0 : 0.0) - n[i] * n[j];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        PH[i][j] = 0.0;
        for (int q = 0; q < 3; ++q) PH[i][j] += P[i][q] * H[q][j];
      }
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        W[i][j] = 0.0;
        for (int q = 0; q < 3; ++q) W[i][j] += PH[i][q] * P[q][j];
        W[i][j] /= gn;
      }
    // the two non-zero eigenvalues: trace and the sum of principal 2x2 minors
    const double tr = W[0][0] + W[1][1] + W[2][2];
    const double m2 = (W[0][0] * W[1][1] - W[0][1] * W[1][0]) + (W[0][0] * W[2][2] - W[0][2] * W[2][0]) +
                      (W[1][1] * W[2][2] - W[1][2] * W[2][1]);
    const double disc = std::sqrt(std::max(0.0, tr * tr - 4.0 * m2));
    kmax = std::max(kmax, std::max(std::fabs(0.5 * (tr + disc)), std::fabs(0.5 * (tr - disc))));
  }
  return kmax > 0.0 ? 1.0 / kmax : std::numeric_limits<double>::infinity();
}

// Threads of the calling thread's OpenMP parallel regions (a batch of bands is built by
// several host threads at once, each single-threaded inside).
void set_host_build_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }

cpm_status build_host_levels(const cpm_surface& s, const cpm_grid& g, int dim,
                             std::vector<HostLevel>& levels, std::string& err) {
  const int L = g.levels;
  double lam2 = g.lam2 > 0 ? g.lam2 : (dim == 2 ? 13.0 : 17.0);
  levels.assign((size_t)L, HostLevel());
  for (int l = 0; l < L; ++l) {
    double h = g.h0 * std::ldexp(1.0, l);
    cpm_status st = enumerate_level(s, dim, h, lam2, levels[(size_t)l], err);
    if (st != CPM_OK) return st;
  }
  for (int l = 0; l < L; ++l) {
    HostLevel& Lv = levels[(size_t)l];
    int64_t bad = -1;
    if (!stencil_runs(Lv, Lv, 3, Lv.runE, Lv.fracE, &bad)) {
      std::ostringstream os;
      os << "cubic stencil of node " << bad << " leaves the band on level " << l;
      err = os.str();
      return CPM_E_BAND;
    }
    build_en_diagonal(Lv);
    // Laplacian neighbours, missing ones marked -1 (they only occur at band edges)
    const int64_t n = Lv.n;
    const int nn = 2 * dim;
    Lv.nbr.assign((size_t)(nn * n), -1);
#pragma omp parallel for
    for (int64_t i = 0; i < n; ++i) {
      const int32_t* m = &Lv.idx[(size_t)(i * dim)];
      for (int a = 0; a < dim; ++a) {
        for (int sg = 0; sg < 2; ++sg) {
          int64_t q[3] = {m[0], m[1], dim == 3 ? m[2] : 0};
          q[a] += sg == 0 ? -1 : 1;
          Lv.nbr[(size_t)((2 * a + sg) * n + i)] = lookup(Lv, q[0], q[1], q[2]);
        }
      }
    }
    // containment: every node of a cubic stencil has all of its Laplacian neighbours
    std::vector<uint8_t> used((size_t)n, 0);
    const int nruns = dim == 2 ? 4 : 16;
    for (int r = 0; r < nruns; ++r)
      for (int64_t i = 0; i < n; ++i) {
        int32_t j = Lv.runE[(size_t)(r * n + i)];
        for (int a = 0; a < 4; ++a) used[(size_t)(j + a)] = 1;
      }
    for (int64_t j = 0; j < n; ++j) {
      if (!used[(size_t)j]) continue;
      for (int k = 0; k < nn; ++k)
        if (Lv.nbr[(size_t)(k * n + j)] < 0) {
          std::ostringstream os;
          os << "band too narrow on level " << l << ": stencil node " << j
             << " lacks a Laplacian neighbour";
          err = os.str();
          return CPM_E_BAND;
        }
    }
  }
  for (int l = 0; l < L; ++l) {
    cpm_status st = build_stencil_order(levels[(size_t)l], l, err);
    if (st != CPM_OK) return st;
    build_tiles(levels[(size_t)l]);
    if (l < 2 && (st = build_patches(levels[(size_t)l], l, err)) != CPM_OK) return st;
  }
  for (int l = 0; l + 1 < L; ++l) {
    HostLevel& F = levels[(size_t)l];
    HostLevel& C = levels[(size_t)(l + 1)];
    int64_t bad = -1;
    if (!stencil_runs(F, C, 1, F.runP, F.fracP, &bad)) {
      std::ostringstream os;
      os << "prolongation stencil of node " << bad << " (level " << l << ") leaves the band of level "
         << l + 1;
      err = os.str();
      return CPM_E_BAND;
    }
    if (!stencil_runs(F, C, 3, F.runP3, F.fracP3, &bad)) {
      std::vector<int32_t>().swap(F.runP3);  // no full-multigrid start on this band
      std::vector<double>().swap(F.fracP3);
    }
    if (!stencil_runs(C, F, 1, C.runR, C.fracR, &bad)) {
      std::ostringstream os;
      os << "restriction stencil of node " << bad << " (level " << l + 1 << ") leaves the band of level "
         << l;
      err = os.str();
      return CPM_E_BAND;
    }
    build_resid_subset(F, C);
  }
  for (auto& Lv : levels) std::vector<int32_t>().swap(Lv.map);
  return CPM_OK;
}

}  // namespace cpm
