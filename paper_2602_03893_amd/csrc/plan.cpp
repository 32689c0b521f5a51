// plan.cpp -- host planner: validation, spatial tiling, workspace layout.
//
// The direct operator pairs every kernel with every sensor (arXiv 2602.03893,
// Methods, start of the "Adaptive supersampling alignment" subsection).  The
// paper precomputes a lookup table of pair distances (Algorithm 1); at 8.4 M
// kernels x 1024 sensors that table would not fit, so this build computes the
// distances on the fly and instead precomputes a spatial tiling: kernels are
// ordered along a Morton curve of the kernel lattice and cut into compact
// tiles, each described by a bounding sphere.  For a tile and a sensor, every
// member's pulse arrives inside the time shell [R - rho, R + rho] widened by
// the window, so one short trace segment per (tile, sensor) holds every tap of
// the tile: that is the binning by sensor-distance shell the kernels use.
#include <algorithm>
#include <climits>
#include <cmath>
#include <cstring>
#include <limits>
#include <numeric>
#include <thread>

#include "gpair_internal.h"

namespace gpair {

namespace {

inline uint64_t spread3(uint64_t x) {
  x &= 0x1fffff;  // 21 bits
  x = (x | (x << 32)) & 0x1f00000000ffffULL;
  x = (x | (x << 16)) & 0x1f0000ff0000ffULL;
  x = (x | (x << 8)) & 0x100f00f00f00f00fULL;
  x = (x | (x << 4)) & 0x10c30c30c30c30c3ULL;
  x = (x | (x << 2)) & 0x1249249249249249ULL;
  return x;
}

inline uint64_t morton3(uint32_t ix, uint32_t iy, uint32_t iz) {
  return spread3(ix) | (spread3(iy) << 1) | (spread3(iz) << 2);
}

bool is_pow2(int64_t x) { return x > 0 && (x & (x - 1)) == 0; }

// Sort of (key, index) records by key, then index: a parallel LSD radix sort
// (11-bit digits, as many passes as the largest key needs).  The input is in
// index order and every pass is stable, so equal keys keep index order.
struct KeyIdx {
  uint64_t key;
  int32_t idx;
};

void parallel_sort(HostVec<KeyIdx> &v) {
  const int64_t n = (int64_t)v.size();
  uint64_t kmax = 0;
  for (const KeyIdx &r : v) kmax = std::max(kmax, r.key);
  int bits = 0;
  while (bits < 64 && (kmax >> bits) != 0) ++bits;
  constexpr int kDigit = 11, kBuckets = 1 << kDigit;
  const int T = (int)std::min<int64_t>(host_threads(), std::max<int64_t>(1, n / 65536));
  HostVec<KeyIdx> tmp((size_t)n);
  std::vector<int64_t> count((size_t)T * kBuckets);
  for (int shift = 0; shift < bits; shift += kDigit) {
    std::fill(count.begin(), count.end(), 0);
    std::vector<std::thread> th;
    for (int t = 0; t < T; ++t)
      th.emplace_back([&, t] {
        int64_t *c = &count[(size_t)t * kBuckets];
        for (int64_t i = n * t / T; i < n * (t + 1) / T; ++i)
          ++c[(v[i].key >> shift) & (kBuckets - 1)];
      });
    for (auto &x : th) x.join();
    th.clear();
    // exclusive offsets in (digit, thread) order: stable
    int64_t off = 0;
    for (int d = 0; d < kBuckets; ++d)
      for (int t = 0; t < T; ++t) {
        const int64_t c = count[(size_t)t * kBuckets + d];
        count[(size_t)t * kBuckets + d] = off;
        off += c;
      }
    for (int t = 0; t < T; ++t)
      th.emplace_back([&, t] {
        int64_t *c = &count[(size_t)t * kBuckets];
        for (int64_t i = n * t / T; i < n * (t + 1) / T; ++i)
          tmp[c[(v[i].key >> shift) & (kBuckets - 1)]++] = v[i];
      });
    for (auto &x : th) x.join();
    v.swap(tmp);
  }
}

int level_for(int64_t tile) {  // smallest l with 8^l >= tile
  int l = 0;
  int64_t b = 1;
  while (b < tile) {
    b *= 8;
    ++l;
  }
  return l;
}

// Sorted unique values of one coordinate axis: chunks sorted and made unique
// in parallel, then the (short, for a lattice) lists merged.
std::vector<float> axis_values(const float *x, int64_t m) {
  const int T = (int)std::min<int64_t>(host_threads(), std::max<int64_t>(1, m / 65536));
  std::vector<std::vector<float>> part(T);
  std::vector<std::thread> th;
  for (int t = 0; t < T; ++t)
    th.emplace_back([&, t] {
      std::vector<float> &v = part[t];
      v.assign(x + m * t / T, x + m * (t + 1) / T);
      std::sort(v.begin(), v.end());
      v.erase(std::unique(v.begin(), v.end()), v.end());
    });
  for (auto &t : th) t.join();
  std::vector<float> v;
  for (const auto &p : part) v.insert(v.end(), p.begin(), p.end());
  std::sort(v.begin(), v.end());
  v.erase(std::unique(v.begin(), v.end()), v.end());
  return v;
}

struct Keys {
  HostVec<uint64_t> key;
  bool lattice = false;
  double quantum = 0.0;  // point clouds: edge of one quantisation cell (m)
};

Keys morton_keys(const gpair_geometry *g) {
  const int64_t m = g->n_kernels;
  Keys out;
  out.key.resize(m);
  std::vector<float> ux = axis_values(g->cx, m), uy = axis_values(g->cy, m),
                     uz = axis_values(g->cz, m);
  const double prod = (double)ux.size() * (double)uy.size() * (double)uz.size();
  if (prod == (double)m && ux.size() < (1u << 21) && uy.size() < (1u << 21) &&
      uz.size() < (1u << 21)) {
    // Candidate full lattice: every kernel must map to a distinct lattice node.
    HostVec<uint32_t> lin((size_t)m);
    parallel_ranges(m, [&](int64_t b, int64_t e) {
      for (int64_t k = b; k < e; ++k) {
        uint32_t ix = (uint32_t)(std::lower_bound(ux.begin(), ux.end(), g->cx[k]) - ux.begin());
        uint32_t iy = (uint32_t)(std::lower_bound(uy.begin(), uy.end(), g->cy[k]) - uy.begin());
        uint32_t iz = (uint32_t)(std::lower_bound(uz.begin(), uz.end(), g->cz[k]) - uz.begin());
        lin[k] = (uint32_t)(((size_t)iz * uy.size() + iy) * ux.size() + ix);
        out.key[k] = morton3(ix, iy, iz);
      }
    });
    std::vector<uint8_t> seen((size_t)m, 0);  // zeroed: read before written
    bool ok = true;
    for (int64_t k = 0; k < m && ok; ++k) {
      if (seen[lin[k]]) ok = false;
      seen[lin[k]] = 1;
    }
    if (ok) {
      out.lattice = true;
      return out;
    }
  }
  // Point cloud: quantise positions on a cubic grid of 2^20 cells per axis.
  double lo[3] = {ux.front(), uy.front(), uz.front()};
  double hi[3] = {ux.back(), uy.back(), uz.back()};
  double ext = std::max({hi[0] - lo[0], hi[1] - lo[1], hi[2] - lo[2]});
  double q = ext > 0 ? ext / double((1u << 20) - 1) : 1.0;
  out.quantum = q;
  const float *c[3] = {g->cx, g->cy, g->cz};
  parallel_ranges(m, [&](int64_t b, int64_t e) {
    for (int64_t k = b; k < e; ++k) {
      uint32_t ii[3];
      for (int a = 0; a < 3; ++a) {
        double t = std::floor(((double)c[a][k] - lo[a]) / q);
        t = std::min(std::max(t, 0.0), double((1u << 20) - 1));
        ii[a] = (uint32_t)t;
      }
      out.key[k] = morton3(ii[0], ii[1], ii[2]);
    }
  });
  return out;
}

// Cut the Morton-ordered kernels [s0, e0) into tiles of at most `tile`
// members that never cross an aligned Morton block of 8^level cells, and
// append them to `tiles`.
void cut_tiles(const HostVec<uint64_t> &sorted_keys, const HostVec<double> &kgeo, int64_t tile,
               int level, int64_t s0, int64_t e0, std::vector<TileInfo> &tiles) {
  const int shift = 3 * level;
  int64_t s = s0;
  while (s < e0) {
    const uint64_t blk = shift >= 64 ? 0 : (sorted_keys[s] >> shift);
    int64_t e = s + 1;
    while (e < e0 && e - s < tile &&
           (shift >= 64 ? 0 : (sorted_keys[e] >> shift)) == blk)
      ++e;
    TileInfo t{};
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int64_t i = s; i < e; ++i)
      for (int a = 0; a < 3; ++a) {
        lo[a] = std::min(lo[a], kgeo[4 * i + a]);
        hi[a] = std::max(hi[a], kgeo[4 * i + a]);
      }
    t.cx = 0.5 * (lo[0] + hi[0]);
    t.cy = 0.5 * (lo[1] + hi[1]);
    t.cz = 0.5 * (lo[2] + hi[2]);
    double r2 = 0;
    for (int64_t i = s; i < e; ++i) {
      double dx = kgeo[4 * i] - t.cx, dy = kgeo[4 * i + 1] - t.cy,
             dz = kgeo[4 * i + 2] - t.cz;
      r2 = std::max(r2, dx * dx + dy * dy + dz * dz);
    }
    t.rho = std::sqrt(r2) * (1.0 + 1e-12) + 1e-15;
    t.start = (int32_t)s;
    t.count = (int32_t)(e - s);
    t.first_block = -1;
    tiles.push_back(t);
    s = e;
  }
}

std::vector<TileInfo> make_tiles(const HostVec<uint64_t> &sorted_keys,
                                 const HostVec<double> &kgeo, int64_t tile, int level) {
  std::vector<TileInfo> tiles;
  cut_tiles(sorted_keys, kgeo, tile, level, 0, (int64_t)sorted_keys.size(), tiles);
  return tiles;
}

// Adjoint tiles cut inside each forward tile (so that every forward tile is
// a whole number of adjoint tiles, its reference blocks); sets each forward
// tile's first_block.
std::vector<TileInfo> make_nested_tiles(const HostVec<uint64_t> &sorted_keys,
                                        const HostVec<double> &kgeo,
                                        std::vector<TileInfo> &ftiles, int64_t tile, int level) {
  std::vector<TileInfo> tiles;
  for (TileInfo &F : ftiles) {
    F.first_block = (int32_t)tiles.size();
    cut_tiles(sorted_keys, kgeo, tile, level, F.start, (int64_t)F.start + F.count, tiles);
  }
  return tiles;
}

double max_rho(const std::vector<TileInfo> &t) {
  double r = 0;
  for (const auto &x : t) r = std::max(r, x.rho);
  return r;
}

// Samples of a (tile, sensor) trace segment: the tile's time shell widened
// by the window on both sides, plus slack for rounding and for the padding
// taps the unrolled forward writes past a window's end.
int segment_len(double rho, double inv_vdt, double hmax) {
  double L = std::ceil(2.0 * rho * inv_vdt + 2.0 * hmax) + 7.0;
  return L > 1e9 ? 1000000000 : (int)L;
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Window half-width (samples) of the widest kernel the records admit: the
// record builder clamps sigma to sigma_max (1 + 1e-6).
double hmax_admitted(const gpair_plan_s *p) { return p->hmax * (1.0 + 1e-6); }

// Lower slot of a (tile, sensor) trace segment, exactly as the operators
// compute it: nb = floor((R - rho) / (v dt) - t0 / dt - h_max) - 1.
int64_t segment_base(const gpair_plan_s *p, const TileInfo &T, const double *s) {
  const double dx = s[0] - T.cx, dy = s[1] - T.cy, dz = s[2] - T.cz;
  const double R = std::sqrt(std::fma(dz, dz, std::fma(dy, dy, dx * dx)));
  return (int64_t)std::floor((R - T.rho) * p->inv_vdt - p->t0_over_dt - p->hmax) - 1;
}

// Slot bound of the trace segments (the binning invariant the operators rely
// on instead of clamping LDS indices).  For a member k of tile T at distance
// r from sensor s, r lies in [R - rho, R + rho], so its first in-window
// sample lo = ceil(r/(v dt) - t0/dt - h_k) satisfies lo - nb >= 1, and its
// last touched sample, with up to two masked padding taps of the unrolled
// loops, is at most lo + ntap_k + 1 <= r/(v dt) - t0/dt + h_k + 3.  Both are
// checked here per (tile, sensor) with the widest admitted window and a
// rounding margin of 1e-6 samples (distances are float64, ~1e-12 samples).
// Returns the largest slot any pair can touch, or -1 if a lower bound fails.
int64_t max_slot(const gpair_plan_s *p, const std::vector<TileInfo> &tiles) {
  const int64_t nt = (int64_t)tiles.size();
  const int nth = (int)std::min<int64_t>(host_threads(), std::max<int64_t>(1, nt / 256));
  const double hm = hmax_admitted(p);
  std::vector<int64_t> worst(nth, 0);
  std::vector<std::thread> th;
  for (int t = 0; t < nth; ++t)
    th.emplace_back([&, t] {
      int64_t w = 0;
      for (int64_t ti = nt * t / nth; ti < nt * (t + 1) / nth; ++ti) {
        const TileInfo &T = tiles[ti];
        for (int32_t j = 0; j < p->Nd; ++j) {
          const double *s = &p->host.sens[4 * (size_t)j];
          const int64_t nb = segment_base(p, T, s);
          const double dx = s[0] - T.cx, dy = s[1] - T.cy, dz = s[2] - T.cz;
          const double R = std::sqrt(dx * dx + dy * dy + dz * dz);
          const double lo_min = std::ceil((R - T.rho) * p->inv_vdt - p->t0_over_dt - hm - 1e-6);
          const double hi_max =
              std::floor((R + T.rho) * p->inv_vdt - p->t0_over_dt + hm + 3.0 + 1e-6);
          if (lo_min - (double)nb < 0.0) {
            w = -1;
            break;
          }
          w = std::max(w, (int64_t)hi_max - nb);
        }
        if (w < 0) break;
      }
      worst[t] = w;
    });
  for (auto &x : th) x.join();
  int64_t w = 0;
  for (int64_t x : worst) {
    if (x < 0) return -1;
    w = std::max(w, x);
  }
  return w;
}

}  // namespace

int filter_steps(double R, double rho, double inv_vdt, double hmax) {
  if (!(R > 4.0 * rho)) return -1;
  // |dr| <= rho; the first estimate D/(2R) is off by dr^2/(2R) <= rho^2/(2R)
  // and each step multiplies the error by at most kappa.
  const double kappa = (2.0 * rho + rho * rho / (2.0 * R)) / (2.0 * R);
  double e = rho * rho / (2.0 * R) * inv_vdt;
  int k = 0;
  while (e > kFilterIterTol && k < kFilterMaxSteps) {
    e *= kappa;
    ++k;
  }
  // Rounding: D carries about 5 float32 units of 2R rho (the rounded
  // coordinates and three fused multiply-adds), the steps and 1/(2R) and
  // 1/(v dt) about 9 units of rho, so dr is within 14 units of rho; the sum
  // z = (Xf - h) + dr/(v dt) adds 2 units of its magnitude.
  const double zmax = 2.0 + hmax + rho * inv_vdt;
  const double bound = 0x1p-24 * (14.0 * rho * inv_vdt + 2.0 * zmax) + e;
  if (e > kFilterIterTol || !(bound < 0.5 * kFilterGuard)) return -1;
  return k;
}

namespace {

// Filter steps of every adjoint tile: from its closest sensor (the step
// count grows as R falls), about the float32-rounded centre the operators
// use as the reference point.
void set_filter_steps(const gpair_plan_s *p, std::vector<TileInfo> &blocks) {
  parallel_ranges((int64_t)blocks.size(), [&](int64_t b0, int64_t b1) {
    for (int64_t b = b0; b < b1; ++b) {
      TileInfo &B = blocks[b];
      const double bx = (float)B.cx, by = (float)B.cy, bz = (float)B.cz;
      double R2 = std::numeric_limits<double>::infinity();
      for (int32_t j = 0; j < p->Nd; ++j) {
        const double *s = &p->host.sens[4 * (size_t)j];
        const double ux = s[0] - bx, uy = s[1] - by, uz = s[2] - bz;
        R2 = std::min(R2, ux * ux + uy * uy + uz * uz);
      }
      const double ex = bx - B.cx, ey = by - B.cy, ez = bz - B.cz;
      const double rho = B.rho + std::sqrt(ex * ex + ey * ey + ez * ez);
      B.filter_steps = filter_steps(std::sqrt(R2) * (1.0 - 1e-12), rho, p->inv_vdt, p->hmax);
    }
  });
}

}  // namespace

gpair_status tiling_slots(const gpair_plan_s *p, int which, int64_t *min_first,
                          int64_t *max_last) {
  const std::vector<TileInfo> &tiles = which == 0 ? p->host.ftiles : p->host.atiles;
  const double h = hmax_admitted(p);
  const int64_t ntap = (int64_t)std::floor(2.0 * h) + 1;
  const int64_t nt = (int64_t)tiles.size();
  const int nth = (int)std::min<int64_t>(host_threads(), std::max<int64_t>(1, nt / 64));
  std::vector<int64_t> lo_t(nth, INT64_MAX), hi_t(nth, INT64_MIN);
  std::vector<std::thread> th;
  for (int t = 0; t < nth; ++t)
    th.emplace_back([&, t] {
      for (int64_t ti = nt * t / nth; ti < nt * (t + 1) / nth; ++ti) {
        const TileInfo &T = tiles[ti];
        for (int32_t j = 0; j < p->Nd; ++j) {
          const double *s = &p->host.sens[4 * (size_t)j];
          const int64_t nb = segment_base(p, T, s);
          for (int32_t i = T.start; i < T.start + T.count; ++i) {
            const double *c = &p->host.kgeo[4 * (size_t)i];
            const double dx = s[0] - c[0], dy = s[1] - c[1], dz = s[2] - c[2];
            const double r = std::sqrt(dx * dx + dy * dy + dz * dz);
            const int64_t lo = (int64_t)std::ceil(r * p->inv_vdt - p->t0_over_dt - h);
            lo_t[t] = std::min(lo_t[t], lo - nb);
            hi_t[t] = std::max(hi_t[t], lo + ntap + 1 - nb);
          }
        }
      }
    });
  for (auto &x : th) x.join();
  *min_first = *std::min_element(lo_t.begin(), lo_t.end());
  *max_last = *std::max_element(hi_t.begin(), hi_t.end());
  return GPAIR_OK;
}

WorkspaceLayout layout_for(int64_t M, int32_t Nd, size_t nft, size_t nat, int64_t det_words) {
  WorkspaceLayout l{};
  size_t off = 0;
  l.sens = off;     off = align256(off + (size_t)Nd * 32);
  l.perm = off;     off = align256(off + (size_t)M * 4);
  l.ftiles = off;   off = align256(off + nft * sizeof(TileInfo));
  l.atiles = off;   off = align256(off + nat * sizeof(TileInfo));
  l.krec = off;     off = align256(off + (size_t)M * sizeof(KernelRec));
  l.counters = off; off = align256(off + 64);
  l.partials = off; off = align256(off + (size_t)kResidualBlocks * 3 * sizeof(double) + 64);
  // det_words int64 accumulators, then the deterministic forward's global unit
  l.det = off;      off = align256(off + (size_t)det_words * sizeof(long long) + (det_words ? 64 : 0));
  l.total = off;
  return l;
}

gpair_status build_plan(const gpair_geometry *g, gpair_plan_s *p) {
  if (!g || !g->cx || !g->cy || !g->cz || !g->sensors) return GPAIR_ERR_INVALID_ARG;
  if (g->n_kernels < 1 || g->n_kernels > (int64_t)INT32_MAX) return GPAIR_ERR_INVALID_ARG;
  if (g->n_sensors < 1 || g->n_samples < 1) return GPAIR_ERR_INVALID_ARG;
  const double scal[] = {g->dt, g->t0, g->c_sound, g->n_sigma, g->sigma_max};
  for (double s : scal)
    if (!std::isfinite(s)) return GPAIR_ERR_NONFINITE;
  if (!(g->dt > 0) || !(g->c_sound > 0) || !(g->n_sigma > 0) || !(g->sigma_max > 0))
    return GPAIR_ERR_INVALID_ARG;
  if (g->fwd_tile != 0 && (!is_pow2(g->fwd_tile) || g->fwd_tile < 64 || g->fwd_tile > 8192))
    return GPAIR_ERR_INVALID_ARG;
  if (g->adj_tile != 0 && g->adj_tile != 64 && g->adj_tile != 128 && g->adj_tile != 256)
    return GPAIR_ERR_INVALID_ARG;
  if (g->fwd_waves != 0 && g->fwd_waves != 1 && g->fwd_waves != 2 && g->fwd_waves != 4 &&
      g->fwd_waves != 8)
    return GPAIR_ERR_INVALID_ARG;
  const int64_t M = g->n_kernels;
  const int32_t Nd = g->n_sensors;
  for (int64_t k = 0; k < M; ++k)
    if (!std::isfinite(g->cx[k]) || !std::isfinite(g->cy[k]) || !std::isfinite(g->cz[k]))
      return GPAIR_ERR_NONFINITE;
  for (int64_t j = 0; j < 3 * (int64_t)Nd; ++j)
    if (!std::isfinite(g->sensors[j])) return GPAIR_ERR_NONFINITE;

  p->M = M;
  p->Nd = Nd;
  p->Nt = g->n_samples;
  p->dt = g->dt;
  p->t0 = g->t0;
  p->v = g->c_sound;
  p->nsig = g->n_sigma;
  p->sigma_max = g->sigma_max;
  p->vdt = g->c_sound * g->dt;
  p->inv_vdt = 1.0 / p->vdt;
  p->t0_over_dt = g->t0 / g->dt;
  p->hmax = g->n_sigma * g->sigma_max / p->vdt;
  if (!(p->hmax < 4096.0)) return GPAIR_ERR_INVALID_ARG;
  p->ntap_max = (int32_t)std::floor(2.0 * p->hmax) + 1;

  // Spatial order.
  Keys keys = morton_keys(g);
  HostTables &h = p->host;
  HostVec<uint64_t> skeys((size_t)M);
  {
    HostVec<KeyIdx> rec((size_t)M);
    parallel_ranges(M, [&](int64_t b, int64_t e) {
      for (int64_t k = b; k < e; ++k) rec[k] = KeyIdx{keys.key[k], (int32_t)k};
    });
    keys.key.clear();
    keys.key.shrink_to_fit();
    parallel_sort(rec);
    h.perm.resize((size_t)M);
    h.kgeo.resize((size_t)M * 4);
    parallel_ranges(M, [&](int64_t b, int64_t e) {
      for (int64_t i = b; i < e; ++i) {
        const int32_t k = rec[i].idx;
        h.perm[i] = k;
        h.kgeo[4 * i + 0] = g->cx[k];
        h.kgeo[4 * i + 1] = g->cy[k];
        h.kgeo[4 * i + 2] = g->cz[k];
        h.kgeo[4 * i + 3] = 0.0;
        skeys[i] = rec[i].key;
      }
    });
  }
  h.sens.assign((size_t)Nd * 4, 0.0);
  for (int32_t j = 0; j < Nd; ++j) {
    for (int a = 0; a < 3; ++a) h.sens[4 * j + a] = g->sensors[3 * j + a];
    const double *q = &h.sens[4 * (size_t)j];
    h.sens[4 * j + 3] = q[0] * q[0] + q[1] * q[1] + q[2] * q[2];  // |s|^2
  }

  // Block level of a tile of T kernels: lattice -> 8^l >= T lattice nodes;
  // point cloud -> a block edge holding about T kernels at the mean density.
  auto level_of = [&](int64_t T) {
    if (keys.lattice) return level_for(T);
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int64_t i = 0; i < M; ++i)
      for (int a = 0; a < 3; ++a) {
        lo[a] = std::min(lo[a], h.kgeo[4 * i + a]);
        hi[a] = std::max(hi[a], h.kgeo[4 * i + a]);
      }
    double ext = std::max({hi[0] - lo[0], hi[1] - lo[1], hi[2] - lo[2]});
    double vol = 1.0;
    for (int a = 0; a < 3; ++a) vol *= std::max(hi[a] - lo[a], ext / 1024.0);
    if (ext <= 0) return 0;
    double edge = std::cbrt((double)T * vol / (double)M);
    int l = (int)std::lround(std::log2(std::max(edge / keys.quantum, 1.0)));
    return std::min(std::max(l, 0), 20);
  };

  // Forward: a workgroup holds one LDS trace segment of Lf samples for 64
  // sensors, and its waves split the tile's kernels, so the tile size sets
  // both the work per workgroup and its LDS.  Tiles of 1024 lattice nodes
  // (a segment near 18 KiB) measured best at the paper-scale shape, for the
  // direct forward and the ASSA forward, which uses the same tiles; smaller
  // tiles are used only when the problem is too small to give every CU
  // several workgroups.
  const int64_t nsg = (Nd + kWave - 1) / kWave;
  int64_t Tf = g->fwd_tile;
  if (Tf == 0) {
    Tf = 1024;
    while (Tf > 64 && ((M + Tf - 1) / Tf) * nsg < 4096) Tf /= 2;
  }
  const int64_t Lcap = kMaxSegmentBytes / (kWave * 4);
  for (;;) {
    h.ftiles = make_tiles(skeys, h.kgeo, Tf, level_of(Tf));
    p->Lf = segment_len(max_rho(h.ftiles), p->inv_vdt, p->hmax);
    if (p->Lf <= Lcap || Tf <= 64) break;
    Tf /= 2;
  }
  if (p->Lf > Lcap) return GPAIR_ERR_INVALID_ARG;
  p->fwd_tile = (int32_t)Tf;
  p->fwd_waves = g->fwd_waves ? g->fwd_waves : 4;

  // Adjoint tiles nest in forward tiles: at most the forward tile size.
  int64_t Ta = std::min<int64_t>(g->adj_tile ? g->adj_tile : 256, Tf);
  for (;;) {
    h.atiles = make_nested_tiles(skeys, h.kgeo, h.ftiles, Ta, level_of(Ta));
    p->La = segment_len(max_rho(h.atiles), p->inv_vdt, p->hmax);
    if ((int64_t)p->La * kAdjSensorsPerStage * 4 <= kMaxSegmentBytes || Ta <= 64) break;
    Ta /= 2;
  }
  if ((int64_t)p->La * kAdjSensorsPerStage * 4 > kMaxSegmentBytes) return GPAIR_ERR_INVALID_ARG;
  p->adj_tile = (int32_t)Ta;
  p->max_rho = std::max(max_rho(h.ftiles), max_rho(h.atiles));
  set_filter_steps(p, h.atiles);

  // The binning invariant: every slot a pair can touch lies in its segment.
  {
    const int64_t wf = max_slot(p, h.ftiles), wa = max_slot(p, h.atiles);
    if (wf < 0 || wf > p->Lf - 1 || wa < 0 || wa > p->La - 1) return GPAIR_ERR_INVALID_ARG;
  }

  // Far-field precondition: every kernel at least 10 sigma_max from every
  // sensor.  Tile spheres give a lower bound; members are checked one by one
  // only where that bound is below the limit.
  const double near = 10.0 * g->sigma_max;
  // Per tile and sensor: the lower bound of the distances; tiles closer than
  // `near` are checked kernel by kernel.  Split over tiles across threads.
  const int64_t nft = (int64_t)h.ftiles.size();
  const int nth = host_threads();
  std::vector<double> lbt(nth, std::numeric_limits<double>::infinity());
  std::vector<uint8_t> nearf(nth, 0);
  {
    std::vector<std::thread> th;
    for (int t = 0; t < nth; ++t)
      th.emplace_back([&, t] {
        double lbm = std::numeric_limits<double>::infinity();
        for (int64_t ti = nft * t / nth; ti < nft * (t + 1) / nth && !nearf[t]; ++ti) {
          const TileInfo &T = h.ftiles[ti];
          for (int32_t j = 0; j < Nd; ++j) {
            double dx = h.sens[4 * j] - T.cx, dy = h.sens[4 * j + 1] - T.cy,
                   dz = h.sens[4 * j + 2] - T.cz;
            double lb = std::sqrt(dx * dx + dy * dy + dz * dz) - T.rho;
            lbm = std::min(lbm, lb);
            if (lb >= near) continue;
            for (int32_t i = T.start; i < T.start + T.count; ++i) {
              double ex = h.sens[4 * j] - h.kgeo[4 * i], ey = h.sens[4 * j + 1] - h.kgeo[4 * i + 1],
                     ez = h.sens[4 * j + 2] - h.kgeo[4 * i + 2];
              if (!(std::sqrt(ex * ex + ey * ey + ez * ez) >= near)) nearf[t] = 1;
            }
          }
        }
        lbt[t] = lbm;
      });
    for (auto &x : th) x.join();
  }
  double lbmin = std::numeric_limits<double>::infinity();
  for (int t = 0; t < nth; ++t) {
    if (nearf[t]) return GPAIR_ERR_NEAR_FIELD;
    lbmin = std::min(lbmin, lbt[t]);
  }
  p->min_dist = std::max(lbmin, near);

  p->deterministic = g->deterministic ? 1 : 0;
  p->lay = layout_for(M, Nd, h.ftiles.size(), h.atiles.size(),
                      p->deterministic ? (int64_t)Nd * g->n_samples : 0);
  return GPAIR_OK;
}

}  // namespace gpair
