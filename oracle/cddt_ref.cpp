// Plain CPU CDDT: the C++ test oracle (test infrastructure only).
//
// Only the tests, the smoke check and the benchmark's CPU-baseline leg load
// this library.  It shares no source with the GPU library and is written
// straight from Walsh & Karaman, "CDDT: Fast Approximate 2D Ray Casting for
// Accelerated Localization":
//   * Sec. IV-A  direct construction: for every stored theta slice, project each
//                edge-map cell and append its along-ray coordinate to every row
//                ("CDDT bin") its footprint overlaps, then sort each row;
//   * Sec. IV-B  query: project, pick the row, successor search, difference;
//   * Sec. IV-C  theta / theta+pi from one slice (predecessor search), edge map
//                from an 8-neighbour erosion plus the overlap check;
//   * Sec. IV-D  incremental update with revealed-neighbour handling;
//   * Sec. VI    beam sensor model: a particle's log-weight is the sum of the
//                per-ray log-likelihoods (summed here in double, in ray order).
//
// Fixed-point reading (units: 2^-16 cell for along-ray values, 2^-30 for the
// direction, 2^-31 for cell lateral extents, 2^-46 for query lateral values):
//   C[s] = llround(cos(2 pi s / n) 2^30), S[s] = llround(sin(2 pi s / n) 2^30)
//   zero point of cell (i,j):  Z  = ((2i+1) C + (2j+1) S) >> 15
//   its bands:                 [(Yc - Hs) >> 31, (Yc + Hs - 1) >> 31],
//                              Yc = (2j+1) C - (2i+1) S, Hs = |C| + |S|
//   query:                     xf = floor(x 2^16), yf = floor(y 2^16),
//                              k = floor(fl(fl(theta K) + 0.5)) mod n, K = (float)(n / 2 pi)
//                              Xq = (xf C + yf S) >> 30, r = (yf C - xf S) >> 46
//   range:                     min(M, (|Z - Xq| + 2^15) >> 16), M when no zero point.
// Right shifts of negative values are arithmetic (floor), as C++20 defines.
//
// 16-bit reading (Sec. IV-C suggests 16-bit zero points at a small precision
// loss): every zero point Z of slice s is replaced by the centre of its
// 1/8-cell bin, zlo + 8192 floor((Z - zlo) / 8192) + 4096, where zlo is the
// lowest projection of the map rectangle, (min(0, W 2^16 C) + min(0, H 2^16 S))
// >> 30; queries, ranges and updates then proceed unchanged on those values.
//
// PCDDT reading (Sec. IV-C, pruning: cast from every state, drop every zero
// point no cast returns): the states are the centres (i + 1/2, j + 1/2) of the
// free cells under every theta bin, each bin at its centre angle 2 pi k / n.
// A state of bin s < n/2 returns the successor of its Xq in its band of slice
// s, one of bin s + n/2 the predecessor, so a pruned band holds the distinct
// values that some state returns, ascending.  Casts from those states answer
// as on the unpruned structure; other queries may see past a dropped point.
// An update of a pruned map rebuilds and prunes again from the new grid (the
// paper leaves incremental edits of a pruned structure open).
//
// Build: g++ -std=c++17 -O2 -ffp-contract=off -shared -fPIC -pthread
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <set>
#include <thread>
#include <tuple>
#include <vector>

namespace {

struct Slice {
  int64_t c, s;
  int64_t row_min;
  int64_t nrows;
  int64_t zlo;  // lowest along-slice projection of the map rectangle (16-bit reading)
  std::vector<std::vector<int32_t>> rows;
};

struct RefMap {
  int w, h, n;
  bool full;
  bool zp16;   // zero points rounded to 1/8-cell bins (the 16-bit reading)
  bool prune;  // PCDDT: only the zero points some discrete state's cast returns
  std::vector<uint8_t> occ;
  std::vector<Slice> slices;
  float k_scale;
  std::vector<int32_t> edge_i, edge_j;  // edge-map cells (brute-force scan)
};

bool occupied(const RefMap& m, int i, int j) {
  return m.occ[(size_t)j * m.w + i] != 0;
}

bool cell_is_edge(const std::vector<uint8_t>& occ, int w, int h, int i, int j, bool full) {
  if (occ[(size_t)j * w + i] == 0) return false;
  if (full) return true;
  for (int dj = -1; dj <= 1; ++dj)
    for (int di = -1; di <= 1; ++di) {
      if (!di && !dj) continue;
      int a = i + di, b = j + dj;
      if (a < 0 || b < 0 || a >= w || b >= h) return true;  // off-map counts as free
      if (occ[(size_t)b * w + a] == 0) return true;
    }
  return false;
}

int32_t zero_point(int64_t i, int64_t j, int64_t c, int64_t s) {
  return (int32_t)(((2 * i + 1) * c + (2 * j + 1) * s) >> 15);
}

void bands(int64_t i, int64_t j, int64_t c, int64_t s, int64_t* lo, int64_t* hi) {
  int64_t yc = (2 * j + 1) * c - (2 * i + 1) * s;
  int64_t hs = std::llabs(c) + std::llabs(s);
  *lo = (yc - hs) >> 31;
  *hi = (yc + hs - 1) >> 31;
}

// The stored zero point: exact, or under the 16-bit reading the centre of its
// 1/8-cell bin counted from the slice's lowest projection zlo.
int32_t stored_point(const RefMap& m, const Slice& sl, int64_t i, int64_t j) {
  const int32_t z = zero_point(i, j, sl.c, sl.s);
  if (!m.zp16) return z;
  const int64_t b = ((int64_t)z - sl.zlo) >> 13;
  return (int32_t)(sl.zlo + b * 8192 + 4096);
}

void touch(RefMap& m, int sidx, int i, int j, int sign) {
  Slice& sl = m.slices[sidx];
  int32_t z = stored_point(m, sl, i, j);
  int64_t lo, hi;
  bands(i, j, sl.c, sl.s, &lo, &hi);
  for (int64_t r = lo; r <= hi; ++r) {
    std::vector<int32_t>& row = sl.rows[(size_t)(r - sl.row_min)];
    if (sign > 0) {
      row.insert(std::upper_bound(row.begin(), row.end(), z), z);
    } else {
      auto it = std::lower_bound(row.begin(), row.end(), z);
      if (it == row.end() || *it != z) std::abort();  // structure inconsistent with the map
      row.erase(it);
    }
  }
}

void build_slice(RefMap& m, int sidx, const std::vector<int32_t>& ci, const std::vector<int32_t>& cj) {
  Slice& sl = m.slices[sidx];
  sl.rows.assign((size_t)sl.nrows, {});
  for (size_t e = 0; e < ci.size(); ++e) {  // every edge cell, appended to each band it covers
    int32_t z = stored_point(m, sl, ci[e], cj[e]);
    int64_t lo, hi;
    bands(ci[e], cj[e], sl.c, sl.s, &lo, &hi);
    for (int64_t r = lo; r <= hi; ++r) sl.rows[(size_t)(r - sl.row_min)].push_back(z);
  }
  for (auto& row : sl.rows) std::sort(row.begin(), row.end());
}

void collect_edges(RefMap& m) {
  m.edge_i.clear();
  m.edge_j.clear();
  for (int j = 0; j < m.h; ++j)
    for (int i = 0; i < m.w; ++i)
      if (cell_is_edge(m.occ, m.w, m.h, i, j, m.full)) {
        m.edge_i.push_back(i);
        m.edge_j.push_back(j);
      }
}

template <class F>
void parallel_for(int64_t n, int threads, F f) {
  if (threads <= 1 || n < 2) {
    f((int64_t)0, n);
    return;
  }
  std::vector<std::thread> pool;
  int64_t chunk = (n + threads - 1) / threads;
  for (int t = 0; t < threads; ++t) {
    int64_t a = t * chunk, b = std::min(n, a + chunk);
    if (a >= b) break;
    pool.emplace_back([=] { f(a, b); });
  }
  for (auto& th : pool) th.join();
}

struct Prepared {
  bool valid;
  int sidx, sigma;
  int64_t xq, r;
};

Prepared prepare(const RefMap& m, float x, float y, float theta) {
  Prepared p{false, 0, 1, 0, 0};
  if (!(std::fabs(theta) < 1e6f)) return p;
  if (!(x >= 0.0f && x < (float)m.w && y >= 0.0f && y < (float)m.h)) return p;
  volatile float sx = x * 65536.0f, sy = y * 65536.0f;
  int64_t xf = (int64_t)std::floor((float)sx);
  int64_t yf = (int64_t)std::floor((float)sy);
  if (occupied(m, (int)(xf >> 16), (int)(yf >> 16))) return p;
  volatile float t = theta * m.k_scale;  // volatile: each float op rounds on its own
  volatile float u = t + 0.5f;
  int64_t k = (int64_t)std::floor((float)u);
  k %= m.n;
  if (k < 0) k += m.n;
  int half = m.n / 2;
  p.sidx = (int)(k % half);
  p.sigma = k < half ? 1 : -1;
  const Slice& sl = m.slices[p.sidx];
  p.xq = (xf * sl.c + yf * sl.s) >> 30;
  p.r = (yf * sl.c - xf * sl.s) >> 46;
  p.valid = true;
  return p;
}

int32_t finish(bool found, int64_t d, int32_t max_range) {
  if (!found) return max_range;
  int64_t v = (d + 32768) >> 16;
  return (int32_t)std::min<int64_t>(max_range, v);
}

// The zero point a valid query's cast returns (Sec. IV-B: successor, or with
// the theta + pi symmetry of Sec. IV-C predecessor); false when there is none.
bool cast_search(const RefMap& m, const Prepared& p, int32_t* z) {
  const Slice& sl = m.slices[p.sidx];
  const std::vector<int32_t>& row = sl.rows[(size_t)(p.r - sl.row_min)];
  if (p.sigma > 0) {
    auto it = std::upper_bound(row.begin(), row.end(), (int32_t)p.xq);
    if (it == row.end()) return false;
    *z = *it;
    return true;
  }
  auto it = std::lower_bound(row.begin(), row.end(), (int32_t)p.xq);
  if (it == row.begin()) return false;
  *z = *(it - 1);
  return true;
}

int32_t cast_cddt(const RefMap& m, float x, float y, float theta, int32_t max_range) {
  Prepared p = prepare(m, x, y, theta);
  if (!p.valid) return 0;
  int32_t z = 0;
  if (!cast_search(m, p, &z)) return max_range;
  return finish(true, p.sigma > 0 ? (int64_t)z - p.xq : p.xq - (int64_t)z, max_range);
}

// PCDDT: cast from every state whose bin is s or s + n/2 (the two directions
// stored in slice s), collect the zero points returned per band, and keep
// only those (distinct, ascending).
void prune_slice(RefMap& m, int sidx) {
  Slice& sl = m.slices[sidx];
  std::vector<std::vector<int32_t>> used(sl.rows.size());
  for (int k : {sidx, sidx + m.n / 2}) {
    const float theta = (float)(2.0 * M_PI * k / m.n);
    for (int j = 0; j < m.h; ++j)
      for (int i = 0; i < m.w; ++i) {
        if (occupied(m, i, j)) continue;
        const Prepared p = prepare(m, (float)i + 0.5f, (float)j + 0.5f, theta);
        if (!p.valid || p.sidx != sidx || (p.sigma > 0) != (k == sidx)) std::abort();  // state outside its bin
        int32_t z = 0;
        if (cast_search(m, p, &z)) used[(size_t)(p.r - sl.row_min)].push_back(z);
      }
  }
  for (size_t b = 0; b < used.size(); ++b) {
    std::vector<int32_t>& u = used[b];
    std::sort(u.begin(), u.end());
    u.erase(std::unique(u.begin(), u.end()), u.end());
  }
  sl.rows.swap(used);
}

void build_all(RefMap& m, int threads) {
  const int half = m.n / 2;
  collect_edges(m);
  parallel_for(half, threads, [&](int64_t a, int64_t b) {
    for (int64_t s = a; s < b; ++s) build_slice(m, (int)s, m.edge_i, m.edge_j);
  });
  if (m.prune)
    parallel_for(half, threads, [&](int64_t a, int64_t b) {
      for (int64_t s = a; s < b; ++s) prune_slice(m, (int)s);
    });
}

int32_t cast_brute(const RefMap& m, float x, float y, float theta, int32_t max_range) {
  Prepared p = prepare(m, x, y, theta);
  if (!p.valid) return 0;
  const Slice& sl = m.slices[p.sidx];
  bool found = false;
  int64_t best = 0;
  for (size_t e = 0; e < m.edge_i.size(); ++e) {
    int64_t lo, hi;
    bands(m.edge_i[e], m.edge_j[e], sl.c, sl.s, &lo, &hi);
    if (p.r < lo || p.r > hi) continue;
    int64_t z = zero_point(m.edge_i[e], m.edge_j[e], sl.c, sl.s);
    if (p.sigma > 0 && z > p.xq && (!found || z < best)) { best = z; found = true; }
    if (p.sigma < 0 && z < p.xq && (!found || z > best)) { best = z; found = true; }
  }
  return finish(found, p.sigma > 0 ? best - p.xq : p.xq - best, max_range);
}

}  // namespace

extern "C" {

void* ref_create(const uint8_t* occ, int32_t w, int32_t h, int32_t n, int32_t full_map, int32_t threads,
                 int32_t zp16, int32_t prune) {
  if (w < 1 || h < 1 || n < 2 || (n & 1)) return nullptr;
  if (zp16 && prune) return nullptr;  // the two readings are not combined
  RefMap* m = new RefMap();
  m->w = w;
  m->h = h;
  m->n = n;
  m->full = full_map != 0;
  m->zp16 = zp16 != 0;
  m->prune = prune != 0;
  m->occ.assign(occ, occ + (size_t)w * h);
  m->k_scale = (float)((double)n / (2.0 * M_PI));
  int half = n / 2;
  m->slices.resize(half);
  for (int s = 0; s < half; ++s) {
    double a = 2.0 * M_PI * s / n;
    Slice& sl = m->slices[s];
    sl.c = std::llround(std::cos(a) * 1073741824.0);
    sl.s = std::llround(std::sin(a) * 1073741824.0);
    {
      const int64_t wc = ((int64_t)w << 16) * sl.c, hs = ((int64_t)h << 16) * sl.s;
      sl.zlo = (std::min<int64_t>(0, wc) + std::min<int64_t>(0, hs)) >> 30;
    }
    int64_t lo = INT64_MAX, hi = INT64_MIN;
    for (int64_t X : {(int64_t)0, (int64_t)w})
      for (int64_t Y : {(int64_t)0, (int64_t)h}) {
        int64_t v = (Y * sl.c - X * sl.s) >> 30;
        lo = std::min(lo, v);
        hi = std::max(hi, v);
      }
    sl.row_min = lo;
    sl.nrows = hi - lo + 1;
  }
  build_all(*m, threads);
  return m;
}

void ref_destroy(void* h) { delete static_cast<RefMap*>(h); }

int64_t ref_edge_count(void* h) { return (int64_t) static_cast<RefMap*>(h)->edge_i.size(); }

void ref_tables(void* h, int64_t* c, int64_t* s, int64_t* row_min, int64_t* nrows, float* k_scale) {
  RefMap* m = static_cast<RefMap*>(h);
  for (int i = 0; i < m->n / 2; ++i) {
    c[i] = m->slices[i].c;
    s[i] = m->slices[i].s;
    row_min[i] = m->slices[i].row_min;
    nrows[i] = m->slices[i].nrows;
  }
  *k_scale = m->k_scale;
}

void ref_sizes(void* h, int64_t* total_rows, int64_t* total_zeros, int64_t* max_row) {
  RefMap* m = static_cast<RefMap*>(h);
  int64_t r = 0, z = 0, mx = 0;
  for (auto& sl : m->slices)
    for (auto& row : sl.rows) {
      ++r;
      z += (int64_t)row.size();
      mx = std::max<int64_t>(mx, (int64_t)row.size());
    }
  *total_rows = r;
  *total_zeros = z;
  *max_row = mx;
}

// Canonical CSR: rows in (slice, band) order, each ascending.
void ref_export(void* h, int32_t* row_len, int32_t* zeros) {
  RefMap* m = static_cast<RefMap*>(h);
  int64_t r = 0, z = 0;
  for (auto& sl : m->slices)
    for (auto& row : sl.rows) {
      row_len[r++] = (int32_t)row.size();
      for (int32_t v : row) zeros[z++] = v;
    }
}

void ref_cast(void* h, const float* x, const float* y, const float* th, int64_t n, int32_t max_range,
              int32_t* out, int32_t threads) {
  const RefMap& m = *static_cast<RefMap*>(h);
  parallel_for(n, threads, [&](int64_t a, int64_t b) {
    for (int64_t i = a; i < b; ++i) out[i] = cast_cddt(m, x[i], y[i], th[i], max_range);
  });
}

void ref_cast_bruteforce(void* h, const float* x, const float* y, const float* th, int64_t n,
                         int32_t max_range, int32_t* out, int32_t threads) {
  const RefMap& m = *static_cast<RefMap*>(h);
  parallel_for(n, threads, [&](int64_t a, int64_t b) {
    for (int64_t i = a; i < b; ++i) out[i] = cast_brute(m, x[i], y[i], th[i], max_range);
  });
}

// Beam sensor model: per particle, sum over rays of log_table[clamp(obs)][range] in double.
void ref_weight(void* h, const float* px, const float* py, const float* pth, int64_t n_particles,
                const float* offsets, const int32_t* obs, int32_t n_rays, const float* log_table,
                int32_t max_range, double* logw, int32_t* ranges, int32_t threads) {
  const RefMap& m = *static_cast<RefMap*>(h);
  const int64_t m1 = (int64_t)max_range + 1;
  parallel_for(n_particles, threads, [&](int64_t a, int64_t b) {
    for (int64_t p = a; p < b; ++p) {
      double acc = 0.0;
      for (int32_t r = 0; r < n_rays; ++r) {
        volatile float th = pth[p] + offsets[r];
        int32_t d = cast_cddt(m, px[p], py[p], th, max_range);
        int64_t z = std::min<int64_t>(std::max<int64_t>(obs[r], 0), max_range);
        acc += (double)log_table[z * m1 + d];
        if (ranges) ranges[p * n_rays + r] = d;
      }
      logw[p] = acc;
    }
  });
}

// Sec. IV-D: ops in array order (last write per cell wins).  Cells within one
// step of a changed cell may change edge status; each flip removes or inserts
// that cell's zero points in every slice.  Returns -1 if an op is off the map.
int32_t ref_update(void* h, const int32_t* xs, const int32_t* ys, const uint8_t* vals, int64_t n_ops) {
  RefMap& m = *static_cast<RefMap*>(h);
  for (int64_t k = 0; k < n_ops; ++k)
    if (xs[k] < 0 || ys[k] < 0 || xs[k] >= m.w || ys[k] >= m.h) return -1;
  std::vector<uint8_t> next = m.occ;
  for (int64_t k = 0; k < n_ops; ++k) next[(size_t)ys[k] * m.w + xs[k]] = vals[k] ? 1 : 0;
  std::set<std::pair<int, int>> cand;
  for (int64_t k = 0; k < n_ops; ++k) {
    int i = xs[k], j = ys[k];
    if (next[(size_t)j * m.w + i] == m.occ[(size_t)j * m.w + i]) continue;
    for (int dj = -1; dj <= 1; ++dj)
      for (int di = -1; di <= 1; ++di) {
        int a = i + di, b = j + dj;
        if (a >= 0 && b >= 0 && a < m.w && b < m.h) cand.insert({b, a});
      }
  }
  std::vector<std::tuple<int, int, int>> flips;  // (i, j, +1 insert / -1 remove)
  for (auto& c : cand) {
    bool was = cell_is_edge(m.occ, m.w, m.h, c.second, c.first, m.full);
    bool now = cell_is_edge(next, m.w, m.h, c.second, c.first, m.full);
    if (was != now) flips.emplace_back(c.second, c.first, now ? 1 : -1);
  }
  m.occ.swap(next);
  if (m.prune) {  // PCDDT: rebuild and prune from the new grid
    build_all(m, 1);
    return (int32_t)flips.size();
  }
  for (auto& f : flips)
    if (std::get<2>(f) < 0)
      for (int s = 0; s < m.n / 2; ++s) touch(m, s, std::get<0>(f), std::get<1>(f), -1);
  for (auto& f : flips)
    if (std::get<2>(f) > 0)
      for (int s = 0; s < m.n / 2; ++s) touch(m, s, std::get<0>(f), std::get<1>(f), +1);
  collect_edges(m);
  return (int32_t)flips.size();
}

}  // extern "C"
