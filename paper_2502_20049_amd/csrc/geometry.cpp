// Host-side geometry field construction (run once per body, section III: the
// body-frame field is built on the host a single time and copied to the
// device once; only its mapping runs every step).
//
// Geometry lattice: spacing h = 2^-s LBM cells in the body frame, cell m has
// its centre at (m + 1/2) h; a bit is set when that centre is inside the
// object.  Meshes use the nonzero-winding rule evaluated along +x rays: per
// (y, z) row of centres, crossings of the row line with the triangles are
// collected (half-open edge rule in the y-z projection), sorted, and the
// signed crossing count left of each centre is its winding number.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <thread>
#include <vector>

#include "psm_internal.hpp"

namespace psm {

namespace {

template <typename F>
void parallel_rows(int64_t n, F &&fn) {
  unsigned nt = std::thread::hardware_concurrency();
  if (nt == 0) nt = 1;
  if (nt > 32) nt = 32;
  if (n < 64) nt = 1;
  std::vector<std::thread> th;
  const int64_t chunk = (n + nt - 1) / nt;
  for (unsigned t = 0; t < nt; ++t) {
    const int64_t lo = (int64_t)t * chunk, hi = std::min<int64_t>(n, lo + chunk);
    if (lo >= hi) break;
    th.emplace_back([&, lo, hi] {
      for (int64_t i = lo; i < hi; ++i) fn(i);
    });
  }
  for (auto &t : th) t.join();
}

inline int64_t words_x(const int32_t dims[3]) { return (dims[0] + 31) / 32; }

}  // namespace

int geom_box(int kind, const double *params, const double *verts, int64_t nv, int s, int32_t mmin[3],
             int32_t dims[3]) {
  double lo[3], hi[3];
  if (verts) {
    if (nv <= 0) return PSM_EINVAL;
    for (int a = 0; a < 3; ++a) lo[a] = hi[a] = verts[a];
    for (int64_t i = 1; i < nv; ++i)
      for (int a = 0; a < 3; ++a) {
        lo[a] = std::min(lo[a], verts[3 * i + a]);
        hi[a] = std::max(hi[a], verts[3 * i + a]);
      }
  } else if (kind == PSM_SHAPE_ELLIPSOID) {
    for (int a = 0; a < 3; ++a) {
      if (!(params[a] > 0)) return PSM_EINVAL;
      lo[a] = -params[a];
      hi[a] = params[a];
    }
  } else if (kind == PSM_SHAPE_CUBE) {
    if (!(params[0] > 0)) return PSM_EINVAL;
    for (int a = 0; a < 3; ++a) {
      lo[a] = -params[0];
      hi[a] = params[0];
    }
  } else {
    return PSM_EINVAL;
  }
  const double sc = ldexp(1.0, s);
  for (int a = 0; a < 3; ++a) {
    // body-frame bounding box plus one LBM cell of padding
    const double m0 = floor((lo[a] - 1.0) * sc), m1 = ceil((hi[a] + 1.0) * sc);
    if (!(m1 - m0 < 2147483647.0)) return PSM_EUNSUP;
    mmin[a] = (int32_t)m0;
    dims[a] = (int32_t)(m1 - m0);
  }
  return PSM_OK;
}

void analytic_rows(int kind, const double *params, int s, const int32_t mmin[3], const int32_t dims[3],
                   uint32_t *bits) {
  const int64_t wx = words_x(dims);
  const int64_t rows = (int64_t)dims[1] * dims[2];
  memset(bits, 0, sizeof(uint32_t) * wx * rows);
  parallel_rows(rows, [&](int64_t r) {
    const int64_t jy = r % dims[1], jz = r / dims[1];
    uint32_t *row = bits + r * wx;
    const double Cy = (double)(2 * ((int64_t)mmin[1] + jy) + 1), Cz = (double)(2 * ((int64_t)mmin[2] + jz) + 1);
    for (int64_t jx = 0; jx < dims[0]; ++jx) {
      const double Cx = (double)(2 * ((int64_t)mmin[0] + jx) + 1);
      bool in;
      if (kind == PSM_SHAPE_ELLIPSOID) {
        // centre C h/2 inside (x/a)^2+(y/b)^2+(z/c)^2 < 1, scaled to integers
        const double a2 = params[0] * params[0], b2 = params[1] * params[1], c2 = params[2] * params[2];
        const double lhs = (Cx * Cx * (b2 * c2) + Cy * Cy * (a2 * c2)) + Cz * Cz * (a2 * b2);
        const double rhs = ldexp(1.0, 2 * (s + 1)) * (a2 * b2 * c2);
        in = lhs < rhs;
      } else {
        const double lim = ldexp(params[0], s + 1);
        in = fabs(Cx) < lim && fabs(Cy) < lim && fabs(Cz) < lim;
      }
      if (in) row[jx >> 5] |= 1u << (jx & 31);
    }
  });
}

void voxelize_rows(const double *V, const int32_t *T, int64_t nt, int s, const int32_t mmin[3],
                   const int32_t dims[3], uint32_t *bits) {
  const double h = ldexp(1.0, -s);
  const int64_t wx = words_x(dims);
  const int64_t ny = dims[1], nz = dims[2];
  const int64_t rows = ny * nz;
  memset(bits, 0, sizeof(uint32_t) * wx * rows);
  // bin triangles over the rows their y-z bounding box covers
  std::vector<int64_t> cnt(rows + 1, 0);
  auto row_range = [&](int64_t t, int64_t &y0, int64_t &y1, int64_t &z0, int64_t &z1) {
    double ylo = 1e300, yhi = -1e300, zlo = 1e300, zhi = -1e300;
    for (int c = 0; c < 3; ++c) {
      const double *p = V + 3 * (int64_t)T[3 * t + c];
      ylo = std::min(ylo, p[1]);
      yhi = std::max(yhi, p[1]);
      zlo = std::min(zlo, p[2]);
      zhi = std::max(zhi, p[2]);
    }
    // row centre (mmin + j + 1/2) h within [lo, hi]
    y0 = std::max<int64_t>(0, (int64_t)ceil(ylo / h - 0.5) - mmin[1]);
    y1 = std::min<int64_t>(ny - 1, (int64_t)floor(yhi / h - 0.5) - mmin[1]);
    z0 = std::max<int64_t>(0, (int64_t)ceil(zlo / h - 0.5) - mmin[2]);
    z1 = std::min<int64_t>(nz - 1, (int64_t)floor(zhi / h - 0.5) - mmin[2]);
  };
  for (int64_t t = 0; t < nt; ++t) {
    int64_t y0, y1, z0, z1;
    row_range(t, y0, y1, z0, z1);
    for (int64_t z = z0; z <= z1; ++z)
      for (int64_t y = y0; y <= y1; ++y) ++cnt[z * ny + y + 1];
  }
  for (int64_t r = 0; r < rows; ++r) cnt[r + 1] += cnt[r];
  std::vector<int32_t> lst(cnt[rows]);
  {
    std::vector<int64_t> pos(cnt.begin(), cnt.end() - 1);
    for (int64_t t = 0; t < nt; ++t) {
      int64_t y0, y1, z0, z1;
      row_range(t, y0, y1, z0, z1);
      for (int64_t z = z0; z <= z1; ++z)
        for (int64_t y = y0; y <= y1; ++y) lst[pos[z * ny + y]++] = (int32_t)t;
    }
  }
  parallel_rows(rows, [&](int64_t r) {
    const int64_t b = cnt[r], e = cnt[r + 1];
    if (b == e) return;
    const int64_t jy = r % ny, jz = r / ny;
    const double py = ((double)(mmin[1] + jy) + 0.5) * h, pz = ((double)(mmin[2] + jz) + 0.5) * h;
    std::vector<std::pair<double, int>> hits;
    for (int64_t i = b; i < e; ++i) {
      const int64_t t = lst[i];
      const double *A = V + 3 * (int64_t)T[3 * t], *B = V + 3 * (int64_t)T[3 * t + 1], *C = V + 3 * (int64_t)T[3 * t + 2];
      // projected signed area (y-z plane); orientation sign decides entry/exit
      const double area = (B[1] - A[1]) * (C[2] - A[2]) - (B[2] - A[2]) * (C[1] - A[1]);
      if (area == 0.0) continue;
      int id[3] = {T[3 * t], T[3 * t + 1], T[3 * t + 2]};
      if (area < 0) std::swap(id[1], id[2]);
      bool inside = true;
      for (int k = 0; k < 3 && inside; ++k) {
        // edge function evaluated from the lower vertex index, so that the two
        // triangles sharing an edge see exactly opposite values
        int iu = id[k], iv = id[(k + 1) % 3];
        const bool flip = iu > iv;
        if (flip) std::swap(iu, iv);
        const double *u = V + 3 * (int64_t)iu, *v = V + 3 * (int64_t)iv;
        double e = (v[1] - u[1]) * (pz - u[2]) - (v[2] - u[2]) * (py - u[1]);
        double dy = v[1] - u[1], dz = v[2] - u[2];
        if (flip) {
          e = -e;
          dy = -dy;
          dz = -dz;
        }
        if (e > 0) continue;
        if (e < 0) {
          inside = false;
          continue;
        }
        // on the edge line: half-open rule keyed on the edge direction
        inside = (dz < 0) || (dz == 0 && dy > 0);
      }
      if (!inside) continue;
      // x of the plane through A, B, C at (py, pz)
      const double nx = (B[1] - A[1]) * (C[2] - A[2]) - (B[2] - A[2]) * (C[1] - A[1]);
      const double nyv = (B[2] - A[2]) * (C[0] - A[0]) - (B[0] - A[0]) * (C[2] - A[2]);
      const double nzv = (B[0] - A[0]) * (C[1] - A[1]) - (B[1] - A[1]) * (C[0] - A[0]);
      const double xh = A[0] - (nyv * (py - A[1]) + nzv * (pz - A[2])) / nx;
      hits.emplace_back(xh, nx < 0 ? 1 : -1);  // outward normal against +x: entering
    }
    if (hits.empty()) return;
    std::sort(hits.begin(), hits.end());
    uint32_t *row = bits + r * wx;
    int w = 0;
    size_t hi_ = 0;
    for (int64_t jx = 0; jx < dims[0]; ++jx) {
      const double px = ((double)(mmin[0] + jx) + 0.5) * h;
      while (hi_ < hits.size() && hits[hi_].first < px) w += hits[hi_++].second;
      if (w != 0) row[jx >> 5] |= 1u << (jx & 31);
    }
  });
}

void coarse_extent(int s, const int32_t mmin[3], const int32_t dims[3], int32_t cmin[3], int32_t cdims[3]) {
  for (int a = 0; a < 3; ++a) {
    const int64_t lo = (int64_t)mmin[a] >> s;  // floor division by 2^s
    const int64_t hi = ((int64_t)mmin[a] + dims[a] - 1) >> s;
    cmin[a] = (int32_t)lo;
    cdims[a] = (int32_t)(hi - lo + 1);
  }
}

void coarse_map(int s, const int32_t mmin[3], const int32_t dims[3], const uint32_t *bits, int32_t cmin[3],
                int32_t cdims[3], uint8_t *out) {
  coarse_extent(s, mmin, dims, cmin, cdims);
  const int64_t wx = words_x(dims);
  const int64_t n = 1 << s;
  const int64_t nblk = (int64_t)cdims[0] * cdims[1] * cdims[2];
  parallel_rows((int64_t)cdims[1] * cdims[2], [&](int64_t r) {
    const int64_t by = r % cdims[1] + cmin[1], bz = r / cdims[1] + cmin[2];
    for (int64_t bx = cmin[0]; bx < cmin[0] + cdims[0]; ++bx) {
      int st = -1;
      for (int64_t kz = 0; kz < n && st != 2; ++kz)
        for (int64_t ky = 0; ky < n && st != 2; ++ky)
          for (int64_t kx = 0; kx < n && st != 2; ++kx) {
            const int64_t jx = bx * n + kx - mmin[0], jy = by * n + ky - mmin[1], jz = bz * n + kz - mmin[2];
            int v = 0;
            if (jx >= 0 && jy >= 0 && jz >= 0 && jx < dims[0] && jy < dims[1] && jz < dims[2])
              v = (bits[(jz * dims[1] + jy) * wx + (jx >> 5)] >> (jx & 31)) & 1;
            st = st < 0 ? v : (st == v ? st : 2);
          }
      out[(r)*cdims[0] + (bx - cmin[0])] = (uint8_t)st;
    }
  });
  // bit 2: the block and its 26 neighbours (outside the box: all out) share
  // one uniform state, so a cell whose centre lies in the block is decided by
  // that block alone (its sub-samples stay within one block of the centre)
  std::vector<uint8_t> st(out, out + nblk);
  auto at = [&](int64_t x, int64_t y, int64_t z) -> int {
    if (x < 0 || y < 0 || z < 0 || x >= cdims[0] || y >= cdims[1] || z >= cdims[2]) return 0;
    return st[(z * cdims[1] + y) * cdims[0] + x];
  };
  parallel_rows((int64_t)cdims[1] * cdims[2], [&](int64_t r) {
    const int64_t y = r % cdims[1], z = r / cdims[1];
    for (int64_t x = 0; x < cdims[0]; ++x) {
      const int v = at(x, y, z);
      bool uni = v != 2;
      for (int dz = -1; dz <= 1 && uni; ++dz)
        for (int dy = -1; dy <= 1 && uni; ++dy)
          for (int dx = -1; dx <= 1 && uni; ++dx) uni = at(x + dx, y + dy, z + dz) == v;
      if (uni) out[r * cdims[0] + x] = (uint8_t)(v | 4);
    }
  });
}

}  // namespace psm
