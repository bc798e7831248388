// Seeded synthetic vessel geometries for the sparse D3Q19 lattice-Boltzmann update.
//
// This file builds INPUTS only: which voxels of a box are fluid, the list of
// fluid sites, their site types and the push-direction neighbour table
// (nbr[x][i] = id of the site at x + c_i, or a boundary code).  It holds no
// part of the lattice-Boltzmann arithmetic (no equilibrium, collision or
// boundary rule); both the CPU oracle and the GPU library consume its output.
//
// Velocity set and its order (the input convention of the neighbour table):
// the D3Q19 set of the paper's Sec. 2.2, ordered so that opposite directions
// are adjacent (i odd, i+1 is its opposite).
//
// Boundary link codes: -1 = wall, -(2+k) = iolet k (inlet/outlet k).
// Site types (paper Sec. 3.2.2): 0 bulk, 1 wall, 2 inlet, 3 outlet,
// 4 inlet+wall, 5 outlet+wall.
//
// Plain C ABI so that Python can call it through ctypes.

#include <cstdint>
#include <cstring>
#include <cmath>
#include <vector>
#include <algorithm>
#include <omp.h>

namespace {

const int CX[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
const int CY[19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
const int CZ[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};

inline bool bit_get(const uint64_t *b, int64_t v) { return (b[v >> 6] >> (v & 63)) & 1ull; }

struct Box {
  int64_t nx, ny, nz;
  int px, py, pz;  // periodic flags
  int64_t nvox() const { return nx * ny * nz; }
};

// Map (x,y,z) (possibly outside the box) to a voxel index, honouring
// periodicity; returns -1 when the point is outside a non-periodic face.
inline int64_t vox_index(const Box &B, int64_t x, int64_t y, int64_t z) {
  if (x < 0 || x >= B.nx) { if (!B.px) return -1; x = ((x % B.nx) + B.nx) % B.nx; }
  if (y < 0 || y >= B.ny) { if (!B.py) return -1; y = ((y % B.ny) + B.ny) % B.ny; }
  if (z < 0 || z >= B.nz) { if (!B.pz) return -1; z = ((z % B.nz) + B.nz) % B.nz; }
  return (z * B.ny + y) * B.nx + x;
}

}  // namespace

extern "C" {

// Number of set bits in a voxel bitmap of nvox voxels.
int64_t gm_count(const uint64_t *bits, int64_t nvox) {
  int64_t nw = (nvox + 63) / 64, s = 0;
#pragma omp parallel for reduction(+ : s) schedule(static)
  for (int64_t w = 0; w < nw; ++w) s += __builtin_popcountll(bits[w]);
  return s;
}

// Voxelise a union of capsules (segment a->b, radius r) into the bitmap of a
// box of nx*ny*nz voxels whose voxel (0,0,0) sits at `origin` in the
// capsules' coordinates.  cut_a[s] != 0 removes the half-space behind a
// (flat end at a, normal along b-a); cut_b[s] != 0 removes the half-space
// beyond b.  A voxel is fluid if it lies inside at least one (cut) capsule.
// The bitmap must be zeroed by the caller; bits are only set.
void gm_capsules(int64_t nseg, const double *a, const double *b, const double *r,
                 const int32_t *cut_a, const int32_t *cut_b, int64_t nx, int64_t ny,
                 int64_t nz, const double *origin, uint64_t *bits) {
  // Work over z-slabs so that no two threads write the same 64-bit word:
  // a word never spans two (y,z) rows when nx is a multiple of 64; otherwise
  // use atomics.
  const bool row_aligned = (nx % 64) == 0;
  for (int64_t s = 0; s < nseg; ++s) {
    const double ax = a[3 * s] - origin[0], ay = a[3 * s + 1] - origin[1], az = a[3 * s + 2] - origin[2];
    const double bx = b[3 * s] - origin[0], by = b[3 * s + 1] - origin[1], bz = b[3 * s + 2] - origin[2];
    const double rr = r[s];
    const double dx = bx - ax, dy = by - ay, dz = bz - az;
    const double len2 = dx * dx + dy * dy + dz * dz;
    int64_t x0 = (int64_t)std::floor(std::min(ax, bx) - rr) - 1, x1 = (int64_t)std::ceil(std::max(ax, bx) + rr) + 1;
    int64_t y0 = (int64_t)std::floor(std::min(ay, by) - rr) - 1, y1 = (int64_t)std::ceil(std::max(ay, by) + rr) + 1;
    int64_t z0 = (int64_t)std::floor(std::min(az, bz) - rr) - 1, z1 = (int64_t)std::ceil(std::max(az, bz) + rr) + 1;
    x0 = std::max<int64_t>(x0, 0); y0 = std::max<int64_t>(y0, 0); z0 = std::max<int64_t>(z0, 0);
    x1 = std::min<int64_t>(x1, nx - 1); y1 = std::min<int64_t>(y1, ny - 1); z1 = std::min<int64_t>(z1, nz - 1);
    const int ca = cut_a ? cut_a[s] : 0, cb = cut_b ? cut_b[s] : 0;
#pragma omp parallel for collapse(2) schedule(dynamic, 4)
    for (int64_t z = z0; z <= z1; ++z) {
      for (int64_t y = y0; y <= y1; ++y) {
        for (int64_t x = x0; x <= x1; ++x) {
          const double px = x - ax, py = y - ay, pz = z - az;
          const double t = (px * dx + py * dy + pz * dz) / len2;  // position along the axis
          if (ca && t < 0.0) continue;
          if (cb && t > 1.0) continue;
          const double tc = t < 0.0 ? 0.0 : (t > 1.0 ? 1.0 : t);
          const double qx = px - tc * dx, qy = py - tc * dy, qz = pz - tc * dz;
          if (qx * qx + qy * qy + qz * qz < rr * rr) {
            const int64_t v = (z * ny + y) * nx + x;
            const uint64_t m = 1ull << (v & 63);
            if (row_aligned) {
              bits[v >> 6] |= m;  // rows of this thread own their words
            } else {
#pragma omp atomic
              bits[v >> 6] |= m;
            }
          }
        }
      }
    }
  }
}

// Build the sparse site list of a voxel bitmap.
//  periodic[3]: wrap flags per axis.
//  Iolet k: plane through centre[k] with unit normal normal[k] pointing into
//  the fluid, disk radius radius[k] (<= 0: unbounded), role[k] (0 inlet,
//  1 outlet).  A link x -> y with y not fluid is an iolet link of the first
//  k for which x is on the fluid side of plane k, y is strictly behind it,
//  and y lies within radius[k] + sqrt(2) of the iolet axis; every other
//  link to a non-fluid point is a wall link.
// Outputs (caller-allocated, n_sites = gm_count(...)):
//  coords[n][3] int32, type[n] uint8, nbr[n][19] int32.
// Sites are numbered in lexicographic (z, y, x) voxel order.
// Returns 0 on success, -1 if a site touches iolets of both roles,
// -2 if n_sites does not match the bitmap.
int gm_build(int64_t nx, int64_t ny, int64_t nz, const uint64_t *bits, const int32_t *periodic,
             int32_t n_iolets, const double *centre, const double *normal, const double *radius,
             const int32_t *role, int64_t n_sites, int32_t *coords, uint8_t *type, int32_t *nbr) {
  Box B{nx, ny, nz, periodic ? periodic[0] : 0, periodic ? periodic[1] : 0, periodic ? periodic[2] : 0};
  const int64_t nvox = B.nvox();
  const int64_t nw = (nvox + 63) / 64;
  std::vector<int64_t> base(nw + 1);
  base[0] = 0;
  {
    // prefix sum of popcounts (two-level for parallelism)
    int nt = omp_get_max_threads();
    std::vector<int64_t> part(nt + 1, 0);
#pragma omp parallel num_threads(nt)
    {
      int t = omp_get_thread_num(), T = omp_get_num_threads();
      int64_t lo = nw * t / T, hi = nw * (t + 1) / T, s = 0;
      for (int64_t w = lo; w < hi; ++w) s += __builtin_popcountll(bits[w]);
      part[t + 1] = s;
#pragma omp barrier
#pragma omp single
      for (int i = 0; i < T; ++i) part[i + 1] += part[i];
      s = part[t];
      for (int64_t w = lo; w < hi; ++w) { base[w] = s; s += __builtin_popcountll(bits[w]); }
      if (t == T - 1) base[nw] = s;
    }
  }
  if (base[nw] != n_sites) return -2;
  auto rank = [&](int64_t v) -> int64_t {
    const uint64_t w = bits[v >> 6];
    const uint64_t below = (v & 63) ? (w & ((1ull << (v & 63)) - 1ull)) : 0ull;
    return base[v >> 6] + __builtin_popcountll(below);
  };
  // Candidate iolets per 16^3 cell, in increasing k so that the first match
  // below is the same as a scan over all iolets.  A link can only cross
  // plane k within (R + sqrt 2) of its centre in the plane and sqrt 2 of it
  // along the normal, so iolet k is listed in every cell that meets the box
  // centre +- (R + 5) (the site is within R + 2 sqrt 2 + 1 of the centre);
  // an iolet without a radius is listed everywhere.
  const int64_t CS = 16;
  const int64_t gx = (nx + CS - 1) / CS, gy = (ny + CS - 1) / CS, gz = (nz + CS - 1) / CS;
  const int64_t ncell = gx * gy * gz;
  std::vector<int64_t> cbeg(ncell + 1, 0);
  std::vector<int32_t> clist;
  {
    auto cell_range = [&](int k, int64_t lo[3], int64_t hi[3]) {
      const int64_t g[3] = {gx, gy, gz};
      for (int d = 0; d < 3; ++d) {
        if (radius[k] > 0.0) {
          const double m = radius[k] + 5.0;
          lo[d] = std::max<int64_t>(0, (int64_t)std::floor((centre[3 * k + d] - m) / CS));
          hi[d] = std::min<int64_t>(g[d] - 1, (int64_t)std::floor((centre[3 * k + d] + m) / CS));
        } else {
          lo[d] = 0;
          hi[d] = g[d] - 1;
        }
      }
    };
    for (int pass = 0; pass < 2; ++pass) {
      std::vector<int64_t> fill(cbeg.begin(), cbeg.end() - 1);
      for (int k = 0; k < n_iolets; ++k) {
        int64_t lo[3], hi[3];
        cell_range(k, lo, hi);
        for (int64_t cz = lo[2]; cz <= hi[2]; ++cz)
          for (int64_t cy = lo[1]; cy <= hi[1]; ++cy)
            for (int64_t cx = lo[0]; cx <= hi[0]; ++cx) {
              const int64_t c = (cz * gy + cy) * gx + cx;
              if (pass == 0) cbeg[c + 1]++;
              else clist[fill[c]++] = k;
            }
      }
      if (pass == 0) {
        for (int64_t c = 0; c < ncell; ++c) cbeg[c + 1] += cbeg[c];
        clist.resize(cbeg[ncell]);
      }
    }
  }
  int bad = 0;
#pragma omp parallel for schedule(dynamic, 1024) reduction(| : bad)
  for (int64_t w = 0; w < nw; ++w) {
    uint64_t word = bits[w];
    while (word) {
      const int bit = __builtin_ctzll(word);
      word &= word - 1;
      const int64_t v = w * 64 + bit;
      const int64_t id = rank(v);
      const int64_t x = v % nx, y = (v / nx) % ny, z = v / (nx * ny);
      coords[3 * id] = (int32_t)x; coords[3 * id + 1] = (int32_t)y; coords[3 * id + 2] = (int32_t)z;
      bool has_wall = false; int roles = 0;
      int32_t *row = nbr + 19 * id;
      row[0] = (int32_t)id;
      for (int i = 1; i < 19; ++i) {
        const int64_t yx = x + CX[i], yy = y + CY[i], yz = z + CZ[i];
        const int64_t u = vox_index(B, yx, yy, yz);
        if (u >= 0 && bit_get(bits, u)) { row[i] = (int32_t)rank(u); continue; }
        int32_t code = -1;
        const int64_t cell = ((z / CS) * gy + y / CS) * gx + x / CS;
        for (int64_t e = cbeg[cell]; e < cbeg[cell + 1]; ++e) {
          const int k = clist[e];
          const double *p = centre + 3 * k, *n = normal + 3 * k;
          const double sx = (x - p[0]) * n[0] + (y - p[1]) * n[1] + (z - p[2]) * n[2];
          const double sy = (yx - p[0]) * n[0] + (yy - p[1]) * n[1] + (yz - p[2]) * n[2];
          if (!(sx >= 0.0 && sy < 0.0)) continue;
          if (radius[k] > 0.0) {
            const double qx = yx - p[0] - sy * n[0], qy = yy - p[1] - sy * n[1], qz = yz - p[2] - sy * n[2];
            const double lim = radius[k] + std::sqrt(2.0);
            if (qx * qx + qy * qy + qz * qz >= lim * lim) continue;
          }
          code = -(2 + k);
          roles |= (role[k] == 0) ? 1 : 2;
          break;
        }
        if (code == -1) has_wall = true;
        row[i] = code;
      }
      uint8_t t;
      if (roles == 3) { bad = 1; t = 0; }
      else if (roles == 1) t = has_wall ? 4 : 2;
      else if (roles == 2) t = has_wall ? 5 : 3;
      else t = has_wall ? 1 : 0;
      type[id] = t;
    }
  }
  return bad ? -1 : 0;
}

}  // extern "C"
