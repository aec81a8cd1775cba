// Cartesian set-up of the elastic example: displacements at voxel corners
// (three components per node, clamped outer walls), each voxel adding the
// stiffness of the trilinear element on the unit cube with its own 6 x 6
// Voigt stiffness (2 x 2 x 2 Gauss rule) and a lumped mass rho / 8 per corner
// and component. A = -sum_v K_v is symmetric and non-positive (Sec. 1), cells
// are the boxes between the cut planes with A_i, B_i the same sums over
// their voxels (eq. splitN_c), and each skeleton piece (face interior, edge
// line, corner point) gets the lowest orthonormal DCT-II modes per
// component (Sec. 4.1). The result goes through the generic ABI calls.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <map>
#include <tuple>
#include <vector>

#include "sfrom_internal.h"

namespace {

// 24 x 24 stiffness of the unit-cube trilinear element for the symmetric
// 6 x 6 Voigt matrix C (strains xx, yy, zz, yz, xz, xy with engineering
// shears); corners x-fastest, dofs corner-major (3 corner + component).
std::array<double, 576> element_stiffness(const double C[6][6]) {
  std::array<double, 576> K{};
  const double gp[2] = {0.5 - 0.5 / std::sqrt(3.0), 0.5 + 0.5 / std::sqrt(3.0)};
  for (int iz = 0; iz < 2; ++iz)
    for (int iy = 0; iy < 2; ++iy)
      for (int ix = 0; ix < 2; ++ix) {
        const double p[3] = {gp[ix], gp[iy], gp[iz]};
        double B[6][24] = {};
        for (int k = 0; k < 8; ++k) {
          const int c[3] = {k & 1, (k >> 1) & 1, (k >> 2) & 1};
          double f[3], d[3];
          for (int a = 0; a < 3; ++a) {
            f[a] = c[a] ? p[a] : 1.0 - p[a];
            d[a] = c[a] ? 1.0 : -1.0;
          }
          const double gx = d[0] * f[1] * f[2], gy = f[0] * d[1] * f[2], gz = f[0] * f[1] * d[2];
          B[0][3 * k] = gx;
          B[1][3 * k + 1] = gy;
          B[2][3 * k + 2] = gz;
          B[3][3 * k + 1] = gz; B[3][3 * k + 2] = gy;
          B[4][3 * k] = gz; B[4][3 * k + 2] = gx;
          B[5][3 * k] = gy; B[5][3 * k + 1] = gx;
        }
        double CB[6][24];
        for (int i = 0; i < 6; ++i)
          for (int j = 0; j < 24; ++j) {
            double s = 0.0;
            for (int q = 0; q < 6; ++q) s += C[i][q] * B[q][j];
            CB[i][j] = s;
          }
        for (int i = 0; i < 24; ++i)
          for (int j = 0; j < 24; ++j) {
            double s = 0.0;
            for (int q = 0; q < 6; ++q) s += B[q][i] * CB[q][j];
            K[i * 24 + j] += s / 8.0;   // unit cube: Gauss weight 1/8 per point
          }
      }
  // symmetric to the last bit, so that the assembled A is exactly symmetric
  for (int i = 0; i < 24; ++i)
    for (int j = i + 1; j < 24; ++j) K[i * 24 + j] = K[j * 24 + i] = 0.5 * (K[i * 24 + j] + K[j * 24 + i]);
  return K;
}

struct EGrid {
  int nx, ny, nz;
  const double* c21;        // 21 upper-triangle Voigt entries per voxel
  const double* rho;
  std::map<std::array<double, 21>, int> kid;
  std::vector<std::array<double, 576>> Ks;
  std::vector<int32_t> vk;  // stiffness id of each voxel
  int64_t vidx(int x, int y, int z) const { return x + (int64_t)nx * (y + (int64_t)ny * z); }
  bool unknown(int x, int y, int z) const { return x >= 1 && x < nx && y >= 1 && y < ny && z >= 1 && z < nz; }
  int64_t gnode(int x, int y, int z) const { return (x - 1) + (int64_t)(nx - 1) * ((y - 1) + (int64_t)(ny - 1) * (z - 1)); }
};

// Voxels with equal stiffness share one element matrix.
void element_matrices(EGrid& g) {
  const int64_t nv = (int64_t)g.nx * g.ny * g.nz;
  g.vk.resize(nv);
  for (int64_t v = 0; v < nv; ++v) {
    std::array<double, 21> key;
    std::copy(g.c21 + 21 * v, g.c21 + 21 * v + 21, key.begin());
    auto it = g.kid.find(key);
    if (it == g.kid.end()) {
      double C[6][6];
      int o = 0;
      for (int i = 0; i < 6; ++i)
        for (int j = i; j < 6; ++j) { C[i][j] = C[j][i] = key[o++]; }
      it = g.kid.emplace(key, (int)g.Ks.size()).first;
      g.Ks.push_back(element_stiffness(C));
    }
    g.vk[v] = it->second;
  }
}

// -sum K_v and the lumped masses over the voxels of [lo, hi) on the node box
// [nlo, nhi] (inclusive, wall nodes excluded), 3 dofs per node numbered
// node-major with nodes x-fastest in the box. CSR rows list the columns of
// the 3 x 3 x 3 neighbour nodes (those in the box) in increasing order.
template <typename RP>
void assemble_elastic_box(const EGrid& g, const int lo[3], const int hi[3], const int nlo[3], const int nhi[3],
                          std::vector<RP>& rp, std::vector<int32_t>& col, std::vector<double>& a,
                          std::vector<double>& m) {
  const int ex = nhi[0] - nlo[0] + 1, ey = nhi[1] - nlo[1] + 1, ez = nhi[2] - nlo[2] + 1;
  const int64_t nn = (int64_t)ex * ey * ez;
  auto lid = [&](int x, int y, int z) -> int64_t { return (x - nlo[0]) + (int64_t)ex * ((y - nlo[1]) + (int64_t)ey * (z - nlo[2])); };
  auto inbox = [&](int x, int y, int z) {
    return x >= nlo[0] && x <= nhi[0] && y >= nlo[1] && y <= nhi[1] && z >= nlo[2] && z <= nhi[2];
  };
  // pattern: per node, the present neighbour slots (dz, dy, dx in -1..1)
  rp.assign(1, 0);
  rp.reserve(3 * nn + 1);
  std::vector<int8_t> slotpos((size_t)nn * 27, -1);
  std::vector<int64_t> rowstart(nn);
  col.clear();
  for (int z = nlo[2]; z <= nhi[2]; ++z)
    for (int y = nlo[1]; y <= nhi[1]; ++y)
      for (int x = nlo[0]; x <= nhi[0]; ++x) {
        const int64_t k = lid(x, y, z);
        std::vector<int64_t> nb;
        for (int dz = -1; dz <= 1; ++dz)
          for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
              const int s = (dz + 1) * 9 + (dy + 1) * 3 + (dx + 1);
              if (inbox(x + dx, y + dy, z + dz)) {
                slotpos[k * 27 + s] = (int8_t)nb.size();
                nb.push_back(lid(x + dx, y + dy, z + dz));
              }
            }
        rowstart[k] = (int64_t)col.size();
        for (int c = 0; c < 3; ++c) {
          for (int64_t q : nb)
            for (int c2 = 0; c2 < 3; ++c2) col.push_back((int32_t)(3 * q + c2));
          rp.push_back((RP)col.size());
        }
      }
  a.assign(col.size(), 0.0);
  m.assign(3 * nn, 0.0);
  for (int vz = lo[2]; vz < hi[2]; ++vz)
    for (int vy = lo[1]; vy < hi[1]; ++vy)
      for (int vx = lo[0]; vx < hi[0]; ++vx) {
        const auto& K = g.Ks[g.vk[g.vidx(vx, vy, vz)]];
        const double mv = g.rho[g.vidx(vx, vy, vz)] / 8.0;
        for (int i = 0; i < 8; ++i) {
          const int xi = vx + (i & 1), yi = vy + ((i >> 1) & 1), zi = vz + ((i >> 2) & 1);
          if (!inbox(xi, yi, zi)) continue;
          const int64_t ki = lid(xi, yi, zi);
          for (int c = 0; c < 3; ++c) m[3 * ki + c] += mv;
          // row (3 ki + c) has 3 n_nb entries; column block of neighbour slot s at 3 pos(s)
          const int64_t nrow = ((int64_t)rp[3 * ki + 1] - (int64_t)rp[3 * ki]);
          for (int j = 0; j < 8; ++j) {
            const int xj = vx + (j & 1), yj = vy + ((j >> 1) & 1), zj = vz + ((j >> 2) & 1);
            if (!inbox(xj, yj, zj)) continue;
            const int s = (zj - zi + 1) * 9 + (yj - yi + 1) * 3 + (xj - xi + 1);
            const int pos = slotpos[ki * 27 + s];
            for (int c = 0; c < 3; ++c)
              for (int c2 = 0; c2 < 3; ++c2)
                a[rowstart[ki] + c * nrow + 3 * pos + c2] -= K[(3 * i + c) * 24 + 3 * j + c2];
          }
        }
      }
}

double dct_e(int n, int k, int j) { return std::cos(M_PI * k * (j + 0.5) / n); }

std::vector<double> dct_unit(int n, int k) {
  std::vector<double> v(n);
  double s = 0.0;
  for (int j = 0; j < n; ++j) { v[j] = dct_e(n, k, j); s += v[j] * v[j]; }
  s = std::sqrt(s);
  for (auto& x : v) x /= s;
  return v;
}

}  // namespace

extern "C" int sfrom_setup_voxel_elastic(sfrom_t* h, const int32_t nvox[3], const double* c21, const double* rho,
                                         const int32_t ncut[3], const int32_t* cuts, int32_t modes_face,
                                         int32_t modes_edge) {
  if (!h) return SFROM_EINVAL;
  if (!nvox || !c21 || !rho || !ncut || (!cuts && ncut[0] + ncut[1] + ncut[2] > 0) || modes_face < 1 ||
      modes_edge < 1) {
    h->err = "bad elastic set-up arguments";
    return SFROM_EINVAL;
  }
  EGrid g;
  g.nx = nvox[0]; g.ny = nvox[1]; g.nz = nvox[2];
  g.c21 = c21; g.rho = rho;
  if (g.nx < 2 || g.ny < 2 || g.nz < 2) { h->err = "need at least 2 voxels per axis"; return SFROM_EINVAL; }
  const int64_t nv = (int64_t)g.nx * g.ny * g.nz;
  for (int64_t v = 0; v < nv; ++v) {
    bool ok = rho[v] > 0.0 && std::isfinite(rho[v]);
    for (int q = 0; q < 21 && ok; ++q) ok = std::isfinite(c21[21 * v + q]);
    if (!ok) { h->err = "rho must be positive and the stiffness finite"; return SFROM_EINVAL; }
  }
  std::array<std::vector<int>, 3> cut;
  {
    int o = 0;
    const int nvx[3] = {g.nx, g.ny, g.nz};
    for (int ax = 0; ax < 3; ++ax)
      for (int k = 0; k < ncut[ax]; ++k) {
        const int c = cuts[o++];
        if (c <= 0 || c >= nvx[ax] || (!cut[ax].empty() && c <= cut[ax].back())) {
          h->err = "cut planes must be increasing and strictly inside the grid";
          return SFROM_EINVAL;
        }
        cut[ax].push_back(c);
      }
  }
  element_matrices(g);
  // ---- fine pencil ------------------------------------------------------------
  int rc;
  {
    const int lo[3] = {0, 0, 0}, hi[3] = {g.nx, g.ny, g.nz};
    const int nlo[3] = {1, 1, 1}, nhi[3] = {g.nx - 1, g.ny - 1, g.nz - 1};
    std::vector<int64_t> rp;
    std::vector<int32_t> col;
    std::vector<double> a, b;
    assemble_elastic_box(g, lo, hi, nlo, nhi, rp, col, a, b);
    rc = sfrom_set_pencil(h, (int64_t)b.size(), rp.data(), col.data(), a.data(), b.data());
    if (rc != SFROM_OK) return rc;
  }
  // ---- cells ----------------------------------------------------------------
  std::array<std::vector<int>, 3> edge;
  const int nvx[3] = {g.nx, g.ny, g.nz};
  for (int ax = 0; ax < 3; ++ax) {
    edge[ax].push_back(0);
    edge[ax].insert(edge[ax].end(), cut[ax].begin(), cut[ax].end());
    edge[ax].push_back(nvx[ax]);
  }
  const int ncx = (int)edge[0].size() - 1, ncy = (int)edge[1].size() - 1, ncz = (int)edge[2].size() - 1;
  std::vector<int32_t> rpl, coll;
  std::vector<double> al, bl;
  std::vector<int64_t> gd;
  for (int cz = 0; cz < ncz; ++cz)
    for (int cy = 0; cy < ncy; ++cy)
      for (int cx = 0; cx < ncx; ++cx) {
        const int clo[3] = {edge[0][cx], edge[1][cy], edge[2][cz]};
        const int chi[3] = {edge[0][cx + 1], edge[1][cy + 1], edge[2][cz + 1]};
        int blo[3], bhi[3];
        for (int ax = 0; ax < 3; ++ax) {
          blo[ax] = std::max(clo[ax], 1);
          bhi[ax] = std::min(chi[ax], nvx[ax] - 1);
        }
        assemble_elastic_box(g, clo, chi, blo, bhi, rpl, coll, al, bl);
        gd.clear();
        for (int z = blo[2]; z <= bhi[2]; ++z)
          for (int y = blo[1]; y <= bhi[1]; ++y)
            for (int x = blo[0]; x <= bhi[0]; ++x)
              for (int c = 0; c < 3; ++c) gd.push_back(3 * g.gnode(x, y, z) + c);
        const int cid = cx + ncx * (cy + ncy * cz);
        rc = sfrom_add_cell(h, cid, (int32_t)gd.size(), gd.data(), rpl.data(), coll.data(), al.data(), bl.data());
        if (rc != SFROM_OK) return rc;
      }
  // ---- pieces: the acoustic set-up's node sets, every scalar mode once per
  // component (columns mode by mode, components x, y, z)
  auto key_of = [&](int ax, int c) {
    const auto it = std::lower_bound(cut[ax].begin(), cut[ax].end(), c);
    const int j = (int)(it - cut[ax].begin());
    return (it != cut[ax].end() && *it == c) ? 2 * j + 1 : 2 * j;
  };
  std::map<std::tuple<int, int, int>, int> pid;
  std::vector<std::vector<int64_t>> pnodes;
  std::vector<std::array<int, 3>> pkey, pmin, pmax;
  for (int z = 1; z < g.nz; ++z) {
    const int kz = key_of(2, z);
    for (int y = 1; y < g.ny; ++y) {
      const int ky = key_of(1, y);
      for (int x = 1; x < g.nx; ++x) {
        const int kx = key_of(0, x);
        if (!((kx & 1) || (ky & 1) || (kz & 1))) continue;
        auto key = std::make_tuple(kx, ky, kz);
        auto it = pid.find(key);
        int p;
        if (it == pid.end()) {
          p = (int)pnodes.size();
          pid.emplace(key, p);
          pnodes.emplace_back();
          pkey.push_back({kx, ky, kz});
          pmin.push_back({x, y, z});
          pmax.push_back({x, y, z});
        } else {
          p = it->second;
        }
        pnodes[p].push_back(g.gnode(x, y, z));
        const int xyz[3] = {x, y, z};
        for (int ax = 0; ax < 3; ++ax) {
          pmin[p][ax] = std::min(pmin[p][ax], xyz[ax]);
          pmax[p][ax] = std::max(pmax[p][ax], xyz[ax]);
        }
      }
    }
  }
  for (size_t p = 0; p < pnodes.size(); ++p) {
    std::vector<int> dims;
    int onplane = 0;
    for (int ax = 0; ax < 3; ++ax) {
      if (pkey[p][ax] & 1) ++onplane;
      else dims.push_back(pmax[p][ax] - pmin[p][ax] + 1);
    }
    const int kp = (int)pnodes[p].size();
    std::vector<std::vector<double>> modes;   // scalar modes over the piece's nodes
    if (onplane == 3) {
      modes.push_back({1.0});
    } else if (onplane == 2) {
      const int ne = dims[0];
      for (int k = 0; k < std::min(modes_edge, ne); ++k) modes.push_back(dct_unit(ne, k));
    } else {
      const int n1 = dims[0], n2 = dims[1];
      std::vector<std::array<int, 2>> pairs;
      for (int pp = 0; pp < n1; ++pp)
        for (int qq = 0; qq < n2; ++qq) pairs.push_back({pp, qq});
      std::stable_sort(pairs.begin(), pairs.end(), [](const std::array<int, 2>& u, const std::array<int, 2>& v) {
        const int mu = std::max(u[0], u[1]), mv = std::max(v[0], v[1]);
        if (mu != mv) return mu < mv;
        if (u[0] != v[0]) return u[0] < v[0];
        return u[1] < v[1];
      });
      const int nm = std::min<int>(modes_face, (int)pairs.size());
      for (int k = 0; k < nm; ++k) {
        const auto v1 = dct_unit(n1, pairs[k][0]);
        const auto v2 = dct_unit(n2, pairs[k][1]);
        std::vector<double> v;
        for (int j2 = 0; j2 < n2; ++j2)
          for (int j1 = 0; j1 < n1; ++j1) v.push_back(v1[j1] * v2[j2]);
        modes.push_back(std::move(v));
      }
    }
    const int bs = (int)modes.size(), bp = 3 * bs, kd = 3 * kp;
    std::vector<int64_t> dofs(kd);
    for (int q = 0; q < kp; ++q)
      for (int c = 0; c < 3; ++c) dofs[3 * q + c] = 3 * pnodes[p][q] + c;
    std::vector<double> S((size_t)kd * bp, 0.0);   // column-major
    for (int l = 0; l < bs; ++l)
      for (int c = 0; c < 3; ++c)
        for (int q = 0; q < kp; ++q) S[(size_t)(3 * l + c) * kd + 3 * q + c] = modes[l][q];
    rc = sfrom_add_piece(h, (int32_t)p, kd, dofs.data(), bp, S.data());
    if (rc != SFROM_OK) return rc;
  }
  h->err.clear();
  return SFROM_OK;
}
