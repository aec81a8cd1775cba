// Cartesian convenience set-up for the 3D acoustic example of Sec. 1 and the
// regular coarse partitions of Sec. 2: voxel-assembled fine pencil, cells as
// boxes between cut planes with voxel-wise splitting (eq. splitN_c), and
// skeleton pieces (face interiors, edge lines, corner points) with the
// lowest orthonormal DCT-II modes as boundary bases (Sec. 4.1). The result is
// handed to the generic ABI calls.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "sfrom_internal.h"

namespace {

struct Grid {
  int nx, ny, nz;           // voxels
  const double* sigma;      // x fastest
  const double* rho;
  double sig(int x, int y, int z) const { return sigma[x + (int64_t)nx * (y + (int64_t)ny * z)]; }
  double rh(int x, int y, int z) const { return rho[x + (int64_t)nx * (y + (int64_t)ny * z)]; }
  bool unknown(int x, int y, int z) const { return x >= 1 && x < nx && y >= 1 && y < ny && z >= 1 && z < nz; }
  int64_t gidx(int x, int y, int z) const {
    return (x - 1) + (int64_t)(nx - 1) * ((y - 1) + (int64_t)(ny - 1) * (z - 1));
  }
};

// Conductance of the edge from node p along axis `ax` (to p + e_ax), summing
// sigma/4 over the voxels that touch the edge and lie in the voxel box
// [lo, hi) (the whole grid for the fine operator, a cell for A_i).
double edge_cond(const Grid& g, int x, int y, int z, int ax, const int lo[3], const int hi[3]) {
  const int p[3] = {x, y, z};
  // the voxel index along ax is p[ax]; along the other two axes p-1 or p
  double s = 0.0;
  const int a1 = (ax + 1) % 3, a2 = (ax + 2) % 3;
  if (p[ax] < lo[ax] || p[ax] >= hi[ax]) return 0.0;
  for (int d1 = -1; d1 <= 0; ++d1)
    for (int d2 = -1; d2 <= 0; ++d2) {
      int v[3];
      v[ax] = p[ax];
      v[a1] = p[a1] + d1;
      v[a2] = p[a2] + d2;
      if (v[a1] < lo[a1] || v[a1] >= hi[a1] || v[a2] < lo[a2] || v[a2] >= hi[a2]) continue;
      s += 0.25 * g.sig(v[0], v[1], v[2]);
    }
  return s;
}

double node_mass(const Grid& g, int x, int y, int z, const int lo[3], const int hi[3]) {
  double s = 0.0;
  for (int dz = -1; dz <= 0; ++dz)
    for (int dy = -1; dy <= 0; ++dy)
      for (int dx = -1; dx <= 0; ++dx) {
        const int vx = x + dx, vy = y + dy, vz = z + dz;
        if (vx < lo[0] || vx >= hi[0] || vy < lo[1] || vy >= hi[1] || vz < lo[2] || vz >= hi[2]) continue;
        s += 0.125 * g.rh(vx, vy, vz);
      }
  return s;
}

// Assemble the operator restricted to the voxel box [lo, hi) on the node box
// [nlo, nhi] (inclusive, wall nodes excluded), nodes numbered x-fastest in
// the node box. Returns CSR (rowptr, col, a) and masses.
void assemble_box(const Grid& g, const int lo[3], const int hi[3], const int nlo[3], const int nhi[3],
                  std::vector<int32_t>* rp32, std::vector<int64_t>* rp64, std::vector<int32_t>& col,
                  std::vector<double>& a, std::vector<double>& m) {
  const int ex = nhi[0] - nlo[0] + 1, ey = nhi[1] - nlo[1] + 1, ez = nhi[2] - nlo[2] + 1;
  auto lid = [&](int x, int y, int z) -> int64_t {
    return (x - nlo[0]) + (int64_t)ex * ((y - nlo[1]) + (int64_t)ey * (z - nlo[2]));
  };
  auto inbox = [&](int x, int y, int z) {
    return x >= nlo[0] && x <= nhi[0] && y >= nlo[1] && y <= nhi[1] && z >= nlo[2] && z <= nhi[2];
  };
  const int64_t nn = (int64_t)ex * ey * ez;
  if (rp32) { rp32->assign(1, 0); rp32->reserve(nn + 1); }
  if (rp64) { rp64->assign(1, 0); rp64->reserve(nn + 1); }
  col.clear(); a.clear(); m.clear();
  col.reserve(nn * 7); a.reserve(nn * 7); m.reserve(nn);
  for (int z = nlo[2]; z <= nhi[2]; ++z)
    for (int y = nlo[1]; y <= nhi[1]; ++y)
      for (int x = nlo[0]; x <= nhi[0]; ++x) {
        // neighbours in increasing index order: z-, y-, x-, self, x+, y+, z+
        const int nb[6][4] = {{x, y, z - 1, 2}, {x, y - 1, z, 1}, {x - 1, y, z, 0},
                              {x + 1, y, z, 0}, {x, y + 1, z, 1}, {x, y, z + 1, 2}};
        double c[6];
        double diag = 0.0;
        for (int k = 0; k < 6; ++k) {
          const int qx = nb[k][0], qy = nb[k][1], qz = nb[k][2], ax = nb[k][3];
          // the edge starts at the smaller endpoint
          const bool minus = (k < 3);
          const int sx = minus ? qx : x, sy = minus ? qy : y, sz = minus ? qz : z;
          c[k] = edge_cond(g, sx, sy, sz, ax, lo, hi);
          diag -= c[k];
        }
        auto push = [&](int k) {
          const int qx = nb[k][0], qy = nb[k][1], qz = nb[k][2];
          if (c[k] != 0.0 && g.unknown(qx, qy, qz) && inbox(qx, qy, qz)) {
            col.push_back((int32_t)lid(qx, qy, qz));
            a.push_back(c[k]);
          }
        };
        push(0); push(1); push(2);
        col.push_back((int32_t)lid(x, y, z));
        a.push_back(diag);
        push(3); push(4); push(5);
        m.push_back(node_mass(g, x, y, z, lo, hi));
        if (rp32) rp32->push_back((int32_t)col.size());
        if (rp64) rp64->push_back((int64_t)col.size());
      }
}

double dct(int n, int k, int j) { return std::cos(M_PI * k * (j + 0.5) / n); }

std::vector<double> dct_vec(int n, int k) {
  std::vector<double> v(n);
  double s = 0.0;
  for (int j = 0; j < n; ++j) { v[j] = dct(n, k, j); s += v[j] * v[j]; }
  s = std::sqrt(s);
  for (auto& x : v) x /= s;
  return v;
}

// Face-mode count of a face interior of n1 x n2 nodes: the first rule whose
// area bound (in voxels, (n1 + 1)(n2 + 1)) it meets, else the fixed count.
struct FaceModes {
  int32_t fixed = 0;
  int32_t n_rules = 0;
  const int32_t* area_max = nullptr;
  const int32_t* modes = nullptr;
  int operator()(int n1, int n2) const {
    if (n_rules == 0) return fixed;
    const int64_t area = (int64_t)(n1 + 1) * (n2 + 1);
    for (int k = 0; k < n_rules; ++k)
      if (area <= area_max[k]) return modes[k];
    return modes[n_rules - 1];
  }
};

int setup_acoustic(sfrom_t* h, const int32_t nvox[3], const double* sigma, const double* rho,
                   const int32_t ncut[3], const int32_t* cuts, const FaceModes& face_modes, int32_t modes_edge);

}  // namespace

extern "C" int sfrom_setup_voxel_acoustic(sfrom_t* h, const int32_t nvox[3], const double* sigma,
                                          const double* rho, const int32_t ncut[3], const int32_t* cuts,
                                          int32_t modes_face, int32_t modes_edge) {
  if (!h) return SFROM_EINVAL;
  if (modes_face < 1) {
    h->err = "bad voxel set-up arguments";
    return SFROM_EINVAL;
  }
  FaceModes fm;
  fm.fixed = modes_face;
  return setup_acoustic(h, nvox, sigma, rho, ncut, cuts, fm, modes_edge);
}

extern "C" int sfrom_setup_voxel_acoustic_rules(sfrom_t* h, const int32_t nvox[3], const double* sigma,
                                                const double* rho, const int32_t ncut[3], const int32_t* cuts,
                                                int32_t n_rules, const int32_t* face_area_max,
                                                const int32_t* face_modes, int32_t modes_edge) {
  if (!h) return SFROM_EINVAL;
  if (n_rules < 1 || !face_area_max || !face_modes) {
    h->err = "bad face-mode rules";
    return SFROM_EINVAL;
  }
  for (int k = 0; k < n_rules; ++k)
    if (face_modes[k] < 1 || (k > 0 && face_area_max[k] <= face_area_max[k - 1])) {
      h->err = "face-mode rules need counts >= 1 and increasing area bounds";
      return SFROM_EINVAL;
    }
  FaceModes fm;
  fm.n_rules = n_rules;
  fm.area_max = face_area_max;
  fm.modes = face_modes;
  return setup_acoustic(h, nvox, sigma, rho, ncut, cuts, fm, modes_edge);
}

namespace {

int setup_acoustic(sfrom_t* h, const int32_t nvox[3], const double* sigma, const double* rho,
                   const int32_t ncut[3], const int32_t* cuts, const FaceModes& face_modes, int32_t modes_edge) {
  if (!nvox || !sigma || !rho || !ncut || (!cuts && ncut[0] + ncut[1] + ncut[2] > 0) || modes_edge < 1) {
    h->err = "bad voxel set-up arguments";
    return SFROM_EINVAL;
  }
  Grid g{nvox[0], nvox[1], nvox[2], sigma, rho};
  if (g.nx < 2 || g.ny < 2 || g.nz < 2) { h->err = "need at least 2 voxels per axis"; return SFROM_EINVAL; }
  const int64_t nv = (int64_t)g.nx * g.ny * g.nz;
  for (int64_t v = 0; v < nv; ++v)
    if (!(sigma[v] > 0.0) || !(rho[v] > 0.0) || !std::isfinite(sigma[v]) || !std::isfinite(rho[v])) {
      h->err = "sigma and rho must be positive and finite";
      return SFROM_EINVAL;
    }
  std::array<std::vector<int>, 3> cut;
  {
    int o = 0;
    const int nvx[3] = {g.nx, g.ny, g.nz};
    for (int ax = 0; ax < 3; ++ax) {
      for (int k = 0; k < ncut[ax]; ++k) {
        const int c = cuts[o++];
        if (c <= 0 || c >= nvx[ax] || (!cut[ax].empty() && c <= cut[ax].back())) {
          h->err = "cut planes must be increasing and strictly inside the grid";
          return SFROM_EINVAL;
        }
        cut[ax].push_back(c);
      }
    }
  }
  // ---- fine pencil -------------------------------------------------------------
  const int lo[3] = {0, 0, 0}, hi[3] = {g.nx, g.ny, g.nz};
  const int nlo[3] = {1, 1, 1}, nhi[3] = {g.nx - 1, g.ny - 1, g.nz - 1};
  std::vector<int64_t> rp;
  std::vector<int32_t> col;
  std::vector<double> a, b;
  assemble_box(g, lo, hi, nlo, nhi, nullptr, &rp, col, a, b);
  const int64_t n = (int64_t)b.size();
  int rc = sfrom_set_pencil(h, n, rp.data(), col.data(), a.data(), b.data());
  if (rc != SFROM_OK) return rc;
  // 7-point form of the same operator for the fine-grid comparator
  {
    const int ux = g.nx - 1, uy = g.ny - 1, uz = g.nz - 1;
    std::vector<double> st((size_t)n * 8, 0.0);
    for (int z = 1; z < g.nz; ++z)
      for (int y = 1; y < g.ny; ++y)
        for (int x = 1; x < g.nx; ++x) {
          const int64_t k = g.gidx(x, y, z);
          const int64_t nbr[6] = {x > 1 ? k - 1 : -1, x < g.nx - 1 ? k + 1 : -1,
                                  y > 1 ? k - ux : -1, y < g.ny - 1 ? k + ux : -1,
                                  z > 1 ? k - (int64_t)ux * uy : -1, z < g.nz - 1 ? k + (int64_t)ux * uy : -1};
          for (int64_t e = rp[k]; e < rp[k + 1]; ++e) {
            const int64_t c = col[e];
            if (c == k) { st[k * 8 + 6] = a[e]; continue; }
            for (int d = 0; d < 6; ++d)
              if (nbr[d] == c) st[k * 8 + d] = a[e];
          }
          st[k * 8 + 7] = 1.0 / b[k];
        }
    h->stencil = std::move(st);
    h->grid_u[0] = ux; h->grid_u[1] = uy; h->grid_u[2] = uz;
  }
  // ---- cells ---------------------------------------------------------------------
  std::array<std::vector<int>, 3> edge;
  const int nvx[3] = {g.nx, g.ny, g.nz};
  for (int ax = 0; ax < 3; ++ax) {
    edge[ax].push_back(0);
    edge[ax].insert(edge[ax].end(), cut[ax].begin(), cut[ax].end());
    edge[ax].push_back(nvx[ax]);
  }
  const int ncx = (int)edge[0].size() - 1, ncy = (int)edge[1].size() - 1, ncz = (int)edge[2].size() - 1;
  std::vector<int32_t> rpl;
  std::vector<int32_t> coll;
  std::vector<double> al, bl;
  std::vector<int64_t> gn;
  for (int cz = 0; cz < ncz; ++cz)
    for (int cy = 0; cy < ncy; ++cy)
      for (int cx = 0; cx < ncx; ++cx) {
        const int clo[3] = {edge[0][cx], edge[1][cy], edge[2][cz]};
        const int chi[3] = {edge[0][cx + 1], edge[1][cy + 1], edge[2][cz + 1]};
        int bl_[3], bh_[3];
        for (int ax = 0; ax < 3; ++ax) {
          bl_[ax] = std::max(clo[ax], 1);
          bh_[ax] = std::min(chi[ax], nvx[ax] - 1);
        }
        assemble_box(g, clo, chi, bl_, bh_, &rpl, nullptr, coll, al, bl);
        gn.clear();
        for (int z = bl_[2]; z <= bh_[2]; ++z)
          for (int y = bl_[1]; y <= bh_[1]; ++y)
            for (int x = bl_[0]; x <= bh_[0]; ++x) gn.push_back(g.gidx(x, y, z));
        const int cid = cx + ncx * (cy + ncy * cz);
        rc = sfrom_add_cell(h, cid, (int32_t)gn.size(), gn.data(), rpl.data(), coll.data(), al.data(), bl.data());
        if (rc != SFROM_OK) return rc;
      }
  // ---- pieces --------------------------------------------------------------------
  // per-axis key: 2j+1 if the coordinate is cut plane j, else 2 * (number of
  // cuts below it); a piece is a set of skeleton nodes with the same key.
  auto key_of = [&](int ax, int c) {
    const auto it = std::lower_bound(cut[ax].begin(), cut[ax].end(), c);
    const int j = (int)(it - cut[ax].begin());
    return (it != cut[ax].end() && *it == c) ? 2 * j + 1 : 2 * j;
  };
  std::map<std::tuple<int, int, int>, int> pid;
  std::vector<std::vector<int64_t>> pnodes;
  std::vector<std::array<int, 3>> pkey;
  std::vector<std::array<int, 3>> pmin, pmax;
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
        pnodes[p].push_back(g.gidx(x, y, z));
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
    std::vector<double> S;
    int bp = 0;
    if (onplane == 3) {
      S.assign(1, 1.0);
      bp = 1;
    } else if (onplane == 2) {
      const int ne = dims[0];
      bp = std::min(modes_edge, ne);
      for (int k = 0; k < bp; ++k) {
        const auto v = dct_vec(ne, k);
        S.insert(S.end(), v.begin(), v.end());
      }
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
      bp = std::min<int>(face_modes(n1, n2), (int)pairs.size());
      for (int k = 0; k < bp; ++k) {
        const auto v1 = dct_vec(n1, pairs[k][0]);
        const auto v2 = dct_vec(n2, pairs[k][1]);
        for (int j2 = 0; j2 < n2; ++j2)
          for (int j1 = 0; j1 < n1; ++j1) S.push_back(v1[j1] * v2[j2]);
      }
    }
    rc = sfrom_add_piece(h, (int32_t)p, kp, pnodes[p].data(), bp, S.data());
    if (rc != SFROM_OK) return rc;
  }
  h->err.clear();
  return SFROM_OK;
}

}  // namespace
