// General sparse pencils: divide-and-conquer partition and splitting (App.
// A: Prop. 1, Alg. 1 with eq. alg1B, the multidomain algorithm Alg. 2) and
// frequency-limited Gramian bases of the skeleton pieces (Sec. 4.1, eq.
// trgr). Host code; the resulting cells and pieces go through the generic
// partition calls, so the off-line build and the on-line stage are the same
// as for any other partition.
//
// Partition (the choices the paper leaves open):
// * k and l are adjacent iff a_kl != 0 in the subdomain's own operator.
// * The set O of Prop. 1 is a union of breadth-first levels of the
//   subdomain's graph from a pseudo-peripheral root (found from the
//   subdomain's smallest node by moving to the least-degree, then
//   least-index, node of the last level while the depth grows): levels
//   0..j, where level j + 1 is the first at which the running node count
//   reaches half the subdomain, with j in [0, depth - 2]. Prop. 1 then gives
//   Gamma = level j + 1. Subdomains of depth < 2 are not split.
// * Alg. 2 splits the largest splittable subdomain (ties: lowest position),
//   swapping it to the last position p; the O_1 side stays at p and the O_2
//   side is appended.
// * Pieces: the nodes held by two or more cells, grouped by the exact set of
//   cells holding them, ordered by their smallest node; a piece's nodes
//   ascend. Each cell's local nodes are renumbered by reverse Cuthill-McKee
//   so that the band factorisation of the off-line build stays narrow.
//
// Gramian bases (the approximate Gramian is only outlined in the paper):
// eigenpairs of the pencil (-A_s, B_s) below omega_max^2 (B-orthonormal, at
// least the lowest one), restricted to the piece, give G = sum v v^T; the
// basis is G's eigenvectors above eps times its largest eigenvalue (at most
// max_modes). (A_s, B_s) is the union of the piece's cells (sum of their
// split operators) cut to the nodes within graph distance depth + 1 of the
// piece by one Prop. 1 / Alg. 1 split (alpha = beta = 1/2) with O the nodes
// within distance depth; depth < 0 keeps the whole union. The dense
// symmetric eigenproblems use Householder tridiagonalisation, Sturm-sequence
// bisection and inverse iteration.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cfloat>
#include <cmath>
#include <complex>
#include <deque>
#include <map>
#include <numeric>
#include <string>
#include <thread>
#include <vector>

#include "sfrom_internal.h"

// Products and sums below are kept as written (no fused multiply-add) so
// that the split operators are reproducible bit for bit.
#pragma STDC FP_CONTRACT OFF

namespace {

struct GFail {
  int code;
  std::string msg;
};

[[noreturn]] void gfail(int code, const std::string& msg) { throw GFail{code, msg}; }

// A subdomain: ascending global nodes and its split operator (local CSR with
// sorted columns) and mass.
struct Sub {
  std::vector<int64_t> nodes;
  std::vector<int32_t> rp, col;
  std::vector<double> a, b;
  int n() const { return (int)nodes.size(); }
};

std::vector<char> neighbourhood(const Sub& s, const std::vector<char>& in) {
  std::vector<char> out(in);
  for (int k = 0; k < s.n(); ++k)
    if (in[k])
      for (int t = s.rp[k]; t < s.rp[k + 1]; ++t)
        if (s.a[t] != 0.0) out[s.col[t]] = 1;
  return out;
}

// Breadth-first levels from root over nodes with allowed[k] (nullptr: all);
// -1 where not reached.
std::vector<int> levels(const Sub& s, int root, const std::vector<char>* allowed = nullptr) {
  std::vector<int> lev(s.n(), -1);
  std::deque<int> q;
  lev[root] = 0;
  q.push_back(root);
  while (!q.empty()) {
    const int k = q.front();
    q.pop_front();
    for (int t = s.rp[k]; t < s.rp[k + 1]; ++t) {
      const int l = s.col[t];
      if (s.a[t] != 0.0 && lev[l] < 0 && (!allowed || (*allowed)[l])) {
        lev[l] = lev[k] + 1;
        q.push_back(l);
      }
    }
  }
  return lev;
}

int degree(const Sub& s, int k) {
  int d = 0;
  for (int t = s.rp[k]; t < s.rp[k + 1]; ++t) d += s.a[t] != 0.0;
  return d;
}

int pseudo_peripheral(const Sub& s, int start, const std::vector<char>* allowed = nullptr) {
  int root = start;
  std::vector<int> lev = levels(s, root, allowed);
  int depth = *std::max_element(lev.begin(), lev.end());
  for (;;) {
    int cand = -1, cdeg = 0;
    for (int k = 0; k < s.n(); ++k)
      if (lev[k] == depth) {
        const int d = degree(s, k);
        if (cand < 0 || d < cdeg) { cand = k; cdeg = d; }
      }
    std::vector<int> lv = levels(s, cand, allowed);
    const int dp = *std::max_element(lv.begin(), lv.end());
    if (dp <= depth) return root;
    root = cand;
    lev.swap(lv);
    depth = dp;
  }
}

// The set O (mask) of a subdomain, or false when it cannot be split.
bool level_set_O(const Sub& s, std::vector<char>& O) {
  const int n = s.n();
  const std::vector<int> lev = levels(s, pseudo_peripheral(s, 0));
  const int e = *std::max_element(lev.begin(), lev.end());
  if (e < 2) return false;
  std::vector<int64_t> cnt(e + 1, 0);
  for (int k = 0; k < n; ++k)
    if (lev[k] >= 0) cnt[lev[k]]++;
  int m = 0;
  for (int64_t c = 0; m <= e; ++m) {
    c += cnt[m];
    if ((double)c >= 0.5 * n) break;
  }
  const int j = std::min(std::max(m - 1, 0), e - 2);
  O.assign(n, 0);
  for (int k = 0; k < n; ++k) O[k] = lev[k] >= 0 && lev[k] <= j;
  return true;
}

// Prop. 1: code 1 = O_1, 2 = O_2, 3 = Gamma.
std::vector<char> prop1(const Sub& s, const std::vector<char>& O) {
  const std::vector<char> AO = neighbourhood(s, O);
  std::vector<char> O2(s.n());
  for (int k = 0; k < s.n(); ++k) O2[k] = !AO[k];
  const std::vector<char> AO2 = neighbourhood(s, O2);
  std::vector<char> code(s.n());
  for (int k = 0; k < s.n(); ++k) code[k] = O2[k] ? 2 : (!AO2[k] ? 1 : 3);
  return code;
}

// Alg. 1 and eq. alg1B: the two split operators.
void alg1(const Sub& s, const std::vector<char>& code, double alpha, double beta, Sub out[2]) {
  const int n = s.n();
  for (int i = 0; i < 2; ++i) {
    const char ci = (char)(i + 1);
    Sub& o = out[i];
    o = Sub();
    std::vector<int32_t> pos(n, -1);
    for (int k = 0; k < n; ++k)
      if (code[k] == ci || code[k] == 3) {
        pos[k] = o.n();
        o.nodes.push_back(s.nodes[k]);
      }
    o.rp.push_back(0);
    for (int k = 0; k < n; ++k) {
      if (pos[k] < 0) continue;
      double sum[2] = {0.0, 0.0};
      int64_t diag_at = -1;
      for (int t = s.rp[k]; t < s.rp[k + 1]; ++t) {
        const int l = s.col[t];
        const double v = s.a[t];
        if ((code[k] == 1 && code[l] == 2) || (code[k] == 2 && code[l] == 1)) {
          if (v != 0.0) gfail(SFROM_EINVAL, "coupling between O_1 and O_2 (Prop. 1)");
          continue;
        }
        const bool own = code[k] == ci || code[l] == ci;
        const bool both_gamma = code[k] == 3 && code[l] == 3;
        if (code[k] == 3) {               // off-diagonal sums of this Gamma row on both sides
          for (int q = 0; q < 2; ++q) {
            if (l == k) continue;
            if (code[l] == q + 1) sum[q] += std::fabs(v);
            else if (code[l] == 3) sum[q] += std::fabs((q == 0 ? alpha : 1.0 - alpha) * v);
          }
        }
        if (own) {                        // entries at a node of this side
          o.col.push_back(pos[l]);
          o.a.push_back(v);
        } else if (both_gamma) {
          o.col.push_back(pos[l]);
          if (l == k) {
            diag_at = (int64_t)o.a.size();
            o.a.push_back(0.0);
          } else {                        // links inside Gamma, split by alpha
            o.a.push_back((i == 0 ? alpha : 1.0 - alpha) * v);
          }
        }
      }
      if (code[k] == 3) {                 // Gamma diagonal from the off-diagonal sums
        if (diag_at < 0) gfail(SFROM_EINVAL, "missing diagonal entry");
        double akk = 0.0;
        for (int t = s.rp[k]; t < s.rp[k + 1]; ++t)
          if (s.col[t] == k) akk = s.a[t];
        o.a[diag_at] = akk * sum[i] / (sum[0] + sum[1]);
      }
      o.rp.push_back((int32_t)o.col.size());
      o.b.push_back(code[k] == ci ? s.b[k] : (i == 0 ? beta : 1.0 - beta) * s.b[k]);
    }
  }
}

// Alg. 2.
std::vector<Sub> alg2(const Sub& whole, int n_cells, double alpha, double beta) {
  std::vector<Sub> subs{whole};
  while ((int)subs.size() < n_cells) {
    std::vector<int> order(subs.size());
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return subs[x].n() > subs[y].n(); });
    int pick = -1;
    std::vector<char> O;
    for (int i : order)
      if (level_set_O(subs[i], O)) { pick = i; break; }
    if (pick < 0)
      gfail(SFROM_EINVAL, "no subdomain can be split further (" + std::to_string(subs.size()) + " of " +
                              std::to_string(n_cells) + " cells)");
    const int p = (int)subs.size() - 1;
    std::swap(subs[pick], subs[p]);
    const std::vector<char> code = prop1(subs[p], O);
    Sub two[2];
    alg1(subs[p], code, alpha, beta, two);
    subs[p] = std::move(two[0]);
    subs.push_back(std::move(two[1]));
  }
  return subs;
}

// Reverse Cuthill-McKee order (new -> old) of a subdomain's graph.
std::vector<int> rcm(const Sub& s) {
  const int n = s.n();
  std::vector<char> free_(n, 1);
  std::vector<int> order;
  order.reserve(n);
  std::vector<int> deg(n);
  for (int k = 0; k < n; ++k) deg[k] = degree(s, k);
  int next = 0;
  while ((int)order.size() < n) {
    while (!free_[next]) ++next;
    const int root = pseudo_peripheral(s, next, &free_);
    std::deque<int> q{root};
    free_[root] = 0;
    while (!q.empty()) {
      const int k = q.front();
      q.pop_front();
      order.push_back(k);
      std::vector<int> nb;
      for (int t = s.rp[k]; t < s.rp[k + 1]; ++t)
        if (s.a[t] != 0.0 && free_[s.col[t]]) {
          nb.push_back(s.col[t]);
          free_[s.col[t]] = 0;
        }
      std::sort(nb.begin(), nb.end(), [&](int x, int y) { return deg[x] != deg[y] ? deg[x] < deg[y] : x < y; });
      for (int l : nb) q.push_back(l);
    }
  }
  std::reverse(order.begin(), order.end());
  return order;
}

// ---------------------------------------------------------------------------
// dense symmetric eigenproblems
// ---------------------------------------------------------------------------

struct Tridiag {
  int n = 0;
  std::vector<double> d, e;                 // diagonal, sub-diagonal
  std::vector<double> tau;                  // reflector scales
  std::vector<std::vector<double>> v;       // reflector k acts on rows k+1..n-1
};

// Householder reduction Q^T C Q = T of a symmetric n x n matrix (row-major,
// full storage, overwritten); Q = H_0 H_1 ... H_{n-3}.
Tridiag tridiagonalize(int n, std::vector<double>& C) {
  Tridiag t;
  t.n = n;
  t.d.assign(n, 0.0);
  t.e.assign(n > 1 ? n - 1 : 0, 0.0);
  t.tau.assign(n, 0.0);
  t.v.resize(n);
  std::vector<double> x, p, w;
  for (int k = 0; k + 2 < n; ++k) {
    const int m = n - k - 1;
    x.assign(m, 0.0);
    double nrm = 0.0;
    for (int i = 0; i < m; ++i) {
      x[i] = C[(size_t)(k + 1 + i) * n + k];
      nrm += x[i] * x[i];
    }
    nrm = std::sqrt(nrm);
    if (nrm == 0.0) continue;
    const double beta = x[0] >= 0.0 ? -nrm : nrm;
    x[0] -= beta;
    double vv = 0.0;
    for (int i = 0; i < m; ++i) vv += x[i] * x[i];
    const double tau = 2.0 / vv;
    t.e[k] = beta;
    p.assign(m, 0.0);
    for (int i = 0; i < m; ++i) {
      const double* row = &C[(size_t)(k + 1 + i) * n + k + 1];
      double acc = 0.0;
      for (int j = 0; j < m; ++j) acc += row[j] * x[j];
      p[i] = tau * acc;
    }
    double pv = 0.0;
    for (int i = 0; i < m; ++i) pv += p[i] * x[i];
    const double K = 0.5 * tau * pv;
    w.assign(m, 0.0);
    for (int i = 0; i < m; ++i) w[i] = p[i] - K * x[i];
    for (int i = 0; i < m; ++i) {
      double* row = &C[(size_t)(k + 1 + i) * n + k + 1];
      for (int j = 0; j < m; ++j) row[j] -= x[i] * w[j] + w[i] * x[j];
    }
    for (int i = 0; i < m; ++i) {          // column k below the diagonal is now beta e_1
      C[(size_t)(k + 1 + i) * n + k] = i == 0 ? beta : 0.0;
      C[(size_t)k * n + k + 1 + i] = i == 0 ? beta : 0.0;
    }
    t.tau[k] = tau;
    t.v[k] = x;
  }
  for (int k = 0; k < n; ++k) t.d[k] = C[(size_t)k * n + k];
  if (n >= 2) t.e[n - 2] = C[(size_t)(n - 1) * n + n - 2];
  return t;
}

// Number of eigenvalues of T below x (Sturm sequence of the LDL^T pivots).
int count_below(const Tridiag& t, double x, double pivmin) {
  int c = 0;
  double q = t.d[0] - x;
  if (std::fabs(q) < pivmin) q = -pivmin;
  c += q < 0.0;
  for (int i = 1; i < t.n; ++i) {
    q = t.d[i] - x - t.e[i - 1] * t.e[i - 1] / q;
    if (std::fabs(q) < pivmin) q = -pivmin;
    c += q < 0.0;
  }
  return c;
}

// Solve (T - lam I) x = b in place by Gaussian elimination with partial
// pivoting on the tridiagonal (one extra super-diagonal of fill).
void tridiag_solve(const Tridiag& t, double lam, double tiny, std::vector<double>& b) {
  const int n = t.n;
  std::vector<double> dl(t.e), d(n), du(t.e), du2(n, 0.0);
  std::vector<char> sw(n, 0);
  for (int i = 0; i < n; ++i) d[i] = t.d[i] - lam;
  for (int i = 0; i + 1 < n; ++i) {
    if (std::fabs(d[i]) >= std::fabs(dl[i])) {
      if (d[i] == 0.0) d[i] = tiny;
      const double f = dl[i] / d[i];
      dl[i] = f;
      d[i + 1] -= f * du[i];
    } else {
      const double f = d[i] / dl[i];
      d[i] = dl[i];
      dl[i] = f;
      const double tmp = du[i];
      du[i] = d[i + 1];
      d[i + 1] = tmp - f * d[i + 1];
      if (i + 2 < n) {
        du2[i] = du[i + 1];
        du[i + 1] = -f * du[i + 1];
      }
      sw[i] = 1;
    }
  }
  if (d[n - 1] == 0.0) d[n - 1] = tiny;
  for (int i = 0; i + 1 < n; ++i) {
    if (!sw[i]) {
      b[i + 1] -= dl[i] * b[i];
    } else {
      const double tmp = b[i];
      b[i] = b[i + 1];
      b[i + 1] = tmp - dl[i] * b[i];
    }
  }
  b[n - 1] /= d[n - 1];
  if (n >= 2) b[n - 2] = (b[n - 2] - du[n - 2] * b[n - 1]) / d[n - 2];
  for (int i = n - 3; i >= 0; --i) b[i] = (b[i] - du[i] * b[i + 1] - du2[i] * b[i + 2]) / d[i];
}

// The eigenpairs of the symmetric matrix C (row-major n x n, destroyed) with
// the `count` smallest eigenvalues; count < 0: every eigenvalue <= upper (at
// least one). lam ascending, Y column-major n x count.
void sym_eig_lowest(int n, std::vector<double>& C, int count, double upper, std::vector<double>& lam,
                    std::vector<double>& Y) {
  if (n == 1) {
    lam.assign(1, C[0]);
    Y.assign(1, 1.0);
    return;
  }
  const Tridiag t = tridiagonalize(n, C);
  double lo = t.d[0], hi = t.d[0], tn = 0.0, emax = 0.0;
  for (int i = 0; i < n; ++i) {
    const double r = (i > 0 ? std::fabs(t.e[i - 1]) : 0.0) + (i + 1 < n ? std::fabs(t.e[i]) : 0.0);
    lo = std::min(lo, t.d[i] - r);
    hi = std::max(hi, t.d[i] + r);
    tn = std::max(tn, std::fabs(t.d[i]) + r);
    if (i + 1 < n) emax = std::max(emax, t.e[i] * t.e[i]);
  }
  const double pivmin = DBL_MIN * std::max(1.0, emax);
  lo -= 2.0 * DBL_EPSILON * tn + pivmin;
  hi += 2.0 * DBL_EPSILON * tn + pivmin;
  int r = count;
  if (r < 0) r = std::max(1, std::min(n, count_below(t, upper, pivmin) + 0));
  r = std::min(r, n);
  lam.assign(r, 0.0);
  for (int j = 0; j < r; ++j) {           // bisection for the j-th smallest eigenvalue
    double a = lo, b = hi;
    for (int it = 0; it < 200 && b - a > 2.0 * DBL_EPSILON * std::max(std::fabs(a), std::fabs(b)) + pivmin; ++it) {
      const double mid = 0.5 * (a + b);
      if (count_below(t, mid, pivmin) > j) b = mid; else a = mid;
    }
    lam[j] = 0.5 * (a + b);
  }
  // inverse iteration, orthogonalised within clusters of close eigenvalues
  const double ortol = 1e-3 * tn, tiny = DBL_EPSILON * std::max(tn, DBL_MIN);
  std::vector<std::vector<double>> X(r);
  int first = 0;
  for (int j = 0; j < r; ++j) {
    if (j > 0 && lam[j] - lam[j - 1] > ortol) first = j;
    std::vector<double> x(n);
    for (int i = 0; i < n; ++i) x[i] = std::sin(0.7071 * (i + 1) * (j + 1)) + 1.0 / (i + 2);
    for (int it = 0; it < 4; ++it) {
      tridiag_solve(t, lam[j], tiny, x);
      for (int q = first; q < j; ++q) {
        double dot = 0.0;
        for (int i = 0; i < n; ++i) dot += X[q][i] * x[i];
        for (int i = 0; i < n; ++i) x[i] -= dot * X[q][i];
      }
      double nr = 0.0;
      for (int i = 0; i < n; ++i) nr += x[i] * x[i];
      nr = std::sqrt(nr);
      if (!(nr > 0.0) || !std::isfinite(nr)) gfail(SFROM_ENONFINITE, "inverse iteration failed");
      for (int i = 0; i < n; ++i) x[i] /= nr;
    }
    X[j] = std::move(x);
  }
  // back to the original basis: y = H_0 (H_1 (... H_{n-3} x))
  Y.assign((size_t)n * r, 0.0);
  for (int j = 0; j < r; ++j) {
    std::vector<double>& x = X[j];
    for (int k = n - 3; k >= 0; --k) {
      if (t.tau[k] == 0.0) continue;
      const std::vector<double>& v = t.v[k];
      double dot = 0.0;
      for (int i = 0; i < (int)v.size(); ++i) dot += v[i] * x[k + 1 + i];
      dot *= t.tau[k];
      for (int i = 0; i < (int)v.size(); ++i) x[k + 1 + i] -= dot * v[i];
    }
    std::copy(x.begin(), x.end(), Y.begin() + (size_t)j * n);
  }
}

// ---------------------------------------------------------------------------
// Gramian basis of one piece
// ---------------------------------------------------------------------------

constexpr int GRAMIAN_MAX_NODES = 4096;

Sub union_pencil(const sfrom_t* h, const std::vector<int32_t>& cells) {
  Sub u;
  for (int32_t c : cells) u.nodes.insert(u.nodes.end(), h->cells[c].gnode.begin(), h->cells[c].gnode.end());
  std::sort(u.nodes.begin(), u.nodes.end());
  u.nodes.erase(std::unique(u.nodes.begin(), u.nodes.end()), u.nodes.end());
  const int n = u.n();
  auto at = [&](int64_t g) { return (int)(std::lower_bound(u.nodes.begin(), u.nodes.end(), g) - u.nodes.begin()); };
  std::vector<std::map<int, double>> rows(n);
  u.b.assign(n, 0.0);
  for (int32_t c : cells) {               // sum of the cells' split operators, cell by cell
    const auto& cd = h->cells[c];
    std::vector<int> loc(cd.n);
    for (int r = 0; r < cd.n; ++r) loc[r] = at(cd.gnode[r]);
    for (int r = 0; r < cd.n; ++r) {
      u.b[loc[r]] += cd.b[r];
      for (int t = cd.rowptr[r]; t < cd.rowptr[r + 1]; ++t) {
        auto it = rows[loc[r]].find(loc[cd.col[t]]);
        if (it == rows[loc[r]].end()) rows[loc[r]].emplace(loc[cd.col[t]], cd.a[t]);
        else it->second += cd.a[t];
      }
    }
  }
  u.rp.push_back(0);
  for (int r = 0; r < n; ++r) {
    for (auto& kv : rows[r]) { u.col.push_back(kv.first); u.a.push_back(kv.second); }
    u.rp.push_back((int32_t)u.col.size());
  }
  return u;
}

// ---------------------------------------------------------------------------
// Zolotarev route to the spectral projector (eq. trgrstep)
// ---------------------------------------------------------------------------

// Host memory of one piece's band solves (each of up to 16 worker threads
// holds one piece at a time).
constexpr double ZOLOTAREV_MAX_BYTES = 2.0 * 1024 * 1024 * 1024;

// K(k) = pi / (2 AGM(1, k')).
double agm_ellipk(double k) {
  double a = 1.0, b = std::sqrt(1.0 - k * k);
  for (int it = 0; it < 64 && std::fabs(a - b) > 1e-16 * a; ++it) {
    const double an = 0.5 * (a + b);
    b = std::sqrt(a * b);
    a = an;
  }
  return M_PI / (2.0 * a);
}

// sn and cn of argument u, modulus k, by the arithmetic-geometric mean
// (descending Landen transformation).
void jacobi_sn_cn(double u, double k, double& sn, double& cn) {
  std::vector<double> a{1.0}, b{std::sqrt(1.0 - k * k)}, c{k};
  for (int it = 0; it < 64 && std::fabs(c.back()) > 1e-17; ++it) {
    const double an = 0.5 * (a.back() + b.back());
    c.push_back(0.5 * (a.back() - b.back()));
    b.push_back(std::sqrt(a.back() * b.back()));
    a.push_back(an);
  }
  const int N = (int)a.size() - 1;
  double phi = std::ldexp(a[N] * u, N);
  for (int n = N; n > 0; --n) phi = 0.5 * (phi + std::asin(c[n] * std::sin(phi) / a[n]));
  sn = std::sin(phi);
  cn = std::cos(phi);
}

// Zolotarev's best rational approximation of sign(x) on [-1, -delta] U
// [delta, 1] with n partial fractions: Z(x) = M x sum_j a_j / (x^2 + beta2_j),
// beta2_j = c_{2j-1}, c_i = delta^2 sn^2 / cn^2 (i K' / (2n); k'); M makes
// the error equioscillate on [delta, 1] (from the extrema on a dense
// geometric grid).
void zolotarev_sign(int n, double delta, double& M, std::vector<double>& beta2, std::vector<double>& a) {
  const double kp = std::sqrt(1.0 - delta * delta);
  const double Kp = agm_ellipk(kp);
  std::vector<double> c(2 * n, 0.0);
  for (int i = 1; i < 2 * n; ++i) {
    double sn, cn;
    jacobi_sn_cn(i * Kp / (2 * n), kp, sn, cn);
    c[i] = delta * delta * sn * sn / (cn * cn);
  }
  beta2.assign(n, 0.0);
  a.assign(n, 0.0);
  for (int j = 0; j < n; ++j) beta2[j] = c[2 * j + 1];
  for (int j = 0; j < n; ++j) {
    double num = 1.0, den = 1.0;
    for (int i = 1; i < n; ++i) num *= c[2 * i] - beta2[j];
    for (int i = 0; i < n; ++i)
      if (i != j) den *= beta2[i] - beta2[j];
    a[j] = num / den;
  }
  const int NG = 20001;
  double fmax = -1e300, fmin = 1e300;
  for (int g = 0; g < NG; ++g) {
    const double x = std::exp(std::log(delta) * (1.0 - (double)g / (NG - 1)));
    double f = 0.0;
    for (int j = 0; j < n; ++j) f += a[j] / (x * x + beta2[j]);
    f *= x;
    fmax = std::max(fmax, f);
    fmin = std::min(fmin, f);
  }
  M = 2.0 / (fmax + fmin);
}

// Rows `rows` of Z_w = sum_{lambda <= w^2} z z^T (z B-orthonormal) for the
// local pencil: Z_w = B^{-1/2} (I + sign(X)) / 2 B^{-1/2}, X = (w^2 I - C) / s,
// C = B^{-1/2} (-A) B^{-1/2}, sign(X) by Zolotarev's approximant; each term
// is Im[(X - i beta I)^{-1}] / beta, one complex symmetric band solve
// (LDL^T without pivoting: i (X - i beta I) has Hermitian part beta I > 0)
// in reverse Cuthill-McKee order. Returns -G (k_p x k_p) for the basis step.
std::vector<double> gramian_zolotarev(const Sub& sl, const std::vector<int>& rows, double omega_max, int npole,
                                      double gamma) {
  using cd = std::complex<double>;
  const int n = sl.n(), kp = (int)rows.size();
  const double w2 = omega_max * omega_max;
  std::vector<double> r(n);
  for (int k = 0; k < n; ++k) r[k] = 1.0 / std::sqrt(sl.b[k]);
  double hi = 0.0;   // Gershgorin bound of C
  for (int k = 0; k < n; ++k) {
    double row = 0.0;
    for (int t = sl.rp[k]; t < sl.rp[k + 1]; ++t) {
      const double c = -(sl.a[t] * r[k]) * r[sl.col[t]];
      row += sl.col[t] == k ? c : std::fabs(c);
    }
    hi = std::max(hi, row);
  }
  const double sc = std::max(w2, hi - w2);
  const double delta = std::min(gamma * w2 / sc, 0.5);
  double M;
  std::vector<double> beta2, coef;
  zolotarev_sign(npole, delta, M, beta2, coef);
  // X in reverse Cuthill-McKee order, lower band
  const std::vector<int> perm = rcm(sl);
  std::vector<int> inv(n);
  for (int i = 0; i < n; ++i) inv[perm[i]] = i;
  int w = 0;
  for (int k = 0; k < n; ++k)
    for (int t = sl.rp[k]; t < sl.rp[k + 1]; ++t) w = std::max(w, std::abs(inv[k] - inv[sl.col[t]]));
  auto xval = [&](int k, int t) {
    const double c = -(sl.a[t] * r[k]) * r[sl.col[t]];
    return sl.col[t] == k ? (w2 - c) / sc : -c / sc;
  };
  const size_t W1 = (size_t)w + 1;
  // band factor (complex) and accumulated columns of one piece, per thread
  const double bytes = (double)n * (double)W1 * 16.0 + (double)n * kp * 8.0;
  if (bytes > ZOLOTAREV_MAX_BYTES)
    gfail(SFROM_EINVAL, "local pencil of " + std::to_string(n) + " nodes with half bandwidth " + std::to_string(w) +
                            " needs " + std::to_string((long long)(bytes / 1048576.0)) +
                            " MiB for the band solves, above the per-piece limit of " +
                            std::to_string((long long)(ZOLOTAREV_MAX_BYTES / 1048576.0)) + " MiB (lower depth)");
  std::vector<double> acc((size_t)n * kp, 0.0);   // sum_j a_j (X^2 + beta_j^2)^{-1} E, permuted rows
  std::vector<cd> L((size_t)n * W1), y(n);
  for (int j = 0; j < npole; ++j) {
    const double beta = std::sqrt(beta2[j]);
    std::fill(L.begin(), L.end(), cd(0.0, 0.0));
    for (int k = 0; k < n; ++k)
      for (int t = sl.rp[k]; t < sl.rp[k + 1]; ++t) {
        const int i = inv[k], l = inv[sl.col[t]];
        if (l <= i) L[(size_t)i * W1 + (i - l)] += cd(xval(k, t), 0.0);
      }
    for (int i = 0; i < n; ++i) L[(size_t)i * W1] -= cd(0.0, beta);
    // right-looking band LDL^T: L[i][0] holds d_i, L[i][i-k] the multiplier l_ik
    std::vector<cd> lk(W1);
    for (int k = 0; k < n; ++k) {
      const cd d = L[(size_t)k * W1];
      const int iend = std::min(n - 1, k + w);
      for (int i = k + 1; i <= iend; ++i) lk[i - k] = L[(size_t)i * W1 + (i - k)] / d;
      for (int i = k + 1; i <= iend; ++i) {
        const cd li = lk[i - k] * d;
        if (li == cd(0.0, 0.0)) continue;
        for (int jj = k + 1; jj <= i; ++jj) L[(size_t)i * W1 + (i - jj)] -= li * lk[jj - k];
      }
      for (int i = k + 1; i <= iend; ++i) L[(size_t)i * W1 + (i - k)] = lk[i - k];
    }
    for (int q = 0; q < kp; ++q) {
      std::fill(y.begin(), y.end(), cd(0.0, 0.0));
      const int e = inv[rows[q]];
      y[e] = cd(r[rows[q]], 0.0);
      for (int i = e + 1; i < n; ++i) {      // forward: y_i -= sum_k l_ik y_k
        cd s(0.0, 0.0);
        for (int k = std::max(e, i - w); k < i; ++k) s += L[(size_t)i * W1 + (i - k)] * y[k];
        y[i] -= s;
      }
      for (int i = 0; i < n; ++i) y[i] /= L[(size_t)i * W1];
      for (int i = n - 1; i >= 0; --i) {      // back: x_i -= sum_l l_li x_l
        cd s(0.0, 0.0);
        const int lend = std::min(n - 1, i + w);
        for (int l = i + 1; l <= lend; ++l) s += L[(size_t)l * W1 + (l - i)] * y[l];
        y[i] -= s;
      }
      const double f = coef[j] / beta;
      for (int i = 0; i < n; ++i) acc[(size_t)i * kp + q] += f * y[i].imag();
    }
  }
  // rows of Z_w: r_row / 2 (E + M X acc) at the piece rows
  std::vector<double> G((size_t)kp * kp, 0.0);
  for (int q = 0; q < kp; ++q) {
    const int k = rows[q];
    std::vector<double> xa(kp, 0.0);
    for (int t = sl.rp[k]; t < sl.rp[k + 1]; ++t) {
      const double x = xval(k, t);
      const double* ar = &acc[(size_t)inv[sl.col[t]] * kp];
      for (int s2 = 0; s2 < kp; ++s2) xa[s2] += x * ar[s2];
    }
    for (int s2 = 0; s2 < kp; ++s2) {
      const double e = (s2 == q) ? r[k] : 0.0;
      G[(size_t)q * kp + s2] = r[k] * 0.5 * (e + M * xa[s2]);
    }
  }
  for (int q = 0; q < kp; ++q)
    for (int s2 = 0; s2 <= q; ++s2) {
      const double v = 0.5 * (G[(size_t)q * kp + s2] + G[(size_t)s2 * kp + q]);
      G[(size_t)q * kp + s2] = G[(size_t)s2 * kp + q] = -v;
    }
  return G;
}

// S (k_p x b_p column-major) of one piece; npole > 0 takes G from the
// Zolotarev projector, else from the eigenpairs of the local pencil.
std::vector<double> piece_gramian_basis(const sfrom_t* h, int p, const std::vector<int32_t>& cells, double omega_max,
                                        double eps, int max_modes, int depth, int& bp, int npole = 0,
                                        double gamma = 0.0) {
  const auto& pc = h->pieces[p];
  const int kp = (int)pc.gnode.size();
  if (kp == 1) { bp = 1; return {1.0}; }
  Sub u = union_pencil(h, cells);
  std::vector<char> in(u.n(), 0);
  for (int64_t g : pc.gnode) in[std::lower_bound(u.nodes.begin(), u.nodes.end(), g) - u.nodes.begin()] = 1;
  Sub sl;
  if (depth < 0) {
    sl = std::move(u);
  } else {
    for (int d = 0; d < depth; ++d) in = neighbourhood(u, in);
    const std::vector<char> AO = neighbourhood(u, in);
    if (std::all_of(AO.begin(), AO.end(), [](char c) { return c != 0; })) {
      sl = std::move(u);
    } else {
      Sub two[2];
      alg1(u, prop1(u, in), 0.5, 0.5, two);
      sl = std::move(two[0]);
    }
  }
  const int n = sl.n();
  std::vector<int> rows(kp);
  for (int q = 0; q < kp; ++q)
    rows[q] = (int)(std::lower_bound(sl.nodes.begin(), sl.nodes.end(), pc.gnode[q]) - sl.nodes.begin());
  std::vector<double> G;
  if (npole > 0) {
    G = gramian_zolotarev(sl, rows, omega_max, npole, gamma);
  } else {
  if (n > GRAMIAN_MAX_NODES)
    gfail(SFROM_EINVAL, "piece " + std::to_string(p) + ": local pencil of " + std::to_string(n) +
                            " nodes exceeds the dense limit " + std::to_string(GRAMIAN_MAX_NODES) + " (lower depth)");
  std::vector<double> C((size_t)n * n, 0.0), r(n);
  for (int k = 0; k < n; ++k) r[k] = 1.0 / std::sqrt(sl.b[k]);
  for (int k = 0; k < n; ++k)
    for (int t = sl.rp[k]; t < sl.rp[k + 1]; ++t) C[(size_t)k * n + sl.col[t]] = -(sl.a[t] * r[k]) * r[sl.col[t]];
  for (int k = 0; k < n; ++k)
    for (int l = 0; l < k; ++l) {
      const double s = 0.5 * (C[(size_t)k * n + l] + C[(size_t)l * n + k]);
      C[(size_t)k * n + l] = C[(size_t)l * n + k] = s;
    }
  std::vector<double> lam, Y;
  sym_eig_lowest(n, C, -1, omega_max * omega_max, lam, Y);
  const int nr = (int)lam.size();
  std::vector<double> V((size_t)kp * nr);  // restricted B-orthonormal eigenvectors, column-major
  for (int j = 0; j < nr; ++j)
    for (int q = 0; q < kp; ++q) V[q + (size_t)j * kp] = Y[rows[q] + (size_t)j * n] * r[rows[q]];
  // eigenvectors of G = V V^T, largest first
  G.assign((size_t)kp * kp, 0.0);
  for (int q = 0; q < kp; ++q)
    for (int s = 0; s <= q; ++s) {
      double acc = 0.0;
      for (int j = 0; j < nr; ++j) acc += V[q + (size_t)j * kp] * V[s + (size_t)j * kp];
      G[(size_t)q * kp + s] = G[(size_t)s * kp + q] = -acc;   // lowest of -G = largest of G
    }
  }
  std::vector<double> mu, U;
  const int want = std::min(kp, std::max(1, max_modes));
  sym_eig_lowest(kp, G, want, 0.0, mu, U);
  bp = 1;
  const double top = -mu[0];
  while (bp < want && -mu[bp] > eps * top) ++bp;
  // re-orthonormalise the kept columns (modified Gram-Schmidt, twice)
  for (int pass = 0; pass < 2; ++pass)
    for (int j = 0; j < bp; ++j) {
      double* uj = &U[(size_t)j * kp];
      for (int q = 0; q < j; ++q) {
        const double* uq = &U[(size_t)q * kp];
        double dot = 0.0;
        for (int i = 0; i < kp; ++i) dot += uq[i] * uj[i];
        for (int i = 0; i < kp; ++i) uj[i] -= dot * uq[i];
      }
      double nr2 = 0.0;
      for (int i = 0; i < kp; ++i) nr2 += uj[i] * uj[i];
      const double s = 1.0 / std::sqrt(nr2);
      for (int i = 0; i < kp; ++i) uj[i] *= s;
    }
  U.resize((size_t)kp * bp);
  return U;
}

int worker_count(int jobs) {
  const unsigned hw = std::thread::hardware_concurrency();
  return std::max(1, std::min({jobs, 16, (int)(hw ? hw : 1)}));
}

}  // namespace

extern "C" int sfrom_partition_graph(sfrom_t* h, int32_t n_cells, double alpha, double beta) {
  if (!h) return SFROM_EINVAL;
  try {
    if (h->n <= 0) gfail(SFROM_ESTATE, "no pencil: call sfrom_set_pencil first");
    if (n_cells < 2) gfail(SFROM_EINVAL, "n_cells must be at least 2");
    if (!(alpha >= 0.0 && alpha <= 1.0)) gfail(SFROM_EINVAL, "alpha must lie in [0, 1] (Alg. 1)");
    if (!(beta > 0.0 && beta < 1.0)) gfail(SFROM_EINVAL, "beta must lie in (0, 1) (eq. alg1B)");
    if (h->n >= ((int64_t)1 << 31)) gfail(SFROM_EINVAL, "pencil too large for a general partition");
    Sub whole;
    const int n = (int)h->n;
    whole.nodes.resize(n);
    std::iota(whole.nodes.begin(), whole.nodes.end(), 0);
    whole.rp.assign(h->rowptr.begin(), h->rowptr.end());
    whole.col = h->col;
    whole.a = h->a;
    whole.b = h->b;
    for (int k = 0; k < n; ++k) {
      bool diag = false;
      for (int t = whole.rp[k]; t < whole.rp[k + 1]; ++t) diag |= whole.col[t] == k && whole.a[t] != 0.0;
      if (!diag) gfail(SFROM_EINVAL, "row " + std::to_string(k) + " has no nonzero diagonal entry (Lemma 1)");
    }
    {
      const std::vector<int> lev = levels(whole, 0);
      for (int k = 0; k < n; ++k)
        if (lev[k] < 0) gfail(SFROM_EINVAL, "the graph of A is not connected");
    }
    const std::vector<Sub> subs = alg2(whole, n_cells, alpha, beta);
    // owner sets and pieces
    std::vector<std::vector<int32_t>> owners(n);
    for (int c = 0; c < (int)subs.size(); ++c)
      for (int64_t g : subs[c].nodes) owners[g].push_back(c);
    std::map<std::vector<int32_t>, std::vector<int64_t>> groups;
    for (int g = 0; g < n; ++g)
      if (owners[g].size() >= 2) groups[owners[g]].push_back(g);
    std::vector<const std::vector<int64_t>*> pieces;
    for (auto& kv : groups) pieces.push_back(&kv.second);
    std::sort(pieces.begin(), pieces.end(), [](const std::vector<int64_t>* x, const std::vector<int64_t>* y) {
      return x->front() < y->front();
    });
    // register: cells in reverse Cuthill-McKee order, pieces with the
    // normalised constant vector as a one-column basis
    h->cells.clear();
    h->pieces.clear();
    for (int c = 0; c < (int)subs.size(); ++c) {
      const Sub& s = subs[c];
      const std::vector<int> perm = rcm(s);
      std::vector<int> inv(s.n());
      for (int r = 0; r < s.n(); ++r) inv[perm[r]] = r;
      std::vector<int64_t> gn(s.n());
      std::vector<int32_t> rp{0}, col;
      std::vector<double> a, b(s.n());
      for (int r = 0; r < s.n(); ++r) {
        const int k = perm[r];
        gn[r] = s.nodes[k];
        b[r] = s.b[k];
        std::vector<std::pair<int32_t, double>> row;
        for (int t = s.rp[k]; t < s.rp[k + 1]; ++t) row.push_back({inv[s.col[t]], s.a[t]});
        std::sort(row.begin(), row.end());
        for (auto& e : row) { col.push_back(e.first); a.push_back(e.second); }
        rp.push_back((int32_t)col.size());
      }
      const int rc = sfrom_add_cell(h, c, s.n(), gn.data(), rp.data(), col.data(), a.data(), b.data());
      if (rc != SFROM_OK) return rc;
    }
    for (int p = 0; p < (int)pieces.size(); ++p) {
      const auto& nodes = *pieces[p];
      std::vector<double> S(nodes.size(), 1.0 / std::sqrt((double)nodes.size()));
      const int rc = sfrom_add_piece(h, p, (int32_t)nodes.size(), nodes.data(), 1, S.data());
      if (rc != SFROM_OK) return rc;
    }
    h->src = sfrom_impl::Columns();
    h->rec = sfrom_impl::Columns();
    h->src_dirty = h->rec_dirty = true;
    h->err.clear();
    return SFROM_OK;
  } catch (const GFail& f) {
    h->err = f.msg;
    return f.code;
  } catch (const std::bad_alloc&) {
    h->err = "host allocation failed";
    return SFROM_ENOMEM;
  }
}

namespace {

int gramian_bases_impl(sfrom_t* h, double omega_max, double eps, int32_t max_modes, int32_t depth, int32_t npole,
                       double gamma) {
  if (!h) return SFROM_EINVAL;
  try {
    if (h->n <= 0 || h->cells.empty() || h->pieces.empty()) gfail(SFROM_ESTATE, "no partition defined");
    if (!(omega_max > 0.0) || !std::isfinite(omega_max)) gfail(SFROM_EINVAL, "omega_max must be positive");
    if (!(eps >= 0.0 && eps < 1.0)) gfail(SFROM_EINVAL, "eps must lie in [0, 1)");
    if (max_modes < 1) gfail(SFROM_EINVAL, "max_modes must be at least 1");
    for (const auto& c : h->cells)
      if (!c.defined) gfail(SFROM_ESTATE, "a cell is not defined");
    for (const auto& p : h->pieces)
      if (!p.defined) gfail(SFROM_ESTATE, "a piece is not defined");
    const int np = (int)h->pieces.size();
    // cells holding each piece (from its first node)
    std::vector<std::vector<int32_t>> node_cells(h->n);
    for (int c = 0; c < (int)h->cells.size(); ++c)
      for (int64_t g : h->cells[c].gnode) node_cells[g].push_back(c);
    std::vector<std::vector<double>> S(np);
    std::vector<int> bp(np, 0);
    std::vector<int> err_code(np, 0);
    std::vector<std::string> err_msg(np);
    std::atomic<int> next{0};
    auto work = [&]() {
      for (;;) {
        const int p = next.fetch_add(1);
        if (p >= np) return;
        try {
          S[p] = piece_gramian_basis(h, p, node_cells[h->pieces[p].gnode[0]], omega_max, eps, max_modes, depth, bp[p],
                                     npole, gamma);
        } catch (const GFail& f) {
          err_code[p] = f.code;
          err_msg[p] = f.msg;
        } catch (const std::bad_alloc&) {
          err_code[p] = SFROM_ENOMEM;
          err_msg[p] = "host allocation failed";
        }
      }
    };
    const int nw = worker_count(np);
    std::vector<std::thread> pool;
    for (int w = 1; w < nw; ++w) pool.emplace_back(work);
    work();
    for (auto& t : pool) t.join();
    for (int p = 0; p < np; ++p)
      if (err_code[p] != 0) gfail(err_code[p], err_msg[p]);
    for (int p = 0; p < np; ++p) {
      const std::vector<int64_t> nodes = h->pieces[p].gnode;
      h->pieces[p].defined = false;
      const int rc = sfrom_add_piece(h, p, (int32_t)nodes.size(), nodes.data(), bp[p], S[p].data());
      if (rc != SFROM_OK) return rc;
    }
    h->src = sfrom_impl::Columns();
    h->rec = sfrom_impl::Columns();
    h->src_dirty = h->rec_dirty = true;
    h->err.clear();
    return SFROM_OK;
  } catch (const GFail& f) {
    h->err = f.msg;
    return f.code;
  } catch (const std::bad_alloc&) {
    h->err = "host allocation failed";
    return SFROM_ENOMEM;
  }
}

}  // namespace

extern "C" int sfrom_gramian_bases(sfrom_t* h, double omega_max, double eps, int32_t max_modes, int32_t depth) {
  return gramian_bases_impl(h, omega_max, eps, max_modes, depth, 0, 0.0);
}

extern "C" int sfrom_gramian_bases_zolotarev(sfrom_t* h, double omega_max, double eps, int32_t max_modes,
                                             int32_t depth, int32_t n_poles, double gamma) {
  if (!h) return SFROM_EINVAL;
  if (n_poles < 1 || n_poles > 64 || !(gamma > 0.0 && gamma < 1.0)) {
    h->err = "n_poles must lie in [1, 64] and gamma in (0, 1)";
    return SFROM_EINVAL;
  }
  return gramian_bases_impl(h, omega_max, eps, max_modes, depth, n_poles, gamma);
}

// ---------------------------------------------------------------------------
// Corner-set removal with hanging nodes (App. B; the 2D example of Sec. 3)
// ---------------------------------------------------------------------------
//
// Readings (the paper leaves these open or states them inconsistently):
// * Corner set: the nodes held by three or more cells.
// * Pairs of a corner node k: the pairs {i, j} of cells holding k that also
//   share a node outside the corner set (faces in the Cartesian case; the
//   four copies of the 2D example); if some cell holding k lies in none of
//   them, every pair of cells holding k. One hanging node per pair, held by
//   the pair's two cells only.
// * Entries: App. B copies each cell's whole row of k into every copy,
//   which repeats links in the rows of k's neighbours (A' indefinite) and
//   multiplies the corner mass. Here cell c's entries at k are shared
//   equally among its n_c(k) copies: a link of weight w to a node l outside
//   the corner set gives w / n_c(k) per copy; a link between two corner
//   nodes joins the copies of the same pair, w / |Q| for each of the Q pairs
//   both have in c (all n_c(k) n_c(l) copy pairs at w / (n_c(k) n_c(l)) if
//   they share none); the row sum of c's row k goes to each copy's diagonal
//   as d_k / n_c(k), minus the weights of the copy's links; the mass is
//   b_c(k) / n_c(k). With E copying each old value to its copies,
//   E^T A' E = A and E^T B' E = B.
// * Numbering: old nodes ascending; a kept node gets one new id, a corner
//   node one per pair (pairs in lexicographic order). Row sums and diagonal
//   updates run over each cell row in ascending old column order. Each
//   cell keeps its local order, a corner node's copies in its place.
// * App. D weights of the copies l of k: b'_l / b_k (they sum to one).

namespace {

struct Copy {
  int32_t pi, pj;     // the pair (-1, -1 for a kept node)
  int64_t id;         // new global id
};

}  // namespace

extern "C" int sfrom_remove_corner_set(sfrom_t* h, int64_t* n_new, int32_t* n_corner, int64_t* n_hanging) {
  if (!h) return SFROM_EINVAL;
  try {
    if (h->n <= 0 || h->cells.empty()) gfail(SFROM_ESTATE, "no partition defined");
    for (size_t c = 0; c < h->cells.size(); ++c)
      if (!h->cells[c].defined) gfail(SFROM_ESTATE, "cell " + std::to_string(c) + " is not defined");
    if (!h->cmap.corner.empty()) gfail(SFROM_ESTATE, "the corner set was already removed");
    const int64_t n0 = h->n;
    const int nc = (int)h->cells.size();
    std::vector<std::vector<int32_t>> owners(n0);
    for (int c = 0; c < nc; ++c)
      for (int64_t g : h->cells[c].gnode) owners[g].push_back(c);
    std::vector<std::pair<int32_t, int32_t>> iface;
    for (int64_t g = 0; g < n0; ++g)
      if (owners[g].size() == 2) iface.push_back({owners[g][0], owners[g][1]});
    std::sort(iface.begin(), iface.end());
    iface.erase(std::unique(iface.begin(), iface.end()), iface.end());
    auto is_iface = [&](int32_t i, int32_t j) { return std::binary_search(iface.begin(), iface.end(), std::make_pair(i, j)); };
    std::vector<int64_t> corner;
    std::vector<std::vector<std::pair<int32_t, int32_t>>> cpairs;
    std::vector<int32_t> corner_of(n0, -1);
    for (int64_t g = 0; g < n0; ++g) {
      const auto& own = owners[g];
      if (own.size() < 3) continue;
      std::vector<std::pair<int32_t, int32_t>> allp, pairs;
      for (size_t a = 0; a < own.size(); ++a)
        for (size_t b = a + 1; b < own.size(); ++b) allp.push_back({own[a], own[b]});
      for (auto& pr : allp)
        if (is_iface(pr.first, pr.second)) pairs.push_back(pr);
      bool covered = true;
      for (int32_t c : own) {
        bool in = false;
        for (auto& pr : pairs) in |= pr.first == c || pr.second == c;
        covered &= in;
      }
      corner_of[g] = (int32_t)corner.size();
      corner.push_back(g);
      cpairs.push_back(covered ? pairs : allp);
    }
    if (n_corner) *n_corner = (int32_t)corner.size();
    if (corner.empty()) {
      if (n_new) *n_new = n0;
      if (n_hanging) *n_hanging = 0;
      h->err.clear();
      return SFROM_OK;
    }
    std::vector<int64_t> new_of_old(n0, -1), cbase(corner.size());
    int64_t nid = 0;
    for (int64_t g = 0; g < n0; ++g) {
      if (corner_of[g] >= 0) {
        cbase[corner_of[g]] = nid;
        nid += (int64_t)cpairs[corner_of[g]].size();
      } else {
        new_of_old[g] = nid++;
      }
    }
    const int64_t n1 = nid;
    if (n1 >= ((int64_t)1 << 31)) gfail(SFROM_EINVAL, "pencil too large after the corner-set removal");
    auto copies = [&](int32_t c, int64_t g, std::vector<Copy>& out) {
      out.clear();
      const int32_t k = corner_of[g];
      if (k < 0) {
        out.push_back({-1, -1, new_of_old[g]});
        return;
      }
      const auto& pr = cpairs[k];
      for (size_t q = 0; q < pr.size(); ++q)
        if (pr[q].first == c || pr[q].second == c) out.push_back({pr[q].first, pr[q].second, cbase[k] + (int64_t)q});
    };
    struct NewCell {
      std::vector<int64_t> gn;
      std::vector<int32_t> rp{0}, col;
      std::vector<double> a, b;
    };
    std::vector<NewCell> ncell(nc);
    std::vector<Copy> cr, cl;
    for (int c = 0; c < nc; ++c) {
      const sfrom_impl::CellDef& cd = h->cells[c];
      NewCell& out = ncell[c];
      std::vector<std::vector<Copy>> cps(cd.n);
      std::vector<int32_t> first(cd.n + 1, 0);
      for (int r = 0; r < cd.n; ++r) {
        copies(c, cd.gnode[r], cps[r]);
        first[r + 1] = first[r] + (int32_t)cps[r].size();
        for (const Copy& x : cps[r]) out.gn.push_back(x.id);
      }
      out.b.resize(first[cd.n]);
      std::vector<std::tuple<int64_t, int32_t, double>> row;
      std::vector<std::pair<int32_t, double>> nrow;
      for (int r = 0; r < cd.n; ++r) {
        const int64_t g = cd.gnode[r];
        row.clear();
        for (int t = cd.rowptr[r]; t < cd.rowptr[r + 1]; ++t) row.emplace_back(cd.gnode[cd.col[t]], cd.col[t], cd.a[t]);
        std::sort(row.begin(), row.end());
        double d = 0.0;
        for (auto& e : row) d += std::get<2>(e);
        const auto& cg = cps[r];
        const int ng = (int)cg.size();
        for (int q = 0; q < ng; ++q) {
          nrow.clear();
          double diag = d / ng;
          for (auto& e : row) {
            const int32_t l = std::get<1>(e);
            if (l == r) continue;
            const double w = std::get<2>(e);
            const auto& cq = cps[l];
            const int nl = (int)cq.size();
            const bool kc = corner_of[g] >= 0, lc = corner_of[std::get<0>(e)] >= 0;
            auto push = [&](int ql, double wt) {
              nrow.push_back({first[l] + ql, wt});
              diag -= wt;
            };
            if (kc && lc) {
              int nq = 0, match = -1;
              for (int a = 0; a < ng; ++a)
                for (int b = 0; b < nl; ++b)
                  if (cg[a].pi == cq[b].pi && cg[a].pj == cq[b].pj) {
                    ++nq;
                    if (a == q) match = b;
                  }
              if (nq > 0) {
                if (match >= 0) push(match, w / nq);
              } else {
                for (int b = 0; b < nl; ++b) push(b, w / (ng * nl));
              }
            } else if (kc) {
              push(0, w / ng);
            } else if (lc) {
              for (int b = 0; b < nl; ++b) push(b, w / nl);
            } else {
              push(0, w);
            }
          }
          nrow.push_back({first[r] + q, diag});
          std::sort(nrow.begin(), nrow.end());
          for (auto& e : nrow) { out.col.push_back(e.first); out.a.push_back(e.second); }
          out.rp.push_back((int32_t)out.col.size());
          out.b[first[r] + q] = cd.b[r] / ng;
        }
      }
    }
    // the pencil: sum of the cells (each new node lies in at most two)
    std::vector<std::vector<std::pair<int32_t, double>>> grow(n1);
    std::vector<double> b1(n1, 0.0);
    for (int c = 0; c < nc; ++c) {
      const NewCell& x = ncell[c];
      for (size_t r = 0; r < x.gn.size(); ++r) {
        b1[x.gn[r]] += x.b[r];
        for (int t = x.rp[r]; t < x.rp[r + 1]; ++t) grow[x.gn[r]].push_back({(int32_t)x.gn[x.col[t]], x.a[t]});
      }
    }
    std::vector<int64_t> rp1{0};
    std::vector<int32_t> col1;
    std::vector<double> a1;
    for (int64_t g = 0; g < n1; ++g) {
      auto& rw = grow[g];
      std::stable_sort(rw.begin(), rw.end(), [](const std::pair<int32_t, double>& x, const std::pair<int32_t, double>& y) {
        return x.first < y.first;
      });
      for (size_t t = 0; t < rw.size(); ++t) {
        if (!col1.empty() && (int64_t)col1.size() > rp1.back() && col1.back() == rw[t].first) a1.back() += rw[t].second;
        else { col1.push_back(rw[t].first); a1.push_back(rw[t].second); }
      }
      rp1.push_back((int64_t)col1.size());
      std::vector<std::pair<int32_t, double>>().swap(rw);
    }
    sfrom::CornerMap cm;
    cm.n_old = n0;
    cm.new_of_old = new_of_old;
    cm.corner = corner;
    cm.hptr.push_back(0);
    for (size_t k = 0; k < corner.size(); ++k) {
      for (size_t q = 0; q < cpairs[k].size(); ++q) {
        const int64_t l = cbase[k] + (int64_t)q;
        cm.hnode.push_back(l);
        cm.hweight.push_back(b1[l] / h->b[corner[k]]);
      }
      cm.hptr.push_back((int64_t)cm.hnode.size());
    }
    // replace the pencil and the partition; pieces get the normalised
    // constant vector as a one-column basis until bases are set
    int rc = sfrom_set_pencil(h, n1, rp1.data(), col1.data(), a1.data(), b1.data());
    if (rc != SFROM_OK) return rc;
    std::vector<std::vector<int32_t>> own1(n1);
    for (int c = 0; c < nc; ++c) {
      const NewCell& x = ncell[c];
      rc = sfrom_add_cell(h, c, (int32_t)x.gn.size(), x.gn.data(), x.rp.data(), x.col.data(), x.a.data(), x.b.data());
      if (rc != SFROM_OK) return rc;
      for (int64_t g : x.gn) own1[g].push_back(c);
    }
    std::map<std::vector<int32_t>, std::vector<int64_t>> groups;
    for (int64_t g = 0; g < n1; ++g)
      if (own1[g].size() >= 2) groups[own1[g]].push_back(g);
    std::vector<const std::vector<int64_t>*> pieces;
    for (auto& kv : groups) pieces.push_back(&kv.second);
    std::sort(pieces.begin(), pieces.end(), [](const std::vector<int64_t>* x, const std::vector<int64_t>* y) {
      return x->front() < y->front();
    });
    for (int p = 0; p < (int)pieces.size(); ++p) {
      const auto& nodes = *pieces[p];
      std::vector<double> S(nodes.size(), 1.0 / std::sqrt((double)nodes.size()));
      rc = sfrom_add_piece(h, p, (int32_t)nodes.size(), nodes.data(), 1, S.data());
      if (rc != SFROM_OK) return rc;
    }
    h->cmap = std::move(cm);
    if (n_new) *n_new = n1;
    if (n_hanging) *n_hanging = (int64_t)h->cmap.hnode.size();
    h->err.clear();
    return SFROM_OK;
  } catch (const GFail& f) {
    h->err = f.msg;
    return f.code;
  } catch (const std::bad_alloc&) {
    h->err = "host allocation failed";
    return SFROM_ENOMEM;
  }
}

extern "C" int sfrom_corner_map(sfrom_t* h, int64_t* new_of_old, int64_t* corner, int64_t* hang_ptr,
                                int64_t* hang_node, double* hang_weight) {
  if (!h) return SFROM_EINVAL;
  const auto& cm = h->cmap;
  if (cm.corner.empty()) {
    h->err = "no corner set was removed: call sfrom_remove_corner_set";
    return SFROM_ESTATE;
  }
  h->err.clear();
  if (new_of_old) std::copy(cm.new_of_old.begin(), cm.new_of_old.end(), new_of_old);
  if (corner) std::copy(cm.corner.begin(), cm.corner.end(), corner);
  if (hang_ptr) std::copy(cm.hptr.begin(), cm.hptr.end(), hang_ptr);
  if (hang_node) std::copy(cm.hnode.begin(), cm.hnode.end(), hang_node);
  if (hang_weight) std::copy(cm.hweight.begin(), cm.hweight.end(), hang_weight);
  return SFROM_OK;
}
