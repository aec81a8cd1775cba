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

// Alg. 1 (steps 1-3) and eq. alg1B: the two split operators.
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
        if (own) {                        // step 1
          o.col.push_back(pos[l]);
          o.a.push_back(v);
        } else if (both_gamma) {
          o.col.push_back(pos[l]);
          if (l == k) {
            diag_at = (int64_t)o.a.size();
            o.a.push_back(0.0);
          } else {                        // step 2
            o.a.push_back((i == 0 ? alpha : 1.0 - alpha) * v);
          }
        }
      }
      if (code[k] == 3) {                 // step 3
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

// S (k_p x b_p column-major) of one piece.
std::vector<double> piece_gramian_basis(const sfrom_t* h, int p, const std::vector<int32_t>& cells, double omega_max,
                                        double eps, int max_modes, int depth, int& bp) {
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
  std::vector<int> rows(kp);
  for (int q = 0; q < kp; ++q)
    rows[q] = (int)(std::lower_bound(sl.nodes.begin(), sl.nodes.end(), pc.gnode[q]) - sl.nodes.begin());
  std::vector<double> V((size_t)kp * nr);  // restricted B-orthonormal eigenvectors, column-major
  for (int j = 0; j < nr; ++j)
    for (int q = 0; q < kp; ++q) V[q + (size_t)j * kp] = Y[rows[q] + (size_t)j * n] * r[rows[q]];
  // eigenvectors of G = V V^T, largest first
  std::vector<double> G((size_t)kp * kp, 0.0);
  for (int q = 0; q < kp; ++q)
    for (int s = 0; s <= q; ++s) {
      double acc = 0.0;
      for (int j = 0; j < nr; ++j) acc += V[q + (size_t)j * kp] * V[s + (size_t)j * kp];
      G[(size_t)q * kp + s] = G[(size_t)s * kp + q] = -acc;   // lowest of -G = largest of G
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
    if (!(alpha >= 0.0 && alpha <= 1.0)) gfail(SFROM_EINVAL, "alpha must lie in [0, 1] (Alg. 1, step 2)");
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

extern "C" int sfrom_gramian_bases(sfrom_t* h, double omega_max, double eps, int32_t max_modes, int32_t depth) {
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
          S[p] = piece_gramian_basis(h, p, node_cells[h->pieces[p].gnode[0]], omega_max, eps, max_modes, depth, bp[p]);
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
