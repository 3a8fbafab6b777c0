// Host-side setup (see host.hpp).  Everything here runs once per context.
#include "host.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>

#ifdef _OPENMP
#include <omp.h>
#endif

namespace stmg {

// ------------------------------------------------------------ polynomials
static double leg(int n, double x) {
  if (n == 0) return 1.0;
  double p0 = 1.0, p1 = x;
  for (int m = 1; m < n; ++m) {
    double p2 = ((2.0 * m + 1.0) * x * p1 - m * p0) / (m + 1.0);
    p0 = p1;
    p1 = p2;
  }
  return p1;
}

// P_n'(x) = sum_{j = n-1, n-3, ...} (2j+1) P_j(x)
static double leg_d(int n, double x) {
  double s = 0.0;
  for (int j = n - 1; j >= 0; j -= 2) s += (2.0 * j + 1.0) * leg(j, x);
  return s;
}

// All roots in (-1,1) of a function with simple roots: bracket on a fine grid,
// then bisect to machine precision.
static std::vector<double> roots(const std::function<double(double)>& f, int expect) {
  std::vector<double> out;
  const int M = 20000;
  double xa = -1.0 + 1e-12, fa = f(xa);
  for (int s = 1; s <= M; ++s) {
    double xb = -1.0 + 2.0 * s / M - (s == M ? 1e-12 : 0.0), fb = f(xb);
    if (fa == 0.0) {
      out.push_back(xa);
    } else if (fa * fb < 0.0) {
      double lo = xa, hi = xb, flo = fa;
      for (int it = 0; it < 200 && hi - lo > 1e-16; ++it) {
        double mid = 0.5 * (lo + hi), fm = f(mid);
        if (fm == 0.0) { lo = hi = mid; break; }
        if ((fm < 0.0) == (flo < 0.0)) { lo = mid; flo = fm; } else { hi = mid; }
      }
      out.push_back(0.5 * (lo + hi));
    }
    xa = xb;
    fa = fb;
  }
  if ((int)out.size() != expect) throw Error(-6, "polynomial root bracketing failed");
  return out;
}

void gauss01(int n, std::vector<double>& x, std::vector<double>& w) {
  std::vector<double> r = roots([n](double t) { return leg(n, t); }, n);
  x.resize(n);
  w.resize(n);
  for (int i = 0; i < n; ++i) {
    double d = leg_d(n, r[i]);
    x[i] = 0.5 * (r[i] + 1.0);
    w[i] = 0.5 * 2.0 / ((1.0 - r[i] * r[i]) * d * d);
  }
}

std::vector<double> lobatto01(int n) {
  std::vector<double> x(n);
  x[0] = 0.0;
  x[n - 1] = 1.0;
  if (n > 2) {
    std::vector<double> r = roots([n](double t) { return leg_d(n - 1, t); }, n - 2);
    for (int i = 0; i < n - 2; ++i) x[i + 1] = 0.5 * (r[i] + 1.0);
  }
  return x;
}

// Right Radau with k+1 points: the roots of P_k - P_{k+1} and t = 1; weights
// (1 + t_i) / ((k+1)^2 P_k(t_i)^2) and 2/(k+1)^2 at t = 1 (mirror image of the
// classical left Radau weights).
void radau_right(int k, std::vector<double>& t, std::vector<double>& w) {
  int n = k + 1;
  t.assign(n, 1.0);
  w.assign(n, 2.0 / (n * n));
  if (k > 0) {
    std::vector<double> r = roots([k](double x) { return leg(k, x) - leg(k + 1, x); }, k);
    for (int i = 0; i < k; ++i) {
      double p = leg(k, r[i]);
      t[i] = r[i];
      w[i] = (1.0 + r[i]) / ((double)n * n * p * p);
    }
  }
}

void lagrange_eval(const std::vector<double>& nodes, double x, double* val, double* der) {
  int n = (int)nodes.size();
  for (int i = 0; i < n; ++i) {
    double v = 1.0, dv = 0.0;
    for (int m = 0; m < n; ++m) {
      if (m == i) continue;
      double inv = 1.0 / (nodes[i] - nodes[m]);
      dv = dv * (x - nodes[m]) * inv + v * inv;  // product rule, running
      v *= (x - nodes[m]) * inv;
    }
    if (val) val[i] = v;
    if (der) der[i] = dv;
  }
}

double legendre01(int m, double x) { return leg(m, 2.0 * x - 1.0); }

int binom(int n, int k) {
  long long r = 1;
  for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
  return (int)r;
}

std::vector<int> pressure_modes(int d, int r) {
  std::vector<int> out;
  for (int t = 0; t <= r; ++t) {
    // exponents (a0, ..., a_{d-1}) with sum t, a0 largest first, then a1, ...
    if (d == 2) {
      for (int a0 = t; a0 >= 0; --a0) { out.push_back(a0); out.push_back(t - a0); }
    } else {
      for (int a0 = t; a0 >= 0; --a0)
        for (int a1 = t - a0; a1 >= 0; --a1) {
          out.push_back(a0); out.push_back(a1); out.push_back(t - a0 - a1);
        }
    }
  }
  return out;
}

TimeData time_data(int k) {
  TimeData T;
  T.k = k;
  radau_right(k, T.t, T.w);
  int n = k + 1;
  T.K.assign(n * n, 0.0);
  T.phim1.assign(n, 0.0);
  std::vector<double> val(n), der(n), vm(n);
  lagrange_eval(T.t, -1.0, vm.data(), nullptr);
  for (int a = 0; a < n; ++a) T.phim1[a] = vm[a];
  // K_ab = int phi_b' phi_a + phi_b(-1) phi_a(-1); the integrand has degree
  // 2k-1, so the Radau rule is exact and only mu = a survives.
  for (int a = 0; a < n; ++a) {
    lagrange_eval(T.t, T.t[a], val.data(), der.data());
    for (int b = 0; b < n; ++b) T.K[a * n + b] = T.w[a] * der[b] + vm[b] * vm[a];
  }
  return T;
}

SpaceTables space_tables(int d, int r) {
  SpaceTables S;
  S.d = d;
  S.r = r;
  S.Q = r + 2;
  int Q = S.Q;
  S.nloc = d == 2 ? Q * Q : Q * Q * Q;
  S.gll = lobatto01(Q);
  gauss01(Q, S.gx, S.gw);
  S.S.resize(Q * Q);
  S.D.resize(Q * Q);
  S.Dg.resize(Q * Q);
  for (int p = 0; p < Q; ++p) {
    lagrange_eval(S.gll, S.gx[p], &S.S[p * Q], &S.D[p * Q]);
    lagrange_eval(S.gx, S.gx[p], nullptr, &S.Dg[p * Q]);
  }
  S.modes = pressure_modes(d, r);
  S.C = (int)S.modes.size() / d;
  S.psi.resize((size_t)S.nloc * S.C);
  for (int p = 0; p < S.nloc; ++p) {
    int pi[3] = {p % Q, (p / Q) % Q, p / (Q * Q)};
    for (int l = 0; l < S.C; ++l) {
      double v = 1.0;
      for (int j = 0; j < d; ++j) v *= legendre01(S.modes[l * d + j], S.gx[pi[j]]);
      S.psi[(size_t)p * S.C + l] = v;
    }
  }
  return S;
}

// ---------------------------------------------------------------- levels
std::vector<LevelSpec> build_levels(int n, int r, int k, int N, int n_coarse, int r_min, int k_min,
                                    bool time_h, int placement) {
  std::vector<LevelSpec> L;
  if (placement == 0) {
    // Alg. 2 for space (p-halving on the fine mesh, then h) and for time
    // (p-halving, then optional h), Alg. 3: pad the shorter list at its fine
    // end and pair level by level -> temporal coarsening on the coarsest levels.
    std::vector<std::pair<int, int>> sp{{n, r}}, tm{{N, k}};
    while (r > r_min) { r = std::max(r / 2, r_min); sp.push_back({n, r}); }
    while (n > n_coarse) { n /= 2; sp.push_back({n, r}); }
    while (k > k_min) { k = std::max(k / 2, k_min); tm.push_back({N, k}); }
    if (time_h)
      while (N > 1) { N /= 2; tm.push_back({N, k}); }
    size_t len = std::max(sp.size(), tm.size());
    while (sp.size() < len) sp.insert(sp.begin(), sp.front());
    while (tm.size() < len) tm.insert(tm.begin(), tm.front());
    for (size_t i = 0; i < len; ++i) L.push_back({sp[i].first, sp[i].second, tm[i].second, tm[i].first});
    return L;
  }
  // placement 1: halve r and k together on the fine mesh first, then h
  L.push_back({n, r, k, N});
  while (r > r_min || k > k_min) {
    if (r > r_min) r = std::max(r / 2, r_min);
    if (k > k_min) k = std::max(k / 2, k_min);
    L.push_back({n, r, k, N});
  }
  int hsteps = 0;
  for (int m = n; m > n_coarse; m /= 2) ++hsteps;
  int tsteps = 0;
  if (time_h)
    for (int M = N; M > 1; M /= 2) ++tsteps;
  for (int s = 0; s < hsteps; ++s) {
    n /= 2;
    if (time_h && s >= hsteps - tsteps) N = std::max(N / 2, 1);
    L.push_back({n, r, k, N});
  }
  return L;
}

// ------------------------------------------------------------ geometry
static void cell_jacobian(const LevelHost& L, int64_t c, const double* xi, double* x, double* J) {
  const int d = L.d;
  int64_t cc[3] = {c % L.n, (c / L.n) % L.n, d == 3 ? c / ((int64_t)L.n * L.n) : 0};
  for (int i = 0; i < d; ++i) {
    x[i] = 0.0;
    for (int j = 0; j < d; ++j) J[i * d + j] = 0.0;
  }
  int64_t nv = L.n + 1;
  for (int v = 0; v < (1 << d); ++v) {
    int64_t idx = 0, stride = 1;
    double N = 1.0, dN[3] = {1.0, 1.0, 1.0};
    for (int j = 0; j < d; ++j) {
      int bit = (v >> j) & 1;
      idx += (cc[j] + bit) * stride;
      stride *= nv;
      double f = bit ? xi[j] : 1.0 - xi[j];
      double df = bit ? 1.0 : -1.0;
      N *= f;
      for (int g = 0; g < d; ++g) dN[g] *= (g == j) ? df : f;
    }
    const double* X = &L.verts[idx * d];
    for (int i = 0; i < d; ++i) {
      x[i] += N * X[i];
      for (int j = 0; j < d; ++j) J[i * d + j] += X[i] * dN[j];
    }
  }
}

static double inv_det(int d, const double* J, double* Ji) {
  if (d == 2) {
    double det = J[0] * J[3] - J[1] * J[2];
    Ji[0] = J[3] / det; Ji[1] = -J[1] / det; Ji[2] = -J[2] / det; Ji[3] = J[0] / det;
    return det;
  }
  double c00 = J[4] * J[8] - J[5] * J[7], c01 = J[5] * J[6] - J[3] * J[8], c02 = J[3] * J[7] - J[4] * J[6];
  double det = J[0] * c00 + J[1] * c01 + J[2] * c02;
  Ji[0] = c00 / det; Ji[3] = c01 / det; Ji[6] = c02 / det;
  Ji[1] = (J[2] * J[7] - J[1] * J[8]) / det;
  Ji[4] = (J[0] * J[8] - J[2] * J[6]) / det;
  Ji[7] = (J[1] * J[6] - J[0] * J[7]) / det;
  Ji[2] = (J[1] * J[5] - J[2] * J[4]) / det;
  Ji[5] = (J[2] * J[3] - J[0] * J[5]) / det;
  Ji[8] = (J[0] * J[4] - J[1] * J[3]) / det;
  return det;
}

int apply_geometry_count(int d) { return 1 + d * d + d * (d + 1) / 2; }

void apply_geometry(const LevelHost& L, std::vector<double>& geo) {
  const int d = L.d, Q = L.Q, NG = apply_geometry_count(d), ZP = d == 3 ? Q : 1;
  geo.assign((size_t)L.ncells * NG * 16 * ZP, 0.0);
#pragma omp parallel for schedule(static)
  for (int64_t c = 0; c < L.ncells; ++c) {
    double J[9], Ji[9], X[3], xi[3];
    for (int z = 0; z < ZP; ++z)
      for (int py = 0; py < Q; ++py)
        for (int px = 0; px < Q; ++px) {
          const int pi[3] = {px, py, z};
          double wq = 1.0;
          for (int j = 0; j < d; ++j) { xi[j] = L.st.gx[pi[j]]; wq *= L.st.gw[pi[j]]; }
          cell_jacobian(L, c, xi, X, J);
          const double det = inv_det(d, J, Ji);
          const double jxw = det * wq;
          const int p = px + Q * py + Q * Q * z;
          const double nu = L.nu_q.empty() ? L.nu_const : L.nu_q[(size_t)c * L.nloc + p];
          double f[16];
          f[0] = jxw;
          for (int j = 0; j < d; ++j)
            for (int i = 0; i < d; ++i) f[1 + j * d + i] = jxw * Ji[j * d + i];
          int o = 1 + d * d;
          for (int j = 0; j < d; ++j)
            for (int k = j; k < d; ++k) {
              double s = 0.0;
              for (int i = 0; i < d; ++i) s += Ji[j * d + i] * Ji[k * d + i];
              f[o++] = nu * jxw * s;
            }
          for (int g = 0; g < NG; ++g) geo[(((size_t)c * NG + g) * 16 + px + 4 * py) * ZP + z] = f[g];
        }
  }
}

void build_level(const Params& P, const LevelSpec& s, LevelHost& L) {
  L.d = P.d; L.n = s.n; L.r = s.r; L.k = s.k; L.N = s.N;
  L.tau = P.tau * P.N / s.N;
  L.st = space_tables(P.d, s.r);
  L.td = time_data(s.k);
  const int d = L.d, Q = L.st.Q;
  L.Q = Q; L.q = s.r + 1; L.nn = s.n * L.q + 1; L.C = L.st.C; L.nloc = L.st.nloc; L.nt = s.k + 1;
  L.ncells = d == 2 ? (int64_t)s.n * s.n : (int64_t)s.n * s.n * s.n;
  L.nodes = d == 2 ? (int64_t)L.nn * L.nn : (int64_t)L.nn * L.nn * L.nn;
  L.Mv = d * L.nodes;
  L.Mp = L.ncells * L.C;
  L.slab = (int64_t)L.nt * (L.Mv + L.Mp);
  L.ndofs = (int64_t)s.N * L.slab;
  // vertices, x fastest, deformed in every coordinate
  int64_t nv = s.n + 1, nvert = d == 2 ? nv * nv : nv * nv * nv;
  L.verts.resize(nvert * d);
  for (int64_t v = 0; v < nvert; ++v) {
    double X[3] = {(double)(v % nv) / s.n, (double)((v / nv) % nv) / s.n,
                   d == 3 ? (double)(v / (nv * nv)) / s.n : 0.0};
    double prod = 1.0;
    for (int j = 0; j < d; ++j) prod *= std::sin(2.0 * M_PI * X[j]);
    for (int j = 0; j < d; ++j) L.verts[v * d + j] = X[j] + P.amp * prod;
  }
  const int nl = L.nloc, C = L.C;
  // quadrature points (x fastest) and physical positions for nu(x)
  std::vector<double> xq((size_t)nl * d), wq(nl);
  for (int p = 0; p < nl; ++p) {
    int pi[3] = {p % Q, (p / Q) % Q, p / (Q * Q)};
    wq[p] = 1.0;
    for (int j = 0; j < d; ++j) { xq[p * d + j] = L.st.gx[pi[j]]; wq[p] *= L.st.gw[pi[j]]; }
  }
  L.nu_const = P.nu;
  if (P.nu_fn) {
    std::vector<double> pts((size_t)L.ncells * nl * d);
    double J[9], x[3];
    for (int64_t c = 0; c < L.ncells; ++c)
      for (int p = 0; p < nl; ++p) {
        cell_jacobian(L, c, &xq[p * d], x, J);
        for (int j = 0; j < d; ++j) pts[((size_t)c * nl + p) * d + j] = x[j];
      }
    L.nu_q.resize((size_t)L.ncells * nl);
    P.nu_fn((int)(L.ncells * nl), pts.data(), L.nu_q.data());
  }
  // basis values / reference gradients at the Gauss points
  std::vector<double> phi((size_t)nl * nl), dphi((size_t)nl * nl * d);
  for (int p = 0; p < nl; ++p) {
    int pi[3] = {p % Q, (p / Q) % Q, p / (Q * Q)};
    for (int i = 0; i < nl; ++i) {
      int ii[3] = {i % Q, (i / Q) % Q, i / (Q * Q)};
      double v = 1.0;
      for (int j = 0; j < d; ++j) v *= L.st.S[pi[j] * Q + ii[j]];
      phi[(size_t)p * nl + i] = v;
      for (int g = 0; g < d; ++g) {
        double dv = 1.0;
        for (int j = 0; j < d; ++j) dv *= (j == g ? L.st.D : L.st.S)[pi[j] * Q + ii[j]];
        dphi[((size_t)p * nl + i) * d + g] = dv;
      }
    }
  }
  L.Me.assign((size_t)L.ncells * nl * nl, 0.0);
  L.Ae.assign((size_t)L.ncells * nl * nl, 0.0);
  L.Be.assign((size_t)L.ncells * C * d * nl, 0.0);
  L.mom.assign((size_t)L.ncells * C, 0.0);
  double vol = 0.0;
#pragma omp parallel reduction(+ : vol)
  {
    std::vector<double> jxw(nl), G((size_t)nl * 9), Jinv((size_t)nl * 9), gphys((size_t)nl * nl * 3),
        gv((size_t)nl * nl * 3);
#pragma omp for schedule(static)
    for (int64_t c = 0; c < L.ncells; ++c) {
      double J[9], x[3];
      for (int p = 0; p < nl; ++p) {
        cell_jacobian(L, c, &xq[p * d], x, J);
        double det = inv_det(d, J, &Jinv[p * 9]);
        if (!(det > 0.0)) throw Error(-1, "inverted cell in the deformed mesh");
        jxw[p] = det * wq[p];
        vol += jxw[p];
        double nu = L.nu_q.empty() ? L.nu_const : L.nu_q[(size_t)c * nl + p];
        // physical gradients grad_i = J^{-T} dphi_i ; G = nu * JxW
        for (int i = 0; i < nl; ++i)
          for (int a = 0; a < d; ++a) {
            double s = 0.0;
            for (int b = 0; b < d; ++b) s += Jinv[p * 9 + b * d + a] * dphi[((size_t)p * nl + i) * d + b];
            gphys[((size_t)p * nl + i) * 3 + a] = s;
            gv[((size_t)p * nl + i) * 3 + a] = s * nu * jxw[p];
          }
      }
      double* me = &L.Me[(size_t)c * nl * nl];
      double* ae = &L.Ae[(size_t)c * nl * nl];
      for (int i = 0; i < nl; ++i)
        for (int j = 0; j < nl; ++j) {
          double sm = 0.0, sa = 0.0;
          for (int p = 0; p < nl; ++p) {
            sm += phi[(size_t)p * nl + i] * phi[(size_t)p * nl + j] * jxw[p];
            const double* gi = &gphys[((size_t)p * nl + i) * 3];
            const double* gj = &gv[((size_t)p * nl + j) * 3];
            for (int a = 0; a < d; ++a) sa += gi[a] * gj[a];
          }
          me[i * nl + j] = sm;
          ae[i * nl + j] = sa;
        }
      double* be = &L.Be[(size_t)c * C * d * nl];
      for (int l = 0; l < C; ++l)
        for (int a = 0; a < d; ++a)
          for (int i = 0; i < nl; ++i) {
            double s = 0.0;
            for (int p = 0; p < nl; ++p)
              s += L.st.psi[(size_t)p * C + l] * gphys[((size_t)p * nl + i) * 3 + a] * jxw[p];
            be[((size_t)l * d + a) * nl + i] = s;
          }
      for (int l = 0; l < C; ++l) {
        double s = 0.0;
        for (int p = 0; p < nl; ++p) s += L.st.psi[(size_t)p * C + l] * jxw[p];
        L.mom[(size_t)c * C + l] = s;
      }
    }
  }
  L.volume = vol;
}

// ------------------------------------------------------------- dense LU
// Column-major LU with partial pivoting; returns false on a zero pivot.
static bool lu_factor(int n, double* A, int* piv) {
  for (int j = 0; j < n; ++j) {
    int p = j;
    double best = std::fabs(A[(size_t)j * n + j]);
    for (int i = j + 1; i < n; ++i)
      if (std::fabs(A[(size_t)j * n + i]) > best) { best = std::fabs(A[(size_t)j * n + i]); p = i; }
    piv[j] = p;
    if (best == 0.0) return false;
    if (p != j)
      for (int c = 0; c < n; ++c) std::swap(A[(size_t)c * n + j], A[(size_t)c * n + p]);
    double inv = 1.0 / A[(size_t)j * n + j];
    for (int i = j + 1; i < n; ++i) A[(size_t)j * n + i] *= inv;
    for (int c = j + 1; c < n; ++c) {
      double f = A[(size_t)c * n + j];
      if (f == 0.0) continue;
      double* col = &A[(size_t)c * n];
      const double* lj = &A[(size_t)j * n];
      for (int i = j + 1; i < n; ++i) col[i] -= lj[i] * f;
    }
  }
  return true;
}

// Solve in place for nrhs column-major right-hand sides.
static void lu_solve(int n, const double* A, const int* piv, double* B, int nrhs) {
  for (int r = 0; r < nrhs; ++r) {
    double* b = &B[(size_t)r * n];
    for (int j = 0; j < n; ++j)
      if (piv[j] != j) std::swap(b[j], b[piv[j]]);
    for (int j = 0; j < n; ++j) {
      double v = b[j];
      if (v != 0.0)
        for (int i = j + 1; i < n; ++i) b[i] -= A[(size_t)j * n + i] * v;
    }
    for (int j = n - 1; j >= 0; --j) {
      b[j] /= A[(size_t)j * n + j];
      double v = b[j];
      if (v != 0.0)
        for (int i = 0; i < j; ++i) b[i] -= A[(size_t)j * n + i] * v;
    }
  }
}

static bool invert(int n, const double* A, double* Ainv) {
  std::vector<double> LU(A, A + (size_t)n * n);
  std::vector<int> piv(n);
  if (!lu_factor(n, LU.data(), piv.data())) return false;
  std::fill(Ainv, Ainv + (size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) Ainv[(size_t)i * n + i] = 1.0;
  lu_solve(n, LU.data(), piv.data(), Ainv, n);
  return true;
}

// ---------------------------------------------------------- Vanka factors
static inline bool node_dirichlet(const LevelHost& L, int64_t c, int i) {
  int64_t cc[3] = {c % L.n, (c / L.n) % L.n, L.d == 3 ? c / ((int64_t)L.n * L.n) : 0};
  int ii[3] = {i % L.Q, (i / L.Q) % L.Q, i / (L.Q * L.Q)};
  for (int j = 0; j < L.d; ++j) {
    int64_t g = cc[j] * L.q + ii[j];
    if (g == 0 || g == L.nn - 1) return true;
  }
  return false;
}

// Scalar mass and Laplacian restricted to the nodes of cell c, assembled from
// every cell that shares a pair of those nodes (the global matrix restricted
// to the patch).
static void patch_matrices(const LevelHost& L, int64_t c, double* Mt, double* At) {
  const int d = L.d, Q = L.Q, nl = L.nloc;
  int64_t cc[3] = {c % L.n, (c / L.n) % L.n, d == 3 ? c / ((int64_t)L.n * L.n) : 0};
  std::fill(Mt, Mt + (size_t)nl * nl, 0.0);
  std::fill(At, At + (size_t)nl * nl, 0.0);
  int no = d == 2 ? 9 : 27;
  std::vector<int> loc(nl);
  for (int o = 0; o < no; ++o) {
    int off[3] = {o % 3 - 1, (o / 3) % 3 - 1, d == 3 ? o / 9 - 1 : 0};
    int64_t nb = 0, stride = 1;
    bool ok = true;
    for (int j = 0; j < d; ++j) {
      int64_t cj = cc[j] + off[j];
      if (cj < 0 || cj >= L.n) ok = false;
      nb += cj * stride;
      stride *= L.n;
    }
    if (!ok) continue;
    // local index in the neighbour of each node of c (or -1)
    for (int i = 0; i < nl; ++i) {
      int ii[3] = {i % Q, (i / Q) % Q, i / (Q * Q)};
      int li = 0, st = 1;
      for (int j = 0; j < d; ++j) {
        int v = ii[j] - off[j] * (Q - 1);
        if (v < 0 || v >= Q) { li = -1; break; }
        li += v * st;
        st *= Q;
      }
      loc[i] = li;
    }
    const double* me = &L.Me[(size_t)nb * nl * nl];
    const double* ae = &L.Ae[(size_t)nb * nl * nl];
    for (int i = 0; i < nl; ++i) {
      if (loc[i] < 0) continue;
      for (int j = 0; j < nl; ++j) {
        if (loc[j] < 0) continue;
        Mt[i * nl + j] += me[(size_t)loc[i] * nl + loc[j]];
        At[i * nl + j] += ae[(size_t)loc[i] * nl + loc[j]];
      }
    }
  }
}

void vanka_factors(const LevelHost& L, VankaFactors& V, int nthreads) {
  const int d = L.d, nl = L.nloc, nt = L.nt, C = L.C;
  const int m = nt * nl, P = nt * C;
  V.m = m;
  V.P = P;
  V.coef.resize(nt);
  for (int a = 0; a < nt; ++a) V.coef[a] = 0.5 * L.tau * L.td.w[a];
  V.As_inv.assign((size_t)L.ncells * m * m, 0.0);
  V.Bm.assign((size_t)L.ncells * C * d * nl, 0.0);
  V.F.assign((size_t)L.ncells * d * m * P, 0.0);
  V.Hinv.assign((size_t)L.ncells * P * P, 0.0);
  int fail = 0;
#pragma omp parallel num_threads(nthreads) reduction(+ : fail)
  {
    std::vector<double> Mt((size_t)nl * nl), At((size_t)nl * nl), As((size_t)m * m), H((size_t)P * P);
    std::vector<char> fr(nl);
#pragma omp for schedule(dynamic, 16)
    for (int64_t c = 0; c < L.ncells; ++c) {
      patch_matrices(L, c, Mt.data(), At.data());
      for (int i = 0; i < nl; ++i) fr[i] = !node_dirichlet(L, c, i);
      // A_s[(a,i),(b,j)] = K_ab M_T + delta_ab c_a A_T on free pairs, identity else
      for (int b = 0; b < nt; ++b)
        for (int j = 0; j < nl; ++j)
          for (int a = 0; a < nt; ++a)
            for (int i = 0; i < nl; ++i) {
              double v;
              if (fr[i] && fr[j])
                v = L.td.K[a * nt + b] * Mt[i * nl + j] + (a == b ? V.coef[a] * At[i * nl + j] : 0.0);
              else
                v = (a == b && i == j) ? 1.0 : 0.0;
              As[(size_t)(b * nl + j) * m + (a * nl + i)] = v;
            }
      double* Ai = &V.As_inv[(size_t)c * m * m];
      if (!invert(m, As.data(), Ai)) { ++fail; continue; }
      double* Bm = &V.Bm[(size_t)c * C * d * nl];
      const double* Be = &L.Be[(size_t)c * C * d * nl];
      for (int l = 0; l < C; ++l)
        for (int a = 0; a < d; ++a)
          for (int i = 0; i < nl; ++i)
            Bm[((size_t)l * d + a) * nl + i] = fr[i] ? Be[((size_t)l * d + a) * nl + i] : 0.0;
      // F_c[:, (a,l)] = -c_a A_s^{-1}[:, (a, .)] B[l][c][.]
      double* F = &V.F[(size_t)c * d * m * P];
      for (int comp = 0; comp < d; ++comp)
        for (int a = 0; a < nt; ++a)
          for (int l = 0; l < C; ++l) {
            double* col = &F[((size_t)comp * P + (a * C + l)) * m];
            const double* bl = &Bm[((size_t)l * d + comp) * nl];
            for (int row = 0; row < m; ++row) {
              double s = 0.0;
              for (int i = 0; i < nl; ++i) s += Ai[(size_t)(a * nl + i) * m + row] * bl[i];
              col[row] = -V.coef[a] * s;
            }
          }
      // H[(a,l),(b,l')] = sum_c sum_i (-c_a) B[l][c][i] F_c[(a,i),(b,l')]
      for (int q = 0; q < P; ++q)
        for (int a = 0; a < nt; ++a)
          for (int l = 0; l < C; ++l) {
            double s = 0.0;
            for (int comp = 0; comp < d; ++comp) {
              const double* col = &F[((size_t)comp * P + q) * m];
              const double* bl = &Bm[((size_t)l * d + comp) * nl];
              for (int i = 0; i < nl; ++i) s += bl[i] * col[a * nl + i];
            }
            H[(size_t)q * P + (a * C + l)] = -V.coef[a] * s;
          }
      if (!invert(P, H.data(), &V.Hinv[(size_t)c * P * P])) ++fail;
    }
  }
  if (fail) throw Error(-5, "a cell-patch matrix is singular");
}

void vanka_dense(const LevelHost& L, const VankaFactors& V, std::vector<double>& dense, int nthreads) {
  const int d = L.d, nl = L.nloc, nt = L.nt, C = L.C, m = V.m, P = V.P;
  const int b = d * m + P;
  dense.assign((size_t)L.ncells * b * b, 0.0);
#pragma omp parallel num_threads(nthreads)
  {
    std::vector<double> E((size_t)d * P * m), FH((size_t)d * m * P);
#pragma omp for schedule(dynamic, 16)
    for (int64_t c = 0; c < L.ncells; ++c) {
      const double* Ai = &V.As_inv[(size_t)c * m * m];
      const double* Bm = &V.Bm[(size_t)c * C * d * nl];
      const double* F = &V.F[(size_t)c * d * m * P];
      const double* Hi = &V.Hinv[(size_t)c * P * P];
      double* A = &dense[(size_t)c * b * b];
      // E_c[q][(b,j)] = -c_{a_q} sum_i B[l_q][c][i] A_s^{-1}[(a_q,i),(b,j)]
      for (int comp = 0; comp < d; ++comp)
        for (int a = 0; a < nt; ++a)
          for (int l = 0; l < C; ++l)
            for (int col = 0; col < m; ++col) {
              double s = 0.0;
              const double* bl = &Bm[((size_t)l * d + comp) * nl];
              for (int i = 0; i < nl; ++i) s += bl[i] * Ai[(size_t)col * m + a * nl + i];
              E[((size_t)comp * P + a * C + l) * m + col] = -V.coef[a] * s;
            }
      // FH_c = F_c H^{-1}   (m x P, col-major)
      for (int comp = 0; comp < d; ++comp)
        for (int q = 0; q < P; ++q)
          for (int row = 0; row < m; ++row) {
            double s = 0.0;
            for (int p = 0; p < P; ++p) s += F[((size_t)comp * P + p) * m + row] * Hi[(size_t)q * P + p];
            FH[((size_t)comp * P + q) * m + row] = s;
          }
      // velocity-velocity: delta_cc' A_s^{-1} - FH_c E_c'
      for (int c2 = 0; c2 < d; ++c2)
        for (int col = 0; col < m; ++col)
          for (int c1 = 0; c1 < d; ++c1)
            for (int row = 0; row < m; ++row) {
              double s = c1 == c2 ? Ai[(size_t)col * m + row] : 0.0;
              for (int q = 0; q < P; ++q)
                s -= FH[((size_t)c1 * P + q) * m + row] * E[((size_t)c2 * P + q) * m + col];
              A[(size_t)(c2 * m + col) * b + (c1 * m + row)] = s;
            }
      // velocity-pressure: FH_c ; pressure-velocity: H^{-1} E_c' ; pressure-pressure: -H^{-1}
      for (int q = 0; q < P; ++q)
        for (int c1 = 0; c1 < d; ++c1)
          for (int row = 0; row < m; ++row)
            A[(size_t)(d * m + q) * b + (c1 * m + row)] = FH[((size_t)c1 * P + q) * m + row];
      for (int c2 = 0; c2 < d; ++c2)
        for (int col = 0; col < m; ++col)
          for (int p = 0; p < P; ++p) {
            double s = 0.0;
            for (int q = 0; q < P; ++q) s += Hi[(size_t)q * P + p] * E[((size_t)c2 * P + q) * m + col];
            A[(size_t)(c2 * m + col) * b + (d * m + p)] = s;
          }
      for (int q = 0; q < P; ++q)
        for (int p = 0; p < P; ++p) A[(size_t)(d * m + q) * b + (d * m + p)] = -Hi[(size_t)q * P + p];
    }
  }
}

// ------------------------------------------------ temporally decoupled Vanka
using cplx = std::complex<double>;

// In-place inverse of a row-major complex n x n matrix (Gauss-Jordan with
// partial pivoting); false if a pivot vanishes.
static bool cinvert(int n, cplx* A) {
  std::vector<int> perm(n);
  for (int i = 0; i < n; ++i) perm[i] = i;
  for (int j = 0; j < n; ++j) {
    int p = j;
    double best = std::abs(A[(size_t)j * n + j]);
    for (int i = j + 1; i < n; ++i) {
      double v = std::abs(A[(size_t)i * n + j]);
      if (v > best) { best = v; p = i; }
    }
    if (!(best > 0.0)) return false;
    if (p != j) {
      for (int c = 0; c < n; ++c) std::swap(A[(size_t)j * n + c], A[(size_t)p * n + c]);
      std::swap(perm[j], perm[p]);
    }
    const cplx inv = 1.0 / A[(size_t)j * n + j];
    A[(size_t)j * n + j] = 1.0;
    for (int c = 0; c < n; ++c) A[(size_t)j * n + c] *= inv;
    for (int i = 0; i < n; ++i) {
      if (i == j) continue;
      const cplx f = A[(size_t)i * n + j];
      if (f == 0.0) continue;
      A[(size_t)i * n + j] = 0.0;
      for (int c = 0; c < n; ++c) A[(size_t)i * n + c] -= f * A[(size_t)j * n + c];
    }
  }
  // the row swaps of the elimination become column swaps of the inverse
  std::vector<cplx> tmp((size_t)n * n);
  for (int i = 0; i < n; ++i)
    for (int c = 0; c < n; ++c) tmp[(size_t)i * n + perm[c]] = A[(size_t)i * n + c];
  std::copy(tmp.begin(), tmp.end(), A);
  return true;
}

TemporalEigen temporal_eigen(const TimeData& td, double tau) {
  const int nt = td.k + 1;
  TemporalEigen E;
  E.nt = nt;
  // Kt = diag(c)^{-1} K, c_a = (tau/2) w_a
  std::vector<double> c(nt), Kt((size_t)nt * nt);
  for (int a = 0; a < nt; ++a) c[a] = 0.5 * tau * td.w[a];
  for (int a = 0; a < nt; ++a)
    for (int b = 0; b < nt; ++b) Kt[(size_t)a * nt + b] = td.K[(size_t)a * nt + b] / c[a];
  // characteristic polynomial det(z I - Kt) = sum_k p[k] z^k (Faddeev-LeVerrier)
  std::vector<double> p(nt + 1, 0.0), Mk((size_t)nt * nt, 0.0), AM((size_t)nt * nt);
  p[nt] = 1.0;
  for (int k = 1; k <= nt; ++k) {
    for (int i = 0; i < nt; ++i)  // Mk = Kt M_{k-1} + p[nt-k+1] I
      for (int j = 0; j < nt; ++j) {
        double s = 0.0;
        for (int l = 0; l < nt; ++l) s += Kt[(size_t)i * nt + l] * Mk[(size_t)l * nt + j];
        AM[(size_t)i * nt + j] = s + (i == j ? p[nt - k + 1] : 0.0);
      }
    Mk = AM;
    double tr = 0.0;
    for (int i = 0; i < nt; ++i)
      for (int l = 0; l < nt; ++l) tr += Kt[(size_t)i * nt + l] * Mk[(size_t)l * nt + i];
    p[nt - k] = -tr / k;
  }
  auto poly = [&](cplx z) {
    cplx v = p[nt];
    for (int k = nt - 1; k >= 0; --k) v = v * z + p[k];
    return v;
  };
  // roots: Durand-Kerner iteration, then Newton polishing
  std::vector<cplx> z(nt);
  double scale = 0.0;
  for (int k = 0; k < nt; ++k) scale = std::max(scale, std::pow(std::abs(p[k]), 1.0 / (nt - k)));
  for (int i = 0; i < nt; ++i) z[i] = scale * std::pow(cplx(0.4, 0.9), i);
  for (int it = 0; it < 500; ++it)
    for (int i = 0; i < nt; ++i) {
      cplx den = 1.0;
      for (int j = 0; j < nt; ++j)
        if (j != i) den *= z[i] - z[j];
      z[i] -= poly(z[i]) / den;
    }
  for (int i = 0; i < nt; ++i)
    for (int it = 0; it < 3; ++it) {
      cplx d = 0.0;  // poly'(z)
      for (int k = nt; k >= 1; --k) d = d * z[i] + double(k) * p[k];
      if (std::abs(d) > 0.0) z[i] -= poly(z[i]) / d;
    }
  // real eigenvalues first, then one representative (Im > 0) per pair
  std::vector<cplx> reals, reps;
  for (cplx v : z) {
    if (std::abs(v.imag()) <= 1e-10 * std::abs(v)) reals.push_back(cplx(v.real(), 0.0));
    else if (v.imag() > 0) reps.push_back(v);
  }
  if ((int)(reals.size() + 2 * reps.size()) != nt) throw Error(-5, "temporal eigenvalues are not separated");
  E.nreal = (int)reals.size();
  E.J = E.nreal + (int)reps.size();
  E.lam = reals;
  E.lam.insert(E.lam.end(), reps.begin(), reps.end());
  // eigenvectors by inverse iteration; W's columns: reals, then rep, conj(rep) per pair
  auto eigvec = [&](cplx lam) {
    const cplx sh = lam + cplx(1e-9 * (1.0 + std::abs(lam)), 0.0);
    std::vector<cplx> A((size_t)nt * nt);
    for (int i = 0; i < nt; ++i)
      for (int j = 0; j < nt; ++j) A[(size_t)i * nt + j] = Kt[(size_t)i * nt + j] - (i == j ? sh : 0.0);
    if (!cinvert(nt, A.data())) throw Error(-5, "temporal eigenvector iteration failed");
    std::vector<cplx> v(nt, 1.0), w(nt);
    for (int it = 0; it < 4; ++it) {
      double nrm = 0.0;
      for (int i = 0; i < nt; ++i) {
        cplx s = 0.0;
        for (int j = 0; j < nt; ++j) s += A[(size_t)i * nt + j] * v[j];
        w[i] = s;
        nrm = std::max(nrm, std::abs(s));
      }
      int im = 0;
      for (int i = 0; i < nt; ++i)
        if (std::abs(w[i]) > std::abs(w[im])) im = i;
      const cplx ph = w[im];
      for (int i = 0; i < nt; ++i) v[i] = w[i] / ph;  // largest component 1
      (void)nrm;
    }
    return v;
  };
  std::vector<cplx> W((size_t)nt * nt);  // row-major W[a][col]
  std::vector<int> col_of_block(E.J);
  int col = 0;
  for (int j = 0; j < E.J; ++j) {
    std::vector<cplx> v = eigvec(E.lam[j]);
    col_of_block[j] = col;
    if (j < E.nreal) {
      for (int a = 0; a < nt; ++a) W[(size_t)a * nt + col] = cplx(v[a].real(), 0.0);
      ++col;
    } else {
      for (int a = 0; a < nt; ++a) {
        W[(size_t)a * nt + col] = v[a];
        W[(size_t)a * nt + col + 1] = std::conj(v[a]);
      }
      col += 2;
    }
  }
  std::vector<cplx> Wi = W;
  if (!cinvert(nt, Wi.data())) throw Error(-5, "temporal eigenvectors are not independent");
  E.T.assign((size_t)E.J * nt, 0.0);
  E.Wt.assign((size_t)nt * E.J, 0.0);
  for (int j = 0; j < E.J; ++j) {
    const int cj = col_of_block[j];
    const bool real = j < E.nreal;
    for (int a = 0; a < nt; ++a) {
      cplx t = Wi[(size_t)cj * nt + a] / c[a];
      cplx w = W[(size_t)a * nt + cj] * (real ? 1.0 : 2.0);
      if (real) { t = cplx(t.real(), 0.0); w = cplx(w.real(), 0.0); }
      E.T[(size_t)j * nt + a] = t;
      E.Wt[(size_t)a * E.J + j] = w;
    }
  }
  return E;
}

void vanka_decoupled(const LevelHost& L, VankaDecoupled& V, int nthreads, bool diagonal) {
  const int d = L.d, nl = L.nloc, C = L.C;
  V.te = temporal_eigen(L.td, L.tau);
  V.diagonal = diagonal;
  const int J = V.te.J;
  if (diagonal) V.Dinv.assign((size_t)L.ncells * J * nl, 0.0);
  else V.Ainv.assign((size_t)L.ncells * J * nl * nl, 0.0);
  V.F.assign((size_t)L.ncells * J * d * nl * C, 0.0);
  V.Hinv.assign((size_t)L.ncells * J * C * C, 0.0);
  V.Bm.assign((size_t)L.ncells * C * d * nl, 0.0);
  int fail = 0;
#pragma omp parallel num_threads(nthreads) reduction(+ : fail)
  {
    std::vector<double> Mt((size_t)nl * nl), At((size_t)nl * nl);
    std::vector<cplx> H((size_t)C * C);
    std::vector<char> fr(nl);
#pragma omp for schedule(dynamic, 16)
    for (int64_t c = 0; c < L.ncells; ++c) {
      patch_matrices(L, c, Mt.data(), At.data());
      for (int i = 0; i < nl; ++i) fr[i] = !node_dirichlet(L, c, i);
      double* Bm = &V.Bm[(size_t)c * C * d * nl];
      const double* Be = &L.Be[(size_t)c * C * d * nl];
      for (int l = 0; l < C; ++l)
        for (int a = 0; a < d; ++a)
          for (int i = 0; i < nl; ++i)
            Bm[((size_t)l * d + a) * nl + i] = fr[i] ? Be[((size_t)l * d + a) * nl + i] : 0.0;
      for (int j = 0; j < J; ++j) {
        const cplx lam = V.te.lam[j];
        cplx* F = &V.F[((size_t)c * J + j) * d * nl * C];
        if (diagonal) {
          // lambda_j diag(M) + diag(A) on free nodes, 1 on Dirichlet nodes
          cplx* Dv = &V.Dinv[((size_t)c * J + j) * nl];
          for (int i = 0; i < nl; ++i) {
            const cplx dd = fr[i] ? lam * Mt[(size_t)i * nl + i] + At[(size_t)i * nl + i] : cplx(1.0, 0.0);
            if (!(std::abs(dd) > 0.0)) { ++fail; break; }
            Dv[i] = 1.0 / dd;
          }
          for (int comp = 0; comp < d; ++comp)
            for (int i = 0; i < nl; ++i)
              for (int l = 0; l < C; ++l)
                F[((size_t)comp * nl + i) * C + l] = -Dv[i] * Bm[((size_t)l * d + comp) * nl + i];
        } else {
          cplx* Ai = &V.Ainv[((size_t)c * J + j) * nl * nl];
          for (int i = 0; i < nl; ++i)
            for (int k = 0; k < nl; ++k)
              Ai[(size_t)i * nl + k] = (fr[i] && fr[k]) ? lam * Mt[(size_t)i * nl + k] + At[(size_t)i * nl + k]
                                                        : cplx(i == k ? 1.0 : 0.0, 0.0);
          if (!cinvert(nl, Ai)) { ++fail; continue; }
          for (int comp = 0; comp < d; ++comp)
            for (int i = 0; i < nl; ++i)
              for (int l = 0; l < C; ++l) {
                const double* bl = &Bm[((size_t)l * d + comp) * nl];
                cplx s = 0.0;
                for (int k = 0; k < nl; ++k) s += Ai[(size_t)i * nl + k] * bl[k];
                F[((size_t)comp * nl + i) * C + l] = -s;
              }
        }
        for (int l = 0; l < C; ++l)
          for (int l2 = 0; l2 < C; ++l2) {
            cplx s = 0.0;
            for (int comp = 0; comp < d; ++comp) {
              const double* bl = &Bm[((size_t)l * d + comp) * nl];
              for (int i = 0; i < nl; ++i) s += bl[i] * F[((size_t)comp * nl + i) * C + l2];
            }
            H[(size_t)l * C + l2] = -s;
          }
        if (!cinvert(C, H.data())) { ++fail; continue; }
        std::copy(H.begin(), H.end(), &V.Hinv[((size_t)c * J + j) * C * C]);
      }
    }
  }
  if (fail) throw Error(-5, "a decoupled cell-patch matrix is singular");
}

// ------------------------------------------------------------ coarse level
void coarse_inverse(const LevelHost& L, std::vector<double>& Dinv, std::vector<double>& G) {
  const int d = L.d, nl = L.nloc, C = L.C, nt = L.nt;
  const int64_t nd = L.slab;  // one subinterval
  if (nd > 12000) throw Error(-1, "coarsest level too large for the dense bordered solve");
  const int64_t nn = L.nodes;
  // global scalar mass / Laplacian and divergence
  std::vector<double> M(nn * nn, 0.0), A(nn * nn, 0.0), B((size_t)L.Mp * L.Mv, 0.0);
  std::vector<int64_t> gn(nl);
  std::vector<char> bnd(nn, 0);
  for (int64_t g = 0; g < nn; ++g) {
    int64_t gi[3] = {g % L.nn, (g / L.nn) % L.nn, d == 3 ? g / ((int64_t)L.nn * L.nn) : 1};
    for (int j = 0; j < d; ++j)
      if (gi[j] == 0 || gi[j] == L.nn - 1) bnd[g] = 1;
  }
  for (int64_t c = 0; c < L.ncells; ++c) {
    int64_t cc[3] = {c % L.n, (c / L.n) % L.n, d == 3 ? c / ((int64_t)L.n * L.n) : 0};
    for (int i = 0; i < nl; ++i) {
      int ii[3] = {i % L.Q, (i / L.Q) % L.Q, i / (L.Q * L.Q)};
      int64_t g = 0, st = 1;
      for (int j = 0; j < d; ++j) { g += (cc[j] * L.q + ii[j]) * st; st *= L.nn; }
      gn[i] = g;
    }
    for (int i = 0; i < nl; ++i)
      for (int j = 0; j < nl; ++j) {
        M[gn[i] * nn + gn[j]] += L.Me[((size_t)c * nl + i) * nl + j];
        A[gn[i] * nn + gn[j]] += L.Ae[((size_t)c * nl + i) * nl + j];
      }
    for (int l = 0; l < C; ++l)
      for (int a = 0; a < d; ++a)
        for (int i = 0; i < nl; ++i)
          B[(size_t)(c * C + l) * L.Mv + a * nn + gn[i]] = L.Be[(((size_t)c * C + l) * d + a) * nl + i];
  }
  // one subinterval block D bordered with nt constraint rows/columns
  const int64_t nb = nd + nt;
  std::vector<double> S((size_t)nb * nb, 0.0);  // column-major
  auto at = [&](int64_t row, int64_t col) -> double& { return S[(size_t)col * nb + row]; };
  auto vidx = [&](int a, int comp, int64_t node) { return a * L.Mv + comp * nn + node; };
  auto pidx = [&](int a, int64_t p) { return nt * L.Mv + a * L.Mp + p; };
  for (int a = 0; a < nt; ++a) {
    double ca = 0.5 * L.tau * L.td.w[a];
    for (int comp = 0; comp < d; ++comp)
      for (int64_t i = 0; i < nn; ++i) {
        int64_t row = vidx(a, comp, i);
        if (bnd[i]) { at(row, row) = 1.0; continue; }
        for (int64_t j = 0; j < nn; ++j) {
          if (bnd[j]) continue;
          double mij = M[i * nn + j], aij = A[i * nn + j];
          if (mij == 0.0 && aij == 0.0) continue;
          for (int b = 0; b < nt; ++b) at(row, vidx(b, comp, j)) += L.td.K[a * nt + b] * mij + (a == b ? ca * aij : 0.0);
        }
        for (int64_t p = 0; p < L.Mp; ++p) {
          double bv = B[(size_t)p * L.Mv + comp * nn + i];
          if (bv != 0.0) {
            at(row, pidx(a, p)) -= ca * bv;
            at(pidx(a, p), row) -= ca * bv;
          }
        }
      }
    // bordering: <P_slice, M^p c_1> = 0
    for (int64_t c = 0; c < L.ncells; ++c)
      for (int l = 0; l < C; ++l) {
        at(pidx(a, c * C + l), nd + a) = L.mom[(size_t)c * C + l];
        at(nd + a, pidx(a, c * C + l)) = L.mom[(size_t)c * C + l];
      }
  }
  std::vector<double> Si((size_t)nb * nb);
  if (!invert((int)nb, S.data(), Si.data())) throw Error(-5, "coarse bordered matrix is singular");
  Dinv.resize((size_t)nd * nd);
  for (int64_t r = 0; r < nd; ++r)
    for (int64_t c = 0; c < nd; ++c) Dinv[(size_t)r * nd + c] = Si[(size_t)c * nb + r];
  // coupling to the previous subinterval (Eq. (DefDtauh), C^n = -C^tau (x) [M_h; 0]):
  // block entry (a, comp, i) <- (k, comp, j) is -phi_a(-1) M_ij on free pairs;
  // G = Dinv * block restricted to the columns (k, comp, j)
  G.assign((size_t)nd * L.Mv, 0.0);
  std::vector<double> col(nd);
  for (int comp = 0; comp < d; ++comp)
    for (int64_t j = 0; j < nn; ++j) {
      if (bnd[j]) continue;
      std::fill(col.begin(), col.end(), 0.0);
      for (int a = 0; a < nt; ++a)
        for (int64_t i = 0; i < nn; ++i)
          if (!bnd[i] && M[i * nn + j] != 0.0) col[vidx(a, comp, i)] = -L.td.phim1[a] * M[i * nn + j];
      for (int64_t r = 0; r < nd; ++r) {
        double s = 0.0;
        for (int64_t q = 0; q < nd; ++q)
          if (col[q] != 0.0) s += Dinv[(size_t)r * nd + q] * col[q];
        G[(size_t)r * L.Mv + comp * nn + j] = s;
      }
    }
}

// ------------------------------------------------------------ transfers
Transfer build_transfer(const LevelHost& F, const LevelHost& Cs) {
  Transfer T;
  T.space_h = F.n != Cs.n;
  T.space_p = F.r != Cs.r;
  T.time_change = F.k != Cs.k || F.N != Cs.N;
  T.nnf = F.nn;
  T.nnc = Cs.nn;
  // 1D velocity embedding: coarse Lagrange basis at the fine Gauss-Lobatto
  // nodes, positions taken in reference (undeformed) coordinates.
  T.P1.assign((size_t)T.nnf * T.nnc, 0.0);
  std::vector<double> val(Cs.Q);
  for (int g = 0; g < T.nnf; ++g) {
    int c = std::min(g / F.q, F.n - 1), i = g - c * F.q;
    double X = (c + F.st.gll[i]) / F.n;
    double Xc = X * Cs.n;
    int cc = std::min((int)std::floor(Xc), Cs.n - 1);
    lagrange_eval(Cs.st.gll, Xc - cc, val.data(), nullptr);
    for (int t = 0; t < Cs.Q; ++t) T.P1[(size_t)g * T.nnc + cc * Cs.q + t] += val[t];
  }
  for (auto& v : T.P1)
    if (std::fabs(v) < 1e-15) v = 0.0;
  T.row_lo.assign(T.nnf, T.nnc); T.row_hi.assign(T.nnf, 0);
  T.col_lo.assign(T.nnc, T.nnf); T.col_hi.assign(T.nnc, 0);
  for (int g = 0; g < T.nnf; ++g)
    for (int h = 0; h < T.nnc; ++h)
      if (T.P1[(size_t)g * T.nnc + h] != 0.0) {
        T.row_lo[g] = std::min(T.row_lo[g], h); T.row_hi[g] = std::max(T.row_hi[g], h + 1);
        T.col_lo[h] = std::min(T.col_lo[h], g); T.col_hi[h] = std::max(T.col_hi[h], g + 1);
      }
  for (int g = 0; g < T.nnf; ++g) if (T.row_hi[g] == 0) T.row_lo[g] = 0;
  for (int h = 0; h < T.nnc; ++h) if (T.col_hi[h] == 0) T.col_lo[h] = 0;
  // pressure: 1D shifted-Legendre embeddings e[o][a][b] = coefficient of P_a(xi)
  // in P_b((o + xi)/2) (h) or delta_ab (p); the d-dimensional map is the
  // product over directions (the basis is a truncated tensor product).
  const int d = F.d, Cf = F.C, Cc = Cs.C;
  int ratio = F.n / Cs.n;
  T.npos = ratio == 2 ? (1 << d) : 1;
  int maxdeg = std::max(F.r, Cs.r);
  std::vector<double> gx, gw;
  gauss01(maxdeg + 2, gx, gw);
  // e1[o][a][b]
  std::vector<double> e1((size_t)2 * (maxdeg + 1) * (maxdeg + 1), 0.0);
  for (int o = 0; o < ratio; ++o)
    for (int a = 0; a <= maxdeg; ++a)
      for (int b = 0; b <= maxdeg; ++b) {
        double s = 0.0;
        for (size_t p = 0; p < gx.size(); ++p) {
          double xc = ratio == 2 ? (o + gx[p]) / 2.0 : gx[p];
          s += gw[p] * legendre01(a, gx[p]) * legendre01(b, xc);
        }
        e1[((size_t)o * (maxdeg + 1) + a) * (maxdeg + 1) + b] = s * (2.0 * a + 1.0);
      }
  T.E.assign((size_t)T.npos * Cf * Cc, 0.0);
  for (int pos = 0; pos < T.npos; ++pos)
    for (int lf = 0; lf < Cf; ++lf)
      for (int lc = 0; lc < Cc; ++lc) {
        double v = 1.0;
        for (int j = 0; j < d; ++j) {
          int o = ratio == 2 ? (pos >> j) & 1 : 0;
          v *= e1[((size_t)o * (maxdeg + 1) + F.st.modes[lf * d + j]) * (maxdeg + 1) + Cs.st.modes[lc * d + j]];
        }
        T.E[((size_t)pos * Cf + lf) * Cc + lc] = std::fabs(v) < 1e-15 ? 0.0 : v;
      }
  // time: coarse Radau-Lagrange basis at the fine Radau points
  T.ntf = F.N * F.nt;
  T.ntc = Cs.N * Cs.nt;
  T.Pt.assign((size_t)T.ntf * T.ntc, 0.0);
  int tr = F.N / Cs.N;
  std::vector<double> tv(Cs.nt);
  for (int nf = 0; nf < F.N; ++nf) {
    int nc = nf / tr, j = nf % tr;
    for (int a = 0; a < F.nt; ++a) {
      double s = tr == 1 ? F.td.t[a] : (F.td.t[a] + 2.0 * j - 1.0) / 2.0;
      lagrange_eval(Cs.td.t, s, tv.data(), nullptr);
      for (int b = 0; b < Cs.nt; ++b) T.Pt[(size_t)(nf * F.nt + a) * T.ntc + nc * Cs.nt + b] = tv[b];
    }
  }
  return T;
}

}  // namespace stmg
