// Host-side setup of the hp space-time multigrid: reference elements, mesh,
// level list, element and cell-patch matrices, smoother factors, transfer
// tables and the bordered coarse inverse.  Pure C++ (no HIP); the device side
// only consumes the arrays built here.
#pragma once
#include <complex>
#include <cstdint>
#include <functional>
#include <stdexcept>
#include <string>
#include <vector>

namespace stmg {

struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

// ----------------------------------------------------------- 1D reference data
// Gauss-Legendre points/weights on [0,1].
void gauss01(int n, std::vector<double>& x, std::vector<double>& w);
// Gauss-Lobatto points on [0,1] (end points included).
std::vector<double> lobatto01(int n);
// Right-sided Gauss-Radau points/weights on [-1,1] (k+1 points, last = 1).
void radau_right(int k, std::vector<double>& t, std::vector<double>& w);
// Lagrange basis on `nodes` evaluated at `x`: val[i] = l_i(x), der[i] = l_i'(x).
void lagrange_eval(const std::vector<double>& nodes, double x, double* val, double* der);
// Shifted Legendre P_m(2x-1) on [0,1].
double legendre01(int m, double x);
// Pressure multi-indices of total degree <= r (total degree ascending,
// x exponent largest first); returns C*d exponents.
std::vector<int> pressure_modes(int d, int r);
int binom(int n, int k);

// Temporal DG(k) data on the reference interval [-1,1].
struct TimeData {
  int k = 0;
  std::vector<double> t, w;   // Radau points and weights
  std::vector<double> K;      // (k+1)^2 row-major, K[a][b]
  std::vector<double> phim1;  // phi_a(-1)
};
TimeData time_data(int k);

// Spatial reference tables for degree r in dimension d (Q = r+2).
struct SpaceTables {
  int d = 0, r = 0, Q = 0, C = 0, nloc = 0;
  std::vector<double> gll;    // Q Gauss-Lobatto nodes on [0,1]
  std::vector<double> gx, gw; // Q Gauss points / weights on [0,1]
  std::vector<double> S;      // S[p*Q + i] = l_i(gx[p])       (nodes -> Gauss points)
  std::vector<double> D;      // D[p*Q + i] = l_i'(gx[p])
  std::vector<double> Dg;     // Dg[p*Q + j] = L_j'(gx[p]), L Lagrange on the Gauss points
  std::vector<int> modes;     // C*d exponents
  std::vector<double> psi;    // psi[p*C + l] at tensor Gauss point p (x fastest)
};
SpaceTables space_tables(int d, int r);

// ------------------------------------------------------------------- levels
struct LevelSpec {
  int n, r, k, N;
};
// placement 0: Alg. 2 + Alg. 3 (temporal coarsening padded at the fine end);
// placement 1: r and k halved together on the fine mesh first.
std::vector<LevelSpec> build_levels(int n, int r, int k, int N, int n_coarse, int r_min, int k_min,
                                    bool time_h, int placement);

struct LevelHost {
  int d = 0, n = 0, r = 0, k = 0, N = 0;
  double tau = 0;
  int Q = 0, q = 0, nn = 0, C = 0, nloc = 0, nt = 0;
  int64_t ncells = 0, nodes = 0, Mv = 0, Mp = 0, slab = 0, ndofs = 0;
  SpaceTables st;
  TimeData td;
  std::vector<double> verts;   // (n+1)^d x d, x fastest
  std::vector<double> nu_q;    // ncells x nloc viscosity at Gauss points (empty: constant)
  double nu_const = 1.0;
  // element matrices (cell-local, Dirichlet not applied)
  std::vector<double> Me, Ae;  // ncells x nloc x nloc
  std::vector<double> Be;      // ncells x C x d x nloc
  std::vector<double> mom;     // ncells x C : int_K psi_l
  double volume = 0;
};

struct Params {
  int d, n, n_coarse, r, k, N, r_min, k_min, placement;
  bool time_h;
  double amp, tau, nu;
  std::function<void(int, const double*, double*)> nu_fn;  // may be empty
};

// Geometry and element matrices of one level.
void build_level(const Params& P, const LevelSpec& s, LevelHost& L);

// Geometry of the operator kernel at the Gauss points of every cell:
// value 0: JxW; 1 + j d + i: JxW Jinv[j][i]; then nu JxW (Jinv Jinv^T)[j][j']
// for j <= j' row by row (apply_geometry_count(d) values).  Layout
// [cell][value][x + 4 y][z]: x and y padded to 4, z < Q in 3D and a single z
// in 2D; padding entries are zero.
int apply_geometry_count(int d);
void apply_geometry(const LevelHost& L, std::vector<double>& geo);

// Smoother factors of one level (Schur-factored local inverse):
// As_inv: ncells x m x m (col-major), m = (k+1) nloc, local velocity order (a, i)
// Bm    : ncells x C x d x nloc, Dirichlet columns zeroed
// F     : ncells x d x m x P (col-major per component), P = (k+1) C
// Hinv  : ncells x P x P (col-major)
// coef  : (k+1) values c_a = (tau/2) w_a
struct VankaFactors {
  int m = 0, P = 0;
  std::vector<double> As_inv, Bm, F, Hinv, coef;
};
void vanka_factors(const LevelHost& L, VankaFactors& V, int nthreads);
// Dense local inverse (ncells x b x b, col-major) from the factors.
void vanka_dense(const LevelHost& L, const VankaFactors& V, std::vector<double>& dense, int nthreads);

// Temporal decoupling of the cell-patch matrix (its tensor-product structure
// in time, the direction the conclusion of the paper points to): the
// velocity block is A_s = K (x) M_T + diag(c) (x) A_T = (diag(c) (x) I)
// (Kt (x) M_T + I (x) A_T) with Kt = diag(c)^{-1} K.  With Kt = W Lambda W^{-1},
// the substitution u = (W (x) I) u~, p = (W (x) I) p~ turns the patch system
// into one spatial Stokes system per eigenvalue lambda_j:
//   [[lambda_j M_T + A_T, -B^T], [-B, 0]] [u~_j; p~_j] = (W^{-1} diag(c)^{-1} (x) I) [r_v; r_p]_j.
// A real Kt has real eigenvalues and complex-conjugate pairs; a pair's
// systems are conjugate, so one representative (positive imaginary part)
// is solved and u_a = sum_real W_aj u~_j + sum_pairs 2 Re(W_aj u~_j).
struct TemporalEigen {
  int nt = 0, J = 0, nreal = 0;           // J blocks: nreal real eigenvalues first, then the pairs
  std::vector<std::complex<double>> lam;  // J eigenvalues of Kt
  std::vector<std::complex<double>> T;    // J x nt: the blocks' rows of W^{-1} diag(c)^{-1}
  std::vector<std::complex<double>> Wt;   // nt x J: W[a][j], doubled for a pair's representative
};
TemporalEigen temporal_eigen(const TimeData& td, double tau);

// Decoupled smoother factors, per cell and block j (FP64, complex):
// Ainv: (lambda_j M + A)^{-1}, nloc x nloc row-major, M and A the patch
//       matrices on free nodes and the identity on Dirichlet nodes;
// F   : F[comp][i][l] = -(Ainv B_comp^T)[i][l] (Dirichlet columns of B zeroed);
// Hinv: (sum_comp B_comp Ainv B_comp^T)^{-1}, C x C row-major.
// Bm as in VankaFactors.
// diagonal = true: the diagonal Vanka's blocks, lambda_j diag(M) + diag(A),
// stored as Dinv (nloc complex values per block) instead of Ainv.
struct VankaDecoupled {
  TemporalEigen te;
  bool diagonal = false;
  std::vector<std::complex<double>> Ainv, Dinv, F, Hinv;
  std::vector<double> Bm;
};
void vanka_decoupled(const LevelHost& L, VankaDecoupled& V, int nthreads, bool diagonal = false);

// Coarsest level: the slab matrix is block lower-bidiagonal in time with one
// diagonal block D per subinterval, so the exact solve is a forward
// substitution x_n = Dinv b_n - G x_{n-1}.  Dinv: the top-left block of the
// inverse of D bordered with the per-slice mean-zero pressure constraints
// (row-major, slab x slab); G = Dinv * (coupling block), restricted to the
// velocity columns of the previous subinterval's last temporal dof
// (row-major, slab x Mv).
void coarse_inverse(const LevelHost& L, std::vector<double>& Dinv, std::vector<double>& G);

// ------------------------------------------------------------ transfer tables
struct Transfer {
  bool space_h = false, space_p = false, time_change = false;
  int nnf = 0, nnc = 0;
  std::vector<double> P1;         // nnf x nnc, row-major (1D velocity embedding)
  std::vector<int> row_lo, row_hi;  // nonzero column range per fine row  [lo, hi)
  std::vector<int> col_lo, col_hi;  // nonzero row range per coarse column
  int npos = 1;
  std::vector<double> E;          // npos x Cf x Cc, row-major (pressure embedding per child position)
  int ntf = 0, ntc = 0;
  std::vector<double> Pt;         // (Nf (kf+1)) x (Nc (kc+1)), row-major
};
Transfer build_transfer(const LevelHost& F, const LevelHost& Cs);

}  // namespace stmg
