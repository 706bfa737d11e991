// Hierarchy data structures of the H(curl) AMG library.
#pragma once
#include <memory>

#include "prims.hpp"

namespace hc {

// One level of the hierarchy.  Level l owns its edge operator, its discrete
// gradient, its nodal operator and (unless it is the coarsest) the transfer to
// level l+1 with everything the energy minimisation built for it.
// A run of consecutive small colour classes that one workgroup sweeps with
// the x entries it touches held in LDS: U lists those entries (sorted), lcol
// gives each matrix entry of the run its slot in U, lrow each row's own slot.
struct ChainRun {
  int k0 = 0, nk = 0, dir = 1;
  int g_lo = 0, g_hi = 0, e_lo = 0, nU = 0;
  DBuf<int> U, lcol, lrow;
};

struct Level {
  bool fine = false;  // level 0: its setup kernels are booked under "_l0" tags
  int n = 0;  // edges (rows of A)
  int m = 0;  // nodes (columns of D)
  Csr A;
  DBuf<int> tail, head;  // endpoints of every edge: D row = -1 at tail, +1 at head
  Csr D, DT;             // D as CSR (+-1 values) and its transpose
  Csr An;                // nodal operator D^T A D
  Csr DTA;               // (A D)^T = D^T A (A symmetric): the Hiptmair nodal right-hand
                         // side D^T (b - A x) is formed as D^T b - DTA x
  Csr ADshape, APshape;  // row pointers and nnz of the setup's A D and A P^(e) (the
                         // products themselves are dropped): an update with the
                         // same patterns redoes only their numeric passes
  DBuf<double> dinvA, dinvAn;
  DBuf<float> dinvA32, dinvAn32;

  // multicolour Gauss-Seidel orderings
  int ncolA = 0, ncolAn = 0;
  std::vector<int> cptrA, cptrAn;  // host offsets of each colour in rowsA / rowsAn
  DBuf<int> cptrA_d, cptrAn_d;     // the same offsets on the device
  DBuf<int> rowsA, rowsAn;         // rows grouped by colour, increasing within a colour
  DBuf<int> colorA, colorAn;
  // colour-major copies: row g is original row rows[g], columns unchanged,
  // so every colour is one contiguous block of rows
  Csr Acm, Ancm;
  std::vector<ChainRun> chainsA, chainsAn;  // LDS plans of the sweeps' small-colour runs
  DBuf<double> dinvAcm, dinvAncm;
  DBuf<float> dinvAcm32, dinvAncm32;

  // transfer to the next level (empty on the coarsest level)
  bool has_transfer = false;
  DBuf<int> agg;          // aggregate of every node (the next level's node id)
  DBuf<int> pbar;         // map of P-bar when it comes from Alg. 1 on the smoothed P^(n)
  Csr Pn;                 // nodal prolongator m x m_H
  Csr R;                  // D P^(n) on the pattern T (n x m_H)
  Csr Pe, PeT;            // edge prolongator n x n_H and its transpose
  DBuf<uint16_t> lpair;   // per pattern entry: local tail | local head << 8 in T_i
  DBuf<double> p0;        // initial guess, kept for export
  int maxJ = 0, maxNp = 0;
  int n_coarse = 0;
  int nsingle = 0;         // Dirichlet edges of this level (one entry in D)
  int nsingle_coarse = 0;  // single-node coarse edges made for the next level
  int64_t irreducible_added = 0;  // coarse edges make_irreducible added
  double rho = 0.0, omega = 0.0;
  double cancel = 0.0;  // max over nodes of (|D|^T |A| |D| 1)_u / (D^T A D)_uu
  std::vector<double> energy;

  // solve workspace
  DBuf<double> x, b, r, rn, cn, dtb;
  DBuf<float> x32, b32, r32, rn32, cn32, dtb32;
};

struct Coarsest {
  int n = 0;
  DBuf<double> inv;  // dense inverse of the coarsest operator (row-major)
};

struct Hierarchy {
  Ctx ctx;
  hipGraphExec_t vgraph = nullptr;  // whole V-cycle on (pr -> pz)
  hipGraphExec_t cgraph = nullptr;  // V-cycle of levels >= 1 on (lv[1].b -> lv[1].x)
  bool capturing = false;
  bool fp32 = false;      // the FP32 form of the V-cycle is in use
  bool pn_given = false;  // level 0's P^(n) came from the caller
  bool valid = true;      // false after a failed update: the levels are mixed
  double update_ms = 0.0;
  ~Hierarchy() {
    if (vgraph) (void)hipGraphExecDestroy(vgraph);
    if (cgraph) (void)hipGraphExecDestroy(cgraph);
  }
  hcurl_amg_opts opts{};
  std::vector<std::unique_ptr<Level>> lv;
  Coarsest co;
  double setup_ms = 0.0, solve_ms = 0.0;
  int last_iters = 0;
  std::vector<double> pcg_hist;  // recursive relative residuals of the last solve
  std::vector<double> pcg_alpha, pcg_beta;  // CG coefficients of the last solve
  double lanczos_min = 0.0, lanczos_max = 0.0;  // extreme Ritz values from them
  bool stagnated = false;
  double last_relres = 0.0;
  DBuf<double> coords;  // level-0 node coordinates (m x 3) when given
  // PCG workspace (level 0, FP64)
  DBuf<double> px, pr, pz, pp, pq, pzold;
};

// setup.hip
void build_hierarchy(Hierarchy& H, const hcurl_csr& A, const hcurl_csr& Dh, const double* coords, const int32_t* const* aggs,
                     int nagg);

// setup reuse for a new edge matrix with the same pattern (HCURL_REUSE_*)
void update_hierarchy(Hierarchy& H, const hcurl_csr& A, int mode, int iters);

// the local min-norm correction x <- x + G~ L~^-1 (r~ - G~^T x) on every row
// (with `ones`, x is first set to ones)
void emin_make_feasible(Level& L, double* x, bool ones, Ctx& c);
// max |P^(e) D_H - D_h P^(n)| over the level's rows and max |D_h P^(n)| on T
void commute_residual(Level& L, double* abs_max, double* ref_max, Ctx& c);
// (|T_i|, n_p) histogram of the level's rows (HCURL_LS_HIST_J x HCURL_LS_HIST_NP)
void ls_histogram(Level& L, int64_t* out, Ctx& c);
// max |S_l D_l| and max |S_l| for l < nlev, S_0 = S, S_{l+1} = P^(e)T S_l P^(e)
void curl_residual(Hierarchy& H, const hcurl_csr& S, int nlev, double* absmax, double* refmax);

// solve.hip
void color_rows(const Csr& A, DBuf<int>& color, DBuf<int>& rows, std::vector<int>& cptr, int& ncol, Ctx& c);
void colour_major(const Csr& A, const DBuf<int>& rows, Csr& Acm, Ctx& c);
void gather_vec(const double* x, const int* rows, double* y, int n, Ctx& c);
void prepare_solve(Hierarchy& H);
void apply_vcycle(Hierarchy& H, const double* r, double* z);
int pcg_solve(Hierarchy& H, const double* f, double* u, double rtol, int maxit, int* iters, double* relres);

}  // namespace hc
