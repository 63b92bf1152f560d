// Batched launches: one launch of a kernel covers G independent GPs.
//
// A launch carries a Tab (by value): GP g owns the blocks [off[g], off[g+1])
// of the grid.  Each block finds its GP by binary search and reads that GP's
// arguments from a device array of job structs.  Arguments that change from
// one Lanczos / CG step to the next are a base pointer plus a per-step stride
// (the step index is a launch argument shared by all GPs, which run in lock
// step), so the job arrays are uploaded once per build.  A single GP is the
// batch of one.
#pragma once
#include "common.h"

namespace love {

constexpr int MAXG = 64;      // GPs per launch
constexpr int RB = 256;       // rows per block of the row kernels: 64 lanes x 4 rows
constexpr int LDP = MAXK + 8; // row stride of the per-block partial-sum rows

struct Tab {
  int G;
  int off[MAXG + 1];
};

// (gp, local block) of grid block b; false past the last GP's blocks
__device__ inline bool tab_find(const Tab& t, int b, int& gp, int& lb) {
  int lo = 0, hi = t.G;   // last g with off[g] <= b
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (t.off[mid] <= b) lo = mid;
    else hi = mid;
  }
  gp = lo;
  lb = b - t.off[lo];
  return b < t.off[t.G];
}

// g = W^T v with v = v_base + j * v_js, into out + j * out_js
// (mode bit 4: W^T (v + ctl->ratio * v2))
template <typename T>
struct ScatterJob {
  GridT<T> g;
  const T* x;                 // sorted coordinates, n x d
  const int32_t* cell_start;  // ctot + 1
  const T* v;
  int64_t v_js;
  const T* v2;
  T* out;                     // m
  int64_t out_js;
  const Ctl* ctl;
  T* cellp;                   // two-stage W^T v scratch (scatter_scratch_bytes): d >= 3 the
                              // tiles' extended-box node partials, else 4^d x ctot products
};

// out = W kg + sigma2 * vsig (vsig nullable)
template <typename T>
struct GatherJob {
  GridT<T> g;
  const T* x;
  int64_t n;
  const T* kg;
  const T* vsig;
  T sigma2;
  T* out;
  const Ctl* ctl;
};

// One axis of K_UU for one GP: out = scale * T_axis in (along the axis).
template <typename T>
struct ToepJob {
  const T* in;
  T* out;
  int64_t in_js, out_js;      // per-step strides of in / out
  const T* c;                 // first column (direct products)
  const T* spec;              // FFT: [lam (N) | twiddles (N)]
  T* partial;                 // per-segment partial sums of the banded product
  int L, bw, seglen, nseg, ntiles, N, logN;
  int64_t inner, outer;
  T scale;
  const Ctl* ctl;
};

// p[i] = val for i < n
template <typename T>
struct FillJob {
  T* p;
  int64_t n;
  T val;
};

// Lanczos run with full reorthogonalisation on rows 0..n-1 (Q column-major,
// column stride ldq, a multiple of 256).  The operator part (g, x, R, m, sigma2) is
// used by the main run on Khat only.
template <typename T>
struct LzJob {
  GridT<T> g;
  const T* x;
  const int32_t* cell_start;
  T sigma2;
  int64_t m;
  T* R;                       // k x m: row j = K W^T q_j
  int64_t n, ldq;
  T* Q;
  T* v;                       // A q_j
  T* r;                       // once-projected residual
  T* gv;                      // m: W^T q_j
  T* gm;                      // m
  double* partial;            // nb x LDP
  // grid-space first pass (gpath = 1, used when m <= n): G = W^T Q, column j
  // at G + j ldg (rows m..ldg-1 zero), and nbc partial rows of G^T R_j
  int gpath;
  const T* G;
  int64_t ldg;
  double* gpart;              // nbc x LDP
  int nbc;
  // gcs = 1 (grids of more than GPASS_NBC_SUM tiles): a column-sum launch
  // adds the nbc rows into c2 before the second pass, which reads them there
  int gcs;
  double* coef;               // LDP
  double* c2;                 // LDP
  double* amax;               // LDP
  double* alpha;
  double* beta;
  double* ldiag;              // T = L L^T
  double* lsub;
  Ctl* ctl;
  double tol;
  int klast;                  // k - 1
  int nb;                     // row blocks of 64 rpl rows
  int rpl;                    // rows per lane of the row kernels (1 or 4)
  // psum = 1: the second pass sums the first pass's partial rows itself
  // (block 0 stores coef) and writes its own rows to partial2, which the
  // finalize step sums (no column-sum launches; for small nb)
  int psum;
  double* partial2;           // nb x LDP
};

// Rt[u, :] = (L^{-1} R[:, u])^T
template <typename T>
struct RtJob {
  const T* R;                 // k x ld row-major (row i: column i of the factor's input)
  int64_t ld;                 // row stride of R (0: m)
  const double* ldiag;
  const double* lsub;
  void* rt;
  uint16_t* rt_lo;
  int64_t m;
  int kpad, split;
  const Ctl* ctl;
};

// Preconditioned CG on Khat x = y in double (the preconditioner reads the
// Lanczos vectors Q of type TQ).
template <typename TQ>
struct CgJob {
  GridT<double> g;
  const double* x;            // sorted coordinates in double
  const double* y;
  int64_t n, m, ldq;
  double* xs;
  double* r;
  double* z;
  double* p;
  double* ap;
  double* gv;
  double* gm;
  const TQ* Q;
  int kq;                     // preconditioner columns (0: plain CG)
  int kpad;
  const double* ldiag;
  const double* lsub;
  double* pg;                 // Gram partials, nbg x kpad x kpad
  double* tinv;               // kpad x kpad
  double* cm;                 // kpad x kpad
  int nbg;
  int64_t rpbg;
  double* partial;            // nb x LDP
  double* coef;               // LDP
  double* dvec;               // LDP
  double sigma2, rscale, tol2;
  int maxit;
  int nb;                     // row blocks of 64 rpl rows
  int rpl;                    // rows per lane (1 or 4)
  Ctl* ctl;
  double* ortho;              // max |G - I| (nullable)
  void* a;                    // cache mean vector (m, cache precision)
  int a_fp64;
};

// Grid-space mean solve (d >= 2, every axis m_e <= SPEC_MAXM): CG on
// (sigma^2 I + B^T W^T W B) z = B^T W^T y with B = kron(B_e), B_e B_e^T = T_e
// and K = kron(T_e); then a = B z.  B_e = V_e diag(sqrt lam_e) U_e, where
// T_e = V_e diag(lam_e) V_e^T and U_e diagonalises the axis's expected
// weight Gram matrix in those coordinates (eigenvalues D_e).
constexpr int SPEC_MAXM = 128;
constexpr int SPW = 4;        // columns of the spectral solve's partial-sum rows
struct SpecJob {
  GridT<double> g;
  const double* x;            // sorted coordinates in double, n x d
  const int32_t* cell_start;
  const double* y;            // sorted targets in double
  int64_t n, mtot;
  int d;
  int m[MAXD];                // grid points per axis
  int ldv[MAXD];              // row stride of the per-axis matrices (m_e rounded up to even)
  int64_t inner[MAXD];        // product of m over later axes
  const double* c64[MAXD];    // first column of T_e (outputscale folded into axis 0)
  double* B[MAXD];            // B_e, ldv x ldv (row: grid node, column: mode)
  double* D[MAXD];            // D_e
  double* pinv;               // mtot: 1 / (sigma^2 + n prod_e D_e)
  double *z, *r, *p, *q, *t0, *t1;   // mtot
  double* un;                 // n: W u
  double* part;               // partial-sum rows (SPW columns)
  int nbm, nbn;               // row counts of the partials over m and over n
  double sigma2, tol2;
  int maxit;
  Ctl* ctl;                   // the solve's own control block
  Ctl* ctl_out;               // the cache's: gets cg_iters, done and the solve's status bits
  void* a;                    // cache mean vector (m, cache precision)
  int a_fp64;
};

}  // namespace love
