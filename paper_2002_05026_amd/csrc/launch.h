// Host-callable launchers of the device kernels (implemented in *.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "d3m_internal.h"

namespace d3m {

// K block placement into panel storage (src/dst offsets in complex elements).
// part: where the scatter writes the |k| sums of the placement's 32x32 tiles
// (tile t = tr + 32-row-tiles * tc: 32 row sums, then 32 column sums, in the
// destination's coordinates; doubles); diag: a diagonal block, of which only
// the lower triangle counts (its diagonal in the row sums).  Fills and
// gathers leave part unused.
struct KPlaceDev {
  int64_t src, dst;
  int32_t rows, cols, ld_dst, trans;  // trans: dst(r,c) = src[c + r*cols]
  int64_t part;
  int32_t diag, pad;
};

// ||K||_inf from the scatter's tile sums: for every 32-row group of every
// interface, the partial vectors to add, ent[ptr[g]..ptr[g+1]) (offsets into
// part, in a fixed order), row l of the group at part[ent + l].
struct KnormDev {
  const double* part;
  const int32_t* ptr;
  const int64_t* ent;
  int32_t ngroups, pad;
};

// Block-row entry for the residual and the norm of K.
struct RBlkDev {
  int64_t koff;
  int32_t J;     // user id of the column interface
  int32_t mode;  // 0 diagonal (symmetric, lower read), 1 K_IJ, 2 K_JI^T
};

// One output tile of the residual: rows [r0, r0+sz) of user interface I.
struct RTaskDev {
  int32_t I, r0, sz, pad;
};

// One output tile of dK: rows [r0, r0+m) x cols [c0, c0+n) of a K block.
struct DkTaskDev {
  int64_t koff;
  int32_t I, J, r0, c0, m, n;
};

// Per-factor constant tables used by the residual, norm and dK kernels.
// The residual splits the K blocks of each block row into kResSplit chunks
// of similar width (one workgroup each, partial products summed afterwards).
constexpr int kResSplit = 4;

struct UserView {
  const int32_t* n;       // sizes, user numbering
  const int64_t* row0;    // user first row of each interface
  const int64_t* prow0;   // internal first row of each user interface
  const int32_t* rptr;    // block-row CSR over RBlkDev
  const RBlkDev* rblk;
  const int32_t* rsplit;  // per interface: kResSplit + 1 bounds into rblk
  const int32_t* perm;    // internal row -> user row
  int64_t N;
};

// IR control block (device memory).
struct IrCtrl {
  int32_t stop;        // 1: converged or given up; later launches return at once
  int32_t iters;       // refinement steps taken
  int32_t status;      // 0 or D3M_IR_NOCONV / D3M_NONFINITE
  int32_t it;          // index of the next eta slot
  double knorm;        // ||K||_inf
  double tol;
  int32_t max_iter;
  int32_t pad;
  double eta_hist[32];
};

hipError_t launch_dag(const DagArgs& a, int prec, int nworkers, bool solve, hipStream_t s);
hipError_t launch_level(const Task* tasks, int begin, int end, const InstView* iv, int prec, hipStream_t s);
hipError_t launch_reset(int32_t* counters, const int32_t* init, int n, int32_t* head, int32_t* abort_flag,
                        const int32_t* skip, hipStream_t s);

hipError_t launch_prepare(int32_t* status, float* growth, int npanel, IrCtrl* ctrl, double tol, int max_iter,
                          hipStream_t s);
// K into panel storage in the factor's precision, the listed zero blocks
// (fill blocks no update stores into, padding row pairs) zeroed, and the
// |k| sums of every placed tile into part (for launch_knorm)
hipError_t launch_scatter(const void* K, void* L, const KPlaceDev* kp, int nkp, const KPlaceDev* fills,
                          int nfill, double* part, int prec, hipStream_t s);
// ctrl->knorm = max over rows of the sums of the scatter's tile sums
hipError_t launch_knorm(const KnormDev& kn, IrCtrl* ctrl, hipStream_t s);
hipError_t launch_perm_in(const void* B, int64_t ld, void* W, int prec, const UserView& uv, int nrhs,
                          const int32_t* skip, hipStream_t s);
hipError_t launch_perm_out(const void* W, void* X, int64_t ld, const UserView& uv, int nrhs, hipStream_t s);
// complex128 rows [q0, q1) of the internal order only; out = 0: user -> internal, 1: internal -> user
hipError_t launch_perm_rows(const void* src, int64_t lds, void* dst, int64_t ldd, const UserView& uv, int64_t q0,
                            int64_t q1, int nrhs, int out, hipStream_t s);
// reduced matrix out of panel storage (the first ndiag entries are diagonal blocks)
hipError_t launch_gather_red(const void* L, void* K, const KPlaceDev* kg, int nkg, int ndiag, int maxelems,
                             hipStream_t s);
// S = M^T U over N rows (bilinear), nports x nrhs, complex128
hipError_t launch_ports(const void* M, int64_t ldm, const void* U, int64_t ldu, int64_t N, int nports, int nrhs,
                        void* S, hipStream_t s);
// R = B - K X (internal order, RHS fastest) and the column maxima of |R|;
// P: kResSplit * N * nrhs complex128 of scratch for the partial products.
hipError_t launch_residual(const void* K, const void* B, int64_t ld, const void* X64, void* R64, void* P,
                           double* colmax, const UserView& uv, const RTaskDev* rt, int nrt, int nrhs,
                           const int32_t* skip, hipStream_t s);
hipError_t launch_colmax(const void* V, int64_t rows, int nrhs, int64_t ld, int rhs_fastest, double* colmax,
                         const int32_t* skip, hipStream_t s);
hipError_t launch_ir_reset(IrCtrl* ctrl, double tol, int max_iter, hipStream_t s);
hipError_t launch_ir_check(IrCtrl* ctrl, double* rmax, double* xmax, const double* bmax, int nrhs,
                           int final_step, hipStream_t s);
hipError_t launch_cvt_down(const void* R64, void* W32, int64_t n, const int32_t* skip, hipStream_t s);
hipError_t launch_cvt_up(const void* W32, void* X64, int64_t n, hipStream_t s);
hipError_t launch_axpy_up(const void* W32, void* X64, int64_t n, const int32_t* skip, hipStream_t s);
hipError_t launch_zero_f64(double* p, int n, hipStream_t s);
hipError_t launch_dk(const void* Lam, const void* X, int64_t ld, int nrhs, void* dK, const UserView& uv,
                     const DkTaskDev* dt, int ndt, int stored, hipStream_t s);
hipError_t launch_all_stop(IrCtrl* const* ctrls, int n, int32_t* out, hipStream_t s);

// One instance of a batch, as the batched refinement kernels see it: the
// user's K, B and X (set before each run), the instance's workspace arrays
// and refinement controls.
struct BatchIrDev {
  const double2* K;
  const double2* B;
  double2* X;
  int64_t ld;
  void* W;         // the factor-precision solve vector (complex128 for a complex128 batch)
  double2* X64;
  double2* R64;
  double2* P64;
  double* rmax;    // 3 x 128 doubles: rmax, xmax, bmax
  double* xmax;
  double* bmax;
  IrCtrl* ctrl;
  UserView uv;
  const RTaskDev* rt;
  int32_t nrt, nrhs;
  double tol;
  // set-up of the factorization (state reset, scatter, ||K||)
  void* L;                      // factor storage (precision of the batch)
  const KPlaceDev* kp;
  const KPlaceDev* fills;
  int32_t nkp, nfill;
  double* part;                 // the scatter's tile sums
  KnormDev kn;
  int32_t* status;
  float* growth;
  int32_t* flag;                // the instance's factor-status flag (copy of the batch's)
  int32_t npanel, max_iter;
  int32_t sb0, pad;             // the instance's first block in the batch's scatter grid
};
constexpr int kBatchUserMax = 32;  // instances whose user pointers one launch sets
struct BatchUserArgs {
  const void* K[kBatchUserMax];
  const void* B[kBatchUserMax];
  void* X[kBatchUserMax];
  int64_t ld[kBatchUserMax];
  int32_t base, count;
};
hipError_t launch_batch_user(BatchIrDev* tab, int n, const void* const* K, const void* const* B, void* const* X,
                             const int64_t* ld, hipStream_t s);
hipError_t launch_batch_begin(BatchIrDev* tab, int n, int prec, int64_t maxtot, hipStream_t s);
// state reset, scatter/convert of K and ||K||_inf of every instance (user K
// pointers set by launch_batch_user first): three launches
hipError_t launch_batch_setup(BatchIrDev* tab, int n, int prec, int totnb, int maxkng, int maxpanel, hipStream_t s);
// every instance's factor-status flag = *src
hipError_t launch_batch_flags(BatchIrDev* tab, int n, const int32_t* src, hipStream_t s);
hipError_t launch_batch_cvt_up(BatchIrDev* tab, int n, int64_t maxtot, hipStream_t s);
hipError_t launch_batch_check(BatchIrDev* tab, int n, int prec, int maxnrt, int minnrhs, int maxnrhs,
                              int64_t maxtot, int final_step, hipStream_t s);
hipError_t launch_batch_cvt_down(BatchIrDev* tab, int n, int64_t maxtot, hipStream_t s);
hipError_t launch_batch_axpy_up(BatchIrDev* tab, int n, int64_t maxtot, hipStream_t s);
hipError_t launch_batch_perm_out(BatchIrDev* tab, int n, int prec, int64_t maxtot, hipStream_t s);
hipError_t launch_debug_gemm(int prec, int m, int n, int k, int amode, int i0, const void* A, int64_t lda,
                             const void* d, const void* B, int64_t ldb, void* C, int64_t ldc, double alpha,
                             double beta, hipStream_t s);
constexpr int kBenchCands = 4;  // engine paths launch_gemm_bench times (see k_gemm_bench)
hipError_t launch_gemm_bench(int prec, void* buf, int reps, int variant, hipStream_t s);

}  // namespace d3m
