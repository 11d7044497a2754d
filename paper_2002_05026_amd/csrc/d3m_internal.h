// Internal data structures shared by the host planner (C++) and the device
// kernels (HIP).  Plain structs only; no behaviour.
#pragma once
#include <stdint.h>

namespace d3m {

constexpr int kTileMax = 128;   // largest tile edge (rows/cols) of any task
constexpr int kThreads = 512;   // threads per workgroup of every MFMA kernel (8 waves)

// Task kinds of the elimination DAG (Sec. II: per nonzero block a dense
// factorization, dense triangular solves and dense updates), and of the
// block forward/backward solve DAG.
enum TaskKind : int32_t {
  TK_XUPD = 3,    // Schur update of one tile: A_rs -= L_rq D_q L_sq^T (q: a tile or a panel)
  TK_FACT = 4,    // LDL^T of one diagonal tile, its D and the inverse of its unit lower factor
  TK_TRSM = 5,    // one tile of the panel: L_rc = A_rc Linv_c^T D_c^-1
  TK_INV = 6,     // one tile of the inverse of a panel's unit lower diagonal block
  TK_FUPD = 11,   // forward update of one row tile: b_r -= L_rI D_I z_I
  TK_BUPD = 12,   // backward push into one column tile: z_c(I) -= L_Jc^T x_J
  TK_FTILE = 14,  // forward, one tile of a diagonal block: z_c = D_c^-1 (L_II^-1 b_I)_c
  TK_BTILE = 15,  // backward, one tile of a diagonal block: x_c = (L_II^-T t_I)_c
  TK_RED = 16,    // forward: b_r += the extra accumulators of tile r
};

// Extra accumulators of the forward solve: the updates into one row tile of
// b go round-robin to b itself and kSolveSlots more copies of b (stored after
// it, N rows each), which a TK_RED task adds into b before the tile is used.
constexpr int kSolveSlots = 3;

// One source of a merged update task: A = LD + a_off (lda), B = L + b_off
// (lda), inner length k.
struct XSrc {
  int64_t a_off, b_off;
  int32_t k, lda;
};

// Sources of one merged update task at most (factor, forward solve); the
// plan's merge option picks the count up to this bound.
constexpr int kMergeSrc = 16;
constexpr int kMergeSolve = 1;
// Forward solve updates from source panels at least this wide are cut into
// two tasks over column halves of the panel.
constexpr int kSolveKSplitMin = 256;
// Plans of at least this many interfaces stop merging update sources in the
// last sixteenth of the elimination order (the chain of the tree's top panels).
constexpr int kChainMin = 64;

// One task, in ticket order.  Offsets are in complex elements, relative to
// the instance's base pointers (panel storage L, solve vector W).
struct Task {
  int32_t kind;
  int32_t inst;      // instance index (batched launches run many factors)
  int32_t panel;     // block column I (elimination position)
  int32_t m, n, k;   // output rows, output cols, inner length
  int32_t lda, ldc;  // leading dims of the A operand and the output
  int32_t dofs;      // offset of D_I in the D vector (internal row of I)
  int32_t aux;       // kind-specific (row tile / column tile index)
  int64_t a_off, b_off, c_off;
  int32_t succ_begin, nsucc;
  int32_t pad0, pad1;  // XUPD/FUPD: merged sources (count, first); FTILE/BTILE: end/start of the factor tile
};
static_assert(sizeof(Task) == 80, "Task layout");

// Block column (panel) I of the factor storage: the n_I x n_I diagonal
// block on top of the blocks L_JI of every J in S_I, column-major with
// leading dimension H = n_I + sum_J n_J.
struct Panel {
  int64_t off;       // element offset of the panel in L storage
  int64_t ioff;      // element offset of the inverse of its unit lower diagonal block (n x n)
  int32_t H, n;      // rows, cols
  int32_t prow0;     // internal (elimination-order) first row of I
  int32_t tile0;     // first tile index of I in the tile table
  int32_t nt;        // tiles of I
  int32_t pb0, npb;  // row-block list: blocks [pb0, pb0+npb) (the first is I itself)
  int32_t user;      // user interface id
  int32_t pad0, pad1;
};

// A row block of a panel: the rows of interface J inside panel I.
struct PBlock {
  int32_t J;         // panel index (elimination position) of J
  int32_t prow;      // first row of J inside the panel
  int32_t n;         // rows (n_J)
  int32_t prow0;     // internal first row of J
};

// A tile of an interface: rows [r0, r0+sz) of interface I.
struct Tile {
  int32_t panel, r0, sz, pad;
  int64_t linv_off;  // element offset of its diagonal tile inside the panel's inverse block (ld n)
};

// Per-instance device view.  The element type of L, D, Linv and W is the
// factor precision (complex64 or complex128).
struct InstView {
  void* L;           // panel storage
  void* LD;          // same layout: L_rc D_c below each diagonal tile (the scaled update operand)
  void* D;           // N diagonal pivots, internal order
  void* Linv;        // per panel: inverse of the unit lower diagonal block
  void* W;           // solve vectors, internal order, RHS fastest: W[row * nrhs + j] (b, then x)
  void* Z;           // second solve vector, same layout (z = D^-1 L^-1 b, then t)
  const Panel* panels;
  const PBlock* pblocks;
  const Tile* tiles;
  const XSrc* xsrc;  // sources of merged update tasks
  int32_t* status;   // [0] first bad pivot (internal row, INT_MAX if none), [1] count, [2] FP64 re-factors
  float* growth;     // per panel: [2*I] min |d|, [2*I+1] max |L|
  int32_t nrhs;
  int32_t npanel;
  int64_t N;
  float gdmin, glmax;  // fallback trigger (complex64 factor): |d| < gdmin max|A|, |l| > glmax
  int32_t fallback;    // 1: re-factor tripped diagonal tiles in FP64
  int32_t pivot;       // 1: Bunch-Kaufman pivoting inside each diagonal tile
  // with pivoting: Linv holds F = L^-1 P of each panel's diagonal block and
  // Ginv holds D^-1 F (the same layout); Doff[r] = D(r+1, r) when a 2x2
  // pivot starts at internal row r; ipiv[r] = original position inside the
  // tile of the unknown at internal row r
  void* Ginv;
  void* Doff;
  int32_t* ipiv;
};

// Arguments of one persistent DAG launch.
struct DagArgs {
  const Task* tasks;
  const int32_t* succ;
  int32_t* counters;     // pending predecessor counts (reset before each launch)
  int32_t* head;         // ticket counter
  int32_t* abort_flag;   // set by the watchdog; every workgroup then exits
  const int32_t* skip;   // if non-null and *skip != 0, the launch does nothing
  const InstView* inst;
  int32_t ntask;
  int32_t nrhs;          // right-hand sides of a solve launch (0: the instance's own)
  int32_t rhs_groups;    // groups of right-hand-side columns of the launched solve DAG (task kind >> 8)
  int64_t spin_limit_ns; // watchdog bound on one dependency wait
  int64_t* trace;        // optional: per ticket {taken, ready, done, workgroup} (100 MHz clock)
};

}  // namespace d3m
