// Host planner: block pattern -> elimination order -> block fill -> tiles and
// panels -> task DAGs (factor and solve) -> ticket order.  CPU only.
#pragma once
#include <array>
#include <cstdint>
#include <string>
#include <vector>

#include "d3m_internal.h"

namespace d3m {

struct TaskDag {
  std::vector<Task> tasks;          // ticket order
  std::vector<int32_t> succ;        // CSR successor lists (ticket indices)
  std::vector<int32_t> npred;       // initial dependency counts (ticket order)
  std::vector<int32_t> gen_of;      // ticket -> generation index
  // generation-order view, kept for the static checker
  std::vector<std::vector<int32_t>> gpreds;  // generation index -> predecessors
  std::vector<double> weight_us;
  double makespan_us = 0;
};

// A resource touched by a task (for the static race check).
struct Access {
  int64_t key;
  bool write;
};

struct PlanImpl {
  // user problem
  int nb = 0;
  std::vector<int32_t> n;                     // sizes, user numbering
  std::vector<std::array<int32_t, 2>> pairs;  // (I, J) with I > J, user order
  std::vector<int64_t> koff;                  // K block offsets
  // elimination
  std::vector<int32_t> order;                 // position -> user id
  std::vector<int32_t> pos;                   // user id -> position
  std::vector<std::vector<int32_t>> S;        // by position: later neighbours (positions, sorted)
  int64_t fill_blocks = 0, L_blocks = 0, nnz_L = 0, nnz_K = 0;
  int etree_height = 0, max_S = 0;
  double flops_diag = 0, flops_trsm = 0, flops_update = 0;
  // storage
  int tile = 128;
  int64_t N = 0;
  std::vector<Panel> panels;                  // by position
  std::vector<PBlock> pblocks;
  std::vector<Tile> tiles;
  int64_t L_elems = 0, Linv_elems = 0;
  // K block placement into panels (for the scatter kernel), one per K block
  // ri, ci: user ids of the interfaces of the destination's rows and columns
  struct KPlace { int64_t src, dst; int32_t rows, cols, ld_dst, trans, ri = 0, ci = 0; };
  std::vector<KPlace> kplace;                 // K blocks -> panel storage
  struct FillPlace { int64_t dst; int32_t rows, cols, ld_dst; };
  // regions of L the scatter zeroes: fill blocks whose tiles are not all
  // first written by an update that stores its product, and the padding
  // row pairs of the others
  std::vector<FillPlace> fills;
  // residual row blocks: for each interface (user id), the K blocks of its block row
  struct RBlk { int64_t koff; int32_t J; int32_t mode; };  // mode 0 diag(sym), 1 K_IJ, 2 K_JI^T
  std::vector<std::vector<RBlk>> rrow;
  // extra operand pairs of merged update tasks (Task.pad1 = first, pad0 = count)
  std::vector<XSrc> xsrc;
  // DAGs
  TaskDag fdag, sdag;
  std::vector<std::vector<Access>> facc, sacc;  // per generation index (small plans only)
  int nworkers = 256;
  int sched = 0;
  // partial elimination (primal reduction): only the first nelim blocks of
  // the order are eliminated; the others (user ids 0..nred-1) keep their
  // Schur complement, the reduced matrix, whose K layout holds those
  // blocks and the first npair_red pairs.  sdag is then the forward part of
  // the solve over the eliminated blocks (it leaves the reduced right-hand
  // side in the rows of the others) and sdag2 the backward part (from the
  // others' given solution).
  int nelim = 0, nred = 0, npair_red = 0;
  int64_t N_elim = 0;                         // internal rows of the eliminated blocks
  std::vector<int64_t> koff_red;              // K offsets of the reduced matrix
  std::vector<KPlace> kgather;                // panel storage -> reduced K (src = panel, dst = K)
  TaskDag sdag2;
  std::vector<std::vector<Access>> sacc2;
  // tuning knobs: solve tile rows, sources per merged update, and the
  // right-hand-side groups of the grouped solve DAG sdagg (rhs_groups > 1)
  int solve_tile = 64, merge = 8, rhs_groups = 1;
  TaskDag sdagg;
  std::vector<std::vector<Access>> saccg;
};

// Builds everything; returns an empty string or an error message.
std::string build_plan(PlanImpl& p, int nb, const int32_t* sizes, int64_t npair, const int32_t* pairs,
                       const int32_t* order, const int32_t* grid, int tile, int nworkers, int sched, int nelim,
                       int solve_tile, int merge, int rhs_groups, int* errcode);

// Union of several instances' DAGs (instance i's tasks get inst = i),
// re-scheduled together on P workers.
TaskDag merge_dags(const std::vector<const TaskDag*>& dags, int P);

// Static serializability check of a DAG against its generation order.
int64_t check_dag(const TaskDag& dag, const std::vector<std::vector<Access>>& acc);

// Grid helpers (the library's own enumeration).
std::vector<std::array<int32_t, 4>> grid_interfaces(const int32_t* grid);
std::vector<int32_t> nd_order(const int32_t* grid);
std::vector<int32_t> min_degree_order(int nb, const std::vector<std::array<int32_t, 2>>& pairs);

}  // namespace d3m
