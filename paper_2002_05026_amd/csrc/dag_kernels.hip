// Device side of the dual factorization and solution (Sec. II of the paper):
// the task bodies -- dense LDL^T of a diagonal block, TRSM + D-scale of a
// row tile, Schur GEMM update of a tile, and the block forward/backward
// solve tasks -- and the persistent kernel that runs a task DAG with
// device-side dependency counters.
//
// The paper schedules its B-DAG statically onto CPU cores and overlaps MPI
// style messages (Sec. II).  On one MI355X the DAG instead runs as one
// persistent launch: each workgroup takes the next ticket of a fixed
// topological order (the planner's list schedule), waits until the ticket's
// dependency counter reaches zero, runs the task, publishes its stores with
// an agent-scope release and decrements its successors' counters.  Because
// a ticket only ever waits on lower tickets, which belong to workgroups that
// are already running, the scheme cannot deadlock whatever the grid size.
#include <hip/hip_runtime.h>
#include <climits>

#include "d3m_internal.h"
#include "gemm_engine.h"
#include "launch.h"
#include "solve_mv.h"
#include "tile_bk.h"
#include "tile_ldlt.h"

namespace d3m {

// ---------------------------------------------------------------- task bodies
template <typename T> struct Ctx {
  typedef typename Cplx<T>::type C;
  C* L;
  C* LD;  // L_rc D_c (written by the TRSM tasks)
  C* D;
  C* Li;
  C* Gi;  // with pivoting: D^-1 L^-1 P of each diagonal block (Li then holds L^-1 P)
  C* W;
  C* Z;
  const InstView* iv;
  lds_char* lds;
  int nrhs;   // right-hand sides of the launch: the row stride of W and Z
  int j0;     // solve tasks: first column of the task's right-hand-side group
  int ncols;  // and its column count
};

// Task bodies are separate functions (each gets its own register
// allocation), and a function's arguments count as per-lane values.  The
// task and its context are the same for the whole workgroup: these copies
// say so (readfirstlane), so that everything derived from them is computed
// once per wave in scalar registers and branches on it are scalar branches.
__device__ __forceinline__ int32_t ufirst(int32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ int64_t ufirst(int64_t v) {
  return (int64_t)(((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)((uint64_t)v >> 32)) << 32) |
                   (uint32_t)__builtin_amdgcn_readfirstlane((int)v));
}
template <typename P> __device__ __forceinline__ P* ufirst_ptr(P* p) {
  return reinterpret_cast<P*>((uintptr_t)ufirst((int64_t)(uintptr_t)p));
}
__device__ __forceinline__ Task uniform_task(const Task& a) {
  Task t;
  t.kind = ufirst(a.kind);
  t.inst = ufirst(a.inst);
  t.panel = ufirst(a.panel);
  t.m = ufirst(a.m);
  t.n = ufirst(a.n);
  t.k = ufirst(a.k);
  t.lda = ufirst(a.lda);
  t.ldc = ufirst(a.ldc);
  t.dofs = ufirst(a.dofs);
  t.aux = ufirst(a.aux);
  t.a_off = ufirst(a.a_off);
  t.b_off = ufirst(a.b_off);
  t.c_off = ufirst(a.c_off);
  t.succ_begin = ufirst(a.succ_begin);
  t.nsucc = ufirst(a.nsucc);
  t.pad0 = ufirst(a.pad0);
  t.pad1 = ufirst(a.pad1);
  return t;
}
template <typename T> __device__ __forceinline__ Ctx<T> uniform_ctx(const Ctx<T>& a) {
  Ctx<T> c;
  c.L = ufirst_ptr(a.L);
  c.LD = ufirst_ptr(a.LD);
  c.D = ufirst_ptr(a.D);
  c.Li = ufirst_ptr(a.Li);
  c.Gi = ufirst_ptr(a.Gi);
  c.W = ufirst_ptr(a.W);
  c.Z = ufirst_ptr(a.Z);
  c.iv = ufirst_ptr(a.iv);
  c.lds = (lds_char*)(uintptr_t)(uint32_t)ufirst((int32_t)(uint32_t)(uintptr_t)a.lds);
  c.nrhs = ufirst(a.nrhs);
  c.j0 = ufirst(a.j0);
  c.ncols = ufirst(a.ncols);
  return c;
}

template <typename T>
__device__ __forceinline__ Opnd<T> opn(const typename Cplx<T>::type* p, int64_t ld, int mode = OP_N, int i0 = 0) {
  Opnd<T> o;
  o.p = p;
  o.ld = ld;
  o.mode = mode;
  o.i0 = i0;
  return o;
}

template <typename T>
__device__ __forceinline__ Out<T> outp(typename Cplx<T>::type* dst, int64_t rs, int64_t cs, T alpha, T beta) {
  Out<T> o;
  o.dst = dst;
  o.rs = rs;
  o.cs = cs;
  o.src = beta != (T)0 ? dst : nullptr;
  o.srs = rs;
  o.scs = cs;
  o.alpha = alpha;
  o.beta = beta;
  o.dst2 = nullptr;
  o.rowdiv = nullptr;
  o.coldiv = nullptr;
  o.wt = false;
  return o;
}

// LDL^T of diagonal tile c of panel I (TK_FACT)
// In the complex64 factor a tile whose growth check trips is factored again
// in FP64 from the same (Schur-complemented) tile and stored rounded to
// complex64.
template <typename T>
__device__ __noinline__ void task_fact(const Ctx<T>& cx_, const Task& t_) {
  const Ctx<T> cx = uniform_ctx(cx_);
  const Task t = uniform_task(t_);
  const Tile tc = cx.iv->tiles[t.aux];
  const Panel P = cx.iv->panels[t.panel];
  if (cx.iv->pivot) {
    typedef typename Cplx<T>::type C;
    tile_bk<T, T>(cx.L + t.a_off, t.lda, t.m, cx.D + t.dofs, reinterpret_cast<C*>(cx.iv->Doff) + t.dofs,
                  cx.iv->ipiv + t.dofs, cx.Li + tc.linv_off, cx.Gi + tc.linv_off, P.n, t.dofs, cx.iv->status,
                  cx.lds);
    return;
  }
  float* gr = cx.iv->growth ? cx.iv->growth + 2 * t.panel : nullptr;
  GrowthCheck gc;
  gc.on = sizeof(T) == 4 && cx.iv->fallback != 0;
  gc.dmin = cx.iv->gdmin;
  gc.lmax = cx.iv->glmax;
  const bool tripped = tile_ldlt<T, T>(cx.L + t.a_off, t.lda, t.m, cx.D + t.dofs, cx.Li + tc.linv_off, P.n, t.dofs,
                                       cx.iv->status, gr, gr ? gr + 1 : nullptr, gc, cx.lds);
  if (sizeof(T) == 4 && tripped) {
    if (threadIdx.x == 0) atomicAdd(&cx.iv->status[2], 1);
    gc.on = false;
    tile_ldlt<double, T>(cx.L + t.a_off, t.lda, t.m, cx.D + t.dofs, cx.Li + tc.linv_off, P.n, t.dofs,
                         cx.iv->status, gr, gr ? gr + 1 : nullptr, gc, cx.lds);
  }
}

// L_rc = A_rc Linv_c^T D_c^-1, in place, and L_rc D_c = A_rc Linv_c^T into
// LD at the same place (TK_TRSM)
// With pivoting (F_c = L_cc^-1 P_c, G_c = D_c^-1 F_c, D_c with 2x2 blocks):
// LD_rc = A_rc F_c^T and L_rc = A_rc G_c^T, two products of the same A.
template <typename T>
__device__ __noinline__ void task_trsm(const Ctx<T>& cx_, const Task& t_) {
  const Ctx<T> cx = uniform_ctx(cx_);
  const Task t = uniform_task(t_);
  Acc<T, true> acc;
  acc.zero();
  if (cx.iv->pivot) {
    gemm_acc<T, 8, GeKB<T>::KB, OP_N, true>(acc, t.m, t.n, t.k, opn<T>(cx.L + t.a_off, t.lda), nullptr,
                                        opn<T>(cx.Li + t.b_off, t.ldc), cx.lds);
    gemm_store<T>(acc, t.m, t.n, outp<T>(cx.LD + t.a_off, 1, t.lda, (T)1, (T)0), cx.lds);
    acc.zero();
    gemm_acc<T, 8, GeKB<T>::KB, OP_N, true>(acc, t.m, t.n, t.k, opn<T>(cx.L + t.a_off, t.lda), nullptr,
                                        opn<T>(cx.Gi + t.b_off, t.ldc), cx.lds);
    gemm_store<T>(acc, t.m, t.n, outp<T>(cx.L + t.a_off, 1, t.lda, (T)1, (T)0), cx.lds);
    return;
  }
  gemm_acc<T, 8, GeKB<T>::KB, OP_N, true>(acc, t.m, t.n, t.k, opn<T>(cx.L + t.a_off, t.lda), nullptr,
                                      opn<T>(cx.Li + t.b_off, t.ldc), cx.lds);
  Out<T> o = outp<T>(cx.L + t.a_off, 1, t.lda, (T)1, (T)0);
  o.dst2 = cx.LD + t.a_off;
  o.coldiv = cx.D + t.dofs;
  gemm_store<T>(acc, t.m, t.n, o, cx.lds);
}

// Whether a Schur update of an m x n tile is formed as its
// transpose, C^T -= (L_sI D_I) L_rI^T.  The engine gives each wave 16 rows
// (two waves per SIMD, so more than 4 row blocks cost two) and issues the
// products of the accumulator's column blocks, so a tile with fewer row
// than column blocks issues fewer products transposed.  The same products
// are summed in the same order; only which side carries D differs.
__device__ __forceinline__ bool xupd_swap(int m, int n) {
  const int mb = (m + 15) >> 4, nb = (n + 15) >> 4;
  return (nb > 4 ? 2 : 1) * mb < (mb > 4 ? 2 : 1) * nb;
}

// C -= sum over the task's sources of (L_rI D_I) L_sI^T on one tile pair
// (TK_XUPD); t.pad0 > 1: the sources are xsrc[t.pad1 ...], else the task's
// own operands
// PRESRC: a merged update's source table is already in LDS (put there
// by the executor while it released the previous task).
template <typename T, bool PRESRC = false>
__device__ __noinline__ void task_xupd(const Ctx<T>& cx_, const Task& t_) {
  const Ctx<T> cx = uniform_ctx(cx_);
  const Task t = uniform_task(t_);
  Acc<T, true> acc;
  acc.zero();
  const int nsrc = t.pad0 > 1 ? t.pad0 : 1;
  // aux bit 1: the first update of a tile of a fill block, which holds no K
  // entries and is not zeroed beforehand: store the product, add nothing
  const T beta = (t.aux & 2) ? (T)0 : (T)1;
  const Out<T> o = outp<T>(cx.L + t.c_off, 1, t.ldc, (T)-1, beta);
  GePre<T> pre;
  pre.ok = false;
  auto src = [&](int q) {
    XSrc x{t.a_off, t.b_off, t.k, t.lda};
    if (t.pad0 > 1) x = cx.iv->xsrc[t.pad1 + q];
    return x;
  };
  bool done = false;
  if constexpr (sizeof(T) == 4) {
    // complex64: the sources go to LDS above the slab buffers, then one
    // direct-load pipeline runs over the slabs of all of them; the target's
    // loads go out with the last slab
    D3M_LDS GeSrc<T>* tab = reinterpret_cast<D3M_LDS GeSrc<T>*>(cx.lds + ge_lds_bytes_dma<T>());
    const bool sw = xupd_swap(t.m, t.n);
    if (!(PRESRC && t.pad0 > 1) && (int)threadIdx.x < nsrc) {
      const XSrc x = src(threadIdx.x);
      GeSrc<T> e;
      e.a = cx.LD + (sw ? x.b_off : x.a_off);
      e.b = cx.L + (sw ? x.a_off : x.b_off);
      e.lda = e.ldb = x.lda;
      e.k = x.k;
      e.pad = 0;
      ge_src_put(tab, (int)threadIdx.x, e);
    }
    __syncthreads();
    bool ok = true;
    for (int q = 0; q < nsrc; ++q) {
      const GeSrc<T> e = ge_src_lds(tab, q);
      ok = ok && ((((uintptr_t)e.a | (uintptr_t)e.b) & 15) == 0) && (((e.lda | e.ldb) & 1) == 0);
    }
    if (ok) {
      if (sw) {
        // its own copy of the pipeline and the store: with the strides
        // fixed at compile time in each, their addressing stays in registers
        const Out<T> ot = outp<T>(cx.L + t.c_off, t.ldc, 1, (T)-1, beta);
        ge_pipe<T, 8, true, true, false, true>(acc, t.n, t.m, nsrc, [&](int q) { return ge_src_lds(tab, q); },
                                               cx.lds, &pre, &ot);
        gemm_store<T>(acc, t.n, t.m, ot, nullptr, pre);
        return;
      }
      ge_pipe<T, 8, true, true, false, true>(acc, t.m, t.n, nsrc, [&](int q) { return ge_src_lds(tab, q); }, cx.lds,
                                             &pre, &o);
      done = true;
    }
  }
  if constexpr (sizeof(T) == 8) {
    // complex128: register slabs, one source at a time; one copy of the
    // source loop per column-block count, so that a tile with a partial last
    // column block issues the products of its own width, and the transpose
    // formed where that issues fewer (as on the direct-load path)
    const bool sw = xupd_swap(t.m, t.n);
    const int mm = sw ? t.n : t.m, nn = sw ? t.m : t.n;
    // A tile of at most 64 x 64 (64-row tiles) splits each source's k over
    // the two wave halves (both waves of each SIMD busy), chosen here, once,
    // outside the source loop.
    auto srcs = [&](auto wc, auto spl) {
      for (int q = 0; q < nsrc; ++q) {
        const XSrc x = src(q);
        gemm_acc_body<T, 8, GeKB<T>::KB, OP_N, true, false, true, false, decltype(spl)::value, decltype(wc)::value>(
            acc, mm, nn, x.k, opn<T>(cx.LD + (sw ? x.b_off : x.a_off), x.lda), nullptr,
            opn<T>(cx.L + (sw ? x.a_off : x.b_off), x.lda), cx.lds, nullptr, nullptr);
      }
    };
    using spl_t = std::integral_constant<bool, true>;
    using spl_f = std::integral_constant<bool, false>;
    if (mm <= 64 && nn <= 64) {
      switch ((nn + 15) >> 4) {
        case 1: srcs(std::integral_constant<int, 1>(), spl_t()); break;
        case 2: srcs(std::integral_constant<int, 2>(), spl_t()); break;
        case 3: srcs(std::integral_constant<int, 3>(), spl_t()); break;
        default: srcs(std::integral_constant<int, 4>(), spl_t()); break;
      }
    } else {
      switch ((nn + 15) >> 4) {
        case 1: srcs(std::integral_constant<int, 1>(), spl_f()); break;
        case 2: srcs(std::integral_constant<int, 2>(), spl_f()); break;
        case 3: srcs(std::integral_constant<int, 3>(), spl_f()); break;
        case 4: srcs(std::integral_constant<int, 4>(), spl_f()); break;
        case 5: srcs(std::integral_constant<int, 5>(), spl_f()); break;
        case 6: srcs(std::integral_constant<int, 6>(), spl_f()); break;
        case 7: srcs(std::integral_constant<int, 7>(), spl_f()); break;
        default: srcs(std::integral_constant<int, 8>(), spl_f()); break;
      }
    }
    if (sw) {
      gemm_store<T>(acc, t.n, t.m, outp<T>(cx.L + t.c_off, t.ldc, 1, (T)-1, beta), nullptr, pre);
      return;
    }
  } else if (!done) {
    for (int q = 0; q < nsrc; ++q) {
      const XSrc x = src(q);
      gemm_acc<T, 8, GeKB<T>::KB, OP_N, true>(acc, t.m, t.n, x.k, opn<T>(cx.LD + x.a_off, x.lda), nullptr,
                                          opn<T>(cx.L + x.b_off, x.lda), cx.lds);
    }
  }
  gemm_store<T>(acc, t.m, t.n, o, nullptr, pre);
}

// tile (r, c) of the inverse of panel I's unit lower diagonal block:
// Y^T = (sum_{c <= q < r} L_rq Linv_qc)^T into the unused upper tile (c, r),
// then Linv_rc = -Linv_rr Y (TK_INV)
template <typename T>
__device__ __noinline__ void task_inv(const Ctx<T>& cx_, const Task& t_) {
  const Ctx<T> cx = uniform_ctx(cx_);
  const Task t = uniform_task(t_);
  const Panel P = cx.iv->panels[t.panel];
  const Tile tr = cx.iv->tiles[t.aux], tc = cx.iv->tiles[t.dofs];
  typedef typename Cplx<T>::type C;
  C* Lb = cx.Li + P.ioff;
  const int n = P.n;
  Acc<T, true> acc;
  acc.zero();
  gemm_acc<T, 8, GeKB<T>::KB, OP_T>(acc, tc.sz, tr.sz, tr.r0 - tc.r0, opn<T>(Lb + tc.r0 + (int64_t)tc.r0 * n, n, OP_T),
                                    nullptr,
              opn<T>(cx.L + P.off + tr.r0 + (int64_t)tc.r0 * P.H, P.H), cx.lds);
  C* stage = Lb + tc.r0 + (int64_t)tr.r0 * n;
  gemm_store<T>(acc, tc.sz, tr.sz, outp<T>(stage, 1, n, (T)1, (T)0));
  acc.zero();
  gemm_acc<T, 8, GeKB<T>::KB, OP_N, true>(acc, tr.sz, tc.sz, tr.sz, opn<T>(Lb + tr.r0 + (int64_t)tr.r0 * n, n), nullptr,
                                    opn<T>(stage, n),
              cx.lds);
  gemm_store<T>(acc, tr.sz, tc.sz, outp<T>(Lb + tr.r0 + (int64_t)tc.r0 * n, 1, n, (T)-1, (T)0));
  if (cx.iv->pivot) {
    // G_rc = -G_rr Y (G = D^-1 F with F in place of Linv)
    C* Gb = cx.Gi + P.ioff;
    acc.zero();
    gemm_acc<T, 8, GeKB<T>::KB, OP_N, true>(acc, tr.sz, tc.sz, tr.sz, opn<T>(Gb + tr.r0 + (int64_t)tr.r0 * n, n),
                                        nullptr, opn<T>(stage, n), cx.lds);
    gemm_store<T>(acc, tr.sz, tc.sz, outp<T>(Gb + tr.r0 + (int64_t)tc.r0 * n, 1, n, (T)-1, (T)0));
  }
}

// forward, one tile: z_c = D_c^-1 sum_{p < r0_c + sz_c} Linv_II(c, p) b_p;
// with pivoting z_c = sum_p G_II(c, p) b_p up to the end of the factor tile
// (t.pad0 columns more: G's diagonal tiles are full)
template <typename T>
__device__ __noinline__ void task_ftile(const Ctx<T>& cx_, const Task& t_) {
  const Ctx<T> cx = uniform_ctx(cx_);
  const Task t = uniform_task(t_);
  const int nr = cx.nrhs, nc = cx.ncols, j0 = cx.j0;
  if (nc <= kMvMaxCols) {
    Out<T> o = outp<T>(cx.Z + t.c_off * nr + j0, nr, 1, (T)1, (T)0);
    o.wt = true;
    if (cx.iv->pivot) {
      solve_mv<T, false>(t.m, nc, t.k + t.pad0, cx.Gi + t.a_off, t.lda, cx.W + t.b_off * nr + j0, nr, o, cx.lds);
    } else {
      o.rowdiv = cx.D + t.dofs;
      solve_mv<T, false>(t.m, nc, t.k, cx.Li + t.a_off, t.lda, cx.W + t.b_off * nr + j0, nr, o, cx.lds);
    }
    return;
  }
  Acc<T> acc;
  acc.zero();
  if (cx.iv->pivot) {
    gemm_acc<T, 8, GeKB<T>::KB, OP_N, true, false, false, true, true>(acc, t.m, nc, t.k + t.pad0,
                                                               opn<T>(cx.Gi + t.a_off, t.lda), nullptr,
                                                               opn<T>(cx.W + t.b_off * nr + j0, nr), cx.lds);
    Out<T> o = outp<T>(cx.Z + t.c_off * nr + j0, nr, 1, (T)1, (T)0);
    o.wt = true;
    gemm_store<T>(acc, t.m, nc, o);
    return;
  }
  gemm_acc<T, 8, GeKB<T>::KB, OP_N, true, false, false, true, true>(acc, t.m, nc, t.k, opn<T>(cx.Li + t.a_off, t.lda),
                                                             nullptr, opn<T>(cx.W + t.b_off * nr + j0, nr),
                                                             cx.lds);
  Out<T> o = outp<T>(cx.Z + t.c_off * nr + j0, nr, 1, (T)1, (T)0);
  o.rowdiv = cx.D + t.dofs;
  o.wt = true;
  gemm_store<T>(acc, t.m, nc, o);
}

// forward update: b_r -= (L_rI D_I) z_I; t.n = 1: the target is an extra
// accumulator written first
template <typename T>
__device__ __noinline__ void task_fupd(const Ctx<T>& cx_, const Task& t_) {
  const Ctx<T> cx = uniform_ctx(cx_);
  const Task t = uniform_task(t_);
  const int nr = cx.nrhs, nc = cx.ncols, j0 = cx.j0;
  if (nc <= kMvMaxCols) {
    Out<T> o = outp<T>(cx.W + t.c_off * nr + j0, nr, 1, (T)-1, t.n ? (T)0 : (T)1);
    o.wt = true;
    solve_mv<T, false>(t.m, nc, t.k, cx.LD + t.a_off, t.lda, cx.Z + t.b_off * nr + j0, nr, o, cx.lds);
    return;
  }
  Acc<T> acc;
  acc.zero();
  // one source (kMergeSolve): a loop over sources around the inlined
  // pipeline would keep all of its state live across the back edge
  static_assert(kMergeSolve == 1, "forward updates have one source");
  gemm_acc<T, 8, GeKB<T>::KB, OP_N, true, false, false, true, true>(acc, t.m, nc, t.k, opn<T>(cx.LD + t.a_off, t.lda),
                                                                     nullptr, opn<T>(cx.Z + t.b_off * nr + j0, nr),
                                                                     cx.lds);
  // the first update into an extra accumulator overwrites it (beta 0)
  Out<T> o = outp<T>(cx.W + t.c_off * nr + j0, nr, 1, (T)-1, t.n ? (T)0 : (T)1);
  o.wt = true;
  gemm_store<T>(acc, t.m, nc, o);
}

// b_r += the t.k extra accumulators of tile r (N rows apart) (TK_RED)
template <typename T>
__device__ __noinline__ void task_red(const Ctx<T>& cx_, const Task& t_) {
  const Ctx<T> cx = uniform_ctx(cx_);
  const Task t = uniform_task(t_);
  const int64_t nr = cx.nrhs, stride = cx.iv->N * nr, nc = cx.ncols;
  D3M_GLB cpx<T>* w = gptr_mut<T>(cx.W + t.c_off * nr + cx.j0);
  const int64_t tot = (int64_t)t.m * nc;
  auto at = [&](int64_t e) { return (e / nc) * nr + e % nc; };  // element e: row e / nc, group column e % nc
  // a thread's elements in batches of E, every load of a batch issued before
  // its first add (one memory latency per batch instead of one per element);
  // element e adds accumulators 1..t.k onto b in that order.  Loads beyond
  // tot or t.k read element 0 of b (a valid address) and are not used.
  constexpr int E = 8;
  for (int64_t e0 = threadIdx.x; e0 < tot; e0 += (int64_t)E * kThreads) {
    cpx<T> v[E], u[kSolveSlots][E];
#pragma unroll
    for (int i = 0; i < E; ++i) {
      const int64_t e = e0 + (int64_t)i * kThreads, ec = e < tot ? at(e) : 0;
      v[i] = w[ec];
#pragma unroll
      for (int q = 0; q < kSolveSlots; ++q) u[q][i] = w[(q < t.k ? (q + 1) * stride : 0) + ec];
    }
#pragma unroll
    for (int i = 0; i < E; ++i) {
      const int64_t e = e0 + (int64_t)i * kThreads;
#pragma unroll
      for (int q = 0; q < kSolveSlots; ++q)
        if (q < t.k) {
          v[i].x += u[q][i].x;
          v[i].y += u[q][i].y;
        }
      if (e < tot) st_out<T>(w + at(e), v[i], true);
    }
  }
}

// backward push: t_c(I) -= L_Jc^T x_J for one row block J of panel I
template <typename T>
__device__ __noinline__ void task_bupd(const Ctx<T>& cx_, const Task& t_) {
  const Ctx<T> cx = uniform_ctx(cx_);
  const Task t = uniform_task(t_);
  const int nr = cx.nrhs, nc = cx.ncols, j0 = cx.j0;
  if (nc <= kMvMaxCols) {
    Out<T> o = outp<T>(cx.Z + t.c_off * nr + j0, nr, 1, (T)-1, (T)1);
    o.wt = true;
    solve_mv<T, true>(t.m, nc, t.k, cx.L + t.a_off, t.lda, cx.W + t.b_off * nr + j0, nr, o, cx.lds);
    return;
  }
  Acc<T> acc;
  acc.zero();
  gemm_acc<T, 8, GeKB<T>::KB, OP_T, false, false, false, true, true>(acc, t.m, nc, t.k, opn<T>(cx.L + t.a_off, t.lda, OP_T),
                                                              nullptr, opn<T>(cx.W + t.b_off * nr + j0, nr), cx.lds);
  Out<T> o = outp<T>(cx.Z + t.c_off * nr + j0, nr, 1, (T)-1, (T)1);
  o.wt = true;
  gemm_store<T>(acc, t.m, nc, o);
}

// backward, one tile: x_c = sum_{p >= r0_c} Linv_II(p, c) t_p; with
// pivoting (Linv holds F = L^-1 P, full in its diagonal tiles) the sum
// starts t.pad0 rows earlier, at the factor tile's first row
template <typename T>
__device__ __noinline__ void task_btile(const Ctx<T>& cx_, const Task& t_) {
  const Ctx<T> cx = uniform_ctx(cx_);
  const Task t = uniform_task(t_);
  const int nr = cx.nrhs, nc = cx.ncols, j0 = cx.j0;
  const int back = cx.iv->pivot ? t.pad0 : 0;
  if (nc <= kMvMaxCols) {
    Out<T> o = outp<T>(cx.W + t.c_off * nr + j0, nr, 1, (T)1, (T)0);
    o.wt = true;
    solve_mv<T, true>(t.m, nc, t.k + back, cx.Li + t.a_off - back, t.lda, cx.Z + (t.b_off - back) * nr + j0, nr, o,
                      cx.lds);
    return;
  }
  Acc<T> acc;
  acc.zero();
  gemm_acc<T, 8, GeKB<T>::KB, OP_T, false, false, false, true, true>(
      acc, t.m, nc, t.k + back, opn<T>(cx.Li + t.a_off - back, t.lda, OP_T), nullptr,
      opn<T>(cx.Z + (t.b_off - back) * nr + j0, nr), cx.lds);
  Out<T> o = outp<T>(cx.W + t.c_off * nr + j0, nr, 1, (T)1, (T)0);
  o.wt = true;
  gemm_store<T>(acc, t.m, nc, o);
}

template <typename T, bool PRESRC = false>
__device__ void run_task(const Task& t, const InstView* ivs, int nrhs, int groups, lds_char* lds) {
  typedef typename Cplx<T>::type C;
  Ctx<T> cx;
  cx.iv = ivs + t.inst;
  cx.L = reinterpret_cast<C*>(cx.iv->L);
  cx.LD = reinterpret_cast<C*>(cx.iv->LD);
  cx.D = reinterpret_cast<C*>(cx.iv->D);
  cx.Li = reinterpret_cast<C*>(cx.iv->Linv);
  cx.Gi = reinterpret_cast<C*>(cx.iv->Ginv);
  cx.W = reinterpret_cast<C*>(cx.iv->W);
  cx.Z = reinterpret_cast<C*>(cx.iv->Z);
  cx.lds = lds;
  cx.nrhs = nrhs > 0 ? nrhs : cx.iv->nrhs;
  // the right-hand-side group of a solve task (bits 8.. of the kind)
  const int grp = t.kind >> 8, per = (cx.nrhs + groups - 1) / groups;
  cx.j0 = grp * per;
  cx.ncols = min(cx.nrhs, cx.j0 + per) - cx.j0;
  if (cx.ncols <= 0) return;
  switch (t.kind & 0xff) {
    case TK_FACT: task_fact<T>(cx, t); break;
    case TK_TRSM: task_trsm<T>(cx, t); break;
    case TK_XUPD: task_xupd<T, PRESRC>(cx, t); break;
    case TK_INV: task_inv<T>(cx, t); break;
    case TK_FTILE: task_ftile<T>(cx, t); break;
    case TK_FUPD: task_fupd<T>(cx, t); break;
    case TK_BUPD: task_bupd<T>(cx, t); break;
    case TK_BTILE: task_btile<T>(cx, t); break;
    case TK_RED: task_red<T>(cx, t); break;
    default: break;
  }
}

// the complex64 kernel also holds the FP64 re-factor of a tile
template <typename T> constexpr int dag_lds_bytes() {
  constexpr int a = tile_ldlt_lds_bytes<double>(), b = ge_lds_bytes_dma<T>(), c = tile_bk_lds_bytes<T>();
  return (a > b ? a : b) > c ? (a > b ? a : b) : c;
}

// ---------------------------------------------------------------- the executor
// PHASE only names the launch (0: factor DAG, 1: solve DAG) so that
// profilers report the two separately.
template <typename T, int PHASE>
__global__ __launch_bounds__(kThreads) void k_dag(DagArgs a) {
  __shared__ __attribute__((aligned(16))) char lds[dag_lds_bytes<T>()];
  // The next ticket and its task record, double-buffered by loop parity:
  // wave 1 fills slot b ^ 1 while the current task (read from slot b) may
  // still be running on other waves, so a task body without any barrier
  // (TK_RED) cannot have its record overwritten before a slow wave copied it.
  // Slot b ^ 1 was last read in the previous iteration, before two barriers.
  __shared__ int s_ticket, s_next[2];
  __shared__ Task s_task[2];
  if (a.skip && __hip_atomic_load(a.skip, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) return;
  // the next ticket, fetched together with the abort flag (a ticket taken
  // after an abort is simply not run); -1: none
  auto take = [&]() {
    const int aborted = __hip_atomic_load(a.abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const int t = __hip_atomic_fetch_add(a.head, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return (aborted != 0 || t >= a.ntask) ? -1 : t;
  };
  // wait until ticket t's predecessors are done (-1: aborted or timed out),
  // then acquire on behalf of the workgroup (its waves share the CU's caches)
  auto wait_ready = [&](int t) {
    const uint64_t t0 = wall_clock64();
    if (t >= 0) {
      while (__hip_atomic_load(&a.counters[t], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) > 0) {
        __builtin_amdgcn_s_sleep(2);
        if (__hip_atomic_load(a.abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) { t = -1; break; }
        // wall_clock64 ticks at 100 MHz: 10 ns per tick
        if ((int64_t)(wall_clock64() - t0) * 10 > a.spin_limit_ns) {
          __hip_atomic_store(a.abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          t = -1;
          break;
        }
      }
    }
    if (t >= 0) __scoped_atomic_thread_fence(__ATOMIC_ACQUIRE, __MEMORY_SCOPE_DEVICE);
    if (t >= 0 && a.trace) {
      a.trace[4 * t] = (int64_t)t0;
      a.trace[4 * t + 1] = (int64_t)wall_clock64();
      a.trace[4 * t + 3] = blockIdx.x;
    }
    return t;
  };
  // every wave's stores are complete (the caller's barrier): every lane of
  // wave 0 releases, then lane l tells successors l, l + 64, ...: their
  // indices come in one vector load and the decrements go out together (one
  // lane telling them in turn waits for each decrement, as atomics count
  // among the outstanding vector-memory operations)
  auto release = [&](const Task& task, int t) {
    if (threadIdx.x < 64) {
      // solve tasks store only with write-through stores (st_out), complete
      // here (each wave waited for its stores before the barrier): no L2
      // write-back; the factor's tile stores are ordinary and need it
      if constexpr (PHASE == 1) __scoped_atomic_thread_fence(__ATOMIC_RELEASE, __MEMORY_SCOPE_WRKGRP);
      else __scoped_atomic_thread_fence(__ATOMIC_RELEASE, __MEMORY_SCOPE_DEVICE);
      if (threadIdx.x == 0 && a.trace) a.trace[4 * t + 2] = (int64_t)wall_clock64();
      for (int s = threadIdx.x; s < task.nsucc; s += 64)
        __hip_atomic_fetch_add(&a.counters[a.succ[task.succ_begin + s]], -1, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
    }
  };
  // Wave 1 takes the next ticket and reads its task record
  // (and a complex64 merged update's source table, into LDS where the
  // update reads it) while the other waves' stores drain; after the
  // barrier it waits for that task's predecessors while wave 0 releases
  // the finished task.  Only read-only tables are read before the wait.
  constexpr bool kPreSrc = sizeof(typename Cplx<T>::type) == 8;
  static_assert(kMergeSrc <= 64, "one lane of wave 1 per source");
  // Lanes of wave 1 learn the ticket from lane 0 by a cross-lane read, not
  // through LDS: lane 0's LDS store and the other lanes' loads would be
  // unsynchronized accesses, which the compiler may reorder (the other
  // lanes would then see an old s_next, e.g. the -1 an earlier launch left,
  // and leave their table entries stale).  Each lane then reads the fields
  // of the task record it needs from global memory.
  auto take_next = [&](int b) {
    if (threadIdx.x >= 64 && threadIdx.x < 128) {
      int t = -1;
      if (threadIdx.x == 64) t = take();
      t = __builtin_amdgcn_readlane(t, 0);
      if (threadIdx.x == 64) {
        s_next[b] = t;
        if (t >= 0) s_task[b] = a.tasks[t];
      }
      if (kPreSrc && t >= 0) {
        const int q = (int)threadIdx.x - 64;
        const Task* nt = a.tasks + t;
        const int kind = nt->kind, pad0 = nt->pad0;
        if ((kind & 0xff) == TK_XUPD && pad0 > 1 && q < pad0) {
          typedef typename Cplx<T>::type C;
          const InstView* iv = a.inst + nt->inst;
          const XSrc x = iv->xsrc[nt->pad1 + q];
          const bool sw = xupd_swap(nt->m, nt->n);
          GeSrc<T> e;
          e.a = reinterpret_cast<const C*>(iv->LD) + (sw ? x.b_off : x.a_off);
          e.b = reinterpret_cast<const C*>(iv->L) + (sw ? x.a_off : x.b_off);
          e.lda = e.ldb = x.lda;
          e.k = x.k;
          e.pad = 0;
          ge_src_put(reinterpret_cast<D3M_LDS GeSrc<T>*>((lds_char*)lds + ge_lds_bytes_dma<T>()), q, e);
        }
      }
    }
  };
  int b = 0;
  take_next(b);
  for (;;) {
    if (threadIdx.x == 64) s_ticket = wait_ready(s_next[b]);
    __syncthreads();
    const int t = __builtin_amdgcn_readfirstlane(s_ticket);
    if (t < 0) break;
    const Task task = uniform_task(s_task[b]);
    run_task<T, kPreSrc>(task, a.inst, a.nrhs, a.rhs_groups > 0 ? a.rhs_groups : 1, (lds_char*)lds);
    // The source table is single-buffered: the only task that reads it (a
    // merged XUPD) ends with a barrier after its last read, and every LDS
    // access of any task after its last barrier lies below the table, so
    // wave 1 may now fill it for the next task.
    __builtin_amdgcn_s_waitcnt(0);
    take_next(b ^ 1);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    release(task, t);
    b ^= 1;
  }
}

// Same task bodies, launched one task per workgroup for one level of the DAG
// (no waits): a stream-ordered fallback executor.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_level(const Task* tasks, int begin, int end, const InstView* iv) {
  __shared__ __attribute__((aligned(16))) char lds[dag_lds_bytes<T>()];
  int t = begin + blockIdx.x;
  if (t >= end) return;
  const Task task = tasks[t];
  run_task<T>(task, iv, 0, 1, (lds_char*)lds);
}

__global__ void k_reset(int32_t* counters, const int32_t* init, int n, int32_t* head, int32_t* abort_flag,
                        const int32_t* skip) {
  if (skip && *skip) return;
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  for (; i < n; i += gridDim.x * blockDim.x) counters[i] = init[i];
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    *head = 0;
    *abort_flag = 0;
  }
}

hipError_t launch_dag(const DagArgs& a, int prec, int nworkers, bool solve, hipStream_t s) {
  if (a.ntask == 0) return hipSuccess;
  if (prec == 0) {
    if (solve) hipLaunchKernelGGL((k_dag<double, 1>), dim3(nworkers), dim3(kThreads), 0, s, a);
    else hipLaunchKernelGGL((k_dag<double, 0>), dim3(nworkers), dim3(kThreads), 0, s, a);
  } else {
    if (solve) hipLaunchKernelGGL((k_dag<float, 1>), dim3(nworkers), dim3(kThreads), 0, s, a);
    else hipLaunchKernelGGL((k_dag<float, 0>), dim3(nworkers), dim3(kThreads), 0, s, a);
  }
  return hipGetLastError();
}

hipError_t launch_level(const Task* tasks, int begin, int end, const InstView* iv, int prec, hipStream_t s) {
  if (end <= begin) return hipSuccess;
  if (prec == 0) hipLaunchKernelGGL(k_level<double>, dim3(end - begin), dim3(kThreads), 0, s, tasks, begin, end, iv);
  else hipLaunchKernelGGL(k_level<float>, dim3(end - begin), dim3(kThreads), 0, s, tasks, begin, end, iv);
  return hipGetLastError();
}

hipError_t launch_reset(int32_t* counters, const int32_t* init, int n, int32_t* head, int32_t* abort_flag,
                        const int32_t* skip, hipStream_t s) {
  int blocks = (n + 255) / 256;
  if (blocks < 1) blocks = 1;
  if (blocks > 1024) blocks = 1024;
  hipLaunchKernelGGL(k_reset, dim3(blocks), dim3(256), 0, s, counters, init, n, head, abort_flag, skip);
  return hipGetLastError();
}

}  // namespace d3m
