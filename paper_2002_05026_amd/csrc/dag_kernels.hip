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

namespace d3m {

// ---------------------------------------------------------------- tile LDL^T
// In-place LDL^T (no pivoting, transposes only) of the m x m tile at `a`
// (column-major, leading dimension lda, lower triangle read), m <= 128, held
// packed in LDS.  Writes L strictly below the diagonal and D on it back to
// `a`, D to dout[0..m), and the full m x m inverse of the unit lower factor
// to linv (column-major, ld m).  Records the first bad pivot (zero or not
// finite) as internal row index row0 + k in status[0].
template <typename T> constexpr int fact_lds_bytes() {
  return (kTileMax * (kTileMax + 1) / 2 + 2 * kTileMax) * (int)sizeof(typename Cplx<T>::type);
}

template <typename T>
__device__ __noinline__ void fact_tile(typename Cplx<T>::type* a_, int64_t lda, int m, typename Cplx<T>::type* dout_,
                                       typename Cplx<T>::type* linv_, int row0, int32_t* status, float* gmin_d,
                                       float* gmax_l, lds_char* lds) {
  D3M_LDS cpx<T>* L = reinterpret_cast<D3M_LDS cpx<T>*>(lds);
  D3M_LDS cpx<T>* U = L + kTileMax * (kTileMax + 1) / 2;
  D3M_GLB cpx<T>* a = gptr_mut<T>(a_);
  D3M_GLB cpx<T>* dout = gptr_mut<T>(dout_);
  D3M_GLB cpx<T>* linv = gptr_mut<T>(linv_);
  const int tid = threadIdx.x;
  auto idx = [m](int i, int j) { return j * (2 * m - j + 1) / 2 + (i - j); };
  wg_sync_global();
  for (int e = tid; e < m * m; e += kThreads) {
    int i = e % m, j = e / m;
    if (i >= j) L[idx(i, j)] = a[i + (int64_t)j * lda];
  }
  __syncthreads();
  // right-looking elimination: u = L(:,k)/d, trailing lower part -= u L(:,k)^T
  for (int k = 0; k < m; ++k) {
    const cpx<T> d = L[idx(k, k)];
    if (tid == 0) {
      T ad = sqrt(d.x * d.x + d.y * d.y);
      bool bad = !(ad > (T)0) || !isfinite(d.x) || !isfinite(d.y);
      if (bad) {
        atomicMin(&status[0], row0 + k);
        atomicAdd(&status[1], 1);
      }
      if (gmin_d) atomicMin(reinterpret_cast<int*>(gmin_d), __float_as_int((float)ad));
    }
    for (int i = k + 1 + tid; i < m; i += kThreads) U[i] = cpx_div(L[idx(i, k)], d);
    __syncthreads();
    const int R = m - k - 1;
    for (int e = tid; e < R * R; e += kThreads) {
      int ii = e % R, jj = e / R;
      if (ii >= jj) {
        int i = k + 1 + ii, j = k + 1 + jj;
        const cpx<T> u = U[i], l = L[idx(j, k)];
        cpx<T> t = L[idx(i, j)];
        t.x -= u.x * l.x - u.y * l.y;
        t.y -= u.x * l.y + u.y * l.x;
        L[idx(i, j)] = t;
      }
    }
    __syncthreads();
    for (int i = k + 1 + tid; i < m; i += kThreads) L[idx(i, k)] = U[i];
    __syncthreads();
  }
  // L and D back to global; D also to dout
  float lmax = 0.f;
  for (int e = tid; e < m * m; e += kThreads) {
    int i = e % m, j = e / m;
    if (i >= j) {
      const cpx<T> v = L[idx(i, j)];
      a[i + (int64_t)j * lda] = v;
      if (i == j) dout[i] = v;
      else lmax = fmaxf(lmax, (float)sqrt(v.x * v.x + v.y * v.y));
    }
  }
  if (gmax_l) atomicMax(reinterpret_cast<int*>(gmax_l), __float_as_int(lmax));
  __syncthreads();
  // invert the unit lower factor in place: for j = m-2 .. 0,
  // Linv(i, j) = -(v_i + sum_{j<q<i} Linv(i, q) v_q), v = L(:, j)
  for (int j = m - 2; j >= 0; --j) {
    for (int i = j + 1 + tid; i < m; i += kThreads) U[i] = L[idx(i, j)];
    __syncthreads();
    for (int i = j + 1 + tid; i < m; i += kThreads) {
      cpx<T> s = U[i];
      for (int q = j + 1; q < i; ++q) {
        const cpx<T> x = L[idx(i, q)], v = U[q];
        s.x += x.x * v.x - x.y * v.y;
        s.y += x.x * v.y + x.y * v.x;
      }
      s.x = -s.x;
      s.y = -s.y;
      L[idx(i, j)] = s;
    }
    __syncthreads();
  }
  for (int e = tid; e < m * m; e += kThreads) {
    int i = e % m, j = e / m;
    cpx<T> v;
    if (i > j) v = L[idx(i, j)];
    else { v.x = (i == j) ? (T)1 : (T)0; v.y = 0; }
    linv[e] = v;
  }
  wg_sync_global();
}

// ---------------------------------------------------------------- task bodies
template <typename T> struct Ctx {
  typedef typename Cplx<T>::type C;
  C* L;
  C* D;
  C* Li;
  C* W;
  const InstView* iv;
  lds_char* lds;
  int nrhs;
};

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
  o.rowdiv = nullptr;
  o.coldiv = nullptr;
  return o;
}

// One row strip (rows of a tile, all columns of panel I) through
// L_rc = (A_rc - sum_{p<c} L_rp D_p L_cp^T) Linv_c^T D_c^-1 for the column
// tiles c < ncol of I (left-looking inside the strip).
template <typename T>
__device__ void strip_solve(const Ctx<T>& cx, const Panel& P, typename Cplx<T>::type* strip, int m, int ncol) {
  typedef typename Cplx<T>::type C;
  for (int c = 0; c < ncol; ++c) {
    const Tile tc = cx.iv->tiles[P.tile0 + c];
    C* tile = strip + (int64_t)tc.r0 * P.H;
    Acc<T> acc;
    if (tc.r0 > 0) {
      acc.zero();
      gemm_acc<T>(acc, m, tc.sz, tc.r0, opn<T>(strip, P.H), cx.D + P.prow0,
                  opn<T>(cx.L + P.off + tc.r0, P.H), cx.lds);
      gemm_store<T>(acc, m, tc.sz, outp<T>(tile, 1, P.H, (T)-1, (T)1));
    }
    acc.zero();
    gemm_acc<T>(acc, m, tc.sz, tc.sz, opn<T>(tile, P.H), nullptr, opn<T>(cx.Li + tc.linv_off, tc.sz),
                cx.lds);
    Out<T> o = outp<T>(tile, 1, P.H, (T)1, (T)0);
    o.coldiv = cx.D + P.prow0 + tc.r0;
    gemm_store<T>(acc, m, tc.sz, o);
  }
}

template <typename T>
__device__ __noinline__ void task_diagf(const Ctx<T>& cx, const Task& t) {
  typedef typename Cplx<T>::type C;
  const Panel P = cx.iv->panels[t.panel];
  float* gr = cx.iv->growth ? cx.iv->growth + 2 * t.panel : nullptr;
  for (int r = 0; r < P.nt; ++r) {
    const Tile tr = cx.iv->tiles[P.tile0 + r];
    C* strip = cx.L + P.off + tr.r0;
    strip_solve<T>(cx, P, strip, tr.sz, r);
    C* diag = strip + (int64_t)tr.r0 * P.H;
    if (tr.r0 > 0) {
      Acc<T> acc;
      acc.zero();
      gemm_acc<T>(acc, tr.sz, tr.sz, tr.r0, opn<T>(strip, P.H), cx.D + P.prow0, opn<T>(strip, P.H),
                  cx.lds);
      gemm_store<T>(acc, tr.sz, tr.sz, outp<T>(diag, 1, P.H, (T)-1, (T)1));
    }
    fact_tile<T>(diag, P.H, tr.sz, cx.D + P.prow0 + tr.r0, cx.Li + tr.linv_off, P.prow0 + tr.r0,
                 cx.iv->status, gr ? gr : nullptr, gr ? gr + 1 : nullptr, cx.lds);
  }
}

template <typename T>
__device__ __noinline__ void task_pstrip(const Ctx<T>& cx, const Task& t) {
  const Panel P = cx.iv->panels[t.panel];
  strip_solve<T>(cx, P, cx.L + t.a_off, t.m, P.nt);
}

template <typename T>
__device__ __noinline__ void task_xupd(const Ctx<T>& cx, const Task& t) {
  Acc<T> acc;
  acc.zero();
  gemm_acc<T>(acc, t.m, t.n, t.k, opn<T>(cx.L + t.a_off, t.lda), cx.D + t.dofs,
              opn<T>(cx.L + t.b_off, t.lda), cx.lds);
  gemm_store<T>(acc, t.m, t.n, outp<T>(cx.L + t.c_off, 1, t.ldc, (T)-1, (T)1));
}

// forward: z_c = D_c^-1 Linv_c (b_c - sum_{p<c} L_cp D_p z_p), tile by tile
template <typename T>
__device__ __noinline__ void task_fdiag(const Ctx<T>& cx, const Task& t) {
  typedef typename Cplx<T>::type C;
  const Panel P = cx.iv->panels[t.panel];
  const int nr = cx.nrhs;
  for (int c = 0; c < P.nt; ++c) {
    const Tile tc = cx.iv->tiles[P.tile0 + c];
    C* wc = cx.W + (int64_t)(P.prow0 + tc.r0) * nr;
    Acc<T> acc;
    if (tc.r0 > 0) {
      acc.zero();
      gemm_acc<T>(acc, tc.sz, nr, tc.r0, opn<T>(cx.L + P.off + tc.r0, P.H), cx.D + P.prow0,
                  opn<T>(cx.W + (int64_t)P.prow0 * nr, nr), cx.lds);
      gemm_store<T>(acc, tc.sz, nr, outp<T>(wc, nr, 1, (T)-1, (T)1));
    }
    acc.zero();
    gemm_acc<T>(acc, tc.sz, nr, tc.sz, opn<T>(cx.Li + tc.linv_off, tc.sz), nullptr, opn<T>(wc, nr), cx.lds);
    Out<T> o = outp<T>(wc, nr, 1, (T)1, (T)0);
    o.rowdiv = cx.D + P.prow0 + tc.r0;
    gemm_store<T>(acc, tc.sz, nr, o);
  }
}

// forward update: b_r -= L_rI D_I z_I
template <typename T>
__device__ __noinline__ void task_fupd(const Ctx<T>& cx, const Task& t) {
  const int nr = cx.nrhs;
  Acc<T> acc;
  acc.zero();
  gemm_acc<T>(acc, t.m, nr, t.k, opn<T>(cx.L + t.a_off, t.lda), cx.D + t.dofs,
              opn<T>(cx.W + t.b_off * nr, nr), cx.lds);
  gemm_store<T>(acc, t.m, nr, outp<T>(cx.W + t.c_off * nr, nr, 1, (T)-1, (T)1));
}

// backward push: z_c(I) -= L_Jc^T x_J for one row block J of panel I
template <typename T>
__device__ __noinline__ void task_bupd(const Ctx<T>& cx, const Task& t) {
  const int nr = cx.nrhs;
  Acc<T> acc;
  acc.zero();
  gemm_acc<T>(acc, t.m, nr, t.k, opn<T>(cx.L + t.a_off, t.lda, OP_T), nullptr, opn<T>(cx.W + t.b_off * nr, nr),
              cx.lds);
  gemm_store<T>(acc, t.m, nr, outp<T>(cx.W + t.c_off * nr, nr, 1, (T)-1, (T)1));
}

// backward: x_c = Linv_c^T (t_c - sum_{p>c} L_pc^T x_p), last tile first
template <typename T>
__device__ __noinline__ void task_bdiag(const Ctx<T>& cx, const Task& t) {
  typedef typename Cplx<T>::type C;
  const Panel P = cx.iv->panels[t.panel];
  const int nr = cx.nrhs;
  for (int c = P.nt - 1; c >= 0; --c) {
    const Tile tc = cx.iv->tiles[P.tile0 + c];
    C* wc = cx.W + (int64_t)(P.prow0 + tc.r0) * nr;
    const int below = tc.r0 + tc.sz;
    Acc<T> acc;
    if (below < P.n) {
      acc.zero();
      gemm_acc<T>(acc, tc.sz, nr, P.n - below,
                  opn<T>(cx.L + P.off + below + (int64_t)tc.r0 * P.H, P.H, OP_T), nullptr,
                  opn<T>(cx.W + (int64_t)(P.prow0 + below) * nr, nr), cx.lds);
      gemm_store<T>(acc, tc.sz, nr, outp<T>(wc, nr, 1, (T)-1, (T)1));
    }
    acc.zero();
    gemm_acc<T>(acc, tc.sz, nr, tc.sz, opn<T>(cx.Li + tc.linv_off, tc.sz, OP_T), nullptr, opn<T>(wc, nr),
                cx.lds);
    gemm_store<T>(acc, tc.sz, nr, outp<T>(wc, nr, 1, (T)1, (T)0));
  }
}

template <typename T>
__device__ void run_task(const Task& t, const InstView* ivs, int nrhs, lds_char* lds) {
  typedef typename Cplx<T>::type C;
  Ctx<T> cx;
  cx.iv = ivs + t.inst;
  cx.L = reinterpret_cast<C*>(cx.iv->L);
  cx.D = reinterpret_cast<C*>(cx.iv->D);
  cx.Li = reinterpret_cast<C*>(cx.iv->Linv);
  cx.W = reinterpret_cast<C*>(cx.iv->W);
  cx.lds = lds;
  cx.nrhs = nrhs > 0 ? nrhs : cx.iv->nrhs;
  switch (t.kind) {
    case TK_DIAGF: task_diagf<T>(cx, t); break;
    case TK_PSTRIP: task_pstrip<T>(cx, t); break;
    case TK_XUPD: task_xupd<T>(cx, t); break;
    case TK_FDIAG: task_fdiag<T>(cx, t); break;
    case TK_FUPD: task_fupd<T>(cx, t); break;
    case TK_BUPD: task_bupd<T>(cx, t); break;
    case TK_BDIAG: task_bdiag<T>(cx, t); break;
    default: break;
  }
}

template <typename T> constexpr int dag_lds_bytes() {
  return fact_lds_bytes<T>() > ge_lds_bytes<T>() ? fact_lds_bytes<T>() : ge_lds_bytes<T>();
}

// ---------------------------------------------------------------- the executor
template <typename T>
__global__ __launch_bounds__(kThreads) void k_dag(DagArgs a) {
  __shared__ __attribute__((aligned(16))) char lds[dag_lds_bytes<T>()];
  __shared__ int s_ticket;
  if (a.skip && __hip_atomic_load(a.skip, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) return;
  for (;;) {
    if (threadIdx.x == 0) {
      int t = -1;
      if (__hip_atomic_load(a.abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0) {
        t = __hip_atomic_fetch_add(a.head, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (t >= a.ntask) t = -1;
      }
      uint64_t t0 = wall_clock64();
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
      // acquire on behalf of the workgroup (its waves share the CU's caches)
      if (t >= 0) __scoped_atomic_thread_fence(__ATOMIC_ACQUIRE, __MEMORY_SCOPE_DEVICE);
      s_ticket = t;
      if (t >= 0 && a.trace) {
        a.trace[4 * t] = (int64_t)t0;
        a.trace[4 * t + 1] = (int64_t)wall_clock64();
        a.trace[4 * t + 3] = blockIdx.x;
      }
    }
    __syncthreads();
    const int t = s_ticket;
    if (t < 0) break;
    const Task task = a.tasks[t];
    run_task<T>(task, a.inst, a.nrhs, (lds_char*)lds);
    // every wave's stores complete, then one agent-scope release for the
    // workgroup before the successors are told
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x == 0) {
      __scoped_atomic_thread_fence(__ATOMIC_RELEASE, __MEMORY_SCOPE_DEVICE);
      if (a.trace) a.trace[4 * t + 2] = (int64_t)wall_clock64();
      for (int s = 0; s < task.nsucc; ++s)
        __hip_atomic_fetch_add(&a.counters[a.succ[task.succ_begin + s]], -1, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
    }
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
  run_task<T>(task, iv, 0, (lds_char*)lds);
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

hipError_t launch_dag(const DagArgs& a, int prec, int nworkers, hipStream_t s) {
  if (a.ntask == 0) return hipSuccess;
  if (prec == 0) hipLaunchKernelGGL(k_dag<double>, dim3(nworkers), dim3(kThreads), 0, s, a);
  else hipLaunchKernelGGL(k_dag<float>, dim3(nworkers), dim3(kThreads), 0, s, a);
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
