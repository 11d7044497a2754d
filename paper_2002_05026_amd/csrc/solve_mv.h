// Products of the block solve with few right-hand sides (Sec. II, dual
// solution: the forward and backward substitutions with the factor blocks).
//
//   out(i, j) = alpha * sum_p A(i, p) B(p, j)  [+ beta * out(i, j)]  [/ rowdiv[i]]
//
// for i < m <= 128 rows of one solve task and j < nc <= 8 columns of the
// right-hand sides (B and out row-major with row strides ldb and o.rs).  With
// so few columns the task reads its block of L once and does little
// arithmetic per byte: the MFMA tile path, which stages the operand in
// slabs and keeps two slabs in flight, waits for memory on every slab.  Here
// every lane issues all its loads of a pass before its products, on the
// vector units, so a task streams its block at the CU's load rate.
//
//   OP_N (A(i, p) at A[i + p*lda]; FTILE and FUPD): lane r of a wave takes
//   row r, the waves split p; B goes through LDS (the same element for the
//   whole wave), and the waves' partial sums are added in LDS in a fixed
//   order.
//   OP_T (A(i, p) at A[p + i*lda]; BUPD and BTILE): lanes take consecutive p
//   (coalesced along the stored columns), each wave a batch of rows; the 64
//   lane sums are reduced by a butterfly that halves the values each lane
//   holds at every step.
//
// Every thread of the workgroup calls; results are deterministic (fixed
// summation order).  LDS use (OP_N) stays below 88 KB.  nc <= kMvMaxCols.
#pragma once
#include <hip/hip_runtime.h>

#include "d3m_internal.h"
#include "gemm_engine.h"

namespace d3m {

constexpr int kMvMaxCols = 8;  // right-hand-side columns of one task handled here
static_assert(kTileMax * kMvMaxCols <= 2 * kThreads, "mv_n: at most two outputs per thread");

template <typename T> __device__ __forceinline__ cpx<T> mv_zero() {
  cpx<T> z;
  z.x = (T)0;
  z.y = (T)0;
  return z;
}

// acc += a * b (complex)
template <typename T> __device__ __forceinline__ void mv_fma(cpx<T>& acc, cpx<T> a, cpx<T> b) {
  acc.x = fma(a.x, b.x, acc.x);
  acc.x = fma(-a.y, b.y, acc.x);
  acc.y = fma(a.x, b.y, acc.y);
  acc.y = fma(a.y, b.x, acc.y);
}

// The beta term and the row divisor of output (i, j), loaded ahead (their
// latency then overlaps the products).
template <typename T> struct MvPre {
  cpx<T> src, div;
};
template <typename T> __device__ __forceinline__ MvPre<T> mv_pre(const Out<T>& o, int i, int j) {
  MvPre<T> q;
  q.src = o.src ? *gptr<T>(o.src + (int64_t)i * o.srs + (int64_t)j * o.scs) : mv_zero<T>();
  q.div = o.rowdiv ? *gptr<T>(o.rowdiv + i) : mv_zero<T>();
  return q;
}
template <typename T> __device__ __forceinline__ void mv_put(const Out<T>& o, int i, int j, cpx<T> acc,
                                                           const MvPre<T>& q) {
  cpx<T> r;
  r.x = acc.x * o.alpha;
  r.y = acc.y * o.alpha;
  if (o.src) {
    r.x += o.beta * q.src.x;
    r.y += o.beta * q.src.y;
  }
  if (o.rowdiv) r = cpx_div(r, q.div);
  st_out<T>(gptr_mut<T>(o.dst) + (int64_t)i * o.rs + (int64_t)j * o.cs, r, o.wt);
}

// OP_N.  NCP: nc rounded up to a power of two.
template <typename T, int NCP>
__device__ __noinline__ void mv_n(int m, int nc, int k, const typename Cplx<T>::type* A, int64_t lda,
                                  const typename Cplx<T>::type* B, int64_t ldb, const Out<T> o, lds_char* lds) {
  constexpr int ES = (int)sizeof(cpx<T>);
  constexpr int KC = 24576 / (NCP * ES);                 // B rows staged per chunk (24 KB)
  constexpr int SLOT = 64 * NCP * ES;                    // one group's partial sums for 64 rows
  const int tid = threadIdx.x;
  const int RM = __builtin_amdgcn_readfirstlane(m > 64 ? 128 : 64);
  const int G = kThreads / RM;                           // groups of columns p
  const int S = min(G, 65536 / (SLOT * (RM / 64)));      // partial-sum slots in 64 KB
  const int r = tid % RM, g = tid / RM;                  // g is the same for the whole wave
  const int rc = r < m ? r : 0;
  D3M_LDS cpx<T>* Bs = reinterpret_cast<D3M_LDS cpx<T>*>(lds);
  D3M_LDS cpx<T>* red = Bs + KC * NCP;
  cpx<T> acc[NCP];
#pragma unroll
  for (int j = 0; j < NCP; ++j) acc[j] = mv_zero<T>();
  // the output terms this thread will need (m * nc <= 1024: outputs tid and
  // tid + 512)
  MvPre<T> pre[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int e = tid + h * kThreads < m * nc ? tid + h * kThreads : 0;
    pre[h] = mv_pre(o, e / nc, e - (e / nc) * nc);
  }
  // UN loads per lane go out before their products: with 512 lanes that
  // keeps UN x 8 KB (complex128) in flight per CU.  The first pass's loads
  // of each chunk are issued before B is staged, which then overlaps them.
  constexpr int UN = 16;
  for (int k0 = 0; k0 < k; k0 += KC) {
    const int kc = min(KC, k - k0);
    const typename Cplx<T>::type* Ar = A + rc + (int64_t)k0 * lda;
    cpx<T> a0[UN];
#pragma unroll
    for (int u = 0; u < UN; ++u) {
      const int p = g + u * G;
      a0[u] = *gptr<T>(Ar + (int64_t)(p < kc ? p : 0) * lda);
    }
    for (int e = tid; e < kc * NCP; e += kThreads) {
      const int p = e / NCP, j = e % NCP;
      Bs[e] = j < nc ? *gptr<T>(B + (int64_t)(k0 + p) * ldb + j) : mv_zero<T>();
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < UN; ++u) {
      const int p = g + u * G;
      if (p < kc)
#pragma unroll
        for (int j = 0; j < NCP; ++j) mv_fma(acc[j], a0[u], Bs[p * NCP + j]);
    }
    int p = g + UN * G;
    for (; p + (UN - 1) * G < kc; p += UN * G) {
      cpx<T> a[UN];
#pragma unroll
      for (int u = 0; u < UN; ++u) a[u] = *gptr<T>(Ar + (int64_t)(p + u * G) * lda);
#pragma unroll
      for (int u = 0; u < UN; ++u)
#pragma unroll
        for (int j = 0; j < NCP; ++j) mv_fma(acc[j], a[u], Bs[(p + u * G) * NCP + j]);
    }
    for (; p + 3 * G < kc; p += 4 * G) {
      cpx<T> a[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) a[u] = *gptr<T>(Ar + (int64_t)(p + u * G) * lda);
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int j = 0; j < NCP; ++j) mv_fma(acc[j], a[u], Bs[(p + u * G) * NCP + j]);
    }
    for (; p < kc; p += G) {
      const cpx<T> a = *gptr<T>(Ar + (int64_t)p * lda);
#pragma unroll
      for (int j = 0; j < NCP; ++j) mv_fma(acc[j], a, Bs[p * NCP + j]);
    }
    __syncthreads();
  }
  // partial sums of the G groups: slot s holds groups s, s + S, ... added in
  // that order (rounds separated by barriers)
  for (int q = 0; q < G; q += S) {
    if (g >= q && g < q + S) {
      D3M_LDS cpx<T>* rs = red + ((g - q) * RM + r) * NCP;
#pragma unroll
      for (int j = 0; j < NCP; ++j) {
        if (q == 0) {
          rs[j] = acc[j];
        } else {
          cpx<T> v = rs[j];
          v.x += acc[j].x;
          v.y += acc[j].y;
          rs[j] = v;
        }
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int e = tid + h * kThreads;
    if (e < m * nc) {
      const int i = e / nc, j = e - (e / nc) * nc;
      cpx<T> s = red[i * NCP + j];
      for (int q = 1; q < S; ++q) {
        const cpx<T> v = red[(q * RM + i) * NCP + j];
        s.x += v.x;
        s.y += v.y;
      }
      mv_put(o, i, j, s, pre[h]);
    }
  }
  __syncthreads();
}

// Sum over the 64 lanes of a wave of V values per lane (V a power of two,
// 16..64): each step exchanges half of the values still held with the lane
// d apart and adds, until one value is left, then the remaining steps add
// that value over the other lanes.  Afterwards lane l holds the sum of value
// (l >> (6 - log2 V)).
template <typename T, int V, int D = 32>
__device__ __forceinline__ void mv_wave_reduce(T (&v)[V], int lane) {
  if constexpr (D >= 1) {
    constexpr int LOGV = V >= 64 ? 6 : V >= 32 ? 5 : V >= 16 ? 4 : V >= 8 ? 3 : V >= 4 ? 2 : V >= 2 ? 1 : 0;
    constexpr int LOGD = D >= 32 ? 5 : D >= 16 ? 4 : D >= 8 ? 3 : D >= 4 ? 2 : D >= 2 ? 1 : 0;
    constexpr int CNT = (5 - LOGD) < LOGV ? (V >> (5 - LOGD)) : 1;  // values held before this step
    if constexpr (CNT > 1) {
      constexpr int H = CNT / 2;
      const bool up = (lane & D) != 0;
#pragma unroll
      for (int i = 0; i < H; ++i) {
        const T send = up ? v[i] : v[i + H];
        const T keep = up ? v[i + H] : v[i];
        v[i] = keep + __shfl_xor(send, D, 64);
      }
    } else {
      v[0] += __shfl_xor(v[0], D, 64);
    }
    mv_wave_reduce<T, V, D / 2>(v, lane);
  }
}

// OP_T.
template <typename T, int NCP>
__device__ __noinline__ void mv_t(int m, int nc, int k, const typename Cplx<T>::type* A, int64_t lda,
                                  const typename Cplx<T>::type* B, int64_t ldb, const Out<T> o) {
  // values per lane and batch: 16 for one or two columns (8 or 4 rows per
  // batch, so that every wave has rows), 32 beyond (4 or 2 rows per batch
  // share the loads of B)
  constexpr int V = NCP <= 2 ? 16 : 32;
  constexpr int RG = V / (2 * NCP);               // rows per batch
  constexpr int SH = V >= 64 ? 0 : V >= 32 ? 1 : 2;  // lane >> SH = value index after the reduction
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int nbat = (m + RG - 1) / RG;
  for (int bt = w; bt < nbat; bt += kThreads / 64) {
    const int i0 = bt * RG;
    // the output term of the value this lane will hold after the reduction
    const int idx0 = lane >> SH;
    const int rr0 = (idx0 >> 1) / NCP, j0 = (idx0 >> 1) % NCP;
    const bool mine = (lane & ((1 << SH) - 1)) == 0 && (idx0 & 1) == 0 && i0 + rr0 < m && j0 < nc;
    const MvPre<T> pre = mv_pre(o, mine ? i0 + rr0 : 0, mine ? j0 : 0);
    T v[V];
#pragma unroll
    for (int q = 0; q < V; ++q) v[q] = (T)0;
    // UP passes over p go out together (their loads before any product)
    constexpr int UP = 2;
    for (int p0 = lane; p0 < k; p0 += 64 * UP) {
      cpx<T> b[UP][NCP], a[UP][RG];
#pragma unroll
      for (int u = 0; u < UP; ++u) {
        const int p = p0 + 64 * u;
        const bool pk = p < k;
#pragma unroll
        for (int j = 0; j < NCP; ++j)
          b[u][j] = (pk && j < nc) ? *gptr<T>(B + (int64_t)p * ldb + j) : mv_zero<T>();
#pragma unroll
        for (int rr = 0; rr < RG; ++rr)
          a[u][rr] = (pk && i0 + rr < m) ? *gptr<T>(A + p + (int64_t)(i0 + rr) * lda) : mv_zero<T>();
      }
#pragma unroll
      for (int u = 0; u < UP; ++u)
#pragma unroll
        for (int rr = 0; rr < RG; ++rr)
#pragma unroll
          for (int j = 0; j < NCP; ++j) {
            cpx<T> s;
            s.x = v[(rr * NCP + j) * 2];
            s.y = v[(rr * NCP + j) * 2 + 1];
            mv_fma(s, a[u][rr], b[u][j]);
            v[(rr * NCP + j) * 2] = s.x;
            v[(rr * NCP + j) * 2 + 1] = s.y;
          }
    }
    mv_wave_reduce<T, V>(v, lane);
    const T im = __shfl_xor(v[0], 1 << SH, 64);  // the partner holds value idx0 ^ 1
    if (mine) {
      cpx<T> s;
      s.x = v[0];
      s.y = im;
      mv_put(o, i0 + rr0, j0, s, pre);
    }
  }
}

// Runtime column count to the padded template width.
template <typename T, bool TRANS>
__device__ __forceinline__ void solve_mv(int m, int nc, int k, const typename Cplx<T>::type* A, int64_t lda,
                                         const typename Cplx<T>::type* B, int64_t ldb, const Out<T>& o,
                                         lds_char* lds) {
  if constexpr (TRANS) {
    if (nc <= 1) mv_t<T, 1>(m, nc, k, A, lda, B, ldb, o);
    else if (nc <= 2) mv_t<T, 2>(m, nc, k, A, lda, B, ldb, o);
    else if (nc <= 4) mv_t<T, 4>(m, nc, k, A, lda, B, ldb, o);
    else mv_t<T, 8>(m, nc, k, A, lda, B, ldb, o);
  } else {
    if (nc <= 1) mv_n<T, 1>(m, nc, k, A, lda, B, ldb, o, lds);
    else if (nc <= 2) mv_n<T, 2>(m, nc, k, A, lda, B, ldb, o, lds);
    else if (nc <= 4) mv_n<T, 4>(m, nc, k, A, lda, B, ldb, o, lds);
    else mv_n<T, 8>(m, nc, k, A, lda, B, ldb, o, lds);
  }
}

}  // namespace d3m
