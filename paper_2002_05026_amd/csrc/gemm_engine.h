// Complex GEMM engine for one 512-thread workgroup on gfx950 (CDNA4).
//
// Every dense operation of the dual step (Sec. II: dense update, dense
// triangular solve through an inverted diagonal tile, block solve updates,
// residual and gradient blocks) reduces to
//     acc(i, j) = sum_p A(i, p) * d(p) * B(j, p),   i < m <= 128, j < n <= 128
// with complex operands (no conjugation) followed by a store
//     out(i, j) = (alpha * acc(i, j) + beta * src(i, j)) / r(i) / c(j).
// The product runs on the matrix cores: 16x16x4 MFMA in FP64 (complex128)
// or FP32 with FP32 accumulation (complex64), four real MFMAs per complex
// block (re*re - im*im, re*im + im*re).  Operand slabs of KB complex columns
// are staged through LDS with a register prefetch of the next slab.
//
// Wave w (of 8) owns output rows [16w, 16w+16) and all (up to 8) 16-column
// blocks.  Blocks outside m x n are skipped wave-uniformly.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace d3m {

template <typename T> struct Cplx;
template <> struct Cplx<double> { typedef double2 type; };
template <> struct Cplx<float> { typedef float2 type; };

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
template <typename T> struct V4;
template <> struct V4<double> { typedef v4d type; };
template <> struct V4<float> { typedef v4f type; };

__device__ __forceinline__ v4d mfma16(double a, double b, v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ v4f mfma16(float a, float b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Row (inside a 16x16 block) of accumulator item v held by a lane of
// 16-lane group lk.  The operand layouts of the two 16x16x4 instructions are
// the same (A(i,k) and B(k,j) in lane i + 16k); their results differ:
// FP32 holds rows 4*lk + v, FP64 holds rows 4*v + lk (measured on gfx950).
template <typename T> __device__ __forceinline__ int acc_row(int lk, int v);
template <> __device__ __forceinline__ int acc_row<float>(int lk, int v) { return 4 * lk + v; }
template <> __device__ __forceinline__ int acc_row<double>(int lk, int v) { return 4 * v + lk; }

template <typename C> __device__ __forceinline__ C cmul(C a, C b) {
  C r;
  r.x = a.x * b.x - a.y * b.y;
  r.y = a.x * b.y + a.y * b.x;
  return r;
}
// a / b computed as a * conj(b) / |b|^2
template <typename C> __device__ __forceinline__ C cdiv(C a, C b) {
  auto den = b.x * b.x + b.y * b.y;
  C r;
  r.x = (a.x * b.x + a.y * b.y) / den;
  r.y = (a.y * b.x - a.x * b.y) / den;
  return r;
}

// Make stores of this workgroup visible to its own later loads, then barrier.
__device__ __forceinline__ void wg_sync_global() {
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
}

constexpr int GE_TM = 128;        // output tile rows
constexpr int GE_TN = 128;        // output tile cols
constexpr int GE_KB = 16;         // complex columns per slab
constexpr int GE_LDP = GE_TM + 2; // padded LDS row (complex elements)
constexpr int GE_THREADS = 512;  // 8 waves

enum OpMode : int { OP_N = 0, OP_T = 1, OP_SYM = 2 };

template <typename T> struct Opnd {
  const typename Cplx<T>::type* p;
  int64_t ld;
  int mode;     // OP_N: X(i,p) = p[i + p*ld]; OP_T: X(i,p) = p[i*ld + p];
                // OP_SYM: symmetric block from its lower triangle, X(i,p) = S(i0+i, p)
  int i0;       // OP_SYM: first row of the tile inside the symmetric block
};

template <typename T> struct Out {
  typename Cplx<T>::type* dst;
  int64_t rs, cs;                           // dst(i,j) = dst[i*rs + j*cs]
  const typename Cplx<T>::type* src;        // beta term (may alias dst), or null
  int64_t srs, scs;
  T alpha, beta;
  const typename Cplx<T>::type* rowdiv;     // divide row i by rowdiv[i], or null
  const typename Cplx<T>::type* coldiv;     // divide column j by coldiv[j], or null
};

template <typename T> struct Acc {
  typename V4<T>::type re[8], im[8];
  __device__ __forceinline__ void zero() {
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      re[b] = typename V4<T>::type{0, 0, 0, 0};
      im[b] = typename V4<T>::type{0, 0, 0, 0};
    }
  }
};

// LDS bytes the engine needs.
template <typename T> constexpr int ge_lds_bytes() {
  return 2 * GE_KB * GE_LDP * (int)sizeof(typename Cplx<T>::type);
}

template <typename T>
__device__ __forceinline__ typename Cplx<T>::type ld_op(const Opnd<T>& A, int i, int p) {
  typedef typename Cplx<T>::type C;
  if (A.mode == OP_N) return A.p[i + (int64_t)p * A.ld];
  if (A.mode == OP_T) return A.p[(int64_t)i * A.ld + p];
  int gi = A.i0 + i;
  C v = (gi >= p) ? A.p[gi + (int64_t)p * A.ld] : A.p[p + (int64_t)gi * A.ld];
  return v;
}

// Load one slab (columns [p0, p0+KB)) of A (m rows) and B (n rows) into
// registers: 4 + 4 complex per thread.
template <typename T>
__device__ __forceinline__ void ge_fetch(typename Cplx<T>::type (&ra)[4], typename Cplx<T>::type (&rb)[4],
                                         const Opnd<T>& A, const typename Cplx<T>::type* dA,
                                         const Opnd<T>& B, int m, int n, int k, int p0) {
  typedef typename Cplx<T>::type C;
  const int tid = threadIdx.x;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    int e = tid + GE_THREADS * q;
    int i, pp;
    if (A.mode == OP_T) { pp = e & (GE_KB - 1); i = e >> 4; }
    else { i = e & (GE_TM - 1); pp = e >> 7; }
    int p = p0 + pp;
    C v;
    v.x = 0; v.y = 0;
    if (i < m && p < k) {
      v = ld_op(A, i, p);
      if (dA) v = cmul(v, dA[p]);
    }
    ra[q] = v;
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    int e = tid + GE_THREADS * q;
    int j = e & (GE_TN - 1), pp = e >> 7;
    int p = p0 + pp;
    C v;
    v.x = 0; v.y = 0;
    if (j < n && p < k) v = B.p[j + (int64_t)p * B.ld];
    rb[q] = v;
  }
}

template <typename T>
__device__ __forceinline__ void ge_stash(const typename Cplx<T>::type (&ra)[4], const typename Cplx<T>::type (&rb)[4],
                                         int amode, typename Cplx<T>::type* As, typename Cplx<T>::type* Bs) {
  const int tid = threadIdx.x;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    int e = tid + GE_THREADS * q;
    int i, pp;
    if (amode == OP_T) { pp = e & (GE_KB - 1); i = e >> 4; }
    else { i = e & (GE_TM - 1); pp = e >> 7; }
    As[pp * GE_LDP + i] = ra[q];
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    int e = tid + GE_THREADS * q;
    Bs[(e >> 7) * GE_LDP + (e & (GE_TN - 1))] = rb[q];
  }
}

// acc += A * diag(dA) * B^T over k columns.  Starts and ends with a barrier,
// so callers may overwrite the operands (or LDS) right after it returns.
template <typename T>
__device__ void gemm_acc(Acc<T>& acc, int m, int n, int k, const Opnd<T>& A,
                         const typename Cplx<T>::type* dA, const Opnd<T>& B, char* lds) {
  typedef typename Cplx<T>::type C;
  C* As = reinterpret_cast<C*>(lds);
  C* Bs = As + GE_KB * GE_LDP;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  const bool rowok = 16 * w < m;
  const int nbj = (n + 15) >> 4;
  C ra[4], rb[4];
  wg_sync_global();
  if (k <= 0 || m <= 0 || n <= 0) return;
  ge_fetch<T>(ra, rb, A, dA, B, m, n, k, 0);
  for (int p0 = 0; p0 < k; p0 += GE_KB) {
    __syncthreads();
    ge_stash<T>(ra, rb, A.mode, As, Bs);
    __syncthreads();
    if (p0 + GE_KB < k) ge_fetch<T>(ra, rb, A, dA, B, m, n, k, p0 + GE_KB);
    if (rowok) {
#pragma unroll
      for (int kk = 0; kk < GE_KB; kk += 4) {
        const C* ap = As + (kk + lk) * GE_LDP + 16 * w + lr;
        const C* bp = Bs + (kk + lk) * GE_LDP + lr;
        const C a0 = ap[0];
        const T nai = -a0.y;
#pragma unroll
        for (int bj = 0; bj < 8; ++bj) {
          if (bj < nbj) {
            const C b = bp[16 * bj];
            acc.re[bj] = mfma16(a0.x, b.x, acc.re[bj]);
            acc.re[bj] = mfma16(nai, b.y, acc.re[bj]);
            acc.im[bj] = mfma16(a0.x, b.y, acc.im[bj]);
            acc.im[bj] = mfma16(a0.y, b.x, acc.im[bj]);
          }
        }
      }
    }
  }
  __syncthreads();
}

// Write the accumulator through the store descriptor.
template <typename T>
__device__ void gemm_store(const Acc<T>& acc, int m, int n, const Out<T>& o) {
  typedef typename Cplx<T>::type C;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  if (16 * w >= m) return;
#pragma unroll
  for (int bj = 0; bj < 8; ++bj) {
    const int j = 16 * bj + lr;
    if (16 * bj >= n) continue;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = 16 * w + acc_row<T>(lk, v);
      if (i < m && j < n) {
        C r;
        r.x = o.alpha * acc.re[bj][v];
        r.y = o.alpha * acc.im[bj][v];
        if (o.src) {
          C s = o.src[(int64_t)i * o.srs + (int64_t)j * o.scs];
          r.x += o.beta * s.x;
          r.y += o.beta * s.y;
        }
        if (o.rowdiv) r = cdiv(r, o.rowdiv[i]);
        if (o.coldiv) r = cdiv(r, o.coldiv[j]);
        o.dst[(int64_t)i * o.rs + (int64_t)j * o.cs] = r;
      }
    }
  }
}

}  // namespace d3m
