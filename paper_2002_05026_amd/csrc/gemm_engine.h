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

#include <type_traits>

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

// LDS pointers keep their address space through non-inlined task bodies so
// that LDS accesses compile to ds_* instructions (a generic pointer would
// turn them into flat accesses that wait on outstanding global loads).
#define D3M_LDS __attribute__((address_space(3)))
#define D3M_GLB __attribute__((address_space(1)))
typedef D3M_LDS char lds_char;

// Complex pair used for LDS and global accesses inside the engine: a
// builtin 2-vector, which loads and stores in every address space.
template <typename T> using cpx = T __attribute__((ext_vector_type(2)));

template <typename T>
__device__ __forceinline__ const D3M_GLB cpx<T>* gptr(const typename Cplx<T>::type* p) {
  return (const D3M_GLB cpx<T>*)(p);
}
template <typename T>
__device__ __forceinline__ D3M_GLB cpx<T>* gptr_mut(typename Cplx<T>::type* p) {
  return (D3M_GLB cpx<T>*)(p);
}

constexpr int GE_TM = 128;        // output tile rows
constexpr int GE_TN = 128;        // output tile cols
constexpr int GE_LDP = GE_TM + 2; // padded LDS row (complex elements)
constexpr int GE_THREADS = 512;  // 8 waves

// Complex columns per slab: 16 for complex64, 8 for complex128 (keeps the
// FP64 accumulator, prefetch and fragment registers within 256 per wave).
template <typename T> struct GeKB;
template <> struct GeKB<float> { static constexpr int KB = 16, LOG = 4; };
template <> struct GeKB<double> { static constexpr int KB = 8, LOG = 3; };

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
  typename Cplx<T>::type* dst2;             // if non-null: also gets the value before the divisions
  const typename Cplx<T>::type* src;        // beta term (may alias dst), or null
  int64_t srs, scs;
  T alpha, beta;
  const typename Cplx<T>::type* rowdiv;     // divide row i by rowdiv[i], or null
  const typename Cplx<T>::type* coldiv;     // divide column j by coldiv[j], or null
  bool wt = false;                          // store with device-scope atomic stores (write-through)
};

// One output element.  wt: as relaxed device-scope atomic stores of 64
// bits (one for complex64, two for complex128), which write through to
// where every XCD sees them; a task whose stores are all of that kind needs
// no L2 write-back before it releases its successors.
template <typename T>
__device__ __forceinline__ void st_out(D3M_GLB cpx<T>* p, const cpx<T>& v, bool wt) {
  if (wt) {
    if constexpr (sizeof(T) == 4) {
      const uint64_t bits = (uint64_t)__float_as_uint(v.x) | ((uint64_t)__float_as_uint(v.y) << 32);
      __hip_atomic_store((D3M_GLB uint64_t*)p, bits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      D3M_GLB uint64_t* q = (D3M_GLB uint64_t*)p;
      __hip_atomic_store(q, (uint64_t)__double_as_longlong(v.x), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(q + 1, (uint64_t)__double_as_longlong(v.y), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  } else {
    *p = v;
  }
}

// Accumulator of one wave: 8 column blocks of 16x16.  complex128 keeps the
// real and imaginary parts.  complex64 uses three real products per complex
// product (Gauss): P1 = sum ar*br, P2 = sum ai*bi, P3 = sum (ar+ai)(br+bi),
// so re = P1 - P2 and im = P3 - P1 - P2; this takes 3 instead of 4 MFMAs per
// block and k-step.  The parts stay separate until read with acc_val, so
// several gemm_acc calls may add into one accumulator.
//
// TR picks the fragment orientation.  false: item v of column block bj in
// lane (lr, lk) of wave w is C(16w + acc_row(lk, v), 16bj + lr), so a store
// instruction covers 16 consecutive columns (whole lines of a row-major C).
// true: the MFMA operands are swapped (the block is formed as (B A^T)^T,
// the same products summed in the same order), and the item is
// C(16w + lr, 16bj + acc_row(lk, v)): 16 consecutive rows, whole lines of a
// column-major C.
template <typename T, bool TR = false> struct Acc {
  typename V4<T>::type re[8], im[8];
  __device__ __forceinline__ void zero() {
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      re[b] = typename V4<T>::type{0, 0, 0, 0};
      im[b] = typename V4<T>::type{0, 0, 0, 0};
    }
  }
};
template <bool TR> struct Acc<float, TR> {
  v4f p1[8], p2[8], p3[8];
  __device__ __forceinline__ void zero() {
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      p1[b] = v4f{0, 0, 0, 0};
      p2[b] = v4f{0, 0, 0, 0};
      p3[b] = v4f{0, 0, 0, 0};
    }
  }
};

// Complex value of accumulator item v of column block bj.
template <bool TR> __device__ __forceinline__ cpx<double> acc_val(const Acc<double, TR>& a, int bj, int v) {
  cpx<double> r;
  r.x = a.re[bj][v];
  r.y = a.im[bj][v];
  return r;
}
template <bool TR> __device__ __forceinline__ cpx<float> acc_val(const Acc<float, TR>& a, int bj, int v) {
  cpx<float> r;
  const float x = a.p1[bj][v], y = a.p2[bj][v];
  r.x = x - y;
  r.y = a.p3[bj][v] - x - y;
  return r;
}

// c + a b^T on the matrix cores with a's fragment as the A operand (or as
// the B operand when TR)
template <bool TR, typename T, typename V> __device__ __forceinline__ V mfma_or(T a, T b, V c) {
  if constexpr (TR) return mfma16(b, a, c);
  else return mfma16(a, b, c);
}

// LDS bytes the engine needs for slabs of KB columns.
// Two slab buffers (double buffering), each holding the A and B slabs.
template <typename T, int KB = GeKB<T>::KB> constexpr int ge_lds_bytes() {
  return 2 * 2 * KB * GE_LDP * (int)sizeof(typename Cplx<T>::type);
}
constexpr int ge_log2(int v) { return v <= 1 ? 0 : 1 + ge_log2(v / 2); }

// Address of A(i, p) for the operand mode (i, p inside the operand); AM >= 0
// fixes the mode at compile time, AM < 0 takes A.mode.
template <int AM, typename T>
__device__ __forceinline__ const typename Cplx<T>::type* op_addr(const Opnd<T>& A, int i, int p) {
  const int mode = AM >= 0 ? AM : A.mode;
  if (mode == OP_N) return A.p + i + (int64_t)p * A.ld;
  if (mode == OP_T) return A.p + (int64_t)i * A.ld + p;
  const int gi = A.i0 + i;
  return (gi >= p) ? A.p + gi + (int64_t)p * A.ld : A.p + p + (int64_t)gi * A.ld;
}

// Slab registers: raw loads of one slab (columns [p0, p0+KB)) of A (m rows)
// and B (n rows), 4 + 4 complex per thread, plus the D entries of A's
// columns.  Loads are issued unconditionally from clamped addresses (out of
// range elements read the operand's first element) so that they stay in
// flight while the previous slab is multiplied; masking and the D scaling
// happen when the slab is written to LDS.
template <typename T, int KB = GeKB<T>::KB> struct Slab {
  static constexpr int NE = KB * GE_TM / GE_THREADS;  // elements per thread per operand
  cpx<T> a[NE], b[NE], d[NE];
  uint32_t amask, bmask;
};

// SPL: split k (see gemm_acc's SK): slab rows 64..127 of A and B hold rows
// 0..63 of the columns ks later, and a half's columns end at ks (first
// half) or k (second half).
template <typename T, int KB, int AM, bool SPL = false>
__device__ __forceinline__ void ge_fetch(Slab<T, KB>& sl, const Opnd<T>& A, const typename Cplx<T>::type* dA,
                                         const Opnd<T>& B, int m, int n, int k, int p0, int ks = 0) {
  typedef typename Cplx<T>::type C;
  const int tid = threadIdx.x;
  constexpr int NE = Slab<T, KB>::NE, LOG = ge_log2(KB);
  const int amode = AM >= 0 ? AM : A.mode;
  sl.amask = 0;
  sl.bmask = 0;
#pragma unroll
  for (int q = 0; q < NE; ++q) {
    const int e = tid + GE_THREADS * q;
    int i, pp;
    if (amode == OP_T) { pp = e & (KB - 1); i = e >> LOG; }
    else { i = e & (GE_TM - 1); pp = e >> 7; }
    int ia = i, p = p0 + pp, ke = k;
    if constexpr (SPL) {
      const int h = i >> 6;
      ia = i & 63;
      p += h * ks;
      ke = h ? k : ks;
    }
    const bool ok = (ia < m) & (p < ke);
    const C* src = ok ? op_addr<AM>(A, ia, p) : A.p;
    sl.a[q] = *gptr<T>(src);
    if (dA) sl.d[q] = *gptr<T>(dA + (ok ? p : 0));
    sl.amask |= (ok ? 1u : 0u) << q;
  }
#pragma unroll
  for (int q = 0; q < NE; ++q) {
    const int e = tid + GE_THREADS * q;
    int j = e & (GE_TN - 1), p = p0 + (e >> 7), ke = k;
    if constexpr (SPL) {
      const int h = j >> 6;
      j &= 63;
      p += h * ks;
      ke = h ? k : ks;
    }
    const bool ok = (j < n) & (p < ke);
    const C* src = ok ? B.p + j + (int64_t)p * B.ld : B.p;
    sl.b[q] = *gptr<T>(src);
    sl.bmask |= (ok ? 1u : 0u) << q;
  }
}

template <typename T, int KB, int AM>
__device__ __forceinline__ void ge_stash(const Slab<T, KB>& sl, int amode_rt, bool scaled, D3M_LDS cpx<T>* As,
                                         D3M_LDS cpx<T>* Bs) {
  const int tid = threadIdx.x;
  constexpr int NE = Slab<T, KB>::NE, LOG = ge_log2(KB);
  const int amode = AM >= 0 ? AM : amode_rt;
#pragma unroll
  for (int q = 0; q < NE; ++q) {
    const int e = tid + GE_THREADS * q;
    int i, pp;
    if (amode == OP_T) { pp = e & (KB - 1); i = e >> LOG; }
    else { i = e & (GE_TM - 1); pp = e >> 7; }
    cpx<T> v = sl.a[q];
    if (scaled) {
      const cpx<T> d = sl.d[q];
      const T re = v.x * d.x - v.y * d.y;
      v.y = v.x * d.y + v.y * d.x;
      v.x = re;
    }
    if (!((sl.amask >> q) & 1u)) { v.x = 0; v.y = 0; }
    As[pp * GE_LDP + i] = v;
  }
#pragma unroll
  for (int q = 0; q < NE; ++q) {
    const int e = tid + GE_THREADS * q;
    cpx<T> v = sl.b[q];
    if (!((sl.bmask >> q) & 1u)) { v.x = 0; v.y = 0; }
    Bs[(e >> 7) * GE_LDP + (e & (GE_TN - 1))] = v;
  }
}

// One LDS slab into the accumulator: NBJ column blocks (compile time, so the
// fragment reads of a k-step are issued together ahead of its MFMAs), k-steps
// below kend (the slab's columns beyond k hold zeros and are skipped).
template <int NBJ, bool TR>
__device__ __forceinline__ void ge_mma(Acc<double, TR>& acc, const D3M_LDS cpx<double>* ap,
                                       const D3M_LDS cpx<double>* bp, int kend) {
  // one k-step at a time keeps the fragment registers few (the other wave
  // on the SIMD covers the LDS latency)
#pragma unroll 1
  for (int kk = 0; kk < kend; kk += 4) {
    const cpx<double> a0 = ap[kk * GE_LDP];
    cpx<double> b[NBJ];
#pragma unroll
    for (int bj = 0; bj < NBJ; ++bj) b[bj] = bp[kk * GE_LDP + 16 * bj];
    const double nai = -a0.y;
#pragma unroll
    for (int bj = 0; bj < NBJ; ++bj) {
      acc.re[bj] = mfma_or<TR>(a0.x, b[bj].x, acc.re[bj]);
      acc.re[bj] = mfma_or<TR>(nai, b[bj].y, acc.re[bj]);
      acc.im[bj] = mfma_or<TR>(a0.x, b[bj].y, acc.im[bj]);
      acc.im[bj] = mfma_or<TR>(a0.y, b[bj].x, acc.im[bj]);
    }
  }
}
template <int NBJ, bool TR>
__device__ __forceinline__ void ge_mma(Acc<float, TR>& acc, const D3M_LDS cpx<float>* ap,
                                       const D3M_LDS cpx<float>* bp, int kend) {
  if constexpr (NBJ <= 4) {
    // narrow accumulators (tiles of at most 64 columns, e.g. the solve's
    // right-hand sides) mostly run one wave per SIMD, which has no second
    // wave to cover the fragment reads: the reads of the next k-step go out
    // before the products of this one
    if (kend <= 0) return;
    cpx<float> a0 = ap[0], b[NBJ];
#pragma unroll
    for (int bj = 0; bj < NBJ; ++bj) b[bj] = bp[16 * bj];
#pragma unroll 1
    for (int kk = 0; kk < kend; kk += 4) {
      const int kn = kk + 4 < kend ? kk + 4 : kk;  // last step: a harmless re-read
      const cpx<float> a1 = ap[kn * GE_LDP];
      cpx<float> b1[NBJ];
#pragma unroll
      for (int bj = 0; bj < NBJ; ++bj) b1[bj] = bp[kn * GE_LDP + 16 * bj];
      const float as = a0.x + a0.y;
#pragma unroll
      for (int bj = 0; bj < NBJ; ++bj) {
        acc.p1[bj] = mfma_or<TR>(a0.x, b[bj].x, acc.p1[bj]);
        acc.p2[bj] = mfma_or<TR>(a0.y, b[bj].y, acc.p2[bj]);
        acc.p3[bj] = mfma_or<TR>(as, b[bj].x + b[bj].y, acc.p3[bj]);
      }
      a0 = a1;
#pragma unroll
      for (int bj = 0; bj < NBJ; ++bj) b[bj] = b1[bj];
    }
  } else {
#pragma unroll 1
    for (int kk = 0; kk < kend; kk += 4) {
      const cpx<float> a0 = ap[kk * GE_LDP];
      cpx<float> b[NBJ];
#pragma unroll
      for (int bj = 0; bj < NBJ; ++bj) b[bj] = bp[kk * GE_LDP + 16 * bj];
      const float as = a0.x + a0.y;
#pragma unroll
      for (int bj = 0; bj < NBJ; ++bj) {
        acc.p1[bj] = mfma_or<TR>(a0.x, b[bj].x, acc.p1[bj]);
        acc.p2[bj] = mfma_or<TR>(a0.y, b[bj].y, acc.p2[bj]);
        acc.p3[bj] = mfma_or<TR>(as, b[bj].x + b[bj].y, acc.p3[bj]);
      }
    }
  }
}

// ---------------------------------------------------------------- direct loads
// Slab depth and LDS buffers of the direct-load path (no slab registers, so
// the depth is bounded by LDS only).
template <typename T> struct GeDma;
template <> struct GeDma<float> { static constexpr int KB = 16, NBUF = 3; };
template <> struct GeDma<double> { static constexpr int KB = 8, NBUF = 2; };  // path not taken
// LDS bytes of the direct-load path.
template <typename T> constexpr int ge_lds_bytes_dma() {
  return GeDma<T>::NBUF * 2 * GeDma<T>::KB * GE_LDP * (int)sizeof(cpx<T>);
}
// Global->LDS load instructions each wave issues per slab (A and B).
template <typename T, int KB> constexpr int ge_dma_per_wave() {
  return 2 * KB * (GE_TM / (64 * (16 / (int)sizeof(cpx<T>)))) / 8;
}

// Wait until at most N vector-memory operations of this wave are in flight
// and its LDS writes are done (gfx9 s_waitcnt encoding: vmcnt in bits 3:0
// and 15:14, expcnt 6:4 left at its maximum, lgkmcnt 11:8 = 0).
template <int N> __device__ __forceinline__ void ge_wait_vm() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | (7 << 4));
}

// Slab layout of the direct-load path (ge_pipe): a slab of KB columns of A
// and B (both OP_N) goes straight from global memory into an LDS buffer,
// column p of A at p*LDP and of B at (KB + p)*LDP; each wave instruction
// moves 16 bytes per lane, a whole 128-row complex64 column (two rows per
// lane).  Columns at or beyond k are loaded from ge_zero_bytes, so the last
// k-step adds nothing from them.  Rows beyond m (n) read row 0 of the
// operand, or the element after an odd last row (inside the operand's
// allocation): they only reach output rows (columns) beyond the tile, which
// are never stored.
// 1 KB of zeros in device memory: the source of slab columns at or beyond k,
// so that every slab is one uninterrupted series of direct loads (an LDS
// store between them would have to wait for all loads in flight).
static __device__ __attribute__((aligned(256))) unsigned char ge_zero_bytes[1024];

// Wait until at most n (0..8) vector-memory operations of this wave are in
// flight (n known only at run time; the instruction takes an immediate).
__device__ __forceinline__ void ge_wait_vm_n(int n) {
  switch (n) {
    case 0: ge_wait_vm<0>(); break;
    case 1: ge_wait_vm<1>(); break;
    case 2: ge_wait_vm<2>(); break;
    case 3: ge_wait_vm<3>(); break;
    case 4: ge_wait_vm<4>(); break;
    case 5: ge_wait_vm<5>(); break;
    case 6: ge_wait_vm<6>(); break;
    case 7: ge_wait_vm<7>(); break;
    default: ge_wait_vm<8>(); break;
  }
}

// One source of a summed product: A (m x k) and B (n x k), both OP_N.
template <typename T> struct GeSrc {
  const typename Cplx<T>::type* a;
  const typename Cplx<T>::type* b;
  int64_t lda, ldb;
  int k, pad;
};
// Entry q of a source table in LDS, as wave-uniform values (and the store).
template <typename T> __device__ __forceinline__ GeSrc<T> ge_src_lds(const D3M_LDS GeSrc<T>* tab, int q) {
  const D3M_LDS GeSrc<T>& e = tab[q];
  auto u64 = [](uint64_t v) {
    return ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(v >> 32)) << 32) |
           (uint32_t)__builtin_amdgcn_readfirstlane((int)v);
  };
  GeSrc<T> r;
  r.a = reinterpret_cast<const typename Cplx<T>::type*>(u64((uint64_t)(uintptr_t)e.a));
  r.b = reinterpret_cast<const typename Cplx<T>::type*>(u64((uint64_t)(uintptr_t)e.b));
  r.lda = (int64_t)u64((uint64_t)e.lda);
  r.ldb = (int64_t)u64((uint64_t)e.ldb);
  r.k = __builtin_amdgcn_readfirstlane(e.k);
  r.pad = 0;
  return r;
}
template <typename T> __device__ __forceinline__ void ge_src_put(D3M_LDS GeSrc<T>* tab, int q, const GeSrc<T>& e) {
  tab[q].a = e.a;
  tab[q].b = e.b;
  tab[q].lda = e.lda;
  tab[q].ldb = e.ldb;
  tab[q].k = e.k;
  tab[q].pad = 0;
}

// Whether gemm_acc may load A and B directly into LDS: complex64, both
// OP_N, no D scaling, 16-byte aligned columns (even leading dimensions and
// even base offsets).  complex128 keeps the register path: its register
// loads already move 16 bytes per lane, and measured the same or faster.
template <typename T>
__device__ __forceinline__ bool ge_dma_ok(const Opnd<T>& A, const typename Cplx<T>::type* dA, const Opnd<T>& B) {
  if (dA != nullptr || sizeof(cpx<T>) != 8) return false;
  return (((uintptr_t)A.p | (uintptr_t)B.p) & 15) == 0 && ((A.ld | B.ld) & 1) == 0;
}

template <typename T> struct GePre;
template <typename T> struct Out;
template <typename T>
__device__ __forceinline__ void ge_preload(GePre<T>& pre, int m, int n, const Out<T>& o);

// Split k: waves 4..7 formed partial sums over the second k range for the
// same rows as waves 0..3 (column blocks 0..3); they pass them through LDS
// to the first half, which adds them, and clear their own accumulators (so
// that a caller may add further products).  Called right after a barrier
// that ends the products (LDS free); ends with a barrier.
template <typename T, bool TR>
__device__ __forceinline__ void ge_sk_reduce(Acc<T, TR>& acc, lds_char* lds) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if constexpr (sizeof(T) == 4) {
    D3M_LDS v4f* buf = reinterpret_cast<D3M_LDS v4f*>(lds);
    if (w >= 4) {
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        buf[((w - 4) * 12 + b) * 64 + lane] = acc.p1[b];
        buf[((w - 4) * 12 + 4 + b) * 64 + lane] = acc.p2[b];
        buf[((w - 4) * 12 + 8 + b) * 64 + lane] = acc.p3[b];
      }
    }
    __syncthreads();
    if (w < 4) {
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        acc.p1[b] += buf[(w * 12 + b) * 64 + lane];
        acc.p2[b] += buf[(w * 12 + 4 + b) * 64 + lane];
        acc.p3[b] += buf[(w * 12 + 8 + b) * 64 + lane];
      }
    } else {
      acc.zero();
    }
  } else {
    typedef typename V4<T>::type V;
    D3M_LDS V* buf = reinterpret_cast<D3M_LDS V*>(lds);
    if (w >= 4) {
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        buf[((w - 4) * 8 + b) * 64 + lane] = acc.re[b];
        buf[((w - 4) * 8 + 4 + b) * 64 + lane] = acc.im[b];
      }
    }
    __syncthreads();
    if (w < 4) {
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        acc.re[b] += buf[(w * 8 + b) * 64 + lane];
        acc.im[b] += buf[(w * 8 + 4 + b) * 64 + lane];
      }
    } else {
      acc.zero();
    }
  }
  __syncthreads();
}

// acc += sum_q A_q B_q^T over nsrc sources (src(q) gives them, wave-uniform),
// all direct-loadable (ge_dma_ok), as one direct-load pipeline over the slabs
// of all sources: a source boundary costs no refill.  Three LDS buffers:
// slab s is multiplied from buffer s % 3 while slab s + 2 loads into buffer
// (s + 2) % 3; before the barrier that ends step s each wave waits for its
// own loads of slab s + 1, letting exactly the loads it issued for slab s + 2
// stay in flight (a slab partly beyond its source's k issues fewer).
// PRE: the store's beta term goes out at the start of the last slab (the
// last slab is peeled off so that those values are live only there).
// Starts and ends with a barrier.
// W2: a two-block accumulator width too (n in 17..32), for callers whose n
// is the right-hand-side count of a solve (the factor keeps three widths).
// ALLW: one copy of the slab loop per column-block count (n rounded up to
// 16, 1..8), so that a tile with a partial last column block issues the
// products of its own width and not of the next of 1, 4 and 8: the Schur
// updates, where most of the factor's products are, take it.
// SK: split k; the caller has one source with m, n <= 64 and k above one
// slab (see gemm_acc).  FIXW > 0: the accumulator width, fixed by the caller.
template <typename T, int NBMAX, bool PRE, bool TR, bool W2 = false, bool ALLW = false, bool SK = false,
          int FIXW = 0, typename SRC>
__device__ __forceinline__ void ge_pipe(Acc<T, TR>& acc, int m, int n, int nsrc, const SRC& src, lds_char* lds,
                                        GePre<T>* pre, const Out<T>* po) {
  constexpr int KD = GeDma<T>::KB, NB = GeDma<T>::NBUF, SL = 2 * KD * GE_LDP;
  static_assert(NB == 3, "the wait counts assume three buffers");
  D3M_LDS cpx<T>* buf0 = reinterpret_cast<D3M_LDS cpx<T>*>(lds);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  const int nbj = (n + 15) >> 4;
  wg_sync_global();
  int nsl = 0;
  for (int q = 0; q < nsrc; ++q) {
    const int kq = src(q).k;
    if (kq > 0) nsl += (kq + KD - 1) / KD;
  }
  if (m <= 0 || n <= 0 || nsl == 0) return;
  // split k: the first ceil(nsl / 2) slabs go to waves 0..3 (LDS rows and
  // columns 0..63), the rest to waves 4..7 (64..127), one step loading a
  // slab of each half
  static_assert(!(SK && PRE), "split k does not preload the store");
  constexpr bool split = SK;
  const int ks = split ? (nsl + 1) / 2 * KD : 0;
  if (split) nsl = (nsl + 1) / 2;
  const int hw = split ? (w >> 2) : 0;
  const bool rowok = (split ? 16 * (w & 3) : 16 * w) < m;
  // load and compute cursors: source, first column of the slab, operands
  int ql = 0, pl = 0, qc = 0, pc = 0;
  GeSrc<T> el = src(0), ec = el;
  while (el.k <= 0) el = src(++ql);
  qc = ql;
  ec = el;
  // Direct loads of the load cursor's slab (the slab layout above): wave
  // instruction q moves column cq[q] of operand opq[q] (A or B), 16 bytes
  // (two rows) per lane.  The per-lane addresses are formed once per source
  // and advance by a whole slab per slab, so a slab costs one add per load;
  // only a source's last, partial slab selects ge_zero_bytes for columns
  // beyond its k.
  static_assert(sizeof(cpx<T>) == 8 && GE_TM == 128, "complex64, one instruction per column");
  constexpr int NW = ge_dma_per_wave<T, KD>();
  const int wq = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const typename Cplx<T>::type* gp[NW];  // column cq[q] of the current slab, this lane's rows
  int64_t gstep[NW];                      // elements per slab
  auto src_start = [&]() {
#pragma unroll
    for (int q = 0; q < NW; ++q) {
      const int g = wq + 8 * q, op = g / KD, cq = g - op * KD;
      const typename Cplx<T>::type* xp = op ? el.b : el.a;
      const int64_t ld = op ? el.ldb : el.lda;
      int r = split ? 2 * (lane & 31) : 2 * lane;
      if (r >= (op ? n : m)) r = 0;
      gp[q] = xp + r + (int64_t)(cq + (split && lane >= 32 ? ks : 0)) * ld;
      gstep[q] = (int64_t)KD * ld;
    }
  };
  src_start();
  auto issue = [&](int slot) -> int {
    D3M_LDS cpx<T>* bs = buf0 + slot * SL;
    const bool full = pl + KD <= el.k;
#pragma unroll
    for (int q = 0; q < NW; ++q) {
      const int g = wq + 8 * q, op = g / KD, cq = g - op * KD;
      D3M_LDS cpx<T>* dst = bs + (op * KD + cq) * GE_LDP;
      // (split: the first half's slabs are all whole)
      const bool okc = split ? (lane < 32 || ks + pl + cq < el.k) : (full || pl + cq < el.k);
      const void* a = okc ? (const void*)gp[q] : (const void*)(ge_zero_bytes + 16 * lane);
      __builtin_amdgcn_global_load_lds(a, (D3M_LDS void*)dst, 16, 0, 0);
      gp[q] += gstep[q];
    }
    pl += KD;
    if (pl >= (split ? ks : el.k)) {
      pl = 0;
      do { ++ql; if (ql < nsrc) el = src(ql); } while (ql < nsrc && el.k <= 0);
      if (ql < nsrc) src_start();
    }
    return NW;
  };
  auto slab = [&](int s, auto nbjc) {
    if (rowok) {
      const D3M_LDS cpx<T>* cur = buf0 + (s % NB) * SL;
      const D3M_LDS cpx<T>* ap = cur + lk * GE_LDP + 16 * w + lr;
      const D3M_LDS cpx<T>* bp = cur + KD * GE_LDP + lk * GE_LDP + lr + 64 * hw;
      int ke = ec.k - pc < KD ? ec.k - pc : KD;
      if (split && hw) {
        ke = ec.k - ks - pc;
        ke = ke < 0 ? 0 : (ke > KD ? KD : ke);
      }
      const int kend = __builtin_amdgcn_readfirstlane(ke);
      ge_mma<decltype(nbjc)::value>(acc, ap, bp, kend);
    }
    pc += KD;
    if (pc >= ec.k) {
      pc = 0;
      do { ++qc; if (qc < nsrc) ec = src(qc); } while (qc < nsrc && ec.k <= 0);
    }
  };
  issue(0);
  const int c1 = nsl > 1 ? issue(1) : 0;
  ge_wait_vm_n(c1);
  __syncthreads();
  // one copy of the loop per accumulator width (no width switch inside it)
  auto run = [&](auto nbjc) {
    for (int s = 0; s < nsl - (PRE ? 1 : 0); ++s) {
      const int c2 = s + 2 < nsl ? issue((s + 2) % NB) : 0;
      slab(s, nbjc);
      ge_wait_vm_n(c2);
      __syncthreads();
    }
    if constexpr (PRE) {
      if (po->src) ge_preload<T>(*pre, m, n, *po);
      slab(nsl - 1, nbjc);
      ge_wait_vm<0>();
      __syncthreads();
    }
    if constexpr (SK) ge_sk_reduce<T, TR>(acc, lds);
  };
  if constexpr (FIXW > 0) {
    run(std::integral_constant<int, FIXW>());
    return;
  }
  if constexpr (ALLW && NBMAX == 8) {
    switch (nbj) {
      case 1: run(std::integral_constant<int, 1>()); break;
      case 2: run(std::integral_constant<int, 2>()); break;
      case 3: run(std::integral_constant<int, 3>()); break;
      case 4: run(std::integral_constant<int, 4>()); break;
      case 5: run(std::integral_constant<int, 5>()); break;
      case 6: run(std::integral_constant<int, 6>()); break;
      case 7: run(std::integral_constant<int, 7>()); break;
      default: run(std::integral_constant<int, 8>()); break;
    }
    return;
  }
  if (NBMAX > 4 && nbj > 4) run(std::integral_constant<int, (NBMAX > 4 ? 8 : 1)>());
  else if (W2 && NBMAX > 1 && nbj == 2) run(std::integral_constant<int, (NBMAX > 1 ? 2 : 1)>());
  else if (NBMAX > 1 && nbj > 1) run(std::integral_constant<int, (NBMAX > 1 ? 4 : 1)>());
  else run(std::integral_constant<int, 1>());
}

// acc += A * diag(dA) * B^T over k columns.  Starts and ends with a barrier,
// so callers may overwrite the operands (or LDS) right after it returns.
// NBMAX (8, 4 or 1) bounds n by 16 * NBMAX at compile time; callers whose n
// is known to be small pass it so that only the narrow accumulators stay live.
// KB: complex columns per slab (lds holds ge_lds_bytes<T, KB>()); callers
// with registers to spare take deeper slabs, which cover more load latency.
// AM: A's mode fixed at compile time (OP_N or OP_T; -1: A.mode at run time),
// which keeps the per-element address and layout choice out of the slab code.
// DMA: the caller's lds holds ge_lds_bytes_dma<T, KB>() and A is OP_N (AM),
// so that aligned operands may take the direct-load path.
// PRE: on the direct-load path the beta term of the store *po is loaded
// into *pre at the start of the last slab's products, so that its latency
// overlaps them (pre->ok tells the store).  A flag rather than a null test:
// a null test of a pointer to a local keeps the local out of registers.
// W2: see ge_pipe.
// FIXW > 0: the accumulator width is exactly FIXW column blocks (the caller
// picked it from n, 16 (FIXW - 1) < n <= 16 FIXW): a caller that loops over
// several products into one accumulator switches on the width once, outside
// its loop, so that each loop holds a single slab loop.
// SK: split k when m and n are at most 64 (the solve's tiles): such a tile
// keeps only waves 0..3 (one per SIMD) busy and half of each slab's rows
// and columns unused, so waves 4..7 take the second half of the k range in
// those unused LDS rows and columns, and their partial sums are added at
// the end (ge_sk_reduce): two waves per SIMD, and half as many slab steps,
// each loading as many bytes as before.  The sum is formed in two halves.
// The body of gemm_acc; SPL: split k, chosen by gemm_acc (m, n <= 64 and k
// above one slab), fixed at compile time so that each form is its own code
// (with the choice left to run time inside, measured 30% slower).
template <typename T, int NBMAX, int KB, int AM, bool DMA, bool PRE, bool TR, bool W2, bool SPL, int FIXW>
__device__ __forceinline__ void gemm_acc_body(Acc<T, TR>& acc, int m, int n, int k, const Opnd<T>& A,
                                              const typename Cplx<T>::type* dA, const Opnd<T>& B, lds_char* lds,
                                              GePre<T>* pre, const Out<T>* po) {
  D3M_LDS cpx<T>* buf0 = reinterpret_cast<D3M_LDS cpx<T>*>(lds);
  D3M_LDS cpx<T>* buf1 = buf0 + 2 * KB * GE_LDP;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  const int nbj = (n + 15) >> 4;
  // split k (SPL): the first half's columns are [0, ks), a whole number of
  // slabs (or all of k when k fits one slab: the second half is then empty);
  // kl is the loop's extent.  The direct-load path needs k above one slab
  // (its first half's lanes take every column as valid): gemm_acc checks.
  constexpr bool split = SPL;
  const int ks = split ? min(((k + KB - 1) / KB + 1) / 2 * KB, k) : 0;
  const int kl = split ? ks : k;
  const int hw = split ? (w >> 2) : 0;
  const bool rowok = (split ? 16 * (w & 3) : 16 * w) < m;
  // one LDS slab of KBX columns into the accumulator; three widths only
  // (more variants make the allocator copy the accumulator); LDS columns
  // beyond n hold zeros or columns of B that only reach discarded outputs
  // (NBJ is fixed for a whole call, below: one copy of the slab loop per
  // accumulator width, so that the allocator keeps the accumulator in place
  // instead of copying it around a width switch inside the loop)
  auto mma = [&](const D3M_LDS cpx<T>* cur, int p0, auto kbx, auto nbjc) {
    constexpr int KBX = decltype(kbx)::value, NBJ = decltype(nbjc)::value;
    if (!rowok) return;
    const D3M_LDS cpx<T>* ap = cur + lk * GE_LDP + 16 * w + lr;
    const D3M_LDS cpx<T>* bp = cur + KBX * GE_LDP + lk * GE_LDP + lr + 64 * hw;
    int ke = k - p0 < KBX ? k - p0 : KBX;
    if (split) {
      ke = hw ? k - ks - p0 : ks - p0;
      ke = ke < 0 ? 0 : (ke > KBX ? KBX : ke);
    }
    const int kend = __builtin_amdgcn_readfirstlane(ke);
    ge_mma<NBJ>(acc, ap, bp, kend);
  };
  if constexpr (DMA && AM == OP_N && sizeof(cpx<T>) == 8) {
    if (ge_dma_ok<T>(A, dA, B)) {
      auto one = [&](int) {
        GeSrc<T> e;
        e.a = A.p; e.b = B.p; e.lda = A.ld; e.ldb = B.ld; e.k = k; e.pad = 0;
        return e;
      };
      ge_pipe<T, NBMAX, PRE, TR, W2, false, SPL, FIXW>(acc, m, n, 1, one, lds, pre, po);
      return;
    }
  }
  using kbc = std::integral_constant<int, KB>;
  const bool scaled = dA != nullptr;
  wg_sync_global();
  if (k <= 0 || m <= 0 || n <= 0) return;
  auto run = [&](auto nbjc) {
  if constexpr (sizeof(cpx<T>) == 8) {
    // complex64: slab s lives in LDS buffer s & 1; while slab s is
    // multiplied, slab s+1 is written to the other buffer and slab s+3 is
    // loaded into the register slab that held s+1 (sb for even s, sa for odd
    // s): each load has two slabs of products to arrive; one barrier per slab
    Slab<T, KB> sa, sb;
    ge_fetch<T, KB, AM, SPL>(sa, A, dA, B, m, n, k, 0, ks);
    if (KB < kl) ge_fetch<T, KB, AM, SPL>(sb, A, dA, B, m, n, k, KB, ks);
    ge_stash<T, KB, AM>(sa, A.mode, scaled, buf0, buf0 + KB * GE_LDP);
    if (2 * KB < kl) ge_fetch<T, KB, AM, SPL>(sa, A, dA, B, m, n, k, 2 * KB, ks);
    __syncthreads();
    for (int p0 = 0; p0 < kl; p0 += 2 * KB) {
      mma(buf0, p0, kbc(), nbjc);
      if (p0 + KB < kl) {
        ge_stash<T, KB, AM>(sb, A.mode, scaled, buf1, buf1 + KB * GE_LDP);
        if (p0 + 3 * KB < kl) ge_fetch<T, KB, AM, SPL>(sb, A, dA, B, m, n, k, p0 + 3 * KB, ks);
      }
      __syncthreads();
      if (p0 + KB >= kl) break;
      mma(buf1, p0 + KB, kbc(), nbjc);
      if (p0 + 2 * KB < kl) {
        ge_stash<T, KB, AM>(sa, A.mode, scaled, buf0, buf0 + KB * GE_LDP);
        if (p0 + 4 * KB < kl) ge_fetch<T, KB, AM, SPL>(sa, A, dA, B, m, n, k, p0 + 4 * KB, ks);
      }
      __syncthreads();
    }
  } else {
    // complex128 (no registers for a second slab): slab s lives in buffer
    // s & 1; while slab s is multiplied, slab s+1 is written to the other
    // buffer and slab s+2 is loaded into registers; one barrier per slab
    Slab<T, KB> sl;
    ge_fetch<T, KB, AM, SPL>(sl, A, dA, B, m, n, k, 0, ks);
    ge_stash<T, KB, AM>(sl, A.mode, scaled, buf0, buf0 + KB * GE_LDP);
    if (KB < kl) ge_fetch<T, KB, AM, SPL>(sl, A, dA, B, m, n, k, KB, ks);
    __syncthreads();
    int s = 0;
    for (int p0 = 0; p0 < kl; p0 += KB, ++s) {
      D3M_LDS cpx<T>* cur = (s & 1) ? buf1 : buf0;
      D3M_LDS cpx<T>* nxt = (s & 1) ? buf0 : buf1;
      mma(cur, p0, kbc(), nbjc);
      if (p0 + KB < kl) {
        ge_stash<T, KB, AM>(sl, A.mode, scaled, nxt, nxt + KB * GE_LDP);
        if (p0 + 2 * KB < kl) ge_fetch<T, KB, AM, SPL>(sl, A, dA, B, m, n, k, p0 + 2 * KB, ks);
      }
      __syncthreads();
    }
  }
  };
  if constexpr (FIXW > 0) run(std::integral_constant<int, FIXW>());
  else if (NBMAX > 4 && nbj > 4) run(std::integral_constant<int, (NBMAX > 4 ? 8 : 1)>());
  else if (W2 && NBMAX > 1 && nbj == 2) run(std::integral_constant<int, (NBMAX > 1 ? 2 : 1)>());
  else if (NBMAX > 1 && nbj > 1) run(std::integral_constant<int, (NBMAX > 1 ? 4 : 1)>());
  else run(std::integral_constant<int, 1>());
  if constexpr (SPL) ge_sk_reduce<T, TR>(acc, lds);
}

template <typename T, int NBMAX = 8, int KB = GeKB<T>::KB, int AM = -1, bool DMA = false, bool PRE = false,
          bool TR = false, bool W2 = false, bool SK = false, int FIXW = 0>
__device__ __forceinline__ void gemm_acc(Acc<T, TR>& acc, int m, int n, int k, const Opnd<T>& A,
                         const typename Cplx<T>::type* dA, const Opnd<T>& B, lds_char* lds,
                         GePre<T>* pre = nullptr, const Out<T>* po = nullptr) {
  if constexpr (SK && !PRE && FIXW == 0) {
    static_assert(GeDma<T>::KB == KB || sizeof(T) == 8, "one split threshold for both load paths");
    if (m <= 64 && n <= 64 && k > KB) {
      // each accumulator width its own copy too (n <= 64: 4, 2 with W2, 1)
      const int nbj = (n + 15) >> 4;
      if (NBMAX >= 4 && (nbj > 2 || (nbj == 2 && !W2)))
        gemm_acc_body<T, 4, KB, AM, DMA, PRE, TR, W2, true, (NBMAX >= 4 ? 4 : 1)>(acc, m, n, k, A, dA, B, lds, pre, po);
      else if (W2 && NBMAX >= 2 && nbj == 2)
        gemm_acc_body<T, 2, KB, AM, DMA, PRE, TR, W2, true, (NBMAX >= 2 ? 2 : 1)>(acc, m, n, k, A, dA, B, lds, pre, po);
      else
        gemm_acc_body<T, 1, KB, AM, DMA, PRE, TR, W2, true, 1>(acc, m, n, k, A, dA, B, lds, pre, po);
      return;
    }
  }
  gemm_acc_body<T, NBMAX, KB, AM, DMA, PRE, TR, W2, false, FIXW>(acc, m, n, k, A, dA, B, lds, pre, po);
}

template <typename T> __device__ __forceinline__ cpx<T> cpx_div(cpx<T> a, cpx<T> b) {
  const T den = b.x * b.x + b.y * b.y;
  cpx<T> r;
  r.x = (a.x * b.x + a.y * b.y) / den;
  r.y = (a.y * b.x - a.x * b.y) / den;
  return r;
}

// Column blocks whose beta-term loads the store issues before its first
// wait: all 8 for complex64, 4 at a time for complex128 (registers).
template <typename T> struct GeStoreBatch;
template <> struct GeStoreBatch<float> { static constexpr int NB = 8; };
template <> struct GeStoreBatch<double> { static constexpr int NB = 4; };

// The beta term of a TR store, loaded ahead (ge_preload) so that its latency
// overlaps the last slab's products; ok is set once the loads are issued.
template <typename T> struct GePre {
  typename V4<T>::type re[8], im[8];  // laid out like an accumulator
  bool ok;
};
template <typename T>
__device__ __forceinline__ void ge_preload(GePre<T>& pre, int m, int n, const Out<T>& o) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  const int i = 16 * w + lr;
  const int ic = (i < m) ? i : 0;
#pragma unroll
  for (int bj = 0; bj < 8; ++bj)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int j = 16 * bj + acc_row<T>(lk, v);
      const int jc = j < n ? j : 0;
      const cpx<T> c = *gptr<T>(o.src + (int64_t)ic * o.srs + (int64_t)jc * o.scs);
      pre.re[bj][v] = c.x;
      pre.im[bj][v] = c.y;
    }
  pre.ok = true;
}

// Write the accumulator through the store descriptor.  All loads of a batch
// of column blocks (beta term, divisors) are issued first from clamped
// addresses, then the results are formed and stored.  With TR the column
// divisors go through LDS (lds: at least n elements, free after gemm_acc)
// and every wave of the workgroup must call, since that takes a barrier.
template <typename T, bool TR, bool PRE = false>
__device__ __forceinline__ void gemm_store_impl(const Acc<T, TR>& acc, int m, int n, const Out<T>& o, lds_char* lds,
                                                const GePre<T>* pre) {
  constexpr int NBB = GeStoreBatch<T>::NB;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  D3M_GLB cpx<T>* dst = gptr_mut<T>(o.dst);
  if constexpr (TR) {
    D3M_LDS cpx<T>* cds = reinterpret_cast<D3M_LDS cpx<T>*>(lds);
    if (o.coldiv) {
      for (int j = threadIdx.x; j < n; j += kThreads) cds[j] = *gptr<T>(o.coldiv + j);
      __syncthreads();
    }
    if (16 * w >= m) return;
    const int i = 16 * w + lr;
    const bool iok = i < m;
    const int ic = iok ? i : 0;
    cpx<T> rd;
    if (o.rowdiv) rd = *gptr<T>(o.rowdiv + ic);
#pragma unroll
    for (int bt = 0; bt < 8 / NBB; ++bt) {
      if (16 * NBB * bt >= n) break;
      cpx<T> src[NBB][4];
      bool have = false;
      if constexpr (PRE) have = pre->ok;
      if (have) {
#pragma unroll
        for (int b4 = 0; b4 < NBB; ++b4)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            src[b4][v].x = pre->re[NBB * bt + b4][v];
            src[b4][v].y = pre->im[NBB * bt + b4][v];
          }
      } else {
#pragma unroll
        for (int b4 = 0; b4 < NBB; ++b4) {
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int j = 16 * (NBB * bt + b4) + acc_row<T>(lk, v);
            const int jc = j < n ? j : 0;
            if (o.src) src[b4][v] = *gptr<T>(o.src + (int64_t)ic * o.srs + (int64_t)jc * o.scs);
          }
        }
      }
      // all results first, then all stores: a use of a loaded value after a
      // store under a branch would wait for that store too
      cpx<T> res[NBB][4];
#pragma unroll
      for (int b4 = 0; b4 < NBB; ++b4) {
        const int bj = NBB * bt + b4;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int j = 16 * bj + acc_row<T>(lk, v);
          cpx<T> r = acc_val(acc, bj, v);
          r.x *= o.alpha;
          r.y *= o.alpha;
          if (o.src) {
            r.x += o.beta * src[b4][v].x;
            r.y += o.beta * src[b4][v].y;
          }
          if (o.rowdiv) r = cpx_div(r, rd);
          if (o.coldiv) r = cpx_div(r, cds[j < n ? j : 0]);
          asm volatile("" : "+v"(r.x), "+v"(r.y));  // formed here, not sunk into the store branches
          res[b4][v] = r;
        }
      }
#pragma unroll
      for (int b4 = 0; b4 < NBB; ++b4) {
        const int bj = NBB * bt + b4;
        if (16 * bj >= n) break;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int j = 16 * bj + acc_row<T>(lk, v);
          if (iok && j < n) {
            if (o.dst2) {
              // the value before the divisions
              cpx<T> r = acc_val(acc, bj, v);
              r.x *= o.alpha;
              r.y *= o.alpha;
              if (o.src) {
                r.x += o.beta * src[b4][v].x;
                r.y += o.beta * src[b4][v].y;
              }
              gptr_mut<T>(o.dst2)[(int64_t)i * o.rs + (int64_t)j * o.cs] = r;
            }
            dst[(int64_t)i * o.rs + (int64_t)j * o.cs] = res[b4][v];
          }
        }
      }
    }
  } else {
    if (16 * w >= m) return;
    cpx<T> rd[4];
    if (o.rowdiv) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = 16 * w + acc_row<T>(lk, v);
        rd[v] = *gptr<T>(o.rowdiv + (i < m ? i : 0));
      }
    }
#pragma unroll
    for (int bt = 0; bt < 8 / NBB; ++bt) {
      if (16 * NBB * bt >= n) break;
      cpx<T> src[NBB][4], cd[NBB];
#pragma unroll
      for (int b4 = 0; b4 < NBB; ++b4) {
        const int bj = NBB * bt + b4;
        const int j = 16 * bj + lr;
        const int jc = j < n ? j : 0;
        if (o.coldiv) cd[b4] = *gptr<T>(o.coldiv + jc);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int i = 16 * w + acc_row<T>(lk, v);
          const int ic = i < m ? i : 0;
          if (o.src) src[b4][v] = *gptr<T>(o.src + (int64_t)ic * o.srs + (int64_t)jc * o.scs);
        }
      }
      // all results first, then all stores (see the TR branch)
      cpx<T> res[NBB][4];
#pragma unroll
      for (int b4 = 0; b4 < NBB; ++b4) {
        const int bj = NBB * bt + b4;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          cpx<T> r = acc_val(acc, bj, v);
          r.x *= o.alpha;
          r.y *= o.alpha;
          if (o.src) {
            r.x += o.beta * src[b4][v].x;
            r.y += o.beta * src[b4][v].y;
          }
          if (o.rowdiv) r = cpx_div(r, rd[v]);
          if (o.coldiv) r = cpx_div(r, cd[b4]);
          asm volatile("" : "+v"(r.x), "+v"(r.y));
          res[b4][v] = r;
        }
      }
#pragma unroll
      for (int b4 = 0; b4 < NBB; ++b4) {
        const int bj = NBB * bt + b4;
        const int j = 16 * bj + lr;
        if (16 * bj >= n) break;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int i = 16 * w + acc_row<T>(lk, v);
          if (i < m && j < n) {
            if (o.dst2) {
              cpx<T> r = acc_val(acc, bj, v);
              r.x *= o.alpha;
              r.y *= o.alpha;
              if (o.src) {
                r.x += o.beta * src[b4][v].x;
                r.y += o.beta * src[b4][v].y;
              }
              gptr_mut<T>(o.dst2)[(int64_t)i * o.rs + (int64_t)j * o.cs] = r;
            }
            st_out<T>(dst + (int64_t)i * o.rs + (int64_t)j * o.cs, res[b4][v], o.wt);
          }
        }
      }
    }
  }
}

template <typename T, bool TR>
__device__ __forceinline__ void gemm_store(const Acc<T, TR>& acc, int m, int n, const Out<T>& o,
                                           lds_char* lds = nullptr) {
  gemm_store_impl<T, TR, false>(acc, m, n, o, lds, nullptr);
}
// the same with the beta term possibly loaded ahead into pre (TR only)
template <typename T, bool TR>
__device__ __forceinline__ void gemm_store(const Acc<T, TR>& acc, int m, int n, const Out<T>& o, lds_char* lds,
                                           const GePre<T>& pre) {
  gemm_store_impl<T, TR, true>(acc, m, n, o, lds, &pre);
}

}  // namespace d3m
