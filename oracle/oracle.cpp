// CPU FP64 oracle for the dual factorization and solution step of D3M
// (Sec. II of the paper: "dual factorization and solution", one task per
// nonzero block of the reduced matrix K doing a dense update, a dense
// triangular solve and a dense factorization).
//
// TEST INFRASTRUCTURE ONLY.  This file is the slow, plain reference that the
// GPU library is checked against.  Only the tests, the smoke check and the
// CPU-baseline leg of the benchmark may load it; the GPU library shares no
// code with it and never calls it.
//
// What it computes (the plain definition): X = K^{-1} B for the block-sparse
// complex-symmetric K (K = K^T, no conjugation anywhere), through the block
// factorization P K P^T = L D L^T with L unit lower triangular and D diagonal
// (both at scalar level), no pivoting.  For a fixed elimination order this
// factorization is unique, so L and D are comparable element by element.
//
// Readings where the paper is silent (it prints no formula):
//  * "block LDL^T" is read as scalar unit-lower L and scalar diagonal D; the
//    dense diagonal blocks are themselves LDL^T-factored (Sec. II, "dense
//    factorization" task; the sytrf of the benchmarked BLAS set).
//  * transpose, never conjugate transpose: K is complex symmetric.
//  * nested dissection over the domain grid: split the axis of largest
//    extent (ties to the lowest axis) at lo + ext/2; low half, high half,
//    then the separator interfaces in interface order.
//
// Everything is plain loops over std::complex<double>, no BLAS, no blocking.
// OpenMP only spreads independent rows/columns over threads; every element
// accumulates its terms in the order the definition gives.

#include <algorithm>
#include <array>
#include <cmath>
#include <complex>
#include <cstdint>
#include <cstring>
#include <set>
#include <vector>

typedef std::complex<double> cplx;

namespace {

// ---------------------------------------------------------------- geometry
// Interfaces of an a x b x c domain grid: axis 0 first, then 1, then 2; the
// lower domain's coordinates run x slowest, z fastest.  Interface (ax, d)
// separates domain d from d + e_ax.  (Sec. III: the mesh is split into
// domains; Fig. 1(a): a four-domain cross section.)
struct Iface { int ax, x, y, z; };

std::vector<Iface> enumerate_ifaces(const int32_t g[3]) {
  std::vector<Iface> out;
  for (int ax = 0; ax < 3; ++ax)
    for (int x = 0; x < g[0]; ++x)
      for (int y = 0; y < g[1]; ++y)
        for (int z = 0; z < g[2]; ++z) {
          int d[3] = {x, y, z};
          d[ax] += 1;
          if (d[0] < g[0] && d[1] < g[1] && d[2] < g[2]) out.push_back({ax, x, y, z});
        }
  return out;
}

bool in_box(const int d[3], const int lo[3], const int hi[3]) {
  for (int t = 0; t < 3; ++t)
    if (d[t] < lo[t] || d[t] >= hi[t]) return false;
  return true;
}

// Nested dissection of the box [lo, hi).
void nd_box(const std::vector<Iface>& ifs, const int lo[3], const int hi[3],
            std::vector<int32_t>& out) {
  int ext[3] = {hi[0] - lo[0], hi[1] - lo[1], hi[2] - lo[2]};
  if (ext[0] * ext[1] * ext[2] <= 1) return;
  int ax = 0;
  for (int t = 1; t < 3; ++t)
    if (ext[t] > ext[ax]) ax = t;
  int s = lo[ax] + ext[ax] / 2;
  int lo2[3] = {lo[0], lo[1], lo[2]}, hi1[3] = {hi[0], hi[1], hi[2]};
  hi1[ax] = s;
  lo2[ax] = s;
  nd_box(ifs, lo, hi1, out);
  nd_box(ifs, lo2, hi, out);
  for (size_t i = 0; i < ifs.size(); ++i) {
    const Iface& f = ifs[i];
    if (f.ax != ax) continue;
    int d0[3] = {f.x, f.y, f.z};
    int d1[3] = {f.x, f.y, f.z};
    d1[ax] += 1;
    if (d0[ax] == s - 1 && in_box(d0, lo, hi) && in_box(d1, lo, hi)) out.push_back((int32_t)i);
  }
}

// ---------------------------------------------------------------- the plan
struct Plan {
  int nb = 0;
  std::vector<int32_t> n;         // interface sizes (user numbering)
  std::vector<int64_t> row0;      // first global row of each interface (user numbering)
  std::vector<int32_t> order;     // elimination order pi (user ids)
  std::vector<int32_t> pos;       // pos[I] = position of I in pi
  std::vector<std::vector<int32_t>> S;   // S_I: later neighbours after fill, sorted by pos
  std::vector<std::array<int32_t, 2>> pairs;  // user pairs (I > J)
  std::vector<int64_t> koff;      // offsets of K blocks (complex elements)
  std::set<std::pair<int, int>> orig;  // original pattern edges (min, max)
  // numeric factor: diag blocks (L strictly below, D on the diagonal) and
  // L_JI for J in S_I, column-major n_J x n_I.
  std::vector<std::vector<cplx>> Ld;
  std::vector<std::vector<std::vector<cplx>>> Lo;
  bool factored = false;
  // with in-block pivoting (orc_factor_bk): segment length, and per
  // interface the permutation (internal position -> original index inside
  // the interface) and D's off-diagonal entries (doff[k] = D(k+1, k) when a
  // 2x2 pivot starts at k, else 0)
  int pivot_tile = 0;
  std::vector<std::vector<int32_t>> perm;
  std::vector<std::vector<cplx>> doff;
};

}  // namespace

extern "C" {

int32_t orc_grid_interfaces(const int32_t* grid, int32_t* out) {
  auto f = enumerate_ifaces(grid);
  if (out)
    for (size_t i = 0; i < f.size(); ++i) {
      out[4 * i] = f[i].ax; out[4 * i + 1] = f[i].x; out[4 * i + 2] = f[i].y; out[4 * i + 3] = f[i].z;
    }
  return (int32_t)f.size();
}

// Pairs of interfaces that border a common domain: block (I,J) of K is
// nonzero exactly for these (Fig. 1(b)).  Written as (I, J), I > J, sorted by
// (J, I).
int64_t orc_grid_pairs(const int32_t* grid, int32_t* out) {
  auto f = enumerate_ifaces(grid);
  std::set<std::pair<int, int>> pr;  // (J, I), J < I
  for (size_t i = 0; i < f.size(); ++i)
    for (size_t j = 0; j < i; ++j) {
      int a0[3] = {f[i].x, f[i].y, f[i].z}, a1[3] = {f[i].x, f[i].y, f[i].z};
      int b0[3] = {f[j].x, f[j].y, f[j].z}, b1[3] = {f[j].x, f[j].y, f[j].z};
      a1[f[i].ax] += 1;
      b1[f[j].ax] += 1;
      auto same = [](const int* p, const int* q) { return p[0] == q[0] && p[1] == q[1] && p[2] == q[2]; };
      if (same(a0, b0) || same(a0, b1) || same(a1, b0) || same(a1, b1)) pr.insert({(int)j, (int)i});
    }
  int64_t k = 0;
  for (auto& p : pr) {
    if (out) { out[2 * k] = p.second; out[2 * k + 1] = p.first; }
    ++k;
  }
  return k;
}

int32_t orc_nd_order(const int32_t* grid, int32_t* order) {
  auto f = enumerate_ifaces(grid);
  std::vector<int32_t> o;
  int lo[3] = {0, 0, 0}, hi[3] = {grid[0], grid[1], grid[2]};
  nd_box(f, lo, hi, o);
  for (size_t i = 0; i < o.size(); ++i) order[i] = o[i];
  return (int32_t)o.size();
}

// Block symbolic factorization (the "symbolic simulation" of the sequential
// algorithm, Sec. II): eliminate interfaces in the order pi; the later
// neighbours S_I of the eliminated I become a clique (block fill).
void* orc_plan(int32_t nb, const int32_t* sizes, int64_t npair, const int32_t* pairs,
               const int32_t* order) {
  Plan* p = new Plan;
  p->nb = nb;
  p->n.assign(sizes, sizes + nb);
  p->row0.assign(nb + 1, 0);
  for (int i = 0; i < nb; ++i) p->row0[i + 1] = p->row0[i] + sizes[i];
  p->order.assign(order, order + nb);
  p->pos.assign(nb, -1);
  for (int k = 0; k < nb; ++k) p->pos[order[k]] = k;
  std::vector<std::set<int>> adj(nb);
  p->koff.assign(nb + npair + 1, 0);
  for (int i = 0; i < nb; ++i) p->koff[i + 1] = p->koff[i] + (int64_t)sizes[i] * sizes[i];
  for (int64_t k = 0; k < npair; ++k) {
    int a = pairs[2 * k], b = pairs[2 * k + 1];
    p->pairs.push_back({a, b});
    adj[a].insert(b);
    adj[b].insert(a);
    p->orig.insert({std::min(a, b), std::max(a, b)});
    p->koff[nb + k + 1] = p->koff[nb + k] + (int64_t)sizes[a] * sizes[b];
  }
  p->S.assign(nb, {});
  for (int k = 0; k < nb; ++k) {
    int I = order[k];
    std::vector<int32_t> later;
    for (int J : adj[I])
      if (p->pos[J] > k) later.push_back(J);
    std::sort(later.begin(), later.end(), [&](int a, int b) { return p->pos[a] < p->pos[b]; });
    for (size_t u = 0; u < later.size(); ++u)
      for (size_t v = u + 1; v < later.size(); ++v) {
        adj[later[u]].insert(later[v]);
        adj[later[v]].insert(later[u]);
      }
    p->S[I] = later;
  }
  return p;
}

void orc_plan_free(void* h) { delete (Plan*)h; }

// Counts: [0] N, [1] fill blocks, [2] L off-diagonal blocks, [3] nnz(L)
// (diagonal blocks counted as lower triangles with diagonal), [4] fact tasks,
// [5] TRSM tasks, [6] update tasks, [7] elimination-tree height,
// [8] max |S_I|, [9] max K degree.  flops[0..3]: diagonal LDL^T, TRSM, GEMM
// update, total (8 real flops per complex multiply-add).
void orc_plan_stats(void* h, int64_t* st, double* flops) {
  Plan* p = (Plan*)h;
  int nb = p->nb;
  int64_t nL = 0, nnz = 0, upd = 0;
  int maxS = 0;
  double fd = 0, ft = 0, fu = 0;
  std::vector<int> deg(nb, 0);
  for (auto& e : p->orig) { deg[e.first]++; deg[e.second]++; }
  for (int I = 0; I < nb; ++I) {
    double nI = p->n[I];
    nnz += (int64_t)p->n[I] * (p->n[I] + 1) / 2;
    fd += 4.0 / 3.0 * nI * nI * nI;
    auto& S = p->S[I];
    maxS = std::max(maxS, (int)S.size());
    nL += S.size();
    for (size_t u = 0; u < S.size(); ++u) {
      double nJ = p->n[S[u]];
      nnz += (int64_t)p->n[S[u]] * p->n[I];
      ft += 4.0 * nJ * nI * nI;
      fu += 4.0 * nJ * nJ * nI;
      upd += 1;
      for (size_t v = 0; v < u; ++v) {
        fu += 8.0 * nJ * p->n[S[v]] * nI;
        upd += 1;
      }
    }
  }
  // elimination tree: parent(I) = first element of S_I
  std::vector<int> ht(nb, 1);
  int height = 0;
  for (int k = 0; k < nb; ++k) {
    int I = p->order[k];
    height = std::max(height, ht[I]);
    if (!p->S[I].empty()) {
      int par = p->S[I][0];
      ht[par] = std::max(ht[par], ht[I] + 1);
    }
  }
  st[0] = p->row0[nb];
  st[1] = nL - (int64_t)p->orig.size();
  st[2] = nL;
  st[3] = nnz;
  st[4] = nb;
  st[5] = nL;
  st[6] = upd;
  st[7] = height;
  st[8] = maxS;
  st[9] = *std::max_element(deg.begin(), deg.end());
  flops[0] = fd; flops[1] = ft; flops[2] = fu; flops[3] = fd + ft + fu;
}

int32_t orc_plan_struct(void* h, int32_t I, int32_t* S) {
  Plan* p = (Plan*)h;
  for (size_t u = 0; u < p->S[I].size(); ++u) S[u] = p->S[I][u];
  return (int32_t)p->S[I].size();
}

// Numeric factorization P K P^T = L D L^T (Sec. II, dual factorization:
// for every block column in elimination order a dense factorization of the
// diagonal block, dense triangular solves of the blocks below it and dense
// updates of the blocks to the right).  K is the flat interleaved complex128
// user layout.  Returns -1, or the global row index (user numbering) of the
// first pivot that is zero or not finite.
int64_t orc_factor(void* h, const double* Kd) {
  Plan* p = (Plan*)h;
  const cplx* K = reinterpret_cast<const cplx*>(Kd);
  int nb = p->nb;
  auto& n = p->n;
  p->Ld.assign(nb, {});
  p->Lo.assign(nb, {});
  // index of J inside S_I
  std::vector<std::vector<int>> slot(nb, std::vector<int>());
  for (int I = 0; I < nb; ++I) {
    p->Ld[I].assign((size_t)n[I] * n[I], cplx(0));
    const cplx* src = K + p->koff[I];
    for (int c = 0; c < n[I]; ++c)
      for (int r = c; r < n[I]; ++r) p->Ld[I][r + (size_t)c * n[I]] = src[r + (size_t)c * n[I]];
    p->Lo[I].resize(p->S[I].size());
    for (size_t u = 0; u < p->S[I].size(); ++u)
      p->Lo[I][u].assign((size_t)n[p->S[I][u]] * n[I], cplx(0));  // fill blocks start at 0
  }
  auto find_slot = [&](int I, int J) -> int {
    auto& S = p->S[I];
    for (size_t u = 0; u < S.size(); ++u)
      if (S[u] == J) return (int)u;
    return -1;
  };
  // copy the off-diagonal blocks: block (row = later, col = earlier)
  for (size_t k = 0; k < p->pairs.size(); ++k) {
    int a = p->pairs[k][0], b = p->pairs[k][1];
    const cplx* src = K + p->koff[nb + k];  // n_a x n_b
    if (p->pos[a] > p->pos[b]) {
      auto& dst = p->Lo[b][find_slot(b, a)];  // n_a x n_b
      for (size_t e = 0; e < (size_t)n[a] * n[b]; ++e) dst[e] = src[e];
    } else {
      auto& dst = p->Lo[a][find_slot(a, b)];  // n_b x n_a = transpose
      for (int c = 0; c < n[b]; ++c)
        for (int r = 0; r < n[a]; ++r) dst[c + (size_t)r * n[b]] = src[r + (size_t)c * n[a]];
    }
  }
  for (int k = 0; k < nb; ++k) {
    int I = p->order[k];
    int nI = n[I];
    std::vector<cplx>& A = p->Ld[I];
    // (a) dense LDL^T of the (already updated) diagonal block, no pivoting:
    //     d_j = a_jj - sum_{q<j} l_jq d_q l_jq,
    //     l_ij = (a_ij - sum_{q<j} l_iq d_q l_jq) / d_j.
    for (int j = 0; j < nI; ++j) {
      cplx s = A[j + (size_t)j * nI];
      for (int q = 0; q < j; ++q) s -= A[j + (size_t)q * nI] * A[q + (size_t)q * nI] * A[j + (size_t)q * nI];
      if (s == cplx(0) || !std::isfinite(s.real()) || !std::isfinite(s.imag()))
        return p->row0[I] + j;
      A[j + (size_t)j * nI] = s;
#pragma omp parallel for schedule(static)
      for (int i = j + 1; i < nI; ++i) {
        cplx t = A[i + (size_t)j * nI];
        for (int q = 0; q < j; ++q) t -= A[i + (size_t)q * nI] * A[q + (size_t)q * nI] * A[j + (size_t)q * nI];
        A[i + (size_t)j * nI] = t / s;
      }
    }
    auto& S = p->S[I];
    // (b) W_JI = A_JI L_II^{-T}, then L_JI = W_JI D_I^{-1}; W kept for (c).
    std::vector<std::vector<cplx>> W(S.size());
    for (size_t u = 0; u < S.size(); ++u) {
      int nJ = n[S[u]];
      std::vector<cplx>& Aj = p->Lo[I][u];
      W[u].assign((size_t)nJ * nI, cplx(0));
      std::vector<cplx>& Wu = W[u];
#pragma omp parallel for schedule(static)
      for (int r = 0; r < nJ; ++r) {
        // row r of W solves w L^T = a: w_c = a_c - sum_{q<c} w_q l_cq
        for (int c = 0; c < nI; ++c) {
          cplx t = Aj[r + (size_t)c * nJ];
          for (int q = 0; q < c; ++q) t -= Wu[r + (size_t)q * nJ] * A[c + (size_t)q * nI];
          Wu[r + (size_t)c * nJ] = t;
        }
        for (int c = 0; c < nI; ++c) Aj[r + (size_t)c * nJ] = Wu[r + (size_t)c * nJ] / A[c + (size_t)c * nI];
      }
    }
    // (c) Schur update: A_JK -= W_JI L_KI^T for J, K in S_I, pos(J) >= pos(K);
    //     the lower triangle only when J = K.
    for (size_t u = 0; u < S.size(); ++u) {
      int J = S[u], nJ = n[J];
      for (size_t v = 0; v <= u; ++v) {
        int Kb = S[v], nK = n[Kb];
        const std::vector<cplx>& Wj = W[u];
        const std::vector<cplx>& Lk = p->Lo[I][v];
        cplx* dst;
        if (u == v) dst = p->Ld[J].data();
        else dst = p->Lo[Kb][find_slot(Kb, J)].data();  // block (J, K) lives in column K
        const int ldd = nJ;
#pragma omp parallel for schedule(dynamic, 4)
        for (int c = 0; c < nK; ++c) {
          int r0 = (u == v) ? c : 0;
          for (int q = 0; q < nI; ++q) {
            cplx l = Lk[c + (size_t)q * nK];
            const cplx* w = Wj.data() + (size_t)q * nJ;
            cplx* d = dst + (size_t)c * ldd;
            for (int r = r0; r < nJ; ++r) d[r] -= w[r] * l;
          }
        }
      }
    }
  }
  p->factored = true;
  return -1;
}

// Factor blocks for checking: (J == I) diagonal block of I with L strictly
// below the diagonal and D on it; otherwise L_JI (J in S_I), n_J x n_I
// column-major.  Returns 0, or -1 when the block is not stored.
int32_t orc_get_block(void* h, int32_t J, int32_t I, double* out) {
  Plan* p = (Plan*)h;
  const std::vector<cplx>* src = nullptr;
  if (J == I) src = &p->Ld[I];
  else {
    auto& S = p->S[I];
    for (size_t u = 0; u < S.size(); ++u)
      if (S[u] == J) src = &p->Lo[I][u];
  }
  if (!src) return -1;
  std::memcpy(out, src->data(), src->size() * sizeof(cplx));
  return 0;
}

// Block solve with the factor (Sec. II, dual solution): forward
// y = L^{-1} P b, diagonal z = D^{-1} y, backward x = P^T L^{-T} z.
// B and X hold m right-hand sides, each a contiguous N-vector.
void orc_solve_bk(Plan* p, const double* Bd, double* Xd, int32_t m);

void orc_solve(void* h, const double* Bd, double* Xd, int32_t m) {
  Plan* p = (Plan*)h;
  if (p->pivot_tile > 0) {
    orc_solve_bk(p, Bd, Xd, m);
    return;
  }
  int nb = p->nb;
  auto& n = p->n;
  const int64_t N = p->row0[nb];
  const cplx* B = reinterpret_cast<const cplx*>(Bd);
  cplx* X = reinterpret_cast<cplx*>(Xd);
#pragma omp parallel for schedule(dynamic, 1)
  for (int rhs = 0; rhs < m; ++rhs) {
    std::vector<cplx> b(B + (size_t)rhs * N, B + (size_t)(rhs + 1) * N);
    // forward, in elimination order
    for (int k = 0; k < nb; ++k) {
      int I = p->order[k], nI = n[I];
      cplx* bi = b.data() + p->row0[I];
      const std::vector<cplx>& A = p->Ld[I];
      for (int r = 0; r < nI; ++r)
        for (int q = 0; q < r; ++q) bi[r] -= A[r + (size_t)q * nI] * bi[q];
      for (size_t u = 0; u < p->S[I].size(); ++u) {
        int J = p->S[I][u], nJ = n[J];
        cplx* bj = b.data() + p->row0[J];
        const std::vector<cplx>& L = p->Lo[I][u];
        for (int q = 0; q < nI; ++q)
          for (int r = 0; r < nJ; ++r) bj[r] -= L[r + (size_t)q * nJ] * bi[q];
      }
    }
    // diagonal
    for (int I = 0; I < nb; ++I) {
      cplx* bi = b.data() + p->row0[I];
      for (int r = 0; r < n[I]; ++r) bi[r] /= p->Ld[I][r + (size_t)r * n[I]];
    }
    // backward, in reverse elimination order
    for (int k = nb - 1; k >= 0; --k) {
      int I = p->order[k], nI = n[I];
      cplx* bi = b.data() + p->row0[I];
      for (size_t u = 0; u < p->S[I].size(); ++u) {
        int J = p->S[I][u], nJ = n[J];
        const cplx* xj = b.data() + p->row0[J];
        const std::vector<cplx>& L = p->Lo[I][u];
        for (int q = 0; q < nI; ++q)
          for (int r = 0; r < nJ; ++r) bi[q] -= L[r + (size_t)q * nJ] * xj[r];
      }
      const std::vector<cplx>& A = p->Ld[I];
      for (int r = nI - 1; r >= 0; --r)
        for (int q = r + 1; q < nI; ++q) bi[r] -= A[q + (size_t)r * nI] * bi[q];
    }
    std::memcpy(X + (size_t)rhs * N, b.data(), sizeof(cplx) * N);
  }
}

// Y = K X with the block-sparse K in the user layout (lower triangle of each
// diagonal block read; every stored off-diagonal block applied as K_IJ and
// as K_JI = K_IJ^T).
void orc_matvec(int32_t nb, const int32_t* sizes, int64_t npair, const int32_t* pairs,
                const double* Kd, const double* Xd, double* Yd, int32_t m) {
  std::vector<int64_t> row0(nb + 1, 0), koff(nb + npair + 1, 0);
  for (int i = 0; i < nb; ++i) row0[i + 1] = row0[i] + sizes[i];
  for (int i = 0; i < nb; ++i) koff[i + 1] = koff[i] + (int64_t)sizes[i] * sizes[i];
  for (int64_t k = 0; k < npair; ++k)
    koff[nb + k + 1] = koff[nb + k] + (int64_t)sizes[pairs[2 * k]] * sizes[pairs[2 * k + 1]];
  const int64_t N = row0[nb];
  const cplx* K = reinterpret_cast<const cplx*>(Kd);
  const cplx* X = reinterpret_cast<const cplx*>(Xd);
  cplx* Y = reinterpret_cast<cplx*>(Yd);
#pragma omp parallel for schedule(dynamic, 1)
  for (int rhs = 0; rhs < m; ++rhs) {
    const cplx* x = X + (size_t)rhs * N;
    cplx* y = Y + (size_t)rhs * N;
    for (int64_t i = 0; i < N; ++i) y[i] = 0;
    for (int I = 0; I < nb; ++I) {
      int nI = sizes[I];
      const cplx* A = K + koff[I];
      for (int c = 0; c < nI; ++c)
        for (int r = 0; r < nI; ++r) {
          cplx a = (r >= c) ? A[r + (size_t)c * nI] : A[c + (size_t)r * nI];
          y[row0[I] + r] += a * x[row0[I] + c];
        }
    }
    for (int64_t k = 0; k < npair; ++k) {
      int I = pairs[2 * k], J = pairs[2 * k + 1];
      int nI = sizes[I], nJ = sizes[J];
      const cplx* A = K + koff[nb + k];
      for (int c = 0; c < nJ; ++c)
        for (int r = 0; r < nI; ++r) {
          y[row0[I] + r] += A[r + (size_t)c * nI] * x[row0[J] + c];
          y[row0[J] + c] += A[r + (size_t)c * nI] * x[row0[I] + r];
        }
    }
  }
}

// Gradient of J(K) on K's block pattern for J = sum_k Re(c_k^T x_k), given
// x = K^{-1} b and lambda = K^{-1} c (K = K^T):  dK = -sym(Lambda X^T),
// sym(A) = (A + A^T)/2, summed over right-hand sides, in the K layout.
void orc_grad_K(int32_t nb, const int32_t* sizes, int64_t npair, const int32_t* pairs,
                const double* Ld, const double* Xd, double* dKd, int32_t m) {
  std::vector<int64_t> row0(nb + 1, 0), koff(nb + npair + 1, 0);
  for (int i = 0; i < nb; ++i) row0[i + 1] = row0[i] + sizes[i];
  for (int i = 0; i < nb; ++i) koff[i + 1] = koff[i] + (int64_t)sizes[i] * sizes[i];
  for (int64_t k = 0; k < npair; ++k)
    koff[nb + k + 1] = koff[nb + k] + (int64_t)sizes[pairs[2 * k]] * sizes[pairs[2 * k + 1]];
  const int64_t N = row0[nb];
  const cplx* Lam = reinterpret_cast<const cplx*>(Ld);
  const cplx* X = reinterpret_cast<const cplx*>(Xd);
  cplx* dK = reinterpret_cast<cplx*>(dKd);
  auto block = [&](int I, int J, cplx* out) {  // -1/2 sum_k (lam_I x_J^T + x_I lam_J^T)
    int nI = sizes[I], nJ = sizes[J];
#pragma omp parallel for schedule(static)
    for (int c = 0; c < nJ; ++c)
      for (int r = 0; r < nI; ++r) {
        cplx s = 0;
        for (int k = 0; k < m; ++k)
          s += Lam[k * N + row0[I] + r] * X[k * N + row0[J] + c] + X[k * N + row0[I] + r] * Lam[k * N + row0[J] + c];
        out[r + (size_t)c * nI] = -0.5 * s;
      }
  };
  for (int I = 0; I < nb; ++I) block(I, I, dK + koff[I]);
  for (int64_t k = 0; k < npair; ++k) block(pairs[2 * k], pairs[2 * k + 1], dK + koff[nb + k]);
}

}  // extern "C"

// ---------------------------------------------------------------- in-block pivoting
// The dense factorization named in Sec. II is LAPACK's sytrf: a symmetric
// indefinite LDL^T with Bunch-Kaufman pivoting (1x1 and 2x2 pivots chosen
// by comparing magnitudes, Bunch & Kaufman 1977, alpha = (1 + sqrt(17))/8).
// Here the pivot search is restricted to segments of `tile` consecutive
// unknowns of one interface (the last segment shorter), so the block pattern
// and the elimination order are unchanged.  Per interface I, in elimination
// order, and per segment c of I in order:
//   (i)   Bunch-Kaufman on the segment's diagonal block A_cc, with symmetric
//         interchanges inside the segment (rows of the segment's already
//         computed columns included):  P_c A_cc P_c^T = L_cc D_c L_cc^T;
//   (ii)  every row r below the segment in the block column (later segments
//         of I and the blocks J in S_I) has its columns permuted by P_c, then
//         W_rc = A_rc L_cc^{-T} and L_rc = W_rc D_c^{-1};
//   (iii) the later columns of the block column: A_rs -= W_rc L_sc^T;
// then the Schur update of the later blocks, A_JK -= W_JI L_KI^T with
// W_JI = L_JI D_I.  Rows of a segment in columns left of it keep their
// original order (LAPACK's product form P(1) L(1) P(2) L(2) ...): the solve
// permutes the vector when it reaches the segment.  Magnitudes are compared
// as |re| + |im|, as LAPACK's complex sytrf does.
namespace {

double cabs1(cplx z) { return std::fabs(z.real()) + std::fabs(z.imag()); }

// one interface's block column: the diagonal block A (n x n, lower triangle
// used) and the blocks below it; element (r, c) of block u at blk[u][r + c*rows[u]]
struct Column {
  int n;
  cplx* A;
  std::vector<cplx*> blk;
  std::vector<int> rows;
};

// symmetric interchange of positions a < b inside the segment [t0, t1) of
// the diagonal block, lower storage; only the segment's rows and columns
// (and the columns of the rows below it) move.
void seg_swap(Column& col, int t0, int t1, int a, int b, std::vector<int32_t>& perm) {
  const int n = col.n;
  cplx* A = col.A;
  auto at = [&](int i, int j) -> cplx& { return A[i + (size_t)j * n]; };
  for (int j = t0; j < a; ++j) std::swap(at(a, j), at(b, j));        // computed columns of the segment
  for (int j = a + 1; j < b; ++j) std::swap(at(j, a), at(b, j));     // between a and b
  for (int i = b + 1; i < t1; ++i) std::swap(at(i, a), at(i, b));    // below b inside the segment
  std::swap(at(a, a), at(b, b));
  for (int i = t1; i < n; ++i) std::swap(at(i, a), at(i, b));        // rows below: columns a, b
  for (size_t u = 0; u < col.blk.size(); ++u)
    for (int r = 0; r < col.rows[u]; ++r)
      std::swap(col.blk[u][r + (size_t)a * col.rows[u]], col.blk[u][r + (size_t)b * col.rows[u]]);
  std::swap(perm[a], perm[b]);
}

// Factor one block column with segment-restricted Bunch-Kaufman; returns -1
// or the position (inside the interface) of a pivot column that is zero.
int factor_column_bk(Column& col, int tile, std::vector<int32_t>& perm, std::vector<cplx>& doff) {
  const int n = col.n;
  const double alpha = (1.0 + std::sqrt(17.0)) / 8.0;
  cplx* A = col.A;
  auto at = [&](int i, int j) -> cplx& { return A[i + (size_t)j * n]; };
  perm.resize(n);
  for (int i = 0; i < n; ++i) perm[i] = i;
  doff.assign(n, cplx(0));
  int bad = -1;
  for (int t0 = 0; t0 < n; t0 += tile) {
    const int t1 = std::min(n, t0 + tile);
    // (i) the segment's diagonal block; L_cc overwrites its strict lower part
    std::vector<int> step(t1 - t0, 0);  // 1 or 2 at the first column of a pivot
    int k = t0;
    while (k < t1) {
      const double akk = cabs1(at(k, k));
      int imax = k;
      double colmax = 0;
      for (int i = k + 1; i < t1; ++i)
        if (cabs1(at(i, k)) > colmax) { colmax = cabs1(at(i, k)); imax = i; }
      int kstep = 1, kp = k;
      if (std::max(akk, colmax) == 0.0) {
        if (bad < 0) bad = k;   // a zero column: recorded, factorization goes on
      } else if (akk >= alpha * colmax) {
      } else {
        double rowmax = 0;
        for (int j = k; j < imax; ++j) rowmax = std::max(rowmax, cabs1(at(imax, j)));
        for (int i = imax + 1; i < t1; ++i) rowmax = std::max(rowmax, cabs1(at(i, imax)));
        if (akk >= alpha * colmax * (colmax / rowmax)) {
        } else if (cabs1(at(imax, imax)) >= alpha * rowmax) {
          kp = imax;
        } else {
          kp = imax;
          kstep = 2;
        }
      }
      const int kk = k + kstep - 1;
      if (kp != kk) seg_swap(col, t0, t1, kk, kp, perm);
      step[k - t0] = kstep;
      if (kstep == 1) {
        const cplx d = at(k, k);
        if (d == cplx(0) || !std::isfinite(d.real()) || !std::isfinite(d.imag())) {
          if (bad < 0) bad = k;
          k += 1;
          continue;
        }
        // trailing block of the segment: A_ij -= A_ik A_jk / d, then l_ik = A_ik / d
        for (int j = k + 1; j < t1; ++j)
          for (int i = j; i < t1; ++i) at(i, j) -= at(i, k) * at(j, k) / d;
        for (int i = k + 1; i < t1; ++i) at(i, k) /= d;
      } else {
        // 2x2 pivot [a b; b c]: [l_ik l_i,k+1] = [A_ik A_i,k+1] D^{-1}
        const cplx a = at(k, k), b = at(k + 1, k), c = at(k + 1, k + 1);
        const cplx det = a * c - b * b;
        if (det == cplx(0) || !std::isfinite(det.real()) || !std::isfinite(det.imag())) {
          if (bad < 0) bad = k;
        } else {
          const cplx i11 = c / det, i12 = -b / det, i22 = a / det;
          for (int j = k + 2; j < t1; ++j)
            for (int i = j; i < t1; ++i) {
              const cplx li0 = at(i, k) * i11 + at(i, k + 1) * i12, li1 = at(i, k) * i12 + at(i, k + 1) * i22;
              at(i, j) -= li0 * at(j, k) + li1 * at(j, k + 1);
            }
          for (int i = k + 2; i < t1; ++i) {
            const cplx w0 = at(i, k), w1 = at(i, k + 1);
            at(i, k) = w0 * i11 + w1 * i12;
            at(i, k + 1) = w0 * i12 + w1 * i22;
          }
          doff[k] = b;   // D(k+1, k); L(k+1, k) = 0 (the slot keeps b)
        }
      }
      k += kstep;
    }
    // (ii) rows below the segment: w solves w L_cc^T = a (forward over the
    // segment's columns), then l = w D_c^{-1}; w kept for (iii)
    auto below = [&](cplx* row, int64_t stride, cplx* wout) {
      for (int c2 = t0; c2 < t1; ++c2) {
        cplx t = row[(size_t)c2 * stride];
        for (int q = t0; q < c2; ++q)
          if (!(q + 1 == c2 && step[q - t0] == 2)) t -= wout[q - t0] * at(c2, q);  // (k+1, k) of a 2x2 holds D
        wout[c2 - t0] = t;
      }
      for (int c2 = t0; c2 < t1;) {
        if (step[c2 - t0] == 2) {
          const cplx a = at(c2, c2), b = doff[c2], c = at(c2 + 1, c2 + 1), det = a * c - b * b;
          const cplx w0 = wout[c2 - t0], w1 = wout[c2 + 1 - t0];
          row[(size_t)c2 * stride] = (w0 * c - w1 * b) / det;
          row[(size_t)(c2 + 1) * stride] = (w1 * a - w0 * b) / det;
          c2 += 2;
        } else {
          row[(size_t)c2 * stride] = wout[c2 - t0] / at(c2, c2);
          c2 += 1;
        }
      }
    };
    const int ts = t1 - t0;
    std::vector<cplx> Wd((size_t)(n - t1) * ts);  // rows t1..n of the diagonal block
    std::vector<std::vector<cplx>> Wb(col.blk.size());
#pragma omp parallel for schedule(static)
    for (int i = t1; i < n; ++i) below(&at(i, 0), n, &Wd[(size_t)(i - t1) * ts]);
    for (size_t u = 0; u < col.blk.size(); ++u) {
      Wb[u].resize((size_t)col.rows[u] * ts);
#pragma omp parallel for schedule(static)
      for (int r = 0; r < col.rows[u]; ++r) below(col.blk[u] + r, col.rows[u], &Wb[u][(size_t)r * ts]);
    }
    // (iii) later columns of the block column: A_rs -= W_rc L_sc^T (lower part
    // of the diagonal block, all rows of the blocks below)
#pragma omp parallel for schedule(dynamic, 4)
    for (int j = t1; j < n; ++j) {
      for (int i = j; i < n; ++i) {
        cplx t = 0;
        for (int q = 0; q < ts; ++q) t += Wd[(size_t)(i - t1) * ts + q] * at(j, t0 + q);
        at(i, j) -= t;
      }
      for (size_t u = 0; u < col.blk.size(); ++u)
        for (int r = 0; r < col.rows[u]; ++r) {
          cplx t = 0;
          for (int q = 0; q < ts; ++q) t += Wb[u][(size_t)r * ts + q] * at(j, t0 + q);
          col.blk[u][r + (size_t)j * col.rows[u]] -= t;
        }
    }
  }
  return bad;
}

}  // namespace

extern "C" {

// Numeric factorization with segment-restricted Bunch-Kaufman pivoting (see
// above).  Returns -1, or the global row (user numbering, original index
// inside the interface) of the first zero pivot column.
int64_t orc_factor_bk(void* h, const double* Kd, int32_t tile) {
  Plan* p = (Plan*)h;
  const cplx* K = reinterpret_cast<const cplx*>(Kd);
  const int nb = p->nb;
  auto& n = p->n;
  p->pivot_tile = tile;
  p->perm.assign(nb, {});
  p->doff.assign(nb, {});
  p->Ld.assign(nb, {});
  p->Lo.assign(nb, {});
  for (int I = 0; I < nb; ++I) {
    p->Ld[I].assign((size_t)n[I] * n[I], cplx(0));
    const cplx* src = K + p->koff[I];
    for (int c = 0; c < n[I]; ++c)
      for (int r = c; r < n[I]; ++r) p->Ld[I][r + (size_t)c * n[I]] = src[r + (size_t)c * n[I]];
    p->Lo[I].resize(p->S[I].size());
    for (size_t u = 0; u < p->S[I].size(); ++u) p->Lo[I][u].assign((size_t)n[p->S[I][u]] * n[I], cplx(0));
  }
  auto find_slot = [&](int I, int J) -> int {
    for (size_t u = 0; u < p->S[I].size(); ++u)
      if (p->S[I][u] == J) return (int)u;
    return -1;
  };
  for (size_t k = 0; k < p->pairs.size(); ++k) {
    int a = p->pairs[k][0], b = p->pairs[k][1];
    const cplx* src = K + p->koff[nb + k];
    if (p->pos[a] > p->pos[b]) {
      auto& dst = p->Lo[b][find_slot(b, a)];
      for (size_t e = 0; e < (size_t)n[a] * n[b]; ++e) dst[e] = src[e];
    } else {
      auto& dst = p->Lo[a][find_slot(a, b)];
      for (int c = 0; c < n[b]; ++c)
        for (int r = 0; r < n[a]; ++r) dst[c + (size_t)r * n[b]] = src[r + (size_t)c * n[a]];
    }
  }
  for (int k = 0; k < nb; ++k) {
    const int I = p->order[k], nI = n[I];
    Column col;
    col.n = nI;
    col.A = p->Ld[I].data();
    for (size_t u = 0; u < p->S[I].size(); ++u) {
      col.blk.push_back(p->Lo[I][u].data());
      col.rows.push_back(n[p->S[I][u]]);
    }
    const int bad = factor_column_bk(col, tile, p->perm[I], p->doff[I]);
    if (bad >= 0) return p->row0[I] + p->perm[I][bad];
    // W_JI = L_JI D_I (D block diagonal with 1x1 and 2x2 blocks)
    auto& S = p->S[I];
    const std::vector<cplx>& A = p->Ld[I];
    std::vector<std::vector<cplx>> W(S.size());
    for (size_t u = 0; u < S.size(); ++u) {
      const int nJ = n[S[u]];
      const std::vector<cplx>& Lb = p->Lo[I][u];
      W[u].assign((size_t)nJ * nI, cplx(0));
      for (int c = 0; c < nI; ++c) {
        const cplx dcc = A[c + (size_t)c * nI];
        const cplx lo = c > 0 ? p->doff[I][c - 1] : cplx(0);   // D(c, c-1)
        const cplx hi = c + 1 < nI ? p->doff[I][c] : cplx(0);  // D(c+1, c)
        for (int r = 0; r < nJ; ++r) {
          cplx t = Lb[r + (size_t)c * nJ] * dcc;
          if (lo != cplx(0)) t += Lb[r + (size_t)(c - 1) * nJ] * lo;
          if (hi != cplx(0)) t += Lb[r + (size_t)(c + 1) * nJ] * hi;
          W[u][r + (size_t)c * nJ] = t;
        }
      }
    }
    // Schur update A_JK -= W_JI L_KI^T, J, K in S_I, pos(J) >= pos(K)
    for (size_t u = 0; u < S.size(); ++u) {
      const int J = S[u], nJ = n[J];
      for (size_t v = 0; v <= u; ++v) {
        const int Kb = S[v], nK = n[Kb];
        const std::vector<cplx>& Lk = p->Lo[I][v];
        cplx* dst = (u == v) ? p->Ld[J].data() : p->Lo[Kb][find_slot(Kb, J)].data();
#pragma omp parallel for schedule(dynamic, 4)
        for (int c = 0; c < nK; ++c) {
          const int r0 = (u == v) ? c : 0;
          for (int q = 0; q < nI; ++q) {
            const cplx l = Lk[c + (size_t)q * nK];
            const cplx* w = W[u].data() + (size_t)q * nJ;
            cplx* d = dst + (size_t)c * nJ;
            for (int r = r0; r < nJ; ++r) d[r] -= w[r] * l;
          }
        }
      }
    }
  }
  p->factored = true;
  return -1;
}

// Pivots of interface I after orc_factor_bk: perm (n_I: internal position ->
// original index inside I) and D's off-diagonal entries (n_I complex,
// doff[k] = D(k+1, k) when a 2x2 pivot starts at k).  Returns 0, or -1 when
// the factor has no pivots.
int32_t orc_get_pivots(void* h, int32_t I, int32_t* perm, double* doff) {
  Plan* p = (Plan*)h;
  if (p->pivot_tile <= 0 || I < 0 || I >= p->nb) return -1;
  std::memcpy(perm, p->perm[I].data(), sizeof(int32_t) * p->n[I]);
  std::memcpy(doff, p->doff[I].data(), sizeof(cplx) * p->n[I]);
  return 0;
}

}  // extern "C"

// Solve with the pivoted factor: the segments' permutations are applied to
// the vector when the forward pass reaches a segment and undone when the
// backward pass leaves it (the product form of the factor).
void orc_solve_bk(Plan* p, const double* Bd, double* Xd, int32_t m) {
  const int nb = p->nb;
  auto& n = p->n;
  const int64_t N = p->row0[nb];
  const int tile = p->pivot_tile;
  const cplx* B = reinterpret_cast<const cplx*>(Bd);
  cplx* X = reinterpret_cast<cplx*>(Xd);
#pragma omp parallel for schedule(dynamic, 1)
  for (int rhs = 0; rhs < m; ++rhs) {
    std::vector<cplx> b(B + (size_t)rhs * N, B + (size_t)(rhs + 1) * N);
    // forward: y = L^{-1} (P b), segment by segment
    for (int k = 0; k < nb; ++k) {
      const int I = p->order[k], nI = n[I];
      cplx* bi = b.data() + p->row0[I];
      const std::vector<cplx>& A = p->Ld[I];
      const std::vector<int32_t>& pm = p->perm[I];
      for (int t0 = 0; t0 < nI; t0 += tile) {
        const int t1 = std::min(nI, t0 + tile);
        std::vector<cplx> tmp(bi + t0, bi + t1);
        for (int i = t0; i < t1; ++i) bi[i] = tmp[pm[i] - t0];
        for (int q = t0; q < t1; ++q)
          for (int r = q + 1; r < nI; ++r)
            if (!(r == q + 1 && p->doff[I][q] != cplx(0))) bi[r] -= A[r + (size_t)q * nI] * bi[q];
      }
      for (size_t u = 0; u < p->S[I].size(); ++u) {
        const int J = p->S[I][u], nJ = n[J];
        cplx* bj = b.data() + p->row0[J];
        const std::vector<cplx>& L = p->Lo[I][u];
        for (int q = 0; q < nI; ++q)
          for (int r = 0; r < nJ; ++r) bj[r] -= L[r + (size_t)q * nJ] * bi[q];
      }
    }
    // diagonal: z = D^{-1} y with 1x1 and 2x2 blocks
    for (int I = 0; I < nb; ++I) {
      cplx* bi = b.data() + p->row0[I];
      const std::vector<cplx>& A = p->Ld[I];
      for (int r = 0; r < n[I];) {
        if (p->doff[I][r] != cplx(0)) {
          const cplx a = A[r + (size_t)r * n[I]], bb = p->doff[I][r], c = A[(r + 1) + (size_t)(r + 1) * n[I]];
          const cplx det = a * c - bb * bb, y0 = bi[r], y1 = bi[r + 1];
          bi[r] = (c * y0 - bb * y1) / det;
          bi[r + 1] = (a * y1 - bb * y0) / det;
          r += 2;
        } else {
          bi[r] /= A[r + (size_t)r * n[I]];
          r += 1;
        }
      }
    }
    // backward: x = P^T L^{-T} z, segments in reverse
    for (int k = nb - 1; k >= 0; --k) {
      const int I = p->order[k], nI = n[I];
      cplx* bi = b.data() + p->row0[I];
      for (size_t u = 0; u < p->S[I].size(); ++u) {
        const int J = p->S[I][u], nJ = n[J];
        const cplx* xj = b.data() + p->row0[J];
        const std::vector<cplx>& L = p->Lo[I][u];
        for (int q = 0; q < nI; ++q)
          for (int r = 0; r < nJ; ++r) bi[q] -= L[r + (size_t)q * nJ] * xj[r];
      }
      const std::vector<cplx>& A = p->Ld[I];
      const std::vector<int32_t>& pm = p->perm[I];
      const int nseg = (nI + tile - 1) / tile;
      for (int sgi = nseg - 1; sgi >= 0; --sgi) {
        const int t0 = sgi * tile, t1 = std::min(nI, t0 + tile);
        // later segments are final (original order): t_c -= L_rc^T x_r
        for (int q = t0; q < t1; ++q)
          for (int r = t1; r < nI; ++r) bi[q] -= A[r + (size_t)q * nI] * bi[r];
        for (int q = t1 - 1; q >= t0; --q)
          for (int r = q + 1; r < t1; ++r)
            if (!(r == q + 1 && p->doff[I][q] != cplx(0))) bi[q] -= A[r + (size_t)q * nI] * bi[r];
        std::vector<cplx> tmp(bi + t0, bi + t1);
        for (int i = t0; i < t1; ++i) bi[pm[i]] = tmp[i - t0];
      }
    }
    std::memcpy(X + (size_t)rhs * N, b.data(), sizeof(cplx) * N);
  }
}
