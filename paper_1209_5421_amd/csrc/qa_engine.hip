// Specialised persistent small-level engine (gfx950).
//
// Below a few thousand cells the K-cycle (Algorithm 2.2, with the nonlinear PCG of Algorithm 2.1 as the coarse
// solver of every level) is a chain of dependent steps on small vectors, run by one workgroup. k_engine in
// qa_solve.hip interprets a generic step list against a level table read at run time. This file holds the variant
// for the common shape of those levels, in which every level size, LDS offset and color of a step is a compile-time
// constant:
//  - the coarsest level is the 64-cell level k = 3, one smoothing sweep, two inner steps of Algorithm 2.1;
//  - on the engine's levels no coupling reaches beyond one cell, so no two cells of one color are coupled;
//  - the top level is k = KT (4, 5 or 6); the levels k <= KL keep their operators and vectors in LDS. A top level
//    above them is held in registers: each thread owns TR rows of every color block of it (k = 6 in FP32: 512
//    threads, two rows each; k = 5 in FP64: 256 threads, one row each) and keeps their nine operator entries and
//    their entries of g, e, r and q0 for the whole launch; only p0 and p1, whose neighbours every color phase
//    gathers, are in LDS. The engine then reads global memory once, in its prologue.
// A step on level k runs on the threads j < 4^(k-1): thread j owns row j of each of the four color blocks, so the
// color of every row a thread touches is a compile-time constant and the neighbour indices of Section 4.4 fold to a
// few integer operations; no level table, no loop over a run-time row count. The whole of B~ on the 256-cell level
// k = 4, with the coarsest solve below it, runs in a single wavefront: its sub-steps (one row per lane per color
// block) are ordered by the wavefront's in-order LDS accesses, with no workgroup barrier between them.
//
// The arithmetic of every value is that of the interpreter (same expressions, same order of the nine slot terms);
// only inner products use a different fixed reduction tree.

#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include <algorithm>
#include <mutex>
#include <type_traits>
#include <utility>
#include <vector>

#include "qa_internal.hpp"

namespace qa {

namespace {

constexpr int kFeMaxThreads = 1024;
constexpr int kFeMaxWaves = kFeMaxThreads / 64;
constexpr int kFeMaxOps = 256;
constexpr int kFeCoarse = 64;                 // cells of the coarsest level k = 3
constexpr int kFeAinvBytes = kFeCoarse * kFeCoarse * 8;

enum FeType : int { FE_FIRST2 = 0, FE_GS, FE_RES, FE_PROLONG, FE_SPMV0, FE_SPMV1, FE_UPDATE2, FE_BTILDE_W };
// step word: type | level << 3 | color << 5 | (second B^ of B~) << 7
constexpr int fe_code(int type, int lvl, int color, int b2) { return type | (lvl << 3) | (color << 5) | (b2 << 7); }

// work vectors of a level: Algorithm 2.1's right-hand side g, result e, residual r, directions p0, p1 (the B^
// outputs) and q0 = A p0
enum FeVec : int { V_G = 0, V_E, V_R, V_P0, V_Q0, V_P1, V_COUNT };
// scalars of a level (LDS, written by thread 0 after a reduction). Algorithm 2.1's stop condition (p0, q0) <= 0 is
// tested on d0 = (p0, q0) itself wherever it is needed rather than stored as a flag: the flag's store, a boolean
// materialised under a one-lane branch, was compiled to a select on a stale scalar condition code.
enum FeScalar : int { S_D0 = 0, S_A0, S_BETA, S_A1 };

constexpr int popc(unsigned v) { return v ? static_cast<int>(v & 1u) + popc(v >> 1) : 0; }

// LDS layout of one configuration. Byte 0: the coarsest inverse (64 x 64 FP64). Then, in units of T: for every LDS
// level down to k = 4 its operator (9 x n, slot-major, color-major rows) and its six vectors; the coarsest level's
// g and e; and, for a top level held in registers, its p0 and p1.
template <class T, int KT, int KL>
struct FeLayout {
  static constexpr int lw = KT - 4;            // level index of k = 4 (B~ in one wavefront)
  static constexpr int first_lds = KT - KL;    // first level index in LDS
  __host__ __device__ static constexpr int n(int i) { return 1 << (2 * (KT - i)); }
  __host__ __device__ static constexpr bool lds(int i) { return i >= first_lds; }
  // top level in registers (TR rows of each color block per thread), else 256 threads
  static constexpr bool reg_top = !lds(0);
  static constexpr int TR = (reg_top && n(0) > 1024) ? 2 : 1;
  static constexpr int threads = reg_top ? n(0) / 4 / TR : 256;
  // vectors of a register top level held in LDS: the B^ outputs p0, p1, whose nine neighbours every color phase
  // gathers
  static constexpr unsigned lvec_mask = reg_top ? ((1u << V_P0) | (1u << V_P1)) : 0u;
  __host__ __device__ static constexpr int ax_off(int i) {
    int o = 0;
    for (int j = first_lds; j < i; j++) o += 15 * n(j);
    return o;
  }
  __host__ __device__ static constexpr int vec_off(int i) { return ax_off(i) + 9 * n(i); }
  static constexpr int c3_off = ax_off(lw + 1);
  static constexpr int lvec_off = c3_off + 2 * kFeCoarse;
  static constexpr int t_units = lvec_off + popc(lvec_mask) * n(0);
  static constexpr size_t bytes = kFeAinvBytes + sizeof(T) * static_cast<size_t>(t_units);
};

// registers of a top level: thread t's rows j + c 4^(k-1) (c = 0..3, j = t + i NT for i < TR), their nine operator
// entries (slot order) and their entries of g, e, r, q0
template <class T, int TR>
struct FeTop {
  T a[TR][4][9];
  T v[TR][4][4];
};
__host__ __device__ constexpr int fe_rv(int v) { return v == V_G ? 0 : v == V_E ? 1 : v == V_R ? 2 : 3; }

template <class T>
struct FeArgs {
  int nops;
  const int32_t *ops;
  const double *ainv;        // coarsest inverse, 64 x 64, storage numbering (bitwise symmetric: Y^t Y in one order)
  const T *ax[4];            // 9 x n operator of each engine level (global)
  T *gv[V_COUNT];            // the top level's work vectors in global memory (g and e are read and written there)
};

template <int C>
using IC = std::integral_constant<int, C>;

// the thread index, opaque to the optimiser: row and neighbour indices derived from it are formed inside each step
// rather than hoisted out of the step loop, where they would stay live across the whole launch
__device__ __forceinline__ int fe_tid() {
  int t;
  asm volatile("v_mov_b32 %0, %1" : "=v"(t) : "v"(static_cast<int>(threadIdx.x)));
  return t;
}

// f(j) for the rows j < N4 of a color block, thread j owning j, j + NT, ... (compile-time trip count)
template <int N4, int NT, class F>
__device__ __forceinline__ void for_rows(F f) {
  constexpr int trips = (N4 + NT - 1) / NT;
  const int t0 = fe_tid();
#pragma unroll 1
  for (int it = 0; it < trips; it++) {
    const int j = t0 + it * NT;
    if (N4 % NT == 0 || j < N4) f(j);
  }
}

template <class F>
__device__ __forceinline__ void for_slots(F f) {
  f(IC<0>{}); f(IC<1>{}); f(IC<2>{}); f(IC<3>{}); f(IC<4>{}); f(IC<5>{}); f(IC<6>{}); f(IC<7>{}); f(IC<8>{});
}

template <class F>
__device__ __forceinline__ void for_colors(F f) {
  f(IC<0>{});
  f(IC<1>{});
  f(IC<2>{});
  f(IC<3>{});
}

// (A x)_q for row q = C 4^(k-1) + j of level k (slots in order 0..8; an absent slot holds 0 and its product is taken
// with x[q])
template <class T, int K, int C, class XV>
__device__ __forceinline__ T fe_row(const T *ax, uint32_t j, XV xv) {
  constexpr int sh = 2 * K - 2;
  constexpr uint32_t n = 1u << (2 * K);
  const uint32_t q = (static_cast<uint32_t>(C) << sh) | j;
  uint32_t nb[9];
  stencil_q(q, j, C, sh, nb);
  T acc = 0;
#pragma unroll
  for (int s = 0; s < 9; s++) acc += ax[s * n + q] * xv(nb[s]);
  return acc;
}

// r = g - a0 q0, the first inner update of Algorithm 2.1 (the interpreter's expression)
template <class T>
__device__ __forceinline__ T fe_upd1_r(T g, T a0, T q0) {
  return g - a0 * q0;
}

// a lane's double moved by a DPP lane pattern (two 32-bit moves)
template <int Ctrl>
__device__ __forceinline__ double fe_dpp(double x) {
  const unsigned long long u = __builtin_bit_cast(unsigned long long, x);
  const int lo = __builtin_amdgcn_update_dpp(0, static_cast<int>(u & 0xffffffffu), Ctrl, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, static_cast<int>(u >> 32), Ctrl, 0xf, 0xf, false);
  return __builtin_bit_cast(double, (static_cast<unsigned long long>(static_cast<unsigned>(hi)) << 32) |
                                        static_cast<unsigned>(lo));
}
__device__ __forceinline__ double fe_readlane(double x, int lane) {
  const unsigned long long u = __builtin_bit_cast(unsigned long long, x);
  const unsigned lo = static_cast<unsigned>(__builtin_amdgcn_readlane(static_cast<int>(u & 0xffffffffu), lane));
  const unsigned hi = static_cast<unsigned>(__builtin_amdgcn_readlane(static_cast<int>(u >> 32), lane));
  return __builtin_bit_cast(double, (static_cast<unsigned long long>(hi) << 32) | lo);
}

// sum over one wavefront, the same value in every lane: within each row of 16 lanes a butterfly over DPP lane
// patterns (pairs, quads, half-row mirror, row mirror: every lane of the row ends with the row sum, added in an
// order that gives the same value in each), then the four row sums (R0 + R1) + (R2 + R3) read from lanes 0, 16, 32,
// 48. A fixed tree: the result depends only on the lanes' values.
template <int ND>
__device__ __forceinline__ void fe_wave_allreduce(double (&v)[ND]) {
#pragma unroll
  for (int j = 0; j < ND; j++) {
    double x = v[j];
    x += fe_dpp<0xb1>(x);   // quad_perm [1, 0, 3, 2]
    x += fe_dpp<0x4e>(x);   // quad_perm [2, 3, 0, 1]
    x += fe_dpp<0x141>(x);  // row_half_mirror
    x += fe_dpp<0x140>(x);  // row_mirror
    v[j] = (fe_readlane(x, 0) + fe_readlane(x, 16)) + (fe_readlane(x, 32) + fe_readlane(x, 48));
  }
}

// sum over the first W wavefronts, delivered to thread 0 (fixed tree: each wavefront's sum as above, then the
// wavefront sums in order). Every thread calls it.
template <int ND, int W>
__device__ __forceinline__ void fe_reduce_t0(double (&v)[ND], double *red) {
  if (static_cast<int>(threadIdx.x >> 6) < W) {
    fe_wave_allreduce<ND>(v);
    if (W > 1 && (threadIdx.x & 63) == 0)
#pragma unroll
      for (int j = 0; j < ND; j++) red[j * kFeMaxWaves + (threadIdx.x >> 6)] = v[j];
  }
  if constexpr (W > 1) {
    __syncthreads();
    if (threadIdx.x == 0)
#pragma unroll
      for (int j = 0; j < ND; j++) {
        double acc = 0.0;
#pragma unroll
        for (int w = 0; w < W; w++) acc += red[j * kFeMaxWaves + w];
        v[j] = acc;
      }
  }
}

// Order between the sub-steps of the one-wavefront B~: a wavefront's LDS accesses are performed in issue order, so
// keeping the compiler from moving memory accesses across this point is all that is needed.
__device__ __forceinline__ void fe_wsync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  asm volatile("" ::: "memory");
}

template <class T, int KT, int KL>
struct FeEngine {
  using Lay = FeLayout<T, KT, KL>;
  static constexpr int lw = Lay::lw;
  static constexpr int NT = Lay::threads;
  static constexpr int TR = Lay::TR;

  T *S;                 // T arrays in LDS
  const double *Ainv;   // LDS
  const FeArgs<T> &A;
  double (*sc)[8];
  double *red;
  FeTop<T, TR> &R;      // the top level's registers (unused unless Lay::reg_top)

  template <int I>
  static constexpr bool reg() {
    return Lay::reg_top && I == 0;
  }

  template <int I, int V>
  __device__ __forceinline__ T *vec() const {
    static_assert(!reg<I>() || V == V_P0 || V == V_P1, "register vector of the top level");
    if constexpr (Lay::lds(I)) {
      return S + Lay::vec_off(I) + V * Lay::n(I);
    } else if constexpr ((Lay::lvec_mask >> V) & 1u) {
      return S + Lay::lvec_off + popc(Lay::lvec_mask & ((1u << V) - 1u)) * Lay::n(I);
    } else {
      return A.gv[V];
    }
  }
  template <int I>
  __device__ __forceinline__ const T *ax() const {
    if constexpr (Lay::lds(I)) return S + Lay::ax_off(I);
    else return A.ax[I];
  }

  // f(j, t) for the rows j < 4^(k-1) of a color block of level I: on the register top level the thread's TR rows
  // (t = IC<i> for the i-th, unrolled), elsewhere a loop with t = IC<0>
  template <int I, class F>
  __device__ __forceinline__ void rows(F f) const {
    if constexpr (reg<I>()) {
      const int t = fe_tid();
      f(t, IC<0>{});
      if constexpr (TR > 1) f(t + NT, IC<1>{});
    } else {
      for_rows<Lay::n(I) / 4, NT>([&](int j) { f(j, IC<0>{}); });
    }
  }

  // entry V of row C 4^(k-1) + j of level I (a register of the top level, else LDS or global memory)
  template <int I, int V, int C, int Tr>
  __device__ __forceinline__ T &own(int j, IC<Tr>) const {
    if constexpr (reg<I>() && V != V_P0 && V != V_P1) return R.v[Tr][fe_rv(V)][C];
    else return vec<I, V>()[C * (Lay::n(I) / 4) + j];
  }
  // operator entry in slot Sl of that row
  template <int I, int C, int Sl, int Tr>
  __device__ __forceinline__ T aop(int j, IC<Tr>) const {
    if constexpr (reg<I>()) return R.a[Tr][C][Sl];
    else return ax<I>()[Sl * Lay::n(I) + C * (Lay::n(I) / 4) + j];
  }

  // (A x)_q for row q = C 4^(k-1) + j of level I (slots in order 0..8; an absent slot holds 0 and its product is
  // taken with x[q])
  template <int I, int C, int Tr, class XV>
  __device__ __forceinline__ T row(int j, IC<Tr> tr, XV xv) const {
    constexpr int K = KT - I, sh = 2 * K - 2;
    const uint32_t ju = static_cast<uint32_t>(j);
    const uint32_t q = (static_cast<uint32_t>(C) << sh) | ju;
    uint32_t nb[9];
    stencil_q(q, ju, C, sh, nb);
    T acc = 0;
    for_slots([&](auto ss) {
      constexpr int sl = decltype(ss)::value;
      acc += aop<I, C, sl>(j, tr) * xv(nb[sl]);
    });
    return acc;
  }

  // ---- steps on a level run by the workgroup (k >= 5) ----

  // the first two color phases of B^ from zero: color 0 takes f / diag, the color-1 rows read those values (their
  // color-0 neighbours are E and W; every other neighbour is still 0), colors 2 and 3 are 0. For the second B^ of B~
  // the right-hand side is r = g - a0 q0, and e = a0 p0 and r are stored here. On an LDS level the color-1 rows form
  // their neighbours' values on the fly (one step); on a register top level the color-0 values go through LDS first.
  template <int I, int B2>
  __device__ __forceinline__ void first2() const {
    constexpr int K = KT - I, N = Lay::n(I), N4 = N / 4, SH = 2 * K - 2;
    T *u = vec<I, B2 ? V_P1 : V_P0>();
    const T *p0 = vec<I, V_P0>();
    const T a0 = B2 ? static_cast<T>(sc[I][S_A0]) : T(0);
    if constexpr (reg<I>()) {
      auto fo = [&](auto cc, auto tr) -> T {
        constexpr int c = decltype(cc)::value, t = decltype(tr)::value;
        if constexpr (B2) return fe_upd1_r(R.v[t][0][c], a0, R.v[t][3][c]);
        else return R.v[t][0][c];
      };
      rows<I>([&](int j, auto tr) {
        constexpr int t = decltype(tr)::value;
        u[j] = fo(IC<0>{}, tr) / R.a[t][0][0];
        u[2 * N4 + j] = T(0);
        u[3 * N4 + j] = T(0);
        if constexpr (B2) {
          for_colors([&](auto cc) {
            constexpr int c = decltype(cc)::value;
            R.v[t][1][c] = a0 * p0[c * N4 + j];
            R.v[t][2][c] = fe_upd1_r(R.v[t][0][c], a0, R.v[t][3][c]);
          });
        }
      });
      __syncthreads();
      rows<I>([&](int j, auto tr) {
        constexpr int t = decltype(tr)::value;
        const uint32_t q1 = static_cast<uint32_t>(N4 + j);
        uint32_t nb[9];
        stencil_q(q1, static_cast<uint32_t>(j), 1, SH, nb);
        auto first = [=](uint32_t i) -> T { return i < static_cast<uint32_t>(N4) ? u[i] : T(0); };
        T acc = R.a[t][1][1] * first(nb[1]);
        acc += R.a[t][1][5] * first(nb[5]);
        u[q1] = T(0) + (fo(IC<1>{}, tr) - acc) / R.a[t][1][0];
      });
    } else {
      const T *a = ax<I>();
      const T *g = vec<I, V_G>(), *q0 = vec<I, V_Q0>();
      T *e = vec<I, V_E>(), *r = vec<I, V_R>();
      auto fv = [=](uint32_t i) -> T {
        if constexpr (B2) return fe_upd1_r(g[i], a0, q0[i]);
        else return g[i];
      };
      for_rows<N4, NT>([&](int j) {
        const uint32_t q1 = static_cast<uint32_t>(N4 + j);
        uint32_t nb[9];
        stencil_q(q1, static_cast<uint32_t>(j), 1, SH, nb);
        auto first = [=](uint32_t i) -> T { return i < static_cast<uint32_t>(N4) ? fv(i) / a[i] : T(0); };
        T acc = a[1 * N + q1] * first(nb[1]);
        acc += a[5 * N + q1] * first(nb[5]);
        const T u1 = T(0) + (fv(q1) - acc) / a[q1];
        u[j] = fv(static_cast<uint32_t>(j)) / a[j];
        u[q1] = u1;
        u[2 * N4 + j] = T(0);
        u[3 * N4 + j] = T(0);
        if constexpr (B2) {
          for_colors([&](auto cc) {
            constexpr int c = decltype(cc)::value;
            const int q = c * N4 + j;
            e[q] = a0 * p0[q];
            r[q] = fe_upd1_r(g[q], a0, q0[q]);
          });
        }
      });
    }
  }

  // one color phase of the pointwise Gauss-Seidel (Section 4.5): x += (f - A x) / diag on the rows of color C; for
  // the second B^'s last phase also beta = -(p1, q0) / d0 of Algorithm 2.1
  template <int I, int C, int B2>
  __device__ __forceinline__ void gs() const {
    constexpr int N4 = Lay::n(I) / 4;
    T *u = vec<I, B2 ? V_P1 : V_P0>();
    rows<I>([&](int j, auto tr) {
      const T f = own<I, B2 ? V_R : V_G, C>(j, tr);
      const T dl = (f - row<I, C>(j, tr, [u](uint32_t i) { return u[i]; })) / aop<I, C, 0>(j, tr);
      u[C * N4 + j] += dl;
    });
    if constexpr (B2 && C == 0) {
      __syncthreads();
      dot_beta<I>();
    }
  }

  template <int I>
  __device__ __forceinline__ void dot_beta() const {
    constexpr int N4 = Lay::n(I) / 4;
    const T *p1 = vec<I, V_P1>();
    double t[1] = {0.0};
    rows<I>([&](int j, auto tr) {
      for_colors([&](auto cc) {
        constexpr int c = decltype(cc)::value;
        t[0] += static_cast<double>(p1[c * N4 + j]) * static_cast<double>(own<I, V_Q0, c>(j, tr));
      });
    });
    fe_reduce_t0<1, (N4 < NT ? N4 : NT) / 64>(t, red);
    if (threadIdx.x == 0) {
      const double d0 = sc[I][S_D0];
      sc[I][S_BETA] = (d0 > 0.0) ? -t[0] / d0 : 0.0;
    }
  }

  // residual f - A u of the four children of each parent cell, summed in the order 0, 1, 3, 2 (Section 4.3's
  // explicit restriction) into the parent's g
  template <int I, int B2>
  __device__ __forceinline__ void res_restrict() const {
    constexpr int K = KT - I;
    constexpr int F = B2 ? V_R : V_G;
    const T *u = vec<I, B2 ? V_P1 : V_P0>();
    T *gc = vec<I + 1, V_G>();
    auto uv = [u](uint32_t i) { return u[i]; };
    rows<I>([&](int m, auto tr) {
      const T r0 = own<I, F, 0>(m, tr) - row<I, 0>(m, tr, uv);
      const T r1 = own<I, F, 1>(m, tr) - row<I, 1>(m, tr, uv);
      const T r3 = own<I, F, 3>(m, tr) - row<I, 3>(m, tr, uv);
      const T r2 = own<I, F, 2>(m, tr) - row<I, 2>(m, tr, uv);
      T acc = 0;
      acc += r0;
      acc += r1;
      acc += r3;
      acc += r2;
      gc[q_of_m(static_cast<uint32_t>(m), K - 1)] = acc;
    });
  }

  // u += P e_c; when the child's B~ ran as steps, its last update e_c + a1 (p1 + beta p0) is formed here
  template <int I, int B2>
  __device__ __forceinline__ void prolong() const {
    constexpr int K = KT - I, N4 = Lay::n(I) / 4;
    constexpr bool defer = (K - 1) >= 5;
    T *u = vec<I, B2 ? V_P1 : V_P0>();
    const T *ec = vec<I + 1, V_E>();
    const T *p1c = vec<I + 1, V_P1>(), *p0c = vec<I + 1, V_P0>();
    const T a1 = defer ? static_cast<T>(sc[I + 1][S_A1]) : T(0);
    const T beta = defer ? static_cast<T>(sc[I + 1][S_BETA]) : T(0);
    rows<I>([&](int j, auto) {
      const uint32_t m = q_of_m(static_cast<uint32_t>(j), K - 1);
      T ecm = ec[m];
      if constexpr (defer) ecm = ec[m] + a1 * (p1c[m] + beta * p0c[m]);
      for_colors([&](auto cc) {
        constexpr int c = decltype(cc)::value;
        u[c * N4 + j] += ecm;
      });
    });
  }

  // q0 = A p0 with (p0, q0) and (g, p0); alpha0 of Algorithm 2.1
  template <int I>
  __device__ __forceinline__ void spmv0() const {
    constexpr int N4 = Lay::n(I) / 4;
    const T *x = vec<I, V_P0>();
    double v[2] = {0.0, 0.0};
    rows<I>([&](int j, auto tr) {
      for_colors([&](auto cc) {
        constexpr int c = decltype(cc)::value;
        const int q = c * N4 + j;
        const T yq = row<I, c>(j, tr, [x](uint32_t i) { return x[i]; });
        own<I, V_Q0, c>(j, tr) = yq;
        v[0] += static_cast<double>(x[q]) * static_cast<double>(yq);
        v[1] += static_cast<double>(own<I, V_G, c>(j, tr)) * static_cast<double>(x[q]);
      });
    });
    fe_reduce_t0<2, (N4 < NT ? N4 : NT) / 64>(v, red);
    if (threadIdx.x == 0) {
      sc[I][S_D0] = v[0];
      sc[I][S_A0] = (v[0] > 0.0) ? v[1] / v[0] : 0.0;
    }
  }

  // A d for the direction d = p1 + beta p0 formed on the fly, with (d, A d) and (r, d); alpha1
  template <int I>
  __device__ __forceinline__ void spmv1() const {
    constexpr int N4 = Lay::n(I) / 4;
    const T beta = static_cast<T>(sc[I][S_BETA]);
    const T *p1 = vec<I, V_P1>(), *p0 = vec<I, V_P0>();
    auto dir = [p1, p0, beta](uint32_t i) { return p1[i] + beta * p0[i]; };
    double v[2] = {0.0, 0.0};
    rows<I>([&](int j, auto tr) {
      for_colors([&](auto cc) {
        constexpr int c = decltype(cc)::value;
        const uint32_t q = static_cast<uint32_t>(c * N4 + j);
        const T yq = row<I, c>(j, tr, dir);
        const T xq = dir(q);
        v[0] += static_cast<double>(xq) * static_cast<double>(yq);
        v[1] += static_cast<double>(own<I, V_R, c>(j, tr)) * static_cast<double>(xq);
      });
    });
    fe_reduce_t0<2, (N4 < NT ? N4 : NT) / 64>(v, red);
    if (threadIdx.x == 0) sc[I][S_A1] = (sc[I][S_D0] > 0.0 && v[0] > 0.0) ? v[1] / v[0] : 0.0;
  }

  // e += a1 (p1 + beta p0)
  template <int I>
  __device__ __forceinline__ void update2() const {
    constexpr int N4 = Lay::n(I) / 4;
    const T a1 = static_cast<T>(sc[I][S_A1]), beta = static_cast<T>(sc[I][S_BETA]);
    const T *p1 = vec<I, V_P1>(), *p0 = vec<I, V_P0>();
    rows<I>([&](int j, auto tr) {
      for_colors([&](auto cc) {
        constexpr int c = decltype(cc)::value;
        const int q = c * N4 + j;
        own<I, V_E, c>(j, tr) += a1 * (p1[q] + beta * p0[q]);
      });
    });
  }

  // ---- B~ on level k = 4 (256 cells) in one wavefront: lane j owns row j of each color block ----

  template <int B2>
  __device__ __forceinline__ void bhat_w(T a0) const {
    constexpr int I = lw, N = 256, N4 = 64, SH = 6;
    const T *a = ax<I>();
    const T *g = vec<I, V_G>(), *q0 = vec<I, V_Q0>(), *p0 = vec<I, V_P0>();
    T *e = vec<I, V_E>(), *r = vec<I, V_R>();
    T *u = vec<I, B2 ? V_P1 : V_P0>();
    const T *f = B2 ? r : g;
    T *g3 = S + Lay::c3_off, *e3 = g3 + kFeCoarse;
    const int j = static_cast<int>(threadIdx.x);
    const uint32_t ju = static_cast<uint32_t>(j);
    auto uv = [u](uint32_t i) { return u[i]; };
    auto fv = [=](uint32_t i) -> T {
      if constexpr (B2) return fe_upd1_r(g[i], a0, q0[i]);
      else return g[i];
    };
    {  // first two phases from zero (and, for the second B^, the first inner update)
      const uint32_t q1 = static_cast<uint32_t>(N4 + j);
      uint32_t nb[9];
      stencil_q(q1, ju, 1, SH, nb);
      auto first = [=](uint32_t i) -> T { return i < static_cast<uint32_t>(N4) ? fv(i) / a[i] : T(0); };
      T acc = a[1 * N + q1] * first(nb[1]);
      acc += a[5 * N + q1] * first(nb[5]);
      const T u1 = T(0) + (fv(q1) - acc) / a[q1];
      const T u0 = fv(ju) / a[j];
      if constexpr (B2) {
        for_colors([&](auto cc) {
          constexpr int c = decltype(cc)::value;
          const int q = c * N4 + j;
          e[q] = a0 * p0[q];
          r[q] = fe_upd1_r(g[q], a0, q0[q]);
        });
      }
      u[j] = u0;
      u[q1] = u1;
      u[2 * N4 + j] = T(0);
      u[3 * N4 + j] = T(0);
    }
    fe_wsync();
    auto phase = [&](auto cc) {
      constexpr int c = decltype(cc)::value;
      const int q = c * N4 + j;
      const T dl = (f[q] - fe_row<T, 4, c>(a, ju, uv)) / a[q];
      u[q] += dl;
      fe_wsync();
    };
    phase(IC<2>{});
    phase(IC<3>{});
    {  // residual and restriction to the coarsest level (lane m = parent)
      const T r0 = f[0 * N4 + j] - fe_row<T, 4, 0>(a, ju, uv);
      const T r1 = f[1 * N4 + j] - fe_row<T, 4, 1>(a, ju, uv);
      const T r3 = f[3 * N4 + j] - fe_row<T, 4, 3>(a, ju, uv);
      const T r2 = f[2 * N4 + j] - fe_row<T, 4, 2>(a, ju, uv);
      T acc = 0;
      acc += r0;
      acc += r1;
      acc += r3;
      acc += r2;
      g3[q_of_m(ju, 3)] = acc;
    }
    fe_wsync();
    {  // coarsest solve e3 = A_3^{-1} g3 in FP64 (row j of the symmetric inverse read as column j), four partial
       // sums over i mod 4 (independent FMA chains), added pairwise
      double acc[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int i = 0; i < kFeCoarse; i += 4)
#pragma unroll
        for (int k = 0; k < 4; k++) acc[k] += Ainv[(i + k) * kFeCoarse + j] * static_cast<double>(g3[i + k]);
      e3[j] = static_cast<T>((acc[0] + acc[1]) + (acc[2] + acc[3]));
    }
    fe_wsync();
    {  // prolongation
      const T ecm = e3[q_of_m(ju, 3)];
      for_colors([&](auto cc) {
        constexpr int c = decltype(cc)::value;
        u[c * N4 + j] += ecm;
      });
    }
    fe_wsync();
    phase(IC<3>{});
    phase(IC<2>{});
    phase(IC<1>{});
    phase(IC<0>{});
  }

  __device__ __forceinline__ void btilde_w() const {
    constexpr int I = lw, N4 = 64;
    if (threadIdx.x >= 64) return;
    const T *a = ax<I>();
    const T *g = vec<I, V_G>();
    T *e = vec<I, V_E>(), *r = vec<I, V_R>(), *p0 = vec<I, V_P0>(), *q0 = vec<I, V_Q0>(), *p1 = vec<I, V_P1>();
    const int j = static_cast<int>(threadIdx.x);
    const uint32_t ju = static_cast<uint32_t>(j);
    bhat_w<0>(T(0));
    double v[2] = {0.0, 0.0};
    for_colors([&](auto cc) {
      constexpr int c = decltype(cc)::value;
      const int q = c * N4 + j;
      const T yq = fe_row<T, 4, c>(a, ju, [p0](uint32_t i) { return p0[i]; });
      q0[q] = yq;
      v[0] += static_cast<double>(p0[q]) * static_cast<double>(yq);
      v[1] += static_cast<double>(g[q]) * static_cast<double>(p0[q]);
    });
    fe_wave_allreduce<2>(v);
    const double d0 = v[0];
    const bool stop = !(d0 > 0.0);
    const double a0 = stop ? 0.0 : v[1] / d0;
    fe_wsync();
    bhat_w<1>(static_cast<T>(a0));
    double t[1] = {0.0};
    for_colors([&](auto cc) {
      constexpr int c = decltype(cc)::value;
      const int q = c * N4 + j;
      t[0] += static_cast<double>(p1[q]) * static_cast<double>(q0[q]);
    });
    fe_wave_allreduce<1>(t);
    const double beta = stop ? 0.0 : -t[0] / d0;
    const T bt = static_cast<T>(beta);
    auto dir = [p1, p0, bt](uint32_t i) { return p1[i] + bt * p0[i]; };
    double w[2] = {0.0, 0.0};
    for_colors([&](auto cc) {
      constexpr int c = decltype(cc)::value;
      const uint32_t q = static_cast<uint32_t>(c * N4 + j);
      const T yq = fe_row<T, 4, c>(a, ju, dir);
      const T xq = dir(q);
      w[0] += static_cast<double>(xq) * static_cast<double>(yq);
      w[1] += static_cast<double>(r[q]) * static_cast<double>(xq);
    });
    fe_wave_allreduce<2>(w);
    const T a1 = static_cast<T>((stop || !(w[0] > 0.0)) ? 0.0 : w[1] / w[0]);
    for_colors([&](auto cc) {
      constexpr int c = decltype(cc)::value;
      const int q = c * N4 + j;
      e[q] += a1 * (p1[q] + bt * p0[q]);
    });
  }

  // ---- dispatch ----

  template <int I>
  __device__ __forceinline__ bool level_steps(int code) const {
    if constexpr (I < lw) {
      switch (code) {
        case fe_code(FE_FIRST2, I, 0, 0): first2<I, 0>(); return true;
        case fe_code(FE_FIRST2, I, 0, 1): first2<I, 1>(); return true;
        case fe_code(FE_GS, I, 0, 0): gs<I, 0, 0>(); return true;
        case fe_code(FE_GS, I, 1, 0): gs<I, 1, 0>(); return true;
        case fe_code(FE_GS, I, 2, 0): gs<I, 2, 0>(); return true;
        case fe_code(FE_GS, I, 3, 0): gs<I, 3, 0>(); return true;
        case fe_code(FE_GS, I, 0, 1): gs<I, 0, 1>(); return true;
        case fe_code(FE_GS, I, 1, 1): gs<I, 1, 1>(); return true;
        case fe_code(FE_GS, I, 2, 1): gs<I, 2, 1>(); return true;
        case fe_code(FE_GS, I, 3, 1): gs<I, 3, 1>(); return true;
        case fe_code(FE_RES, I, 0, 0): res_restrict<I, 0>(); return true;
        case fe_code(FE_RES, I, 0, 1): res_restrict<I, 1>(); return true;
        case fe_code(FE_PROLONG, I, 0, 0): prolong<I, 0>(); return true;
        case fe_code(FE_PROLONG, I, 0, 1): prolong<I, 1>(); return true;
        case fe_code(FE_SPMV0, I, 0, 0): spmv0<I>(); return true;
        case fe_code(FE_SPMV1, I, 0, 0): spmv1<I>(); return true;
        case fe_code(FE_UPDATE2, I, 0, 0): update2<I>(); return true;
        default: return false;
      }
    } else {
      return false;
    }
  }

  __device__ __forceinline__ void step(int code) const {
    if (code == fe_code(FE_BTILDE_W, lw, 0, 0)) {
      btilde_w();
      return;
    }
    if (level_steps<0>(code)) return;
    level_steps<1>(code);
  }
};

// dst[i] = src[i] for i < N: a thread's loads issued in rounds of eight before any of them is stored (a plain copy
// loop waits for each load before the next)
template <class V, int N, int NT>
__device__ __forceinline__ void fe_stage(V *dst, const V *__restrict__ src, int tid) {
  constexpr int per = (N + NT - 1) / NT, R = 8;
#pragma unroll
  for (int k0 = 0; k0 < per; k0 += R) {
    V tmp[R];
#pragma unroll
    for (int k = 0; k < R; k++) {
      const int i = tid + (k0 + k) * NT;
      if (k0 + k < per) tmp[k] = src[i < N ? i : N - 1];
    }
#pragma unroll
    for (int k = 0; k < R; k++) {
      const int i = tid + (k0 + k) * NT;
      if (k0 + k < per && i < N) dst[i] = tmp[k];
    }
  }
}

template <class T, int KT, int KL>
__global__ void __launch_bounds__((FeLayout<T, KT, KL>::threads)) k_engine_fast(FeArgs<T> A) {
  using Lay = FeLayout<T, KT, KL>;
  constexpr int NT = Lay::threads;
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ double sc[4][8];
  __shared__ double red[2 * kFeMaxWaves];
  __shared__ int32_t ops[kFeMaxOps];
  double *ainv = reinterpret_cast<double *>(smem);
  T *S = reinterpret_cast<T *>(smem + kFeAinvBytes);
  const int tid = static_cast<int>(threadIdx.x);
  FeTop<T, Lay::TR> R;
  if constexpr (Lay::reg_top) {  // the top level's rows of this thread
    constexpr int N = Lay::n(0), N4 = N / 4;
#pragma unroll
    for (int t = 0; t < Lay::TR; t++)
      for_colors([&](auto cc) {
        constexpr int c = decltype(cc)::value;
        const int j = tid + t * NT;
        for_slots([&](auto ss) {
          constexpr int sl = decltype(ss)::value;
          R.a[t][c][sl] = A.ax[0][sl * N + c * N4 + j];
        });
        R.v[t][0][c] = A.gv[V_G][c * N4 + j];
      });
  }
  for (int i = tid; i < A.nops; i += NT) ops[i] = A.ops[i];
  fe_stage<double, kFeCoarse * kFeCoarse, NT>(ainv, A.ainv, tid);
  // operators of the LDS levels
  auto stage_level = [&](auto ll) {
    constexpr int l = decltype(ll)::value;
    if constexpr (l >= Lay::first_lds && l <= Lay::lw)
      fe_stage<T, 9 * Lay::n(l), NT>(S + Lay::ax_off(l), A.ax[l], tid);
  };
  stage_level(IC<0>{});
  stage_level(IC<1>{});
  stage_level(IC<2>{});
  if constexpr (Lay::lds(0)) fe_stage<T, Lay::n(0), NT>(S + Lay::vec_off(0) + V_G * Lay::n(0), A.gv[V_G], tid);
  __syncthreads();
  const FeEngine<T, KT, KL> E{S, ainv, A, sc, red, R};
  for (int oi = 0; oi < A.nops; oi++) {
    E.step(__builtin_amdgcn_readfirstlane(ops[oi]));
    __syncthreads();
  }
  if constexpr (Lay::reg_top) {
    constexpr int N4 = Lay::n(0) / 4;
#pragma unroll
    for (int t = 0; t < Lay::TR; t++)
      for_colors([&](auto cc) {
        constexpr int c = decltype(cc)::value;
        A.gv[V_E][c * N4 + tid + t * NT] = R.v[t][1][c];
      });
  } else {
    const T *e = S + Lay::vec_off(0) + V_E * Lay::n(0);
    for (int i = tid; i < Lay::n(0); i += NT) A.gv[V_E][i] = e[i];
  }
}

// ---- host side ----

void fe_emit_btilde(std::vector<int32_t> &ops, int kt, int l, bool defer);

// B^ of Algorithm 2.2 on engine level l (k >= 5), one sweep: the first two phases from zero as one step, then
// colors 2 and 3, residual and restriction, the coarse B~, prolongation, colors 3..0
void fe_emit_bhat(std::vector<int32_t> &ops, int kt, int l, int b2) {
  ops.push_back(fe_code(FE_FIRST2, l, 0, b2));
  ops.push_back(fe_code(FE_GS, l, 2, b2));
  ops.push_back(fe_code(FE_GS, l, 3, b2));
  ops.push_back(fe_code(FE_RES, l, 0, b2));
  fe_emit_btilde(ops, kt, l + 1, kt - (l + 1) >= 5);
  ops.push_back(fe_code(FE_PROLONG, l, 0, b2));
  for (int c = 3; c >= 0; c--) ops.push_back(fe_code(FE_GS, l, c, b2));
}

// B~ of Algorithm 2.1 (n = 2) on engine level l; on k = 4 one step for the whole of it. defer: the last update is
// formed by the parent's prolongation.
void fe_emit_btilde(std::vector<int32_t> &ops, int kt, int l, bool defer) {
  if (kt - l == 4) {
    ops.push_back(fe_code(FE_BTILDE_W, l, 0, 0));
    return;
  }
  fe_emit_bhat(ops, kt, l, 0);
  ops.push_back(fe_code(FE_SPMV0, l, 0, 0));
  fe_emit_bhat(ops, kt, l, 1);
  ops.push_back(fe_code(FE_SPMV1, l, 0, 0));
  if (!defer) ops.push_back(fe_code(FE_UPDATE2, l, 0, 0));
}

// configuration ids: FP32 (6,5), (5,5), (4,4); FP64 (5,4), (4,4)
struct FeCfg {
  int pi, kt, kl;
};
constexpr FeCfg kFeCfgs[] = {{1, 6, 5}, {1, 5, 5}, {1, 4, 4}, {0, 5, 4}, {0, 4, 4}};

template <class T, int KT, int KL>
size_t fe_bytes() {
  return FeLayout<T, KT, KL>::bytes;
}

size_t fe_cfg_bytes(int id) {
  switch (id) {
    case 0: return fe_bytes<float, 6, 5>();
    case 1: return fe_bytes<float, 5, 5>();
    case 2: return fe_bytes<float, 4, 4>();
    case 3: return fe_bytes<double, 5, 4>();
    default: return fe_bytes<double, 4, 4>();
  }
}

const void *fe_kernel(int id) {
  switch (id) {
    case 0: return reinterpret_cast<const void *>(k_engine_fast<float, 6, 5>);
    case 1: return reinterpret_cast<const void *>(k_engine_fast<float, 5, 5>);
    case 2: return reinterpret_cast<const void *>(k_engine_fast<float, 4, 4>);
    case 3: return reinterpret_cast<const void *>(k_engine_fast<double, 5, 4>);
    default: return reinterpret_cast<const void *>(k_engine_fast<double, 4, 4>);
  }
}

constexpr size_t kFeStatic = sizeof(double) * 4 * 8 + sizeof(double) * 2 * kFeMaxWaves + sizeof(int32_t) * kFeMaxOps;

amg_status fe_lds_limits(int device, size_t lds_max) {
  static std::once_flag once[64];
  if (device < 0 || device >= 64) return AMG_ERR_DEVICE;
  amg_status st = AMG_OK;
  std::call_once(once[device], [&]() {
    const int dyn = static_cast<int>(lds_max - kFeStatic);
    for (int id = 0; id < 5; id++)
      if (hipFuncSetAttribute(fe_kernel(id), hipFuncAttributeMaxDynamicSharedMemorySize, dyn) != hipSuccess)
        st = AMG_ERR_DEVICE;
  });
  return st;
}

template <class T>
std::vector<LevelWork<T>> &fe_work(amg_hierarchy *h) {
  if constexpr (std::is_same<T, float>::value) return h->w32;
  else return h->w64;
}
template <class T>
const T *fe_level_ax(const QuadLevel &Q) {
  if constexpr (std::is_same<T, float>::value) return Q.ax32;
  else return Q.ax64;
}

template <class T>
void fe_fill(amg_hierarchy *h, int pi, FeArgs<T> &A) {
  const int top = h->engine_top[pi];
  A.nops = h->fe_nops[pi];
  A.ops = static_cast<const int32_t *>(h->fe_ops[pi]);
  A.ainv = h->ainv;
  for (int i = 0; i < 4; i++) {
    const int l = top + i;
    A.ax[i] = l < h->nlev ? fe_level_ax<T>(h->lev[l]) : nullptr;
  }
  const LevelWork<T> &w = fe_work<T>(h)[top];
  A.gv[V_G] = w.g;
  A.gv[V_E] = w.e;
  A.gv[V_R] = w.r;
  A.gv[V_P0] = w.p0;
  A.gv[V_Q0] = w.q0;
  A.gv[V_P1] = w.p1;
}

template <class T, int KT, int KL>
void fe_launch(amg_hierarchy *h, int pi) {
  FeArgs<T> A{};
  fe_fill<T>(h, pi, A);
  const size_t lds = FeLayout<T, KT, KL>::bytes;
  Timing &t = h->timing;
  const int kind = pi ? KK_ENGINE32 : KK_ENGINE64;
  if (t.kind == kind && t.used + 2 <= t.ev.size()) {  // dispatch-stamped start / stop
    hipExtLaunchKernelGGL(k_engine_fast<T, KT, KL>, dim3(1), dim3(FeLayout<T, KT, KL>::threads), lds, h->stream,
                          t.ev[t.used],
                          t.ev[t.used + 1], 0, A);
    t.used += 2;
  } else {
    k_engine_fast<T, KT, KL><<<1, FeLayout<T, KT, KL>::threads, lds, h->stream>>>(A);
  }
}

}  // namespace

amg_status plan_engine_fast(amg_hierarchy *h) {
  h->fe_cfg[0] = h->fe_cfg[1] = -1;
  if (h->use_engine != 1 || h->nlev < 3 || h->L < 4 || h->lev[h->nlev - 1].k != 3 || h->nc != kFeCoarse ||
      h->opt.sweeps != 1 || h->opt.inner_iters != 2)
    return AMG_OK;
  if (h->lds_max == 0) {
    int lds = 0;
    QA_HIP(hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, h->device));
    h->lds_max = static_cast<size_t>(lds);
  }
  for (int id = 0; id < 5; id++) {
    const FeCfg c = kFeCfgs[id];
    // the top is the largest level the count allows (k = min(L, 6) in FP32, min(L, 5) in FP64); LDS holds k <= 5 in
    // FP32 and k <= 4 in FP64
    const int kt = std::min(h->L, c.pi ? 6 : 5);
    const int kl = std::min(kt, c.pi ? 5 : 4);
    if (kt != c.kt || kl != c.kl) continue;
    const int top = 1 + (h->L - c.kt);  // hierarchy index of level k = kt
    bool ok = fe_cfg_bytes(id) + kFeStatic <= h->lds_max;
    for (int l = top; l + 1 < h->nlev && ok; l++)
      if (h->lev[l].ovf_nnz != 0 || h->lev[l].same_color_ovf) ok = false;
    if (!ok) continue;
    std::vector<int32_t> ops;
    fe_emit_btilde(ops, c.kt, 0, false);
    if (ops.size() > static_cast<size_t>(kFeMaxOps)) continue;
    int32_t *d = static_cast<int32_t *>(dalloc(h, sizeof(int32_t) * ops.size()));
    if (!d) return AMG_ERR_NOMEM;
    QA_HIP(hipMemcpyAsync(d, ops.data(), sizeof(int32_t) * ops.size(), hipMemcpyHostToDevice, h->stream));
    QA_HIP(hipStreamSynchronize(h->stream));
    h->fe_cfg[c.pi] = id;
    h->fe_ops[c.pi] = d;
    h->fe_nops[c.pi] = static_cast<int>(ops.size());
    h->engine_top[c.pi] = top;
    h->engine_lds_top[c.pi] = top + (c.kt - c.kl);
    h->engine_lds[c.pi] = fe_cfg_bytes(id);
    h->engine_nops[c.pi] = static_cast<int>(ops.size());
  }
  if (h->fe_cfg[0] >= 0 || h->fe_cfg[1] >= 0) QA_TRY(fe_lds_limits(h->device, h->lds_max));
  return AMG_OK;
}

void launch_engine_fast(amg_hierarchy *h, int pi) {
  switch (h->fe_cfg[pi]) {
    case 0: fe_launch<float, 6, 5>(h, pi); break;
    case 1: fe_launch<float, 5, 5>(h, pi); break;
    case 2: fe_launch<float, 4, 4>(h, pi); break;
    case 3: fe_launch<double, 5, 4>(h, pi); break;
    case 4: fe_launch<double, 4, 4>(h, pi); break;
    default: break;
  }
}

}  // namespace qa
