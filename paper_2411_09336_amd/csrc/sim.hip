// Batched truncated MPS simulation of the feature-map circuit (Sec. II-B,
// Fig. 1; circuit of Sec. II-C).
//
// Every circuit of a batch shares one gate list, hence one step list (runs
// of Rz records, centre moves and two-qubit gates); a launch runs a chunk of
// steps with one workgroup per circuit, each walking its own circuit through
// the chunk.  Rz layers are diagonal and applied in place (Fig. 1a).  A
// two-qubit gate on sites (p, p+1) (Fig. 1b):
//   * theta[(s,a),(t,b)] = sum_{s',t'} G[st,s't'] P[(s',a),(t',b)] with the
//     pair product P[(s',a),(t',b)] = sum_c A_p[s'][a][c] A_{p+1}[t'][c][b],
//     formed once per step as a block-wide GEMM through LDS;
//   * its SVD is taken by one-sided (Hestenes) Jacobi in FP64: pairs of
//     columns are rotated until every pair is orthogonal to relative
//     tolerance 1e-14; the columns then are U S.  To absorb S to the right
//     the columns of theta are orthogonalised (U = W / |W|, the new right
//     tensor is U^H theta); to absorb it to the left the columns of theta^H
//     are (giving V, the new left tensor is theta V).  The isometric factor
//     is therefore always a set of normalised Jacobi columns and the other
//     factor an exact projection, so no V matrix is accumulated;
//   * truncation keeps k = max(1, min(chi, k_cut)) columns by decreasing norm
//     (Eq. (8): k_cut is the smallest count whose discarded weight is at most
//     cutoff times the total; cutoff <= 0 keeps all non-zero columns) and the
//     kept weight is renormalised to one.
// Orthogonality-centre moves (canonicalisation before each truncation) use
// the same machinery without truncation: the site matrix is orthogonalised
// and the remainder is pushed into the neighbour via the identity two-site
// theta.
//
// Register layout of the Jacobi matrix M (<= 128 x 128 complex): wave w of
// 16 owns rows 8w .. 8w+7; lane l owns column positions 2l and 2l+1 (slots A
// and B).  Rounds alternate between pairs inside a lane and pairs across
// neighbouring lanes (odd-even transposition ordering, each pair exchanged
// after its rotation), so n rounds visit every pair once per sweep and the
// only data movement is one DPP lane shift each way in every second round.
// Each round the partial inner products of the 16 waves go through LDS to
// four waves that form the rotation parameters, which all waves then apply.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "qk_internal.h"

namespace qk {

namespace {

constexpr int kSvWaves = 16;
constexpr int kSvRows = 8;                // rows per wave
constexpr int kSvThreads = kSvWaves * 64; // 1024
constexpr int kSvMaxN = 128;
constexpr int kMaxSweeps = 30;
// Two-site steps next to a bond above 64 (bond caps up to 128): Jacobi
// matrices up to 256 x 256, streamed through a per-circuit slot of global
// scratch (Jacobi columns and projection source, 1 MiB each).
constexpr int kWideN = 256;
constexpr int kWideFrom = 64;     // a neighbouring bond above this takes the wide step
constexpr size_t kWideSlot = size_t(2) * kWideN * kWideN;
constexpr double kJacobiTol = 1e-14;
// A sweep whose rotations all have |<X,Y>| below kJacobiLarge |X| |Y| ends
// the iteration: cyclic Jacobi converges quadratically, so the next sweep's
// would fall below kJacobiTol and rotate nothing.
constexpr double kJacobiLarge = 1e-8;
// columns whose weight is below this fraction of ||M||_F^2 are numerical zeros
constexpr double kZeroWeight = 1e-28;
constexpr double kDegenerateGap = 1e-10;

enum SvMode { GATE_RIGHT = 0, GATE_LEFT = 1, MOVE_RIGHT = 2, MOVE_LEFT = 3 };
enum GateOp { OP_RZ = 0, OP_RXX = 1, OP_SWAP = 2, OP_ID = 3 };

struct SvParams {
  double2 *f64;
  int64_t mps_stride;
  const int64_t *site_off;
  const int32_t *pad;
  int32_t *dims;
  int32_t m;
  int32_t chi;
  int32_t gate_split;  // cap the kept count at rank(G) x the middle bond
  double coef_xx;
  double cutoff;
  const double *X;
  int64_t ldx;
  double2 *scratch;  // per circuit 2 * kSvMaxN * kSvMaxN
  double2 *wscratch; // per circuit kWideSlot (bond caps above 64), else nullptr
  double *disc;
  double *maxdisc;
  int32_t *degen;
  int32_t *unconv;
  int64_t n;
  int32_t *trace;     // optional: per circuit and two-qubit gate (cut bond, sum_l D_l D_{l+1})
  int32_t trace_n2q;  // two-qubit gates per circuit (row length of the trace / 2)
  const int64_t *base;  // graph replays: first circuit of the replay (nullptr: 0)
};

// Circuit of this workgroup: workgroup i of a launch simulates circuit
// base + i, where base is read from device memory in a graph replay (each
// replay advances it by the launch's grid) and is 0 otherwise.  The SVD
// scratch slot is the workgroup index, so a graph needs scratch only for
// the circuits of one replay.
__device__ inline int64_t circuit_of(const int64_t *base) { return (base ? *base : 0) + blockIdx.x; }

// DPP lane moves of a double.  Lanes without a source lane receive zero
// (bound_ctrl), so no copy of the source is needed as the fallback value.
template <int CTRL>
__device__ inline double dpp_mov(double x) {
  const int lo = __double2loint(x), hi = __double2hiint(x);
  return __hiloint2double(__builtin_amdgcn_mov_dpp(hi, CTRL, 0xf, 0xf, true),
                          __builtin_amdgcn_mov_dpp(lo, CTRL, 0xf, 0xf, true));
}
// shr1: lane l receives lane l-1 (lane 0: zero); shl1: lane l receives lane
// l+1 (lane 63: zero)
__device__ inline double dpp_shr1(double x) { return dpp_mov<0x138>(x); }
__device__ inline double dpp_shl1(double x) { return dpp_mov<0x130>(x); }

// Sum over the 16 lanes of a DPP row (all 16 lanes receive the total).
__device__ inline double row_sum16(double x) {
  x += dpp_mov<0x128>(x);   // row_ror:8
  x += dpp_mov<0x124>(x);   // row_ror:4
  x += dpp_mov<0x122>(x);   // row_ror:2
  x += dpp_mov<0x121>(x);   // row_ror:1
  return x;
}

__device__ inline double2 cconj(double2 a) { return make_double2(a.x, -a.y); }

// Sum over the 64 lanes of the wave (every lane receives the total).
__device__ inline double wave_sum(double x) {
  x = row_sum16(x);
  x += __shfl_xor(x, 16, 64);
  x += __shfl_xor(x, 32, 64);
  return x;
}

// Lane-half and row exchanges of two doubles (gfx950 permlane swaps):
// swap32 leaves a = [a_lo, b_lo], b = [a_hi, b_hi] (32-lane halves);
// swap16 leaves a = [a_0, b_0, a_2, b_2], b = [a_1, b_1, a_3, b_3] (rows).
__device__ inline void swap32(double &a, double &b) {
  const auto lo = __builtin_amdgcn_permlane32_swap(__double2loint(a), __double2loint(b), false, false);
  const auto hi = __builtin_amdgcn_permlane32_swap(__double2hiint(a), __double2hiint(b), false, false);
  a = __hiloint2double(int(hi[0]), int(lo[0]));
  b = __hiloint2double(int(hi[1]), int(lo[1]));
}
__device__ inline void swap16(double &a, double &b) {
  const auto lo = __builtin_amdgcn_permlane16_swap(__double2loint(a), __double2loint(b), false, false);
  const auto hi = __builtin_amdgcn_permlane16_swap(__double2hiint(a), __double2hiint(b), false, false);
  a = __hiloint2double(int(hi[0]), int(lo[0]));
  b = __hiloint2double(int(hi[1]), int(lo[1]));
}

// Sixteen wave sums at once (every lane receives all sixteen totals): a
// reduce-scatter over the lane halves and rows (each exchange halves the
// values a lane carries), a row sum of the remaining four, then the reverse
// exchanges to spread the totals.  About a third of the instructions of
// sixteen separate wave sums.
__device__ inline void wave_sum16(double (&v)[16]) {
  double u[8], t[4];
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    swap32(v[2 * k], v[2 * k + 1]);
    u[k] = v[2 * k] + v[2 * k + 1];  // lanes 0-31: value 2k, lanes 32-63: value 2k+1
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    swap16(u[2 * k], u[2 * k + 1]);
    // rows 0, 1, 2, 3: values 4k, 4k+2, 4k+1, 4k+3, each over 4 lanes
    t[k] = row_sum16(u[2 * k] + u[2 * k + 1]);
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    double a = t[k], b = t[k];
    swap16(a, b);  // rows 0, 1: a = value 4k, b = 4k+2; rows 2, 3: a = 4k+1, b = 4k+3
    double a2 = a, b2 = b;
    swap32(a, a2);
    swap32(b, b2);
    v[4 * k] = a;
    v[4 * k + 1] = a2;
    v[4 * k + 2] = b;
    v[4 * k + 3] = b2;
  }
}

constexpr int kKC = 16;  // contraction chunk of the pair product staged in LDS

// Block-wide complex product acc[rr][q] = sum_{k < K} L(y, k) R(k, x) with
// y = ROWS w + rr (wave w) and x = 2 l + q (lane l); ldL / ldR return the
// operands (zero outside the matrices).  Chunks of kKC contraction indices
// of both operands are staged in LDS; the row operand is read by the whole
// wave at one address.
template <int ROWS, class FL, class FR>
__device__ inline void staged_tile_gemm(int K, const FL &ldL, const FR &ldR, double2 (*sL)[kSvMaxN],
                                        double2 (*sR)[kSvMaxN], double2 (&acc)[ROWS][2]) {
  const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  constexpr int kRowsAll = ROWS * kSvWaves;
#pragma unroll
  for (int rr = 0; rr < ROWS; ++rr) {
    acc[rr][0] = make_double2(0.0, 0.0);
    acc[rr][1] = make_double2(0.0, 0.0);
  }
  for (int k0 = 0; k0 < K; k0 += kKC) {
    __syncthreads();  // the previous chunk (or earlier use of the buffers) is done
    for (int e = tid; e < kKC * kRowsAll; e += kSvThreads) {
      // consecutive threads walk the contraction index of one row
      const int kk = e % kKC, y = e / kKC;
      sL[kk][y] = k0 + kk < K ? ldL(y, k0 + kk) : make_double2(0.0, 0.0);
    }
    for (int e = tid; e < kKC * kSvMaxN; e += kSvThreads) {
      const int x = e % kSvMaxN, kk = e / kSvMaxN;
      sR[kk][x] = k0 + kk < K ? ldR(k0 + kk, x) : make_double2(0.0, 0.0);
    }
    __syncthreads();
    const int kc = min(kKC, K - k0);
    for (int kk = 0; kk < kc; ++kk) {
      const double2 r0 = sR[kk][2 * lane], r1 = sR[kk][2 * lane + 1];
#pragma unroll
      for (int rr = 0; rr < ROWS; ++rr) {
        const double2 l = sL[kk][wave * ROWS + rr];
        acc[rr][0].x = fma(l.x, r0.x, fma(-l.y, r0.y, acc[rr][0].x));
        acc[rr][0].y = fma(l.x, r0.y, fma(l.y, r0.x, acc[rr][0].y));
        acc[rr][1].x = fma(l.x, r1.x, fma(-l.y, r1.y, acc[rr][1].x));
        acc[rr][1].y = fma(l.x, r1.y, fma(l.y, r1.x, acc[rr][1].y));
      }
    }
  }
}

// Two-site theta element theta[(s, a), (t, b)] of this step's gate from the
// pair product P (row stride ld).
__device__ inline double2 theta_from_pair(const double2 *Pp2, int op, double cg, double sg, int Dp, int Dn, int s,
                                          int a, int t, int b, int ld = kSvMaxN) {
  if (op == OP_SWAP) return Pp2[(t * Dp + a) * ld + s * Dn + b];
  const double2 d = Pp2[(s * Dp + a) * ld + t * Dn + b];
  if (op == OP_RXX) {
    // Rxx = cos(phi/2) I - i sin(phi/2) X(x)X
    const double2 x = Pp2[((1 - s) * Dp + a) * ld + (1 - t) * Dn + b];
    return make_double2(cg * d.x + sg * x.y, cg * d.y - sg * x.x);
  }
  return d;
}

struct JacobiShared {
  double2 (*red)[kSvWaves][64];  // [0]: (|X|^2, |Y|^2), [1]: <X, Y>; per wave and lane
  double (*upd)[64][8];          // per round type and lane: pa, wa, -, -, pb, wb, -, -
  double *w;                     // squared norm of the column at each position
};

// Sum over the 4 lanes of a DPP quad (every lane receives the same total).
__device__ inline double quad_sum(double x) {
  x += dpp_mov<0xB1>(x);   // quad_perm [1,0,3,2]
  x += dpp_mov<0x4E>(x);   // quad_perm [2,3,0,1]
  return x;
}

// One round of the parallel Jacobi sweep.  The pair of a lane is (X, Y) =
// (A, B) for TYPE 0 and (B_l, A_{l+1}) for TYPE 1.  Its rotation
// X' = c X - s u Y, Y' = s X + c u Y (u = conj<X,Y> / |<X,Y>|, the
// Hermitian 2x2 Jacobi rotation of the Gram block of the pair) zeroes
// <X', Y'>; the outputs are stored exchanged, Y' in the slot of X and X' in
// the slot of Y.  Every lane then forms A' = pa P + wa Q, B' = pb R + wb S
// with (P, Q, R, S) = (A, B, A, B) for TYPE 0 and (B_{l-1}, A, B, A_{l+1})
// for TYPE 1.  Returns whether this wave rotated some pair by more than
// kJacobiLarge (relative |<X,Y>|).
//
// Column norms: a FULL round reduces |X|^2 and |Y|^2 with <X, Y> and stores
// them; the other rounds reduce <X, Y> only and update the stored norms by
// |X'|^2 = |X|^2 - t |<X,Y>|, |Y'|^2 = |Y|^2 + t |<X,Y>| (t = s / c), which
// holds exactly for the rotation above.  The first round of every sweep is
// FULL, so rounding in the updates never outlives a sweep.
template <int TYPE, bool FULL>
__device__ __forceinline__ bool jacobi_round(double (&Ar)[kSvRows], double (&Ai)[kSvRows], double (&Br)[kSvRows],
                                             double (&Bi)[kSvRows], const JacobiShared &sh, int wave,
                                             int H, double zero_w) {
  // The lane index is formed afresh every round (two instructions the
  // compiler cannot hoist), so the LDS addresses derived from it are not
  // held, or spilled, across the sweep loop.
  int lane;
  asm volatile("v_mbcnt_lo_u32_b32 %0, -1, 0\n\tv_mbcnt_hi_u32_b32 %0, -1, %0" : "=v"(lane));
  double Nr[kSvRows], Ni[kSvRows];  // A_{l+1} (TYPE 1)
  if (TYPE == 1) {
#pragma unroll
    for (int rr = 0; rr < kSvRows; ++rr) {
      Nr[rr] = dpp_shl1(Ar[rr]);
      Ni[rr] = dpp_shl1(Ai[rr]);
    }
  }
  {
    double al = 0.0, be = 0.0, gr = 0.0, gi = 0.0;
#pragma unroll
    for (int rr = 0; rr < kSvRows; ++rr) {
      const double xr = TYPE == 0 ? Ar[rr] : Br[rr], xi = TYPE == 0 ? Ai[rr] : Bi[rr];
      const double yr = TYPE == 0 ? Br[rr] : Nr[rr], yi = TYPE == 0 ? Bi[rr] : Ni[rr];
      if (FULL) {
        al = fma(xr, xr, fma(xi, xi, al));
        be = fma(yr, yr, fma(yi, yi, be));
      }
      gr = fma(xr, yr, fma(xi, yi, gr));
      gi = fma(xr, yi, fma(-xi, yr, gi));
    }
    if (FULL) sh.red[0][wave][lane] = make_double2(al, be);
    sh.red[1][wave][lane] = make_double2(gr, gi);
  }
  __syncthreads();
  // rotation parameters: waves 0..3, lane = 4 j + q sums the partials of
  // pair 16 wave + j over waves 4q..4q+3, then over the quad
  const int npairs = TYPE == 0 ? H : H - 1;
  bool large = false;
  if (wave < 4 && 16 * wave < npairs) {
    const int j = lane >> 2, q = lane & 3, pr = 16 * wave + j;
    // positions of X and Y
    const int px = TYPE == 0 ? 2 * pr : 2 * pr + 1, py = px + 1;
    double a = 0.0, b = 0.0, x = 0.0, y = 0.0;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (FULL) {
        const double2 n = sh.red[0][4 * q + u][pr];
        a += n.x;
        b += n.y;
      }
      const double2 g = sh.red[1][4 * q + u][pr];
      x += g.x;
      y += g.y;
    }
    if (FULL) {
      a = quad_sum(a);
      b = quad_sum(b);
    } else {
      a = sh.w[px];
      b = sh.w[py];
    }
    x = quad_sum(x);
    y = quad_sum(y);
    const double g2 = fma(x, x, y * y);
    const bool rot = pr < npairs && a > zero_w && b > zero_w && g2 > (kJacobiTol * kJacobiTol) * (a * b);
    large = __any(rot && g2 > (kJacobiLarge * kJacobiLarge) * (a * b));
    if (pr < npairs && q < 2) {
      double c = 1.0, s = 0.0, ur = 1.0, ui = 0.0, tg = 0.0;
      if (rot) {
        // rsqrt: the hardware estimate with one correction step (about 1
        // ulp), a third of the instructions of a divided square root on
        // this per-round critical path
        const double rg = rsqrt(g2);
        const double zeta = 0.5 * (b - a) * rg;
        // t = sign(zeta) / (|zeta| + sqrt(1 + zeta^2)); the denominator is >= 1, so
        // its reciprocal is the hardware estimate refined by two Newton steps
        // (the rotation is orthogonal for any t: c and s follow from t)
        const double den = fabs(zeta) + sqrt(fma(zeta, zeta, 1.0));
        double rd = __builtin_amdgcn_rcp(den);
        rd = fma(rd, fma(-den, rd, 1.0), rd);
        rd = fma(rd, fma(-den, rd, 1.0), rd);
        const double t = zeta >= 0.0 ? rd : -rd;
        c = rsqrt(fma(t, t, 1.0));
        s = c * t;
        ur = x * rg;
        ui = -y * rg;
        tg = t * (g2 * rg);
      }
      // exchanged: the slot of X receives |Y'|^2, the slot of Y |X'|^2
      if (q == 0) sh.w[px] = b + tg;
      else sh.w[py] = fmax(a - tg, 0.0);
      // q == 0 stores Y' = s X + (c u) Y, q == 1 stores X' = c X - (s u) Y
      const double p0 = q == 0 ? s : c, w = q == 0 ? c : -s;
      const int slot_lane = (TYPE == 1 && q == 1) ? pr + 1 : pr;
      const int slot = (TYPE == 0) == (q == 0) ? 0 : 4;
      double *o = sh.upd[TYPE][slot_lane] + slot;
      o[0] = p0;
      o[1] = w * ur;
      o[2] = w * ui;
    }
  }
  __syncthreads();
  const double *up = sh.upd[TYPE][lane];
  const double pa = up[0], war = up[1], wai = up[2], pb = up[4], wbr = up[5], wbi = up[6];
#pragma unroll
  for (int rr = 0; rr < kSvRows; ++rr) {
    double pr_, pi_, qr, qi, rr_, ri, sr, si;
    if (TYPE == 0) {
      pr_ = Ar[rr]; pi_ = Ai[rr]; qr = Br[rr]; qi = Bi[rr];
      rr_ = Ar[rr]; ri = Ai[rr]; sr = Br[rr]; si = Bi[rr];
    } else {
      pr_ = dpp_shr1(Br[rr]); pi_ = dpp_shr1(Bi[rr]); qr = Ar[rr]; qi = Ai[rr];
      rr_ = Br[rr]; ri = Bi[rr]; sr = Nr[rr]; si = Ni[rr];
    }
    Ar[rr] = fma(pa, pr_, fma(war, qr, -wai * qi));
    Ai[rr] = fma(pa, pi_, fma(war, qi, wai * qr));
    Br[rr] = fma(pb, rr_, fma(wbr, sr, -wbi * si));
    Bi[rr] = fma(pb, ri, fma(wbr, si, wbi * sr));
  }
  return large;
}

// One entry of the step list shared by every circuit of a batch: a run of
// Rz records, or a two-site step (a two-qubit gate or a centre move).
enum StepKind { STEP_RZ = 0, STEP_TWO_SITE = 1 };
struct SimStep {
  int32_t kind;
  int32_t p, mode, op, fi, fj;  // two-site step: sites (p, p+1), SvMode, GateOp, features of Rxx
  int32_t r0, nr;               // Rz run: gate records [r0, r0 + nr); two-site step: r0 = index of
                                // the two-qubit gate among the circuit's (-1 for a centre move)
};

// Rows j0 .. j0 + 63 of the projection out[j][x] = nrm sum_y conj(U[y][j])
// S[y][x] (j < k, x < ncs, y < nr) of a two-site step, written to the
// non-isometric site tensor; U is the isometric factor already written to
// A_p (absorb right) or, conjugated, to A_{p+1}.  Wave w forms rows
// j0 + 4w .. j0 + 4w + 3.
__device__ __attribute__((noinline)) void project_rows(double2 *Ap, double2 *Aq, const double2 *S, int Dp, int Dn,
                                                       int Pp, int Pm, int Pn, int nr, int ncs, int k, int j0,
                                                       double nrm, bool right, double2 (*sL)[kSvMaxN],
                                                       double2 (*sR)[kSvMaxN]) {
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  double2 acc[4][2];
  staged_tile_gemm<4>(
      nr,
      [&](int jj, int y) {
        const int j = j0 + jj;
        if (j >= k) return make_double2(0.0, 0.0);
        return right ? cconj(Ap[(size_t(y / Dp) * Pp + y % Dp) * Pm + j]) : Aq[(size_t(y / Dn) * Pm + j) * Pn + y % Dn];
      },
      [&](int y, int x) { return x < ncs ? S[y * kSvMaxN + x] : make_double2(0.0, 0.0); }, sL, sR, acc);
#pragma unroll
  for (int rr = 0; rr < 4; ++rr)
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int j = j0 + wave * 4 + rr, x = 2 * lane + q;
      if (j < k && x < ncs) {
        if (right) Aq[(size_t(x / Dn) * Pm + j) * Pn + x % Dn] = make_double2(nrm * acc[rr][q].x, nrm * acc[rr][q].y);
        else Ap[(size_t(x / Dp) * Pp + x % Dp) * Pm + j] = make_double2(nrm * acc[rr][q].x, -nrm * acc[rr][q].y);
      }
    }
}

// Two-site step of circuit ci (one 1024-thread workgroup).
__device__ __attribute__((noinline)) void svd_step(const SvParams &P, const int64_t ci, const SimStep &st) {
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave-uniform: scalar register

  // the pair-product staging is dead once the Jacobi matrix is built; the
  // reduction buffers are used from then on
  __shared__ union {
    struct {
      double2 L[kKC][kSvMaxN];
      double2 R[kKC][kSvMaxN];
    } stage;
    struct {
      double part[4][kSvWaves][65];  // [component][wave][pair], rows padded (bank spread)
      double2 red[2][kSvWaves][64];
    } jac;
  } s_u;
  auto &s_part = s_u.jac.part;
  auto &s_red = s_u.jac.red;
  __shared__ double s_upd[2][64][8];
  __shared__ double s_w[kSvMaxN];
  __shared__ double s_norm[kSvMaxN];
  __shared__ int s_piv[kSvMaxN];    // LQ pivot of each step
  __shared__ int s_prank[kSvMaxN];  // step at which each row is the pivot
  __shared__ double s_sorted[kSvMaxN];
  __shared__ int s_rank[kSvMaxN];
  __shared__ int s_k;
  __shared__ double s_nrm;

  int32_t *dims = P.dims + ci * (P.m + 1);
  const int p = st.p;
  const int Dp = dims[p], Dm = dims[p + 1], Dn = dims[p + 2];
  const int Pp = P.pad[p], Pm = P.pad[p + 1], Pn = P.pad[p + 2];
  double2 *Ap = P.f64 + ci * P.mps_stride + P.site_off[p];
  double2 *Aq = P.f64 + ci * P.mps_stride + P.site_off[p + 1];
  double2 *S = P.scratch + int64_t(blockIdx.x) * (2 * kSvMaxN * kSvMaxN);

  double cg = 1.0, sg = 0.0;
  if (st.op == OP_RXX) {
    const double xi = P.X[ci * P.ldx + st.fi], xj = P.X[ci * P.ldx + st.fj];
    const double phi = P.coef_xx * (1.0 - xi) * (1.0 - xj);
    sincos(0.5 * phi, &sg, &cg);
  }

  const bool right = (st.mode == GATE_RIGHT || st.mode == MOVE_RIGHT);
  const bool gate = (st.mode == GATE_RIGHT || st.mode == GATE_LEFT);
  // Jacobi matrix shape and projection-source width
  int nr, nc, ncs;
  if (st.mode == GATE_RIGHT) { nr = 2 * Dp; nc = 2 * Dn; ncs = nc; }
  else if (st.mode == GATE_LEFT) { nr = 2 * Dn; nc = 2 * Dp; ncs = nc; }
  else if (st.mode == MOVE_RIGHT) { nr = 2 * Dp; nc = Dm; ncs = 2 * Dn; }
  else { nr = 2 * Dn; nc = Dm; ncs = 2 * Dp; }

  // ---------------------------------------------------------- build M
  // M (Jacobi matrix) goes to scratch region SM, the projection source to S;
  // for gates they coincide and the pair product is kept in region 2.
  double2 *SM = gate ? S : S + kSvMaxN * kSvMaxN;
  {
    // pair product of the two sites, the two-site tensor before the gate
    // (Fig. 1b): P[(s', a)][(t', b)] = sum_c A_p[s'][a][c] A_{p+1}[t'][c][b]
    double2 pt[kSvRows][2];
    staged_tile_gemm<kSvRows>(
        Dm,
        [&](int y, int c) {
          return y < 2 * Dp ? Ap[(size_t(y / Dp) * Pp + y % Dp) * Pm + c] : make_double2(0.0, 0.0);
        },
        [&](int c, int x) {
          return x < 2 * Dn ? Aq[(size_t(x / Dn) * Pm + c) * Pn + x % Dn] : make_double2(0.0, 0.0);
        },
        s_u.stage.L, s_u.stage.R, pt);
    double2 *P2 = S + kSvMaxN * kSvMaxN;
#pragma unroll
    for (int rr = 0; rr < kSvRows; ++rr)
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const int y = wave * kSvRows + rr, x = 2 * lane + q;
        if (y < 2 * Dp && x < 2 * Dn) {
          if (gate) P2[y * kSvMaxN + x] = pt[rr][q];
          else if (st.mode == MOVE_RIGHT) S[y * kSvMaxN + x] = pt[rr][q];   // identity theta
          else S[x * kSvMaxN + y] = cconj(pt[rr][q]);                        // its adjoint
        }
      }
  }
  if (!gate) {
    // the site being orthogonalised, as a matrix
    for (int e = tid; e < nr * nc; e += kSvThreads) {
      const int r = e / nc, c = e % nc;
      SM[r * kSvMaxN + c] = st.mode == MOVE_RIGHT ? Ap[(size_t(r / Dp) * Pp + r % Dp) * Pm + c]
                                                 : cconj(Aq[(size_t(r / Dn) * Pm + c) * Pn + r % Dn]);
    }
  }
  __syncthreads();
  if (gate) {
    const double2 *P2 = S + kSvMaxN * kSvMaxN;
    for (int e = tid; e < nr * nc; e += kSvThreads) {
      const int r = e / nc, c = e % nc;
      SM[r * kSvMaxN + c] = st.mode == GATE_RIGHT
                                ? theta_from_pair(P2, st.op, cg, sg, Dp, Dn, r / Dp, r % Dp, c / Dn, c % Dn)
                                : cconj(theta_from_pair(P2, st.op, cg, sg, Dp, Dn, c / Dp, c % Dp, r / Dn, r % Dn));
    }
    __syncthreads();
  }
  double Ar[kSvRows], Ai[kSvRows], Br[kSvRows], Bi[kSvRows];
#pragma unroll
  for (int rr = 0; rr < kSvRows; ++rr) {
    const int r = wave * kSvRows + rr;
    const int c0 = 2 * lane, c1 = 2 * lane + 1;
    const double2 va = (r < nr && c0 < nc) ? SM[r * kSvMaxN + c0] : make_double2(0.0, 0.0);
    const double2 vb = (r < nr && c1 < nc) ? SM[r * kSvMaxN + c1] : make_double2(0.0, 0.0);
    Ar[rr] = va.x;
    Ai[rr] = va.y;
    Br[rr] = vb.x;
    Bi[rr] = vb.y;
  }
  // ||M||_F^2 (invariant under the rotations)
  {
    double w = 0.0;
#pragma unroll
    for (int rr = 0; rr < kSvRows; ++rr)
      w = fma(Ar[rr], Ar[rr], fma(Ai[rr], Ai[rr], fma(Br[rr], Br[rr], fma(Bi[rr], Bi[rr], w))));
    s_part[0][wave][lane] = w;
    __syncthreads();
    if (tid < 64) {
      double t = 0.0;
      for (int u = 0; u < kSvWaves; ++u) t += s_part[0][u][tid];
      for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o, 64);
      if (tid == 0) s_nrm = t;
    }
    __syncthreads();
  }
  const double zero_w = kZeroWeight * s_nrm;
  __syncthreads();

  // ---------------------------------------------------------- LQ preconditioning
  // M <- M H_0 H_1 ... (Householder reflections from the right, M = L Q with
  // the rows taken in order of decreasing norm): the Jacobi columns of M W
  // are U S for any unitary W, so the factors are unchanged, while the
  // triangular factor of these graded matrices needs 40 % fewer sweeps than M
  // itself.  Step i reflects the i-th heaviest row (its pivot) onto column i:
  // with x = that row restricted to columns >= i and
  // w = x + e^{i arg x_i} |x| e_i, every row r becomes r - beta (r . conj w) w,
  // beta = 1 / (|x| (|x| + |x_i|)).  Rows stay in place (a row permutation
  // changes no column inner product); the pivot's wave publishes w in LDS
  // (two buffers, one barrier per step), and waves whose rows all were
  // pivots of earlier steps hold only rounding-level entries in columns >= i
  // and skip the step.
  {
    double2(*lqw)[kSvMaxN] = reinterpret_cast<double2(*)[kSvMaxN]>(&s_red[0][0][0]);  // [2][kSvMaxN]
    double *lqb = reinterpret_cast<double *>(&s_red[1][0][0]);                          // [2]
    const int nref = min(nr, nc);
    const int c0 = 2 * lane, c1 = 2 * lane + 1;
    // pivot order: rows by decreasing norm, ties by index
#pragma unroll
    for (int rr = 0; rr < kSvRows; ++rr) {
      const double w2 = wave_sum(fma(Ar[rr], Ar[rr], fma(Ai[rr], Ai[rr], fma(Br[rr], Br[rr], Bi[rr] * Bi[rr]))));
      if (lane == 0) s_norm[wave * kSvRows + rr] = w2;
    }
    __syncthreads();
    if (tid < kSvMaxN) {
      const double v = s_norm[tid];
      int rank = 0;
#pragma unroll 1
      for (int u = 0; u < kSvMaxN; ++u) {
        const double o = s_norm[u];
        rank += (o > v || (o == v && u < tid)) ? 1 : 0;
      }
      s_piv[rank] = tid;
      s_prank[tid] = rank;
    }
    __syncthreads();
    int last = 0;  // latest step at which a row of this wave is the pivot
#pragma unroll
    for (int rr = 0; rr < kSvRows; ++rr) last = max(last, s_prank[wave * kSvRows + rr]);
    last = __builtin_amdgcn_readfirstlane(last);
    for (int i = 0; i < nref; ++i) {
      const int buf = i & 1;
      const int pv = __builtin_amdgcn_readfirstlane(s_piv[i]);
      if (wave == (pv >> 3)) {
        const int ri = pv & 7;
        double xr0 = 0.0, xi0 = 0.0, xr1 = 0.0, xi1 = 0.0;
#pragma unroll
        for (int rr = 0; rr < kSvRows; ++rr)
          if (rr == ri) {
            xr0 = Ar[rr];
            xi0 = Ai[rr];
            xr1 = Br[rr];
            xi1 = Bi[rr];
          }
        if (c0 < i) xr0 = xi0 = 0.0;
        if (c1 < i) xr1 = xi1 = 0.0;
        const double nx = sqrt(wave_sum(fma(xr0, xr0, fma(xi0, xi0, fma(xr1, xr1, xi1 * xi1)))));
        const double dr = __shfl((i & 1) ? xr1 : xr0, i >> 1, 64);
        const double di = __shfl((i & 1) ? xi1 : xi0, i >> 1, 64);
        const double ax = sqrt(fma(dr, dr, di * di));
        const double pr = ax > 0.0 ? dr / ax : 1.0, pi = ax > 0.0 ? di / ax : 0.0;
        const double wdr = pr * (ax + nx), wdi = pi * (ax + nx);
        lqw[buf][c0] = c0 == i ? make_double2(wdr, wdi) : make_double2(xr0, xi0);
        lqw[buf][c1] = c1 == i ? make_double2(wdr, wdi) : make_double2(xr1, xi1);
        if (lane == 0) lqb[buf] = nx > 0.0 ? 1.0 / (nx * (nx + ax)) : 0.0;
      }
      __syncthreads();
      if (last >= i) {
        const double2 w0 = lqw[buf][c0], w1 = lqw[buf][c1];
        const double beta = lqb[buf];
        double d[16];  // d = r . conj(w) for the wave's rows (re, im)
#pragma unroll
        for (int rr = 0; rr < kSvRows; ++rr) {
          d[2 * rr] = fma(Ar[rr], w0.x, fma(Ai[rr], w0.y, fma(Br[rr], w1.x, Bi[rr] * w1.y)));
          d[2 * rr + 1] = fma(Ai[rr], w0.x, fma(-Ar[rr], w0.y, fma(Bi[rr], w1.x, -Br[rr] * w1.y)));
        }
        wave_sum16(d);
#pragma unroll
        for (int rr = 0; rr < kSvRows; ++rr) {
          const double dr = beta * d[2 * rr], di = beta * d[2 * rr + 1];
          Ar[rr] -= dr * w0.x - di * w0.y;
          Ai[rr] -= dr * w0.y + di * w0.x;
          Br[rr] -= dr * w1.x - di * w1.y;
          Bi[rr] -= dr * w1.y + di * w1.x;
        }
      }
    }
    __syncthreads();  // the reflector buffers alias the Jacobi reduction buffers
  }

  // ---------------------------------------------------------- Jacobi sweeps
  // Odd-even transposition ordering of the positions 0..NP-1 (A_l = 2l,
  // B_l = 2l+1): type-0 rounds pair (A_l, B_l) inside each lane, type-1
  // rounds pair (B_l, A_{l+1}) across neighbouring lanes, and each pair is
  // exchanged after its rotation, so every two columns meet exactly once in
  // the NP rounds of a sweep.  Lanes >= H hold empty positions and keep them.
  for (int e = tid; e < 2 * 64; e += kSvThreads) {
    // identity updates (slots that no pair of the round writes)
    const int type = e >> 6;
    double *u = s_upd[type][e & 63];
    u[0] = type == 0 ? 1.0 : 0.0;  // A' = pa P + wa Q
    u[1] = type == 0 ? 0.0 : 1.0;
    u[2] = 0.0;
    u[3] = 0.0;
    u[4] = type == 0 ? 0.0 : 1.0;  // B' = pb R + wb S
    u[5] = type == 0 ? 1.0 : 0.0;
    u[6] = 0.0;
    u[7] = 0.0;
  }
  __syncthreads();
  const int NP = (nc + (nc & 1)) < 2 ? 2 : (nc + (nc & 1));
  const int H = NP / 2;
  const JacobiShared sh{s_red, s_upd, s_w};
  // wave-uniform: kept in scalar registers
  const double zw = __hiloint2double(__builtin_amdgcn_readfirstlane(__double2hiint(zero_w)),
                                     __builtin_amdgcn_readfirstlane(__double2loint(zero_w)));
  bool converged = false;
  int sweep = 0;
  for (; sweep < kMaxSweeps && !converged; ++sweep) {
    bool large = jacobi_round<0, true>(Ar, Ai, Br, Bi, sh, wave, H, zw);  // wave-uniform
    if (H > 1) large |= jacobi_round<1, false>(Ar, Ai, Br, Bi, sh, wave, H, zw);
    for (int half = 1; half < H; ++half) {
      large |= jacobi_round<0, false>(Ar, Ai, Br, Bi, sh, wave, H, zw);
      large |= jacobi_round<1, false>(Ar, Ai, Br, Bi, sh, wave, H, zw);
    }
    converged = __syncthreads_or(large ? 1 : 0) == 0;
  }

  // ---------------------------------------------------------- norms, order, k
  {
    double na = 0.0, nb = 0.0;
#pragma unroll
    for (int rr = 0; rr < kSvRows; ++rr) {
      na = fma(Ar[rr], Ar[rr], fma(Ai[rr], Ai[rr], na));
      nb = fma(Br[rr], Br[rr], fma(Bi[rr], Bi[rr], nb));
    }
    s_part[0][wave][lane] = na;
    s_part[1][wave][lane] = nb;
    __syncthreads();
    const int pr = tid >> 4, w = tid & 15;
    const double a = row_sum16(s_part[0][w][pr]), b = row_sum16(s_part[1][w][pr]);
    if (w == 0) {
      s_norm[2 * pr] = (2 * pr < NP) ? a : 0.0;
      s_norm[2 * pr + 1] = (2 * pr + 1 < NP) ? b : 0.0;
    }
    __syncthreads();
    if (tid < kSvMaxN) {
      const double v = s_norm[tid];
      int rank = 0;
#pragma unroll 1
      for (int u = 0; u < kSvMaxN; ++u) {
        const double o = s_norm[u];
        rank += (o > v || (o == v && u < tid)) ? 1 : 0;
      }
      s_rank[tid] = rank;
      s_sorted[rank] = v;
    }
    __syncthreads();
    if (tid == 0) {
      const int nsv = min(nr, nc);
      int nnz = 0;
#pragma unroll 1
      for (int u = 0; u < kSvMaxN; ++u) nnz += s_sorted[u] > zero_w ? 1 : 0;
      double total = 0.0;
#pragma unroll 1
      for (int u = kSvMaxN - 1; u >= 0; --u) total += s_sorted[u];
      int k;
      double disc = 0.0;
      if (gate) {
        int kcut = nsv;
        if (P.cutoff > 0.0) {
          // smallest k with sum_{r >= k} w_r <= cutoff * total
          double tail = 0.0;
          kcut = nsv;
    #pragma unroll 1
      for (int kk = nsv; kk >= 0; --kk) {
            if (kk < nsv) tail += s_sorted[kk];
            if (tail <= P.cutoff * total) kcut = kk;
            else break;
          }
        }
        k = max(1, min(min(P.chi, kcut), max(nnz, 1)));
        if (P.gate_split) {
          // theta = sum_r (L_r A_p)(R_r A_{p+1}) over the rank(G) terms of
          // the gate's operator-Schmidt decomposition: rank <= rank(G) Dm.
          // Rxx(phi) = cos(phi/2) II - i sin(phi/2) XX: a term counts when its
          // coefficient exceeds 1e-12 of the larger one (cos(pi/2) rounds to
          // ~6e-17, not zero); SWAP has four terms
          const double cmax = fmax(fabs(cg), fabs(sg));
          const int rg = st.op == OP_RXX
                             ? (fabs(cg) > 1e-12 * cmax ? 1 : 0) + (fabs(sg) > 1e-12 * cmax ? 1 : 0)
                             : 4;
          k = max(1, min(k, rg * Dm));
        }
        double kept = 0.0;
  #pragma unroll 1
      for (int u = k - 1; u >= 0; --u) kept += s_sorted[u];
        double tail = 0.0;
  #pragma unroll 1
      for (int u = kSvMaxN - 1; u >= k; --u) tail += s_sorted[u];
        disc = total > 0.0 ? tail / total : 0.0;
        s_nrm = kept > 0.0 ? 1.0 / sqrt(kept) : 1.0;
        P.disc[ci] += disc;
        P.maxdisc[ci] = fmax(P.maxdisc[ci], disc);
        if (k < nsv && s_sorted[0] > 0.0 &&
            (sqrt(s_sorted[k - 1]) - sqrt(s_sorted[k])) / sqrt(s_sorted[0]) < kDegenerateGap)
          P.degen[ci] += 1;
      } else {
        k = max(1, min(nsv, max(nnz, 1)));
        s_nrm = 1.0;
      }
      if (!converged) P.unconv[ci] += 1;
      s_k = k;
    }
    __syncthreads();
  }
  const int k = s_k;
  const double nrm = s_nrm;

  // ---------------------------------------------------------- write factors
  // zero both site tensors (padded blocks), then the isometric factor
  for (int e = tid; e < 2 * Pp * Pm; e += kSvThreads) Ap[e] = make_double2(0.0, 0.0);
  for (int e = tid; e < 2 * Pm * Pn; e += kSvThreads) Aq[e] = make_double2(0.0, 0.0);
  __syncthreads();
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int pos = 2 * lane + q;
    const int j = s_rank[pos];
    if (pos < NP && j < k) {
      const double inv = 1.0 / sqrt(s_norm[pos]);
#pragma unroll
      for (int rr = 0; rr < kSvRows; ++rr) {
        const int r = wave * kSvRows + rr;
        if (r < nr) {
          const double vr = (q == 0 ? Ar[rr] : Br[rr]) * inv;
          const double vi = (q == 0 ? Ai[rr] : Bi[rr]) * inv;
          if (right) Ap[(size_t(r / Dp) * Pp + r % Dp) * Pm + j] = make_double2(vr, vi);
          else Aq[(size_t(r / Dn) * Pm + j) * Pn + r % Dn] = make_double2(vr, -vi);
        }
      }
    }
  }
  __syncthreads();
  // projection: out[j][x] = sum_y conj(U[y][j]) S[y][x] in blocks of 64 rows
  // j (bond caps above 64 keep up to 128)
  project_rows(Ap, Aq, S, Dp, Dn, Pp, Pm, Pn, nr, ncs, k, 0, nrm, right, s_u.stage.L, s_u.stage.R);
  if (k > 64) project_rows(Ap, Aq, S, Dp, Dn, Pp, Pm, Pn, nr, ncs, k, 64, nrm, right, s_u.stage.L, s_u.stage.R);
  if (tid == 0) dims[p + 1] = k;
}

// Sum over the 32 lanes of lane half hf (rows 2 hf, 2 hf + 1), as the value
// of the half's first lane in every lane of the half: identical rotation
// parameters for all rows of a column pair.
__device__ inline double half_sum(double x, int hf) {
  x = row_sum16(x);
  x += __shfl_xor(x, 16, 64);
  return __shfl(x, hf << 5, 64);
}

// A value of lane 0, in every lane (wave-uniform control flow and
// identical rotation parameters across the rows of a column pair).
__device__ inline double lane0(double x) {
  return __hiloint2double(__builtin_amdgcn_readfirstlane(__double2hiint(x)),
                          __builtin_amdgcn_readfirstlane(__double2loint(x)));
}

// Two-site step of circuit ci whose Jacobi matrix may exceed 128 x 128 (a
// neighbouring bond above 64; one 1024-thread workgroup).  The same
// operation as svd_step -- pair product, theta, one-sided Jacobi on the
// columns, truncation by Eq. (8) with the bond cap, isometric factor from the
// normalised columns and the other factor as an exact projection -- with the
// matrices in the circuit's global scratch slot (L2-resident) instead of
// registers:
//   W: the pair product (row-major), then the Jacobi matrix M column-major
//      (column c at W + c kWideN, rows 0..255, zero beyond nr);
//   S: the projection source (row-major, row stride kWideN).
// M is first reduced as in svd_step (M <- M H_0 H_1 ..., Householder
// reflections from the right with the rows in order of decreasing norm), so
// that only its first min(nr, nc) columns carry more than rounding-level
// weight; the Jacobi sweeps then pair those columns in round-robin order
// (NP - 1 rounds of NP/2 disjoint pairs: every pair once per sweep).  Wave w
// rotates pairs w, w + 16, ... of a round, two at a time (one per lane half,
// each lane holding 8 rows of both columns), with one barrier per round.
__device__ __attribute__((noinline)) void svd_step_wide(const SvParams &P, const int64_t ci, const SimStep &st) {
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  __shared__ double w_norm[kWideN];   // squared norm of each Jacobi column (row norms during the LQ)
  __shared__ double w_sorted[kWideN]; // norms in decreasing order
  __shared__ int w_col[kWideN];       // column of each rank (pivot row of each LQ step)
  __shared__ double2 w_vec[kWideN];   // Householder vector of an LQ step
  __shared__ double2 w_dot[4][kWideN];// partial products row . conj(w)
  __shared__ double w_part[kSvWaves];
  __shared__ double w_beta;
  __shared__ int w_k;
  __shared__ double w_nrm, w_tot;

  int32_t *dims = P.dims + ci * (P.m + 1);
  const int p = st.p;
  const int Dp = dims[p], Dm = dims[p + 1], Dn = dims[p + 2];
  const int Pp = P.pad[p], Pm = P.pad[p + 1], Pn = P.pad[p + 2];
  double2 *Ap = P.f64 + ci * P.mps_stride + P.site_off[p];
  double2 *Aq = P.f64 + ci * P.mps_stride + P.site_off[p + 1];
  double2 *W = P.wscratch + int64_t(blockIdx.x) * kWideSlot;
  double2 *S = W + kWideN * kWideN;

  double cg = 1.0, sg = 0.0;
  if (st.op == OP_RXX) {
    const double xi = P.X[ci * P.ldx + st.fi], xj = P.X[ci * P.ldx + st.fj];
    const double phi = P.coef_xx * (1.0 - xi) * (1.0 - xj);
    sincos(0.5 * phi, &sg, &cg);
  }
  const bool right = (st.mode == GATE_RIGHT || st.mode == MOVE_RIGHT);
  const bool gate = (st.mode == GATE_RIGHT || st.mode == GATE_LEFT);
  int nr, nc, ncs;
  if (st.mode == GATE_RIGHT) { nr = 2 * Dp; nc = 2 * Dn; ncs = nc; }
  else if (st.mode == GATE_LEFT) { nr = 2 * Dn; nc = 2 * Dp; ncs = nc; }
  else if (st.mode == MOVE_RIGHT) { nr = 2 * Dp; nc = Dm; ncs = 2 * Dn; }
  else { nr = 2 * Dn; nc = Dm; ncs = 2 * Dp; }

  // ---------------------------------------------------------- pair product -> W
  // P[(s', a)][(t', b)] = sum_c A_p[s'][a][c] A_{p+1}[t'][c][b]; consecutive
  // threads take consecutive b (coalesced reads of A_{p+1})
  for (int e = tid; e < 4 * Dp * Dn; e += kSvThreads) {
    const int y = e / (2 * Dn), x = e % (2 * Dn);
    const double2 *ar = Ap + (size_t(y / Dp) * Pp + y % Dp) * Pm;
    const double2 *bc = Aq + size_t(x / Dn) * Pm * Pn + x % Dn;
    double re = 0.0, im = 0.0;
    for (int c = 0; c < Dm; ++c) {
      const double2 u = ar[c], v = bc[size_t(c) * Pn];
      re = fma(u.x, v.x, fma(-u.y, v.y, re));
      im = fma(u.x, v.y, fma(u.y, v.x, im));
    }
    W[size_t(y) * kWideN + x] = make_double2(re, im);
  }
  __syncthreads();
  // ---------------------------------------------------------- projection source -> S
  // gates: theta (absorb right) or theta^H (absorb left), which is also the
  // Jacobi matrix; centre moves: the identity theta P or its adjoint
  for (int e = tid; e < nr * ncs; e += kSvThreads) {
    const int r = e / ncs, c = e % ncs;
    double2 v;
    if (st.mode == GATE_RIGHT) v = theta_from_pair(W, st.op, cg, sg, Dp, Dn, r / Dp, r % Dp, c / Dn, c % Dn, kWideN);
    else if (st.mode == GATE_LEFT)
      v = cconj(theta_from_pair(W, st.op, cg, sg, Dp, Dn, c / Dp, c % Dp, r / Dn, r % Dn, kWideN));
    else if (st.mode == MOVE_RIGHT) v = W[size_t(r) * kWideN + c];
    else v = cconj(W[size_t(c) * kWideN + r]);
    S[size_t(r) * kWideN + c] = v;
  }
  __syncthreads();
  // ---------------------------------------------------------- Jacobi matrix -> W (column-major)
  const int NC = nc + (nc & 1);
  for (int e = tid; e < NC * kWideN; e += kSvThreads) {
    const int c = e / kWideN, r = e % kWideN;
    double2 v = make_double2(0.0, 0.0);
    if (r < nr && c < nc) {
      if (gate) v = S[size_t(r) * kWideN + c];
      else if (st.mode == MOVE_RIGHT) v = Ap[(size_t(r / Dp) * Pp + r % Dp) * Pm + c];
      else v = cconj(Aq[(size_t(r / Dn) * Pm + c) * Pn + r % Dn]);
    }
    W[size_t(c) * kWideN + r] = v;
  }
  // ||M||_F^2 (invariant under the rotations), from the values just written
  {
    double t = 0.0;
    for (int e = tid; e < NC * kWideN; e += kSvThreads) {
      const int c = e / kWideN, r = e % kWideN;
      if (r < nr && c < nc) {
        double2 v;
        if (gate) v = S[size_t(r) * kWideN + c];
        else if (st.mode == MOVE_RIGHT) v = Ap[(size_t(r / Dp) * Pp + r % Dp) * Pm + c];
        else v = cconj(Aq[(size_t(r / Dn) * Pm + c) * Pn + r % Dn]);
        t = fma(v.x, v.x, fma(v.y, v.y, t));
      }
    }
    t = wave_sum(t);
    if (lane == 0) w_part[wave] = t;
    __syncthreads();
    if (tid == 0) {
      double u = 0.0;
      for (int w = 0; w < kSvWaves; ++w) u += w_part[w];
      w_tot = u;
    }
    __syncthreads();
  }
  const double zero_w = lane0(kZeroWeight * w_tot);

  // ---------------------------------------------------------- LQ preconditioning
  // Step i reflects the i-th heaviest row x (restricted to columns >= i) onto
  // column i: w = x + e^{i arg x_i} |x| e_i, beta = 1 / (|x| (|x| + |x_i|)),
  // every row r <- r - beta (r . conj w) w.  Thread (r, q) = (tid % 256,
  // tid / 256) takes row r and the columns c = q mod 4.
  const int nref = min(nr, nc);
  {
    if (tid < kWideN) {
      double t = 0.0;
      if (tid < nr)
        for (int c = 0; c < nc; ++c) {
          const double2 v = W[size_t(c) * kWideN + tid];
          t = fma(v.x, v.x, fma(v.y, v.y, t));
        }
      w_norm[tid] = t;
    }
    __syncthreads();
    if (tid < kWideN) {
      const double v = w_norm[tid];
      int rank = 0;
#pragma unroll 1
      for (int u = 0; u < kWideN; ++u) {
        const double o = w_norm[u];
        rank += (o > v || (o == v && u < tid)) ? 1 : 0;
      }
      w_col[rank] = tid;
    }
    __syncthreads();
    const int r = tid & (kWideN - 1), q = tid >> 8;
    for (int i = 0; i < nref; ++i) {
      const int pv = w_col[i];
      if (tid < kWideN) {
        // the pivot row restricted to columns >= i, and |x|
        const double2 x = (tid >= i && tid < nc) ? W[size_t(tid) * kWideN + pv] : make_double2(0.0, 0.0);
        w_vec[tid] = x;
        const double n2 = wave_sum(fma(x.x, x.x, x.y * x.y));
        if (lane == 0) w_part[wave] = n2;
      }
      __syncthreads();
      if (tid == 0) {
        const double nx = sqrt(w_part[0] + w_part[1] + w_part[2] + w_part[3]);
        const double2 xi = w_vec[i];
        const double ax = sqrt(fma(xi.x, xi.x, xi.y * xi.y));
        const double pr = ax > 0.0 ? xi.x / ax : 1.0, pi = ax > 0.0 ? xi.y / ax : 0.0;
        w_vec[i] = make_double2(pr * (ax + nx), pi * (ax + nx));
        w_beta = nx > 0.0 ? 1.0 / (nx * (nx + ax)) : 0.0;
      }
      __syncthreads();
      double dr = 0.0, di = 0.0;
      if (r < nr)
        for (int c = i + q; c < nc; c += 4) {
          const double2 v = W[size_t(c) * kWideN + r], w = w_vec[c];
          dr = fma(v.x, w.x, fma(v.y, w.y, dr));
          di = fma(v.y, w.x, fma(-v.x, w.y, di));
        }
      w_dot[q][r] = make_double2(dr, di);
      __syncthreads();
      if (r < nr) {
        const double beta = w_beta;
        const double2 d0 = w_dot[0][r], d1 = w_dot[1][r], d2 = w_dot[2][r], d3 = w_dot[3][r];
        const double br = beta * ((d0.x + d1.x) + (d2.x + d3.x)), bi = beta * ((d0.y + d1.y) + (d2.y + d3.y));
        for (int c = i + q; c < nc; c += 4) {
          const double2 w = w_vec[c];
          double2 *m = W + size_t(c) * kWideN + r;
          const double2 v = *m;
          *m = make_double2(v.x - (br * w.x - bi * w.y), v.y - (br * w.y + bi * w.x));
        }
      }
      __syncthreads();  // the next step reads its pivot row and rewrites the LDS vectors
    }
  }

  // ---------------------------------------------------------- Jacobi sweeps
  const int NP = max(2, nref + (nref & 1));
  bool converged = false;
  const int half = NP / 2, rounds = NP - 1;
  // two pairs in flight per wave: lane half hf takes pair k0 + 16 hf, its
  // lane hl rows hl + 32 q (q < 8); sums over a half, then the value of the
  // half's first lane in all its lanes (the same rotation for every row)
  const int hf = lane >> 5, hl = lane & 31;
  for (int sweep = 0; sweep < kMaxSweeps && !converged; ++sweep) {
    bool large = false;
    for (int rd = 0; rd < rounds; ++rd) {
      for (int k0 = wave; k0 < half; k0 += 2 * kSvWaves) {
        // round-robin pairing: column NP-1 meets column rd, the others pair
        // symmetrically around rd (indices mod NP-1)
        const int k = k0 + hf * kSvWaves;
        const bool act = k < half;
        const int i = !act ? 0 : k == 0 ? NP - 1 : (rd + k) % rounds;
        const int j = !act ? 0 : k == 0 ? rd : (rd - k + rounds) % rounds;
        double2 *X = W + size_t(i) * kWideN + hl;
        double2 *Y = W + size_t(j) * kWideN + hl;
        double2 x[8], y[8];
        double a = 0.0, b = 0.0, gr = 0.0, gi = 0.0;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          x[q] = act ? X[32 * q] : make_double2(0.0, 0.0);
          y[q] = act ? Y[32 * q] : make_double2(0.0, 0.0);
          a = fma(x[q].x, x[q].x, fma(x[q].y, x[q].y, a));
          b = fma(y[q].x, y[q].x, fma(y[q].y, y[q].y, b));
          gr = fma(x[q].x, y[q].x, fma(x[q].y, y[q].y, gr));
          gi = fma(x[q].x, y[q].y, fma(-x[q].y, y[q].x, gi));
        }
        a = half_sum(a, hf);
        b = half_sum(b, hf);
        gr = half_sum(gr, hf);
        gi = half_sum(gi, hf);
        const double g2 = fma(gr, gr, gi * gi);
        if (act && a > zero_w && b > zero_w && g2 > (kJacobiTol * kJacobiTol) * (a * b)) {
          if (g2 > (kJacobiLarge * kJacobiLarge) * (a * b)) large = true;
          // the Hermitian 2 x 2 rotation of the pair's Gram block (as in
          // jacobi_round): X' = c X - s u Y, Y' = s X + c u Y,
          // u = conj<X,Y> / |<X,Y>|
          const double rg = rsqrt(g2);
          const double zeta = 0.5 * (b - a) * rg;
          const double den = fabs(zeta) + sqrt(fma(zeta, zeta, 1.0));
          double rdn = __builtin_amdgcn_rcp(den);
          rdn = fma(rdn, fma(-den, rdn, 1.0), rdn);
          rdn = fma(rdn, fma(-den, rdn, 1.0), rdn);
          const double t = zeta >= 0.0 ? rdn : -rdn;
          const double c = rsqrt(fma(t, t, 1.0));
          const double sn = c * t;
          const double ur = gr * rg, ui = -gi * rg;
          const double xr_ = -sn * ur, xi_ = -sn * ui;   // -s u
          const double yr_ = c * ur, yi_ = c * ui;       //  c u
#pragma unroll
          for (int q = 0; q < 8; ++q) {
            const double2 xo = x[q], yo = y[q];
            X[32 * q] = make_double2(fma(c, xo.x, fma(xr_, yo.x, -xi_ * yo.y)), fma(c, xo.y, fma(xr_, yo.y, xi_ * yo.x)));
            Y[32 * q] = make_double2(fma(sn, xo.x, fma(yr_, yo.x, -yi_ * yo.y)),
                                     fma(sn, xo.y, fma(yr_, yo.y, yi_ * yo.x)));
          }
        }
      }
      __syncthreads();  // the next round reads the columns this one wrote
    }
    converged = __syncthreads_or(large ? 1 : 0) == 0;
  }

  // ---------------------------------------------------------- norms, order, k
  for (int c = wave; c < kWideN; c += kSvWaves) {
    double t = 0.0;
    if (c < NP) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const double2 v = W[size_t(c) * kWideN + lane + 64 * q];
        t = fma(v.x, v.x, fma(v.y, v.y, t));
      }
      t = wave_sum(t);
    }
    if (lane == 0) w_norm[c] = t;
  }
  __syncthreads();
  if (tid < kWideN) {
    const double v = w_norm[tid];
    int rank = 0;
#pragma unroll 1
    for (int u = 0; u < kWideN; ++u) {
      const double o = w_norm[u];
      rank += (o > v || (o == v && u < tid)) ? 1 : 0;
    }
    w_sorted[rank] = v;
    w_col[rank] = tid;
  }
  __syncthreads();
  if (tid == 0) {
    const int nsv = min(nr, nc);
    int nnz = 0;
#pragma unroll 1
    for (int u = 0; u < kWideN; ++u) nnz += w_sorted[u] > zero_w ? 1 : 0;
    double total = 0.0;
#pragma unroll 1
    for (int u = kWideN - 1; u >= 0; --u) total += w_sorted[u];
    int k;
    if (gate) {
      int kcut = nsv;
      if (P.cutoff > 0.0) {
        // smallest k with sum_{r >= k} w_r <= cutoff * total
        double tail = 0.0;
#pragma unroll 1
        for (int kk = nsv; kk >= 0; --kk) {
          if (kk < nsv) tail += w_sorted[kk];
          if (tail <= P.cutoff * total) kcut = kk;
          else break;
        }
      }
      k = max(1, min(min(P.chi, kcut), max(nnz, 1)));
      if (P.gate_split) {
        const double cmax = fmax(fabs(cg), fabs(sg));
        const int rg = st.op == OP_RXX ? (fabs(cg) > 1e-12 * cmax ? 1 : 0) + (fabs(sg) > 1e-12 * cmax ? 1 : 0) : 4;
        k = max(1, min(k, rg * Dm));
      }
      double kept = 0.0;
#pragma unroll 1
      for (int u = k - 1; u >= 0; --u) kept += w_sorted[u];
      double tail = 0.0;
#pragma unroll 1
      for (int u = kWideN - 1; u >= k; --u) tail += w_sorted[u];
      const double disc = total > 0.0 ? tail / total : 0.0;
      w_nrm = kept > 0.0 ? 1.0 / sqrt(kept) : 1.0;
      P.disc[ci] += disc;
      P.maxdisc[ci] = fmax(P.maxdisc[ci], disc);
      if (k < nsv && w_sorted[0] > 0.0 &&
          (sqrt(w_sorted[k - 1]) - sqrt(w_sorted[k])) / sqrt(w_sorted[0]) < kDegenerateGap)
        P.degen[ci] += 1;
    } else {
      k = max(1, min(nsv, max(nnz, 1)));
      w_nrm = 1.0;
    }
    if (!converged) P.unconv[ci] += 1;
    w_k = k;
  }
  __syncthreads();
  const int k = w_k;
  const double nrm = w_nrm;

  // ---------------------------------------------------------- write factors
  for (int e = tid; e < 2 * Pp * Pm; e += kSvThreads) Ap[e] = make_double2(0.0, 0.0);
  for (int e = tid; e < 2 * Pm * Pn; e += kSvThreads) Aq[e] = make_double2(0.0, 0.0);
  __syncthreads();
  // isometric factor: U[:, j] = column w_col[j] / its norm
  for (int e = tid; e < k * nr; e += kSvThreads) {
    const int j = e / nr, r = e % nr;
    const int c = w_col[j];
    const double inv = 1.0 / sqrt(w_norm[c]);
    const double2 v = W[size_t(c) * kWideN + r];
    const double vr = v.x * inv, vi = v.y * inv;
    if (right) Ap[(size_t(r / Dp) * Pp + r % Dp) * Pm + j] = make_double2(vr, vi);
    else Aq[(size_t(r / Dn) * Pm + j) * Pn + r % Dn] = make_double2(vr, -vi);
  }
  // projection: out[j][x] = nrm sum_y conj(U[y][j]) S[y][x]; consecutive
  // threads take consecutive x (one column of W per wave, coalesced rows of S)
  for (int e = tid; e < k * ncs; e += kSvThreads) {
    const int j = e / ncs, x = e % ncs;
    const int c = w_col[j];
    const double inv = 1.0 / sqrt(w_norm[c]);
    const double2 *u = W + size_t(c) * kWideN;
    double re = 0.0, im = 0.0;
    for (int y = 0; y < nr; ++y) {
      const double2 uv = u[y], sv = S[size_t(y) * kWideN + x];
      const double ur = uv.x * inv, ui = uv.y * inv;
      re = fma(ur, sv.x, fma(ui, sv.y, re));
      im = fma(ur, sv.y, fma(-ui, sv.x, im));
    }
    if (right) Aq[(size_t(x / Dn) * Pm + j) * Pn + x % Dn] = make_double2(nrm * re, nrm * im);
    else Ap[(size_t(x / Dp) * Pp + x % Dp) * Pm + j] = make_double2(nrm * re, -nrm * im);
  }
  if (tid == 0) dims[p + 1] = k;
}

// Rz on a run of gate records (Fig. 1a) for circuit ci: A[site][s] *=
// exp(-/+ i theta / 2).  The records of a run act on distinct sites.
__device__ inline void rz_run(const SvParams &P, int64_t ci, const qk_gate *recs, int n_recs, double coef_z) {
  for (int r = 0; r < n_recs; ++r) {
    const qk_gate g = recs[r];
    const double th = coef_z * P.X[ci * P.ldx + g.feat_i];
    double sn, cs;
    sincos(0.5 * th, &sn, &cs);
    const int pl = P.pad[g.site], pr = P.pad[g.site + 1];
    double2 *A = P.f64 + ci * P.mps_stride + P.site_off[g.site];
    const int half = pl * pr;
    for (int e = threadIdx.x; e < 2 * half; e += kSvThreads) {
      const double2 v = A[e];
      const double ph = e < half ? -sn : sn;  // s = 0: exp(-i th/2), s = 1: exp(+i th/2)
      A[e] = make_double2(cs * v.x - ph * v.y, cs * v.y + ph * v.x);
    }
  }
}

// Steps [s0, s1) of the step list for every circuit, one workgroup each.
// Circuits do not wait for one another between steps, so a launch lasts as
// long as the slowest circuit's total over the chunk rather than the sum,
// over the steps, of each step's slowest SVD (whose sweep count varies from
// circuit to circuit).
__global__ __launch_bounds__(kSvThreads) void sim_steps_kernel(SvParams P, const SimStep *steps, int s0, int s1,
                                                              const qk_gate *recs, double coef_z) {
  const int64_t ci = circuit_of(P.base);
  if (ci >= P.n) return;
  for (int s = s0; s < s1; ++s) {
    const SimStep st = steps[s];
    if (st.kind == STEP_RZ) {
      rz_run(P, ci, recs + st.r0, st.nr, coef_z);
    } else {
      const int32_t *dims = P.dims + ci * (P.m + 1);
      if (P.wscratch && (dims[st.p] > kWideFrom || dims[st.p + 2] > kWideFrom)) svd_step_wide(P, ci, st);
      else svd_step(P, ci, st);
    }
    __syncthreads();  // the next step reads the tensors and bond dims this one wrote
    if (P.trace && st.kind == STEP_TWO_SITE && st.r0 >= 0 && threadIdx.x < 64) {
      // memory trace after a two-qubit gate: the bond at its cut and
      // sum_l D_l D_{l+1} (complex entries per physical index) over the MPS.
      // Only reads of the bond dims, which the next step's first thread
      // rewrites after this wave has passed here.
      const int32_t *dims = P.dims + ci * (P.m + 1);
      int acc = 0;
      for (int l = threadIdx.x; l < P.m; l += 64) acc += dims[l] * dims[l + 1];
      for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
      if (threadIdx.x == 0) {
        int32_t *t = P.trace + (ci * P.trace_n2q + st.r0) * 2;
        t[0] = dims[st.p + 1];
        t[1] = acc;
      }
    }
  }
}

__global__ void init_plus_kernel(double2 *f64, int64_t mps_stride, const int64_t *site_off, const int32_t *pad,
                                 int32_t *dims, int32_t m, int64_t n, const int64_t *base) {
  const int64_t ci = circuit_of(base);
  if (ci >= n) return;
  const double h = 0.70710678118654752440;
  for (int l = threadIdx.x; l <= m; l += blockDim.x) {
    dims[ci * (m + 1) + l] = 1;
    if (l < m) {
      double2 *A = f64 + ci * mps_stride + site_off[l];
      A[0] = make_double2(h, 0.0);                                  // s = 0, a = 0, b = 0
      A[size_t(pad[l]) * pad[l + 1]] = make_double2(h, 0.0);        // s = 1
    }
  }
}

__global__ void normalize_last_kernel(double2 *f64, int64_t mps_stride, const int64_t *site_off,
                                      const int32_t *pad, int32_t m, int64_t n, const int64_t *base) {
  const int64_t ci = circuit_of(base);
  if (ci >= n) return;
  __shared__ double s_red[256];
  double2 *A = f64 + ci * mps_stride + site_off[m - 1];
  const int cnt = 2 * pad[m - 1] * pad[m];
  double acc = 0.0;
  for (int e = threadIdx.x; e < cnt; e += blockDim.x) acc = fma(A[e].x, A[e].x, fma(A[e].y, A[e].y, acc));
  s_red[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (int(threadIdx.x) < o) s_red[threadIdx.x] += s_red[threadIdx.x + o];
    __syncthreads();
  }
  const double nrm = s_red[0];
  if (nrm <= 0.0) return;
  const double inv = 1.0 / sqrt(nrm);
  for (int e = threadIdx.x; e < cnt; e += blockDim.x) A[e] = make_double2(A[e].x * inv, A[e].y * inv);
}

// First circuit of the next graph replay (one thread).
__global__ void set_base_kernel(int64_t *base, int64_t v, int64_t add) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *base = add ? *base + v : v;
}

}  // namespace

// FP64 tensors of src copied into dst, whose pads are no larger (and no
// smaller than every bond dimension of src): block (mps i, site l) of dst is
// [s][r][c] with r < dst pad[l], c < dst pad[l+1].  Grid (m, MPS chunk).
__global__ __launch_bounds__(256) void repad_f64_kernel(const double2 *__restrict__ src, double2 *__restrict__ dst,
                                                        const int32_t *__restrict__ spad,
                                                        const int32_t *__restrict__ dpad,
                                                        const int64_t *__restrict__ soff,
                                                        const int64_t *__restrict__ doff, int64_t sstride,
                                                        int64_t dstride, int32_t m, int64_t n) {
  const int l = blockIdx.x;
  const int64_t i = blockIdx.y;
  if (l >= m || i >= n) return;
  const int sl = spad[l], sr = spad[l + 1], dl = dpad[l], dr = dpad[l + 1];
  const double2 *a = src + i * sstride + soff[l];
  double2 *b = dst + i * dstride + doff[l];
  for (int e = threadIdx.x; e < 2 * dl * dr; e += blockDim.x) {
    const int s = e / (dl * dr), r = (e / dr) % dl, c = e % dr;
    b[e] = a[(size_t(s) * sl + r) * sr + c];
  }
}

qk_status launch_repad_f64(const qk_mps_batch *src, qk_mps_batch *dst, hipStream_t stream) {
  if (src->n == 0) return QK_OK;
  for (int l = 0; l <= src->m; ++l)
    if (dst->pad[l] > src->pad[l]) return fail(QK_EINVAL, "repad to a larger pad");
  const int64_t chunk = 65535;
  for (int64_t i0 = 0; i0 < src->n; i0 += chunk) {
    const int64_t cnt = std::min(chunk, src->n - i0);
    hipLaunchKernelGGL(repad_f64_kernel, dim3(unsigned(src->m), unsigned(cnt)), dim3(256), 0, stream,
                       src->f64 + i0 * src->mps_stride, dst->f64 + i0 * dst->mps_stride, src->pad_dev,
                       dst->pad_dev, src->site_off_dev, dst->site_off_dev, src->mps_stride, dst->mps_stride,
                       src->m, cnt);
    QK_HIP_CHECK(hipGetLastError());
  }
  return QK_OK;
}

qk_status run_simulation(qk_mps_batch *b, const double *features_dev, const std::vector<qk_gate> &gates,
                         const qk_circuit_spec &spec, int chi, double cutoff, hipStream_t stream, qk_progress_fn fn,
                         void *user, int64_t every, int64_t graph_circuits, int32_t *trace) {
  const int64_t n = b->n;
  const int m = b->m;
  int n2q = 0;
  for (const auto &g : gates) n2q += g.op != OP_RZ ? 1 : 0;
  b->n_two_qubit_gates = n2q;
  if (n == 0) return QK_OK;
  if (n > 0x7fffffff) return fail(QK_EINVAL, "too many points for one launch");
  if (graph_circuits > 0 && fn) return fail(QK_EINVAL, "progress callbacks are not available with graph replay");

  // reject non-finite features before any launch
  {
    std::vector<double> xh(size_t(n) * m);
    QK_HIP_CHECK(hipMemcpyAsync(xh.data(), features_dev, sizeof(double) * xh.size(), hipMemcpyDeviceToHost, stream));
    QK_HIP_CHECK(hipStreamSynchronize(stream));
    for (double v : xh)
      if (!std::isfinite(v)) return fail(QK_EINVAL, "non-finite feature value");
  }

  // Graph mode: one graph records the launches that simulate `grid` circuits
  // from start to end and is replayed until every circuit is done; otherwise
  // the launches cover the whole batch.
  const bool graph = graph_circuits > 0;
  const int64_t grid = graph ? std::min(n, graph_circuits) : n;
  const int64_t replays = (n + grid - 1) / grid;

  // The step list shared by every circuit: runs of Rz records, centre moves
  // and two-qubit gates in circuit order, then the final moves to the last
  // site.  gate_no[i] is the number of two-qubit gates done after step i
  // when step i is a gate, and 0 otherwise.
  std::vector<SimStep> steps;
  std::vector<int64_t> gate_no;
  {
    std::vector<int> next2q(gates.size(), -1);  // site of the next two-qubit gate
    int nxt = -1;
    for (int gi = int(gates.size()) - 1; gi >= 0; --gi) {
      next2q[gi] = nxt;
      if (gates[gi].op != OP_RZ) nxt = gates[gi].site;
    }
    auto push = [&](const SimStep &x, int64_t g) {
      steps.push_back(x);
      gate_no.push_back(g);
    };
    int center = 0;
    int64_t d2q = 0;
    size_t gi = 0;
    while (gi < gates.size()) {
      if (gates[gi].op == OP_RZ) {
        size_t ge = gi;
        while (ge < gates.size() && gates[ge].op == OP_RZ) ++ge;
        push({STEP_RZ, 0, 0, 0, -1, -1, int32_t(gi), int32_t(ge - gi)}, 0);
        gi = ge;
        continue;
      }
      const int p = gates[gi].site;
      for (; center < p; ++center) push({STEP_TWO_SITE, center, MOVE_RIGHT, OP_ID, -1, -1, -1, 0}, 0);
      for (; center > p + 1; --center) push({STEP_TWO_SITE, center - 1, MOVE_LEFT, OP_ID, -1, -1, -1, 0}, 0);
      const bool absorb_right = next2q[gi] < 0 || next2q[gi] > p;
      push({STEP_TWO_SITE, p, absorb_right ? GATE_RIGHT : GATE_LEFT, gates[gi].op == 1 ? OP_RXX : OP_SWAP,
            gates[gi].feat_i, gates[gi].feat_j, int32_t(d2q), 0},
           d2q + 1);
      ++d2q;
      center = absorb_right ? p + 1 : p;
      ++gi;
    }
    for (; center < m - 1; ++center) push({STEP_TWO_SITE, center, MOVE_RIGHT, OP_ID, -1, -1, -1, 0}, 0);
  }

  // Device buffers: gate records, step list, SVD scratch of one slot per
  // workgroup of a launch, and (graph mode) the first circuit of a replay.
  const DevAlloc al = allocator_for_current_device();
  void *recs_dev = nullptr, *steps_dev = nullptr, *scratch = nullptr, *wscratch = nullptr, *base_dev = nullptr;
  auto release = [&]() {
    for (void *ptr : {recs_dev, steps_dev, scratch, wscratch, base_dev})
      if (ptr) dev_free(al, ptr, stream, true);
  };
  recs_dev = dev_alloc(al, sizeof(qk_gate) * std::max<size_t>(gates.size(), 1), stream, true);
  steps_dev = dev_alloc(al, sizeof(SimStep) * std::max<size_t>(steps.size(), 1), stream, true);
  scratch = dev_alloc(al, sizeof(double2) * 2 * kSvMaxN * kSvMaxN * size_t(grid), stream, true);
  if (chi > kWideFrom) wscratch = dev_alloc(al, sizeof(double2) * kWideSlot * size_t(grid), stream, true);
  if (graph) base_dev = dev_alloc(al, 256, stream, true);
  if (!recs_dev || !steps_dev || !scratch || (chi > kWideFrom && !wscratch) || (graph && !base_dev)) {
    release();
    return fail(QK_ENOMEM, "device allocation of the simulation buffers failed");
  }
  if ((!gates.empty() && hipMemcpyAsync(recs_dev, gates.data(), sizeof(qk_gate) * gates.size(),
                                        hipMemcpyHostToDevice, stream) != hipSuccess) ||
      (!steps.empty() && hipMemcpyAsync(steps_dev, steps.data(), sizeof(SimStep) * steps.size(),
                                        hipMemcpyHostToDevice, stream) != hipSuccess)) {
    (void)hipGetLastError();
    release();
    return fail(QK_EDEVICE, "copy of the gate and step lists failed");
  }
  const auto *recs = static_cast<const qk_gate *>(recs_dev);
  const auto *steps_d = static_cast<const SimStep *>(steps_dev);
  auto *base = static_cast<int64_t *>(base_dev);

  SvParams P{};
  P.f64 = b->f64;
  P.mps_stride = b->mps_stride;
  P.site_off = b->site_off_dev;
  P.pad = b->pad_dev;
  P.dims = b->dims_dev;
  P.m = m;
  P.chi = chi;
  P.gate_split = spec.gate_split;
  P.coef_xx = spec.coef_xx;
  P.cutoff = cutoff;
  P.X = features_dev;
  P.ldx = m;
  P.scratch = static_cast<double2 *>(scratch);
  P.wscratch = static_cast<double2 *>(wscratch);
  P.disc = b->disc_dev;
  P.maxdisc = b->maxdisc_dev;
  P.degen = b->degen_dev;
  P.unconv = b->unconv_dev;
  P.n = n;
  P.trace = trace;
  P.trace_n2q = n2q;
  P.base = base;

  // The launches of one pass over `grid` circuits on stream s: the |+>
  // state, the step list in launches of at most kMaxChunkSteps steps (a
  // launch also ends where a progress callback is due), the normalisation of
  // the last site, and in graph mode the advance of the first circuit.
  constexpr size_t kMaxChunkSteps = 256;
  auto pass = [&](hipStream_t s) -> qk_status {
    hipLaunchKernelGGL(init_plus_kernel, dim3(unsigned(grid)), dim3(64), 0, s, b->f64, b->mps_stride,
                       b->site_off_dev, b->pad_dev, b->dims_dev, m, n, P.base);
    if (hipGetLastError() != hipSuccess) return fail(QK_EDEVICE, "initial-state launch failed");
    size_t s0 = 0;
    while (s0 < steps.size()) {
      size_t s1 = s0;
      bool report = false;
      while (s1 < steps.size() && s1 - s0 < kMaxChunkSteps) {
        const int64_t g = gate_no[s1++];
        if (g > 0 && fn && every > 0 && g % every == 0) {
          report = true;
          break;
        }
      }
      hipLaunchKernelGGL(sim_steps_kernel, dim3(unsigned(grid)), dim3(kSvThreads), 0, s, P, steps_d, int(s0),
                         int(s1), recs, spec.coef_z);
      if (hipGetLastError() != hipSuccess) return fail(QK_EDEVICE, "simulation launch failed");
      if (report) {
        if (hipStreamSynchronize(s) != hipSuccess) return fail(QK_EDEVICE, "simulation step failed");
        if (fn(gate_no[s1 - 1], n2q, user) != 0)
          return fail(QK_EABORTED, "simulation aborted by the progress callback");
      }
      s0 = s1;
    }
    hipLaunchKernelGGL(normalize_last_kernel, dim3(unsigned(grid)), dim3(256), 0, s, b->f64, b->mps_stride,
                       b->site_off_dev, b->pad_dev, m, n, P.base);
    if (hipGetLastError() != hipSuccess) return fail(QK_EDEVICE, "normalisation launch failed");
    if (graph) {
      hipLaunchKernelGGL(set_base_kernel, dim3(1), dim3(64), 0, s, base, grid, int64_t(1));
      if (hipGetLastError() != hipSuccess) return fail(QK_EDEVICE, "replay-advance launch failed");
    }
    return QK_OK;
  };

  qk_status st = QK_OK;
  if (!graph) {
    st = pass(stream);
  } else {
    // The pass is recorded by stream capture on a private stream (the
    // caller's stream may be the legacy null stream, which cannot be
    // captured) and replayed `replays` times there; events order the
    // private stream after the caller's earlier work and the caller's stream
    // after the replays.  The first circuit starts at 0 (a kernel, not a
    // memset, so that the sequence could itself be captured).
    hipLaunchKernelGGL(set_base_kernel, dim3(1), dim3(64), 0, stream, base, int64_t(0), int64_t(0));
    if (hipGetLastError() != hipSuccess) {
      release();
      return fail(QK_EDEVICE, "replay-start launch failed");
    }
    hipStream_t cap = nullptr;
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    hipGraph_t g = nullptr;
    hipGraphExec_t exec = nullptr;
    if (hipStreamCreateWithFlags(&cap, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&ev_in, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&ev_out, hipEventDisableTiming) != hipSuccess ||
        hipEventRecord(ev_in, stream) != hipSuccess || hipStreamWaitEvent(cap, ev_in, 0) != hipSuccess) {
      st = fail(QK_EDEVICE, "graph stream set-up failed");
    } else if (hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal) != hipSuccess) {
      st = fail(QK_EDEVICE, "graph capture failed to start");
    } else {
      st = pass(cap);
      // the capture is ended on every path so that the stream stays usable
      const hipError_t ce = hipStreamEndCapture(cap, &g);
      if (st == QK_OK && ce != hipSuccess) st = fail(QK_EDEVICE, std::string("graph capture failed: ") + hipGetErrorString(ce));
      if (st == QK_OK) {
        const hipError_t ie = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
        if (ie != hipSuccess) st = fail(QK_EDEVICE, std::string("graph instantiation failed: ") + hipGetErrorString(ie));
      }
      for (int64_t r = 0; st == QK_OK && r < replays; ++r) {
        const hipError_t le = hipGraphLaunch(exec, cap);
        if (le != hipSuccess) st = fail(QK_EDEVICE, std::string("graph launch failed: ") + hipGetErrorString(le));
      }
    }
    if (cap) {
      // the caller's stream continues after the replays
      if (ev_out && hipEventRecord(ev_out, cap) == hipSuccess) (void)hipStreamWaitEvent(stream, ev_out, 0);
      (void)hipStreamSynchronize(cap);
    }
    if (exec) (void)hipGraphExecDestroy(exec);
    if (g) (void)hipGraphDestroy(g);
    if (ev_in) (void)hipEventDestroy(ev_in);
    if (ev_out) (void)hipEventDestroy(ev_out);
    if (cap) (void)hipStreamDestroy(cap);
  }
  release();
  if (st != QK_OK) {
    (void)hipStreamSynchronize(stream);
    return st;
  }
  QK_HIP_CHECK(hipStreamSynchronize(stream));
  if (fn && fn(n2q, n2q, user) != 0) return fail(QK_EABORTED, "simulation aborted by the progress callback");
  return QK_OK;
}

}  // namespace qk
