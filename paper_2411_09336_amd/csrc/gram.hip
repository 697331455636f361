// Gram matrix of MPS overlaps on MI355X (gfx950).
//
// For every pair (bra a_i, ket b_j) the overlap <a_i|b_j> is contracted site
// by site as in Fig. 2 of the paper:
//     E_0 = [[1]],   E_{l+1} = sum_s A_a[l][s]^H E_l A_b[l][s],
// and K[i][j] = |E_m|^2 (Eq. (1)).  Each site update is two complex GEMMs:
//     GEMM1  T_s  = E A_b[s]              (contract the ket's left bond)
//     GEMM2  E'^T = sum_s T_s^T conj(A_a[s])   (contract the bra's left bond)
// E (and T) live in LDS; MFMA accumulator rows of one GEMM are laid out so
// that they feed the next GEMM as A-operand rows, and the site tensors stream
// from HBM / L2 in MFMA fragment order.
//
// Four arithmetic forms:
//  * FP64 and FP32: plain operands, v_mfma_f64_16x16x4 / v_mfma_f32_16x16x4,
//    E rescaled by a power of two after every site (exact) against underflow;
//    four waves per pair, wave w computes E' for the ket column block w.
//  * split-BF16 and split-int8: 31-bit fixed-point codes with one exponent
//    per row (E, T^T) or column (site tensors), cut into four 8-bit digits;
//    the digit products are carried by bf16 MFMAs (exact leading-digit
//    accumulator, FP64 combination) or by int8 MFMAs (all products exact in
//    int32).  These forms reach FP64-level accuracy (|dK| ~ 1e-8) on
//    low-precision matrix cores.
//
// Pairs are taken from device work queues over 16 x 16 pair tiles that may
// span several jobs (batches with different qubit counts and pads).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "qk_internal.h"

namespace qk {

namespace {

constexpr int kDefaultTileSide = 16;   // pair tiles are side x side entries

// Site tensors and K live in global memory, but their pointers come from the
// job table, so the compiler cannot infer the address space and would emit
// flat accesses, which also count against the LDS wait counter (an LDS wait
// then waits for every global load in flight).  Accesses go through these
// global-address-space views instead.
template <typename T>
__device__ inline const T __attribute__((address_space(1))) *gview(const T *p) {
  return (const T __attribute__((address_space(1))) *)p;
}
template <typename T>
__device__ inline T __attribute__((address_space(1))) *gview_rw(T *p) {
  return (T __attribute__((address_space(1))) *)p;
}

// Complex loads through global views (native vector types: the HIP vector
// structs cannot be copied from address-space-qualified lvalues).
template <typename T2>
__device__ inline T2 gload_c(const T2 *p) {
  typedef decltype(T2().x) T;
  typedef T v2 __attribute__((ext_vector_type(2)));
  const v2 v = *gview(reinterpret_cast<const v2 *>(p));
  T2 r;
  r.x = v.x;
  r.y = v.y;
  return r;
}
template <typename T2>
__device__ inline void gstore_c(T2 *p, T2 v) {
  typedef decltype(T2().x) T;
  typedef T v2 __attribute__((ext_vector_type(2)));
  v2 w;
  w.x = v.x;
  w.y = v.y;
  *gview_rw(reinterpret_cast<v2 *>(p)) = w;
}
constexpr int kThreads = 256;

struct GramTile {
  int32_t job;
  int32_t ti;
  int32_t tj;
  int32_t unused;
};

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x8 __attribute__((__vector_size__(8 * sizeof(__bf16))));

__device__ inline f32x4 mma(float a, float b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ inline f64x4 mma(double a, double b, f64x4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ inline f32x4 mma16(uint4 a, uint4 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a),
                                                 __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
}

__device__ inline uint4 neg_bf16(uint4 v) {
  return make_uint4(v.x ^ 0x80008000u, v.y ^ 0x80008000u, v.z ^ 0x80008000u, v.w ^ 0x80008000u);
}

__device__ inline float wave_max(float v) {
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ inline double wave_max(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

// Work queues: nq queues, one per XCD (workgroups are dispatched to the
// XCDs round-robin, so workgroup b runs on XCD b mod 8).  Queue x serves the
// tiles x, x + nq, x + 2 nq, ... so that the workgroups of one XCD work on
// the same tile and share its site tensors in their L2.  Counters are 64
// bytes apart.
constexpr int kQueues = 8;
constexpr int kCounterStride = 8;   // unsigned long long elements
constexpr size_t kGramCounterBytes = sizeof(unsigned long long) * kQueues * kCounterStride;

// Decode the next pair of this workgroup's queue.  Returns false when the
// queue is empty; *valid is false for pairs outside the job's range or below
// the diagonal.
__device__ inline bool next_pair(const GramJobDev *jobs, const GramTile *tiles, int64_t n_tiles, int nq, int side,
                                 unsigned long long *counters, int64_t *s_slot, int *job, int64_t *i,
                                 int64_t *j, bool *valid) {
  const int tile_pairs = side * side;
  const int x = int(blockIdx.x % unsigned(nq));
  if (threadIdx.x == 0) *s_slot = int64_t(atomicAdd(counters + x * kCounterStride, 1ull));
  __syncthreads();
  // the slot is the same for the whole workgroup: make it wave-uniform so
  // that the job, pair and site addresses derived from it live in scalar
  // registers
  const uint64_t pv = uint64_t(*s_slot);
  const int64_t p = int64_t((uint64_t(uint32_t(__builtin_amdgcn_readfirstlane(uint32_t(pv >> 32)))) << 32) |
                            uint32_t(__builtin_amdgcn_readfirstlane(uint32_t(pv))));
  __syncthreads();
  const int64_t tile = x + int64_t(nq) * (p / tile_pairs);
  if (tile >= n_tiles) return false;
  const GramTile t = tiles[tile];
  const int q = int(p % tile_pairs);
  const GramJobDev &J = jobs[t.job];
  const int64_t li = int64_t(t.ti) * side + q / side;
  const int64_t lj = int64_t(t.tj) * side + q % side;
  *job = t.job;
  *i = li;
  *j = lj;
  bool ok = li < J.na && lj < J.nb;
  if (ok && J.upper) ok = (J.b0 + lj) >= (J.a0 + li);
  *valid = ok;
  return true;
}

__device__ inline void write_k(const GramJobDev &J, int64_t li, int64_t lj, double k) {
  const auto K = gview_rw(J.K);
  K[li * J.ldk + lj] = k;
  if (J.upper) {
    // mirror inside the written block when the transposed entry is in range
    const int64_t gi = J.a0 + li, gj = J.b0 + lj;
    const int64_t mi = gj - J.a0, mj = gi - J.b0;
    if (gi != gj && mi >= 0 && mi < J.na && mj >= 0 && mj < J.nb) K[mi * J.ldk + mj] = k;
  }
}

// Row held by element e of lane j + 16 g in a 16 x 16 MFMA accumulator: the
// FP32 and BF16 instructions hold rows 4 g + e, the FP64 instruction holds
// rows 4 e + g (both verified on gfx950).
template <typename T>
__device__ constexpr int acc_row(int g, int e) {
  return sizeof(T) == 8 ? 4 * e + g : 4 * g + e;
}

// ------------------------------------------------------------------------
// FP64 / FP32 forms.  E in LDS in MFMA A-operand fragment order:
// fragment (rt, kq) holds E[16 rt + i][4 kq + g] at lane i + 16 g, as an
// interleaved complex value.
template <typename T, typename V4, typename T2, int MAXP>
__device__ void overlap_plain(const GramJobDev &J, int64_t ia, int64_t ib, T2 *E, T *s_red,
                              T &ov_re, T &ov_im, int &ov_exp) {
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int j = lane & 15, g = lane >> 4;
  const T2 *abase = reinterpret_cast<const T2 *>(J.a_base) + ia * J.a_stride;
  const T2 *bbase = reinterpret_cast<const T2 *>(J.b_base) + ib * J.b_stride;
  {
    const int n0 = gview(J.a_pad)[0] * gview(J.b_pad)[0];
    for (int x = tid; x < n0; x += kThreads) {
      T2 z;
      z.x = T(0);
      z.y = T(0);
      E[x] = z;
    }
    __syncthreads();
    if (tid == 0) E[0].x = T(1);
    __syncthreads();
  }
  int expacc = 0;
  constexpr int NT = MAXP / 16;
  constexpr int CT_PER_WAVE = (NT + 3) / 4;
  for (int l = 0; l < J.m; ++l) {
    const int Da = gview(J.a_pad)[l], Dan = gview(J.a_pad)[l + 1], Db = gview(J.b_pad)[l], Dbn = gview(J.b_pad)[l + 1];
    const T2 *A = abase + gview(J.a_off)[l];
    const T2 *B = bbase + gview(J.b_off)[l];
    const int nrt = Da / 16, nkq = Db / 4, nat = Dan / 16, nct = Dbn / 16, nkqn = Dbn / 4;
    V4 Ep[CT_PER_WAVE][NT][2];
    T lmax = T(0);
#pragma unroll
    for (int c = 0; c < CT_PER_WAVE; ++c) {
      const int ct = wave + 4 * c;
#pragma unroll
      for (int at = 0; at < NT; ++at) {
        Ep[c][at][0] = V4{0, 0, 0, 0};
        Ep[c][at][1] = V4{0, 0, 0, 0};
      }
      if (ct >= nct) continue;
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        V4 Tt[NT][2];
#pragma unroll
        for (int rt = 0; rt < NT; ++rt) {
          Tt[rt][0] = V4{0, 0, 0, 0};
          Tt[rt][1] = V4{0, 0, 0, 0};
        }
        // GEMM1: T_s[a][b'] = sum_b E[a][b] B_s[b][b'],  b' in block ct
        for (int kq = 0; kq < nkq; ++kq) {
          const T2 bv = gload_c(B + (size_t(s) * Db + 4 * kq + g) * Dbn + 16 * ct + j);
          const T bneg = -bv.y;
#pragma unroll
          for (int rt = 0; rt < NT; ++rt) {
            if (rt < nrt) {
              const T2 ev = E[(rt * nkq + kq) * 64 + lane];
              Tt[rt][0] = mma(ev.x, bv.x, Tt[rt][0]);
              Tt[rt][0] = mma(ev.y, bneg, Tt[rt][0]);
              Tt[rt][1] = mma(ev.x, bv.y, Tt[rt][1]);
              Tt[rt][1] = mma(ev.y, bv.x, Tt[rt][1]);
            }
          }
        }
        // GEMM2: E'^T[b'][a'] += sum_a T_s[a][b'] conj(A_s[a][a'])
#pragma unroll
        for (int rt = 0; rt < NT; ++rt) {
          if (rt < nrt) {
#pragma unroll
            for (int e = 0; e < 4; ++e) {
              const T tr = Tt[rt][0][e], ti = Tt[rt][1][e];
              const int a = 16 * rt + acc_row<T>(g, e);
              const T2 *arow = A + (size_t(s) * Da + a) * Dan + j;
#pragma unroll
              for (int at = 0; at < NT; ++at) {
                if (at < nat) {
                  const T2 av = gload_c(arow + 16 * at);
                  Ep[c][at][0] = mma(tr, av.x, Ep[c][at][0]);
                  Ep[c][at][0] = mma(ti, av.y, Ep[c][at][0]);
                  Ep[c][at][1] = mma(ti, av.x, Ep[c][at][1]);
                  Ep[c][at][1] = mma(-tr, av.y, Ep[c][at][1]);
                }
              }
            }
          }
        }
      }
#pragma unroll
      for (int at = 0; at < NT; ++at)
#pragma unroll
        for (int e = 0; e < 4; ++e)
          lmax = fmax(lmax, fmax(fabs(Ep[c][at][0][e]), fabs(Ep[c][at][1][e])));
    }
    lmax = wave_max(lmax);
    if (lane == 0) s_red[wave] = lmax;
    __syncthreads();  // every wave is done reading E
    const T gmax = fmax(fmax(s_red[0], s_red[1]), fmax(s_red[2], s_red[3]));
    const int e2 = gmax > T(0) ? ilogb(gmax) : 0;
    const T scale = ldexp(T(1), -e2);
    expacc += e2;
#pragma unroll
    for (int c = 0; c < CT_PER_WAVE; ++c) {
      const int ct = wave + 4 * c;
      if (ct >= nct) continue;
#pragma unroll
      for (int at = 0; at < NT; ++at) {
        if (at < nat) {
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            T2 v;
            v.x = Ep[c][at][0][e] * scale;
            v.y = Ep[c][at][1][e] * scale;
            // E'[16 at + j][bp] -> fragment (at, bp / 4), lane j + 16 (bp % 4)
            const int bp = 16 * ct + acc_row<T>(g, e);
            E[(at * nkqn + (bp >> 2)) * 64 + j + 16 * (bp & 3)] = v;
          }
        }
      }
    }
    __syncthreads();
  }
  ov_re = E[0].x;
  ov_im = E[0].y;
  ov_exp = expacc;
  __syncthreads();
}

// ------------------------------------------------------------------------
// FP64 / FP32 forms for bond pads up to 128.  E (128 x 128 complex, 256 KiB
// in FP64) is above one CU's LDS, so it lives in a slot of global scratch
// per workgroup, where it stays in L2: two buffers, E read and E' written,
// each in the A-operand fragment order of the LDS variant above.  Eight
// waves; wave w computes E' for the ket column block w.  T_s passes from
// GEMM1 to GEMM2 one 16-row block at a time, so only the accumulators of
// the wave's E' block (8 x 16 x 16 complex) are held across the site.
constexpr int kWideP = 128;
constexpr int kWideThreads = 512;
constexpr int kWideWaves = kWideThreads / 64;

template <typename T, typename V4, typename T2>
__device__ void overlap_wide(const GramJobDev &J, int64_t ia, int64_t ib, T2 *E0, T2 *E1, T *s_red,
                             T &ov_re, T &ov_im, int &ov_exp) {
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int j = lane & 15, g = lane >> 4;
  const T2 *abase = reinterpret_cast<const T2 *>(J.a_base) + ia * J.a_stride;
  const T2 *bbase = reinterpret_cast<const T2 *>(J.b_base) + ib * J.b_stride;
  T2 *Ec = E0, *En = E1;
  {
    // E_0 = [[1]] on the first site's pads (element [0][0] is lane 0 of
    // fragment 0)
    const int n0 = gview(J.a_pad)[0] * gview(J.b_pad)[0];
    for (int x = tid; x < n0; x += kWideThreads) {
      T2 z;
      z.x = x == 0 ? T(1) : T(0);
      z.y = T(0);
      gstore_c(Ec + x, z);
    }
    __syncthreads();
  }
  int expacc = 0;
  constexpr int NT = kWideP / 16;
  const int ct = wave;
  for (int l = 0; l < J.m; ++l) {
    const int Da = gview(J.a_pad)[l], Dan = gview(J.a_pad)[l + 1], Db = gview(J.b_pad)[l], Dbn = gview(J.b_pad)[l + 1];
    const T2 *A = abase + gview(J.a_off)[l];
    const T2 *B = bbase + gview(J.b_off)[l];
    const int nrt = Da / 16, nkq = Db / 4, nat = Dan / 16, nct = Dbn / 16, nkqn = Dbn / 4;
    V4 Ep[NT][2];
#pragma unroll
    for (int at = 0; at < NT; ++at) {
      Ep[at][0] = V4{0, 0, 0, 0};
      Ep[at][1] = V4{0, 0, 0, 0};
    }
    if (ct < nct) {
      for (int s = 0; s < 2; ++s) {
        const T2 *Bc = B + size_t(s) * Db * Dbn + 16 * ct + j;
        for (int rt = 0; rt < nrt; ++rt) {
          // GEMM1 on row block rt: T_s[a][b'] = sum_b E[a][b] B_s[b][b'],
          // real and imaginary parts of E in separate accumulators (two
          // independent MFMA chains per output)
          V4 t0 = V4{0, 0, 0, 0}, t1 = V4{0, 0, 0, 0}, u0 = V4{0, 0, 0, 0}, u1 = V4{0, 0, 0, 0};
          const T2 *Er = Ec + size_t(rt) * nkq * 64 + lane;
#pragma unroll 4
          for (int kq = 0; kq < nkq; ++kq) {
            const T2 bv = gload_c(Bc + size_t(4 * kq + g) * Dbn);
            const T2 ev = gload_c(Er + kq * 64);
            t0 = mma(ev.x, bv.x, t0);
            t1 = mma(ev.x, bv.y, t1);
            u0 = mma(ev.y, -bv.y, u0);
            u1 = mma(ev.y, bv.x, u1);
          }
          t0 += u0;
          t1 += u1;
          // GEMM2: E'^T[b'][a'] += sum_{a in block rt} T_s[a][b'] conj(A_s[a][a'])
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const T tr = t0[e], ti = t1[e];
            const int a = 16 * rt + acc_row<T>(g, e);
            const T2 *arow = A + (size_t(s) * Da + a) * Dan + j;
#pragma unroll
            for (int at = 0; at < NT; ++at) {
              if (at < nat) {
                const T2 av = gload_c(arow + 16 * at);
                Ep[at][0] = mma(tr, av.x, Ep[at][0]);
                Ep[at][0] = mma(ti, av.y, Ep[at][0]);
                Ep[at][1] = mma(ti, av.x, Ep[at][1]);
                Ep[at][1] = mma(-tr, av.y, Ep[at][1]);
              }
            }
          }
        }
      }
    }
    T lmax = T(0);
#pragma unroll
    for (int at = 0; at < NT; ++at)
#pragma unroll
      for (int e = 0; e < 4; ++e) lmax = fmax(lmax, fmax(fabs(Ep[at][0][e]), fabs(Ep[at][1][e])));
    lmax = wave_max(lmax);
    if (lane == 0) s_red[wave] = lmax;
    __syncthreads();
    T gmax = s_red[0];
#pragma unroll
    for (int w = 1; w < kWideWaves; ++w) gmax = fmax(gmax, s_red[w]);
    const int e2 = gmax > T(0) ? ilogb(gmax) : 0;
    const T scale = ldexp(T(1), -e2);
    expacc += e2;
    if (ct < nct) {
#pragma unroll
      for (int at = 0; at < NT; ++at) {
        if (at < nat) {
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            T2 v;
            v.x = Ep[at][0][e] * scale;
            v.y = Ep[at][1][e] * scale;
            // E'[16 at + j][bp] -> fragment (at, bp / 4), lane j + 16 (bp % 4)
            const int bp = 16 * ct + acc_row<T>(g, e);
            gstore_c(En + (at * nkqn + (bp >> 2)) * 64 + j + 16 * (bp & 3), v);
          }
        }
      }
    }
    // E' complete and visible to the workgroup; s_red free for the next site
    __syncthreads();
    T2 *t = Ec;
    Ec = En;
    En = t;
  }
  const T2 r = gload_c(Ec);
  ov_re = r.x;
  ov_im = r.y;
  ov_exp = expacc;
  __syncthreads();   // every wave has read the result before the next pair overwrites it
}

// A pointer that is the same in every lane, moved to scalar registers.
template <typename T>
__device__ inline T *uniform_ptr(T *p) {
  const uint64_t v = reinterpret_cast<uint64_t>(p);
  return reinterpret_cast<T *>((uint64_t(__builtin_amdgcn_readfirstlane(uint32_t(v >> 32))) << 32) |
                               uint32_t(__builtin_amdgcn_readfirstlane(uint32_t(v))));
}

// Fragments are read with buffer loads through a descriptor of the whole
// site block (scalar base, 32-bit lane offset, scalar fragment offset): no
// 64-bit vector address arithmetic per fragment, and a read outside the
// block's bytes returns zero.  Word 3 is the gfx9-family raw-buffer format.
typedef __amdgpu_buffer_rsrc_t SiteRsrc;
template <int64_t BYTES>
__device__ inline SiteRsrc site_rsrc(const uint8_t *site) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<uint8_t *>(uniform_ptr(site)), 0, int(BYTES), 0x00020000);
}

__device__ inline uint4 rsrc_load_u4(SiteRsrc r, int voff, int soff) {
  typedef unsigned int v4u __attribute__((ext_vector_type(4)));
  const v4u v = __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0);
  return make_uint4(v.x, v.y, v.z, v.w);
}


// ------------------------------------------------------------------------
// Split-BF16 form with fixed-point slices (layout in qk_internal.h).
//
// Every GEMM operand is cut into four bf16 slices that share one exponent per
// row (A-operand) or column (B-operand), so each slice is an integer
// |n| <= 128 times a power of two.  A real product X Y is then
//     2^(eX + eY - 14) * ( X0.Y0  +  sum of ten smaller slice products )
// where X0.Y0 accumulates EXACTLY in one FP32 MFMA accumulator (integers below
// 2^22) and the other ten slice pairs (weights 2^-8 .. 2^-32, smallest first)
// share a second FP32 accumulator, whose rounding is then ~2^-32 of the result.
// The two accumulators are combined in FP64.  This removes the FP32
// accumulation error that otherwise grows along the chain (about 2e-6 at 50
// sites and 2e-5 at 100 sites for K = 1 with plain FP32 operands).
//
// E lives in LDS as slices plus one exponent per row; T and E' are formed in
// FP64 registers and re-sliced for the next GEMM.
__device__ inline int exp_above(double mx) {
  // Smallest e with mx (1 + 2^-30) < 2^e (0 for mx == 0).  The margin keeps
  // |x| 2^(31-e) below 2^31 - 1 after rounding for every |x| <= mx, so the
  // 31-bit fixed-point code never saturates (saturation would bias values
  // just below a power of two, e.g. the unit diagonal of a self-overlap).
  return mx > 0.0 ? ilogb(mx * (1.0 + 0x1p-30)) + 1 : 0;
}

__device__ inline uint32_t bf16_bits_exact(float v) { return __float_as_uint(v) >> 16; }

// Four pre-scaled slices n_k 2^-8k (k = 0..3) of x * 2^-e (|x| < 2^e), as
// bf16 bits: X = round(x 2^(31-e)) (saturated to int32) is split into
// balanced base-256 digits X = n0 2^24 + n1 2^16 + n2 2^8 + n3, with
// n1..n3 in [-128, 127] and n0 in [-128, 128].  Each step takes the low byte
// as a signed digit and carries one when it is negative; the carry is formed
// from the shifted value, never from X - digit, which overflows int32 for X
// near 2^31 (values just below the top of their exponent range).
__device__ inline int balanced_digit(int &r) {
  const int d = int(int8_t(r & 0xff));
  r = (r >> 8) + ((r >> 7) & 1);
  return d;
}

__device__ inline void slice4e(double x, int e, uint32_t (&o)[4]) {
  int r = int(fmin(fmax(rint(ldexp(x, 31 - e)), -2147483647.0), 2147483647.0));
  const int n3 = balanced_digit(r);
  const int n2 = balanced_digit(r);
  const int n1 = balanced_digit(r);
  const int n0 = r;
  o[0] = bf16_bits_exact(float(n0));
  o[1] = bf16_bits_exact(float(n1) * 0x1p-8f);
  o[2] = bf16_bits_exact(float(n2) * 0x1p-16f);
  o[3] = bf16_bits_exact(float(n3) * 0x1p-24f);
}


// Row exponent of the values the kernel slices itself (T and E'): smallest e
// with mx (1 + 2^-7) < 2^e, so that |X| + 0x808080 < 2^31 in slice4_word.
__device__ inline int exp_above_w(double mx) { return mx > 0.0 ? ilogb(mx * (1.0 + 0x1p-7)) + 1 : 0; }

// The same four slices as slice4e, as floats n_k 2^-8k, from one FP64 FMA:
// with scale = 2^(31-e), the low word of x scale + 1.5 2^52 + 0x808080 is
// Y = X + 0x808080 for X = round(x 2^(31-e)), whose top byte is the signed
// leading digit n0 and whose lower bytes are n_k + 128 (k = 1..3) -- the
// same balanced digits, without carries.  Each slice is then one byte
// conversion and one exact FMA; its bf16 bits are the float's upper half.
__device__ inline void slice4_word(double x, double scale, float (&f)[4]) {
  const uint32_t y = uint32_t(__double_as_longlong(fma(x, scale, 0x1.8p52 + 0x808080)));
  f[0] = float(int(y) >> 24);
  f[1] = fmaf(float(uint8_t(y >> 16)), 0x1p-8f, -0x1p-1f);
  f[2] = fmaf(float(uint8_t(y >> 8)), 0x1p-16f, -0x1p-9f);
  f[3] = fmaf(float(uint8_t(y)), 0x1p-24f, -0x1p-17f);
}

// bf16 bits of two exact floats packed in one word (a low, b high).
__device__ inline uint32_t pack_bf16_pair(float a, float b) {
  return __builtin_amdgcn_perm(__float_as_uint(b), __float_as_uint(a), 0x07060302u);
}

struct Sl4 {
  uint4 v[4];
};

__device__ inline Sl4 neg4(const Sl4 &x) {
  Sl4 y;
#pragma unroll
  for (int k = 0; k < 4; ++k) y.v[k] = neg_bf16(x.v[k]);
  return y;
}

// hi += X0 Y0 (exact); lo += the smaller slice products, smallest first:
// the nine others of weight >= 2^-24 and, if P22, the (2, 2) product, which
// is kept only where bra ~ ket makes it one-signed (the real part of GEMM2;
// the reasoning of the split-int8 form below applies to the same digits).
template <bool P22>
__device__ inline void slice_mac(const Sl4 &X, const Sl4 &Y, f32x4 &hi, f32x4 &lo) {
  hi = mma16(X.v[0], Y.v[0], hi);
  lo = mma16(X.v[3], Y.v[0], lo);
  lo = mma16(X.v[0], Y.v[3], lo);
  lo = mma16(X.v[2], Y.v[1], lo);
  lo = mma16(X.v[1], Y.v[2], lo);
  if (P22) lo = mma16(X.v[2], Y.v[2], lo);
  lo = mma16(X.v[2], Y.v[0], lo);
  lo = mma16(X.v[1], Y.v[1], lo);
  lo = mma16(X.v[0], Y.v[2], lo);
  lo = mma16(X.v[1], Y.v[0], lo);
  lo = mma16(X.v[0], Y.v[1], lo);
}

// Work split per site (eight waves): wave w owns column block c = w % 4 and
// row half h = w / 4.  GEMM1 produces T_s[rows 32h..32h+31][ket block c]; the
// exponent of each T^T row (ket column) combines both halves through LDS and
// T is stored in LDS as slices.  GEMM2 produces E'^T[ket rows 32h..][bra
// block c].  Two 64 KiB LDS buffers alternate roles so that slicing one
// operand overlaps the MFMAs of the next GEMM:
//   1. GEMM1(s=0) reads E (buffer X)                     -> T0 in registers
//   2. slice T0 -> Y            ||  GEMM1(s=1) reads X    -> T1 in registers
//   3. slice T1 -> X            ||  GEMM2(s=0) reads Y    (E no longer needed)
//   4. GEMM2(s=1) reads X; E' row exponents
//   5. slice E' -> Y, which holds E for the next site (X and Y swap).
// The split form is stored with 64 x 64 blocks at every site, so the body is
// straight-line code.
constexpr int kSplitThreads = 512;
constexpr int kSP = 64;

struct SplitCtx {
  int lane, j, g, cb, hf;
};

constexpr int64_t kSplitSiteBytes = kSplitExpBytes + int64_t(2) * 4 * 2 * 2 * 4 * kFragBytes;
static_assert(kSplitSiteBytes == split_site_bytes(), "split-BF16 site block size");

__device__ inline uint4 split_frag(SiteRsrc site, int s, int k, int q, int kc, int c, int lane) {
  return rsrc_load_u4(site, lane * 16, kSplitExpBytes + ((((s * 4 + k) * 2 + q) * 2 + kc) * 4 + c) * kFragBytes);
}

// GEMM1 for physical index s: T[a][b'] (a in rows 32h.., b' in block c) in
// FP64, and the local max |T| over this wave's part of each T^T row.
__device__ inline void split_gemm1(const SplitCtx &C, const uint8_t *B, const uint8_t *Ebuf, const int *s_ea, int s,
                                   double (&Td)[2][2][4], double &tmax) {
  f32x4 h1[2][2], l1[2][2];
#pragma unroll
  for (int u = 0; u < 2; ++u)
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      h1[u][q] = f32x4{0, 0, 0, 0};
      l1[u][q] = f32x4{0, 0, 0, 0};
    }
  const SiteRsrc rB = site_rsrc<kSplitSiteBytes>(B);
#pragma unroll
  for (int kc = 0; kc < 2; ++kc) {
    Sl4 Br, Bi;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      Br.v[k] = split_frag(rB, s, k, 0, kc, C.cb, C.lane);
      Bi.v[k] = split_frag(rB, s, k, 1, kc, C.cb, C.lane);
    }
    const Sl4 Bin = neg4(Bi);
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int rt = 2 * C.hf + u;
      const uint8_t *eg = Ebuf + size_t(rt * 2 + kc) * 8192 + C.lane * 16;
      Sl4 Er, Ei;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        Er.v[k] = *reinterpret_cast<const uint4 *>(eg + (k * 2 + 0) * 1024);
        Ei.v[k] = *reinterpret_cast<const uint4 *>(eg + (k * 2 + 1) * 1024);
      }
      // re += Er Br - Ei Bi ; im += Er Bi + Ei Br
      __builtin_amdgcn_s_setprio(1);   // MFMA burst first when both waves of a SIMD are ready
      slice_mac<false>(Er, Br, h1[u][0], l1[u][0]);
      slice_mac<false>(Ei, Bin, h1[u][0], l1[u][0]);
      slice_mac<false>(Er, Bi, h1[u][1], l1[u][1]);
      slice_mac<false>(Ei, Br, h1[u][1], l1[u][1]);
      __builtin_amdgcn_s_setprio(0);
    }
  }
  const int ebc = int(gview(reinterpret_cast<const int8_t *>(B))[s * 128 + 16 * C.cb + C.j]);
  tmax = 0.0;
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int rt = 2 * C.hf + u;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int ex = s_ea[16 * rt + 4 * C.g + e] + ebc - 14;
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const double v = ldexp(double(h1[u][q][e]) + double(l1[u][q][e]), ex);
        Td[u][q][e] = v;
        tmax = fmax(tmax, fabs(v));
      }
    }
  }
  tmax = fmax(tmax, __shfl_xor(tmax, 16, 64));
  tmax = fmax(tmax, __shfl_xor(tmax, 32, 64));
}

// Slice four 4-value rows (u = 0, 1; q = re, im) with exponent ex into LDS
// group row `grow` of buffer `buf`: the 16-row tiles t = 2 h + u of the
// contraction index are slots 0..3 (u = 0) and 4..7 (u = 1) of A-operand
// group (grow, kc = h), so each lane stores one full 16-byte slot per slice
// and plane (contiguous across the wave: no bank conflicts).
__device__ inline void split_store(const SplitCtx &C, uint8_t *buf, int grow, const double (&V)[2][2][4], int ex) {
  const double scale = ldexp(1.0, 31 - ex);
  uint8_t *dst = buf + size_t(grow * 2 + C.hf) * 8192 + C.lane * 16;
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    float sl[2][4][4];
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
      for (int e = 0; e < 4; ++e) slice4_word(V[u][q][e], scale, sl[u][e]);
#pragma unroll
    for (int k = 0; k < 4; ++k)
      *reinterpret_cast<uint4 *>(dst + (k * 2 + q) * 1024) =
          make_uint4(pack_bf16_pair(sl[0][0][k], sl[0][1][k]), pack_bf16_pair(sl[0][2][k], sl[0][3][k]),
                     pack_bf16_pair(sl[1][0][k], sl[1][1][k]), pack_bf16_pair(sl[1][2][k], sl[1][3][k]));
  }
}

// GEMM2 for physical index s: E'^T[b'][a'] += sum_a T_s[a][b'] conj(A_s[a][a'])
// with b' in rows 32h.., a' in bra block c.
__device__ inline void split_gemm2(const SplitCtx &C, const uint8_t *A, const uint8_t *Tbuf, const int *s_eTs, int s,
                                   double (&Ep)[2][2][4]) {
  f32x4 h2[2][2], l2[2][2];
#pragma unroll
  for (int u = 0; u < 2; ++u)
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      h2[u][q] = f32x4{0, 0, 0, 0};
      l2[u][q] = f32x4{0, 0, 0, 0};
    }
  const SiteRsrc rA = site_rsrc<kSplitSiteBytes>(A);
#pragma unroll
  for (int kc = 0; kc < 2; ++kc) {
    Sl4 Ar, Ai;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      Ar.v[k] = split_frag(rA, s, k, 0, kc, C.cb, C.lane);
      Ai.v[k] = split_frag(rA, s, k, 1, kc, C.cb, C.lane);
    }
    const Sl4 Ain = neg4(Ai);   // shared by both row tiles (the products are those of -Tr Ai)
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int bt = 2 * C.hf + u;
      const uint8_t *tg = Tbuf + size_t(bt * 2 + kc) * 8192 + C.lane * 16;
      Sl4 Tr, Ti;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        Tr.v[k] = *reinterpret_cast<const uint4 *>(tg + (k * 2 + 0) * 1024);
        Ti.v[k] = *reinterpret_cast<const uint4 *>(tg + (k * 2 + 1) * 1024);
      }
      // re += Tr Ar + Ti Ai ; im += Ti Ar + Tr (-Ai)
      __builtin_amdgcn_s_setprio(1);
      slice_mac<true>(Tr, Ar, h2[u][0], l2[u][0]);
      slice_mac<true>(Ti, Ai, h2[u][0], l2[u][0]);
      slice_mac<false>(Ti, Ar, h2[u][1], l2[u][1]);
      slice_mac<false>(Tr, Ain, h2[u][1], l2[u][1]);
      __builtin_amdgcn_s_setprio(0);
    }
  }
  const int eac = int(gview(reinterpret_cast<const int8_t *>(A))[s * 128 + 16 * C.cb + C.j]);
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int bt = 2 * C.hf + u;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int ex = s_eTs[16 * bt + 4 * C.g + e] + eac - 14;
#pragma unroll
      for (int q = 0; q < 2; ++q) Ep[u][q][e] += ldexp(double(h2[u][q][e]) + double(l2[u][q][e]), ex);
    }
  }
}

template <int MAXP>
__device__ void overlap_split(const GramJobDev &J, int64_t ia, int64_t ib, uint8_t *buf0, uint8_t *buf1,
                              int *s_ea, int *s_eT, double *s_mx, double *s_ov, double &ov_re, double &ov_im,
                              int &ov_exp) {
  static_assert(MAXP == kSP, "the split form uses 64 x 64 site blocks");
  const int tid = threadIdx.x, wave = tid >> 6;
  SplitCtx C;
  C.lane = tid & 63;
  C.j = C.lane & 15;
  C.g = C.lane >> 4;
  // wave-uniform (scalar) block indices: fragment offsets stay in SGPRs
  C.cb = __builtin_amdgcn_readfirstlane(wave & 3);
  C.hf = __builtin_amdgcn_readfirstlane(wave >> 2);
  const uint8_t *abase = reinterpret_cast<const uint8_t *>(J.a_base) + ia * J.a_stride;
  const uint8_t *bbase = reinterpret_cast<const uint8_t *>(J.b_base) + ib * J.b_stride;
  uint8_t *X = buf0, *Y = buf1;
  {
    uint4 *X16 = reinterpret_cast<uint4 *>(X);
    for (int x = tid; x < kSP * kSP; x += kSplitThreads) X16[x] = make_uint4(0, 0, 0, 0);
    for (int x = tid; x < kSP; x += kSplitThreads) s_ea[x] = 0;
    __syncthreads();
    // E_0 = [[1]]: row exponent 1, leading slice 64 (= 0.5 * 128)
    if (tid == 0) {
      reinterpret_cast<uint16_t *>(X)[0] = uint16_t(bf16_bits_exact(64.0f));
      s_ea[0] = 1;
    }
    __syncthreads();
  }
  const int col = 16 * C.cb + C.j;
  for (int l = 0; l < J.m; ++l) {
    const uint8_t *A = abase + gview(J.a_off)[l];
    const uint8_t *B = bbase + gview(J.b_off)[l];
    double Td0[2][2][4], Td1[2][2][4], Ep[2][2][4];
    double tmax;
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
      for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int e = 0; e < 4; ++e) Ep[u][q][e] = 0.0;
    // 1. GEMM1(s = 0)
    split_gemm1(C, B, X, s_ea, 0, Td0, tmax);
    if (C.g == 0) s_mx[(0 * 2 + C.hf) * kSP + col] = tmax;
    __syncthreads();
    // 2. slice T0 -> Y  ||  GEMM1(s = 1)
    {
      const int eT0 = exp_above_w(fmax(s_mx[(0 * 2 + 0) * kSP + col], s_mx[(0 * 2 + 1) * kSP + col]));
      if (C.hf == 0 && C.g == 0) s_eT[0 * kSP + col] = eT0;
      split_store(C, Y, C.cb, Td0, eT0);
      split_gemm1(C, B, X, s_ea, 1, Td1, tmax);
      if (C.g == 0) s_mx[(1 * 2 + C.hf) * kSP + col] = tmax;
    }
    __syncthreads();
    // 3. slice T1 -> X  ||  GEMM2(s = 0)
    {
      const int eT1 = exp_above_w(fmax(s_mx[(1 * 2 + 0) * kSP + col], s_mx[(1 * 2 + 1) * kSP + col]));
      if (C.hf == 0 && C.g == 0) s_eT[1 * kSP + col] = eT1;
      split_store(C, X, C.cb, Td1, eT1);
      split_gemm2(C, A, Y, s_eT, 0, Ep);
    }
    __syncthreads();
    // 4. GEMM2(s = 1) and the row maxima of E' (rows a' = 16 c + j)
    split_gemm2(C, A, X, s_eT + kSP, 1, Ep);
    {
      double rm = 0.0;
#pragma unroll
      for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int e = 0; e < 4; ++e) rm = fmax(rm, fmax(fabs(Ep[u][0][e]), fabs(Ep[u][1][e])));
      rm = fmax(rm, __shfl_xor(rm, 16, 64));
      rm = fmax(rm, __shfl_xor(rm, 32, 64));
      if (C.g == 0) s_mx[(0 * 2 + C.hf) * kSP + col] = rm;
    }
    __syncthreads();
    // 5. E' -> Y (E of the next site)
    if (l + 1 == J.m) {
      // E_m[0][0] = E'^T[0][0]: block 0, half 0, lane 0, u = 0, e = 0
      if (wave == 0 && C.lane == 0) {
        s_ov[0] = Ep[0][0][0];
        s_ov[1] = Ep[0][1][0];
      }
    } else {
      const int er = exp_above_w(fmax(s_mx[(0 * 2 + 0) * kSP + col], s_mx[(0 * 2 + 1) * kSP + col]));
      split_store(C, Y, C.cb, Ep, er);
      if (C.hf == 0 && C.g == 0) s_ea[col] = er;
    }
    __syncthreads();
    uint8_t *t = X;
    X = Y;
    Y = t;
  }
  ov_re = s_ov[0];
  ov_im = s_ov[1];
  ov_exp = 0;
  __syncthreads();
}

// ------------------------------------------------------------------------
// Split-int8 form: the same 31-bit fixed-point codes with one exponent per
// row (E, T^T) or column (site tensors), cut into four balanced base-256
// digits that are int8 MFMA operands (v_mfma_i32_16x16x64_i8, twice the
// bf16 rate).  Digit products accumulate EXACTLY in int32, grouped by weight
// 2^(-8 c), c = a + b for digit pair (a, b): c = 0..3 (ten pairs) and, in
// the real part of GEMM2, the (2, 2) pair.  A product with a negated operand
// uses ~x = -x - 1: the
// accumulator then lacks a column digit sum of the other operand, which the
// packed site block carries and the combination adds back.
//
// Code of x with exponent e: X = round(x 2^(31-e)), formed by one FMA with
// 1.5 * 2^52 (the low word of the sum is X).  The margin of exp_above_i8
// keeps |X| <= 2^31 * 128/129, so the leading digit lies in [-127, 127].
// Digit word (X + 0x808080) ^ 0x808080 holds the digits d3, d2, d1, d0 as
// two's-complement bytes 0..3 (X = d0 2^24 + d1 2^16 + d2 2^8 + d3); the
// addition is folded into the FMA constant and the XOR applied once per
// four-value slice word.
typedef int i32x4 __attribute__((ext_vector_type(4)));

// The (2, 2) digit pair (weight 2^-32, like the omitted (1, 3) and (3, 1))
// is kept only in the real part of GEMM2.  There, for a bra equal (or close)
// to the ket, T is the site tensor itself (E = I for left-canonical states)
// and the pair's products Tr Ar + Ti Ai are sums of squares: dropping them
// biases every self-overlap one way (max |dK| on 165-site chi = 64 states
// 2.7e-9 -> 4.0e-7).  In the imaginary part Ti Ar - Tr Ai they cancel for
// T = A, and in GEMM1 the LDS operand is E, whose digit 2 vanishes for E = I
// and whose products with the site digits carry no common sign, so the pair
// is omitted there (CPU emulation on 100-site chi = 64 states: max |dK|
// 1.8e-8 with the pair everywhere, 2.5e-8 with it in GEMM2's real part only,
// the diagonal 1.6e-8; without it in GEMM2's real part: 2.6e-6).
#ifndef QK_I8_PAIR22
#define QK_I8_PAIR22 1
#endif

__device__ inline i32x4 mma_i8(const uint4 &a, const uint4 &b, const i32x4 &c) {
  return __builtin_amdgcn_mfma_i32_16x16x64_i8(*reinterpret_cast<const i32x4 *>(&a),
                                               *reinterpret_cast<const i32x4 *>(&b), c, 0, 0, 0);
}

__device__ inline int exp_above_i8(double mx) {
  // smallest e with mx (1 + 2^-7) < 2^e (0 for mx == 0)
  return mx > 0.0 ? ilogb(mx * (1.0 + 0x1p-7)) + 1 : 0;
}

// Digit word with the bias of the three low digits still applied (bytes
// 0..2 hold d + 128); transpose_digits removes it.
__device__ inline uint32_t biased_digit_word(double x, double scale) {
  const double w = fma(x, scale, 0x1.8p52 + 0x808080);   // low word: X + 0x808080
  return uint32_t(__double_as_longlong(w));
}

// Byte transpose of four biased digit words (values e = 0..3) into four
// slice words: byte e of slice k is digit k of value e (slice 0 = leading
// digit); the bias of digits 1..3 is removed by one XOR per slice word.
__device__ inline void transpose_digits(uint32_t d0, uint32_t d1, uint32_t d2, uint32_t d3, uint32_t (&s)[4]) {
  const uint32_t lo01 = __builtin_amdgcn_perm(d1, d0, 0x05010400u);
  const uint32_t hi01 = __builtin_amdgcn_perm(d1, d0, 0x07030602u);
  const uint32_t lo23 = __builtin_amdgcn_perm(d3, d2, 0x05010400u);
  const uint32_t hi23 = __builtin_amdgcn_perm(d3, d2, 0x07030602u);
  s[3] = __builtin_amdgcn_perm(lo23, lo01, 0x05040100u) ^ 0x80808080u;
  s[2] = __builtin_amdgcn_perm(lo23, lo01, 0x07060302u) ^ 0x80808080u;
  s[1] = __builtin_amdgcn_perm(hi23, hi01, 0x05040100u) ^ 0x80808080u;
  s[0] = __builtin_amdgcn_perm(hi23, hi01, 0x07060302u);
}

__device__ inline uint4 not4(const uint4 &v) { return make_uint4(~v.x, ~v.y, ~v.z, ~v.w); }

// Completes one row tile before the next one starts: the tile's results are
// formed before this point and no later LDS or global load moves above it,
// so only one tile's accumulators are live (register budget of two waves
// per SIMD).
__device__ inline void tile_fence(double (&v)[2][4]) {
#pragma unroll
  for (int q = 0; q < 2; ++q)
#pragma unroll
    for (int e = 0; e < 4; ++e) asm volatile("" : "+v"(v[q][e])::"memory");
}

// Fragment (s, slice k, plane q, column block ct) of a packed int8 site block.
__device__ inline uint4 i8_frag(SiteRsrc site, int s, int k, int q, int ct, int lane) {
  return rsrc_load_u4(site, lane * 16, kI8ExpBytes + kI8SumBytes + (((s * 4 + k) * 2 + q) * 4 + ct) * kI8FragBytes);
}

// Class accumulators of one complex 16 x 16 tile: class c holds the digit
// products of weight 2^(-8 c) (c = 0..3) and class 4 the (2, 2) product
// (real part of GEMM2 only; unused accumulators are never formed).
struct I8Acc {
  i32x4 re[5], im[5];
};

// Same products with the LDS operand read one digit at a time (tile base tg:
// fragments (digit a, plane 0 / 1) at (2 a + q) KiB).  CPL1: complement plane 1
// in the real part (GEMM1: re += X0 Y0 + (~X1) Y1, im += X0 Y1 + X1 Y0);
// otherwise complement plane 0 in the imaginary part (GEMM2: re += X0 Y0 +
// X1 Y1, im += (~X0) Y1 + X1 Y0).  The part with the complemented operand
// starts from the class corrections `corr` (so its sums come out exact), the
// other from zero.  P22_RE: include the (2, 2) pair (class 4) in the real
// part.  Only one digit's operands are live.
template <bool CPL1, bool P22_RE>
__device__ inline void i8_block_lds(const uint8_t *tg, const uint4 (&Y0)[4], const uint4 (&Y1)[4],
                                    const i32x4 (&corr)[4], I8Acc &acc) {
#pragma unroll
  for (int c = 0; c < 5; ++c) {
    acc.re[c] = (CPL1 && c < 4) ? corr[c] : i32x4{0, 0, 0, 0};
    acc.im[c] = (!CPL1 && c < 4) ? corr[c] : i32x4{0, 0, 0, 0};
  }
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const uint4 x0 = *reinterpret_cast<const uint4 *>(tg + (a * 2 + 0) * kI8FragBytes);
    const uint4 x1 = *reinterpret_cast<const uint4 *>(tg + (a * 2 + 1) * kI8FragBytes);
    const uint4 P = x0, Q = CPL1 ? not4(x1) : x1, R = CPL1 ? x0 : not4(x0), S = x1;
    // digit pairs (a, b) with a + b <= 3
    const int nb = a == 0 ? 4 : a == 1 ? 3 : a == 2 ? 2 : 1;
#pragma unroll
    for (int b = 0; b < nb; ++b) {
      const int c = a + b;
      acc.re[c] = mma_i8(P, Y0[b], acc.re[c]);
      acc.im[c] = mma_i8(R, Y1[b], acc.im[c]);
      acc.re[c] = mma_i8(Q, Y1[b], acc.re[c]);
      acc.im[c] = mma_i8(S, Y0[b], acc.im[c]);
    }
    if (P22_RE && a == 2) {   // (2, 2) into class 4 of the real part
      acc.re[4] = mma_i8(P, Y0[2], acc.re[4]);
      acc.re[4] = mma_i8(Q, Y1[2], acc.re[4]);
    }
  }
}

// Exact digit sum of element e of a class accumulator set (corrections
// already in the accumulators), as a double in units of 2^24 of the code
// product (class c weighs 2^(24 - 8 c); class 4, if P22, 2^-8: one rounding).
template <bool P22>
__device__ inline double i8_value(const i32x4 (&a)[5], int e) {
  const int hiw = int((uint32_t(a[0][e]) << 8) + uint32_t(a[1][e]));
  const int low = int((uint32_t(a[2][e]) << 8) + uint32_t(a[3][e]));
  if (P22) return fma(double(a[4][e]), 0x1p-8, fma(double(hiw), 65536.0, double(low)));
  return fma(double(hiw), 65536.0, double(low));
}

// Class corrections from the column digit sums cs0..cs3 of the operand that
// was multiplied by a complemented one: class c gets the sum over its pairs
// (a, b) of cs_b, the same for the four accumulator rows of a lane (its
// column).  Class 4 is only formed where no operand is complemented (the
// real part of GEMM2), so it needs none.
__device__ inline void i8_corrections(const int (&cs)[4], i32x4 (&corr)[4]) {
  const int k0 = cs[0], k1 = k0 + cs[1], k2 = k1 + cs[2], k3 = k2 + cs[3];
  corr[0] = i32x4{k0, k0, k0, k0};
  corr[1] = i32x4{k1, k1, k1, k1};
  corr[2] = i32x4{k2, k2, k2, k2};
  corr[3] = i32x4{k3, k3, k3, k3};
}

// Work split of the int8 kernel: workgroups of four waves, two per CU, each
// workgroup on its own pair, so the two workgroups of a CU interleave their
// MFMA and VALU phases.  Wave w owns column block c = w of every 64 x 64
// product: it holds whole columns of T (rows of T^T) and whole rows of E',
// so their exponents are formed in registers.  Three barriers per site:
//   I.   GEMM1(s=0) reads E (buffer X) -> T0 -> Y ; GEMM1(s=1) reads X -> T1
//   II.  T1 -> X (E consumed) ; GEMM2(s=0) reads Y
//   III. GEMM2(s=1) reads X ; E' -> Y (T0 consumed), which is the next E
constexpr int kI8Threads = 256;

struct I8Ctx {
  int lane, j, g, cb;
};

// This lane's digit fragments of column block c of one physical index of a
// packed site block (real plane, then imaginary plane), loaded one GEMM
// ahead of their use so that global latency overlaps the current GEMM; the
// column exponent and digit sums are read at the start of the GEMM itself
// (first needed after its first tile of MFMAs).
struct I8Operand {
  uint4 f[8];
  const uint8_t *site;
  int s;
};

__device__ inline void i8_load(const I8Ctx &C, const uint8_t *site, int s, I8Operand &o) {
  const SiteRsrc r = site_rsrc<kI8SiteBytes>(site);
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    o.f[k] = i8_frag(r, s, k, 0, C.cb, C.lane);
    o.f[4 + k] = i8_frag(r, s, k, 1, C.cb, C.lane);
  }
  o.site = site;
  o.s = s;
}

__device__ inline void i8_column_meta(const I8Ctx &C, const I8Operand &o, int &e, int (&cs)[4]) {
  const int col = 16 * C.cb + C.j;
  e = int(gview(reinterpret_cast<const int8_t *>(o.site))[o.s * 128 + col]);
  const auto p = gview(reinterpret_cast<const int *>(o.site + kI8ExpBytes) + o.s * 256 + col);
#pragma unroll
  for (int k = 0; k < 4; ++k) cs[k] = p[64 * k];
}

// GEMM1: T_s[a][b'] for all rows a (tiles rt = 0..3) and b' in block c;
// tmax = max |T| over the whole column b' = 16 c + j.
__device__ inline void i8_gemm1(const I8Ctx &C, const I8Operand &Bs, const uint8_t *Ebuf, const int *s_ea,
                                double (&Td)[4][2][4], double &tmax) {
  const uint4(&Br)[4] = *reinterpret_cast<const uint4(*)[4]>(&Bs.f[0]);
  const uint4(&Bi)[4] = *reinterpret_cast<const uint4(*)[4]>(&Bs.f[4]);
  int ebc, cs[4];
  i8_column_meta(C, Bs, ebc, cs);
  i32x4 corr[4];
  i8_corrections(cs, corr);
  tmax = 0.0;
#pragma unroll
  for (int rt = 0; rt < 4; ++rt) {
    // re = Er Br - Ei Bi = Er Br + (~Ei) Bi + colsum(Bi) ; im = Er Bi + Ei Br
    I8Acc acc;
    __builtin_amdgcn_s_setprio(1);
    i8_block_lds<true, false>(Ebuf + size_t(rt * 8) * kI8FragBytes + C.lane * 16, Br, Bi, corr, acc);
    __builtin_amdgcn_s_setprio(0);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      // a code product is x_E x_B 2^(62 - ea - eb); i8_value counts units of 2^24 of it
      const int ex = s_ea[16 * rt + 4 * C.g + e] + ebc - 38;
      const double vr = ldexp(i8_value<false>(acc.re, e), ex);
      const double vi = ldexp(i8_value<false>(acc.im, e), ex);
      Td[rt][0][e] = vr;
      Td[rt][1][e] = vi;
      tmax = fmax(tmax, fmax(fabs(vr), fabs(vi)));
    }
    tile_fence(Td[rt]);
  }
  tmax = fmax(tmax, __shfl_xor(tmax, 16, 64));
  tmax = fmax(tmax, __shfl_xor(tmax, 32, 64));
}

// Slice the wave's values (A-operand rows 16 c + j, contraction
// 16 rt + 4 g + e) with row exponent ex into buffer buf: fragment (row tile
// c, digit k, plane q), lane bytes 4 rt .. 4 rt + 3.
__device__ inline void i8_store(const I8Ctx &C, uint8_t *buf, const double (&V)[4][2][4], int ex) {
  const double scale = ldexp(1.0, 31 - ex);
  uint8_t *dst = buf + size_t(C.cb * 8) * kI8FragBytes + C.lane * 16;
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    uint32_t w[4][4];
#pragma unroll
    for (int rt = 0; rt < 4; ++rt)
      transpose_digits(biased_digit_word(V[rt][q][0], scale), biased_digit_word(V[rt][q][1], scale),
                       biased_digit_word(V[rt][q][2], scale), biased_digit_word(V[rt][q][3], scale), w[rt]);
#pragma unroll
    for (int k = 0; k < 4; ++k)
      *reinterpret_cast<uint4 *>(dst + (k * 2 + q) * kI8FragBytes) = make_uint4(w[0][k], w[1][k], w[2][k], w[3][k]);
  }
}

// GEMM2: E'^T[b'][a'] += sum_a T_s[a][b'] conj(A_s[a][a']) for all b' (tiles
// bt = 0..3) and a' in block c.
__device__ inline void i8_gemm2(const I8Ctx &C, const I8Operand &As, const uint8_t *Tbuf, const int *s_eTs,
                                double (&Ep)[4][2][4]) {
  const uint4(&Ar)[4] = *reinterpret_cast<const uint4(*)[4]>(&As.f[0]);
  const uint4(&Ai)[4] = *reinterpret_cast<const uint4(*)[4]>(&As.f[4]);
  int eac, cs[4];
  i8_column_meta(C, As, eac, cs);
  i32x4 corr[4];
  i8_corrections(cs, corr);
#pragma unroll
  for (int bt = 0; bt < 4; ++bt) {
    // re = Tr Ar + Ti Ai ; im = Ti Ar - Tr Ai = Ti Ar + (~Tr) Ai + colsum(Ai)
    I8Acc acc;
    __builtin_amdgcn_s_setprio(1);
    i8_block_lds<false, QK_I8_PAIR22>(Tbuf + size_t(bt * 8) * kI8FragBytes + C.lane * 16, Ar, Ai, corr, acc);
    __builtin_amdgcn_s_setprio(0);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int ex = s_eTs[16 * bt + 4 * C.g + e] + eac - 38;
      Ep[bt][0][e] += ldexp(i8_value<QK_I8_PAIR22>(acc.re, e), ex);
      Ep[bt][1][e] += ldexp(i8_value<false>(acc.im, e), ex);
    }
    tile_fence(Ep[bt]);
  }
}

__device__ void overlap_i8(const GramJobDev &J, int64_t ia, int64_t ib, uint8_t *buf0, uint8_t *buf1, int *s_ea,
                           int *s_eT, double *s_ov, double &ov_re, double &ov_im) {
  const int tid = threadIdx.x;
  I8Ctx C;
  C.lane = tid & 63;
  C.j = C.lane & 15;
  C.g = C.lane >> 4;
  C.cb = __builtin_amdgcn_readfirstlane(tid >> 6);   // wave-uniform: scalar addressing
  const uint8_t *abase = reinterpret_cast<const uint8_t *>(J.a_base) + ia * J.a_stride;
  const uint8_t *bbase = reinterpret_cast<const uint8_t *>(J.b_base) + ib * J.b_stride;
  uint8_t *X = buf0, *Y = buf1;
  {
    uint4 *X16 = reinterpret_cast<uint4 *>(X);
    for (int x = tid; x < kI8BufBytes / 16; x += kI8Threads) X16[x] = make_uint4(0, 0, 0, 0);
    for (int x = tid; x < kSP; x += kI8Threads) s_ea[x] = 0;
    __syncthreads();
    // E_0 = [[1]]: exponent 1, code 2^30, leading digit 64
    if (tid == 0) {
      X[0] = 64;
      s_ea[0] = 1;
    }
    __syncthreads();
  }
  const int col = 16 * C.cb + C.j;
  I8Operand P0, P1;   // operands of the current and the next GEMM
  i8_load(C, uniform_ptr(bbase + gview(J.b_off)[0]), 0, P0);
  for (int l = 0; l < J.m; ++l) {
    const uint8_t *A = uniform_ptr(abase + gview(J.a_off)[l]);
    const uint8_t *B = uniform_ptr(bbase + gview(J.b_off)[l]);
    double Td[4][2][4], Ep[4][2][4];
    double tmax;
    // I
    i8_load(C, B, 1, P1);
    i8_gemm1(C, P0, X, s_ea, Td, tmax);
    {
      const int eT0 = exp_above_i8(tmax);
      if (C.g == 0) s_eT[col] = eT0;
      i8_store(C, Y, Td, eT0);
    }
    i8_load(C, A, 0, P0);
    i8_gemm1(C, P1, X, s_ea, Td, tmax);
    __syncthreads();
    // II
    i8_load(C, A, 1, P1);
    {
      const int eT1 = exp_above_i8(tmax);
      if (C.g == 0) s_eT[kSP + col] = eT1;
      i8_store(C, X, Td, eT1);
    }
#pragma unroll
    for (int bt = 0; bt < 4; ++bt)
#pragma unroll
      for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int e = 0; e < 4; ++e) Ep[bt][q][e] = 0.0;
    i8_gemm2(C, P0, Y, s_eT, Ep);
    __syncthreads();
    // III
    if (l + 1 < J.m) i8_load(C, uniform_ptr(bbase + gview(J.b_off)[l + 1]), 0, P0);
    i8_gemm2(C, P1, X, s_eT + kSP, Ep);
    if (l + 1 == J.m) {
      // E_m[0][0] = E'^T[0][0]: wave 0, lane 0, tile 0, e = 0
      if (tid == 0) {
        s_ov[0] = Ep[0][0][0];
        s_ov[1] = Ep[0][1][0];
      }
    } else {
      double rm = 0.0;
#pragma unroll
      for (int bt = 0; bt < 4; ++bt)
#pragma unroll
        for (int e = 0; e < 4; ++e) rm = fmax(rm, fmax(fabs(Ep[bt][0][e]), fabs(Ep[bt][1][e])));
      rm = fmax(rm, __shfl_xor(rm, 16, 64));
      rm = fmax(rm, __shfl_xor(rm, 32, 64));
      const int er = exp_above_i8(rm);
      i8_store(C, Y, Ep, er);
      if (C.g == 0) s_ea[col] = er;
    }
    __syncthreads();
    uint8_t *t = X;
    X = Y;
    Y = t;
  }
  ov_re = s_ov[0];
  ov_im = s_ov[1];
  __syncthreads();
}

template <int PREC>
constexpr int threads_of() {
  return PREC == QK_SPLIT_BF16 ? kSplitThreads : PREC == QK_SPLIT_I8 ? kI8Threads : kThreads;
}

template <int PREC, int MAXP>
__global__ __launch_bounds__(threads_of<PREC>(), 2) void gram_kernel(const GramJobDev *__restrict__ jobs,
                                                        const GramTile *__restrict__ tiles,
                                                        int64_t n_tiles, int nq, int side,
                                                        unsigned long long *counters) {
  extern __shared__ __align__(16) uint8_t smem[];
  __shared__ int64_t s_slot;
  __shared__ double s_red[4];
  __shared__ double s_ov[2];
  __shared__ int s_ea[MAXP];
  __shared__ int s_eT[2 * MAXP];
  __shared__ double s_mx[4 * MAXP];
  int job;
  int64_t i, j;
  bool valid;
  while (next_pair(jobs, tiles, n_tiles, nq, side, counters, &s_slot, &job, &i, &j, &valid)) {
    if (!valid) continue;
    const GramJobDev &J = jobs[job];
    double k;
    if constexpr (PREC == QK_FP64) {
      double re, im;
      int ex;
      overlap_plain<double, f64x4, double2, MAXP>(J, J.a0 + i, J.b0 + j,
                                                  reinterpret_cast<double2 *>(smem), s_red, re, im, ex);
      k = ldexp(re * re + im * im, 2 * ex);
    } else if constexpr (PREC == QK_FP32) {
      float re, im;
      int ex;
      overlap_plain<float, f32x4, float2, MAXP>(J, J.a0 + i, J.b0 + j, reinterpret_cast<float2 *>(smem),
                                                reinterpret_cast<float *>(s_red), re, im, ex);
      k = ldexp(double(re) * re + double(im) * im, 2 * ex);
    } else if constexpr (PREC == QK_SPLIT_BF16) {
      double re, im;
      int ex;
      overlap_split<MAXP>(J, J.a0 + i, J.b0 + j, smem, smem + size_t(MAXP) * MAXP * 16, s_ea, s_eT, s_mx, s_ov,
                          re, im, ex);
      k = ldexp(re * re + im * im, 2 * ex);
    } else {
      static_assert(MAXP == kSP, "the split-int8 form uses 64 x 64 site blocks");
      double re, im;
      overlap_i8(J, J.a0 + i, J.b0 + j, smem, smem + kI8BufBytes, s_ea, s_eT, s_ov, re, im);
      k = re * re + im * im;
    }
    if (threadIdx.x == 0) write_k(J, i, j, k);
  }
}

template <int PREC, int MAXP>
size_t lds_bytes() {
  if (PREC == QK_FP64) return size_t(MAXP) * MAXP * 16;
  if (PREC == QK_FP32) return size_t(MAXP) * MAXP * 8;
  if (PREC == QK_SPLIT_BF16) return size_t(MAXP) * MAXP * 32;   // E slices + T slices
  return size_t(2) * kI8BufBytes;                                  // two int8 operand buffers
}

template <int PREC, int MAXP>
qk_status launch_one(const GramJobDev *jobs_dev, const GramTile *tiles_dev, int64_t n_tiles,
                     unsigned long long *counters, const GramConfig &cfg, hipStream_t stream, int *grid_out,
                     hipEvent_t ev0, hipEvent_t ev1) {
  int dev = 0, cus = 256;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  const size_t lds = lds_bytes<PREC, MAXP>();
  auto kern = gram_kernel<PREC, MAXP>;
  QK_HIP_CHECK(hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, int(lds)));
  int per_cu = 0;
  QK_HIP_CHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, threads_of<PREC>(), lds));
  per_cu = std::max(per_cu, 1);
  int64_t grid = int64_t(cus) * per_cu;
  grid = std::min<int64_t>(grid, std::max<int64_t>(n_tiles * cfg.tile_side * cfg.tile_side, 1));
  // every queue needs workgroups: at most one queue per workgroup
  const int nq = int(std::min<int64_t>(cfg.queues, grid));
  if (ev0) QK_HIP_CHECK(hipEventRecord(ev0, stream));
  hipLaunchKernelGGL(kern, dim3(unsigned(grid)), dim3(threads_of<PREC>()), lds, stream, jobs_dev, tiles_dev,
                     n_tiles, nq, cfg.tile_side, counters);
  QK_HIP_CHECK(hipGetLastError());
  if (ev1) QK_HIP_CHECK(hipEventRecord(ev1, stream));
  *grid_out = int(grid);
  return QK_OK;
}

// Gram kernel of the plain forms for bond pads up to 128: one pair per
// workgroup at a time, E and E' in the workgroup's slot of escratch.
constexpr size_t kWideSlot = size_t(2) * kWideP * kWideP;   // complex elements per workgroup

template <int PREC>
__global__ __launch_bounds__(kWideThreads, 1) void gram_wide_kernel(const GramJobDev *__restrict__ jobs,
                                                                  const GramTile *__restrict__ tiles,
                                                                  int64_t n_tiles, int nq, int side,
                                                                  unsigned long long *counters, uint8_t *escratch) {
  __shared__ int64_t s_slot;
  __shared__ double s_red[kWideWaves];
  int job;
  int64_t i, j;
  bool valid;
  while (next_pair(jobs, tiles, n_tiles, nq, side, counters, &s_slot, &job, &i, &j, &valid)) {
    if (!valid) continue;
    const GramJobDev &J = jobs[job];
    double k;
    if constexpr (PREC == QK_FP64) {
      double2 *E = reinterpret_cast<double2 *>(escratch) + blockIdx.x * kWideSlot;
      double re, im;
      int ex;
      overlap_wide<double, f64x4, double2>(J, J.a0 + i, J.b0 + j, E, E + kWideP * kWideP, s_red, re, im, ex);
      k = ldexp(re * re + im * im, 2 * ex);
    } else {
      float2 *E = reinterpret_cast<float2 *>(escratch) + blockIdx.x * kWideSlot;
      float re, im;
      int ex;
      overlap_wide<float, f32x4, float2>(J, J.a0 + i, J.b0 + j, E, E + kWideP * kWideP,
                                         reinterpret_cast<float *>(s_red), re, im, ex);
      k = ldexp(double(re) * re + double(im) * im, 2 * ex);
    }
    if (threadIdx.x == 0) write_k(J, i, j, k);
  }
}

template <int PREC>
qk_status launch_wide(const GramJobDev *jobs_dev, const GramTile *tiles_dev, int64_t n_tiles,
                      unsigned long long *counters, const GramConfig &cfg, const DevAlloc &al, hipStream_t stream,
                      int *grid_out, hipEvent_t ev0, hipEvent_t ev1) {
  int dev = 0, cus = 256;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  auto kern = gram_wide_kernel<PREC>;
  int per_cu = 0;
  QK_HIP_CHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, kWideThreads, 0));
  per_cu = std::max(per_cu, 1);
  int64_t grid = int64_t(cus) * per_cu;
  grid = std::min<int64_t>(grid, std::max<int64_t>(n_tiles * cfg.tile_side * cfg.tile_side, 1));
  const int nq = int(std::min<int64_t>(cfg.queues, grid));
  // one E / E' slot per workgroup
  const size_t slot = (PREC == QK_FP64 ? sizeof(double2) : sizeof(float2)) * kWideSlot;
  uint8_t *es = static_cast<uint8_t *>(dev_alloc(al, slot * size_t(grid), stream, true));
  if (!es) return fail(QK_ENOMEM, "device allocation of the Gram E scratch failed");
  qk_status st = QK_OK;
  if (ev0 && hipEventRecord(ev0, stream) != hipSuccess) st = fail(QK_EDEVICE, "event record failed");
  if (st == QK_OK) {
    hipLaunchKernelGGL(kern, dim3(unsigned(grid)), dim3(kWideThreads), 0, stream, jobs_dev, tiles_dev, n_tiles, nq,
                       cfg.tile_side, counters, es);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) st = fail(QK_EDEVICE, std::string("Gram kernel launch -> ") + hipGetErrorString(e));
  }
  if (st == QK_OK && ev1 && hipEventRecord(ev1, stream) != hipSuccess) st = fail(QK_EDEVICE, "event record failed");
  dev_free(al, es, stream, true);
  *grid_out = int(grid);
  return st;
}

}  // namespace

// Device scratch of the allocation-free Gram entry point: work-queue
// counters, job table and pair-tile list of one launch.  Each device holds
// its own copy until the process ends; host code reaches it only through the
// address that hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) uint8_t scratch[kNoAllocScratchBytes];

namespace {
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxScratchDevices] = {};
}  // namespace

qk_status noalloc_scratch(void **ptr) {
  int dev = 0;
  QK_HIP_CHECK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxScratchDevices) return fail(QK_EINVAL, "device index out of range");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      (void)hipGetLastError();
      return fail(QK_EDEVICE, std::string("hipGetSymbolAddress of the Gram scratch -> ") + hipGetErrorString(e));
    }
    g_scratch_ptr[dev] = p;
  }
  *ptr = g_scratch_ptr[dev];
  return QK_OK;
}

qk_status launch_gram_cfg(const std::vector<GramJobDev> &jobs_in, int max_pad, qk_precision prec,
                          const GramConfig &cfg, hipStream_t stream, qk_gram_stats *stats, void *ws_given,
                          size_t ws_cap) {
  if (max_pad > kWideP) return fail(QK_ENOTSUP, "Gram kernels support bond pads up to 128");
  if (max_pad > 64 && prec != QK_FP64 && prec != QK_FP32)
    return fail(QK_ENOTSUP, "the split forms support bond pads up to 64");
  if (max_pad > 64 && ws_given)
    return fail(QK_ENOTSUP, "the allocation-free Gram supports bond pads up to 64");
  if (cfg.maxp < max_pad) return fail(QK_EINVAL, "tile configuration smaller than the batch's bond pads");
  const int side = cfg.tile_side;
  std::vector<GramJobDev> jobs = jobs_in;
  std::vector<GramTile> tiles;
  for (size_t k = 0; k < jobs.size(); ++k) {
    GramJobDev &J = jobs[k];
    J.tiles_i = (J.na + side - 1) / side;
    J.tiles_j = (J.nb + side - 1) / side;
    J.pair_begin = int64_t(tiles.size()) * (side * side);
    for (int64_t ti = 0; ti < J.tiles_i; ++ti)
      for (int64_t tj = 0; tj < J.tiles_j; ++tj) {
        if (J.upper) {
          // skip tiles entirely below the global diagonal
          const int64_t max_col = J.b0 + std::min(J.nb, (tj + 1) * side) - 1;
          const int64_t min_row = J.a0 + ti * side;
          if (max_col < min_row) continue;
        }
        tiles.push_back(GramTile{int32_t(k), int32_t(ti), int32_t(tj), 0});
      }
  }
  if (stats) {
    stats->tiles = int64_t(tiles.size());
    stats->tile_side = side;
    stats->queues = cfg.queues;
    stats->block = cfg.maxp;
    stats->workgroups = 0;
    stats->kernel_ms = 0.0;
  }
  if (tiles.empty()) return QK_OK;
  const int64_t n_tiles = int64_t(tiles.size());
  const size_t jbytes = sizeof(GramJobDev) * jobs.size();
  const size_t tbytes = sizeof(GramTile) * tiles.size();
  // workspace: [queue counters | job table | tile list], uploaded in one copy
  // whose counter bytes are zero (no memset node in the stream)
  const size_t ws_bytes = kGramCounterBytes + jbytes + tbytes;
  if (ws_given && ws_bytes > ws_cap)
    return fail(QK_EINVAL, "the Gram work queue needs " + std::to_string(ws_bytes) + " bytes (" +
                               std::to_string(n_tiles) + " pair tiles of side " + std::to_string(side) +
                               "), above the " + std::to_string(ws_cap) + "-byte scratch");
  std::vector<uint8_t> host(ws_bytes, 0);
  std::memcpy(host.data() + kGramCounterBytes, jobs.data(), jbytes);
  std::memcpy(host.data() + kGramCounterBytes + jbytes, tiles.data(), tbytes);
  const DevAlloc al = allocator_for_current_device();
  uint8_t *ws = static_cast<uint8_t *>(ws_given);
  if (!ws) {
    ws = static_cast<uint8_t *>(dev_alloc(al, ws_bytes, stream, true));
    if (!ws) return fail(QK_ENOMEM, "device allocation of the Gram work queue failed");
  }
  auto *counters = reinterpret_cast<unsigned long long *>(ws);
  auto *jobs_dev = reinterpret_cast<GramJobDev *>(ws + kGramCounterBytes);
  auto *tiles_dev = reinterpret_cast<GramTile *>(ws + kGramCounterBytes + jbytes);
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  qk_status st = QK_OK;
  if (hipMemcpyAsync(ws, host.data(), ws_bytes, hipMemcpyHostToDevice, stream) != hipSuccess ||
      // the host buffer must stay alive until the copy has run
      hipStreamSynchronize(stream) != hipSuccess)
    st = fail(QK_EDEVICE, "upload of the Gram work queue failed");
  if (st == QK_OK && stats &&
      (hipEventCreate(&ev0) != hipSuccess || hipEventCreate(&ev1) != hipSuccess))
    st = fail(QK_EDEVICE, "event creation failed");
  int grid = 0;
  if (st == QK_OK) {
    if (cfg.maxp == kWideP && (prec == QK_FP64 || prec == QK_FP32))
      st = prec == QK_FP64 ? launch_wide<QK_FP64>(jobs_dev, tiles_dev, n_tiles, counters, cfg, al, stream, &grid, ev0, ev1)
                           : launch_wide<QK_FP32>(jobs_dev, tiles_dev, n_tiles, counters, cfg, al, stream, &grid, ev0, ev1);
    else if (prec == QK_FP64)
      st = cfg.maxp == 32 ? launch_one<QK_FP64, 32>(jobs_dev, tiles_dev, n_tiles, counters, cfg, stream, &grid, ev0, ev1)
                          : launch_one<QK_FP64, 64>(jobs_dev, tiles_dev, n_tiles, counters, cfg, stream, &grid, ev0, ev1);
    else if (prec == QK_FP32)
      st = cfg.maxp == 32 ? launch_one<QK_FP32, 32>(jobs_dev, tiles_dev, n_tiles, counters, cfg, stream, &grid, ev0, ev1)
                          : launch_one<QK_FP32, 64>(jobs_dev, tiles_dev, n_tiles, counters, cfg, stream, &grid, ev0, ev1);
    else if (prec == QK_SPLIT_BF16)
      st = launch_one<QK_SPLIT_BF16, 64>(jobs_dev, tiles_dev, n_tiles, counters, cfg, stream, &grid, ev0, ev1);
    else
      st = launch_one<QK_SPLIT_I8, 64>(jobs_dev, tiles_dev, n_tiles, counters, cfg, stream, &grid, ev0, ev1);
  }
  if (!ws_given) dev_free(al, ws, stream, true);
  if (st == QK_OK && stats) {
    float ms = 0.f;
    if (hipEventSynchronize(ev1) != hipSuccess || hipEventElapsedTime(&ms, ev0, ev1) != hipSuccess)
      st = fail(QK_EDEVICE, "Gram kernel failed");
    stats->workgroups = grid;
    stats->kernel_ms = ms;
  }
  if (ev0) (void)hipEventDestroy(ev0);
  if (ev1) (void)hipEventDestroy(ev1);
  return st;
}


// ------------------------------------------------------------------------
// Kernel configurations and the autotuner.  A configuration is the block
// size of the plain forms (32, 64, or 128 with E in global scratch), the pair-tile side and the number of
// work queues.  Defaults were chosen by measurement on 165-site chi = 64
// batches; mps_gram_autotune times every valid configuration on a sample of
// the caller's batch and stores the fastest per (device, form, pad bucket).

namespace {
std::mutex g_tune_mu;
std::map<std::tuple<int, int, int>, GramConfig> g_tuned;

int pad_bucket(int max_pad) { return max_pad <= 32 ? 32 : max_pad <= 64 ? 64 : 128; }
}  // namespace

GramConfig default_gram_config(qk_precision prec, int max_pad) {
  GramConfig c;
  c.maxp = max_pad > 64 ? kWideP : 64;
  c.tile_side = kDefaultTileSide;
  c.queues = prec == QK_SPLIT_I8 ? kQueues : 1;
  return c;
}

std::vector<GramConfig> gram_config_candidates(qk_precision prec, int max_pad) {
  std::vector<GramConfig> out;
  std::vector<int> maxps{max_pad > 64 ? kWideP : 64};
  if ((prec == QK_FP64 || prec == QK_FP32) && max_pad <= 32) maxps.push_back(32);
  for (int mp : maxps)
    for (int side : {8, 16, 32})
      for (int nq : {1, kQueues}) {
        GramConfig c;
        c.maxp = mp;
        c.tile_side = side;
        c.queues = nq;
        out.push_back(c);
      }
  return out;
}

GramConfig current_gram_config(qk_precision prec, int max_pad) {
  int dev = 0;
  (void)hipGetDevice(&dev);
  std::lock_guard<std::mutex> lk(g_tune_mu);
  auto it = g_tuned.find(std::make_tuple(dev, int(prec), pad_bucket(max_pad)));
  return it != g_tuned.end() ? it->second : default_gram_config(prec, max_pad);
}

void store_gram_config(qk_precision prec, int max_pad, const GramConfig &c) {
  int dev = 0;
  (void)hipGetDevice(&dev);
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tuned[std::make_tuple(dev, int(prec), pad_bucket(max_pad))] = c;
}

void clear_gram_configs() {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tuned.clear();
}

qk_status launch_gram(const std::vector<GramJobDev> &jobs, int max_pad, qk_precision prec, hipStream_t stream,
                      qk_gram_stats *stats) {
  return launch_gram_cfg(jobs, max_pad, prec, current_gram_config(prec, max_pad), stream, stats);
}

// ------------------------------------------------------------------------
// Packing of the FP64 master into the FP32 and split-BF16 operand forms.

__global__ void pack_f32_kernel(const double2 *__restrict__ src, float2 *__restrict__ dst, int64_t count) {
  for (int64_t x = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; x < count;
       x += int64_t(gridDim.x) * blockDim.x) {
    const double2 v = src[x];
    dst[x] = make_float2(float(v.x), float(v.y));
  }
}

// One block per (site, mps): column exponents e[s][c] (max |x| < 2^e over the
// column's rows and both planes), then the four fixed-point slices of every
// value, in B-operand fragment order, on a 64 x 64 block (zero beyond the
// batch's pads).
__global__ __launch_bounds__(256) void pack_split_kernel(const double2 *__restrict__ src, uint8_t *__restrict__ dst,
                                                         const int32_t *__restrict__ pad,
                                                         const int64_t *__restrict__ site_off,
                                                         const int64_t *__restrict__ split_off, int64_t mps_stride,
                                                         int64_t split_stride, int32_t m, int64_t n) {
  const int l = blockIdx.x;
  const int64_t i = blockIdx.y;
  if (i >= n || l >= m) return;
  __shared__ int s_e[2 * 128];
  const int pl = pad[l], pr = pad[l + 1];
  const double2 *site = src + i * mps_stride + site_off[l];
  uint8_t *out = dst + i * split_stride + split_off[l];
  for (int t = threadIdx.x; t < 2 * 128; t += blockDim.x) {
    const int s = t / 128, c = t % 128;
    int e = 0;
    if (c < pr) {
      double mx = 0.0;
      for (int r = 0; r < pl; ++r) {
        const double2 x = site[(size_t(s) * pl + r) * pr + c];
        mx = fmax(mx, fmax(fabs(x.x), fabs(x.y)));
      }
      e = max(exp_above(mx), -127);   // int8 storage; |x| < 2^e still holds
    }
    s_e[t] = e;
    out[t] = uint8_t(int8_t(e));
  }
  __syncthreads();
  const int work = 2 * 2 * 4 * 64;   // (s, kc, ct, lane)
  for (int w = threadIdx.x; w < work; w += blockDim.x) {
    const int lane = w % 64;
    const int ct = (w / 64) % 4;
    const int kc = (w / 256) % 2;
    const int s = w / 512;
    const int jj = lane & 15, gg = lane >> 4;
    const int col = 16 * ct + jj;
    const int e = s_e[s * 128 + col];
    uint32_t sl[2][8][4];
#pragma unroll
    for (int v = 0; v < 8; ++v) {
      const int row = 32 * kc + (v < 4 ? 4 * gg + v : 16 + 4 * gg + (v - 4));
      double2 x = make_double2(0.0, 0.0);
      if (row < pl && col < pr) x = site[(size_t(s) * pl + row) * pr + col];
      slice4e(x.x, e, sl[0][v]);
      slice4e(x.y, e, sl[1][v]);
    }
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        uint4 o;
        o.x = sl[q][0][k] | (sl[q][1][k] << 16);
        o.y = sl[q][2][k] | (sl[q][3][k] << 16);
        o.z = sl[q][4][k] | (sl[q][5][k] << 16);
        o.w = sl[q][6][k] | (sl[q][7][k] << 16);
        *reinterpret_cast<uint4 *>(out + kSplitExpBytes + ((size_t(((s * 4 + k) * 2 + q) * 2 + kc) * 4 + ct) * 1024 +
                                                           lane * 16)) = o;
      }
  }
}

// ------------------------------------------------------------------------
// Gather: record k of the destination is record idx[k] of the source.  One
// launch per form instead of one copy per MPS.

__global__ __launch_bounds__(256) void gather_records_kernel(const uint4 *__restrict__ src, uint4 *__restrict__ dst,
                                                             const int64_t *__restrict__ idx, int64_t rec_vecs,
                                                             int64_t k0, int64_t count) {
  const int64_t k = k0 + blockIdx.y;
  if (k >= count) return;
  const uint4 *s = src + idx[k] * rec_vecs;
  uint4 *d = dst + k * rec_vecs;
  for (int64_t x = int64_t(blockIdx.x) * 256 + threadIdx.x; x < rec_vecs; x += int64_t(gridDim.x) * 256) d[x] = s[x];
}

__global__ __launch_bounds__(256) void gather_meta_kernel(const qk_mps_batch_meta src, qk_mps_batch_meta dst,
                                                          const int64_t *__restrict__ idx, int32_t m1,
                                                          int64_t count) {
  const int64_t k = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (k >= count) return;
  const int64_t i = idx[k];
  for (int t = 0; t < m1; ++t) dst.dims[k * m1 + t] = src.dims[i * m1 + t];
  dst.disc[k] = src.disc[i];
  dst.maxdisc[k] = src.maxdisc[i];
  dst.degen[k] = src.degen[i];
  dst.unconv[k] = src.unconv[i];
}

qk_status launch_gather_records(const void *src, void *dst, const int64_t *idx_dev, int64_t rec_bytes,
                                int64_t count, hipStream_t stream) {
  if (count == 0 || rec_bytes == 0) return QK_OK;
  if (rec_bytes % 16) return fail(QK_EINVAL, "gather record size is not a multiple of 16 bytes");
  const int64_t vecs = rec_bytes / 16;
  const unsigned gx = unsigned(std::min<int64_t>((vecs + 255) / 256, 64));
  for (int64_t k0 = 0; k0 < count; k0 += 65535) {
    const unsigned gy = unsigned(std::min<int64_t>(65535, count - k0));
    hipLaunchKernelGGL(gather_records_kernel, dim3(gx, gy), dim3(256), 0, stream,
                       reinterpret_cast<const uint4 *>(src), reinterpret_cast<uint4 *>(dst), idx_dev, vecs, k0,
                       count);
    QK_HIP_CHECK(hipGetLastError());
  }
  return QK_OK;
}

qk_status launch_gather_meta(const qk_mps_batch_meta &src, const qk_mps_batch_meta &dst, const int64_t *idx_dev,
                             int32_t m1, int64_t count, hipStream_t stream) {
  if (count == 0) return QK_OK;
  hipLaunchKernelGGL(gather_meta_kernel, dim3(unsigned((count + 255) / 256)), dim3(256), 0, stream, src, dst,
                     idx_dev, m1, count);
  QK_HIP_CHECK(hipGetLastError());
  return QK_OK;
}

// One block per (site, mps) for the split-int8 form: column exponents (with
// the int8 margin), the int8 digit fragments in B-operand order and the
// column digit sums of the imaginary plane.
__global__ __launch_bounds__(256) void pack_i8_kernel(const double2 *__restrict__ src, uint8_t *__restrict__ dst,
                                                      const int32_t *__restrict__ pad,
                                                      const int64_t *__restrict__ site_off, int64_t mps_stride,
                                                      int64_t i8_stride, int32_t m, int64_t n) {
  const int l = blockIdx.x;
  const int64_t i = blockIdx.y;
  if (i >= n || l >= m) return;
  __shared__ int s_e[2 * 128];
  const int pl = pad[l], pr = pad[l + 1];
  const double2 *site = src + i * mps_stride + site_off[l];
  uint8_t *out = dst + i * i8_stride + int64_t(l) * kI8SiteBytes;
  auto value = [&](int s, int row, int col, int q) -> double {
    if (row >= pl || col >= pr) return 0.0;
    const double2 x = site[(size_t(s) * pl + row) * pr + col];
    return q ? x.y : x.x;
  };
  for (int t = threadIdx.x; t < 2 * 128; t += blockDim.x) {
    const int s = t / 128, c = t % 128;
    int e = 0;
    if (c < pr) {
      double mx = 0.0;
      for (int r = 0; r < pl; ++r) {
        const double2 x = site[(size_t(s) * pl + r) * pr + c];
        mx = fmax(mx, fmax(fabs(x.x), fabs(x.y)));
      }
      e = max(exp_above_i8(mx), -127);   // int8 storage; |x| < 2^e still holds
    }
    s_e[t] = e;
    out[t] = uint8_t(int8_t(e));
  }
  __syncthreads();
  // fragments: work item (s, q, ct, lane), 16 rows each
  for (int w = threadIdx.x; w < 2 * 2 * 4 * 64; w += blockDim.x) {
    const int lane = w % 64;
    const int ct = (w / 64) % 4;
    const int q = (w / 256) % 2;
    const int s = w / 512;
    const int jj = lane & 15, gg = lane >> 4;
    const int col = 16 * ct + jj;
    const double scale = ldexp(1.0, 31 - s_e[s * 128 + col]);
    uint32_t sl[4][4];   // [group of four rows][digit]
#pragma unroll
    for (int vv = 0; vv < 4; ++vv) {
      uint32_t d[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int v = 4 * vv + r;
        const int row = 16 * (2 * (v >> 3) + ((v >> 2) & 1)) + 4 * gg + (v & 3);
        d[r] = biased_digit_word(value(s, row, col, q), scale);
      }
      transpose_digits(d[0], d[1], d[2], d[3], sl[vv]);
    }
#pragma unroll
    for (int k = 0; k < 4; ++k)
      *reinterpret_cast<uint4 *>(out + kI8ExpBytes + kI8SumBytes +
                                 size_t(((s * 4 + k) * 2 + q) * 4 + ct) * kI8FragBytes + lane * 16) =
          make_uint4(sl[0][k], sl[1][k], sl[2][k], sl[3][k]);
  }
  // column digit sums of the imaginary plane: item (s, k, c)
  int *cs = reinterpret_cast<int *>(out + kI8ExpBytes);
  for (int t = threadIdx.x; t < 2 * 4 * 64; t += blockDim.x) {
    const int c = t % 64, k = (t / 64) % 4, s = t / 256;
    const double scale = ldexp(1.0, 31 - s_e[s * 128 + c]);
    int sum = 0;
    for (int r = 0; r < 64; ++r)
      sum += int(int8_t((biased_digit_word(value(s, r, c, 1), scale) ^ 0x808080u) >> (8 * (3 - k))));
    cs[(s * 4 + k) * 64 + c] = sum;
  }
}

qk_status launch_pack_i8(const qk_mps_batch *b, hipStream_t stream) {
  if (b->n == 0) return QK_OK;
  const int64_t chunk = 65535;
  for (int64_t i0 = 0; i0 < b->n; i0 += chunk) {
    const int64_t cnt = std::min(chunk, b->n - i0);
    hipLaunchKernelGGL(pack_i8_kernel, dim3(unsigned(b->m), unsigned(cnt)), dim3(256), 0, stream,
                       b->f64 + i0 * b->mps_stride, b->si8 + i0 * b->i8_stride, b->pad_dev, b->site_off_dev,
                       b->mps_stride, b->i8_stride, b->m, cnt);
    QK_HIP_CHECK(hipGetLastError());
  }
  return QK_OK;
}

qk_status launch_pack_f32(const qk_mps_batch *b, hipStream_t stream) {
  const int64_t count = b->n * b->mps_stride;
  if (count == 0) return QK_OK;
  const int64_t blocks = std::min<int64_t>((count + 255) / 256, 65536);
  hipLaunchKernelGGL(pack_f32_kernel, dim3(unsigned(blocks)), dim3(256), 0, stream, b->f64, b->f32, count);
  QK_HIP_CHECK(hipGetLastError());
  return QK_OK;
}

qk_status launch_pack_split(const qk_mps_batch *b, hipStream_t stream) {
  if (b->n == 0) return QK_OK;
  if (b->n > 65535 * 16) return fail(QK_ENOTSUP, "batch too large for the packing grid");
  // grid.y = MPS (chunked), grid.z = site
  const int64_t chunk = 65535;
  for (int64_t i0 = 0; i0 < b->n; i0 += chunk) {
    const int64_t cnt = std::min(chunk, b->n - i0);
    hipLaunchKernelGGL(pack_split_kernel, dim3(unsigned(b->m), unsigned(cnt)), dim3(256), 0, stream,
                       b->f64 + i0 * b->mps_stride, b->sbf16 + i0 * b->split_stride, b->pad_dev,
                       b->site_off_dev, b->split_off_dev, b->mps_stride, b->split_stride, b->m, cnt);
    QK_HIP_CHECK(hipGetLastError());
  }
  return QK_OK;
}

}  // namespace qk
