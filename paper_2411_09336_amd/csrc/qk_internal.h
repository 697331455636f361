// Internal declarations shared by the host library and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/qkmps.h"

namespace qk {

// Thread-local error reporting used by every C-ABI entry point.
void set_error(const std::string &msg);
qk_status fail(qk_status st, const std::string &msg);

#define QK_HIP_CHECK(expr)                                                     \
  do {                                                                         \
    hipError_t _e = (expr);                                                    \
    if (_e != hipSuccess)                                                      \
      return ::qk::fail(QK_EDEVICE, std::string(#expr " -> ") +               \
                                        hipGetErrorString(_e));                \
  } while (0)

constexpr int kPadQuantum = 32;      // bond pads are multiples of 32
constexpr int kMaxBond = 128;        // largest supported pad in a batch
constexpr int kMaxSimChi = 128;      // largest bond cap in simulation

inline int pad_of(int d) { return ((d + kPadQuantum - 1) / kPadQuantum) * kPadQuantum; }

// Split-BF16 operand form (fixed-point slices).  Every real value x of a
// site tensor column c (per physical index s) is written as
//   x = 2^(e[s][c] - 7) * (n0 + n1 2^-8 + n2 2^-16 + n3 2^-24) + O(2^(e-32))
// with a shared column exponent e[s][c] (max |x| of the column times
// 1 + 2^-30 is below 2^e, so codes never saturate; e >= -127) and
// integers |n_k| <= 128; slice k is stored as the bf16 value n_k 2^(-8k),
// which is exact.  Products of leading slices are integers below 2^14, so
// the (0,0) slice product accumulates exactly in an FP32 MFMA accumulator.
// A site block is:
//   [int8 exponents e[s][c], s in {0,1}, c < 128 : 256 bytes]
//   [fragments: [s][slice 0..3][plane 0..1 = re, im][kc][ct][lane][8 bf16]]
// where fragment (kc, ct) is the MFMA B-operand of K = 32 rows by 16
// columns: lane l = j + 16 g, slot v holds row perm(kc, g, v), column
// 16 ct + j, with
//   perm(kc, g, v) = 32 kc + 4 g + v          for v < 4
//                  = 32 kc + 16 + 4 g + v - 4 for v >= 4.
constexpr int kFragBytes = 64 * 8 * 2;   // 1 KiB
constexpr int kSlices = 4;
constexpr int kSplitExpBytes = 256;

// Every site of the split form is a 64 x 64 block (zero beyond the batch's
// pads); batches with pads above 64 have no split form.
constexpr int kSplitMaxPad = 64;
constexpr int64_t split_site_bytes() {
  return kSplitExpBytes + int64_t(2) * kSlices * 2 * (kSplitMaxPad / 32) * (kSplitMaxPad / 16) * kFragBytes;
}

// Split-int8 operand form: the same 31-bit codes (row / column exponent e
// with max |x| (1 + 2^-7) < 2^e, so the leading digit is in [-127, 127]) cut
// into four balanced base-256 digits stored as int8.  A site block is:
//   [int8 exponents e[s][c], s in {0,1}, c < 128 : 256 bytes]
//   [int32 column digit sums of the imaginary plane cs[s][k][c], c < 64 :
//    2048 bytes]
//   [fragments [s][digit k 0..3][plane 0..1][ct 0..3][lane][16 int8]]
// where fragment ct is the B operand of v_mfma_i32_16x16x64_i8 for columns
// 16 ct .. 16 ct + 15: lane l = j + 16 g, byte v holds row
//   perm(g, v) = 16 (2 (v >> 3) + ((v >> 2) & 1)) + 4 g + (v & 3)
// of column 16 ct + j.  Every site is a 64 x 64 block (zero beyond the pads).
constexpr int kI8ExpBytes = 256;
constexpr int kI8SumBytes = 2 * 4 * 64 * 4;
constexpr int kI8FragBytes = 64 * 16;
constexpr int kI8BufBytes = 4 * 4 * 2 * kI8FragBytes;   // one A-operand buffer (64 rows)
constexpr int64_t kI8SiteBytes = kI8ExpBytes + kI8SumBytes + int64_t(2) * 4 * 2 * 4 * kI8FragBytes;

// Device memory of the library.  Batch arrays, packed planes and scratch
// buffers come from the allocator registered for the device with qk_init
// (for example a framework's caching allocator), else from hipMalloc /
// hipFree (batches) and hipMallocAsync / hipFreeAsync (stream-ordered
// scratch).  A batch keeps the allocator that made it.
struct DevAlloc {
  qk_allocator user{};
  bool custom() const { return user.alloc != nullptr; }
};
DevAlloc allocator_for_current_device();
void *dev_alloc(const DevAlloc &al, size_t bytes, hipStream_t stream, bool scratch);
void dev_free(const DevAlloc &al, void *p, hipStream_t stream, bool scratch);

}  // namespace qk

// Opaque batch.  Every MPS of a batch has m sites with the pad profile
// pad[0..m]; site l of MPS i starts at complex offset
//   i * mps_stride + site_off[l]
// in the FP64 (complex128) and FP32 (complex64) forms, and at byte offset
//   i * split_stride + split_off[l]
// in the split-BF16 form.
struct qk_mps_batch {
  int device = 0;
  qk::DevAlloc alloc;              // allocator of every array below
  int64_t n = 0;
  int32_t m = 0;
  std::vector<int32_t> pad;        // m + 1 entries
  std::vector<int64_t> site_off;   // m + 1 entries (last = mps_stride)
  int64_t mps_stride = 0;          // complex elements per MPS
  std::vector<int64_t> split_off;  // m + 1 entries, bytes
  int64_t split_stride = 0;        // bytes per MPS
  std::vector<int64_t> i8_off;     // m + 1 entries, bytes (split-int8 form)
  int64_t i8_stride = 0;           // bytes per MPS

  double2 *f64 = nullptr;          // n * mps_stride
  float2 *f32 = nullptr;           // packed on demand
  uint8_t *sbf16 = nullptr;        // packed on demand
  uint8_t *si8 = nullptr;          // packed on demand

  int32_t *dims_dev = nullptr;     // n * (m + 1)
  int32_t *pad_dev = nullptr;      // m + 1
  int64_t *site_off_dev = nullptr; // m + 1
  int64_t *split_off_dev = nullptr;// m + 1
  int64_t *i8_off_dev = nullptr;   // m + 1
  double *disc_dev = nullptr;      // n: summed discarded weight
  double *maxdisc_dev = nullptr;   // n: largest single discarded weight
  int32_t *degen_dev = nullptr;    // n: near-degenerate cuts
  int32_t *unconv_dev = nullptr;   // n: SVDs at the sweep limit

  int32_t n_two_qubit_gates = 0;
};

namespace qk {

// Allocate a batch with the given pad profile (device memory zeroed).
qk_status batch_create(int64_t n, int32_t m, const std::vector<int32_t> &pad,
                       hipStream_t stream, qk_mps_batch **out, bool with_f64 = true);
qk_status batch_ensure_packed(qk_mps_batch *b, qk_precision prec, hipStream_t stream);

// Per-MPS metadata arrays of a batch (device pointers).
struct qk_mps_batch_meta {
  int32_t *dims;
  double *disc, *maxdisc;
  int32_t *degen, *unconv;
};

// Launchers implemented in the .hip files.
qk_status launch_gather_records(const void *src, void *dst, const int64_t *idx_dev, int64_t rec_bytes,
                                int64_t count, hipStream_t stream);
qk_status launch_gather_meta(const qk_mps_batch_meta &src, const qk_mps_batch_meta &dst, const int64_t *idx_dev,
                             int32_t m1, int64_t count, hipStream_t stream);
qk_status launch_pack_f32(const qk_mps_batch *b, hipStream_t stream);
qk_status launch_pack_split(const qk_mps_batch *b, hipStream_t stream);
qk_status launch_pack_i8(const qk_mps_batch *b, hipStream_t stream);

struct GramJobDev {
  const void *a_base;              // form-specific base pointer of batch a
  const void *b_base;
  const int64_t *a_off;            // per-site offsets (complex elems or bytes)
  const int64_t *b_off;
  const int32_t *a_pad;            // m + 1
  const int32_t *b_pad;
  int64_t a_stride, b_stride;      // per-MPS stride (complex elems or bytes)
  int64_t a0, na, b0, nb;
  double *K;
  int64_t ldk;
  int32_t m;
  int32_t upper;                   // symmetric: only global j >= i
  int64_t tiles_i, tiles_j;        // tile grid of this job
  int64_t pair_begin;              // first flat pair index of this job
};

// Gram kernel configuration: block size of the plain forms (32, 64 or 128), pair
// tile side, number of work queues (1, or one per XCD).
struct GramConfig {
  int maxp = 64;
  int tile_side = 16;
  int queues = 1;
};

qk_status launch_gram(const std::vector<GramJobDev> &jobs, int max_pad,
                      qk_precision prec, hipStream_t stream, qk_gram_stats *stats = nullptr);
// ws / ws_cap: caller-provided workspace for the work queue (nullptr: drawn
// from the device's allocator for the launch).
qk_status launch_gram_cfg(const std::vector<GramJobDev> &jobs, int max_pad,
                          qk_precision prec, const GramConfig &cfg, hipStream_t stream,
                          qk_gram_stats *stats = nullptr, void *ws = nullptr, size_t ws_cap = 0);

// Scratch of the allocation-free Gram entry point: a static device array of
// kNoAllocScratchBytes per device.  noalloc_scratch returns its address on
// the current device (looked up once per device with hipGetSymbolAddress).
constexpr size_t kNoAllocScratchBytes = size_t(8) << 20;
constexpr int kMaxScratchDevices = 64;
qk_status noalloc_scratch(void **ptr);
GramConfig default_gram_config(qk_precision prec, int max_pad);
GramConfig current_gram_config(qk_precision prec, int max_pad);
std::vector<GramConfig> gram_config_candidates(qk_precision prec, int max_pad);
void store_gram_config(qk_precision prec, int max_pad, const GramConfig &c);
void clear_gram_configs();

// Simulation launchers.
qk_status run_simulation(qk_mps_batch *b, const double *features_dev,
                         const std::vector<qk_gate> &gates,
                         const qk_circuit_spec &spec, int chi, double cutoff,
                         hipStream_t stream, qk_progress_fn fn = nullptr,
                         void *user = nullptr, int64_t every = 0, int64_t graph_circuits = 0,
                         int32_t *trace = nullptr);

std::vector<qk_gate> compile_circuit(const qk_circuit_spec &spec);
qk_status validate_spec(const qk_circuit_spec *spec);

}  // namespace qk
static_assert(qk::kNoAllocScratchBytes == QK_NOALLOC_SCRATCH_BYTES, "scratch size of the header");
