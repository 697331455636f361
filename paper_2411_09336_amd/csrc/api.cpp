// C-ABI entry points of libqkmps: argument checking, batch management and
// dispatch to the HIP launchers.  No device arithmetic lives here.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <mutex>
#include <string>
#include <vector>

#include "qk_internal.h"

namespace qk {

static thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }

qk_status fail(qk_status st, const std::string &msg) {
  g_last_error = msg;
  return st;
}

static qk_status ok() {
  g_last_error.clear();
  return QK_OK;
}

// Allocator per device index, set by qk_init.
constexpr int kMaxDevices = 64;
static std::mutex g_alloc_mu;
static DevAlloc g_alloc[kMaxDevices];

DevAlloc allocator_for_current_device() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    (void)hipGetLastError();
    dev = 0;
  }
  if (dev < 0 || dev >= kMaxDevices) return DevAlloc{};
  std::lock_guard<std::mutex> lk(g_alloc_mu);
  return g_alloc[dev];
}

void *dev_alloc(const DevAlloc &al, size_t bytes, hipStream_t stream, bool scratch) {
  if (bytes == 0) bytes = 16;
  if (al.custom()) return al.user.alloc(bytes, al.user.ctx, reinterpret_cast<void *>(stream));
  void *p = nullptr;
  const hipError_t e = scratch ? hipMallocAsync(&p, bytes, stream) : hipMalloc(&p, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  return p;
}

void dev_free(const DevAlloc &al, void *p, hipStream_t stream, bool scratch) {
  if (!p) return;
  if (al.custom()) {
    al.user.free(p, al.user.ctx, reinterpret_cast<void *>(stream));
    return;
  }
  if (scratch)
    (void)hipFreeAsync(p, stream);
  else
    (void)hipFree(p);
}

qk_status validate_spec(const qk_circuit_spec *spec) {
  if (!spec) return fail(QK_EINVAL, "circuit spec is NULL");
  if (spec->n_qubits < 1 || spec->n_qubits > 100000)
    return fail(QK_EINVAL, "n_qubits must be in [1, 100000]");
  if (spec->interaction_distance < 0) return fail(QK_EINVAL, "interaction_distance < 0");
  if (spec->repetitions < 0) return fail(QK_EINVAL, "repetitions < 0");
  if (spec->routing != 0 && spec->routing != 1) return fail(QK_EINVAL, "routing must be 0 or 1");
  if (!std::isfinite(spec->coef_z) || !std::isfinite(spec->coef_xx))
    return fail(QK_EINVAL, "angle coefficients must be finite");
  if (spec->gate_split != 0 && spec->gate_split != 1) return fail(QK_EINVAL, "gate_split must be 0 or 1");
  for (int k = 0; k < 3; ++k)
    if (spec->reserved[k] != 0) return fail(QK_EINVAL, "reserved fields must be zero");
  return QK_OK;
}

// Gate list: per repetition the Z layer (one Rz per qubit), then the XX
// layer in E_i-block order; an Rxx between qubits i and i+k is applied on
// sites (i+k-1, i+k) after SWAPs carry qubit i up to site i+k-1.
std::vector<qk_gate> compile_circuit(const qk_circuit_spec &spec) {
  const int m = spec.n_qubits, d = spec.interaction_distance;
  std::vector<qk_gate> g;
  auto push = [&](int op, int site, int fi, int fj) { g.push_back(qk_gate{op, site, fi, fj}); };
  for (int r = 0; r < spec.repetitions; ++r) {
    for (int q = 0; q < m; ++q) push(0, q, q, -1);
    for (int i = 0; i + 1 < m; ++i) {
      const int kmax = std::min(d, m - 1 - i);
      if (spec.routing == 0) {
        for (int k = 1; k <= kmax; ++k) {
          for (int p = i; p <= i + k - 2; ++p) push(2, p, -1, -1);
          push(1, i + k - 1, i, i + k);
          for (int p = i + k - 2; p >= i; --p) push(2, p, -1, -1);
        }
      } else {
        for (int k = 1; k <= kmax; ++k) {
          if (k > 1) push(2, i + k - 2, -1, -1);
          push(1, i + k - 1, i, i + k);
        }
        for (int p = i + kmax - 2; p >= i; --p) push(2, p, -1, -1);
      }
    }
  }
  return g;
}

static void compute_layout(qk_mps_batch *b) {
  const int m = b->m;
  b->site_off.assign(m + 1, 0);
  b->split_off.assign(m + 1, 0);
  b->i8_off.assign(m + 1, 0);
  for (int l = 0; l < m; ++l) {
    b->site_off[l + 1] = b->site_off[l] + int64_t(2) * b->pad[l] * b->pad[l + 1];
    b->split_off[l + 1] = b->split_off[l] + split_site_bytes();
    b->i8_off[l + 1] = b->i8_off[l] + kI8SiteBytes;
  }
  b->mps_stride = b->site_off[m];
  b->split_stride = b->split_off[m];
  b->i8_stride = b->i8_off[m];
}

static void batch_release(qk_mps_batch *b) {
  if (!b) return;
  int cur = 0;
  (void)hipGetDevice(&cur);
  (void)hipSetDevice(b->device);
  void *ptrs[] = {b->f64,          b->f32,        b->sbf16,       b->si8,       b->dims_dev,
                  b->pad_dev,      b->site_off_dev, b->split_off_dev, b->i8_off_dev, b->disc_dev,
                  b->maxdisc_dev,  b->degen_dev,   b->unconv_dev};
  // the batch may still be in use by enqueued work: wait before the memory
  // goes back to the allocator
  if (b->alloc.custom()) (void)hipDeviceSynchronize();
  for (void *p : ptrs) dev_free(b->alloc, p, nullptr, false);
  (void)hipSetDevice(cur);
  delete b;
}

qk_status batch_create(int64_t n, int32_t m, const std::vector<int32_t> &pad,
                       hipStream_t stream, qk_mps_batch **out, bool with_f64) {
  auto *b = new qk_mps_batch();
  if (hipGetDevice(&b->device) != hipSuccess) {
    (void)hipGetLastError();
    b->device = 0;
  }
  b->alloc = allocator_for_current_device();
  b->n = n;
  b->m = m;
  b->pad = pad;
  compute_layout(b);
  auto alloc = [&](void **p, size_t bytes) -> bool {
    if (bytes == 0) bytes = 16;
    *p = dev_alloc(b->alloc, bytes, stream, false);
    if (!*p) return false;
    return hipMemsetAsync(*p, 0, bytes, stream) == hipSuccess;
  };
  const size_t nn = size_t(std::max<int64_t>(n, 1));
  bool good = (!with_f64 || alloc((void **)&b->f64, sizeof(double2) * nn * size_t(b->mps_stride))) &&
              alloc((void **)&b->dims_dev, sizeof(int32_t) * nn * size_t(m + 1)) &&
              alloc((void **)&b->pad_dev, sizeof(int32_t) * size_t(m + 1)) &&
              alloc((void **)&b->site_off_dev, sizeof(int64_t) * size_t(m + 1)) &&
              alloc((void **)&b->split_off_dev, sizeof(int64_t) * size_t(m + 1)) &&
              alloc((void **)&b->i8_off_dev, sizeof(int64_t) * size_t(m + 1)) &&
              alloc((void **)&b->disc_dev, sizeof(double) * nn) &&
              alloc((void **)&b->maxdisc_dev, sizeof(double) * nn) &&
              alloc((void **)&b->degen_dev, sizeof(int32_t) * nn) &&
              alloc((void **)&b->unconv_dev, sizeof(int32_t) * nn);
  if (!good) {
    (void)hipGetLastError();
    batch_release(b);
    return fail(QK_ENOMEM, "device allocation failed for an MPS batch of " + std::to_string(n) +
                               " x " + std::to_string(m) + " sites");
  }
  if (hipMemcpyAsync(b->pad_dev, pad.data(), sizeof(int32_t) * (m + 1), hipMemcpyHostToDevice, stream) != hipSuccess ||
      hipMemcpyAsync(b->site_off_dev, b->site_off.data(), sizeof(int64_t) * (m + 1), hipMemcpyHostToDevice, stream) != hipSuccess ||
      hipMemcpyAsync(b->split_off_dev, b->split_off.data(), sizeof(int64_t) * (m + 1), hipMemcpyHostToDevice, stream) != hipSuccess ||
      hipMemcpyAsync(b->i8_off_dev, b->i8_off.data(), sizeof(int64_t) * (m + 1), hipMemcpyHostToDevice, stream) != hipSuccess ||
      hipStreamSynchronize(stream) != hipSuccess) {
    batch_release(b);
    return fail(QK_EDEVICE, "copy of batch layout failed");
  }
  *out = b;
  return QK_OK;
}

qk_status batch_ensure_packed(qk_mps_batch *b, qk_precision prec, hipStream_t stream) {
  if (prec == QK_FP64) {
    if (!b->f64) return fail(QK_ENOTSUP, "batch holds no FP64 form");
    return QK_OK;
  }
  if ((prec == QK_FP32 && b->f32) || (prec == QK_SPLIT_BF16 && b->sbf16) || (prec == QK_SPLIT_I8 && b->si8))
    return QK_OK;
  if (!b->f64) return fail(QK_ENOTSUP, "batch holds no FP64 form to pack from");
  if (prec == QK_FP32) {
    if (b->f32) return QK_OK;
    size_t bytes = sizeof(float2) * size_t(std::max<int64_t>(b->n, 1)) * size_t(b->mps_stride);
    b->f32 = static_cast<float2 *>(dev_alloc(b->alloc, bytes, stream, false));
    if (!b->f32) return fail(QK_ENOMEM, "device allocation of FP32 planes failed");
    return launch_pack_f32(b, stream);
  }
  if (prec == QK_SPLIT_BF16) {
    if (b->sbf16) return QK_OK;
    if (*std::max_element(b->pad.begin(), b->pad.end()) > kSplitMaxPad)
      return fail(QK_ENOTSUP, "the split-BF16 form supports bond dimensions up to 64");
    size_t bytes = size_t(std::max<int64_t>(b->n, 1)) * size_t(b->split_stride);
    b->sbf16 = static_cast<uint8_t *>(dev_alloc(b->alloc, bytes, stream, false));
    if (!b->sbf16) return fail(QK_ENOMEM, "device allocation of split-BF16 planes failed");
    return launch_pack_split(b, stream);
  }
  if (prec == QK_SPLIT_I8) {
    if (*std::max_element(b->pad.begin(), b->pad.end()) > kSplitMaxPad)
      return fail(QK_ENOTSUP, "the split-int8 form supports bond dimensions up to 64");
    size_t bytes = size_t(std::max<int64_t>(b->n, 1)) * size_t(b->i8_stride);
    b->si8 = static_cast<uint8_t *>(dev_alloc(b->alloc, bytes, stream, false));
    if (!b->si8) return fail(QK_ENOMEM, "device allocation of split-int8 planes failed");
    return launch_pack_i8(b, stream);
  }
  return fail(QK_EINVAL, "unknown precision");
}

}  // namespace qk

using namespace qk;

extern "C" {

qk_status qk_init(int device, const qk_allocator *alloc) {
  if (device < 0 || device >= kMaxDevices) return fail(QK_EINVAL, "device index out of range");
  if (alloc && (!alloc->alloc || !alloc->free)) return fail(QK_EINVAL, "allocator with a NULL function");
  {
    std::lock_guard<std::mutex> lk(g_alloc_mu);
    g_alloc[device] = DevAlloc{};
    if (alloc) g_alloc[device].user = *alloc;
  }
  int count = 0;
  QK_HIP_CHECK(hipGetDeviceCount(&count));
  if (device >= count) return fail(QK_EINVAL, "device index out of range");
  QK_HIP_CHECK(hipSetDevice(device));
  // address of this device's copy of the allocation-free Gram scratch
  void *scratch_ptr = nullptr;
  const qk_status st = noalloc_scratch(&scratch_ptr);
  if (st != QK_OK) return st;
  return ok();
}

const char *qk_last_error(void) { return g_last_error.c_str(); }

const char *qk_version(void) { return "qkmps 0.1 (gfx950)"; }

qk_status qk_circuit_compile(const qk_circuit_spec *spec, qk_gate *out_host, int64_t cap,
                             int64_t *n_gates) {
  qk_status st = validate_spec(spec);
  if (st != QK_OK) return st;
  if (!n_gates) return fail(QK_EINVAL, "n_gates is NULL");
  auto g = compile_circuit(*spec);
  *n_gates = int64_t(g.size());
  if (cap < int64_t(g.size())) {
    if (cap == 0 && out_host == nullptr) return ok();
    return fail(QK_EINVAL, "gate buffer too small");
  }
  if (!out_host && !g.empty()) return fail(QK_EINVAL, "out_host is NULL");
  if (!g.empty()) std::memcpy(out_host, g.data(), g.size() * sizeof(qk_gate));
  return ok();
}

qk_status mps_simulate(const double *features_dev, int64_t n_points, const qk_circuit_spec *spec,
                       int32_t chi_max, double cutoff, void *hip_stream, qk_mps_batch **out) {
  return mps_simulate_progress(features_dev, n_points, spec, chi_max, cutoff, hip_stream, nullptr, nullptr, 0, out);
}

static qk_status simulate_impl(const double *features_dev, int64_t n_points, const qk_circuit_spec *spec,
                               int32_t chi_max, double cutoff, void *hip_stream, qk_progress_fn fn, void *user,
                               int64_t every, int64_t graph_circuits, int32_t *trace_dev, qk_mps_batch **out);

qk_status mps_simulate_progress(const double *features_dev, int64_t n_points, const qk_circuit_spec *spec,
                                int32_t chi_max, double cutoff, void *hip_stream, qk_progress_fn fn, void *user,
                                int64_t every, qk_mps_batch **out) {
  return simulate_impl(features_dev, n_points, spec, chi_max, cutoff, hip_stream, fn, user, every, 0, nullptr, out);
}

qk_status mps_simulate_trace(const double *features_dev, int64_t n_points, const qk_circuit_spec *spec,
                             int32_t chi_max, double cutoff, int32_t *trace_dev, void *hip_stream,
                             qk_mps_batch **out) {
  if (!out) return fail(QK_EINVAL, "out is NULL");
  *out = nullptr;
  const qk_status st = validate_spec(spec);
  if (st != QK_OK) return st;
  int64_t n2q = 0;
  for (const auto &g : compile_circuit(*spec)) n2q += g.op != 0 ? 1 : 0;   // op 0: Rz
  if (n_points > 0 && n2q > 0 && !trace_dev) return fail(QK_EINVAL, "trace_dev is NULL");
  return simulate_impl(features_dev, n_points, spec, chi_max, cutoff, hip_stream, nullptr, nullptr, 0, 0,
                       trace_dev, out);
}

qk_status mps_simulate_graph(const double *features_dev, int64_t n_points, const qk_circuit_spec *spec,
                             int32_t chi_max, double cutoff, int64_t circuits_per_graph, void *hip_stream,
                             qk_mps_batch **out) {
  if (circuits_per_graph < 0) return fail(QK_EINVAL, "circuits_per_graph < 0");
  int64_t c = circuits_per_graph;
  if (c == 0 && n_points > 0) {
    // the batch in equal replays of at most QK_GRAPH_CIRCUITS circuits
    const int64_t r = (n_points + QK_GRAPH_CIRCUITS - 1) / QK_GRAPH_CIRCUITS;
    c = (n_points + r - 1) / r;
  }
  return simulate_impl(features_dev, n_points, spec, chi_max, cutoff, hip_stream, nullptr, nullptr, 0,
                       std::max<int64_t>(c, 1), nullptr, out);
}

extern "C++" {
namespace qk {
// Copy of a batch's FP64 tensors into a batch with smaller pads (sim.hip).
qk_status launch_repad_f64(const qk_mps_batch *src, qk_mps_batch *dst, hipStream_t stream);
}  // namespace qk
}

// The simulation allocates for the largest bonds its chi cap allows; once
// the states are known, the batch is re-laid with the pads of the bonds they
// reached (pad of the largest bond at each site), so Gram kernels of the
// plain forms work on blocks that size (bond-2 states: 32-wide pads instead
// of 64).  Tensors, bond dimensions and statistics are copied unchanged.
static qk_status shrink_to_bonds(qk_mps_batch **pb, hipStream_t stream) {
  qk_mps_batch *b = *pb;
  const int m = b->m;
  if (b->n == 0) return QK_OK;
  std::vector<int32_t> dims(size_t(b->n) * (m + 1));
  QK_HIP_CHECK(hipMemcpyAsync(dims.data(), b->dims_dev, sizeof(int32_t) * dims.size(), hipMemcpyDeviceToHost, stream));
  QK_HIP_CHECK(hipStreamSynchronize(stream));
  std::vector<int32_t> pad(m + 1, 1);
  for (int64_t i = 0; i < b->n; ++i)
    for (int l = 0; l <= m; ++l) pad[l] = std::max(pad[l], dims[size_t(i) * (m + 1) + l]);
  for (int l = 0; l <= m; ++l) pad[l] = std::min(pad_of(pad[l]), b->pad[l]);
  if (pad == b->pad) return QK_OK;
  qk_mps_batch *c = nullptr;
  qk_status st = batch_create(b->n, m, pad, stream, &c);
  if (st != QK_OK) return st;
  st = launch_repad_f64(b, c, stream);
  const size_t n = size_t(b->n);
  if (st == QK_OK &&
      (hipMemcpyAsync(c->dims_dev, b->dims_dev, sizeof(int32_t) * n * (m + 1), hipMemcpyDeviceToDevice, stream) !=
           hipSuccess ||
       hipMemcpyAsync(c->disc_dev, b->disc_dev, sizeof(double) * n, hipMemcpyDeviceToDevice, stream) != hipSuccess ||
       hipMemcpyAsync(c->maxdisc_dev, b->maxdisc_dev, sizeof(double) * n, hipMemcpyDeviceToDevice, stream) !=
           hipSuccess ||
       hipMemcpyAsync(c->degen_dev, b->degen_dev, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, stream) !=
           hipSuccess ||
       hipMemcpyAsync(c->unconv_dev, b->unconv_dev, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, stream) !=
           hipSuccess ||
       hipStreamSynchronize(stream) != hipSuccess))
    st = fail(QK_EDEVICE, "copy into the re-laid batch failed");
  if (st != QK_OK) {
    batch_release(c);
    return st;
  }
  c->n_two_qubit_gates = b->n_two_qubit_gates;
  batch_release(b);
  *pb = c;
  return QK_OK;
}

static qk_status simulate_impl(const double *features_dev, int64_t n_points, const qk_circuit_spec *spec,
                               int32_t chi_max, double cutoff, void *hip_stream, qk_progress_fn fn, void *user,
                               int64_t every, int64_t graph_circuits, int32_t *trace_dev, qk_mps_batch **out) {
  if (!out) return fail(QK_EINVAL, "out is NULL");
  *out = nullptr;
  qk_status st = validate_spec(spec);
  if (st != QK_OK) return st;
  if (n_points < 0) return fail(QK_EINVAL, "n_points < 0");
  if (n_points > 0 && !features_dev) return fail(QK_EINVAL, "features_dev is NULL");
  if (chi_max < 1) return fail(QK_EINVAL, "chi_max must be >= 1");
  if (chi_max > kMaxSimChi) return fail(QK_ENOTSUP, "chi_max above 128 is not supported in simulation");
  if (!std::isfinite(cutoff)) return fail(QK_EINVAL, "cutoff must be finite");
  hipStream_t stream = reinterpret_cast<hipStream_t>(hip_stream);
  const int m = spec->n_qubits;
  // Worst-case bond profile: D_l <= min(chi, 2^min(l, m-l)).
  std::vector<int32_t> pad(m + 1);
  for (int l = 0; l <= m; ++l) {
    int e = std::min(l, m - l);
    int64_t cap = e >= 30 ? (int64_t(1) << 30) : (int64_t(1) << e);
    pad[l] = pad_of(int(std::min<int64_t>(chi_max, cap)));
  }
  qk_mps_batch *b = nullptr;
  st = batch_create(n_points, m, pad, stream, &b);
  if (st != QK_OK) return st;
  auto gates = compile_circuit(*spec);
  st = run_simulation(b, features_dev, gates, *spec, chi_max, cutoff, stream, fn, user, every, graph_circuits,
                      trace_dev);
  if (st == QK_OK) st = shrink_to_bonds(&b, stream);
  if (st != QK_OK) {
    batch_release(b);
    return st;
  }
  *out = b;
  return ok();
}

static qk_status check_pair_batches(const qk_mps_batch *a, const qk_mps_batch *b) {
  if (!a || !b) return fail(QK_EINVAL, "batch is NULL");
  if (a->m != b->m) return fail(QK_EINVAL, "batches have different qubit counts");
  int dev = 0;
  QK_HIP_CHECK(hipGetDevice(&dev));
  if (a->device != dev || b->device != dev)
    return fail(QK_EINVAL, "batch lives on another device than the current one");
  return QK_OK;
}

static qk_status make_job(const qk_mps_batch *a, int64_t a0, int64_t na, const qk_mps_batch *b,
                          int64_t b0, int64_t nb, int32_t upper, double *K, int64_t ldk,
                          qk_precision prec, hipStream_t stream, GramJobDev *job, bool pack = true) {
  qk_status st = check_pair_batches(a, b);
  if (st != QK_OK) return st;
  if (na < 0 || nb < 0 || a0 < 0 || b0 < 0 || a0 + na > a->n || b0 + nb > b->n)
    return fail(QK_EINVAL, "row/column range outside the batch");
  if (na > 0 && nb > 0 && !K) return fail(QK_EINVAL, "K_dev is NULL");
  if (ldk < nb) return fail(QK_EINVAL, "ldk < number of columns");
  if (upper && a != b) return fail(QK_EINVAL, "upper_only requires a == b");
  if (prec != QK_FP64 && prec != QK_FP32 && prec != QK_SPLIT_BF16 && prec != QK_SPLIT_I8)
    return fail(QK_EINVAL, "unknown precision");
  auto *am = const_cast<qk_mps_batch *>(a);
  auto *bm = const_cast<qk_mps_batch *>(b);
  if (pack) {
    st = batch_ensure_packed(am, prec, stream);
    if (st != QK_OK) return st;
    st = batch_ensure_packed(bm, prec, stream);
    if (st != QK_OK) return st;
  } else {
    auto present = [&](const qk_mps_batch *x) {
      return prec == QK_FP64 ? x->f64 != nullptr : prec == QK_FP32 ? x->f32 != nullptr
                                                 : prec == QK_SPLIT_BF16 ? x->sbf16 != nullptr : x->si8 != nullptr;
    };
    if (!present(a) || !present(b))
      return fail(QK_ENOTSUP, "the precision's packed form is not built: call mps_batch_pack first");
  }
  auto base = [&](qk_mps_batch *x) -> const void * {
    switch (prec) {
      case QK_FP64: return x->f64;
      case QK_FP32: return x->f32;
      case QK_SPLIT_BF16: return x->sbf16;
      default: return x->si8;
    }
  };
  auto offsets = [&](qk_mps_batch *x) -> const int64_t * {
    return prec == QK_SPLIT_BF16 ? x->split_off_dev : prec == QK_SPLIT_I8 ? x->i8_off_dev : x->site_off_dev;
  };
  auto stride = [&](qk_mps_batch *x) -> int64_t {
    return prec == QK_SPLIT_BF16 ? x->split_stride : prec == QK_SPLIT_I8 ? x->i8_stride : x->mps_stride;
  };
  job->a_base = base(am);
  job->b_base = base(bm);
  job->a_off = offsets(am);
  job->b_off = offsets(bm);
  job->a_pad = am->pad_dev;
  job->b_pad = bm->pad_dev;
  job->a_stride = stride(am);
  job->b_stride = stride(bm);
  job->a0 = a0;
  job->na = na;
  job->b0 = b0;
  job->nb = nb;
  job->K = K;
  job->ldk = ldk;
  job->m = a->m;
  job->upper = upper ? 1 : 0;
  job->tiles_i = 0;
  job->tiles_j = 0;
  job->pair_begin = 0;
  return QK_OK;
}

static int max_pad_of(const qk_mps_batch *x) {
  return *std::max_element(x->pad.begin(), x->pad.end());
}

// Entries and algorithmic flops of one Gram job.  An overlap costs, per site
// l (Fig. 2), 2 Da_l Db_{l+1} (Db_l + Da_{l+1}) complex MACs of 8 flops for
// bra bonds Da and ket bonds Db.  Summed over a block of pairs the terms
// separate into per-row and per-column sums (prefix sums over the rows for
// the upper triangle), so the count is exact and costs O(m (na + nb)).
static qk_status job_work(const qk_mps_batch *a, int64_t a0, int64_t na, const qk_mps_batch *b, int64_t b0,
                          int64_t nb, bool upper, double *entries, double *flops) {
  const int m = a->m, m1 = m + 1;
  std::vector<int32_t> da(size_t(na) * m1), db(size_t(nb) * m1);
  QK_HIP_CHECK(hipDeviceSynchronize());
  if (na > 0)
    QK_HIP_CHECK(hipMemcpy(da.data(), a->dims_dev + a0 * m1, sizeof(int32_t) * da.size(), hipMemcpyDeviceToHost));
  if (nb > 0)
    QK_HIP_CHECK(hipMemcpy(db.data(), b->dims_dev + b0 * m1, sizeof(int32_t) * db.size(), hipMemcpyDeviceToHost));
  double e = 0.0, f = 0.0;
  if (!upper) {
    e = double(na) * double(nb);
    for (int l = 0; l < m; ++l) {
      double sa = 0, qa = 0, pb = 0, sb = 0;
      for (int64_t i = 0; i < na; ++i) {
        sa += da[i * m1 + l];
        qa += double(da[i * m1 + l]) * da[i * m1 + l + 1];
      }
      for (int64_t j = 0; j < nb; ++j) {
        pb += double(db[j * m1 + l]) * db[j * m1 + l + 1];
        sb += db[j * m1 + l + 1];
      }
      f += 2.0 * (sa * pb + qa * sb);
    }
  } else {
    // pairs (i, j) with global column b0 + j >= global row a0 + i
    std::vector<double> ps(size_t(na) + 1), pq(size_t(na) + 1);
    for (int64_t j = 0; j < nb; ++j) {
      const int64_t rows = std::min<int64_t>(na, std::max<int64_t>(0, b0 + j - a0 + 1));
      e += double(rows);
    }
    for (int l = 0; l < m; ++l) {
      ps[0] = pq[0] = 0.0;
      for (int64_t i = 0; i < na; ++i) {
        ps[i + 1] = ps[i] + da[i * m1 + l];
        pq[i + 1] = pq[i] + double(da[i * m1 + l]) * da[i * m1 + l + 1];
      }
      for (int64_t j = 0; j < nb; ++j) {
        const int64_t rows = std::min<int64_t>(na, std::max<int64_t>(0, b0 + j - a0 + 1));
        f += 2.0 * (ps[rows] * double(db[j * m1 + l]) * db[j * m1 + l + 1] + pq[rows] * db[j * m1 + l + 1]);
      }
    }
  }
  *entries += e;
  *flops += 8.0 * f;
  return QK_OK;
}

qk_status mps_gram_block(const qk_mps_batch *a, int64_t a0, int64_t na, const qk_mps_batch *b,
                         int64_t b0, int64_t nb, int32_t upper_only, qk_precision prec,
                         double *K_dev, int64_t ldk, void *hip_stream, qk_gram_stats *stats) {
  hipStream_t stream = reinterpret_cast<hipStream_t>(hip_stream);
  if (stats) std::memset(stats, 0, sizeof(*stats));
  GramJobDev job;
  qk_status st = make_job(a, a0, na, b, b0, nb, upper_only, K_dev, ldk, prec, stream, &job);
  if (st != QK_OK) return st;
  if (na == 0 || nb == 0) return ok();
  std::vector<GramJobDev> jobs{job};
  st = launch_gram(jobs, std::max(max_pad_of(a), max_pad_of(b)), prec, stream, stats);
  if (st != QK_OK) return st;
  if (stats) {
    double e = 0.0, f = 0.0;
    st = job_work(a, a0, na, b, b0, nb, upper_only != 0, &e, &f);
    if (st != QK_OK) return st;
    stats->entries = int64_t(e);
    stats->flops = f;
  }
  return ok();
}

qk_status mps_gram_block_noalloc(const qk_mps_batch *a, int64_t a0, int64_t na, const qk_mps_batch *b,
                                 int64_t b0, int64_t nb, int32_t upper_only, qk_precision prec, double *K_dev,
                                 int64_t ldk, void *hip_stream) {
  hipStream_t stream = reinterpret_cast<hipStream_t>(hip_stream);
  GramJobDev job;
  // pack = false: the precision's planes must exist already (no allocation)
  qk_status st = make_job(a, a0, na, b, b0, nb, upper_only, K_dev, ldk, prec, stream, &job, false);
  if (st != QK_OK) return st;
  if (na == 0 || nb == 0) return ok();
  void *ws = nullptr;
  st = noalloc_scratch(&ws);
  if (st != QK_OK) return st;
  const int max_pad = std::max(max_pad_of(a), max_pad_of(b));
  std::vector<GramJobDev> jobs{job};
  st = launch_gram_cfg(jobs, max_pad, prec, current_gram_config(prec, max_pad), stream, nullptr, ws,
                       kNoAllocScratchBytes);
  if (st != QK_OK) return st;
  return ok();
}

qk_status mps_gram(const qk_mps_batch *a, const qk_mps_batch *b, qk_precision prec, double *K_dev,
                   int64_t ldk, void *hip_stream, qk_gram_stats *stats) {
  if (!a) return fail(QK_EINVAL, "batch a is NULL");
  if (b == nullptr || b == a)
    return mps_gram_block(a, 0, a->n, a, 0, a->n, 1, prec, K_dev, ldk, hip_stream, stats);
  return mps_gram_block(a, 0, a->n, b, 0, b->n, 0, prec, K_dev, ldk, hip_stream, stats);
}

constexpr double kTuneMargin = 0.02;

qk_status mps_gram_autotune(qk_mps_batch *b, qk_precision prec, int64_t sample, void *hip_stream,
                            qk_tune_report *report) {
  if (!b) return fail(QK_EINVAL, "NULL batch");
  if (sample < 1) return fail(QK_EINVAL, "sample must be >= 1");
  hipStream_t stream = reinterpret_cast<hipStream_t>(hip_stream);
  const int64_t n = std::min<int64_t>(sample, b->n);
  if (n < 1) return fail(QK_EINVAL, "empty batch");
  const DevAlloc al = allocator_for_current_device();
  auto *K = static_cast<double *>(dev_alloc(al, sizeof(double) * size_t(n) * size_t(n), stream, true));
  if (!K) return fail(QK_ENOMEM, "device allocation of the autotuning Gram failed");
  GramJobDev job;
  qk_status st = make_job(b, 0, n, b, 0, n, 1, K, n, prec, stream, &job);
  const int max_pad = max_pad_of(b);
  std::vector<GramJobDev> jobs{job};
  auto run_ms = [&](const GramConfig &c, double &ms) -> qk_status {
    double best = 1e300;
    for (int rep = 0; rep < 3; ++rep) {
      const auto t0 = std::chrono::steady_clock::now();
      qk_status s2 = launch_gram_cfg(jobs, max_pad, prec, c, stream);
      if (s2 != QK_OK) return s2;
      QK_HIP_CHECK(hipStreamSynchronize(stream));
      const double dt = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
      if (rep > 0) best = std::min(best, dt);   // rep 0 warms up
    }
    ms = best;
    return QK_OK;
  };
  GramConfig best_cfg = default_gram_config(prec, max_pad);
  double default_ms = 0.0, best_ms = 1e300;
  const auto cands = gram_config_candidates(prec, max_pad);
  if (st == QK_OK) st = run_ms(best_cfg, default_ms);
  best_ms = default_ms;
  GramConfig fastest = best_cfg;
  double fastest_ms = default_ms;
  for (size_t k = 0; k < cands.size() && st == QK_OK; ++k) {
    double ms = 0.0;
    st = run_ms(cands[k], ms);
    if (st == QK_OK && ms < fastest_ms) {
      fastest_ms = ms;
      fastest = cands[k];
    }
  }
  // the default stays unless a candidate beats it by more than the
  // run-to-run spread of the timing (about 1 %), so that the choice is
  // stable between runs
  if (fastest_ms < (1.0 - kTuneMargin) * default_ms) {
    best_cfg = fastest;
    best_ms = fastest_ms;
  }
  dev_free(al, K, stream, true);
  if (st != QK_OK) return st;
  store_gram_config(prec, max_pad, best_cfg);
  if (report) {
    report->maxp = best_cfg.maxp;
    report->tile_side = best_cfg.tile_side;
    report->queues = best_cfg.queues;
    report->n_candidates = int32_t(cands.size());
    report->best_ms = best_ms;
    report->default_ms = default_ms;
  }
  return ok();
}

qk_status mps_gram_tune_reset(void) {
  clear_gram_configs();
  return ok();
}

qk_status mps_gram_multi(const qk_gram_job *jobs, int32_t n_jobs, qk_precision prec, void *hip_stream,
                         qk_gram_stats *stats) {
  if (stats) std::memset(stats, 0, sizeof(*stats));
  if (n_jobs < 0 || (n_jobs > 0 && !jobs)) return fail(QK_EINVAL, "invalid job list");
  hipStream_t stream = reinterpret_cast<hipStream_t>(hip_stream);
  std::vector<GramJobDev> dj;
  int max_pad = 32;
  for (int k = 0; k < n_jobs; ++k) {
    const qk_gram_job &j = jobs[k];
    if (j.reserved != 0) return fail(QK_EINVAL, "reserved job field must be zero");
    GramJobDev job;
    qk_status st = make_job(j.a, j.a0, j.na, j.b, j.b0, j.nb, j.upper_only, j.K_dev, j.ldk, prec,
                            stream, &job);
    if (st != QK_OK) return st;
    if (j.na == 0 || j.nb == 0) continue;
    max_pad = std::max({max_pad, max_pad_of(j.a), max_pad_of(j.b)});
    dj.push_back(job);
  }
  if (dj.empty()) return ok();
  qk_status st = launch_gram(dj, max_pad, prec, stream, stats);
  if (st != QK_OK) return st;
  if (stats) {
    double e = 0.0, f = 0.0;
    for (int k = 0; k < n_jobs && st == QK_OK; ++k) {
      const qk_gram_job &j = jobs[k];
      if (j.na > 0 && j.nb > 0) st = job_work(j.a, j.a0, j.na, j.b, j.b0, j.nb, j.upper_only != 0, &e, &f);
    }
    if (st != QK_OK) return st;
    stats->entries = int64_t(e);
    stats->flops = f;
  }
  return ok();
}

qk_status mps_batch_import(const double *tensors_host, const int32_t *dims_host, int64_t n, int32_t m,
                           void *hip_stream, qk_mps_batch **out) {
  if (!out) return fail(QK_EINVAL, "out is NULL");
  *out = nullptr;
  if (n < 0 || m < 1) return fail(QK_EINVAL, "need n >= 0 and m >= 1");
  if (n > 0 && (!tensors_host || !dims_host)) return fail(QK_EINVAL, "NULL host buffer");
  hipStream_t stream = reinterpret_cast<hipStream_t>(hip_stream);
  std::vector<int32_t> maxd(m + 1, 1);
  int64_t total = 0;
  for (int64_t i = 0; i < n; ++i) {
    const int32_t *d = dims_host + i * (m + 1);
    if (d[0] != 1 || d[m] != 1) return fail(QK_EINVAL, "first and last bond dimensions must be 1");
    for (int l = 0; l <= m; ++l) {
      if (d[l] < 1 || d[l] > kMaxBond) return fail(QK_EINVAL, "bond dimension outside [1, 128]");
      maxd[l] = std::max(maxd[l], d[l]);
    }
    for (int l = 0; l < m; ++l) total += int64_t(2) * d[l] * d[l + 1];
  }
  for (int64_t k = 0; k < 2 * total; ++k)
    if (!std::isfinite(tensors_host[k])) return fail(QK_EINVAL, "non-finite tensor entry");
  std::vector<int32_t> pad(m + 1);
  for (int l = 0; l <= m; ++l) pad[l] = pad_of(maxd[l]);
  qk_mps_batch *b = nullptr;
  qk_status st = batch_create(n, m, pad, stream, &b);
  if (st != QK_OK) return st;
  std::vector<double2> host(size_t(std::max<int64_t>(n, 1)) * size_t(b->mps_stride), double2{0.0, 0.0});
  const double *src = tensors_host;
  for (int64_t i = 0; i < n; ++i) {
    const int32_t *d = dims_host + i * (m + 1);
    for (int l = 0; l < m; ++l) {
      double2 *dst = host.data() + i * b->mps_stride + b->site_off[l];
      for (int s = 0; s < 2; ++s)
        for (int a = 0; a < d[l]; ++a)
          for (int c = 0; c < d[l + 1]; ++c) {
            dst[(size_t(s) * pad[l] + a) * pad[l + 1] + c] = double2{src[0], src[1]};
            src += 2;
          }
    }
  }
  if (n > 0) {
    if (hipMemcpyAsync(b->f64, host.data(), sizeof(double2) * host.size(), hipMemcpyHostToDevice, stream) != hipSuccess ||
        hipMemcpyAsync(b->dims_dev, dims_host, sizeof(int32_t) * n * (m + 1), hipMemcpyHostToDevice, stream) != hipSuccess ||
        hipStreamSynchronize(stream) != hipSuccess) {
      batch_release(b);
      return fail(QK_EDEVICE, "copy of imported tensors failed");
    }
  }
  *out = b;
  return ok();
}

qk_status mps_batch_info(const qk_mps_batch *b, qk_batch_info *info) {
  if (!b || !info) return fail(QK_EINVAL, "NULL argument");
  std::memset(info, 0, sizeof(*info));
  info->n = b->n;
  info->m = b->m;
  info->pad_max = max_pad_of(b);
  info->n_two_qubit_gates = b->n_two_qubit_gates;
  const size_t n = size_t(b->n);
  if (n > 0) {
    std::vector<int32_t> dims(n * (b->m + 1));
    std::vector<double> disc(n), maxd(n);
    std::vector<int32_t> deg(n), unc(n);
    QK_HIP_CHECK(hipDeviceSynchronize());
    QK_HIP_CHECK(hipMemcpy(dims.data(), b->dims_dev, sizeof(int32_t) * dims.size(), hipMemcpyDeviceToHost));
    QK_HIP_CHECK(hipMemcpy(disc.data(), b->disc_dev, sizeof(double) * n, hipMemcpyDeviceToHost));
    QK_HIP_CHECK(hipMemcpy(maxd.data(), b->maxdisc_dev, sizeof(double) * n, hipMemcpyDeviceToHost));
    QK_HIP_CHECK(hipMemcpy(deg.data(), b->degen_dev, sizeof(int32_t) * n, hipMemcpyDeviceToHost));
    QK_HIP_CHECK(hipMemcpy(unc.data(), b->unconv_dev, sizeof(int32_t) * n, hipMemcpyDeviceToHost));
    info->max_bond = *std::max_element(dims.begin(), dims.end());
    double sum = 0.0;
    for (size_t i = 0; i < n; ++i) {
      sum += disc[i];
      info->max_discarded = std::max(info->max_discarded, maxd[i]);
      info->degenerate_cuts += deg[i];
      info->unconverged_svds += unc[i];
    }
    info->mean_total_discarded = sum / double(n);
  }
  info->bytes_f64 = b->f64 ? int64_t(sizeof(double2)) * b->n * b->mps_stride : 0;
  info->bytes_f32 = b->f32 ? int64_t(sizeof(float2)) * b->n * b->mps_stride : 0;
  info->bytes_split_bf16 = b->sbf16 ? b->n * b->split_stride : 0;
  info->bytes_split_i8 = b->si8 ? b->n * b->i8_stride : 0;
  return ok();
}

qk_status mps_batch_bond_dims(const qk_mps_batch *b, int32_t *dims_host) {
  if (!b || !dims_host) return fail(QK_EINVAL, "NULL argument");
  if (b->n == 0) return ok();
  QK_HIP_CHECK(hipDeviceSynchronize());
  QK_HIP_CHECK(hipMemcpy(dims_host, b->dims_dev, sizeof(int32_t) * b->n * (b->m + 1), hipMemcpyDeviceToHost));
  return ok();
}

qk_status mps_batch_trunc_stats(const qk_mps_batch *b, double *discarded_host, int32_t *degenerate_host) {
  if (!b) return fail(QK_EINVAL, "NULL batch");
  if (b->n == 0) return ok();
  QK_HIP_CHECK(hipDeviceSynchronize());
  if (discarded_host)
    QK_HIP_CHECK(hipMemcpy(discarded_host, b->disc_dev, sizeof(double) * b->n, hipMemcpyDeviceToHost));
  if (degenerate_host)
    QK_HIP_CHECK(hipMemcpy(degenerate_host, b->degen_dev, sizeof(int32_t) * b->n, hipMemcpyDeviceToHost));
  return ok();
}

qk_status mps_batch_export(const qk_mps_batch *b, int64_t idx, double *host_buf, int64_t cap,
                           int64_t *written) {
  if (!b || !written) return fail(QK_EINVAL, "NULL argument");
  if (idx < 0 || idx >= b->n) return fail(QK_EINVAL, "index out of range");
  if (!b->f64) return fail(QK_ENOTSUP, "batch holds no FP64 form");
  const int m = b->m;
  std::vector<int32_t> d(m + 1);
  QK_HIP_CHECK(hipDeviceSynchronize());
  QK_HIP_CHECK(hipMemcpy(d.data(), b->dims_dev + idx * (m + 1), sizeof(int32_t) * (m + 1), hipMemcpyDeviceToHost));
  int64_t need = 0;
  for (int l = 0; l < m; ++l) need += int64_t(4) * d[l] * d[l + 1];
  *written = need;
  if (cap < need || !host_buf) return fail(QK_EINVAL, "export buffer too small");
  std::vector<double2> mps(size_t(b->mps_stride));
  QK_HIP_CHECK(hipMemcpy(mps.data(), b->f64 + idx * b->mps_stride, sizeof(double2) * mps.size(), hipMemcpyDeviceToHost));
  double *dst = host_buf;
  for (int l = 0; l < m; ++l) {
    const double2 *src = mps.data() + b->site_off[l];
    for (int s = 0; s < 2; ++s)
      for (int a = 0; a < d[l]; ++a)
        for (int c = 0; c < d[l + 1]; ++c) {
          double2 v = src[(size_t(s) * b->pad[l] + a) * b->pad[l + 1] + c];
          *dst++ = v.x;
          *dst++ = v.y;
        }
  }
  return ok();
}

qk_status mps_batch_pack(qk_mps_batch *b, qk_precision prec, void *hip_stream) {
  if (!b) return fail(QK_EINVAL, "NULL batch");
  qk_status st = batch_ensure_packed(b, prec, reinterpret_cast<hipStream_t>(hip_stream));
  if (st != QK_OK) return st;
  return ok();
}

qk_status mps_batch_drop(qk_mps_batch *b, qk_precision prec) {
  if (!b) return fail(QK_EINVAL, "NULL batch");
  QK_HIP_CHECK(hipDeviceSynchronize());
  if (prec == QK_FP32 && b->f32) {
    dev_free(b->alloc, b->f32, nullptr, false);
    b->f32 = nullptr;
  } else if (prec == QK_SPLIT_BF16 && b->sbf16) {
    dev_free(b->alloc, b->sbf16, nullptr, false);
    b->sbf16 = nullptr;
  } else if (prec == QK_SPLIT_I8 && b->si8) {
    dev_free(b->alloc, b->si8, nullptr, false);
    b->si8 = nullptr;
  } else if (prec == QK_FP64) {
    return fail(QK_EINVAL, "the FP64 form cannot be dropped");
  }
  return ok();
}

qk_status mps_batch_gather(const qk_mps_batch *src, const int64_t *idx_host, int64_t count, uint32_t forms,
                           void *hip_stream, qk_mps_batch **out) {
  if (!src || !out) return fail(QK_EINVAL, "NULL argument");
  *out = nullptr;
  if (count < 0 || (count > 0 && !idx_host)) return fail(QK_EINVAL, "invalid index list");
  if (forms == 0 || (forms & ~15u)) return fail(QK_EINVAL, "invalid forms mask");
  if (((forms & QK_FORM_FP64) && !src->f64) || ((forms & QK_FORM_FP32) && !src->f32) ||
      ((forms & QK_FORM_SPLIT_BF16) && !src->sbf16) || ((forms & QK_FORM_SPLIT_I8) && !src->si8))
    return fail(QK_EINVAL, "requested form is not present in the source batch");
  for (int64_t k = 0; k < count; ++k)
    if (idx_host[k] < 0 || idx_host[k] >= src->n) return fail(QK_EINVAL, "gather index out of range");
  hipStream_t stream = reinterpret_cast<hipStream_t>(hip_stream);
  qk_mps_batch *b = nullptr;
  qk_status st = batch_create(count, src->m, src->pad, stream, &b, (forms & QK_FORM_FP64) != 0);
  if (st != QK_OK) return st;
  b->n_two_qubit_gates = src->n_two_qubit_gates;
  const size_t nn = size_t(std::max<int64_t>(count, 1));
  if (forms & QK_FORM_FP32) {
    b->f32 = static_cast<float2 *>(dev_alloc(b->alloc, sizeof(float2) * nn * size_t(b->mps_stride), stream, false));
    if (!b->f32) {
      batch_release(b);
      return fail(QK_ENOMEM, "device allocation of FP32 planes failed");
    }
  }
  if (forms & QK_FORM_SPLIT_BF16) {
    b->sbf16 = static_cast<uint8_t *>(dev_alloc(b->alloc, nn * size_t(b->split_stride), stream, false));
    if (!b->sbf16) {
      batch_release(b);
      return fail(QK_ENOMEM, "device allocation of split-BF16 planes failed");
    }
  }
  if (forms & QK_FORM_SPLIT_I8) {
    b->si8 = static_cast<uint8_t *>(dev_alloc(b->alloc, nn * size_t(b->i8_stride), stream, false));
    if (!b->si8) {
      batch_release(b);
      return fail(QK_ENOMEM, "device allocation of split-int8 planes failed");
    }
  }
  const int m1 = src->m + 1;
  if (count > 0) {
    auto *idx_dev = static_cast<int64_t *>(dev_alloc(b->alloc, sizeof(int64_t) * size_t(count), stream, true));
    if (!idx_dev) {
      batch_release(b);
      return fail(QK_ENOMEM, "device allocation of the gather index failed");
    }
    const qk_mps_batch_meta ms{src->dims_dev, src->disc_dev, src->maxdisc_dev, src->degen_dev, src->unconv_dev};
    const qk_mps_batch_meta md{b->dims_dev, b->disc_dev, b->maxdisc_dev, b->degen_dev, b->unconv_dev};
    qk_status gs = QK_OK;
    if (hipMemcpyAsync(idx_dev, idx_host, sizeof(int64_t) * size_t(count), hipMemcpyHostToDevice, stream) !=
        hipSuccess)
      gs = fail(QK_EDEVICE, "copy of the gather index failed");
    if (gs == QK_OK && (forms & QK_FORM_FP64))
      gs = launch_gather_records(src->f64, b->f64, idx_dev, int64_t(sizeof(double2)) * src->mps_stride, count,
                                 stream);
    if (gs == QK_OK && (forms & QK_FORM_FP32))
      gs = launch_gather_records(src->f32, b->f32, idx_dev, int64_t(sizeof(float2)) * src->mps_stride, count,
                                 stream);
    if (gs == QK_OK && (forms & QK_FORM_SPLIT_BF16))
      gs = launch_gather_records(src->sbf16, b->sbf16, idx_dev, src->split_stride, count, stream);
    if (gs == QK_OK && (forms & QK_FORM_SPLIT_I8))
      gs = launch_gather_records(src->si8, b->si8, idx_dev, src->i8_stride, count, stream);
    if (gs == QK_OK) gs = launch_gather_meta(ms, md, idx_dev, m1, count, stream);
    // the host index list must stay valid until the copy has run
    const bool synced = hipStreamSynchronize(stream) == hipSuccess;
    dev_free(b->alloc, idx_dev, stream, true);
    if (gs != QK_OK || !synced) {
      batch_release(b);
      return gs != QK_OK ? gs : fail(QK_EDEVICE, "gather failed");
    }
  }
  *out = b;
  return ok();
}

static const char kBatchMagic[8] = {'Q', 'K', 'M', 'P', 'S', 'B', '0', '1'};

qk_status mps_batch_save(const qk_mps_batch *b, const char *path) {
  if (!b || !path) return fail(QK_EINVAL, "NULL argument");
  if (!b->f64) return fail(QK_ENOTSUP, "batch holds no FP64 form");
  const int m = b->m, m1 = m + 1;
  const size_t n = size_t(b->n);
  std::vector<int32_t> dims(n * m1), degen(n), unconv(n);
  std::vector<double> disc(n), maxdisc(n);
  QK_HIP_CHECK(hipDeviceSynchronize());
  if (n > 0) {
    QK_HIP_CHECK(hipMemcpy(dims.data(), b->dims_dev, sizeof(int32_t) * dims.size(), hipMemcpyDeviceToHost));
    QK_HIP_CHECK(hipMemcpy(disc.data(), b->disc_dev, sizeof(double) * n, hipMemcpyDeviceToHost));
    QK_HIP_CHECK(hipMemcpy(maxdisc.data(), b->maxdisc_dev, sizeof(double) * n, hipMemcpyDeviceToHost));
    QK_HIP_CHECK(hipMemcpy(degen.data(), b->degen_dev, sizeof(int32_t) * n, hipMemcpyDeviceToHost));
    QK_HIP_CHECK(hipMemcpy(unconv.data(), b->unconv_dev, sizeof(int32_t) * n, hipMemcpyDeviceToHost));
  }
  std::ofstream f(path, std::ios::binary | std::ios::trunc);
  if (!f) return fail(QK_EINVAL, std::string("cannot open ") + path + " for writing");
  const int32_t hdr32[2] = {m, b->n_two_qubit_gates};
  const int64_t n64 = b->n;
  f.write(kBatchMagic, 8);
  f.write(reinterpret_cast<const char *>(hdr32), sizeof(hdr32));
  f.write(reinterpret_cast<const char *>(&n64), sizeof(n64));
  f.write(reinterpret_cast<const char *>(b->pad.data()), sizeof(int32_t) * m1);
  f.write(reinterpret_cast<const char *>(dims.data()), sizeof(int32_t) * dims.size());
  f.write(reinterpret_cast<const char *>(disc.data()), sizeof(double) * n);
  f.write(reinterpret_cast<const char *>(maxdisc.data()), sizeof(double) * n);
  f.write(reinterpret_cast<const char *>(degen.data()), sizeof(int32_t) * n);
  f.write(reinterpret_cast<const char *>(unconv.data()), sizeof(int32_t) * n);
  // tensors in chunks of whole MPS (about 256 MiB of host memory at a time)
  const size_t per = sizeof(double2) * size_t(b->mps_stride);
  const size_t chunk = std::max<size_t>(1, (size_t(256) << 20) / std::max<size_t>(per, 1));
  std::vector<double2> host;
  for (size_t i0 = 0; i0 < n && f; i0 += chunk) {
    const size_t cnt = std::min(chunk, n - i0);
    host.resize(cnt * size_t(b->mps_stride));
    QK_HIP_CHECK(hipMemcpy(host.data(), b->f64 + i0 * b->mps_stride, per * cnt, hipMemcpyDeviceToHost));
    f.write(reinterpret_cast<const char *>(host.data()), std::streamsize(per * cnt));
  }
  f.flush();
  if (!f) return fail(QK_EINVAL, std::string("write to ") + path + " failed");
  return ok();
}

qk_status mps_batch_load(const char *path, void *hip_stream, qk_mps_batch **out) {
  if (!path || !out) return fail(QK_EINVAL, "NULL argument");
  *out = nullptr;
  hipStream_t stream = reinterpret_cast<hipStream_t>(hip_stream);
  std::ifstream f(path, std::ios::binary);
  if (!f) return fail(QK_EINVAL, std::string("cannot open ") + path);
  f.seekg(0, std::ios::end);
  const int64_t fsize = int64_t(f.tellg());
  f.seekg(0, std::ios::beg);
  char magic[8];
  int32_t hdr32[2];
  int64_t n = -1;
  f.read(magic, 8);
  f.read(reinterpret_cast<char *>(hdr32), sizeof(hdr32));
  f.read(reinterpret_cast<char *>(&n), sizeof(n));
  if (!f || std::memcmp(magic, kBatchMagic, 8) != 0) return fail(QK_EINVAL, "not an MPS batch file");
  const int32_t m = hdr32[0];
  if (m < 1 || m > 100000 || n < 0 || hdr32[1] < 0) return fail(QK_EINVAL, "malformed batch header");
  const int m1 = m + 1;
  std::vector<int32_t> pad(m1);
  f.read(reinterpret_cast<char *>(pad.data()), sizeof(int32_t) * m1);
  if (!f) return fail(QK_EINVAL, "truncated batch file");
  for (int l = 0; l <= m; ++l)
    if (pad[l] < kPadQuantum || pad[l] > kMaxBond || pad[l] % kPadQuantum)
      return fail(QK_EINVAL, "pad outside [32, 128] or not a multiple of 32");
  int64_t stride = 0;
  for (int l = 0; l < m; ++l) stride += int64_t(2) * pad[l] * pad[l + 1];
  const int64_t meta = int64_t(8 + 8 + 8) + 4 * int64_t(m1) + n * (4 * int64_t(m1) + 8 + 8 + 4 + 4);
  if (n > (int64_t(1) << 40) / std::max<int64_t>(stride, 1) || fsize != meta + n * stride * 16)
    return fail(QK_EINVAL, "batch file size does not match its header");
  const size_t nn = size_t(n);
  std::vector<int32_t> dims(nn * m1), degen(nn), unconv(nn);
  std::vector<double> disc(nn), maxdisc(nn);
  f.read(reinterpret_cast<char *>(dims.data()), sizeof(int32_t) * dims.size());
  f.read(reinterpret_cast<char *>(disc.data()), sizeof(double) * nn);
  f.read(reinterpret_cast<char *>(maxdisc.data()), sizeof(double) * nn);
  f.read(reinterpret_cast<char *>(degen.data()), sizeof(int32_t) * nn);
  f.read(reinterpret_cast<char *>(unconv.data()), sizeof(int32_t) * nn);
  if (!f) return fail(QK_EINVAL, "truncated batch file");
  for (size_t i = 0; i < nn; ++i) {
    const int32_t *d = dims.data() + i * m1;
    if (d[0] != 1 || d[m] != 1) return fail(QK_EINVAL, "first and last bond dimensions must be 1");
    for (int l = 0; l <= m; ++l)
      if (d[l] < 1 || d[l] > pad[l]) return fail(QK_EINVAL, "bond dimension outside [1, pad]");
  }
  qk_mps_batch *b = nullptr;
  qk_status st = batch_create(n, m, pad, stream, &b);
  if (st != QK_OK) return st;
  b->n_two_qubit_gates = hdr32[1];
  const size_t per = sizeof(double2) * size_t(b->mps_stride);
  const size_t chunk = std::max<size_t>(1, (size_t(256) << 20) / std::max<size_t>(per, 1));
  std::vector<double2> host;
  for (size_t i0 = 0; i0 < nn && st == QK_OK; i0 += chunk) {
    const size_t cnt = std::min(chunk, nn - i0);
    host.resize(cnt * size_t(b->mps_stride));
    f.read(reinterpret_cast<char *>(host.data()), std::streamsize(per * cnt));
    if (!f) {
      st = fail(QK_EINVAL, "truncated batch file");
      break;
    }
    for (const double2 &v : host)
      if (!std::isfinite(v.x) || !std::isfinite(v.y)) {
        st = fail(QK_EINVAL, "non-finite tensor entry");
        break;
      }
    if (st == QK_OK &&
        (hipMemcpyAsync(b->f64 + i0 * b->mps_stride, host.data(), per * cnt, hipMemcpyHostToDevice, stream) !=
             hipSuccess ||
         hipStreamSynchronize(stream) != hipSuccess))
      st = fail(QK_EDEVICE, "copy of loaded tensors failed");
  }
  if (st == QK_OK && nn > 0 &&
      (hipMemcpyAsync(b->dims_dev, dims.data(), sizeof(int32_t) * dims.size(), hipMemcpyHostToDevice, stream) !=
           hipSuccess ||
       hipMemcpyAsync(b->disc_dev, disc.data(), sizeof(double) * nn, hipMemcpyHostToDevice, stream) != hipSuccess ||
       hipMemcpyAsync(b->maxdisc_dev, maxdisc.data(), sizeof(double) * nn, hipMemcpyHostToDevice, stream) !=
           hipSuccess ||
       hipMemcpyAsync(b->degen_dev, degen.data(), sizeof(int32_t) * nn, hipMemcpyHostToDevice, stream) !=
           hipSuccess ||
       hipMemcpyAsync(b->unconv_dev, unconv.data(), sizeof(int32_t) * nn, hipMemcpyHostToDevice, stream) !=
           hipSuccess ||
       hipStreamSynchronize(stream) != hipSuccess))
    st = fail(QK_EDEVICE, "copy of loaded metadata failed");
  if (st != QK_OK) {
    batch_release(b);
    return st;
  }
  *out = b;
  return ok();
}

void mps_batch_free(qk_mps_batch *b) { batch_release(b); }

}  // extern "C"
