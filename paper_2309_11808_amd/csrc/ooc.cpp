// Out-of-core SPOD: the snapshot matrix reaches the device in chunks of rows.
// Pass 1 adds every chunk's weighted Gram into the Gram of every frequency,
// the eigenproblems are solved once, and pass 2 recomputes every chunk's
// Fourier blocks to form the rows of the modes it owns.  The kernels are the
// in-memory path's, run on a view of the plan restricted to the chunk's rows.
//
// Streams: `st` (the caller's) runs the kernels, `cin` the copies in and
// `cout` the copies out; events hand the device slots and mode buffers over
// between them, so the copy of chunk c+1 and the copy out of chunk c-1 overlap
// the kernels of chunk c.  Measured on the 1M-DOF, 8192-snapshot float32
// field with 32 chunks: a pinned host -> device copy runs at 56.8 GB/s; the
// streamed forward moves 68.7 GB in and 10.8 GB of modes out in 1.27 s.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <new>
#include <string>
#include <system_error>
#include <thread>
#include <vector>

#include "internal.h"

namespace spod {
namespace {

enum class Mem { Device, Pinned, Pageable };

Mem classify(const void* ptr) {
  hipPointerAttribute_t a;
  std::memset(&a, 0, sizeof(a));
  hipError_t e = hipPointerGetAttributes(&a, ptr);
  if (e != hipSuccess) {
    (void)hipGetLastError();   // not known to the runtime: ordinary host memory
    return Mem::Pageable;
  }
  if (a.type == hipMemoryTypeUnregistered) return Mem::Pageable;
  return a.type == hipMemoryTypeHost ? Mem::Pinned : Mem::Device;
}

hipMemcpyKind kind_in(Mem src) {
  return src == Mem::Pinned ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
}

// Device address of pinned host memory at p, when [p, p + bytes) lies inside
// one allocation mapped for the device; NULL otherwise.
char* mapped_range(void* p, size_t bytes) {
  hipPointerAttribute_t a;
  std::memset(&a, 0, sizeof(a));
  if (hipPointerGetAttributes(&a, p) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  if (a.type != hipMemoryTypeHost || !a.devicePointer) return nullptr;
  hipDeviceptr_t base = nullptr;
  size_t size = 0;
  if (hipMemGetAddressRange(&base, &size, a.devicePointer) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  char* d = static_cast<char*>(a.devicePointer);
  char* b = static_cast<char*>(base);
  if (d < b || bytes > size || (size_t)(d - b) > size - bytes) return nullptr;
  return d;
}

size_t up256(size_t x) { return (x + 255) / 256 * 256; }

// Runs part(0) .. part(t - 1), on threads where they can be started and on
// this thread otherwise; returns once every part has finished.
template <class F>
void run_parts(unsigned t, F part) {
  std::vector<std::thread> th;
  th.reserve(t);
  for (unsigned i = 0; i < t; ++i) {
    try {
      th.emplace_back(part, i);
    } catch (const std::system_error&) {
      part(i);
    }
  }
  for (auto& x : th) x.join();
}

// Host copies of `n` rows of `width` bytes (strides in bytes), split over a
// few threads once there is enough to copy.
void copy_rows(char* dst, size_t dpitch, const char* src, size_t spitch, size_t width, size_t n) {
  const size_t total = width * n;
  unsigned t = std::min<unsigned>(8, std::max(1u, std::thread::hardware_concurrency()));
  if (total < (size_t(64) << 20) || t < 2) t = 1;
  if (t == 1) {
    for (size_t r = 0; r < n; ++r) std::memcpy(dst + r * dpitch, src + r * spitch, width);
    return;
  }
  if (n == 1) {   // one long row: split the bytes instead
    const size_t step = (width + t - 1) / t;
    run_parts(t, [=](unsigned i) {
      const size_t b0 = std::min(width, i * step), b1 = std::min(width, b0 + step);
      std::memcpy(dst + b0, src + b0, b1 - b0);
    });
    return;
  }
  const size_t step = (n + t - 1) / t;
  run_parts(t, [=](unsigned i) {
    const size_t r0 = std::min(n, i * step), r1 = std::min(n, r0 + step);
    if (dpitch == width && spitch == width) {
      std::memcpy(dst + r0 * width, src + r0 * width, (r1 - r0) * width);
    } else {
      for (size_t r = r0; r < r1; ++r) std::memcpy(dst + r * dpitch, src + r * spitch, width);
    }
  });
}

}  // namespace

struct Ooc {
  Plan* plan = nullptr;          // the caller's; not owned
  spod_dtype dtype = SPOD_F32;
  int n_modes = 0;
  int64_t rows = 0, nchunks = 0, nres = 0, nstream = 0;   // nstream: slots of streamed chunks
  size_t esz = 4, csz = 8;
  size_t slot_bytes = 0, qhat_bytes = 0, phi_bytes = 0, ws_bytes = 0;
  size_t device_bytes = 0, pinned_bytes = 0;

  std::vector<void*> slot;       // device chunks of q, [rows][nt]
  void* qhat = nullptr;          // Fourier blocks of one chunk, [K][L][rows]
  void* phi_c[2] = {nullptr, nullptr};   // modes of one chunk, [K][n_modes][rows]
  double2* gram = nullptr;       // [K][L][L]
  double* mean = nullptr;        // [M]
  int32_t* info = nullptr;       // [K], when the caller passes no info array
  void* ws = nullptr;
  void* pin_q[2] = {nullptr, nullptr};   // pinned staging (allocated on demand)
  void* pin_phi[2] = {nullptr, nullptr};

  hipStream_t cin = nullptr, cout = nullptr;
  std::vector<hipEvent_t> loaded, freed;            // per slot
  hipEvent_t pin_free[2] = {nullptr, nullptr};      // copy in from pin_q[b] done
  hipEvent_t phi_ready[2] = {nullptr, nullptr};     // modes written to phi_c[b]
  hipEvent_t phi_free[2] = {nullptr, nullptr};      // copy out of phi_c[b] done
  hipEvent_t start = nullptr;

  int64_t row0(int64_t c) const { return c * rows; }
  int64_t nrows(int64_t c) const { return std::min(rows, plan->M - c * rows); }
  bool resident(int64_t c) const { return c >= nchunks - nres; }
  int slot_of(int64_t c) const {
    return resident(c) ? (int)(nstream + (c - (nchunks - nres))) : (int)(c % nstream);
  }
};

namespace {

void release(Ooc* o) {
  if (o->cin) (void)hipStreamSynchronize(o->cin);
  if (o->cout) (void)hipStreamSynchronize(o->cout);
  for (void* s : o->slot)
    if (s) (void)hipFree(s);
  void* dev[] = {o->qhat, o->phi_c[0], o->phi_c[1], o->gram, o->mean, o->info, o->ws};
  for (void* b : dev)
    if (b) (void)hipFree(b);
  void* pin[] = {o->pin_q[0], o->pin_q[1], o->pin_phi[0], o->pin_phi[1]};
  for (void* b : pin)
    if (b) (void)hipHostFree(b);
  for (hipEvent_t e : o->loaded)
    if (e) (void)hipEventDestroy(e);
  for (hipEvent_t e : o->freed)
    if (e) (void)hipEventDestroy(e);
  hipEvent_t ev[] = {o->pin_free[0], o->pin_free[1], o->phi_ready[0], o->phi_ready[1],
                     o->phi_free[0], o->phi_free[1], o->start};
  for (hipEvent_t e : ev)
    if (e) (void)hipEventDestroy(e);
  if (o->cin) (void)hipStreamDestroy(o->cin);
  if (o->cout) (void)hipStreamDestroy(o->cout);
  delete o;
}

// One forward pass: the pipeline state of a call.
struct Run {
  Ooc& o;
  const char* q;                 // the source (NULL with a reader)
  Mem q_mem;
  spod_read_fn read;
  void* user;
  char* phi;
  Mem phi_mem;
  char* phi_mapped;              // device address of a pinned phi (modes stored by a kernel)
  hipStream_t st;
  int next_pin = 0;              // pinned staging buffer of the next copy in
  int64_t pending[2] = {-1, -1}; // chunk whose modes wait in pin_phi[b] to be scattered

  spod_status hip(hipError_t e, const char* where) {
    return e == hipSuccess ? SPOD_OK : hip_fail(e, where);
  }

  // enqueue the copy of chunk c into its slot on `cin`
  spod_status load(int64_t c) {
    const int s = o.slot_of(c);
    const size_t bytes = (size_t)o.nrows(c) * (size_t)o.plan->nt * o.esz;
    const size_t off = (size_t)o.row0(c) * (size_t)o.plan->nt * o.esz;
    spod_status r = hip(hipStreamWaitEvent(o.cin, o.freed[s], 0), "hipStreamWaitEvent");
    if (r != SPOD_OK) return r;
    if (q && q_mem != Mem::Pageable) {
      r = hip(hipMemcpyAsync(o.slot[s], q + off, bytes, kind_in(q_mem), o.cin), "hipMemcpyAsync");
    } else {
      const int b = next_pin;
      next_pin ^= 1;
      r = hip(hipEventSynchronize(o.pin_free[b]), "hipEventSynchronize");
      if (r != SPOD_OK) return r;
      if (read) {
        const int rc = read(user, o.row0(c), o.nrows(c), o.pin_q[b]);
        if (rc != 0)
          return fail(SPOD_ERR_IO, "reader returned " + std::to_string(rc) + " for rows " +
                                       std::to_string(o.row0(c)) + "..");
      } else {
        copy_rows(static_cast<char*>(o.pin_q[b]), bytes, q + off, bytes, bytes, 1);
      }
      r = hip(hipMemcpyAsync(o.slot[s], o.pin_q[b], bytes, hipMemcpyHostToDevice, o.cin),
              "hipMemcpyAsync");
      if (r == SPOD_OK) r = hip(hipEventRecord(o.pin_free[b], o.cin), "hipEventRecord");
    }
    if (r == SPOD_OK) r = hip(hipEventRecord(o.loaded[s], o.cin), "hipEventRecord");
    return r;
  }

  // host side: scatter the modes staged in pin_phi[b] into the caller's phi
  spod_status drain(int b) {
    if (pending[b] < 0) return SPOD_OK;
    spod_status r = hip(hipEventSynchronize(o.phi_free[b]), "hipEventSynchronize");
    if (r != SPOD_OK) return r;
    const int64_t c = pending[b];
    const size_t width = (size_t)o.nrows(c) * o.csz;
    const size_t nrow = (size_t)o.plan->nfreq * (size_t)o.n_modes;
    copy_rows(phi + (size_t)o.row0(c) * o.csz, (size_t)o.plan->M * o.csz,
              static_cast<const char*>(o.pin_phi[b]), width, width, nrow);
    pending[b] = -1;
    return SPOD_OK;
  }

  // enqueue the copy of chunk c's modes (in phi_c[b]) to the caller's phi on `cout`
  spod_status store(int64_t c, int b) {
    spod_status r = hip(hipStreamWaitEvent(o.cout, o.phi_ready[b], 0), "hipStreamWaitEvent");
    if (r != SPOD_OK) return r;
    const size_t width = (size_t)o.nrows(c) * o.csz;
    const size_t nrow = (size_t)o.plan->nfreq * (size_t)o.n_modes;
    if (phi_mapped) {
      r = launch_store_rows(o.phi_c[b], phi_mapped + (size_t)o.row0(c) * o.csz, width,
                            (size_t)o.plan->M * o.csz, (int64_t)nrow, o.cout);
    } else if (phi_mem != Mem::Pageable) {
      r = hip(hipMemcpy2DAsync(phi + (size_t)o.row0(c) * o.csz, (size_t)o.plan->M * o.csz,
                               o.phi_c[b], width, width, nrow, hipMemcpyDefault, o.cout),
              "hipMemcpy2DAsync");
    } else {
      r = drain(b);
      if (r != SPOD_OK) return r;
      r = hip(hipMemcpyAsync(o.pin_phi[b], o.phi_c[b], width * nrow, hipMemcpyDeviceToHost,
                             o.cout),
              "hipMemcpyAsync");
      if (r == SPOD_OK) pending[b] = c;
    }
    if (r == SPOD_OK) r = hip(hipEventRecord(o.phi_free[b], o.cout), "hipEventRecord");
    return r;
  }

  spod_status pass1() {
    const Plan& p = *o.plan;
    for (int64_t c = 0; c < o.nchunks; ++c) {
      const int s = o.slot_of(c);
      spod_status r = load(c);
      if (r != SPOD_OK) return r;
      r = hip(hipStreamWaitEvent(st, o.loaded[s], 0), "hipStreamWaitEvent");
      if (r != SPOD_OK) return r;
      const Plan cp = plan_rows(p, o.row0(c), o.nrows(c));
      r = launch_blocks_fft(cp, o.slot[s], o.dtype, o.qhat, o.mean + o.row0(c), o.ws, st);
      if (r == SPOD_OK) r = hip(hipEventRecord(o.freed[s], st), "hipEventRecord");
      if (r == SPOD_OK) r = launch_csd(cp, o.qhat, o.gram, o.ws, st, c > 0);
      if (r != SPOD_OK) return r;
    }
    return SPOD_OK;
  }

  spod_status pass2(const double* lam, const void* psi, int32_t* n_valid) {
    const Plan& p = *o.plan;
    std::vector<int64_t> order;
    for (int64_t c = o.nchunks - o.nres; c < o.nchunks; ++c) order.push_back(c);
    for (int64_t c = 0; c < o.nchunks - o.nres; ++c) order.push_back(c);
    for (size_t i = 0; i < order.size(); ++i) {
      const int64_t c = order[i];
      const int s = o.slot_of(c);
      const int b = (int)(i & 1);
      spod_status r = SPOD_OK;
      if (!o.resident(c)) {
        r = load(c);
        if (r != SPOD_OK) return r;
        r = hip(hipStreamWaitEvent(st, o.loaded[s], 0), "hipStreamWaitEvent");
        if (r != SPOD_OK) return r;
      }
      const Plan cp = plan_rows(p, o.row0(c), o.nrows(c));
      r = launch_blocks_fft(cp, o.slot[s], o.dtype, o.qhat, o.mean + o.row0(c), o.ws, st);
      if (r == SPOD_OK) r = hip(hipEventRecord(o.freed[s], st), "hipEventRecord");
      if (r == SPOD_OK) r = hip(hipStreamWaitEvent(st, o.phi_free[b], 0), "hipStreamWaitEvent");
      if (r == SPOD_OK)
        r = launch_modes(cp, o.qhat, lam, psi, o.n_modes, o.phi_c[b], n_valid, o.ws, st);
      if (r == SPOD_OK) r = hip(hipEventRecord(o.phi_ready[b], st), "hipEventRecord");
      if (r == SPOD_OK) r = store(c, b);
      if (r != SPOD_OK) return r;
    }
    spod_status r = drain(0);
    if (r == SPOD_OK) r = drain(1);
    return r;
  }
};

// The allocations of spod_ooc_create (o is released on an error status).
spod_status ooc_create_body(Ooc* o, Plan* p, spod_dtype dtype, int64_t chunk_rows,
                            int64_t n_modes, int64_t resident, spod_ooc* out) {
  hipError_t e;
  o->plan = p;
  o->dtype = dtype;
  o->n_modes = (int)n_modes;
  // chunk rows: a multiple of 256 keeps every chunk's weights and blocks
  // 16-byte aligned for the vector loads of the kernels
  int64_t rows = (std::min(chunk_rows, p->M) + 255) / 256 * 256;
  if (rows >= p->M) rows = p->M;
  o->rows = rows;
  o->nchunks = (p->M + rows - 1) / rows;
  o->nres = std::min(resident, o->nchunks);
  o->nstream = std::min<int64_t>(2, o->nchunks - o->nres);
  o->esz = dtype == SPOD_F32 ? 4 : 8;
  o->csz = is_complex128(*p) ? 16 : 8;
  const size_t K = (size_t)p->nfreq, L = (size_t)p->nblocks;
  o->slot_bytes = up256((size_t)rows * (size_t)p->nt * o->esz);
  o->qhat_bytes = up256(qhat_bytes(plan_rows(*p, 0, rows)));
  o->phi_bytes = up256(K * (size_t)n_modes * (size_t)rows * o->csz);
  o->ws_bytes = std::max<size_t>(256, plan_rows(*p, 0, rows).ws_bytes);
  const size_t gram_bytes = up256(K * L * L * sizeof(double2));
  const size_t mean_bytes = up256((size_t)p->M * sizeof(double));
  const int64_t nslots = o->nstream + o->nres;
  o->device_bytes = (size_t)nslots * o->slot_bytes + o->qhat_bytes + 2 * o->phi_bytes +
                    gram_bytes + mean_bytes + o->ws_bytes;
  o->pinned_bytes = 2 * ((size_t)rows * (size_t)p->nt * o->esz) +
                    2 * (K * (size_t)n_modes * (size_t)rows * o->csz);

  auto bail = [&](hipError_t err, const char* where) {
    release(o);
    return err == hipErrorOutOfMemory ? fail(SPOD_ERR_ALLOC, where) : hip_fail(err, where);
  };
  o->slot.assign((size_t)nslots, nullptr);
  for (auto& s : o->slot)
    if ((e = hipMalloc(&s, o->slot_bytes)) != hipSuccess) return bail(e, "device chunk slots");
  if ((e = hipMalloc(&o->qhat, o->qhat_bytes)) != hipSuccess) return bail(e, "chunk blocks");
  for (auto& b : o->phi_c)
    if ((e = hipMalloc(&b, o->phi_bytes)) != hipSuccess) return bail(e, "chunk modes");
  if ((e = hipMalloc(&o->gram, gram_bytes)) != hipSuccess) return bail(e, "gram");
  if ((e = hipMalloc(&o->mean, mean_bytes)) != hipSuccess) return bail(e, "mean");
  if ((e = hipMalloc(&o->info, up256(K * sizeof(int32_t)))) != hipSuccess) return bail(e, "info");
  if ((e = hipMalloc(&o->ws, o->ws_bytes)) != hipSuccess) return bail(e, "workspace");
  if ((e = hipStreamCreateWithFlags(&o->cin, hipStreamNonBlocking)) != hipSuccess)
    return bail(e, "hipStreamCreateWithFlags");
  if ((e = hipStreamCreateWithFlags(&o->cout, hipStreamNonBlocking)) != hipSuccess)
    return bail(e, "hipStreamCreateWithFlags");
  o->loaded.assign((size_t)nslots, nullptr);
  o->freed.assign((size_t)nslots, nullptr);
  std::vector<hipEvent_t*> evs;
  for (auto& x : o->loaded) evs.push_back(&x);
  for (auto& x : o->freed) evs.push_back(&x);
  for (int b = 0; b < 2; ++b) {
    evs.push_back(&o->pin_free[b]);
    evs.push_back(&o->phi_ready[b]);
    evs.push_back(&o->phi_free[b]);
  }
  evs.push_back(&o->start);
  for (hipEvent_t* x : evs)
    if ((e = hipEventCreateWithFlags(x, hipEventDisableTiming)) != hipSuccess)
      return bail(e, "hipEventCreateWithFlags");
  freeze(*p);
  *out = reinterpret_cast<spod_ooc>(o);
  return SPOD_OK;
}

}  // namespace
}  // namespace spod

using namespace spod;

extern "C" {

spod_status spod_ooc_create(spod_plan plan, spod_dtype dtype, int64_t chunk_rows, int64_t n_modes,
                            int64_t resident, spod_ooc* out) {
  return guarded([&]() -> spod_status {
    if (!out) return fail(SPOD_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    Plan* p = reinterpret_cast<Plan*>(plan);
    if (!p) return fail(SPOD_ERR_INVALID_ARG, "plan is NULL");
    if (dtype != SPOD_F32 && dtype != SPOD_F64) return fail(SPOD_ERR_INVALID_ARG, "dtype");
    if (chunk_rows < 1) return fail(SPOD_ERR_INVALID_ARG, "chunk_rows must be >= 1");
    if (n_modes < 1 || n_modes > p->nblocks)
      return fail(SPOD_ERR_INVALID_ARG, "n_modes must be in [1, nblocks]");
    if (resident < 0) return fail(SPOD_ERR_INVALID_ARG, "resident must be >= 0");
    if (p->nblocks > SPOD_MAX_NBLOCKS) return fail(SPOD_ERR_UNSUPPORTED, "nblocks > 160");
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (cur != p->device) return fail(SPOD_ERR_INVALID_ARG, "plan belongs to another device");

    Ooc* o = new (std::nothrow) Ooc();
    if (!o) return fail(SPOD_ERR_ALLOC, "out-of-core object");
    try {
      return ooc_create_body(o, p, dtype, chunk_rows, n_modes, resident, out);
    } catch (...) {
      release(o);
      throw;
    }
  });
}

spod_status spod_ooc_query(spod_ooc ooc, int64_t* chunk_rows, int64_t* n_chunks,
                           int64_t* n_resident, size_t* device_bytes, size_t* pinned_bytes) {
  Ooc* o = reinterpret_cast<Ooc*>(ooc);
  if (!o) return fail(SPOD_ERR_INVALID_ARG, "ooc is NULL");
  if (chunk_rows) *chunk_rows = o->rows;
  if (n_chunks) *n_chunks = o->nchunks;
  if (n_resident) *n_resident = o->nres;
  if (device_bytes) *device_bytes = o->device_bytes;
  if (pinned_bytes) *pinned_bytes = o->pinned_bytes;
  return SPOD_OK;
}

spod_status spod_ooc_forward(spod_ooc ooc, const void* q, spod_read_fn read, void* user,
                             double* mean, double* lam, void* psi, int32_t* info, void* phi,
                             int32_t* n_valid, spod_stream stream) {
  return guarded([&]() -> spod_status {
    Ooc* o = reinterpret_cast<Ooc*>(ooc);
    if (!o) return fail(SPOD_ERR_INVALID_ARG, "ooc is NULL");
    if ((q == nullptr) == (read == nullptr))
      return fail(SPOD_ERR_INVALID_ARG, "exactly one of q and read is required");
    if (!mean || !lam || !psi || !phi)
      return fail(SPOD_ERR_INVALID_ARG, "mean, lam, psi and phi are required");
    const Plan& p = *o->plan;
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (cur != p.device) return fail(SPOD_ERR_INVALID_ARG, "plan belongs to another device");

    const Mem q_mem = q ? classify(q) : Mem::Pageable;
    const Mem phi_mem = classify(phi);
    // pinned staging, kept for later calls
    if (q_mem == Mem::Pageable && !o->pin_q[0]) {
      const size_t b = (size_t)o->rows * (size_t)p.nt * o->esz;
      for (auto& x : o->pin_q)
        if ((e = hipHostMalloc(&x, b, hipHostMallocDefault)) != hipSuccess)
          return e == hipErrorOutOfMemory ? fail(SPOD_ERR_ALLOC, "pinned staging")
                                          : hip_fail(e, "hipHostMalloc");
    }
    if (phi_mem == Mem::Pageable && !o->pin_phi[0]) {
      const size_t b = (size_t)p.nfreq * (size_t)o->n_modes * (size_t)o->rows * o->csz;
      for (auto& x : o->pin_phi)
        if ((e = hipHostMalloc(&x, b, hipHostMallocDefault)) != hipSuccess)
          return e == hipErrorOutOfMemory ? fail(SPOD_ERR_ALLOC, "pinned staging")
                                          : hip_fail(e, "hipHostMalloc");
    }

    hipStream_t st = (hipStream_t)stream;
    // Modes going to pinned host memory while chunks are still coming in are
    // stored by a kernel through the memory's device address: a DMA copy out
    // was measured to wait for the DMA copies in (one engine), a kernel's
    // stores run beside them.  With every chunk resident nothing comes in
    // during the modes pass and the DMA copy is the faster one.
    char* phi_mapped =
        phi_mem == Mem::Pinned && o->nres < o->nchunks
            ? mapped_range(phi, (size_t)p.nfreq * (size_t)o->n_modes * (size_t)p.M * o->csz)
            : nullptr;
    Run run{*o, static_cast<const char*>(q), q_mem, read, user, static_cast<char*>(phi), phi_mem,
            phi_mapped, st};
    spod_status r = run.hip(hipEventRecord(o->start, st), "hipEventRecord");
    if (r == SPOD_OK) r = run.hip(hipStreamWaitEvent(o->cin, o->start, 0), "hipStreamWaitEvent");
    if (r == SPOD_OK) r = run.hip(hipStreamWaitEvent(o->cout, o->start, 0), "hipStreamWaitEvent");
    try {
      if (r == SPOD_OK) r = run.pass1();
      if (r == SPOD_OK) r = launch_eig(p, o->gram, lam, psi, info ? info : o->info, o->ws, st);
      if (r == SPOD_OK) r = run.pass2(lam, psi, n_valid);
    } catch (const std::bad_alloc&) {
      r = fail(SPOD_ERR_ALLOC, "host memory");
    } catch (...) {
      r = fail(SPOD_ERR_INTERNAL, "unexpected exception");
    }
    // nothing of this call may still run when it returns, error or not
    hipError_t e1 = hipStreamSynchronize(st);
    hipError_t e2 = hipStreamSynchronize(o->cin);
    hipError_t e3 = hipStreamSynchronize(o->cout);
    if (r != SPOD_OK) return r;
    if (e1 != hipSuccess) return hip_fail(e1, "hipStreamSynchronize");
    if (e2 != hipSuccess) return hip_fail(e2, "hipStreamSynchronize");
    if (e3 != hipSuccess) return hip_fail(e3, "hipStreamSynchronize");
    e = hipMemcpy(mean, o->mean, sizeof(double) * (size_t)p.M, hipMemcpyDefault);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpy");
    // every output is written; a frequency whose Gram was not finite (NaN or
    // infinite data) is reported as a numeric failure of the whole call
    std::vector<int32_t> h_info((size_t)p.nfreq);
    e = hipMemcpy(h_info.data(), info ? info : o->info, sizeof(int32_t) * (size_t)p.nfreq,
                  hipMemcpyDefault);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpy");
    for (int32_t v : h_info)
      if (v == SPOD_INFO_NONFINITE) return fail(SPOD_ERR_NUMERIC, "non-finite data (see info)");
    return SPOD_OK;
  });
}

void spod_ooc_destroy(spod_ooc ooc) {
  Ooc* o = reinterpret_cast<Ooc*>(ooc);
  if (o) release(o);
}

}  // extern "C"
