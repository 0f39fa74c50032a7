// fsmp_server.hip -- continuous-batching serving loop of libfsmp.so (include/fsmp.h).
//
// Host runtime only.  A pool of slots, each with its own HIP stream, fsmp_ctx
// (workspace) and device / pinned buffers; queued events are packed in arrival order
// into micro-batches that fit the device-memory budget and launched on idle slots, so
// requests that arrive while others run are admitted as slots and memory free up and
// their work overlaps on the device.  Results are scattered back per event.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <deque>
#include <memory>
#include <string>
#include <unordered_map>
#include <vector>

#include "fsmp_internal.h"

namespace {

using Clock = std::chrono::steady_clock;

struct Event {
  uint64_t id = 0;
  int64_t n_wave = 0;
  std::vector<float> wave;
  std::vector<int64_t> offsets;
  std::vector<double> lambda;
  std::vector<int32_t> kmax;
  Clock::time_point t_submit;
  std::vector<double> mean, mcse;
  std::vector<uint32_t> status;
  double latency = 0.0;
  int state = 0;  // 0 queued, 1 in flight, 2 done
};

template <typename T>
struct DBuf {
  T *p = nullptr;
  size_t n = 0;
  hipError_t ensure(size_t want) {
    if (want <= n && p) return hipSuccess;
    if (p) (void)hipFree(p);
    p = nullptr;
    n = 0;
    hipError_t e = hipMalloc((void **)&p, std::max<size_t>(want, 1) * sizeof(T));
    if (e == hipSuccess) n = std::max<size_t>(want, 1);
    return e;
  }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    n = 0;
  }
};

template <typename T>
struct HBuf {
  T *p = nullptr;
  size_t n = 0;
  hipError_t ensure(size_t want) {
    if (want <= n && p) return hipSuccess;
    if (p) (void)hipHostFree(p);
    p = nullptr;
    n = 0;
    hipError_t e = hipHostMalloc((void **)&p, std::max<size_t>(want, 1) * sizeof(T), hipHostMallocDefault);
    if (e == hipSuccess) n = std::max<size_t>(want, 1);
    return e;
  }
  void release() {
    if (p) (void)hipHostFree(p);
    p = nullptr;
    n = 0;
  }
};

struct Slot {
  fsmp_ctx *ctx = nullptr;
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  bool busy = false;
  std::vector<uint64_t> events;
  std::vector<int64_t> ev_first;  // first waveform of each event in the micro-batch
  int64_t n_wave = 0;
  size_t bytes = 0;
  // device
  DBuf<float> wave;
  DBuf<int32_t> n_pe, z, nhist, counts, status;
  DBuf<double> t0, charge, acc;
  DBuf<double> mean, var, mcse, accept;
  DBuf<uint32_t> pstatus;
  // host (pinned for the copies; plain vectors for the metadata fsmp_sample reads)
  HBuf<float> h_wave;
  HBuf<double> h_mean, h_mcse;
  HBuf<uint32_t> h_status;
  std::vector<int64_t> offsets;
  std::vector<double> lambda;
  std::vector<int32_t> kmax;
  std::vector<uint64_t> wid;
};

}  // namespace

struct fsmp_server {
  int device = 0;
  fsmp_config cfg{};
  fsmp_server_config scfg{};
  std::vector<std::unique_ptr<Slot>> slots;
  std::deque<uint64_t> queue;
  std::unordered_map<uint64_t, std::unique_ptr<Event>> events;
  size_t bytes_held = 0;
  int64_t n_done = 0;
  std::string err = "no error";
};

namespace {

fsmp_status sfail(fsmp_server *s, fsmp_status st, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (s) s->err = buf;
  return st;
}

std::string g_server_create_error = "no error";

int kcap_of(int kmax) {
  const int k = fsmp::chain_kcap_for(kmax);
  return k > 0 ? k : 192;
}

// device bytes a micro-batch holds: samples, matched filter over the whole window,
// per-chain state of the chain kernels, outputs
size_t event_bytes(const Event &e, int n_chains, int kz) {
  size_t b = 0;
  for (int64_t i = 0; i < e.n_wave; ++i) {
    const size_t L = (size_t)(e.offsets[i + 1] - e.offsets[i]);
    const size_t K = (size_t)kcap_of(e.kmax[i]);
    b += 4 * L + 8 * 4 * L + 64;
    b += (size_t)n_chains * (8 * (K * K + 5 * K) + 4 * (2 * K + 1));
    b += (size_t)n_chains * (8 * kz + 4 * kz + 4 * (kz + 1) + 12 * 8 + 8 * 4 + 32);
  }
  return b;
}

void retire(fsmp_server *s, Slot &sl, int &completed) {
  const auto now = Clock::now();
  for (size_t q = 0; q < sl.events.size(); ++q) {
    auto it = s->events.find(sl.events[q]);
    if (it == s->events.end()) continue;
    Event &e = *it->second;
    const int64_t f = sl.ev_first[q];
    e.mean.assign(sl.h_mean.p + 3 * f, sl.h_mean.p + 3 * (f + e.n_wave));
    e.mcse.assign(sl.h_mcse.p + 3 * f, sl.h_mcse.p + 3 * (f + e.n_wave));
    e.status.assign(sl.h_status.p + f, sl.h_status.p + f + e.n_wave);
    e.latency = std::chrono::duration<double>(now - e.t_submit).count();
    e.state = 2;
    e.wave.clear();
    e.wave.shrink_to_fit();
    ++completed;
    ++s->n_done;
  }
  s->bytes_held -= std::min(s->bytes_held, sl.bytes);
  sl.busy = false;
  sl.events.clear();
  sl.ev_first.clear();
}

fsmp_status launch(fsmp_server *s, Slot &sl, const std::vector<Event *> &batch) {
  const fsmp_config &cf = s->cfg;
  int64_t n = 0, samples = 0;
  int kz = 1;
  for (Event *e : batch) {
    n += e->n_wave;
    samples += e->offsets[e->n_wave];
    for (int32_t k : e->kmax) kz = std::max(kz, (int)k);
  }
  const int64_t C = n * cf.n_chains;
  hipError_t r = hipSuccess;
  r = sl.wave.ensure(samples);
  if (r == hipSuccess) r = sl.n_pe.ensure(C);
  if (r == hipSuccess) r = sl.t0.ensure(C);
  if (r == hipSuccess) r = sl.z.ensure((size_t)C * kz);
  if (r == hipSuccess) r = sl.charge.ensure((size_t)C * kz);
  if (r == hipSuccess) r = sl.acc.ensure((size_t)C * 12);
  if (r == hipSuccess) r = sl.nhist.ensure((size_t)C * (kz + 1));
  if (r == hipSuccess) r = sl.counts.ensure((size_t)C * 8);
  if (r == hipSuccess) r = sl.status.ensure(C);
  if (r == hipSuccess) r = sl.mean.ensure(3 * n);
  if (r == hipSuccess) r = sl.var.ensure(3 * n);
  if (r == hipSuccess) r = sl.mcse.ensure(3 * n);
  if (r == hipSuccess) r = sl.accept.ensure(4 * n);
  if (r == hipSuccess) r = sl.pstatus.ensure(n);
  if (r == hipSuccess) r = sl.h_wave.ensure(samples);
  if (r == hipSuccess) r = sl.h_mean.ensure(3 * n);
  if (r == hipSuccess) r = sl.h_mcse.ensure(3 * n);
  if (r == hipSuccess) r = sl.h_status.ensure(n);
  if (r != hipSuccess) return sfail(s, FSMP_ENOMEM, "server buffers: %s", hipGetErrorString(r));
  sl.offsets.assign(1, 0);
  sl.lambda.clear();
  sl.kmax.clear();
  sl.wid.clear();
  sl.events.clear();
  sl.ev_first.clear();
  int64_t w0 = 0, s0 = 0;
  for (Event *e : batch) {
    std::memcpy(sl.h_wave.p + s0, e->wave.data(), sizeof(float) * e->offsets[e->n_wave]);
    for (int64_t i = 0; i < e->n_wave; ++i) {
      sl.offsets.push_back(s0 + e->offsets[i + 1]);
      sl.lambda.push_back(e->lambda[i]);
      sl.kmax.push_back(e->kmax[i]);
      sl.wid.push_back((e->id << 16) | (uint64_t)i);
    }
    sl.events.push_back(e->id);
    sl.ev_first.push_back(w0);
    e->state = 1;
    w0 += e->n_wave;
    s0 += e->offsets[e->n_wave];
  }
  r = hipMemcpyAsync(sl.wave.p, sl.h_wave.p, sizeof(float) * samples, hipMemcpyHostToDevice, sl.stream);
  if (r != hipSuccess) return sfail(s, FSMP_EDEVICE, "upload: %s", hipGetErrorString(r));
  fsmp_batch b{};
  b.n_wave = n;
  b.wave = sl.wave.p;
  b.offsets = sl.offsets.data();
  b.lambda = sl.lambda.data();
  b.kmax = sl.kmax.data();
  b.wave_id = sl.wid.data();
  fsmp_samples o{};
  o.n_pe = sl.n_pe.p;
  o.t0 = sl.t0.p;
  o.z = sl.z.p;
  o.charge = sl.charge.p;
  o.acc = sl.acc.p;
  o.nhist = sl.nhist.p;
  o.counts = sl.counts.p;
  o.status = (uint32_t *)sl.status.p;
  o.kz = kz;
  fsmp_status st = fsmp_sample(sl.ctx, &b, &o, sl.stream);
  if (st != FSMP_OK) return sfail(s, st, "fsmp_sample: %s", fsmp_last_error(sl.ctx));
  fsmp_posterior_out po{};
  po.mean = sl.mean.p;
  po.var = sl.var.p;
  po.mcse = sl.mcse.p;
  po.accept = sl.accept.p;
  po.status = sl.pstatus.p;
  st = fsmp_posterior(sl.ctx, n, &o, &po, sl.stream);
  if (st != FSMP_OK) return sfail(s, st, "fsmp_posterior: %s", fsmp_last_error(sl.ctx));
  r = hipMemcpyAsync(sl.h_mean.p, sl.mean.p, sizeof(double) * 3 * n, hipMemcpyDeviceToHost, sl.stream);
  if (r == hipSuccess)
    r = hipMemcpyAsync(sl.h_mcse.p, sl.mcse.p, sizeof(double) * 3 * n, hipMemcpyDeviceToHost, sl.stream);
  if (r == hipSuccess)
    r = hipMemcpyAsync(sl.h_status.p, sl.pstatus.p, sizeof(uint32_t) * n, hipMemcpyDeviceToHost, sl.stream);
  if (r == hipSuccess) r = hipEventRecord(sl.done, sl.stream);
  if (r != hipSuccess) return sfail(s, FSMP_EDEVICE, "result copy: %s", hipGetErrorString(r));
  sl.n_wave = n;
  sl.busy = true;
  return FSMP_OK;
}

}  // namespace

extern "C" {

fsmp_status fsmp_server_create(fsmp_server **out, const fsmp_ser *ser, const fsmp_intensity *phi,
                               const fsmp_config *cfg, int device, const fsmp_server_config *scfg) {
  if (!out) return FSMP_EINVAL;
  *out = nullptr;
  if (cfg && cfg->record_flags != 0) {
    g_server_create_error = "the server returns posterior summaries only: record_flags must be 0";
    return FSMP_EINVAL;
  }
  if (!scfg || scfg->n_streams < 1 || scfg->n_streams > 16 || scfg->max_batch_wave < 1) {
    g_server_create_error = "server config: need 1..16 streams and max_batch_wave >= 1";
    return FSMP_EINVAL;
  }
  auto s = std::make_unique<fsmp_server>();
  s->device = device;
  s->cfg = *cfg;
  s->scfg = *scfg;
  int prev = 0;
  (void)hipGetDevice(&prev);
  for (int i = 0; i < scfg->n_streams; ++i) {
    auto sl = std::make_unique<Slot>();
    fsmp_status st = fsmp_create(&sl->ctx, ser, phi, cfg, device);
    if (st != FSMP_OK) {
      g_server_create_error = fsmp_last_error(nullptr);
      for (auto &x : s->slots) fsmp_destroy(x->ctx);
      return st;
    }
    // latency: the lane-group kernels finish a sweep in microseconds; one lane per chain
    // with its state in device memory needs many memory round trips per sweep.  The FP32
    // form has lane groups with G^-1 in device memory only: its wide groups (16 lanes per
    // chain at capacities 16 and 32, the narrow ones above, which are 32-64 lanes wide
    // from capacity 64 up).
    if (cfg->precision == FSMP_FP32_REFRESH) {
      (void)fsmp_set_design(sl->ctx, 0, FSMP_DESIGN_GROUP_DEVMEM);
      (void)fsmp_set_design(sl->ctx, 0, FSMP_DESIGN_GROUP_DEVMEM_WIDE);
    } else {
      (void)fsmp_set_design(sl->ctx, 0, FSMP_DESIGN_GROUP);
    }
    (void)hipSetDevice(device);
    if (hipStreamCreateWithFlags(&sl->stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&sl->done, hipEventDisableTiming) != hipSuccess) {
      g_server_create_error = "stream or event creation failed";
      fsmp_destroy(sl->ctx);
      for (auto &x : s->slots) fsmp_destroy(x->ctx);
      (void)hipSetDevice(prev);
      return FSMP_EDEVICE;
    }
    s->slots.push_back(std::move(sl));
  }
  (void)hipSetDevice(prev);
  *out = s.release();
  return FSMP_OK;
}

fsmp_status fsmp_server_submit(fsmp_server *s, uint64_t event_id, int64_t n_wave, const float *wave,
                               const int64_t *offsets, const double *lambda, const int32_t *kmax) {
  if (!s) return FSMP_EINVAL;
  if (n_wave < 1 || n_wave > 65536) return sfail(s, FSMP_EINVAL, "event %llu: n_wave %lld outside 1..65536",
                                                 (unsigned long long)event_id, (long long)n_wave);
  if (event_id >= (1ull << 48)) return sfail(s, FSMP_EINVAL, "event id must be below 2^48");
  if (!wave || !offsets || !lambda) return sfail(s, FSMP_EINVAL, "wave, offsets and lambda are required");
  if (s->events.count(event_id)) return sfail(s, FSMP_EINVAL, "event %llu already pending", (unsigned long long)event_id);
  if (offsets[0] != 0) return sfail(s, FSMP_EINVAL, "offsets[0] must be 0");
  auto e = std::make_unique<Event>();
  e->id = event_id;
  e->n_wave = n_wave;
  e->offsets.assign(offsets, offsets + n_wave + 1);
  for (int64_t i = 0; i < n_wave; ++i)
    if (e->offsets[i + 1] <= e->offsets[i] || e->offsets[i + 1] - e->offsets[i] > 65536)
      return sfail(s, FSMP_EINVAL, "event %llu: bad window %lld", (unsigned long long)event_id, (long long)i);
  e->wave.assign(wave, wave + e->offsets[n_wave]);
  e->lambda.assign(lambda, lambda + n_wave);
  if (kmax) e->kmax.assign(kmax, kmax + n_wave);
  else e->kmax.assign(n_wave, s->cfg.k_max);
  for (int64_t i = 0; i < n_wave; ++i)
    if (e->kmax[i] < 1 || e->kmax[i] > 192) return sfail(s, FSMP_EINVAL, "kmax outside 1..192");
  e->t_submit = Clock::now();
  s->queue.push_back(event_id);
  s->events[event_id] = std::move(e);
  return FSMP_OK;
}

int32_t fsmp_server_progress(fsmp_server *s, int32_t wait) {
  if (!s) return FSMP_EINVAL;
  int completed = 0;
  int prev = 0;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(s->device);
  for (auto &sl : s->slots)
    if (sl->busy && hipEventQuery(sl->done) == hipSuccess) retire(s, *sl, completed);
  // admit queued events into idle slots, in arrival order, within the memory budget
  for (auto &sl : s->slots) {
    if (sl->busy || s->queue.empty()) continue;
    std::vector<Event *> batch;
    int64_t nw = 0;
    size_t bytes = 0;
    const int kz_all = 192;
    while (!s->queue.empty()) {
      Event *e = s->events[s->queue.front()].get();
      const size_t eb = event_bytes(*e, s->cfg.n_chains, kz_all);
      const bool nothing_held = s->bytes_held == 0 && batch.empty();
      if (!batch.empty() && nw + e->n_wave > s->scfg.max_batch_wave) break;
      if (!nothing_held && s->bytes_held + bytes + eb > s->scfg.memory_budget) break;
      batch.push_back(e);
      nw += e->n_wave;
      bytes += eb;
      s->queue.pop_front();
    }
    if (batch.empty()) break;
    fsmp_status st = launch(s, *sl, batch);
    if (st != FSMP_OK) {
      (void)hipSetDevice(prev);
      return st;
    }
    sl->bytes = bytes;
    s->bytes_held += bytes;
  }
  if (wait && completed == 0) {
    Slot *oldest = nullptr;
    for (auto &sl : s->slots)
      if (sl->busy) {
        oldest = sl.get();
        break;
      }
    if (oldest) {
      (void)hipEventSynchronize(oldest->done);
      for (auto &sl : s->slots)
        if (sl->busy && hipEventQuery(sl->done) == hipSuccess) retire(s, *sl, completed);
    }
  }
  (void)hipSetDevice(prev);
  return completed;
}

fsmp_status fsmp_server_result(fsmp_server *s, uint64_t event_id, double *mean, double *mcse, uint32_t *status,
                               double *latency_s) {
  if (!s) return FSMP_EINVAL;
  auto it = s->events.find(event_id);
  if (it == s->events.end()) return sfail(s, FSMP_EINVAL, "unknown event %llu", (unsigned long long)event_id);
  Event &e = *it->second;
  if (e.state != 2) return FSMP_EBUSY;
  if (mean) std::memcpy(mean, e.mean.data(), sizeof(double) * e.mean.size());
  if (mcse) std::memcpy(mcse, e.mcse.data(), sizeof(double) * e.mcse.size());
  if (status) std::memcpy(status, e.status.data(), sizeof(uint32_t) * e.status.size());
  if (latency_s) *latency_s = e.latency;
  s->events.erase(it);
  return FSMP_OK;
}

fsmp_status fsmp_server_stats(const fsmp_server *s, int64_t *queued, int64_t *in_flight, int64_t *done,
                              size_t *bytes_held) {
  if (!s) return FSMP_EINVAL;
  int64_t fl = 0, dn = 0;
  for (const auto &kv : s->events) {
    if (kv.second->state == 1) ++fl;
    if (kv.second->state == 2) ++dn;
  }
  if (queued) *queued = (int64_t)s->queue.size();
  if (in_flight) *in_flight = fl;
  if (done) *done = dn;
  if (bytes_held) *bytes_held = s->bytes_held;
  return FSMP_OK;
}

const char *fsmp_server_last_error(const fsmp_server *s) { return s ? s->err.c_str() : g_server_create_error.c_str(); }

void fsmp_server_destroy(fsmp_server *s) {
  if (!s) return;
  int prev = 0;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(s->device);
  for (auto &sl : s->slots) {
    if (sl->stream) (void)hipStreamSynchronize(sl->stream);
    sl->wave.release();
    sl->n_pe.release();
    sl->z.release();
    sl->nhist.release();
    sl->counts.release();
    sl->status.release();
    sl->t0.release();
    sl->charge.release();
    sl->acc.release();
    sl->mean.release();
    sl->var.release();
    sl->mcse.release();
    sl->accept.release();
    sl->pstatus.release();
    sl->h_wave.release();
    sl->h_mean.release();
    sl->h_mcse.release();
    sl->h_status.release();
    if (sl->done) (void)hipEventDestroy(sl->done);
    if (sl->stream) (void)hipStreamDestroy(sl->stream);
    fsmp_destroy(sl->ctx);
  }
  (void)hipSetDevice(prev);
  delete s;
}

}  // extern "C"
