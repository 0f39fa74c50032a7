// Runs fsmp_sample of the library built for the CPU emulation (hip/hip_runtime.h here) on a
// batch written by tests/test_cpu_emu.py, and writes the chains' outputs.  Test
// infrastructure only.  Files in the directory argv[1] (raw little-endian):
//   ser.bin, intensity.bin, config.bin   fsmp_ser, fsmp_intensity, fsmp_config as in fsmp.h
//   design.txt                           one design per PE capacity (8 integers, -1: the default)
//   kz.txt                               the output row length
//   wave.f32, offsets.i64, lam.f64, kmax.i32, and when present g_range.i32, t0_init.f64,
//   noalloc (empty: call fsmp_sample_noalloc instead of fsmp_sample)
// and written there: n_pe.i32, t0.f64, z.i32, charge.f64, acc.f64, nhist.i32, counts.i32,
// status.u32, work.f64, rec_steps.i32, comp.i32 (with a mixture charge law), and as the
// configuration's record flags ask, log.bin (fsmp_logrec per chain and step), trace.f64,
// qdraw.f64, zdraw.i32.
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "fsmp.h"

static bool exists(const std::string &path) {
  std::FILE *f = std::fopen(path.c_str(), "rb");
  if (f) std::fclose(f);
  return f != nullptr;
}

static std::vector<char> slurp(const std::string &path) {
  std::FILE *f = std::fopen(path.c_str(), "rb");
  if (!f) {
    std::fprintf(stderr, "cannot open %s\n", path.c_str());
    std::exit(2);
  }
  std::vector<char> v;
  char buf[1 << 16];
  size_t n;
  while ((n = std::fread(buf, 1, sizeof buf, f)) > 0) v.insert(v.end(), buf, buf + n);
  std::fclose(f);
  return v;
}

template <typename T>
static void spit(const std::string &path, const std::vector<T> &v) {
  std::FILE *f = std::fopen(path.c_str(), "wb");
  if (!f || std::fwrite(v.data(), sizeof(T), v.size(), f) != v.size()) {
    std::fprintf(stderr, "cannot write %s\n", path.c_str());
    std::exit(2);
  }
  std::fclose(f);
}

template <typename T>
static std::vector<T> as(const std::vector<char> &raw) {
  std::vector<T> v(raw.size() / sizeof(T));
  std::memcpy(v.data(), raw.data(), v.size() * sizeof(T));
  return v;
}

int main(int argc, char **argv) {
  if (argc != 2) return 2;
  const std::string d = std::string(argv[1]) + "/";
  fsmp_ser ser;
  fsmp_intensity phi;
  fsmp_config cfg;
  const auto rs = slurp(d + "ser.bin"), ri = slurp(d + "intensity.bin"), rc = slurp(d + "config.bin");
  if (rs.size() != sizeof ser || ri.size() != sizeof phi || rc.size() != sizeof cfg) {
    std::fprintf(stderr, "struct sizes differ: %zu/%zu %zu/%zu %zu/%zu\n", rs.size(), sizeof ser, ri.size(),
                 sizeof phi, rc.size(), sizeof cfg);
    return 2;
  }
  std::memcpy(&ser, rs.data(), sizeof ser);
  std::memcpy(&phi, ri.data(), sizeof phi);
  std::memcpy(&cfg, rc.data(), sizeof cfg);
  const auto wave = as<float>(slurp(d + "wave.f32"));
  const auto offsets = as<int64_t>(slurp(d + "offsets.i64"));
  const auto lam = as<double>(slurp(d + "lam.f64"));
  const auto kmax = as<int32_t>(slurp(d + "kmax.i32"));
  const auto g_range = exists(d + "g_range.i32") ? as<int32_t>(slurp(d + "g_range.i32")) : std::vector<int32_t>();
  const auto t0_init = exists(d + "t0_init.f64") ? as<double>(slurp(d + "t0_init.f64")) : std::vector<double>();
  const int64_t n = (int64_t)lam.size();
  int kz = 0, design[8];
  {
    std::FILE *f = std::fopen((d + "kz.txt").c_str(), "r");
    if (!f || std::fscanf(f, "%d", &kz) != 1) return 2;
    std::fclose(f);
    f = std::fopen((d + "design.txt").c_str(), "r");
    for (int q = 0; q < 8; ++q)
      if (!f || std::fscanf(f, "%d", &design[q]) != 1) return 2;
    std::fclose(f);
  }
  fsmp_ctx *ctx = nullptr;
  if (fsmp_create(&ctx, &ser, &phi, &cfg, 0) != FSMP_OK) {
    std::fprintf(stderr, "create: %s\n", fsmp_last_error(nullptr));
    return 1;
  }
  static const int caps[8] = {16, 32, 48, 64, 96, 128, 160, 192};
  for (int q = 0; q < 8; ++q)
    if (design[q] >= 0 && fsmp_set_design(ctx, caps[q], design[q]) != FSMP_OK) {
      std::fprintf(stderr, "set_design %d %d: %s\n", caps[q], design[q], fsmp_last_error(ctx));
      return 1;
    }
  const int64_t C = n * cfg.n_chains;
  // "device" buffers: host memory, each its own allocation, exactly sized
  std::vector<int32_t> n_pe(C), z((size_t)C * kz), nhist((size_t)C * (kz + 1)), counts((size_t)C * 8);
  std::vector<double> t0(C), charge((size_t)C * kz), acc((size_t)C * 12);
  std::vector<uint32_t> status(C);
  std::vector<fsmp_logrec> log((size_t)C * cfg.n_steps);
  const int64_t n_rec = cfg.thin > 0 ? (cfg.n_steps - cfg.burn_in + cfg.thin - 1) / cfg.thin : 0;
  std::vector<double> trace((size_t)C * n_rec * 3), qdraw((size_t)C * n_rec * kz), work((size_t)C * 5);
  std::vector<int32_t> zdraw((size_t)C * n_rec * kz), rec_steps(C), comp((size_t)C * kz);
  fsmp_batch b{};
  b.n_wave = n;
  b.wave = wave.data();
  b.offsets = offsets.data();
  b.lambda = lam.data();
  b.kmax = kmax.data();
  b.g_range = g_range.empty() ? nullptr : g_range.data();
  b.t0_init = t0_init.empty() ? nullptr : t0_init.data();
  fsmp_samples o{};
  o.n_pe = n_pe.data();
  o.t0 = t0.data();
  o.z = z.data();
  o.charge = charge.data();
  o.acc = acc.data();
  o.nhist = nhist.data();
  o.counts = counts.data();
  o.status = status.data();
  o.log = (cfg.record_flags & FSMP_REC_LOG) ? log.data() : nullptr;
  o.trace = (cfg.record_flags & FSMP_REC_TRACE) ? trace.data() : nullptr;
  o.qdraw = (cfg.record_flags & FSMP_REC_CHARGE) ? qdraw.data() : nullptr;
  o.zdraw = (cfg.record_flags & FSMP_REC_CHARGE) ? zdraw.data() : nullptr;
  o.work = work.data();
  o.rec_steps = rec_steps.data();
  o.comp = cfg.n_mix > 0 ? comp.data() : nullptr;
  o.kz = kz;
  const bool noalloc = exists(d + "noalloc");
  if ((noalloc ? fsmp_sample_noalloc(ctx, &b, &o, nullptr) : fsmp_sample(ctx, &b, &o, nullptr)) != FSMP_OK) {
    std::fprintf(stderr, "sample: %s\n", fsmp_last_error(ctx));
    return 1;
  }
  fsmp_destroy(ctx);
  spit(d + "n_pe.i32", n_pe);
  spit(d + "t0.f64", t0);
  spit(d + "z.i32", z);
  spit(d + "charge.f64", charge);
  spit(d + "acc.f64", acc);
  spit(d + "nhist.i32", nhist);
  spit(d + "counts.i32", counts);
  spit(d + "status.u32", status);
  if (o.log) spit(d + "log.bin", log);
  if (o.trace) spit(d + "trace.f64", trace);
  if (o.qdraw) spit(d + "qdraw.f64", qdraw);
  if (o.zdraw) spit(d + "zdraw.i32", zdraw);
  spit(d + "work.f64", work);
  spit(d + "rec_steps.i32", rec_steps);
  if (o.comp) spit(d + "comp.i32", comp);
  std::printf("cpu emulation: %lld waveforms x %d chains x %d sweeps done\n", (long long)n, cfg.n_chains,
              cfg.n_steps);
  return 0;
}
