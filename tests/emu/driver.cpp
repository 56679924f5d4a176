// CPU emulation driver: runs the library's own trajectory code (the real
// runtime and kernel sources, emulated on the host by emu.cpp) for one
// configuration and writes the recorded x_t and y_t.
//
// usage: driver ENS N T KIND A B PATTERN SEED TRIAL F64 CPT X1_FILE OUT_PREFIX
//   ENS 0 Gaussian (sigma = 1/sqrt(N)) / 1 Haar; KIND as HD_DYN_*; PATTERN
//   0 = Q only, 1 = alternating; CPT 0 = the built-in shape, else forced;
//   X1_FILE holds N values of the storage type.  Writes OUT_PREFIX.X
//   ((T+1) x N) and OUT_PREFIX.Y (T x N) and prints "rc <code> status <code>".
// usage: driver ista M N L COUNT SEED TRIAL0 SIGMA A THETA XSTAR NOISE OUT
//          [G_FILE GRAD_OUT]
//   an FP32 batch of unrolled-ISTA trials with constant (A, THETA); XSTAR
//   (COUNT x N) and NOISE (COUNT x M) files; writes OUT (COUNT x (L+1) x N).
//   With G_FILE (COUNT x N, dL/dx_{L+1}) the batch also runs its reverse
//   pass and writes GRAD_OUT: dL/da (COUNT x L), dL/dtheta (COUNT x L), FP64.
// usage: driver cplx ENS M N F64 SEED TRIAL SIGMA PATTERN X_FILE OUT
//   complex queries on one handle: PATTERN is a string of Q (y = Q x),
//   H (y = Q^H x) and G (GUE step); X_FILE holds the query vectors back to
//   back (interleaved complex, storage type), OUT receives the answers.
// usage: driver crun N T A B F64 SEED TRIAL X1_FILE OUT_PREFIX
//   a complex Haar trajectory (hd_crun); writes OUT_PREFIX.X and .Y.
// usage: driver batch SPEC_FILE X1_FILE OUT [SHAPES]
//   a batch of FP32 Haar trials (hd_batch_run, tanh(2y), Q-queries): SPEC_FILE
//   holds int64 pairs (n, T) per trial (seed 0, trial = index); X1_FILE the
//   x_1 of every trial back to back; OUT receives every trial's
//   trajectory (T + 1) x n back to back.  With SHAPES (digits 1, 2, 4 and
//   'a'): one run per digit after hd_batch_set_shape, written to OUT.0,
//   OUT.1, ...; 'a' runs hd_batch_autotune.
#include "hd_api.hip"

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

static void* read_file(const char* path, size_t bytes) {
  void* p = std::malloc(bytes);
  FILE* f = std::fopen(path, "rb");
  if (!f || std::fread(p, 1, bytes, f) != bytes) {
    std::fprintf(stderr, "cannot read %s\n", path);
    std::exit(2);
  }
  std::fclose(f);
  return p;
}

static void write_file(const char* path, const void* p, size_t bytes) {
  FILE* f = std::fopen(path, "wb");
  if (!f || std::fwrite(p, 1, bytes, f) != bytes) {
    std::fprintf(stderr, "cannot write %s\n", path);
    std::exit(2);
  }
  std::fclose(f);
}

static int ista_main(char** argv) {
  const int64_t m = std::atoll(argv[2]), n = std::atoll(argv[3]);
  const int L = std::atoi(argv[4]), C = std::atoi(argv[5]);
  const uint32_t seed = (uint32_t)std::atol(argv[6]);
  const uint32_t trial0 = (uint32_t)std::atol(argv[7]);
  const double sigma = std::atof(argv[8]);
  std::vector<float> a(L, (float)std::atof(argv[9]));
  std::vector<float> th(L, (float)std::atof(argv[10]));
  void* xs = read_file(argv[11], 4 * (size_t)C * n);
  void* w = read_file(argv[12], 4 * (size_t)C * m);
  const size_t xb = 4 * (size_t)C * (L + 1) * n;
  void* X = std::calloc(1, xb);
  const bool grad = argv[14] != nullptr;
  hd_ista b = nullptr;
  int rc = hd_ista_init(HD_F32, m, n, L, C, seed, trial0, sigma,
                        grad ? HD_ISTA_GRAD : 0, nullptr, &b);
  if (!rc) rc = hd_ista_run(b, a.data(), th.data(), xs, w, X);
  if (grad) {
    void* G = read_file(argv[14], 4 * (size_t)C * n);
    std::vector<double> gr(2 * (size_t)C * L, 0.0);
    if (!rc)
      rc = hd_ista_grad(b, a.data(), th.data(), G, gr.data(),
                        gr.data() + (size_t)C * L);
    write_file(argv[15], gr.data(), gr.size() * sizeof(double));
    std::free(G);
  }
  const int st = rc ? 0 : hd_ista_status(b);
  write_file(argv[13], X, xb);
  std::printf("rc %d status %d\n", rc, st);
  hd_ista_free(b);
  std::free(xs);
  std::free(w);
  std::free(X);
  return rc ? 1 : 0;
}

static int cplx_main(char** argv) {
  const int ens = std::atoi(argv[2]);
  const int64_t m = std::atoll(argv[3]), n = std::atoll(argv[4]);
  const int f64 = std::atoi(argv[5]);
  const uint32_t seed = (uint32_t)std::atol(argv[6]);
  const uint32_t trial = (uint32_t)std::atol(argv[7]);
  const double sigma = std::atof(argv[8]);
  const std::string pat = argv[9];
  const size_t es = f64 ? 16 : 8;
  size_t in = 0, out = 0;
  int tq = 0;
  for (char c : pat) {
    in += es * (c == 'H' ? m : n);
    out += es * (c == 'Q' ? m : n);
    tq += c == 'G' ? 2 : 1;
  }
  char* X = (char*)read_file(argv[10], in);
  char* Y = (char*)std::calloc(1, out);
  hd_chandle h = nullptr;
  int rc = hd_cinit(ens, f64 ? HD_F64 : HD_F32, m, n, tq, seed, trial, sigma,
                    nullptr, &h);
  size_t xi = 0, yi = 0;
  for (char c : pat) {
    if (rc) break;
    if (c == 'G')
      rc = hd_cgue_step(h, X + xi, Y + yi);
    else
      rc = hd_cstep(h, c == 'H', X + xi, Y + yi);
    xi += es * (c == 'H' ? m : n);
    yi += es * (c == 'Q' ? m : n);
  }
  const int st = rc ? 0 : hd_cstatus(h);
  write_file(argv[11], Y, out);
  std::printf("rc %d status %d\n", rc, st);
  hd_cfree(h);
  std::free(X);
  std::free(Y);
  return rc ? 1 : 0;
}

static int crun_main(char** argv) {
  const int64_t n = std::atoll(argv[2]);
  const int T = std::atoi(argv[3]);
  const double a = std::atof(argv[4]), b = std::atof(argv[5]);
  const int f64 = std::atoi(argv[6]);
  const uint32_t seed = (uint32_t)std::atol(argv[7]);
  const uint32_t trial = (uint32_t)std::atol(argv[8]);
  const size_t row = (f64 ? 16 : 8) * (size_t)n;
  char* X = (char*)std::calloc(1, row * (T + 1));
  char* Y = (char*)std::calloc(1, row * T);
  void* x1 = read_file(argv[9], row);
  std::memcpy(X, x1, row);
  hd_chandle h = nullptr;
  int rc = hd_cinit(HD_HAAR, f64 ? HD_F64 : HD_F32, n, n, T, seed, trial, 1.0,
                    nullptr, &h);
  if (!rc) rc = hd_crun(h, T, a, b, X, Y);
  const int st = rc ? 0 : hd_cstatus(h);
  const std::string pre = argv[10];
  write_file((pre + ".X").c_str(), X, row * (T + 1));
  write_file((pre + ".Y").c_str(), Y, row * T);
  std::printf("rc %d status %d\n", rc, st);
  hd_cfree(h);
  std::free(X);
  std::free(Y);
  std::free(x1);
  return rc ? 1 : 0;
}

static int batch_main(char** argv, const char* shapes) {
  FILE* f = std::fopen(argv[2], "rb");
  std::vector<int64_t> spec;
  int64_t v;
  while (f && std::fread(&v, sizeof(v), 1, f) == 1) spec.push_back(v);
  if (f) std::fclose(f);
  const int count = (int)(spec.size() / 2);
  std::vector<hd_batch_trial> tr(count);
  size_t xin = 0, xout = 0;
  for (int i = 0; i < count; ++i) {
    tr[i].n = spec[2 * i];
    tr[i].T = (int32_t)spec[2 * i + 1];
    tr[i].seed = 0;
    tr[i].trial = (uint32_t)i;
    xin += (size_t)tr[i].n;
    xout += (size_t)tr[i].n * (tr[i].T + 1);
  }
  float* x1 = (float*)read_file(argv[3], 4 * xin);
  float* X = (float*)std::calloc(xout, 4);
  std::vector<const void*> px(count);
  std::vector<void*> ptx(count);
  size_t oi = 0, oo = 0;
  for (int i = 0; i < count; ++i) {
    px[i] = x1 + oi;
    ptx[i] = X + oo;
    oi += (size_t)tr[i].n;
    oo += (size_t)tr[i].n * (tr[i].T + 1);
  }
  hd_batch b = nullptr;
  int rc = hd_batch_init(HD_F32, tr.data(), count, nullptr, &b);
  hd_dynamics dyn;
  dyn.kind = HD_DYN_TANH;
  dyn.pattern = HD_PATTERN_Q;
  dyn.a = 2.0;
  dyn.b = 0.0;
  if (!shapes) {
    if (!rc)
      rc = hd_batch_run(b, &dyn, px.data(), nullptr, ptx.data(), nullptr);
    const int st = rc ? 0 : hd_batch_status(b);
    write_file(argv[4], X, 4 * xout);
    std::printf("rc %d status %d\n", rc, st);
  } else {
    // one run per shape digit, each after hd_batch_set_shape; 'a' runs the
    // autotuner (one timed run per shape) and reports what it installed
    int k = 0;
    for (const char* c = shapes; *c && !rc; ++c) {
      if (*c == 'a') {
        int32_t ch = 0;
        double ms[3];
        rc = hd_batch_autotune(b, &dyn, px.data(), 1, ms, &ch);
        std::printf("tuned %d shape %d\n", ch, hd_batch_shape(b));
        continue;
      }
      rc = hd_batch_set_shape(b, *c - '0');
      std::memset(X, 0, 4 * xout);
      if (!rc)
        rc = hd_batch_run(b, &dyn, px.data(), nullptr, ptx.data(), nullptr);
      const int st = rc ? 0 : hd_batch_status(b);
      write_file((std::string(argv[4]) + "." + std::to_string(k++)).c_str(),
                 X, 4 * xout);
      std::printf("shape %d rc %d status %d\n", hd_batch_shape(b), rc, st);
    }
  }
  hd_batch_free(b);
  std::free(x1);
  std::free(X);
  return rc ? 1 : 0;
}

int main(int argc, char** argv) {
  if ((argc == 5 || argc == 6) && std::string(argv[1]) == "batch")
    return batch_main(argv, argc == 6 ? argv[5] : nullptr);
  if ((argc == 14 || argc == 16) && std::string(argv[1]) == "ista")
    return ista_main(argv);
  if (argc == 12 && std::string(argv[1]) == "cplx") return cplx_main(argv);
  if (argc == 11 && std::string(argv[1]) == "crun") return crun_main(argv);
  if (argc != 14) {
    std::fprintf(stderr, "usage: see the header of driver.cpp\n");
    return 2;
  }
  const int ens = std::atoi(argv[1]);
  const int64_t n = std::atoll(argv[2]);
  const int T = std::atoi(argv[3]);
  hd_dynamics dyn;
  dyn.kind = std::atoi(argv[4]);
  dyn.a = std::atof(argv[5]);
  dyn.b = std::atof(argv[6]);
  dyn.pattern = std::atoi(argv[7]);
  const uint32_t seed = (uint32_t)std::atol(argv[8]);
  const uint32_t trial = (uint32_t)std::atol(argv[9]);
  const int f64 = std::atoi(argv[10]);
  const int cpt = std::atoi(argv[11]);
  if (cpt) setenv("HD_CPT", argv[11], 1);
  hd_config cfg;
  std::memset(&cfg, 0, sizeof(cfg));
  cfg.ensemble = ens;
  cfg.storage = f64 ? HD_F64 : HD_F32;
  cfg.m = cfg.n = n;
  cfg.t_max = T;
  cfg.seed = seed;
  cfg.trial = trial;
  cfg.sigma = 1.0 / std::sqrt((double)n);
  hd_handle h = nullptr;
  int rc = hd_init(&cfg, &h);
  if (rc) {
    std::printf("rc %d status 0\n", rc);
    return 1;
  }
  const size_t es = f64 ? 8 : 4;
  void* x1 = read_file(argv[12], es * (size_t)n);
  void* X = std::malloc(es * (size_t)n * (size_t)(T + 1));
  void* Y = std::malloc(es * (size_t)n * (size_t)T);
  rc = run_dynamics(h, &dyn, T, x1, nullptr, nullptr, X, Y);
  const int st = hd_status(h);
  std::string pre = argv[13];
  write_file((pre + ".X").c_str(), X, es * (size_t)n * (size_t)(T + 1));
  write_file((pre + ".Y").c_str(), Y, es * (size_t)n * (size_t)T);
  std::printf("rc %d status %d\n", rc, st);
  hd_free(h);
  std::free(x1);
  std::free(X);
  std::free(Y);
  return rc ? 1 : 0;
}
