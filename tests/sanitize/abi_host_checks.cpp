// Host code of libepm under AddressSanitizer and UndefinedBehaviorSanitizer.
//
// Runs, on a machine without a GPU, every host path that comes before the
// first device call: argument validation, the FP64 pair setup (Eq. 1-2,
// pencil basis, rank check) over many geometries, the workspace layout, the
// pose-prior and tolerance-feature tables, and the clean-up after every error.
// With no device, a call that gets as far as the runtime returns EPM_ERR_HIP,
// and that is checked as well.  Exits non-zero on the first failed check; the
// sanitizers abort on the first memory error or undefined behaviour.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <vector>

#include "epm.h"

#define CHECK(cond)                                                          \
  do {                                                                       \
    if (!(cond)) {                                                           \
      std::fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #cond); \
      std::exit(1);                                                          \
    }                                                                        \
  } while (0)

namespace {

void mul3(const double* A, const double* B, double* C) {
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) {
      double s = 0.0;
      for (int k = 0; k < 3; ++k) s += A[3 * r + k] * B[3 * k + c];
      C[3 * r + c] = s;
    }
}

void rot(double ax, double ay, double az, double* R) {
  const double cx = std::cos(ax), sx = std::sin(ax), cy = std::cos(ay), sy = std::sin(ay);
  const double cz = std::cos(az), sz = std::sin(az);
  const double X[9] = {1, 0, 0, 0, cx, -sx, 0, sx, cx};
  const double Y[9] = {cy, 0, sy, 0, 1, 0, -sy, 0, cy};
  const double Z[9] = {cz, -sz, 0, sz, cz, 0, 0, 0, 1};
  double T[9];
  mul3(X, Y, T);
  mul3(T, Z, R);
}

// F = K^-T [t]x R K^-1 for K = [[f, 0, w/2], [0, f, h/2], [0, 0, 1]].
void fundamental(double f, int w, int h, const double* R, const double* t, double* F) {
  const double cx = 0.5 * w, cy = 0.5 * h;
  const double Ki[9] = {1 / f, 0, -cx / f, 0, 1 / f, -cy / f, 0, 0, 1};
  const double KiT[9] = {Ki[0], Ki[3], Ki[6], Ki[1], Ki[4], Ki[7], Ki[2], Ki[5], Ki[8]};
  const double Tx[9] = {0, -t[2], t[1], t[2], 0, -t[0], -t[1], t[0], 0};
  double A[9], B[9];
  mul3(KiT, Tx, A);
  mul3(A, R, B);
  mul3(B, Ki, F);
}

struct Batch {
  std::vector<epm_pair> pairs;
  int64_t n1 = 0, n2 = 0;
  void add(const double* F, int w, int h, int64_t m, int64_t n) {
    epm_pair p;
    std::memcpy(p.F, F, sizeof(p.F));
    p.w2 = w;
    p.h2 = h;
    p.q_begin = n1;
    p.m = m;
    p.k_begin = n2;
    p.n = n;
    n1 += m;
    n2 += n;
    pairs.push_back(p);
  }
};

// Aligned host buffer standing in for device memory (only its address and
// size are used on the host).
struct Buf {
  void* p = nullptr;
  size_t bytes = 0;
  explicit Buf(size_t b) : bytes(b ? b : 256) {
    p = std::aligned_alloc(256, (bytes + 255) / 256 * 256);
    std::memset(p, 0, (bytes + 255) / 256 * 256);
  }
  ~Buf() { std::free(p); }
  template <class T> T* as() const { return static_cast<T*>(p); }
};

Batch random_batch(std::mt19937_64& rng, int num) {
  std::uniform_real_distribution<double> U(-1.0, 1.0);
  std::uniform_int_distribution<int> kind(0, 5), sz(0, 3000);
  Batch b;
  for (int k = 0; k < num; ++k) {
    const int w = 320 + (int)(rng() % 6000), h = 240 + (int)(rng() % 4000);
    const double f = 0.5 * w + (double)(rng() % 4000);
    double R[9], t[3], F[9];
    switch (kind(rng)) {
      case 0:  // sideways: epipole at infinity
        rot(0, 0, 0, R);
        t[0] = 1; t[1] = 0; t[2] = 0;
        break;
      case 1:  // forward: epipole in the image
        rot(0.01 * U(rng), 0.01 * U(rng), 0, R);
        t[0] = 0; t[1] = 0; t[2] = -1;
        break;
      case 2:  // epipole far outside
        rot(0.1 * U(rng), 0.1 * U(rng), 0.1 * U(rng), R);
        t[0] = 1; t[1] = 0.2 * U(rng); t[2] = 1e-7 * U(rng);
        break;
      default:  // general
        rot(0.3 * U(rng), 0.3 * U(rng), 0.3 * U(rng), R);
        t[0] = U(rng); t[1] = U(rng); t[2] = U(rng);
    }
    fundamental(f, w, h, R, t, F);
    const double s = std::ldexp(1.0, (int)(rng() % 41) - 20);  // scale of F is free
    for (double& v : F) v *= s;
    b.add(F, w, h, k % 7 == 3 ? 0 : sz(rng), k % 11 == 5 ? 0 : sz(rng));
  }
  return b;
}

void check_build(const Batch& b, epm_status want) {
  const size_t ws = epm_workspace_bytes(b.pairs.data(), (int32_t)b.pairs.size());
  CHECK(ws > 0);
  Buf W(ws), kp2(8 * (size_t)b.n2 + 8), eps2(4 * (size_t)b.n2 + 4);
  epm_index* idx = reinterpret_cast<epm_index*>(0x1);
  const epm_status st = epm_build_intervals(b.pairs.data(), (int32_t)b.pairs.size(),
                                            kp2.as<float>(), nullptr, 2.0f, W.p, ws, &idx,
                                            nullptr);
  CHECK(st == want);
  CHECK(idx == nullptr);
  idx = reinterpret_cast<epm_index*>(0x1);
  CHECK(epm_build_intervals(b.pairs.data(), (int32_t)b.pairs.size(), kp2.as<float>(),
                            eps2.as<float>(), 0.0f, W.p, ws, &idx, nullptr) == want);
  CHECK(idx == nullptr);
}

}  // namespace

int main() {
  std::mt19937_64 rng(20260601);

  // status strings and version
  for (int s = 0; s <= 6; ++s) CHECK(std::strncmp(epm_status_string((epm_status)s), "EPM_", 4) == 0);
  CHECK(std::strstr(epm_version(), "gfx950") != nullptr);

  // workspace sizes and the pair setup of many geometries: valid batches get
  // past the host and stop at the missing device
  for (int trial = 0; trial < 40; ++trial) {
    const Batch b = random_batch(rng, 1 + (int)(rng() % (trial < 4 ? 600 : 40)));
    check_build(b, EPM_ERR_HIP);
  }

  // degenerate F anywhere in the batch
  {
    Batch b = random_batch(rng, 5);
    const double zero[9] = {0}, rank1[9] = {1, 2, 3, 2, 4, 6, -1, -2, -3};
    double nan[9];
    for (double& v : nan) v = NAN;
    for (const double* F : {zero, rank1, (const double*)nan}) {
      Batch c = b;
      std::memcpy(c.pairs[2].F, F, sizeof(double) * 9);
      const size_t ws = epm_workspace_bytes(c.pairs.data(), 5);
      Buf W(ws ? ws : 1 << 20), kp2(8 * (size_t)c.n2 + 8);
      epm_index* idx = nullptr;
      CHECK(epm_build_intervals(c.pairs.data(), 5, kp2.as<float>(), nullptr, 2.0f, W.p,
                                ws ? ws : 1 << 20, &idx, nullptr) == EPM_ERR_DEGENERATE_F);
      CHECK(idx == nullptr);
    }
  }

  // argument errors of the build
  {
    Batch b = random_batch(rng, 3);
    const size_t ws = epm_workspace_bytes(b.pairs.data(), 3);
    Buf W(ws + 512), kp2(8 * (size_t)b.n2 + 8);
    epm_index* idx = nullptr;
    const epm_pair* P = b.pairs.data();
    CHECK(epm_build_intervals(P, 3, kp2.as<float>(), nullptr, 2.0f, W.p, ws, nullptr, nullptr) ==
          EPM_ERR_ARG);
    CHECK(epm_build_intervals(P, 3, kp2.as<float>(), nullptr, -1.0f, W.p, ws, &idx, nullptr) ==
          EPM_ERR_ARG);
    CHECK(epm_build_intervals(P, 3, kp2.as<float>(), nullptr, INFINITY, W.p, ws, &idx,
                              nullptr) == EPM_ERR_ARG);
    CHECK(epm_build_intervals(P, 3, kp2.as<float>(), nullptr, 2.0f, nullptr, ws, &idx,
                              nullptr) == EPM_ERR_WORKSPACE);
    CHECK(epm_build_intervals(P, 3, kp2.as<float>(), nullptr, 2.0f, W.as<char>() + 8, ws, &idx,
                              nullptr) == EPM_ERR_WORKSPACE);
    CHECK(epm_build_intervals(P, 3, kp2.as<float>(), nullptr, 2.0f, W.p, ws - 1, &idx,
                              nullptr) == EPM_ERR_WORKSPACE);
    CHECK(epm_build_intervals(nullptr, 3, kp2.as<float>(), nullptr, 2.0f, W.p, ws, &idx,
                              nullptr) == EPM_ERR_ARG);
    CHECK(epm_build_intervals(P, -1, kp2.as<float>(), nullptr, 2.0f, W.p, ws, &idx, nullptr) ==
          EPM_ERR_ARG);
    Batch c = b;
    c.pairs[1].q_begin += 1;  // slices not contiguous
    CHECK(epm_workspace_bytes(c.pairs.data(), 3) == 0);
    CHECK(epm_build_intervals(c.pairs.data(), 3, kp2.as<float>(), nullptr, 2.0f, W.p, ws, &idx,
                              nullptr) == EPM_ERR_ARG);
    c = b;
    c.pairs[0].w2 = 0;
    CHECK(epm_workspace_bytes(c.pairs.data(), 3) == 0);
    c = b;
    c.pairs[2].n = -5;
    CHECK(epm_workspace_bytes(c.pairs.data(), 3) == 0);
  }

  // calls on a missing index or batch
  {
    int64_t nnz = 0;
    Buf a(4096);
    CHECK(epm_query_candidates(nullptr, a.as<float>(), a.as<int64_t>(), a.as<int32_t>(), 10, &nnz,
                               nullptr) == EPM_ERR_ARG);
    CHECK(epm_match(nullptr, a.as<int64_t>(), a.as<int32_t>(), EPM_F32, 128, a.p, a.p, nullptr,
                    nullptr, nullptr, nullptr, 0.0f, a.as<int32_t>(), a.as<float>(),
                    a.as<float>(), nullptr, nullptr) == EPM_ERR_ARG);
    CHECK(epm_query_match(nullptr, a.as<float>(), a.as<int64_t>(), a.as<int32_t>(), 10, &nnz,
                          a.as<float>(), a.as<float>(), 0.0f, a.as<int32_t>(), a.as<float>(),
                          a.as<float>(), nullptr) == EPM_ERR_ARG);
    CHECK(epm_query_match_bf16(nullptr, a.as<float>(), a.as<int64_t>(), a.as<int32_t>(), 10,
                               &nnz, a.as<uint16_t>(), a.as<uint16_t>(), a.as<float>(),
                               a.as<float>(), 0.0f, a.as<int32_t>(), a.as<float>(), a.as<float>(),
                               nullptr) == EPM_ERR_ARG);
    CHECK(epm_query_match_fp8(nullptr, a.as<float>(), a.as<int64_t>(), a.as<int32_t>(), 10, &nnz,
                              a.as<uint8_t>(), a.as<float>(), a.as<float>(), a.as<float>(),
                              a.as<float>(), 0.0f, a.as<int32_t>(), a.as<float>(), a.as<float>(),
                              nullptr) == EPM_ERR_ARG);
    CHECK(epm_get_query_stats(nullptr, nullptr) == EPM_ERR_ARG);
    CHECK(epm_get_match_stats(nullptr, nullptr) == EPM_ERR_ARG);
    CHECK(epm_index_set_sched(nullptr, nullptr) == EPM_ERR_ARG);
    CHECK(epm_index_set_timing_events(nullptr, nullptr, nullptr) == EPM_ERR_ARG);
    CHECK(epm_mutual_check(nullptr, nullptr, nullptr, nullptr, nullptr) == EPM_ERR_ARG);
    CHECK(epm_gms(nullptr, nullptr, 20, 6.0f, nullptr, nullptr, nullptr, nullptr, nullptr, 0,
                  nullptr) == EPM_ERR_ARG);
    CHECK(epm_batch_launch(nullptr, nullptr) == EPM_ERR_ARG);
    CHECK(epm_batch_nnz(nullptr, &nnz, nullptr) == EPM_ERR_ARG);
    CHECK(epm_batch_index(nullptr) == nullptr);
    epm_batch_destroy(nullptr);
    epm_index_destroy(nullptr);
    CHECK(epm_point_line_terms(nullptr, nullptr, nullptr, nullptr, 0.0f, nullptr, nullptr, 5,
                               nullptr, nullptr, nullptr) == EPM_ERR_ARG);
    CHECK(epm_quantize(a.as<float>(), 4, 0, EPM_BF16, a.p, nullptr, nullptr) == EPM_ERR_ARG);
    CHECK(epm_quantize(a.as<float>(), 4, 128, EPM_F32, a.p, nullptr, nullptr) == EPM_ERR_ARG);
    CHECK(epm_quantize(a.as<float>(), 0, 128, EPM_BF16, a.p, nullptr, nullptr) == EPM_OK);
  }

  // batched graphs: a valid description reaches the device
  {
    Batch b = random_batch(rng, 24);
    const size_t ws = epm_workspace_bytes(b.pairs.data(), 24);
    Buf W(ws), kp1(8 * (size_t)b.n1 + 8), kp2(8 * (size_t)b.n2 + 8),
        d1(512 * (size_t)b.n1 + 512), d2(512 * (size_t)b.n2 + 512), ro(8 * (size_t)b.n1 + 8),
        ci(4 << 20), bi(4 * (size_t)b.n1 + 4), bd(4 * (size_t)b.n1 + 4), sd(4 * (size_t)b.n1 + 4);
    epm_batch_desc d;
    std::memset(&d, 0, sizeof(d));
    d.kp1_xy = kp1.as<float>();
    d.kp2_xy = kp2.as<float>();
    d.eps_scalar = 2.0f;
    d.row_offsets = ro.as<int64_t>();
    d.col_indices = ci.as<int32_t>();
    d.capacity = 1 << 20;
    d.dtype = EPM_F32;
    d.dim = 128;
    d.desc1 = d1.p;
    d.desc2 = d2.p;
    d.best_idx = bi.as<int32_t>();
    d.best_dist = bd.as<float>();
    d.second_dist = sd.as<float>();
    epm_batch* out = reinterpret_cast<epm_batch*>(0x1);
    CHECK(epm_batch_create(b.pairs.data(), 24, &d, W.p, ws, &out, nullptr) == EPM_ERR_HIP);
    CHECK(out == nullptr);
    d.dim = 64;  // descriptors are 128-dimensional
    out = reinterpret_cast<epm_batch*>(0x1);
    CHECK(epm_batch_create(b.pairs.data(), 24, &d, W.p, ws, &out, nullptr) == EPM_ERR_ARG);
    CHECK(out == nullptr);
  }

  // the allocation-free entry point: beyond its scratch, and a valid call
  {
    Batch b = random_batch(rng, 4);
    Buf kp1(8 * (size_t)b.n1 + 8), kp2(8 * (size_t)b.n2 + 8), d1(512 * (size_t)b.n1 + 512),
        d2(512 * (size_t)b.n2 + 512), ro(8 * (size_t)b.n1 + 8), ci(1 << 20),
        bi(4 * (size_t)b.n1 + 4), bd(4 * (size_t)b.n1 + 4), sd(4 * (size_t)b.n1 + 4);
    CHECK(epm_query_match_noalloc(b.pairs.data(), 4, kp1.as<float>(), kp2.as<float>(), nullptr,
                                  2.0f, ro.as<int64_t>(), ci.as<int32_t>(), 1 << 18, nullptr,
                                  d1.as<float>(), d2.as<float>(), 0.0f, bi.as<int32_t>(),
                                  bd.as<float>(), sd.as<float>(), nullptr) == EPM_ERR_HIP);
    Batch big;
    const double* F = b.pairs[0].F;
    for (int k = 0; k < 64; ++k) big.add(F, 6048, 4032, 1, 2000000);
    CHECK(epm_query_match_noalloc(big.pairs.data(), 64, kp1.as<float>(), kp2.as<float>(),
                                  nullptr, 2.0f, ro.as<int64_t>(), ci.as<int32_t>(), 1 << 18,
                                  nullptr, d1.as<float>(), d2.as<float>(), 0.0f,
                                  bi.as<int32_t>(), bd.as<float>(), sd.as<float>(),
                                  nullptr) == EPM_ERR_WORKSPACE);
  }

  // tolerance features and the pose-covariance tolerance: host tables
  {
    Batch b = random_batch(rng, 9);
    const int P = 9;
    Buf kp2(8 * (size_t)b.n2 + 8), attrs(12 * (size_t)b.n2 + 12), feat(24 * (size_t)b.n2 + 24),
        eps2(4 * (size_t)b.n2 + 4);
    const size_t wf = epm_eps_workspace_bytes(P);
    Buf W(wf);
    CHECK(epm_eps_features(b.pairs.data(), P, kp2.as<float>(), attrs.as<float>(),
                           feat.as<float>(), W.p, wf, nullptr) ==
          (b.n2 > 0 ? EPM_ERR_HIP : EPM_OK));
    CHECK(epm_eps_features(b.pairs.data(), P, kp2.as<float>(), attrs.as<float>(),
                           feat.as<float>(), W.p, wf - 1, nullptr) == EPM_ERR_WORKSPACE);
    std::vector<epm_pose_prior> pri(P);
    for (int p = 0; p < P; ++p) {
      epm_pose_prior& q = pri[p];
      std::memset(&q, 0, sizeof(q));
      const double f = 1000.0 + p;
      const double K[9] = {f, 0, 320, 0, f, 240, 0, 0, 1};
      std::memcpy(q.K1, K, sizeof(K));
      std::memcpy(q.K2, K, sizeof(K));
      rot(0.01 * p, -0.02, 0.005 * p, q.R);
      q.t[0] = 1.0; q.t[1] = 0.1 * p; q.t[2] = 0.05;
      for (int k = 0; k < 6; ++k) q.cov[7 * k] = 1e-4 * (k + 1);
      q.w1 = 640;
      q.h1 = 480;
      q.zmin = p % 2 ? 2.0 : 0.0;
      q.zmax = p % 3 ? 30.0 : INFINITY;
    }
    const size_t wp = epm_pose_eps_workspace_bytes(P);
    Buf WP(wp);
    CHECK(epm_pose_eps(b.pairs.data(), pri.data(), P, kp2.as<float>(), 2.0f, 3.0f, 100.0f,
                       eps2.as<float>(), WP.p, wp, nullptr) ==
          (b.n2 > 0 ? EPM_ERR_HIP : EPM_OK));
    std::vector<epm_pose_prior> bad = pri;
    bad[4].K1[0] = 0.0;
    bad[4].K1[4] = 0.0;  // singular intrinsics
    CHECK(epm_pose_eps(b.pairs.data(), bad.data(), P, kp2.as<float>(), 2.0f, 3.0f, 100.0f,
                       eps2.as<float>(), WP.p, wp, nullptr) == EPM_ERR_DEGENERATE_F);
    bad = pri;
    bad[6].cov[13] = NAN;
    CHECK(epm_pose_eps(b.pairs.data(), bad.data(), P, kp2.as<float>(), 2.0f, 3.0f, 100.0f,
                       eps2.as<float>(), WP.p, wp, nullptr) == EPM_ERR_DEGENERATE_F);
    bad = pri;
    bad[1].zmax = 1.0;  // zmax below zmin
    CHECK(epm_pose_eps(b.pairs.data(), bad.data(), P, kp2.as<float>(), 2.0f, 3.0f, 100.0f,
                       eps2.as<float>(), WP.p, wp, nullptr) == EPM_ERR_ARG);
    CHECK(epm_pose_eps(b.pairs.data(), pri.data(), P, kp2.as<float>(), 2.0f, 3.0f, 1.0f,
                       eps2.as<float>(), WP.p, wp, nullptr) == EPM_ERR_ARG);
    CHECK(epm_pose_eps(b.pairs.data(), pri.data(), P, kp2.as<float>(), 2.0f, 3.0f, 100.0f,
                       eps2.as<float>(), WP.as<char>() + 4, wp, nullptr) == EPM_ERR_WORKSPACE);
  }

  std::printf("libepm host checks passed\n");
  return 0;
}
