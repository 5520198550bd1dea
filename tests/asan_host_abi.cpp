// Host-side AddressSanitizer driver for the C ABI (built by
// tests/test_asan_host.py with the sanitizer on the host compilation only; no
// GPU is touched).  It runs the library's host-only routines -- pose k-means
// and its default normaliser, the segment partition, cluster selection and
// active segments (Sec. 3.3 "Offline Clustering" / "Algorithm"), pose
// extrapolation and resident-set planning (Sec. 3.3 "Scene Prefetching"),
// tile counts and workspace sizes -- on randomised inputs held in heap
// buffers of exactly the documented sizes, so any read or write past a
// buffer, use after free or leak in that host code stops the run.  It also
// drives the argument validation of the device entry points with inputs that
// must be rejected before anything is enqueued.  Results are checked for the
// invariants the header states; parity with the float64 oracle is covered by
// the Python ABI tests.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <random>
#include <vector>

#include "seele.h"

namespace {

int g_fail = 0;

#define CHECK(cond)                                                              \
  do {                                                                           \
    if (!(cond)) {                                                               \
      std::fprintf(stderr, "%s:%d: check failed: %s\n", __FILE__, __LINE__, #cond); \
      ++g_fail;                                                                  \
    }                                                                            \
  } while (0)

// Heap array of exactly n elements (never a zero-size allocation).
template <typename T>
std::unique_ptr<T[]> arr(size_t n) {
  return std::unique_ptr<T[]>(new T[n > 0 ? n : 1]());
}

seele_camera look_at(double cx, double cy, double cz, int w, int h) {
  double f[3] = {-cx, -cy, -cz};
  const double fn = std::sqrt(f[0] * f[0] + f[1] * f[1] + f[2] * f[2]);
  for (double& v : f) v /= fn;
  const double up[3] = {0.0, -1.0, 0.0};
  double x[3] = {f[1] * up[2] - f[2] * up[1], f[2] * up[0] - f[0] * up[2],
                 f[0] * up[1] - f[1] * up[0]};
  const double xn = std::sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
  for (double& v : x) v /= xn;
  const double y[3] = {f[1] * x[2] - f[2] * x[1], f[2] * x[0] - f[0] * x[2],
                       f[0] * x[1] - f[1] * x[0]};
  seele_camera c{};
  for (int i = 0; i < 3; ++i) {
    c.R[i] = (float)x[i];
    c.R[3 + i] = (float)y[i];
    c.R[6 + i] = (float)f[i];
  }
  const double C[3] = {cx, cy, cz};
  for (int r = 0; r < 3; ++r)
    c.t[r] = (float)-(c.R[3 * r] * C[0] + c.R[3 * r + 1] * C[1] + c.R[3 * r + 2] * C[2]);
  c.fx = c.fy = (float)(w / 2.0 / std::tan(M_PI / 6.0));
  c.cx = w / 2.0f;
  c.cy = h / 2.0f;
  c.width = w;
  c.height = h;
  return c;
}

void test_kmeans_select_segments(std::mt19937& rng) {
  std::uniform_real_distribution<double> u(-1.0, 1.0);
  for (int trial = 0; trial < 40; ++trial) {
    const int n = 1 + (int)(rng() % 70);
    auto cams = arr<seele_camera>(n);
    for (int i = 0; i < n; ++i) {
      double d[3] = {u(rng), 0.3 * u(rng), u(rng)};
      const double r = 2.0 + 3.0 * (0.5 + 0.5 * u(rng));
      const double dn = std::sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]) + 1e-9;
      cams[i] = look_at(r * d[0] / dn, r * d[1] / dn, r * d[2] / dn, 64, 48);
    }
    const float ps = seele_hp_pos_scale(cams.get(), n);
    CHECK(ps > 0.0f);
    const int K = 1 + (int)(rng() % n);
    auto cents = arr<float>((size_t)K * 6);
    auto labels = arr<int32_t>(n);
    const float pos_scale = (trial % 2) ? 0.0f : ps;
    CHECK(seele_hp_kmeans(cams.get(), n, pos_scale, 1.0f, K, 50, cents.get(), labels.get()) ==
          SEELE_OK);
    for (int i = 0; i < n; ++i) CHECK(labels[i] >= 0 && labels[i] < K);
    const int M = (int)(rng() % K);
    auto clusters = arr<int32_t>(1 + M);
    CHECK(seele_hp_select(cents.get(), K, &cams[0], ps, 1.0f, M, clusters.get()) == SEELE_OK);
    for (int i = 0; i <= M; ++i) CHECK(clusters[i] >= 0 && clusters[i] < K);
    // a layout over K clusters, some empty
    auto lb = arr<int64_t>(1 + K);
    auto lc = arr<int64_t>(1 + K);
    int64_t at = 0;
    for (int s = 0; s <= K; ++s) {
      lb[s] = at;
      lc[s] = (rng() % 4 == 0) ? 0 : (int64_t)(rng() % 1000);
      at += lc[s];
    }
    auto ob = arr<int64_t>(2 + M);
    auto oc = arr<int64_t>(2 + M);
    int32_t n_out = -1;
    CHECK(seele_hp_segments(lb.get(), lc.get(), K, clusters.get(), 1 + M, ob.get(), oc.get(),
                            &n_out) == SEELE_OK);
    CHECK(n_out >= 0 && n_out <= 2 + M);
    for (int i = 1; i < n_out; ++i) CHECK(ob[i] > ob[i - 1]);
    // rejected: M too large, cluster out of range, null outputs
    CHECK(seele_hp_select(cents.get(), K, &cams[0], ps, 1.0f, K, clusters.get()) != SEELE_OK);
    clusters[0] = K;
    CHECK(seele_hp_segments(lb.get(), lc.get(), K, clusters.get(), 1, ob.get(), oc.get(),
                            &n_out) != SEELE_OK);
    CHECK(seele_hp_kmeans(cams.get(), n, 1.0f, 1.0f, n + 1, 5, cents.get(), labels.get()) !=
          SEELE_OK);
    CHECK(seele_hp_kmeans(cams.get(), n, NAN, 1.0f, 1, 5, cents.get(), labels.get()) != SEELE_OK);
  }
}

void test_partition(std::mt19937& rng) {
  for (int trial = 0; trial < 40; ++trial) {
    const int64_t n = (int64_t)(rng() % 500);
    const int K = 1 + (int)(rng() % 9);
    auto shared = arr<uint8_t>(n);
    auto best = arr<float>(n);
    auto bc = arr<int32_t>(n);
    for (int64_t i = 0; i < n; ++i) {
      shared[i] = rng() % 5 == 0;
      best[i] = (rng() % 3 == 0) ? 0.0f : (float)(rng() % 100) / 7.0f;
      bc[i] = (int32_t)(rng() % (K + 2)) - 1;  // -1 .. K (K is not a cluster)
    }
    auto perm = arr<int64_t>(n);
    auto b = arr<int64_t>(1 + K);
    auto c = arr<int64_t>(1 + K);
    CHECK(seele_hp_partition(shared.get(), best.get(), bc.get(), n, K, perm.get(), b.get(),
                             c.get()) == SEELE_OK);
    std::vector<int> seen((size_t)n, 0);
    for (int64_t i = 0; i < n; ++i) {
      CHECK(perm[i] >= 0 && perm[i] < n);
      if (perm[i] >= 0 && perm[i] < n) ++seen[(size_t)perm[i]];
    }
    for (int64_t i = 0; i < n; ++i) CHECK(seen[(size_t)i] == 1);
    int64_t tot = 0;
    for (int s = 0; s <= K; ++s) {
      CHECK(b[s] == tot);
      tot += c[s];
    }
    CHECK(tot <= n);
  }
}

void test_prefetch(std::mt19937& rng) {
  std::uniform_real_distribution<float> u(-1.0f, 1.0f);
  for (int trial = 0; trial < 30; ++trial) {
    seele_camera a = look_at(4.0 * u(rng), u(rng), 4.0 + u(rng), 320, 200);
    seele_camera b = look_at(4.0 * u(rng), u(rng), 4.0 + u(rng), 320, 200);
    seele_camera out{};
    CHECK(seele_pose_extrapolate(&a, &b, 0.5f + u(rng), &out) == SEELE_OK);
    CHECK(out.width == b.width && out.height == b.height);
    const int K = 2 + (int)(rng() % 10);
    const int n_slots = 1 + (int)(rng() % 6);
    auto cc = arr<int64_t>(K);
    int64_t cap = 0;
    for (int k = 0; k < K; ++k) {
      cc[k] = (int64_t)(rng() % 100);
      cap = std::max(cap, cc[k]);
    }
    auto slot_c = arr<int32_t>(n_slots);
    auto slot_s = arr<int64_t>(n_slots);
    for (int s = 0; s < n_slots; ++s) {
      slot_c[s] = -1;
      slot_s[s] = 0;
    }
    auto lcl = arr<int32_t>(n_slots);
    auto lsl = arr<int32_t>(n_slots);
    for (int64_t frame = 1; frame <= 25; ++frame) {
      const int n_need = 1 + (int)(rng() % n_slots);
      const int n_want = (int)(rng() % (K + 1));
      auto need = arr<int32_t>(n_need);
      auto want = arr<int32_t>(n_want);
      // distinct needed clusters (at most n_slots of them)
      for (int i = 0; i < n_need; ++i) need[i] = (int32_t)((frame + 3 * i) % K);
      for (int i = 0; i < n_want; ++i) want[i] = (int32_t)(rng() % K);
      int32_t n_loads = -1, n_demand = -1;
      const int32_t st = seele_resident_plan(slot_c.get(), slot_s.get(), n_slots, cc.get(), K, cap,
                                             need.get(), n_need, want.get(), n_want, frame,
                                             lcl.get(), lsl.get(), &n_loads, &n_demand);
      if (st == SEELE_OK) {
        CHECK(n_loads >= 0 && n_loads <= n_slots && n_demand >= 0 && n_demand <= n_loads);
        for (int i = 0; i < n_loads; ++i) CHECK(lsl[i] >= 0 && lsl[i] < n_slots);
      }
    }
    // rejected: a cluster larger than a slot, an out-of-range need
    int32_t bad = K;
    int32_t nl = 0, nd = 0;
    CHECK(seele_resident_plan(slot_c.get(), slot_s.get(), n_slots, cc.get(), K, cap, &bad, 1,
                              nullptr, 0, 99, lcl.get(), lsl.get(), &nl, &nd) != SEELE_OK);
  }
}

void test_sizes_and_validation(std::mt19937& rng) {
  for (int trial = 0; trial < 30; ++trial) {
    const int V = 1 + (int)(rng() % 9);
    auto cams = arr<seele_camera>(V);
    for (int v = 0; v < V; ++v)
      cams[v] = look_at(0.0, 0.0, -3.0 - v, 1 + (int)(rng() % 2000), 1 + (int)(rng() % 1200));
    for (int tile : {8, 16}) {
      CHECK(seele_total_tiles(cams.get(), V, tile) > 0);
      CHECK(seele_total_super_tiles(cams.get(), V, tile) > 0);
    }
    CHECK(seele_total_tiles(cams.get(), V, 12) < 0);
    CHECK(seele_photometric_loss_workspace_size(cams.get(), V) > 0);
    CHECK(seele_flip_loss_workspace_size(cams.get(), V) > 0);
    CHECK(seele_bin_sort_workspace_size(1000, 5000, 64) > 0);
    CHECK(seele_raster_queue_workspace_size(1000) > 0);
    CHECK(seele_spatial_order_workspace_size(1000) > 0);
    // device entry points: arguments rejected on the host before any launch
    seele_preprocess_opts po{};
    po.tile = 7;  // not 8 or 16
    po.alpha_min = 1.0f / 255.0f;
    po.lowpass = 0.3f;
    po.z_near = 0.2f;
    seele_gaussians g{};
    g.n = 10;
    CHECK(seele_preprocess(&g, cams.get(), V, &po, nullptr, nullptr, nullptr) != SEELE_OK);
    seele_raster_opts ro{};
    ro.tile = 16;
    ro.mode = 5;  // unknown
    CHECK(seele_rasterize_fwd(nullptr, nullptr, nullptr, cams.get(), V, &ro, nullptr, nullptr,
                              nullptr, nullptr) != SEELE_OK);
    CHECK(seele_bin_sort(nullptr, nullptr, -1, cams.get(), V, 16, nullptr, 0, nullptr, 0, nullptr,
                         nullptr, nullptr) != SEELE_OK);
    CHECK(seele_photometric_loss(nullptr, nullptr, cams.get(), V, 0.2f, nullptr, 0, nullptr,
                                 nullptr, nullptr) != SEELE_OK);
    CHECK(seele_flip_loss(nullptr, nullptr, cams.get(), V, 67.0f, 1.0f, 0, nullptr, 0, nullptr,
                          nullptr, nullptr) != SEELE_OK);
    CHECK(std::strlen(seele_last_error()) > 0);
  }
  for (int s = -1; s <= 5; ++s) CHECK(seele_status_string(s) != nullptr);
}

}  // namespace

int main() {
  std::mt19937 rng(12345);
  test_kmeans_select_segments(rng);
  test_partition(rng);
  test_prefetch(rng);
  test_sizes_and_validation(rng);
  std::printf("asan host ABI driver: %d failed checks\n", g_fail);
  return g_fail == 0 ? 0 : 1;
}
