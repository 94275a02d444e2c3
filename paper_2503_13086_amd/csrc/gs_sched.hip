// Host-side schedule of progressive training (Sec. IV-C and IV-D): hierarchical
// image weights (Eq. 3-4), the per-arrival iteration plan (Eq. 5 for the local
// half, an even spread for the semi-global half) and the per-image learning rate
// (Eq. 6-8).  Plain C++ on host arrays; no device work.  The floating-point
// evaluation order is fixed (documented per function) so results are reproducible.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <numeric>
#include <vector>

#include "gs.h"

namespace {

bool bad_overlap(const double* M, int32_t n) {
  for (int64_t k = 0; k < (int64_t)n * n; ++k)
    if (!(M[k] >= 0.0) || std::isinf(M[k])) return true;   // rejects negatives and NaN
  return false;
}

}  // namespace

extern "C" {

gs_status gs_sched_weights(const double* overlap, int32_t n, int32_t new_image, double* weights,
                           int32_t* layer) {
  if (n <= 0 || !overlap || !weights || new_image < 0 || new_image >= n) return GS_ERR_INVALID;
  if (bad_overlap(overlap, n)) return GS_ERR_INVALID;
  std::vector<int32_t> lay(n, 0);
  for (int32_t i = 0; i < n; ++i) weights[i] = -1.0;
  weights[new_image] = 1.0;
  lay[new_image] = 1;
  std::vector<int32_t> prev{new_image}, next;
  for (int32_t k = 2; !prev.empty(); ++k) {
    next.clear();
    for (int32_t i = 0; i < n; ++i) {
      if (lay[i]) continue;
      bool linked = false;
      for (int32_t j : prev) linked = linked || overlap[(int64_t)j * n + i] > 0.0;
      if (linked) next.push_back(i);
    }
    // Eq. 4 (Eq. 3 is its first layer, where the previous layer is the new image
    // alone with weight 1): mean over the previous layer of weight times overlap,
    // summed in ascending image order.
    for (int32_t i : next) {
      double s = 0.0;
      for (int32_t j : prev) s += weights[j] * overlap[(int64_t)j * n + i];
      weights[i] = s / (double)prev.size();
    }
    for (int32_t i : next) lay[i] = k;
    prev.swap(next);
  }
  if (layer) std::memcpy(layer, lay.data(), sizeof(int32_t) * n);
  return GS_OK;
}

gs_status gs_sched_plan(const double* weights, int32_t n, int32_t n_m, int32_t t_i, const double* u,
                        int32_t* plan, int32_t* local_iters) {
  if (n <= 0 || !weights || !u || !plan || n_m < 1 || t_i < 0) return GS_ERR_INVALID;
  for (int32_t i = 0; i < n; ++i)
    if (std::isnan(weights[i]) || std::isnan(u[i])) return GS_ERR_INVALID;
  // key images: the n_m largest weights among the reached images (weight >= 0),
  // ties by the smaller index
  std::vector<int32_t> cand;
  for (int32_t i = 0; i < n; ++i)
    if (weights[i] >= 0.0) cand.push_back(i);
  std::stable_sort(cand.begin(), cand.end(), [&](int32_t a, int32_t b) { return weights[a] > weights[b]; });
  if ((int32_t)cand.size() > n_m) cand.resize(n_m);
  std::vector<int32_t> share(n, 0);
  const int32_t half = t_i / 2;
  double tot = 0.0;
  for (int32_t i : cand) tot += 1.0 - std::exp(-weights[i]);
  int32_t n_local = 0;
  if (tot > 0.0 && half > 0) {
    // Eq. 5 shares, rounded by largest remainder (ties by the smaller index) so
    // they sum to exactly t_i / 2
    std::vector<double> exact(n, 0.0);
    int32_t assigned = 0;
    for (int32_t i : cand) {
      exact[i] = (1.0 - std::exp(-weights[i])) / (2.0 * tot) * (double)t_i;
      share[i] = (int32_t)std::floor(exact[i]);
      assigned += share[i];
    }
    std::vector<int32_t> byrem(cand);
    std::sort(byrem.begin(), byrem.end(), [&](int32_t a, int32_t b) {
      const double ra = exact[a] - share[a], rb = exact[b] - share[b];
      return ra != rb ? ra > rb : a < b;
    });
    for (int32_t k = 0; k < half - assigned && k < (int32_t)byrem.size(); ++k) share[byrem[k]] += 1;
    // local half: round robin over the key images in weight order while budget remains
    std::vector<int32_t> left(share);
    while (n_local < half) {
      bool any = false;
      for (int32_t i : cand) {
        if (left[i] > 0 && n_local < half) {
          plan[n_local++] = i;
          --left[i];
          any = true;
        }
      }
      if (!any) break;
    }
  }
  // semi-global half: the images outside the key set (all images when every image
  // is a key image) ordered by the caller's uniform draws u (ties by index), used
  // cyclically: an even spread, and a draw without replacement when there are more
  // images than iterations
  std::vector<char> is_key(n, 0);
  for (int32_t i : cand) is_key[i] = 1;
  std::vector<int32_t> other;
  for (int32_t i = 0; i < n; ++i)
    if (!is_key[i]) other.push_back(i);
  if (other.empty()) {
    other.resize(n);
    std::iota(other.begin(), other.end(), 0);
  }
  std::stable_sort(other.begin(), other.end(), [&](int32_t a, int32_t b) { return u[a] < u[b]; });
  for (int32_t k = 0; n_local + k < t_i; ++k) plan[n_local + k] = other[k % other.size()];
  if (local_iters) std::memcpy(local_iters, share.data(), sizeof(int32_t) * n);
  return GS_OK;
}

gs_status gs_sched_lr(const int64_t* trained, const double* overlap, int32_t n, double eta0, double etaf,
                      double t_a, double* lr_current, double* lr) {
  if (n <= 0 || !trained || !overlap || !lr || !(eta0 > 0.0) || !(etaf > 0.0) || !(t_a > 0.0))
    return GS_ERR_INVALID;
  if (bad_overlap(overlap, n)) return GS_ERR_INVALID;
  std::vector<double> c(n);
  const double l0 = std::log(eta0), lf = std::log(etaf);
  for (int32_t j = 0; j < n; ++j) {
    if (trained[j] < 0) return GS_ERR_INVALID;
    // Eq. 7: progress capped at 1; Eq. 6: log-linear between eta0 and etaf
    const double t = (double)trained[j] > t_a ? 1.0 : (double)trained[j] / t_a;
    c[j] = std::exp(l0 * (1.0 - t) + lf * t);
  }
  for (int32_t j = 0; j < n; ++j) {
    // Eq. 8: own rate plus overlap-weighted rates of the overlapping images, over
    // their count plus one (neighbour terms summed first, in ascending order)
    double s = 0.0;
    int32_t cnt = 0;
    for (int32_t i = 0; i < n; ++i) {
      const double m = overlap[(int64_t)i * n + j];
      if (i != j && m > 0.0) {
        s += m * c[i];
        ++cnt;
      }
    }
    lr[j] = (c[j] + s) / (double)(cnt + 1);
  }
  if (lr_current) std::memcpy(lr_current, c.data(), sizeof(double) * n);
  return GS_OK;
}

}  // extern "C"
