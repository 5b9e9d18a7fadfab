// Host side of the prefetch predictor's data path: pose features, the
// union-of-cameras Level-1 bitset used both for logging training pairs and
// for judging predictions, and the block sphere of a parameter sample.
#include <cstring>

#include "blocks.h"
#include "common.h"

using namespace tide;

extern "C" tide_status tide_pose_features(const tide_camera* cams, int32_t n_poses, double t_scale, float* out) {
  TIDE_CHECK_ARG(cams && out, "null argument");
  TIDE_CHECK_ARG(n_poses >= 1, "n_poses must be positive");
  TIDE_CHECK_ARG(t_scale > 0, "t_scale must be positive");
  double prev[3] = {0, 0, 0};
  for (int p = 0; p < n_poses; ++p) {
    const tide_camera& c = cams[p];
    float* o = out + 14 * (size_t)p;
    for (int i = 0; i < 9; ++i) o[i] = (float)c.R[i];
    for (int i = 0; i < 3; ++i) o[9 + i] = (float)(c.t[i] / t_scale);
    // camera centre: -R^T t
    double e[3];
    for (int i = 0; i < 3; ++i) e[i] = -(c.R[i] * c.t[0] + c.R[3 + i] * c.t[1] + c.R[6 + i] * c.t[2]);
    o[12] = p ? (float)(e[0] - prev[0]) : 0.0f;
    o[13] = p ? (float)(e[1] - prev[1]) : 0.0f;
    std::memcpy(prev, e, sizeof(e));
  }
  return TIDE_OK;
}

extern "C" tide_status tide_cull_bits(const float* spheres, int64_t n_blocks, const tide_camera* cams, int32_t n_cams,
                                      uint32_t* out, int64_t n_words) {
  TIDE_CHECK_ARG(spheres && cams && out, "null argument");
  TIDE_CHECK_ARG(n_cams >= 1 && n_cams <= TIDE_MAX_CAMS, "bad n_cams");
  TIDE_CHECK_ARG(n_blocks >= 0 && n_words * 32 >= n_blocks, "n_words %lld too small for %lld blocks",
                 (long long)n_words, (long long)n_blocks);
  std::memset(out, 0, sizeof(uint32_t) * (size_t)n_words);
  for (int ci = 0; ci < n_cams; ++ci) {
    const CullCam cc(cams[ci]);
    for (int64_t k = 0; k < n_blocks; ++k)
      if (cc.keep(spheres + 4 * k)) out[k >> 5] |= 1u << (k & 31);
  }
  return TIDE_OK;
}

extern "C" tide_status tide_block_sphere(const float* params, int64_t ld, int64_t rows, double kappa, float* out) {
  TIDE_CHECK_ARG(params && out, "null argument");
  TIDE_CHECK_ARG(rows >= 1 && rows <= ld, "need 1 <= rows <= ld");
  block_sphere(params, ld, rows, kappa, out);
  return TIDE_OK;
}
