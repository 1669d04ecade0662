// Learned refinement tagger: launchers shared by the host core (gf_host.cpp)
// and the kernels (gf_net.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gfnet {

// parameter vector layout (float): W1[16][3][3][4] b1[16] W2[32][3][3][16] b2[32]
// W3[32][3][3][32] b3[32] Wf[3][32] bf[3]
constexpr int OFF_W1 = 0, OFF_B1 = 576, OFF_W2 = 592, OFF_B2 = 5200, OFF_W3 = 5232, OFF_B3 = 14448;
constexpr int OFF_WF = 14480, OFF_BF = 14576, N_PARAMS = 14579;
constexpr int TILE = 24, CIN = 4, FEAT = TILE * TILE * CIN;   // 2304 feature values per patch

struct NetArgs {
    const float *x;          // [n][FEAT] features (rounded to bf16 in the kernel), or null
    const uint16_t *xb;      // [rows][FEAT] bf16 features, used when x is null
    int n;
    const float *w;          // FP32 parameters
    const uint16_t *wb;      // bf16 copies (conv weights read from here)
    float *logits;           // [n][3]
    // training only
    const int8_t *y;         // class 0 (coarsen), 1 (keep), 2 (refine)
    float cw[3];             // class weights
    float wtot;              // sum over the batch of cw[y]
    const float *wtot_dev;   // the same sum in device memory, used when not null
    float *loss_i;           // [n] per-sample loss contributions
    float *part;             // [n][N_PARAMS] per-sample gradients
};

// One pixel source of the feature images: a leaf-slot map per level.
struct FeatLevel {
    int64_t map_off;         // offset of the level's slot map (mj 2^l rows x mi 2^l columns)
    int32_t map_w;           // patches per row at this level
    int64_t img_off;         // offset of the level's image: 4 channels x ny x nx floats
    int32_t nx, ny;          // pixels (8 per patch side)
};

}  // namespace gfnet

hipError_t gfnet_launch_forward(const gfnet::NetArgs &a, hipStream_t s);
hipError_t gfnet_launch_train(const gfnet::NetArgs &a, hipStream_t s);
hipError_t gfnet_launch_reduce(const float *part, int n, float *grad, hipStream_t s);
// class-weight sum of a batch whose labels are in device memory (labels
// outside 0..2 count 0)
hipError_t gfnet_launch_weight_sum(const int8_t *y, int n, float c0, float c1, float c2, float *wtot, hipStream_t s);
hipError_t gfnet_launch_adam(float *w, float *m, float *v, uint16_t *wb, const float *g, float lr, float bc1, float bc2,
                             hipStream_t s);
hipError_t gfnet_launch_to_bf16(const float *w, uint16_t *wb, int n, hipStream_t s);
// finest feature image of one scenario from its leaves (state in float or double)
hipError_t gfnet_launch_image_f32(const float *q, const float *b, int64_t cap, int m, const int32_t *map,
                                  const gfnet::FeatLevel *lv_dev, const gfnet::FeatLevel &finest, int Lf, float *img,
                                  hipStream_t s);
hipError_t gfnet_launch_image_f64(const double *q, const double *b, int64_t cap, int m, const int32_t *map,
                                  const gfnet::FeatLevel *lv_dev, const gfnet::FeatLevel &finest, int Lf, float *img,
                                  hipStream_t s);
hipError_t gfnet_launch_pyramid(const float *fine, int fnx, int fny, float *coarse, int cnx, int cny, hipStream_t s);
// tiles of n leaves: level, global patch indices, image of that level
hipError_t gfnet_launch_tiles(const float *img, const gfnet::FeatLevel *lv_dev, const int32_t *leaf_lij, int n,
                              float *featf, uint16_t *featb, hipStream_t s);
