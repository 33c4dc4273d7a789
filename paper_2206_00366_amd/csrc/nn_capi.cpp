// C ABI of the warm-start surrogate kernels (declared in include/rmrt.h).
#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <string>

#include "../../include/rmrt.h"

namespace rmrt {
namespace nn {
hipError_t launch_conv(const uint16_t*, const uint16_t*, const float*, float*, uint16_t*, const float*, int, int, int,
                       int, int, int, int, hipStream_t);
hipError_t launch_flip(const uint16_t*, uint16_t*, int, int, hipStream_t);
size_t wgrad_partial_floats(long, int, int, int);
hipError_t launch_wgrad(const uint16_t*, const uint16_t*, int, int, int, int, int, int, float*, float*, float*, size_t,
                        hipStream_t);
hipError_t launch_mse(const float*, int, const float*, const float*, long, int, uint16_t*, double*, float*, double*,
                      hipStream_t);
hipError_t launch_adam(float*, uint16_t*, const float*, float*, float*, long, float, float, float, float, float, float,
                       hipStream_t);
hipError_t launch_to_bf16(const float*, uint16_t*, long, hipStream_t);
hipError_t launch_features(const uint8_t*, const float*, int, int, int, int, float, float, uint16_t*, int, float*,
                           hipStream_t);
hipError_t launch_targets(const double*, const double*, const uint8_t*, int, int, int, int, float, float, float, float*,
                          float*, hipStream_t);
hipError_t launch_warm_fields(const float*, int, int, int, int, int, float, float, float, const uint8_t*, double*,
                              double*, hipStream_t);
}  // namespace nn
}  // namespace rmrt

int rmrt_set_error_(int code, const char* msg);  // defined in rmrt_capi.cpp

namespace {
int nn_fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  return rmrt_set_error_(code, buf);
}
int hip_rc(hipError_t e, const char* what) {
  if (e == hipSuccess) return RMRT_OK;
  return nn_fail(RMRT_EHIP, "%s: %s", what, hipGetErrorString(e));
}
bool ch_ok(int c) { return c == 16 || c == 32; }
}  // namespace

using namespace rmrt::nn;

extern "C" {

int rmrt_nn_conv_forward(const void* x, const void* w, const float* bias, float* y_pre, void* a_out, const float* aux,
                         int B, int H, int W, int Cin, int Cout, int dil, int epilogue, void* stream) {
  if (!x || !w) return nn_fail(RMRT_EINVAL, "x and w are required");
  if (!ch_ok(Cin) || !ch_ok(Cout)) return nn_fail(RMRT_EUNSUPPORTED, "channels must be 16 or 32");
  if (B < 1 || H < 1 || W < 1 || dil < 1) return nn_fail(RMRT_EINVAL, "bad sizes");
  if (epilogue < 0 || epilogue > 2) return nn_fail(RMRT_EINVAL, "bad epilogue");
  if (epilogue == 2 && !aux) return nn_fail(RMRT_EINVAL, "epilogue 2 needs aux");
  if (!y_pre && !a_out) return nn_fail(RMRT_EINVAL, "no output");
  return hip_rc(launch_conv((const uint16_t*)x, (const uint16_t*)w, bias, y_pre, (uint16_t*)a_out, aux, B, H, W, Cin,
                            Cout, dil, epilogue, (hipStream_t)stream),
                "conv launch");
}

int rmrt_nn_flip_weights(const void* w, void* wt, int Cout, int Cin, void* stream) {
  if (!w || !wt) return nn_fail(RMRT_EINVAL, "NULL pointer");
  if (!ch_ok(Cin) || !ch_ok(Cout)) return nn_fail(RMRT_EUNSUPPORTED, "channels must be 16 or 32");
  return hip_rc(launch_flip((const uint16_t*)w, (uint16_t*)wt, Cout, Cin, (hipStream_t)stream), "flip launch");
}

size_t rmrt_nn_wgrad_scratch_floats(int B, int H, int W, int Cin, int Cout) {
  const size_t a = wgrad_partial_floats((long)B * H * W, Cin, Cout, 1024);
  const size_t b = (size_t)1024 * Cout;
  return a > b ? a : b;
}

int rmrt_nn_conv_backward_weight(const void* x, const void* dy, int B, int H, int W, int Cin, int Cout, int dil,
                                 float* dw, float* db, float* scratch, size_t scratch_floats, void* stream) {
  if (!x || !dy || !dw || !scratch) return nn_fail(RMRT_EINVAL, "NULL pointer");
  if (!ch_ok(Cin) || !ch_ok(Cout)) return nn_fail(RMRT_EUNSUPPORTED, "channels must be 16 or 32");
  if (scratch_floats < rmrt_nn_wgrad_scratch_floats(B, H, W, Cin, Cout))
    return nn_fail(RMRT_EINVAL, "scratch too small");
  return hip_rc(launch_wgrad((const uint16_t*)x, (const uint16_t*)dy, B, H, W, Cin, Cout, dil, dw, db, scratch,
                             scratch_floats, (hipStream_t)stream),
                "wgrad launch");
}

int rmrt_nn_masked_mse(const float* out, int out_stride, const float* target, const float* weight, long P, int C,
                       void* dout, double* scratch, float* inv_den, double* loss, void* stream) {
  if (!out || !target || !weight || !dout || !scratch || !inv_den || !loss) return nn_fail(RMRT_EINVAL, "NULL pointer");
  if (C < 1 || C > out_stride || P < 1) return nn_fail(RMRT_EINVAL, "bad sizes");
  return hip_rc(launch_mse(out, out_stride, target, weight, P, C, (uint16_t*)dout, scratch, inv_den, loss,
                           (hipStream_t)stream),
                "mse launch");
}

int rmrt_nn_adam(float* w, void* w_bf16, const float* g, float* m, float* v, long n, float lr, float b1, float b2,
                 float eps, int t, void* stream) {
  if (!w || !g || !m || !v || n < 1 || t < 1) return nn_fail(RMRT_EINVAL, "bad arguments");
  const float c1 = 1.f - powf(b1, (float)t), c2 = 1.f - powf(b2, (float)t);
  return hip_rc(launch_adam(w, (uint16_t*)w_bf16, g, m, v, n, lr, b1, b2, eps, c1, c2, (hipStream_t)stream),
                "adam launch");
}

int rmrt_nn_to_bf16(const float* src, void* dst, long n, void* stream) {
  if (!src || !dst || n < 0) return nn_fail(RMRT_EINVAL, "bad arguments");
  if (n == 0) return RMRT_OK;
  return hip_rc(launch_to_bf16(src, (uint16_t*)dst, n, (hipStream_t)stream), "bf16 launch");
}

int rmrt_nn_features(const uint8_t* solid, const float* re, int B, int nx, int ny, int k, float dy, float re_scale,
                     void* x0, int channels, float* scratch, void* stream) {
  if (!solid || !re || !x0 || !scratch) return nn_fail(RMRT_EINVAL, "NULL pointer");
  if (k < 1 || nx % k || ny % k || channels < 5) return nn_fail(RMRT_EINVAL, "bad sizes");
  return hip_rc(launch_features(solid, re, B, nx, ny, k, dy, re_scale, (uint16_t*)x0, channels, scratch,
                                (hipStream_t)stream),
                "features launch");
}

int rmrt_nn_targets(const double* rho, const double* u, const uint8_t* solid, int B, int nx, int ny, int k, float dy,
                    float Ut, float rho_scale, float* tgt, float* wgt, void* stream) {
  if (!rho || !u || !solid || !tgt || !wgt) return nn_fail(RMRT_EINVAL, "NULL pointer");
  if (k < 1 || nx % k || ny % k) return nn_fail(RMRT_EINVAL, "bad sizes");
  return hip_rc(launch_targets(rho, u, solid, B, nx, ny, k, dy, Ut, rho_scale, tgt, wgt, (hipStream_t)stream),
                "targets launch");
}

int rmrt_nn_warm_fields(const float* out, int out_stride, int B, int nx, int ny, int k, float dy, float Ut,
                        float rho_scale, const uint8_t* solid, double* rho, double* u, void* stream) {
  if (!out || !rho || !u) return nn_fail(RMRT_EINVAL, "NULL pointer");
  if (k < 1 || nx % k || ny % k || out_stride < 3) return nn_fail(RMRT_EINVAL, "bad sizes");
  return hip_rc(launch_warm_fields(out, out_stride, B, nx, ny, k, dy, Ut, rho_scale, solid, rho, u, (hipStream_t)stream),
                "warm fields launch");
}

}  // extern "C"
