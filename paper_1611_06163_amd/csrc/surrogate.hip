// surrogate.hip -- host side of the membrane-surrogate network behind the C
// ABI (tdpd_mlp_*): parameters and Adam state on the device, forward pass,
// loss gradient and training steps built from the kernels of
// kernels_surrogate.hip.
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "launch.h"
#include "../../include/tdpd.h"

using namespace tdpd;

struct tdpd_mlp {
  hipStream_t st = nullptr;
  tdpd_alloc_fn alloc = nullptr;
  tdpd_free_fn free_fn = nullptr;
  void *user = nullptr;
  std::string err;
  std::vector<void *> blocks;
  float *params = nullptr, *grad = nullptr, *m = nullptr, *v = nullptr;
  int64_t adam_t = 0;
  // per-batch buffers, sized for cap rows
  int64_t cap = 0;
  float *X = nullptr, *T = nullptr, *Z[3] = {}, *H[3] = {}, *Y = nullptr, *dY = nullptr;
  float *dA = nullptr, *dB = nullptr;
  double *part = nullptr, *loss = nullptr;

  int fail(int code, const std::string &msg) {
    err = msg;
    return code;
  }
  void *dalloc(size_t bytes) {
    bytes = (bytes + 255) & ~size_t(255);
    if (bytes == 0) bytes = 256;
    void *p = nullptr;
    if (alloc) p = alloc(bytes, user);
    else if (hipMalloc(&p, bytes) != hipSuccess) p = nullptr;
    if (p) blocks.push_back(p);
    return p;
  }
  void dfree(void *p) {
    if (!p) return;
    for (size_t i = 0; i < blocks.size(); ++i)
      if (blocks[i] == p) {
        blocks.erase(blocks.begin() + long(i));
        break;
      }
    if (free_fn) free_fn(p, user);
    else if (!alloc) (void)hipFree(p);
  }
};

#define MLPCHK(call)                                                                    \
  do {                                                                                  \
    hipError_t e_ = (call);                                                             \
    if (e_ != hipSuccess)                                                               \
      return m->fail(TDPD_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_));  \
  } while (0)

namespace {

// (re)size the per-batch buffers for n rows
int ensure_cap(tdpd_mlp *m, int64_t n) {
  if (n <= m->cap) return TDPD_OK;
  MLPCHK(hipStreamSynchronize(m->st));
  void *old[] = {m->X, m->T, m->Z[0], m->Z[1], m->Z[2], m->H[0], m->H[1], m->H[2],
                 m->Y, m->dY, m->dA, m->dB, m->part, m->loss};
  for (void *p : old) m->dfree(p);
  const size_t h = sizeof(float) * size_t(n) * kSurrHid;
  m->X = static_cast<float *>(m->dalloc(sizeof(float) * size_t(n) * kSurrIn));
  m->T = static_cast<float *>(m->dalloc(sizeof(float) * size_t(n) * kSurrOut));
  for (int l = 0; l < 3; ++l) {
    m->Z[l] = static_cast<float *>(m->dalloc(h));
    m->H[l] = static_cast<float *>(m->dalloc(h));
  }
  m->Y = static_cast<float *>(m->dalloc(sizeof(float) * size_t(n) * kSurrOut));
  m->dY = static_cast<float *>(m->dalloc(sizeof(float) * size_t(n) * kSurrOut));
  m->dA = static_cast<float *>(m->dalloc(h));
  m->dB = static_cast<float *>(m->dalloc(h));
  m->part = static_cast<double *>(m->dalloc(sizeof(double) * size_t(loss_grad_blocks(n))));
  m->loss = static_cast<double *>(m->dalloc(sizeof(double)));
  bool ok = m->X && m->T && m->Y && m->dY && m->dA && m->dB && m->part && m->loss;
  for (int l = 0; l < 3; ++l) ok = ok && m->Z[l] && m->H[l];
  if (!ok) {
    m->cap = 0;
    return m->fail(TDPD_ERR_OOM, "device allocation failed");
  }
  m->cap = n;
  return TDPD_OK;
}

// forward pass keeping pre-activations, loss and full gradient of the mean
// squared error for the n rows at X, T (device), targets divided by scale
void forward_backward(tdpd_mlp *m, const float *X, const float *T, int64_t n, float scale) {
  const MlpLayout L;
  const float *P = m->params;
  float *G = m->grad;
  hipStream_t st = m->st;
  GemmArgs g{};
  // forward
  const float *in = X;
  int64_t kin = kSurrIn;
  const int Wo[3] = {L.W1, L.W2, L.W3}, bo[3] = {L.b1, L.b2, L.b3};
  for (int l = 0; l < 3; ++l) {
    g = GemmArgs{};
    g.A = in; g.sa_i = kin; g.sa_p = 1;
    g.B = P + Wo[l]; g.sb_p = 1; g.sb_j = kin;
    g.C = m->Z[l]; g.ldc = kSurrHid; g.M = n; g.N = kSurrHid; g.K = kin;
    g.bias = P + bo[l]; g.epi = kEpiSilu; g.H = m->H[l];
    launch_gemm_bf16(g, st);
    in = m->H[l];
    kin = kSurrHid;
  }
  g = GemmArgs{};
  g.A = m->H[2]; g.sa_i = kSurrHid; g.sa_p = 1;
  g.B = P + L.W4; g.sb_p = 1; g.sb_j = kSurrHid;
  g.C = m->Y; g.ldc = kSurrOut; g.M = n; g.N = kSurrOut; g.K = kSurrHid;
  g.bias = P + L.b4; g.epi = kEpiStore;
  launch_gemm_bf16(g, st);
  launch_loss_grad(m->Y, T, n, 1.f / scale, m->dY, m->part, st);
  launch_sum_parts(m->part, loss_grad_blocks(n), m->loss, st);
  // output layer: dW4 = dY^T H3, db4 = column sums of dY, dZ3 = (dY W4) * silu'(Z3)
  g = GemmArgs{};
  g.A = m->dY; g.sa_i = 1; g.sa_p = kSurrOut;
  g.B = m->H[2]; g.sb_p = kSurrHid; g.sb_j = 1;
  g.C = G + L.W4; g.ldc = kSurrHid; g.M = kSurrOut; g.N = kSurrHid; g.K = n; g.epi = kEpiStore;
  launch_gemm_bf16(g, st);
  launch_colsum(m->dY, n, kSurrOut, kSurrOut, G + L.b4, st);
  g = GemmArgs{};
  g.A = m->dY; g.sa_i = kSurrOut; g.sa_p = 1;
  g.B = P + L.W4; g.sb_p = kSurrHid; g.sb_j = 1;
  g.C = m->dA; g.ldc = kSurrHid; g.M = n; g.N = kSurrHid; g.K = kSurrOut;
  g.epi = kEpiSiluGrad; g.Z = m->Z[2];
  launch_gemm_bf16(g, st);
  // hidden layers 3, 2, 1: dz in cur; weight gradient against the layer input
  float *cur = m->dA, *nxt = m->dB;
  for (int l = 2; l >= 0; --l) {
    const float *lin = l > 0 ? m->H[l - 1] : X;
    const int64_t kl = l > 0 ? kSurrHid : kSurrIn;
    g = GemmArgs{};
    g.A = cur; g.sa_i = 1; g.sa_p = kSurrHid;
    g.B = lin; g.sb_p = kl; g.sb_j = 1;
    g.C = G + Wo[l]; g.ldc = kl; g.M = kSurrHid; g.N = kl; g.K = n; g.epi = kEpiStore;
    launch_gemm_bf16(g, st);
    launch_colsum(cur, n, kSurrHid, kSurrHid, G + bo[l], st);
    if (l > 0) {
      g = GemmArgs{};
      g.A = cur; g.sa_i = kSurrHid; g.sa_p = 1;
      g.B = P + Wo[l]; g.sb_p = kl; g.sb_j = 1;
      g.C = nxt; g.ldc = kSurrHid; g.M = n; g.N = kSurrHid; g.K = kSurrHid;
      g.epi = kEpiSiluGrad; g.Z = m->Z[l - 1];
      launch_gemm_bf16(g, st);
      std::swap(cur, nxt);
    }
  }
}

int check_launch(tdpd_mlp *m) {
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return m->fail(TDPD_ERR_HIP, std::string("kernel launch: ") + hipGetErrorString(e));
  return TDPD_OK;
}

}  // namespace

extern "C" int tdpd_mlp_create(void *hip_stream, tdpd_alloc_fn alloc, tdpd_free_fn free_fn,
                               void *user, tdpd_mlp **out) {
  if (!out || (alloc == nullptr) != (free_fn == nullptr)) return TDPD_ERR_INVALID_ARG;
  tdpd_mlp *m = new tdpd_mlp();
  m->st = reinterpret_cast<hipStream_t>(hip_stream);
  m->alloc = alloc;
  m->free_fn = free_fn;
  m->user = user;
  const size_t pb = sizeof(float) * kSurrParams;
  m->params = static_cast<float *>(m->dalloc(pb));
  m->grad = static_cast<float *>(m->dalloc(pb));
  m->m = static_cast<float *>(m->dalloc(pb));
  m->v = static_cast<float *>(m->dalloc(pb));
  if (!m->params || !m->grad || !m->m || !m->v) {
    for (void *p : std::vector<void *>(m->blocks)) m->dfree(p);
    delete m;
    return TDPD_ERR_OOM;
  }
  *out = m;
  return TDPD_OK;
}

extern "C" void tdpd_mlp_destroy(tdpd_mlp *m) {
  if (!m) return;
  (void)hipStreamSynchronize(m->st);
  for (void *p : std::vector<void *>(m->blocks)) m->dfree(p);
  delete m;
}

extern "C" const char *tdpd_mlp_last_error(const tdpd_mlp *m) {
  return m ? m->err.c_str() : "null network";
}

extern "C" int64_t tdpd_mlp_num_params(void) { return kSurrParams; }

extern "C" int tdpd_mlp_set_params(tdpd_mlp *m, const float *params) {
  if (!m || !params) return TDPD_ERR_INVALID_ARG;
  for (int i = 0; i < kSurrParams; ++i)
    if (!std::isfinite(params[i])) return m->fail(TDPD_ERR_INVALID_ARG, "set_params: non-finite value");
  const size_t pb = sizeof(float) * kSurrParams;
  MLPCHK(hipMemcpyAsync(m->params, params, pb, hipMemcpyHostToDevice, m->st));
  MLPCHK(hipMemsetAsync(m->m, 0, pb, m->st));
  MLPCHK(hipMemsetAsync(m->v, 0, pb, m->st));
  MLPCHK(hipStreamSynchronize(m->st));
  m->adam_t = 0;
  return TDPD_OK;
}

extern "C" int tdpd_mlp_get_params(tdpd_mlp *m, float *params) {
  if (!m || !params) return TDPD_ERR_INVALID_ARG;
  MLPCHK(hipMemcpyAsync(params, m->params, sizeof(float) * kSurrParams, hipMemcpyDeviceToHost, m->st));
  MLPCHK(hipStreamSynchronize(m->st));
  return TDPD_OK;
}

// device pointer of the parameters (for tdpd_surrogate_enable)
const float *mlp_device_params(const tdpd_mlp *m) { return m ? m->params : nullptr; }

extern "C" int tdpd_mlp_forward(tdpd_mlp *m, const float *X, int64_t n, float *Y) {
  if (!m || n < 0 || (n > 0 && (!X || !Y))) return TDPD_ERR_INVALID_ARG;
  if (n == 0) return TDPD_OK;
  int rc = ensure_cap(m, n);
  if (rc) return rc;
  MLPCHK(hipMemcpyAsync(m->X, X, sizeof(float) * n * kSurrIn, hipMemcpyHostToDevice, m->st));
  mlp_forward(m->params, m->X, n, m->Y, m->st);
  if ((rc = check_launch(m))) return rc;
  MLPCHK(hipMemcpyAsync(Y, m->Y, sizeof(float) * n * kSurrOut, hipMemcpyDeviceToHost, m->st));
  MLPCHK(hipStreamSynchronize(m->st));
  return TDPD_OK;
}

extern "C" int tdpd_mlp_forward_hidden(tdpd_mlp *m, const float *X, int64_t n, float *Y,
                                       float *H) {
  if (!m || n < 0 || (n > 0 && (!X || !Y || !H))) return TDPD_ERR_INVALID_ARG;
  if (n == 0) return TDPD_OK;
  int rc = ensure_cap(m, n);
  if (rc) return rc;
  float *dH = static_cast<float *>(m->dalloc(sizeof(float) * size_t(n) * 3 * kSurrHid));
  if (!dH) return m->fail(TDPD_ERR_OOM, "device allocation failed");
  hipError_t e = hipMemcpyAsync(m->X, X, sizeof(float) * n * kSurrIn, hipMemcpyHostToDevice, m->st);
  if (e == hipSuccess) {
    mlp_forward(m->params, m->X, n, m->Y, m->st, dH);
    e = hipGetLastError();
  }
  if (e == hipSuccess)
    e = hipMemcpyAsync(Y, m->Y, sizeof(float) * n * kSurrOut, hipMemcpyDeviceToHost, m->st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(H, dH, sizeof(float) * size_t(n) * 3 * kSurrHid, hipMemcpyDeviceToHost, m->st);
  if (e == hipSuccess) e = hipStreamSynchronize(m->st);
  m->dfree(dH);
  if (e != hipSuccess) return m->fail(TDPD_ERR_HIP, std::string("mlp_forward_hidden: ") + hipGetErrorString(e));
  return TDPD_OK;
}

extern "C" int tdpd_mlp_loss_grad(tdpd_mlp *m, const float *X, const float *T, int64_t n,
                                  float target_scale, double *loss, float *grad) {
  if (!m || n <= 0 || !X || !T || !(target_scale > 0.f)) return TDPD_ERR_INVALID_ARG;
  int rc = ensure_cap(m, n);
  if (rc) return rc;
  MLPCHK(hipMemcpyAsync(m->X, X, sizeof(float) * n * kSurrIn, hipMemcpyHostToDevice, m->st));
  MLPCHK(hipMemcpyAsync(m->T, T, sizeof(float) * n * kSurrOut, hipMemcpyHostToDevice, m->st));
  forward_backward(m, m->X, m->T, n, target_scale);
  if ((rc = check_launch(m))) return rc;
  double s = 0.0;
  MLPCHK(hipMemcpyAsync(&s, m->loss, sizeof(double), hipMemcpyDeviceToHost, m->st));
  if (grad)
    MLPCHK(hipMemcpyAsync(grad, m->grad, sizeof(float) * kSurrParams, hipMemcpyDeviceToHost, m->st));
  MLPCHK(hipStreamSynchronize(m->st));
  if (loss) *loss = s / double(3 * n);
  return TDPD_OK;
}

extern "C" int tdpd_mlp_train(tdpd_mlp *m, const float *X, const float *T, int64_t n,
                              float target_scale, int32_t batch, int32_t steps, float lr,
                              double *loss_out) {
  if (!m || !X || !T || batch <= 0 || n < batch || steps < 0 || !(target_scale > 0.f) ||
      !(lr > 0.f))
    return TDPD_ERR_INVALID_ARG;
  int rc = ensure_cap(m, batch);
  if (rc) return rc;
  // the data set stays on the device for the whole call
  float *dX = static_cast<float *>(m->dalloc(sizeof(float) * size_t(n) * kSurrIn));
  float *dT = static_cast<float *>(m->dalloc(sizeof(float) * size_t(n) * kSurrOut));
  double *dl = static_cast<double *>(m->dalloc(sizeof(double) * size_t(steps > 0 ? steps : 1)));
  if (!dX || !dT || !dl) {
    m->dfree(dX);
    m->dfree(dT);
    m->dfree(dl);
    return m->fail(TDPD_ERR_OOM, "device allocation failed");
  }
  hipError_t e = hipMemcpyAsync(dX, X, sizeof(float) * n * kSurrIn, hipMemcpyHostToDevice, m->st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(dT, T, sizeof(float) * n * kSurrOut, hipMemcpyHostToDevice, m->st);
  const int64_t nb = n / batch;  // full batches, taken in order (the caller shuffles)
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  for (int32_t s = 0; s < steps && e == hipSuccess; ++s) {
    const int64_t off = (s % nb) * batch;
    forward_backward(m, dX + off * kSurrIn, dT + off * kSurrOut, batch, target_scale);
    (void)hipMemcpyAsync(dl + s, m->loss, sizeof(double), hipMemcpyDeviceToDevice, m->st);
    ++m->adam_t;
    const float bc1 = float(1.0 - std::pow(double(b1), double(m->adam_t)));
    const float bc2 = float(1.0 - std::pow(double(b2), double(m->adam_t)));
    launch_adam(m->params, m->grad, m->m, m->v, kSurrParams, lr, b1, b2, eps, bc1, bc2, m->st);
    e = hipGetLastError();
  }
  std::vector<double> hl(size_t(steps > 0 ? steps : 1));
  if (e == hipSuccess && steps > 0)
    e = hipMemcpyAsync(hl.data(), dl, sizeof(double) * steps, hipMemcpyDeviceToHost, m->st);
  const hipError_t es = hipStreamSynchronize(m->st);  // before the buffers go
  if (e == hipSuccess) e = es;
  m->dfree(dX);
  m->dfree(dT);
  m->dfree(dl);
  if (e != hipSuccess) return m->fail(TDPD_ERR_HIP, std::string("train: ") + hipGetErrorString(e));
  if (loss_out)
    for (int32_t s = 0; s < steps; ++s) loss_out[s] = hl[s] / double(3 * batch);
  return TDPD_OK;
}
