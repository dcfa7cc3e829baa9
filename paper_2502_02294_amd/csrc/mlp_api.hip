// libdiffhydro: the learned star-formation closure network (C ABI part, include/diffhydro.h).
// Training runs entirely on the device: per step one launch computes the per-wave partial
// gradients of a batch on the matrix cores, one sums them in a fixed order and applies Adam,
// and one repacks the weights into their matrix-core fragments.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "../../include/diffhydro.h"
#include "dh_kernels.h"
#include "dh_mlp.h"

namespace {

using dh::ArgError;
using dh::HipError;
namespace mlp = dh::mlp;

constexpr uint32_t kTagMlpInit = 0x4D490000u;

}  // namespace

struct dh_mlp {
  hipStream_t st = nullptr;
  float *theta = nullptr, *m = nullptr, *v = nullptr;
  uint4* packed = nullptr;
  float* partial = nullptr;
  double* loss_part = nullptr;
  long long part_cap = 0;
  double* grad = nullptr;
  double* scalars = nullptr;       // device: loss
  double* hist = nullptr;
  int hist_cap = 0;
  double* host = nullptr;          // pinned: loss
  std::vector<void*> allocs;
  std::string err;

  template <typename T>
  T* alloc(long long count) {
    void* p = nullptr;
    if (hipMalloc(&p, static_cast<size_t>(count) * sizeof(T)) != hipSuccess)
      throw std::bad_alloc();
    allocs.push_back(p);
    return static_cast<T*>(p);
  }
  void release(void* p) {
    if (!p) return;
    auto it = std::find(allocs.begin(), allocs.end(), p);
    if (it != allocs.end()) allocs.erase(it);
    (void)hipFree(p);
  }
};

namespace {

int fail(dh_mlp* s, int code, const std::string& msg) {
  if (s) s->err = msg;
  return code;
}

template <typename F>
int guarded(dh_mlp* s, F&& f) {
  try {
    return f();
  } catch (const ArgError& e) {
    return fail(s, DH_E_INVAL, e.what());
  } catch (const HipError& e) {
    return fail(s, DH_E_HIP, e.what());
  } catch (const std::bad_alloc&) {
    return fail(s, DH_E_OOM, "device or host allocation failed");
  } catch (const std::exception& e) {
    return fail(s, DH_E_HIP, e.what());
  }
}

void sync(dh_mlp* s) { DH_HIP(hipStreamSynchronize(s->st)); }

void ensure_parts(dh_mlp* s, long long parts) {
  if (parts <= s->part_cap) return;
  s->release(s->partial);
  s->release(s->loss_part);
  s->partial = nullptr;
  s->loss_part = nullptr;
  s->part_cap = 0;
  s->partial = s->alloc<float>(parts * mlp::kParams);
  s->loss_part = s->alloc<double>(parts);
  s->part_cap = parts;
}

void upload_weights(dh_mlp* s, const float* h_theta) {
  DH_HIP(hipMemcpyAsync(s->theta, h_theta, mlp::kParams * sizeof(float), hipMemcpyHostToDevice,
                        s->st));
  dh::launch_mlp_pack(s->st, s->theta, s->packed);
  sync(s);
}

}  // namespace

extern "C" {

void dh_mlp_train_defaults(dh_mlp_train_opts* o) {
  if (!o) return;
  o->batch = 16384;
  o->steps = 20000;
  o->lr = 3e-3;
  o->lr_final = 3e-5;
  o->beta1 = 0.9;
  o->beta2 = 0.999;
  o->eps = 1e-8;
}

void dh_mlp_sample_defaults(dh_mlp_sample_opts* o) {
  if (!o) return;
  o->lnd_lo = std::log(1e-2);
  o->lnd_hi = std::log(3e4);
  o->lnt_lo = 0.0;
  o->lnt_hi = std::log(3e8);
  o->lna_lo = std::log(0.008);
  o->lna_hi = std::log(0.32);
  o->eps_lo = 0.01;
  o->eps_hi = 0.03;
  o->dc_lo = 50.0;
  o->dc_hi = 150.0;
}

int dh_mlp_create(dh_mlp** out) {
  if (!out) return DH_E_INVAL;
  *out = nullptr;
  auto s = std::make_unique<dh_mlp>();
  int rc = guarded(s.get(), [&]() -> int {
    s->theta = s->alloc<float>(mlp::kParams);
    s->m = s->alloc<float>(mlp::kParams);
    s->v = s->alloc<float>(mlp::kParams);
    s->packed = s->alloc<uint4>(static_cast<long long>(mlp::kPackedBytes / sizeof(uint4)));
    s->grad = s->alloc<double>(mlp::kParams);
    s->scalars = s->alloc<double>(8);
    void* hp = nullptr;
    DH_HIP(hipHostMalloc(&hp, 8 * sizeof(double), hipHostMallocDefault));
    s->host = static_cast<double*>(hp);
    DH_HIP(hipMemset(s->theta, 0, mlp::kParams * sizeof(float)));
    dh::launch_mlp_pack(s->st, s->theta, s->packed);
    DH_HIP(hipDeviceSynchronize());
    return DH_OK;
  });
  if (rc != DH_OK) {
    dh_mlp_destroy(s.release());
    return rc;
  }
  *out = s.release();
  return DH_OK;
}

int dh_mlp_destroy(dh_mlp* s) {
  if (!s) return DH_OK;
  if (s->st) (void)hipStreamSynchronize(s->st);
  else (void)hipDeviceSynchronize();
  for (void* p : s->allocs) (void)hipFree(p);
  if (s->host) (void)hipHostFree(s->host);
  delete s;
  return DH_OK;
}

int dh_mlp_set_stream(dh_mlp* s, void* stream) {
  if (!s) return DH_E_INVAL;
  s->st = static_cast<hipStream_t>(stream);
  return DH_OK;
}

int dh_mlp_init_weights(dh_mlp* s, uint64_t seed) {
  if (!s) return DH_E_INVAL;
  return guarded(s, [&]() -> int {
    std::vector<float> th(mlp::kParams);
    const int fan[8] = {mlp::kIn, mlp::kIn, mlp::kHid, mlp::kHid, mlp::kHid, mlp::kHid, mlp::kHid,
                        mlp::kHid};
    const int off[9] = {mlp::kOffW1, mlp::kOffB1, mlp::kOffW2, mlp::kOffB2, mlp::kOffW3,
                        mlp::kOffB3, mlp::kOffW4, mlp::kOffB4, mlp::kParams};
    for (int part = 0; part < 8; ++part) {
      const double bound = 1.0 / std::sqrt(static_cast<double>(fan[part]));
      for (int i = off[part]; i < off[part + 1]; ++i) {
        uint32_t c[4] = {static_cast<uint32_t>(i), 0u, kTagMlpInit, 0u};
        dh::philox4x32_10(c, static_cast<uint32_t>(seed), static_cast<uint32_t>(seed >> 32));
        th[i] = static_cast<float>(bound * (2.0 * dh::uniform_open_d(c[0]) - 1.0));
      }
    }
    upload_weights(s, th.data());
    return DH_OK;
  });
}

int dh_mlp_set_weights(dh_mlp* s, const float* h_theta) {
  if (!s || !h_theta) return DH_E_INVAL;
  return guarded(s, [&]() -> int {
    upload_weights(s, h_theta);
    return DH_OK;
  });
}

int dh_mlp_get_weights(dh_mlp* s, float* h_theta) {
  if (!s || !h_theta) return DH_E_INVAL;
  return guarded(s, [&]() -> int {
    DH_HIP(hipMemcpyAsync(h_theta, s->theta, mlp::kParams * sizeof(float), hipMemcpyDeviceToHost,
                          s->st));
    sync(s);
    return DH_OK;
  });
}

int dh_mlp_sample(dh_mlp* s, const dh_mlp_sample_opts* opts, double omega_b, const dh_params* p,
                  uint64_t seed, int64_t first, int64_t count, float* d_x, float* d_y) {
  if (!s || !p || !d_x || !d_y || count <= 0 || first < 0) return DH_E_INVAL;
  dh_mlp_sample_opts o;
  if (opts) o = *opts;
  else dh_mlp_sample_defaults(&o);
  if (!(o.lnd_lo <= o.lnd_hi && o.lnt_lo <= o.lnt_hi && o.lna_lo <= o.lna_hi &&
        o.eps_lo > 0 && o.eps_lo <= o.eps_hi && o.dc_lo > 0 && o.dc_lo <= o.dc_hi &&
        omega_b > 0 && p->t_c > 0 && p->w_rho > 0 && p->w_t > 0))
    return fail(s, DH_E_INVAL, "bad sampling ranges or parameters");
  return guarded(s, [&]() -> int {
    dh::MlpSampleArgs a{};
    a.first = first;
    a.seed_lo = static_cast<uint32_t>(seed);
    a.seed_hi = static_cast<uint32_t>(seed >> 32);
    a.lnd_lo = o.lnd_lo;
    a.lnd_hi = o.lnd_hi;
    a.lnt_lo = o.lnt_lo;
    a.lnt_hi = o.lnt_hi;
    a.lna_lo = o.lna_lo;
    a.lna_hi = o.lna_hi;
    a.eps_lo = o.eps_lo;
    a.eps_hi = o.eps_hi;
    a.dc_lo = o.dc_lo;
    a.dc_hi = o.dc_hi;
    a.t_c = p->t_c;
    a.omega_b = omega_b;
    a.w_rho = p->w_rho;
    a.w_t = p->w_t;
    dh::launch_mlp_sample(s->st, a, d_x, d_y, count);
    return DH_OK;
  });
}

int dh_mlp_eval(dh_mlp* s, const float* d_x, int64_t count, float* d_out) {
  if (!s || !d_x || !d_out || count < 0) return DH_E_INVAL;
  if (count == 0) return DH_OK;
  return guarded(s, [&]() -> int {
    dh::launch_mlp_eval(s->st, s->packed, d_x, d_out, count);
    return DH_OK;
  });
}

int dh_mlp_vjp(dh_mlp* s, const float* d_x, const float* d_gout, int64_t count, float* d_gx) {
  if (!s || !d_x || !d_gout || !d_gx || count < 0) return DH_E_INVAL;
  if (count == 0) return DH_OK;
  return guarded(s, [&]() -> int {
    dh::launch_mlp_vjp(s->st, s->packed, d_x, d_gout, d_gx, count);
    return DH_OK;
  });
}

int dh_mlp_grad(dh_mlp* s, const float* d_x, const float* d_y, int64_t count, double* h_grad,
                double* loss_out) {
  if (!s || !d_x || !d_y || !h_grad || count <= 0) return DH_E_INVAL;
  return guarded(s, [&]() -> int {
    const int parts = dh::mlp_train_parts(count);
    ensure_parts(s, parts);
    dh::launch_mlp_train_grad(s->st, s->packed, d_x, d_y, count, 0, count, s->partial,
                              s->loss_part);
    dh::launch_mlp_reduce_grad(s->st, s->partial, parts, s->loss_part,
                               1.0 / static_cast<double>(count), s->grad, s->scalars);
    DH_HIP(hipMemcpyAsync(h_grad, s->grad, mlp::kParams * sizeof(double), hipMemcpyDeviceToHost,
                          s->st));
    DH_HIP(hipMemcpyAsync(s->host, s->scalars, sizeof(double), hipMemcpyDeviceToHost, s->st));
    sync(s);
    if (loss_out) *loss_out = s->host[0];
    return DH_OK;
  });
}

int dh_mlp_train(dh_mlp* s, const float* d_x, const float* d_y, int64_t count,
                 const dh_mlp_train_opts* opts, double* h_loss) {
  if (!s || !d_x || !d_y || !opts || count <= 0) return DH_E_INVAL;
  const dh_mlp_train_opts o = *opts;
  if (o.batch <= 0 || o.batch > count || o.steps < 0 || !(o.lr > 0) || !(o.lr_final >= 0) ||
      !(o.beta1 >= 0 && o.beta1 < 1) || !(o.beta2 >= 0 && o.beta2 < 1) || !(o.eps > 0))
    return fail(s, DH_E_INVAL, "bad training options");
  return guarded(s, [&]() -> int {
    const int parts = dh::mlp_train_parts(o.batch);
    ensure_parts(s, parts);
    if (o.steps > s->hist_cap) {
      s->release(s->hist);
      s->hist = nullptr;
      s->hist_cap = 0;
      s->hist = s->alloc<double>(o.steps);
      s->hist_cap = o.steps;
    }
    DH_HIP(hipMemsetAsync(s->m, 0, mlp::kParams * sizeof(float), s->st));
    DH_HIP(hipMemsetAsync(s->v, 0, mlp::kParams * sizeof(float), s->st));
    const double pi = 3.14159265358979323846;
    double b1t = 1.0, b2t = 1.0;
    for (int k = 0; k < o.steps; ++k) {
      const long long start = (static_cast<long long>(k) * o.batch) % count;
      dh::launch_mlp_train_grad(s->st, s->packed, d_x, d_y, count, start, o.batch, s->partial,
                                s->loss_part);
      b1t *= o.beta1;
      b2t *= o.beta2;
      dh::AdamArgs a{};
      a.lr = static_cast<float>(o.lr_final + 0.5 * (o.lr - o.lr_final) *
                                                 (1.0 + std::cos(pi * k / std::max(1, o.steps))));
      a.beta1 = static_cast<float>(o.beta1);
      a.beta2 = static_cast<float>(o.beta2);
      a.eps = static_cast<float>(o.eps);
      a.corr1 = static_cast<float>(1.0 / (1.0 - b1t));
      a.corr2 = static_cast<float>(1.0 / (1.0 - b2t));
      a.step = k;
      dh::launch_mlp_adam(s->st, s->partial, parts, s->loss_part,
                          1.0 / static_cast<double>(o.batch), s->theta, s->m, s->v, a, s->hist);
      dh::launch_mlp_pack(s->st, s->theta, s->packed);
    }
    if (h_loss && o.steps > 0)
      DH_HIP(hipMemcpyAsync(h_loss, s->hist, o.steps * sizeof(double), hipMemcpyDeviceToHost,
                            s->st));
    sync(s);
    return DH_OK;
  });
}

const char* dh_mlp_last_error(const dh_mlp* s) { return s ? s->err.c_str() : "null handle"; }

}  // extern "C"
