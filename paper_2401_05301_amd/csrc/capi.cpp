// extern "C" entry points: argument validation, error translation, handle lifecycle.
#include <cmath>
#include <cstring>
#include <string>
#include <thread>
#include <vector>

#include "../../include/ptebd_diag.h"
#include "engine.hpp"

namespace {

thread_local std::string g_err;

}  // namespace

namespace ptebd {
void set_last_error(const std::string& msg) { g_err = msg; }
}  // namespace ptebd

namespace {

tebd_status fail(int code, const std::string& msg) {
  g_err = msg;
  return (tebd_status)code;
}

// Routes the launchers' timing records to the handle's profiler for the
// duration of one call.
struct ProfBind {
  ProfBind(tebd_mps* M) { ptebd::active_profiler() = (M && M->prof_on) ? &M->prof : nullptr; }
  ~ProfBind() { ptebd::active_profiler() = nullptr; }
};

template <class F>
tebd_status guard(F&& f) {
  try {
    f();
    return TEBD_OK;
  } catch (const ptebd::Error& e) {
    return fail(e.code, e.what());
  } catch (const std::bad_alloc&) {
    return fail(TEBD_ENOMEM, "host allocation failed");
  } catch (const std::exception& e) {
    return fail(TEBD_EDEVICE, e.what());
  }
}

bool finite(double x) { return std::isfinite(x); }

tebd_status check_model(const tebd_model* m) {
  if (!m) return fail(TEBD_EINVAL, "model is NULL");
  if (m->L < 3) return fail(TEBD_EINVAL, "L must be >= 3 for three-site gates");
  if (m->d < 2) return fail(TEBD_EINVAL, "d must be >= 2");
  if (m->d > 8) return fail(TEBD_EINVAL, "d must be <= 8");
  if (!finite(m->U) || !finite(m->J) || !finite(m->Jnnn) || !finite(m->K) || !finite(m->jc))
    return fail(TEBD_EINVAL, "model parameters must be finite");
  return TEBD_OK;
}

tebd_status check_opts(const tebd_opts* o, int d) {
  if (!o) return fail(TEBD_EINVAL, "opts is NULL");
  if (o->chi_max < 1) return fail(TEBD_EINVAL, "chi_max must be >= 1");
  if (o->supersite != 0 && o->supersite != 1) return fail(TEBD_EINVAL, "supersite must be 0 or 1");
  if (o->u1 != 0 && o->u1 != 1) return fail(TEBD_EINVAL, "u1 must be 0 or 1");
  const int64_t dl = o->supersite ? (int64_t)d * d : d;   // local dimension of the chain the MPS lives on
  if ((int64_t)o->chi_max * dl > 8192) return fail(TEBD_EINVAL, "chi_max * (local dimension) must be <= 8192");
  if (!finite(o->trunc_weight) || o->trunc_weight < 0) return fail(TEBD_EINVAL, "trunc_weight must be >= 0");
  if (!finite(o->trunc_rel) || o->trunc_rel < 0) return fail(TEBD_EINVAL, "trunc_rel must be >= 0");
  if (o->prec < TEBD_FP64 || o->prec > TEBD_FP32_SPLIT) return fail(TEBD_EINVAL, "bad precision");
  if (o->svd < TEBD_SVD_JACOBI || o->svd > TEBD_SVD_RANDOMIZED) return fail(TEBD_EINVAL, "bad svd variant");
  if (o->svd != TEBD_SVD_JACOBI && !(o->trunc_rel >= TEBD_GRAM_EPS_MIN))
    return fail(TEBD_EINVAL,
                "the Gram route resolves singular values down to 1e-6 of the largest: trunc_rel must be >= "
                "TEBD_GRAM_EPS_MIN (1e-6); use TEBD_SVD_JACOBI for a smaller eps");
  if (o->workers < 0) return fail(TEBD_EINVAL, "workers must be >= 0");
  if (o->fuse != 0 && o->fuse != 1) return fail(TEBD_EINVAL, "fuse must be 0 or 1");
  if (o->fuse && (o->svd != TEBD_SVD_JACOBI || o->u1 || o->supersite))
    return fail(TEBD_EINVAL, "fuse needs the Jacobi route on a dense three-site chain (svd = TEBD_SVD_JACOBI, "
                             "u1 = 0, supersite = 0)");
  if ((o->dev_alloc == nullptr) != (o->dev_free == nullptr))
    return fail(TEBD_EINVAL, "dev_alloc and dev_free must be given together");
  return TEBD_OK;
}

ptebd::ModelP to_model(const tebd_model* m) { return ptebd::ModelP{m->L, m->d, m->U, m->J, m->Jnnn, m->K, m->jc}; }

tebd_status create(const tebd_model* model, const tebd_opts* opts, tebd_mps** out, tebd_mps** made) {
  if (!out) return fail(TEBD_EINVAL, "out is NULL");
  *out = nullptr;
  tebd_status st = check_model(model);
  if (st) return st;
  st = check_opts(opts, model->d);
  if (st) return st;
  if (opts->supersite && (model->L % 2 != 0 || model->L < 4))
    return fail(TEBD_EINVAL, "a super-site chain needs an even number of physical sites, at least 4");
  tebd_mps* M = new tebd_mps();
  st = guard([&] {
    M->opts = *opts;
    M->phys_L = model->L;
    M->pd = model->d;
    M->super = opts->supersite != 0;
    M->L = M->super ? model->L / 2 : model->L;
    M->d = M->super ? model->d * model->d : model->d;
    M->u1 = opts->u1 != 0;
    // bosons of every local level: s, or s1 + s2 for the super-site index s1 d + s2
    M->qs.resize(M->d);
    for (int t = 0; t < M->d; ++t) M->qs[t] = M->super ? t / model->d + t % model->d : t;
    M->chi_max = opts->chi_max;
    if (opts->stream) {
      M->stream = (hipStream_t)opts->stream;
    } else {
      PTEBD_HIP(hipStreamCreateWithFlags(&M->stream, hipStreamNonBlocking));
      M->own_stream = true;
    }
    ptebd::mps_allocate(M);
    ptebd::set_model(M, to_model(model));
  });
  if (st) {
    ptebd::mps_release(M);
    if (M->own_stream) (void)hipStreamDestroy(M->stream);
    delete M;
    return st;
  }
  *made = M;
  return TEBD_OK;
}

tebd_status usable(const tebd_mps* M) {
  if (!M) return fail(TEBD_EINVAL, "handle is NULL");
  if (M->failed) return fail(TEBD_ESTATE, "handle is in an error state (an SVD failed to converge)");
  return TEBD_OK;
}

// One second-order (Strang) step of the handle's chain.
void strang(tebd_mps* M, double dt) {
  const double h = 0.5 * dt;
  if (M->super) {   // A(dt/2) B(dt) A(dt/2), A = even K, B = odd K
    ptebd::layer(M, 0, h);
    ptebd::layer(M, 1, dt);
    ptebd::layer(M, 0, h);
    return;
  }
  ptebd::layer(M, 0, h);
  ptebd::layer(M, 1, h);
  ptebd::layer(M, 2, dt);
  ptebd::layer(M, 1, h);
  ptebd::layer(M, 0, h);
}

// Byte image of a checkpoint: a fixed header, then chi[L + 1] (int32, padded
// to a multiple of 8 bytes), the Schmidt values of bonds 0..L and the site
// tensors 0..L-1 in stored form, back to back.
struct CkHeader {
  char tag[8];                // "ptebdck" and a NUL
  uint32_t version;
  int32_t L, d;               // sites and local dimension of the chain the MPS lives on
  int32_t phys_L, phys_d;     // physical chain
  int32_t supersite, u1;
  int32_t reserved;
  double ledger;
  uint64_t payload;           // bytes after the header
  uint64_t checksum;          // over header (this field zero) and payload
};
static_assert(sizeof(CkHeader) == 64, "checkpoint header layout");
constexpr char kCkTag[8] = {'p', 't', 'e', 'b', 'd', 'c', 'k', '\0'};
constexpr uint32_t kCkVersion = 1;

// 64-bit FNV-1a over 8-byte words (tail bytes one at a time): detects a
// damaged or truncated image, not tampering.
uint64_t ck_hash(const unsigned char* p, size_t n, uint64_t h = 14695981039346656037ull) {
  constexpr uint64_t prime = 1099511628211ull;
  size_t i = 0;
  for (; i + 8 <= n; i += 8) {
    uint64_t w;
    std::memcpy(&w, p + i, 8);
    h = (h ^ w) * prime;
  }
  for (; i < n; ++i) h = (h ^ p[i]) * prime;
  return h;
}

size_t ck_chi_bytes(int L) { return ((size_t)(L + 1) * sizeof(int32_t) + 7) / 8 * 8; }

// Payload bytes of a state with bond dimensions chi[L + 1] and local dimension d.
size_t ck_payload(const int32_t* chi, int L, int d) {
  size_t n = 0;
  for (int b = 0; b <= L; ++b) n += (size_t)chi[b];
  for (int i = 0; i < L; ++i) n += 2 * (size_t)chi[i] * d * chi[i + 1];
  return ck_chi_bytes(L) + n * sizeof(double);
}

uint64_t ck_checksum(const CkHeader& h, const unsigned char* payload) {
  CkHeader z = h;
  z.checksum = 0;
  return ck_hash(payload, h.payload, ck_hash(reinterpret_cast<const unsigned char*>(&z), sizeof z));
}

}  // namespace

extern "C" {

void tebd_opts_default(tebd_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->chi_max = 64;
  o->trunc_weight = 1e-12;
  o->trunc_rel = 1e-12;
  o->prec = TEBD_FP64;
  o->svd = TEBD_SVD_JACOBI;
  o->max_sweeps = 80;
}

tebd_status mps_init_product(const tebd_model* model, const tebd_opts* opts, const int32_t* occ, tebd_mps** out) {
  if (!occ) return fail(TEBD_EINVAL, "occ is NULL");
  tebd_status st = check_model(model);
  if (st) return st;
  for (int i = 0; i < model->L; ++i)
    if (occ[i] < 0 || occ[i] >= model->d) return fail(TEBD_EINVAL, "occupation outside 0..d-1");
  tebd_mps* M = nullptr;
  st = create(model, opts, out, &M);
  if (st) return st;
  st = guard([&] { ptebd::upload_product(M, occ); });
  if (st) {
    mps_free(M);
    return st;
  }
  *out = M;
  return TEBD_OK;
}

tebd_status mps_init_cdw(const tebd_model* model, const tebd_opts* opts, int32_t first_occupied, tebd_mps** out) {
  if (first_occupied != 0 && first_occupied != 1) return fail(TEBD_EINVAL, "first_occupied must be 0 or 1");
  tebd_status st = check_model(model);
  if (st) return st;
  std::vector<int32_t> occ(model->L);
  for (int i = 0; i < model->L; ++i) occ[i] = ((i % 2 == 0) == (first_occupied == 1)) ? 1 : 0;
  return mps_init_product(model, opts, occ.data(), out);
}

tebd_status mps_init_state(const tebd_model* model, const tebd_opts* opts, const int32_t* chi, const double* B,
                           const double* lam, tebd_mps** out) {
  if (!chi || !B || !lam) return fail(TEBD_EINVAL, "chi, B and lam must be non-NULL");
  tebd_status st = check_model(model);
  if (st) return st;
  st = check_opts(opts, model->d);
  if (st) return st;
  if (opts->supersite) return fail(TEBD_EINVAL, "mps_init_state loads three-site chains only");
  ptebd::Sizes sz = ptebd::plan_sizes(model->L, model->d, opts->chi_max);
  if (chi[0] != 1 || chi[model->L] != 1) return fail(TEBD_EINVAL, "chi[0] and chi[L] must be 1");
  for (int b = 0; b <= model->L; ++b)
    if (chi[b] < 1 || chi[b] > sz.cap[b]) return fail(TEBD_EINVAL, "bond dimension outside 1..min(d^b, d^(L-b), chi_max)");
  tebd_mps* M = nullptr;
  st = create(model, opts, out, &M);
  if (st) return st;
  st = guard([&] { ptebd::upload_state(M, chi, B, lam); });
  if (st) {
    mps_free(M);
    return st;
  }
  *out = M;
  return TEBD_OK;
}

tebd_status tebd_layer(tebd_mps* M, int32_t group, double tau) {
  tebd_status st = usable(M);
  if (st) return st;
  if (group < 0 || group > (M->super ? 1 : 2))
    return fail(TEBD_EINVAL, M->super ? "group must be 0 or 1 on a super-site chain" : "group must be 0, 1 or 2");
  if (!std::isfinite(tau)) return fail(TEBD_EINVAL, "tau must be finite");
  ProfBind pb(M);
  return guard([&] { ptebd::layer(M, group, tau); });
}

tebd_status tebd_step(tebd_mps* M, double dt) {
  tebd_status st = usable(M);
  if (st) return st;
  if (!std::isfinite(dt)) return fail(TEBD_EINVAL, "dt must be finite");
  ProfBind pb(M);
  return guard([&] { strang(M, dt); });
}

tebd_status tebd_step4(tebd_mps* M, double dt) {
  tebd_status st = usable(M);
  if (st) return st;
  if (!std::isfinite(dt)) return fail(TEBD_EINVAL, "dt must be finite");
  ProfBind pb(M);
  return guard([&] {
    // Suzuki's fractal weights: 4p + (1 - 4p) = 1 and 4p^3 + (1 - 4p)^3 = 0
    const double p = 1.0 / (4.0 - std::cbrt(4.0));
    const double w[5] = {p, p, 1.0 - 4.0 * p, p, p};
    for (double x : w) strang(M, x * dt);
  });
}

tebd_status tebd_step_many(tebd_mps* const* mps, int32_t n, const double* dt) {
  if (n < 0 || (n > 0 && (!mps || !dt))) return fail(TEBD_EINVAL, "bad handle list");
  for (int i = 0; i < n; ++i) {
    tebd_status st = usable(mps[i]);
    if (st) return st;
    if (!std::isfinite(dt[i])) return fail(TEBD_EINVAL, "dt must be finite");
    for (int k = 0; k < i; ++k)
      if (mps[k] == mps[i]) return fail(TEBD_EINVAL, "handles must be distinct");
  }
  if (n == 1) return tebd_step(mps[0], dt[0]);
  bool fused = n > 1;
  for (int i = 0; i < n; ++i) fused = fused && mps[i]->opts.fuse != 0 && !mps[i]->super;
  if (fused) {
    // one fused batch per layer over all handles: the Strang layers of
    // tebd_step, each handle with its own dt
    ProfBind pb(mps[0]);
    std::vector<tebd_mps*> hs(mps, mps + n);
    return guard([&] {
      const int groups[5] = {0, 1, 2, 1, 0};
      const double frac[5] = {0.5, 0.5, 1.0, 0.5, 0.5};
      std::vector<double> tau(n);
      for (int l = 0; l < 5; ++l) {
        for (int i = 0; i < n; ++i) tau[i] = frac[l] == 1.0 ? dt[i] : 0.5 * dt[i];
        ptebd::layers_many(hs, groups[l], tau);
      }
    });
  }
  // Each handle runs its own stream(s); one host thread per handle issues its
  // step, so that the handles' kernels overlap on the device.
  std::vector<tebd_status> status(n, TEBD_OK);
  std::vector<std::string> message(n);
  std::vector<std::thread> threads;
  threads.reserve(n);
  for (int i = 0; i < n; ++i)
    threads.emplace_back([&, i] {
      status[i] = tebd_step(mps[i], dt[i]);
      if (status[i]) message[i] = g_err;
    });
  for (auto& t : threads) t.join();
  for (int i = 0; i < n; ++i)
    if (status[i]) return fail(status[i], "handle " + std::to_string(i) + ": " + message[i]);
  return TEBD_OK;
}

tebd_status measure_local(tebd_mps* M, double* n, double* c_nn, double* c_nnn) {
  tebd_status st = usable(M);
  if (st) return st;
  ProfBind pb(M);
  return guard([&] { ptebd::measure(M, n, c_nn, c_nnn); });
}

tebd_status measure_quasi_local(tebd_mps* M, int32_t centre, double* out) {
  tebd_status st = usable(M);
  if (st) return st;
  if (!out) return fail(TEBD_EINVAL, "out is NULL");
  if (centre < 0 || centre >= M->phys_L) return fail(TEBD_EINVAL, "centre must be a site index");
  ProfBind pb(M);
  return guard([&] {
    const int L = M->phys_L;
    std::vector<double> n(L), c(2 * (L - 1));
    ptebd::measure(M, n.data(), c.data(), nullptr);
    // j = i - centre; the centre site is even
    double N = 0.0, nodd = 0.0, neven = 0.0, cr = 0.0, ci = 0.0, re_all = 0.0;
    for (int i = 0; i < L; ++i) {
      N += n[i];
      if (((i - centre) & 1) == 0) neven += n[i];
      else nodd += n[i];
    }
    for (int i = 0; i + 1 < L; ++i) {
      re_all += c[2 * i];
      if (((i - centre) & 1) == 0) {
        cr += c[2 * i];
        ci += c[2 * i + 1];
      }
    }
    if (!(N > 0.0)) throw ptebd::Error(TEBD_ESTATE, "quasi-local observables need a state with particles");
    nodd /= N;
    neven /= N;
    cr /= N;
    ci /= N;
    const double zr = neven - nodd, zi = -2.0 * ci;   // A e^{i phi} = n_even - n_odd - 2 i Im C_even
    out[0] = N;
    out[1] = nodd;
    out[2] = neven;
    out[3] = cr;
    out[4] = ci;
    out[5] = std::hypot(zr, zi);
    out[6] = std::atan2(zi, zr);
    out[7] = 2.0 * re_all / N;                          // nu = (1/N) sum_j (C_j + C_j^*)
  });
}

tebd_status mps_set_model(tebd_mps* M, const tebd_model* model) {
  tebd_status st = usable(M);
  if (st) return st;
  st = check_model(model);
  if (st) return st;
  if (model->L != M->phys_L || model->d != M->pd) return fail(TEBD_EINVAL, "set_model must keep L and d");
  return guard([&] {
    PTEBD_HIP(hipStreamSynchronize(M->stream));
    ptebd::set_model(M, to_model(model));
  });
}

tebd_status mps_bond_dims(const tebd_mps* M, int32_t* chi) {
  if (!M || !chi) return fail(TEBD_EINVAL, "NULL argument");
  std::memcpy(chi, M->chi.data(), sizeof(int32_t) * (M->L + 1));
  return TEBD_OK;
}

tebd_status mps_lambda(const tebd_mps* M, int32_t bond, double* s, int32_t cap, int32_t* len) {
  if (!M || !s || !len) return fail(TEBD_EINVAL, "NULL argument");
  if (bond < 0 || bond > M->L) return fail(TEBD_EINVAL, "bond out of range");
  const int n = M->chi[bond];
  *len = n;
  if (cap < n) return fail(TEBD_EINVAL, "output capacity smaller than the bond dimension");
  return guard([&] {
    PTEBD_HIP(hipMemcpyAsync(s, M->lam[bond], sizeof(double) * n, hipMemcpyDeviceToHost, M->stream));
    PTEBD_HIP(hipStreamSynchronize(M->stream));
  });
}

tebd_status mps_bond_charges(const tebd_mps* M, int32_t bond, int32_t* q, int32_t cap, int32_t* len) {
  if (!M || !q || !len) return fail(TEBD_EINVAL, "NULL argument");
  if (!M->u1) return fail(TEBD_ESTATE, "particle numbers are tracked only with opts.u1 = 1");
  if (bond < 0 || bond > M->L) return fail(TEBD_EINVAL, "bond out of range");
  const int n = M->chi[bond];
  *len = n;
  if (cap < n) return fail(TEBD_EINVAL, "output capacity smaller than the bond dimension");
  for (int a = 0; a < n; ++a) q[a] = M->q[bond][a];
  return TEBD_OK;
}

tebd_status mps_site(const tebd_mps* M, int32_t site, double* buf, int64_t cap) {
  if (!M || !buf) return fail(TEBD_EINVAL, "NULL argument");
  if (site < 0 || site >= M->L) return fail(TEBD_EINVAL, "site out of range");
  const int64_t n = (int64_t)M->chi[site] * M->d * M->chi[site + 1];
  if (cap < 2 * n) return fail(TEBD_EINVAL, "output capacity too small");
  return guard([&] {
    PTEBD_HIP(hipMemcpyAsync(buf, M->Br[site], sizeof(double) * n, hipMemcpyDeviceToHost, M->stream));
    PTEBD_HIP(hipMemcpyAsync(buf + n, M->Bi[site], sizeof(double) * n, hipMemcpyDeviceToHost, M->stream));
    PTEBD_HIP(hipStreamSynchronize(M->stream));
  });
}

tebd_status mps_discarded_weight(const tebd_mps* M, double* w) {
  if (!M || !w) return fail(TEBD_EINVAL, "NULL argument");
  return guard([&] {
    PTEBD_HIP(hipMemcpyAsync(w, M->ledger, sizeof(double), hipMemcpyDeviceToHost, M->stream));
    PTEBD_HIP(hipStreamSynchronize(M->stream));
  });
}

tebd_status mps_checkpoint(const tebd_mps* M, void* buf, size_t cap, size_t* bytes) {
  if (!bytes) return fail(TEBD_EINVAL, "NULL argument");
  tebd_status st0 = usable(M);   // a half-applied layer is no state to resume from
  if (st0) return st0;
  const int L = M->L, d = M->d;
  const size_t payload = ck_payload(M->chi.data(), L, d);
  *bytes = sizeof(CkHeader) + payload;
  if (!buf) return TEBD_OK;
  if (cap < *bytes) return fail(TEBD_EINVAL, "output capacity smaller than the checkpoint");
  unsigned char* out = static_cast<unsigned char*>(buf);
  unsigned char* body = out + sizeof(CkHeader);
  CkHeader h{};
  std::memcpy(h.tag, kCkTag, sizeof h.tag);
  h.version = kCkVersion;
  h.L = L;
  h.d = d;
  h.phys_L = M->phys_L;
  h.phys_d = M->pd;
  h.supersite = M->super ? 1 : 0;
  h.u1 = M->u1 ? 1 : 0;
  h.payload = payload;
  std::memset(body, 0, ck_chi_bytes(L));
  std::memcpy(body, M->chi.data(), sizeof(int32_t) * (L + 1));
  tebd_status st = guard([&] {
    // the caller's buffer may sit at any alignment: addressed in bytes
    unsigned char* v = body + ck_chi_bytes(L);
    PTEBD_HIP(hipMemcpyAsync(&h.ledger, M->ledger, sizeof(double), hipMemcpyDeviceToHost, M->stream));
    for (int b = 0; b <= L; ++b) {
      const size_t n = sizeof(double) * M->chi[b];
      PTEBD_HIP(hipMemcpyAsync(v, M->lam[b], n, hipMemcpyDeviceToHost, M->stream));
      v += n;
    }
    for (int i = 0; i < L; ++i) {
      const size_t n = sizeof(double) * (size_t)M->chi[i] * d * M->chi[i + 1];
      PTEBD_HIP(hipMemcpyAsync(v, M->Br[i], n, hipMemcpyDeviceToHost, M->stream));
      PTEBD_HIP(hipMemcpyAsync(v + n, M->Bi[i], n, hipMemcpyDeviceToHost, M->stream));
      v += 2 * n;
    }
    PTEBD_HIP(hipStreamSynchronize(M->stream));
  });
  if (st) return st;
  h.checksum = ck_checksum(h, body);
  std::memcpy(out, &h, sizeof h);
  return TEBD_OK;
}

tebd_status mps_restore(const tebd_model* model, const tebd_opts* opts, const void* buf, size_t len,
                        tebd_mps** out) {
  if (!out) return fail(TEBD_EINVAL, "out is NULL");
  *out = nullptr;
  if (!buf) return fail(TEBD_EINVAL, "buf is NULL");
  tebd_status st = check_model(model);
  if (st) return st;
  st = check_opts(opts, model->d);
  if (st) return st;
  if (len < sizeof(CkHeader)) return fail(TEBD_EINVAL, "checkpoint cut short (no header)");
  const unsigned char* in = static_cast<const unsigned char*>(buf);
  CkHeader h;
  std::memcpy(&h, in, sizeof h);
  if (std::memcmp(h.tag, kCkTag, sizeof h.tag) != 0) return fail(TEBD_EINVAL, "not a checkpoint image");
  if (h.version != kCkVersion) return fail(TEBD_EINVAL, "unsupported checkpoint version");
  const bool super = opts->supersite != 0;
  if (h.supersite != (super ? 1 : 0)) return fail(TEBD_EINVAL, "checkpoint and opts differ in supersite");
  if (h.phys_L != model->L || h.phys_d != model->d)
    return fail(TEBD_EINVAL, "checkpoint and model differ in L or d");
  if (super && (model->L % 2 != 0 || model->L < 4))
    return fail(TEBD_EINVAL, "a super-site chain needs an even number of physical sites, at least 4");
  const int L = super ? model->L / 2 : model->L;
  const int d = super ? model->d * model->d : model->d;
  if (h.L != L || h.d != d) return fail(TEBD_EINVAL, "checkpoint header is inconsistent");
  const unsigned char* body = in + sizeof(CkHeader);
  const size_t avail = len - sizeof(CkHeader);
  if (avail < ck_chi_bytes(L) || h.payload > avail) return fail(TEBD_EINVAL, "checkpoint cut short");
  if (h.checksum != ck_checksum(h, body)) return fail(TEBD_EINVAL, "checkpoint checksum mismatch");
  std::vector<int32_t> chi(L + 1);
  std::memcpy(chi.data(), body, sizeof(int32_t) * (L + 1));
  const ptebd::Sizes sz = super ? ptebd::plan_sizes2(L, d, opts->chi_max) : ptebd::plan_sizes(L, d, opts->chi_max);
  if (chi[0] != 1 || chi[L] != 1) return fail(TEBD_EINVAL, "checkpoint has chi[0] or chi[L] != 1");
  for (int b = 0; b <= L; ++b)
    if (chi[b] < 1 || chi[b] > sz.cap[b])
      return fail(TEBD_EINVAL, "checkpointed bond dimension outside 1..min(d^b, d^(L-b), chi_max)");
  if (h.payload != ck_payload(chi.data(), L, d)) return fail(TEBD_EINVAL, "checkpoint size does not match its bonds");
  if (!std::isfinite(h.ledger) || h.ledger < 0) return fail(TEBD_EINVAL, "checkpointed ledger is not a weight");
  // the image may sit at any alignment: the values are copied out
  size_t nv = 0;
  for (int b = 0; b <= L; ++b) nv += (size_t)chi[b];
  size_t nb = 0;
  for (int i = 0; i < L; ++i) nb += 2 * (size_t)chi[i] * d * chi[i + 1];
  std::vector<double> lam, B;
  st = guard([&] {
    lam.resize(nv);
    B.resize(nb);
  });
  if (st) return st;
  const unsigned char* v = body + ck_chi_bytes(L);
  std::memcpy(lam.data(), v, sizeof(double) * nv);
  std::memcpy(B.data(), v + sizeof(double) * nv, sizeof(double) * nb);
  tebd_mps* M = nullptr;
  st = create(model, opts, out, &M);
  if (st) return st;
  const double ledger = h.ledger;
  st = guard([&] {
    ptebd::upload_state(M, chi.data(), B.data(), lam.data());
    PTEBD_HIP(hipMemcpyAsync(M->ledger, &ledger, sizeof(double), hipMemcpyHostToDevice, M->stream));
    PTEBD_HIP(hipStreamSynchronize(M->stream));
  });
  if (st) {
    mps_free(M);
    return st;
  }
  *out = M;
  return TEBD_OK;
}

tebd_status mps_sweep_stats(const tebd_mps* M, int64_t* last, int64_t* total) {
  if (!M || !last || !total) return fail(TEBD_EINVAL, "NULL argument");
  ptebd::sweep_stats(M, last, total);
  return TEBD_OK;
}

tebd_status mps_trunc_stats(const tebd_mps* M, int64_t* counts) {
  if (!M || !counts) return fail(TEBD_EINVAL, "NULL argument");
  ptebd::trunc_stats(M, counts);
  return TEBD_OK;
}

tebd_status mps_footprint(const tebd_model* model, const tebd_opts* opts, size_t* bytes) {
  if (!bytes) return fail(TEBD_EINVAL, "bytes is NULL");
  tebd_status st = check_model(model);
  if (st) return st;
  st = check_opts(opts, model->d);
  if (st) return st;
  if (opts->supersite) {
    if (model->L % 2 != 0 || model->L < 4)
      return fail(TEBD_EINVAL, "a super-site chain needs an even number of physical sites, at least 4");
    const int Ls = model->L / 2;
    *bytes = ptebd::plan_sizes2(Ls, model->d * model->d, opts->chi_max)
                 .bytes(ptebd::auto_workers(Ls, opts->workers, true, opts->u1 != 0), opts->u1 != 0);   // fuse is 0 here
    return TEBD_OK;
  }
  const bool fuse = opts->fuse != 0;
  *bytes = ptebd::plan_sizes(model->L, model->d, opts->chi_max)
               .bytes(ptebd::auto_workers(model->L, opts->workers, false, opts->u1 != 0, fuse), opts->u1 != 0, fuse);
  return TEBD_OK;
}

tebd_status tebd_prepare(tebd_mps* M, double dt) {
  tebd_status st = usable(M);
  if (st) return st;
  if (!std::isfinite(dt)) return fail(TEBD_EINVAL, "dt must be finite");
  return guard([&] {
    ptebd::prepare_gates(M, 0, 0.5 * dt);
    if (M->super) {
      ptebd::prepare_gates(M, 1, dt);
      return;
    }
    ptebd::prepare_gates(M, 1, 0.5 * dt);
    ptebd::prepare_gates(M, 2, dt);
  });
}

tebd_status mps_canonicalize(tebd_mps* M) {
  tebd_status st = usable(M);
  if (st) return st;
  ProfBind pb(M);
  return guard([&] { ptebd::canonicalize(M); });
}

tebd_status mps_profile(tebd_mps* M, int32_t enable) {
  if (!M) return fail(TEBD_EINVAL, "handle is NULL");
  return guard([&] {
    PTEBD_HIP(hipStreamSynchronize(M->stream));
    if (enable)
      M->prof.start(M->stream);
    else
      M->prof.fold(true);
    M->prof_on = enable != 0;
  });
}

tebd_status mps_profile_read(tebd_mps* M, int32_t kclass, double* ms, int64_t* launches, double* flops) {
  if (!M || !ms || !launches || !flops) return fail(TEBD_EINVAL, "NULL argument");
  if (kclass < 0 || kclass >= ptebd::K_NCLASS) return fail(TEBD_EINVAL, "unknown kernel class");
  return guard([&] {
    // the handle's stream follows every worker stream at the end of a call
    PTEBD_HIP(hipStreamSynchronize(M->stream));
    M->prof.fold(true);
    *ms = M->prof.ms[kclass];
    *launches = M->prof.launches[kclass];
    *flops = M->prof.flops[kclass];
  });
}

tebd_status mps_profile_busy(tebd_mps* M, int32_t kclass, double* busy_ms) {
  if (!M || !busy_ms) return fail(TEBD_EINVAL, "NULL argument");
  if (kclass < 0 || kclass >= ptebd::K_NCLASS) return fail(TEBD_EINVAL, "unknown kernel class");
  return guard([&] {
    PTEBD_HIP(hipStreamSynchronize(M->stream));
    M->prof.fold(true);
    *busy_ms = M->prof.busy_ms(kclass);
  });
}

extern "C" tebd_status tebd_diag_profile_sites(tebd_mps* M, char* out, int64_t cap) {
  if (!M || !out || cap < 1) return fail(TEBD_EINVAL, "NULL argument");
  return guard([&] {
    PTEBD_HIP(hipStreamSynchronize(M->stream));
    M->prof.fold(true);
    std::string txt;
    for (const auto& kv : M->prof.by_tag) {
      char line[160];
      std::snprintf(line, sizeof(line), "%s %lld %.6f %.6e\n", kv.first.c_str(), (long long)kv.second.launches,
                    kv.second.ms, kv.second.flops);
      txt += line;
    }
    if ((int64_t)txt.size() + 1 > cap) throw ptebd::Error(TEBD_EINVAL, "output buffer too small");
    std::memcpy(out, txt.c_str(), txt.size() + 1);
  });
}

extern "C" tebd_status tebd_diag_tile_tuner(int64_t* counts) {
  if (!counts) return fail(TEBD_EINVAL, "NULL argument");
  ptebd::TileTuner& T = ptebd::tile_tuner();
  std::lock_guard<std::mutex> lk(T.mu);
  counts[0] = T.shapes_tuned;
  counts[1] = T.launches_64;
  counts[2] = T.launches_128;
  return TEBD_OK;
}

tebd_status mps_sync(tebd_mps* M) {
  if (!M) return fail(TEBD_EINVAL, "handle is NULL");
  return guard([&] { PTEBD_HIP(hipStreamSynchronize(M->stream)); });
}

tebd_status mps_free(tebd_mps* M) {
  if (!M) return TEBD_OK;
  tebd_status st = guard([&] { ptebd::mps_release(M); });
  if (M->own_stream) (void)hipStreamDestroy(M->stream);
  delete M;
  return st;
}

const char* tebd_last_error(void) { return g_err.c_str(); }

}  // extern "C"
