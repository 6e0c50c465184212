// C ABI of the hps library (include/hps.h).  Argument checking, call-order
// state and error capture; the work is in the host modules and device.hip.
#include <dlfcn.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <new>
#include <sstream>
#include <thread>

#include "device.h"
#include "hps_internal.h"

struct hps_ctx {
  int device = -1;
  void *stream = nullptr;
  std::string err;
  hps_params params{};
  bool have_params = false;
  hps::Mesh mesh;
  bool have_mesh = false;
  hps::HMatrix H;
  bool have_h = false;
  hps::Plan plan;
  bool have_setup = false;
  std::unique_ptr<hps::DeviceState> dev;
  double build_ms = 0.0, symbolic_ms = 0.0, setup_ms = 0.0;
  // batch of independent problems (n_prob > 0): per-problem meshes and
  // H-matrices, merged into mesh / H above once all are present
  int32_t n_prob = 0;
  std::vector<hps::Mesh> pmesh;
  std::vector<hps::HMatrix> pH;
  std::vector<char> pmesh_ok, pH_ok;
  std::vector<int64_t> nseg, gseg;   // unknown / group offsets per problem
  int32_t problems() const { return n_prob > 0 ? n_prob : 1; }
};

namespace {

thread_local std::string g_create_error;

hps_status fail(hps_ctx *c, hps_status s, const std::string &m) {
  if (c) c->err = m;
  return s;
}

template <class F>
hps_status guarded(hps_ctx *c, F &&f) {
  try {
    c->err.clear();
    return f();
  } catch (const hps::Error &e) {
    return fail(c, e.code, e.msg);
  } catch (const std::bad_alloc &) {
    return fail(c, HPS_ENOMEM, "host allocation failed");
  } catch (const std::exception &e) {
    return fail(c, HPS_EINVAL, e.what());
  } catch (...) {
    return fail(c, HPS_EINVAL, "unknown error");
  }
}

hps_status check_params(hps_ctx *c, const hps_params *p) {
  if (!p) return fail(c, HPS_EINVAL, "params is NULL");
  if (!(p->freq_hz > 0.0) || !std::isfinite(p->freq_hz)) return fail(c, HPS_EINVAL, "freq_hz must be > 0");
  if (p->leaf_max < 1) return fail(c, HPS_EINVAL, "leaf_max must be >= 1");
  if (p->leaf_max > 1024) return fail(c, HPS_EINVAL, "leaf_max must be <= 1024");
  if (!(p->aca_tol > 0.0 && p->aca_tol < 1.0)) return fail(c, HPS_EINVAL, "aca_tol must be in (0, 1)");
  if (p->terms < 1) return fail(c, HPS_EINVAL, "terms must be >= 1");
  if (p->refine_passes < 0) return fail(c, HPS_EINVAL, "refine_passes must be >= 0");
  if (p->precision < 0 || p->precision > 2) return fail(c, HPS_EINVAL, "precision must be 0, 1 or 2");
  if (p->ordering != 0 && p->ordering != 1) return fail(c, HPS_EINVAL, "ordering must be 0 or 1");
  if (p->graphs < 0 || p->graphs > 2) return fail(c, HPS_EINVAL, "graphs must be 0, 1 or 2");
  if (!(p->leaf_box_min >= 0.0) || !std::isfinite(p->leaf_box_min))
    return fail(c, HPS_EINVAL, "leaf_box_min must be >= 0");
  if (!(p->series_tol >= 0.0) || !std::isfinite(p->series_tol))
    return fail(c, HPS_EINVAL, "series_tol must be >= 0");
  if (!(p->eta >= 0.0) || !std::isfinite(p->eta)) return fail(c, HPS_EINVAL, "eta must be >= 0");
  if (p->formulation != 0 && p->formulation != 1) return fail(c, HPS_EINVAL, "formulation must be 0 or 1");
  if (p->formulation == 1 && !(p->cfie_alpha >= 0.0 && p->cfie_alpha <= 1.0))
    return fail(c, HPS_EINVAL, "cfie_alpha must be in [0, 1]");
  if (p->formulation == 1 && c && c->have_mesh) {
    bool open = c->mesh.open;
    for (size_t q = 0; q < c->pmesh.size(); ++q) open = open || (c->pmesh_ok[q] && c->pmesh[q].open);
    if (open) return fail(c, HPS_EINVAL, "the CFIE needs a closed surface (the MFIE part holds on closed surfaces only)");
  }
  return HPS_OK;
}

void single_segments(hps_ctx *c) {
  c->nseg = {0, c->H.N};
  c->gseg = {0, c->H.M};
}

void merge_batch(hps_ctx *c) {
  hps::Mesh m;
  hps::HMatrix H;
  hps::merge_problems(c->pmesh, c->pH, m, H, c->nseg, c->gseg);
  c->mesh = std::move(m);
  c->H = std::move(H);
}

// Checked copy of an H-matrix given as flat arrays (layout in hps.h).
hps::HMatrix read_hmatrix(int64_t N, const int64_t *perm, int64_t M, const int64_t *group_ptr, int64_t n_near,
                                 const int32_t *near_ts, const int64_t *near_off, const double *near_vals,
                                 int64_t n_far, const int64_t *far_rng, const int32_t *far_rank,
                                 const int64_t *far_off, const double *far_uv, bool nonsym) {
  if (!perm || !group_ptr || M <= 0 || n_near <= 0 || !near_ts || !near_off || !near_vals)
    throw hps::Error{HPS_EINVAL, "missing near-field arrays"};
  if (n_far < 0 || (n_far > 0 && (!far_rng || !far_rank || !far_off || !far_uv)))
    throw hps::Error{HPS_EINVAL, "missing far-field arrays"};
  hps::HMatrix H;
  H.N = N;
  H.M = M;
  H.nonsym = nonsym;
  H.perm.assign(perm, perm + N);
  std::vector<char> seen(N, 0);
  for (int64_t i = 0; i < N; ++i) {
    if (perm[i] < 0 || perm[i] >= N || seen[perm[i]]) throw hps::Error{HPS_EINVAL, "perm is not a permutation"};
    seen[perm[i]] = 1;
  }
  H.gptr.assign(group_ptr, group_ptr + M + 1);
  if (H.gptr[0] != 0 || H.gptr[M] != N) throw hps::Error{HPS_EINVAL, "group_ptr must span [0, N)"};
  for (int64_t g = 0; g < M; ++g) {
    const int64_t sz = H.gptr[g + 1] - H.gptr[g];
    if (sz < 1) throw hps::Error{HPS_EINVAL, "empty group"};
  }
  H.near_ts.assign(near_ts, near_ts + 2 * n_near);
  H.near_off.assign(near_off, near_off + n_near + 1);
  if (near_off[0] != 0) throw hps::Error{HPS_EINVAL, "near_off must start at 0"};
  std::vector<char> diag(M, 0);
  for (int64_t b = 0; b < n_near; ++b) {
    const int64_t t = near_ts[2 * b], s = near_ts[2 * b + 1];
    if (t < 0 || s < 0 || t >= M || s >= M || (t > s && !nonsym)) throw hps::Error{HPS_EINVAL, "bad near pair"};
    if (near_off[b + 1] - near_off[b] != (H.gptr[t + 1] - H.gptr[t]) * (H.gptr[s + 1] - H.gptr[s]))
      throw hps::Error{HPS_EINVAL, "near_off does not match the block sizes"};
    if (t == s) diag[t] = 1;
  }
  for (int64_t g = 0; g < M; ++g)
    if (!diag[g]) throw hps::Error{HPS_EINVAL, "every group needs its diagonal near block"};
  const int64_t ne = near_off[n_near];
  H.near_vals.resize(ne);
  std::memcpy((void *)H.near_vals.data(), near_vals, ne * sizeof(hps::cplx));
  H.far_off.assign(1, 0);
  if (n_far > 0) {
    H.far_rng.assign(far_rng, far_rng + 4 * n_far);
    H.far_rank.assign(far_rank, far_rank + n_far);
    H.far_off.assign(far_off, far_off + n_far + 1);
    if (far_off[0] != 0) throw hps::Error{HPS_EINVAL, "far_off must start at 0"};
  }
  for (int64_t b = 0; b < n_far; ++b) {
    const int64_t m = far_rng[4 * b + 1] - far_rng[4 * b], n = far_rng[4 * b + 3] - far_rng[4 * b + 2];
    if (m <= 0 || n <= 0 || far_rng[4 * b] < 0 || far_rng[4 * b + 3] > N || far_rng[4 * b + 1] > N ||
        far_rng[4 * b + 2] < 0 || far_rank[b] < 0 || far_off[b + 1] - far_off[b] != (int64_t)far_rank[b] * (m + n))
      throw hps::Error{HPS_EINVAL, "bad far block"};
  }
  const int64_t fe = n_far > 0 ? far_off[n_far] : 0;
  H.far_uv.resize(fe);
  if (fe) std::memcpy((void *)H.far_uv.data(), far_uv, fe * sizeof(hps::cplx));
  hps::split_groups(H, hps::kMaxPivot);
  return H;
}

double now_ms() {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

}  // namespace

extern "C" {

hps_status hps_params_default(hps_params *p) {
  if (!p) return HPS_EINVAL;
  std::memset(p, 0, sizeof(*p));
  p->freq_hz = 0.0;
  p->leaf_max = 128;
  p->aca_tol = 1e-3;
  p->precision = 0;
  p->terms = 2;
  p->refine_passes = 0;
  p->ratio_warn = 0.1;
  p->device_mem_cap = 0;
  p->host_threads = 0;
  p->ordering = 0;
  p->graphs = 1;
  p->verbose = 0;
  p->leaf_box_min = 0.0;
  p->series_tol = 0.0;
  p->host_near = 0;
  p->formulation = 0;
  p->cfie_alpha = 0.5;
  p->eta = 2.0;
  return HPS_OK;
}

// <directory of this library>/tuning/gfx950.json, or "" when unknown.
static std::string default_tuning_path() {
  Dl_info info;
  if (!dladdr((void *)&hps_create, &info) || !info.dli_fname) return "";
  std::string lib(info.dli_fname);
  const size_t slash = lib.rfind('/');
  return (slash == std::string::npos ? std::string(".") : lib.substr(0, slash)) + "/tuning/gfx950.json";
}

hps_status hps_create(hps_ctx **out, int device, void *stream) {
  if (!out) return HPS_EINVAL;
  *out = nullptr;
  hps_ctx *c = new (std::nothrow) hps_ctx();
  if (!c) return HPS_ENOMEM;
  c->device = device;
  c->stream = stream;
  if (device >= 0) {
    hps_status st = guarded(c, [&]() {
      c->dev.reset(new hps::DeviceState(device, stream));
      // the tile-shape table written by the autotuner, if the library's
      // directory holds one (tuning/gfx950.json next to libhps.so)
      const std::string path = default_tuning_path();
      if (!path.empty()) {
        FILE *f = std::fopen(path.c_str(), "rb");
        if (f) {
          std::fclose(f);
          c->dev->set_tuning(hps::read_tuning(path), path);
        }
      }
      return HPS_OK;
    });
    if (st != HPS_OK) {
      g_create_error = c->err;
      delete c;
      return st;
    }
  }
  *out = c;
  return HPS_OK;
}

void hps_destroy(hps_ctx *c) {
  if (!c) return;
  try {
    c->dev.reset();
  } catch (...) {
  }
  delete c;
}

const char *hps_last_error(const hps_ctx *c) { return c ? c->err.c_str() : g_create_error.c_str(); }

static hps_status set_mesh(hps_ctx *c, const double *xyz, int64_t nv, const int32_t *tri, int64_t nt, bool open) {
  if (!c) return HPS_EINVAL;
  if (c->n_prob) return fail(c, HPS_EINVAL, "batch context: use hps_batch_set_mesh");
  if (!xyz || !tri || nv <= 0 || nt <= 0) return fail(c, HPS_EINVAL, "empty mesh");
  return guarded(c, [&]() {
    hps::Mesh m;
    m.nv = nv;
    m.nt = nt;
    m.xyz.assign(xyz, xyz + 3 * nv);
    m.tri.assign(tri, tri + 3 * nt);
    hps::build_rwg(m, open);
    c->mesh = std::move(m);
    c->have_mesh = true;
    c->have_h = false;
    c->have_setup = false;
    return HPS_OK;
  });
}

hps_status hps_set_mesh(hps_ctx *c, const double *xyz, int64_t nv, const int32_t *tri, int64_t nt) {
  return set_mesh(c, xyz, nv, tri, nt, false);
}

hps_status hps_set_open_mesh(hps_ctx *c, const double *xyz, int64_t nv, const int32_t *tri, int64_t nt) {
  return set_mesh(c, xyz, nv, tri, nt, true);
}

hps_status hps_num_unknowns(const hps_ctx *c, int64_t *N) {
  if (!c || !N) return HPS_EINVAL;
  if (!c->have_mesh) return HPS_ESTATE;
  if (c->n_prob) {
    int64_t t = 0;
    for (const hps::Mesh &m : c->pmesh) t += m.N;
    *N = t;
  } else {
    *N = c->mesh.N;
  }
  return HPS_OK;
}

hps_status hps_batch_create(hps_ctx **out, int device, void *stream, int32_t n_problems) {
  if (!out) return HPS_EINVAL;
  *out = nullptr;
  if (n_problems < 1 || n_problems > 65535) {
    g_create_error = "n_problems must be in [1, 65535]";
    return HPS_EINVAL;
  }
  hps_status st = hps_create(out, device, stream);
  if (st != HPS_OK) return st;
  hps_ctx *c = *out;
  try {
    c->n_prob = n_problems;
    c->pmesh.resize(n_problems);
    c->pH.resize(n_problems);
    c->pmesh_ok.assign(n_problems, 0);
    c->pH_ok.assign(n_problems, 0);
  } catch (...) {
    hps_destroy(c);
    *out = nullptr;
    g_create_error = "host allocation failed";
    return HPS_ENOMEM;
  }
  return HPS_OK;
}

hps_status hps_num_problems(const hps_ctx *c, int32_t *n_problems) {
  if (!c || !n_problems) return HPS_EINVAL;
  *n_problems = c->problems();
  return HPS_OK;
}

hps_status hps_problem_unknowns(const hps_ctx *c, int32_t p, int64_t *N) {
  if (!c || !N || p < 0 || p >= c->problems()) return HPS_EINVAL;
  if (c->n_prob) {
    if (!c->pmesh_ok[p]) return HPS_ESTATE;
    *N = c->pmesh[p].N;
  } else {
    if (!c->have_mesh) return HPS_ESTATE;
    *N = c->mesh.N;
  }
  return HPS_OK;
}

hps_status hps_batch_set_mesh(hps_ctx *c, int32_t p, const double *xyz, int64_t nv, const int32_t *tri, int64_t nt) {
  if (!c) return HPS_EINVAL;
  if (!c->n_prob) return fail(c, HPS_EINVAL, "not a batch context: use hps_set_mesh");
  if (p < 0 || p >= c->n_prob) return fail(c, HPS_EINVAL, "problem index out of range");
  if (!xyz || !tri || nv <= 0 || nt <= 0) return fail(c, HPS_EINVAL, "empty mesh");
  return guarded(c, [&]() {
    hps::Mesh m;
    m.nv = nv;
    m.nt = nt;
    m.xyz.assign(xyz, xyz + 3 * nv);
    m.tri.assign(tri, tri + 3 * nt);
    hps::build_rwg(m);
    c->pmesh[p] = std::move(m);
    c->pmesh_ok[p] = 1;
    c->pH_ok[p] = 0;
    c->pH[p] = hps::HMatrix();
    c->have_mesh = std::all_of(c->pmesh_ok.begin(), c->pmesh_ok.end(), [](char x) { return x != 0; });
    c->have_h = false;
    c->have_setup = false;
    return HPS_OK;
  });
}

hps_status hps_batch_set_hmatrix(hps_ctx *c, int32_t p, const hps_params *prm, int64_t N, const int64_t *perm,
                                 int64_t M, const int64_t *group_ptr, int64_t n_near, const int32_t *near_ts,
                                 const int64_t *near_off, const double *near_vals, int64_t n_far,
                                 const int64_t *far_rng, const int32_t *far_rank, const int64_t *far_off,
                                 const double *far_uv) {
  if (!c) return HPS_EINVAL;
  if (!c->n_prob) return fail(c, HPS_EINVAL, "not a batch context: use hps_set_hmatrix");
  if (p < 0 || p >= c->n_prob) return fail(c, HPS_EINVAL, "problem index out of range");
  if (!c->pmesh_ok[p]) return fail(c, HPS_ESTATE, "hps_batch_set_mesh for this problem first");
  hps_status st = check_params(c, prm);
  if (st != HPS_OK) return st;
  if (N != c->pmesh[p].N) return fail(c, HPS_EINVAL, "N does not match the mesh of this problem");
  for (int32_t q = 0; q < c->n_prob; ++q)
    if (c->pH_ok[q] && q != p && std::memcmp(&c->params, prm, sizeof(hps_params)) != 0)
      return fail(c, HPS_EINVAL, "every problem of a batch takes the same parameters");
  return guarded(c, [&]() {
    hps::HMatrix H = read_hmatrix(N, perm, M, group_ptr, n_near, near_ts, near_off, near_vals, n_far, far_rng,
                                  far_rank, far_off, far_uv, prm->formulation == 1);
    c->have_h = false;
    c->have_setup = false;
    c->pH[p] = std::move(H);
    c->pH_ok[p] = 1;
    c->params = *prm;
    c->have_params = true;
    if (c->have_mesh && std::all_of(c->pH_ok.begin(), c->pH_ok.end(), [](char x) { return x != 0; })) {
      merge_batch(c);
      if (c->dev) c->dev->upload(c->mesh, c->H, *prm, c->nseg);
      c->have_h = true;
    }
    return HPS_OK;
  });
}

hps_status hps_build_hmatrix(hps_ctx *c, const hps_params *p) {
  if (!c) return HPS_EINVAL;
  if (!c->have_mesh) return fail(c, HPS_ESTATE, c->n_prob ? "hps_batch_set_mesh for every problem first"
                                                         : "hps_set_mesh first");
  hps_status st = check_params(c, p);
  if (st != HPS_OK) return st;
  return guarded(c, [&]() {
    const double t0 = now_ms();
    c->have_h = false;
    c->have_setup = false;
    if (c->n_prob) {
      for (int32_t q = 0; q < c->n_prob; ++q) {
        hps::HMatrix H;
        const hps::Mesh &mq = c->pmesh[q];
        const hps::NearFill fill = [&](hps::HMatrix &h) { c->dev->near_fill(mq, p->freq_hz, p->formulation, p->cfie_alpha, h); };
        const hps::FarSample sample = [&](const hps::HMatrix &h, const hps::FarEmit &emit) {
          c->dev->far_sample(mq, p->freq_hz, p->formulation, p->cfie_alpha, h, p->aca_tol, emit);
        };
        const bool dev = c->dev && !p->host_near;
        hps::build_hmatrix(mq, *p, H, dev ? &fill : nullptr, dev ? &sample : nullptr);
        hps::split_groups(H, hps::kMaxPivot);
        c->pH[q] = std::move(H);
        c->pH_ok[q] = 1;
      }
      merge_batch(c);
    } else {
      hps::HMatrix H;
      const hps::NearFill fill = [&](hps::HMatrix &h) { c->dev->near_fill(c->mesh, p->freq_hz, p->formulation, p->cfie_alpha, h); };
      const hps::FarSample sample = [&](const hps::HMatrix &h, const hps::FarEmit &emit) {
        c->dev->far_sample(c->mesh, p->freq_hz, p->formulation, p->cfie_alpha, h, p->aca_tol, emit);
      };
      const bool dev = c->dev && !p->host_near;
      hps::build_hmatrix(c->mesh, *p, H, dev ? &fill : nullptr, dev ? &sample : nullptr);
      hps::split_groups(H, hps::kMaxPivot);
      c->H = std::move(H);
      single_segments(c);
    }
    c->params = *p;
    c->have_params = true;
    if (c->dev) c->dev->upload(c->mesh, c->H, *p, c->nseg);
    c->have_h = true;
    c->build_ms = now_ms() - t0;
    return HPS_OK;
  });
}

hps_status hps_set_hmatrix(hps_ctx *c, const hps_params *p, int64_t N, const int64_t *perm, int64_t M,
                           const int64_t *group_ptr, int64_t n_near, const int32_t *near_ts, const int64_t *near_off,
                           const double *near_vals, int64_t n_far, const int64_t *far_rng, const int32_t *far_rank,
                           const int64_t *far_off, const double *far_uv) {
  if (!c) return HPS_EINVAL;
  if (c->n_prob) return fail(c, HPS_EINVAL, "batch context: use hps_batch_set_hmatrix");
  if (!c->have_mesh) return fail(c, HPS_ESTATE, "hps_set_mesh first");
  hps_status st = check_params(c, p);
  if (st != HPS_OK) return st;
  if (N != c->mesh.N) return fail(c, HPS_EINVAL, "N does not match the mesh");
  return guarded(c, [&]() {
    hps::HMatrix H = read_hmatrix(N, perm, M, group_ptr, n_near, near_ts, near_off, near_vals, n_far, far_rng,
                                  far_rank, far_off, far_uv, p->formulation == 1);
    c->have_h = false;
    c->have_setup = false;
    c->H = std::move(H);
    single_segments(c);
    c->params = *p;
    c->have_params = true;
    if (c->dev) c->dev->upload(c->mesh, c->H, *p, c->nseg);
    c->have_h = true;
    return HPS_OK;
  });
}

hps_status hps_hmatrix_sizes(const hps_ctx *c, int64_t *M, int64_t *n_near, int64_t *n_far, int64_t *near_elems,
                             int64_t *far_elems) {
  if (!c) return HPS_EINVAL;
  if (!c->have_h) return HPS_ESTATE;
  if (M) *M = c->H.M;
  if (n_near) *n_near = c->H.n_near();
  if (n_far) *n_far = c->H.n_far();
  if (near_elems) *near_elems = (int64_t)c->H.near_vals.size();
  if (far_elems) *far_elems = (int64_t)c->H.far_uv.size();
  return HPS_OK;
}

hps_status hps_get_hmatrix(const hps_ctx *c, int64_t *perm, int64_t *group_ptr, int32_t *near_ts, int64_t *near_off,
                           double *near_vals, int64_t *far_rng, int32_t *far_rank, int64_t *far_off,
                           double *far_uv) {
  if (!c) return HPS_EINVAL;
  if (!c->have_h) return HPS_ESTATE;
  const hps::HMatrix &H = c->H;
  if (perm) std::memcpy(perm, H.perm.data(), H.perm.size() * 8);
  if (group_ptr) std::memcpy(group_ptr, H.gptr.data(), H.gptr.size() * 8);
  if (near_ts) std::memcpy(near_ts, H.near_ts.data(), H.near_ts.size() * 4);
  if (near_off) std::memcpy(near_off, H.near_off.data(), H.near_off.size() * 8);
  if (near_vals) std::memcpy(near_vals, H.near_vals.data(), H.near_vals.size() * 16);
  if (far_rng) std::memcpy(far_rng, H.far_rng.data(), H.far_rng.size() * 8);
  if (far_rank) std::memcpy(far_rank, H.far_rank.data(), H.far_rank.size() * 4);
  if (far_off) std::memcpy(far_off, H.far_off.data(), H.far_off.size() * 8);
  if (far_uv) std::memcpy(far_uv, H.far_uv.data(), H.far_uv.size() * 16);
  return HPS_OK;
}

hps_status hps_rwg(const hps_ctx *c, int32_t *edge_v, int32_t *tri_pm, int32_t *free_v) {
  if (!c) return HPS_EINVAL;
  if (!c->have_mesh) return HPS_ESTATE;
  std::vector<const hps::Mesh *> ms;
  if (c->n_prob)
    for (const hps::Mesh &m : c->pmesh) ms.push_back(&m);
  else
    ms.push_back(&c->mesh);
  int64_t o = 0, voff = 0, toff = 0;
  for (const hps::Mesh *m : ms) {
    for (int64_t n = 0; n < m->N; ++n, ++o) {
      if (edge_v) {
        edge_v[2 * o] = (int32_t)(m->edge[2 * n] + voff);
        edge_v[2 * o + 1] = (int32_t)(m->edge[2 * n + 1] + voff);
      }
      if (tri_pm) {
        tri_pm[2 * o] = (int32_t)(m->tp[n] + toff);
        tri_pm[2 * o + 1] = (int32_t)(m->tm[n] + toff);
      }
      if (free_v) {
        free_v[2 * o] = (int32_t)(m->vp[n] + voff);
        free_v[2 * o + 1] = (int32_t)(m->vm[n] + voff);
      }
    }
    voff += m->nv;
    toff += m->nt;
  }
  return HPS_OK;
}

namespace {

const char kHmatMagic[8] = {'H', 'P', 'S', 'H', 'M', 'A', 'T', '1'};

struct File {
  std::FILE *f = nullptr;
  ~File() {
    if (f) std::fclose(f);
  }
};

}  // namespace

hps_status hps_export_hmatrix(const hps_ctx *cc, const char *path) {
  if (!cc) return HPS_EINVAL;
  hps_ctx *c = const_cast<hps_ctx *>(cc);     // only the error text is written
  if (!path) return fail(c, HPS_EINVAL, "path is NULL");
  if (c->n_prob) return fail(c, HPS_EINVAL, "batch context: export the problems one by one");
  if (!c->have_h) return fail(c, HPS_ESTATE, "no H-matrix installed");
  return guarded(c, [&]() {
    const hps::HMatrix &H = c->H;
    const std::string name(path);
    File out;
    out.f = std::fopen(name.c_str(), "wb");
    if (!out.f) throw hps::Error{HPS_EIO, "cannot open " + name + " for writing"};
    bool ok = std::fwrite(kHmatMagic, 1, 8, out.f) == 8;
    const int64_t hdr[8] = {H.N, H.M, H.n_near(), (int64_t)H.near_vals.size(), H.n_far(),
                            (int64_t)H.far_uv.size(), H.nonsym ? 1 : 0, (int64_t)sizeof(hps_params)};
    ok = ok && std::fwrite(hdr, 8, 8, out.f) == 8;
    ok = ok && std::fwrite(&c->params, sizeof(hps_params), 1, out.f) == 1;
    auto put = [&](const void *p, size_t bytes) {
      ok = ok && (bytes == 0 || std::fwrite(p, 1, bytes, out.f) == bytes);
    };
    put(H.perm.data(), H.perm.size() * 8);
    put(H.gptr.data(), H.gptr.size() * 8);
    put(H.near_ts.data(), H.near_ts.size() * 4);
    put(H.near_off.data(), H.near_off.size() * 8);
    put(H.near_vals.data(), H.near_vals.size() * 16);
    put(H.far_rng.data(), H.far_rng.size() * 8);
    put(H.far_rank.data(), H.far_rank.size() * 4);
    put(H.far_off.data(), H.far_off.size() * 8);
    put(H.far_uv.data(), H.far_uv.size() * 16);
    ok = ok && std::fflush(out.f) == 0;
    const int rc = std::fclose(out.f);
    out.f = nullptr;
    if (!ok || rc != 0) throw hps::Error{HPS_EIO, "write to " + name + " failed"};
    return HPS_OK;
  });
}

hps_status hps_import_hmatrix(hps_ctx *c, const char *path) {
  if (!c) return HPS_EINVAL;
  if (!path) return fail(c, HPS_EINVAL, "path is NULL");
  if (c->n_prob) return fail(c, HPS_EINVAL, "batch context: use hps_batch_set_hmatrix");
  if (!c->have_mesh) return fail(c, HPS_ESTATE, "hps_set_mesh first");
  hps_params prm{};
  std::vector<int64_t> perm, gptr, near_off, far_rng, far_off;
  std::vector<int32_t> near_ts, far_rank;
  std::vector<double> near_vals, far_uv;
  int64_t hdr[8] = {0};
  {
    File in;
    in.f = std::fopen(path, "rb");
    if (!in.f) return fail(c, HPS_EIO, std::string("cannot open ") + path);
    char magic[8];
    if (std::fread(magic, 1, 8, in.f) != 8 || std::memcmp(magic, kHmatMagic, 8) != 0)
      return fail(c, HPS_EIO, std::string(path) + " is not an H-matrix file");
    if (std::fread(hdr, 8, 8, in.f) != 8) return fail(c, HPS_EIO, std::string(path) + ": truncated header");
    const int64_t N = hdr[0], M = hdr[1], nn = hdr[2], ne = hdr[3], nf = hdr[4], fe = hdr[5];
    if (hdr[7] != (int64_t)sizeof(hps_params))
      return fail(c, HPS_EIO, std::string(path) + ": written with another hps_params layout");
    if (N != c->mesh.N) return fail(c, HPS_EINVAL, "N of the file does not match the mesh");
    if (M < 1 || M > N || nn < 1 || ne < 1 || nf < 0 || fe < 0 || (hdr[6] != 0 && hdr[6] != 1))
      return fail(c, HPS_EIO, std::string(path) + ": bad header");
    // sizes against the file length before allocating
    const long here = std::ftell(in.f);
    if (here < 0 || std::fseek(in.f, 0, SEEK_END) != 0) return fail(c, HPS_EIO, "cannot seek in " + std::string(path));
    const long end = std::ftell(in.f);
    if (std::fseek(in.f, here, SEEK_SET) != 0) return fail(c, HPS_EIO, "cannot seek in " + std::string(path));
    const double need = (double)sizeof(hps_params) + 8.0 * (N + M + 1 + nn + 1 + 4 * nf + nf + 1) + 4.0 * (2 * nn + nf) +
                        16.0 * ((double)ne + (double)fe);
    if ((double)(end - here) != need) return fail(c, HPS_EIO, std::string(path) + ": truncated or oversized");
    bool ok = std::fread(&prm, sizeof(hps_params), 1, in.f) == 1;
    hps_status st = guarded(c, [&]() {
      perm.resize(N); gptr.resize(M + 1); near_ts.resize(2 * nn); near_off.resize(nn + 1);
      near_vals.resize(2 * ne); far_rng.resize(4 * nf); far_rank.resize(nf); far_off.resize(nf + 1);
      far_uv.resize(2 * fe);
      return HPS_OK;
    });
    if (st != HPS_OK) return st;
    auto get = [&](void *p, size_t bytes) { ok = ok && (bytes == 0 || std::fread(p, 1, bytes, in.f) == bytes); };
    get(perm.data(), perm.size() * 8);
    get(gptr.data(), gptr.size() * 8);
    get(near_ts.data(), near_ts.size() * 4);
    get(near_off.data(), near_off.size() * 8);
    get(near_vals.data(), near_vals.size() * 8);
    get(far_rng.data(), far_rng.size() * 8);
    get(far_rank.data(), far_rank.size() * 4);
    get(far_off.data(), far_off.size() * 8);
    get(far_uv.data(), far_uv.size() * 8);
    if (!ok) return fail(c, HPS_EIO, std::string(path) + ": read failed");
  }
  if ((prm.formulation == 1) != (hdr[6] == 1)) return fail(c, HPS_EIO, std::string(path) + ": inconsistent symmetry flag");
  // offsets of the file must stay inside the arrays read
  if (near_off.back() != hdr[3] || far_off.back() != hdr[5]) return fail(c, HPS_EIO, std::string(path) + ": offsets do not match the sizes");
  return hps_set_hmatrix(c, &prm, hdr[0], perm.data(), hdr[1], gptr.data(), hdr[2], near_ts.data(), near_off.data(),
                         near_vals.data(), hdr[4], far_rng.data(), far_rank.data(), far_off.data(), far_uv.data());
}

// Device bytes a setup with plan P holds: the H-matrix (near blocks, far
// factors, excitation quadrature data), the working and factor panel sets
// (both triangles for a non-symmetric field) and, in the precision form, the
// FP32 panels, FP32 near blocks and the FP32 and 16-bit far factors.
static uint64_t plan_device_bytes(const hps::Plan &P, const hps::HMatrix &H, const hps_params &prm) {
  const uint64_t near = H.near_vals.size(), far = H.far_uv.size();
  const uint64_t pe = (uint64_t)std::max<int64_t>(P.panel_elems, 1) * (H.nonsym ? 2 : 1);
  uint64_t b = 16 * (near + far) + (uint64_t)H.N * 14 * 10 * 8 + 2 * 16 * pe;
  if (prm.precision > 0) b += 8 * pe + 8 * near + 8 * far + 4 * far + 8 * (uint64_t)H.n_far();
  return b;
}

hps_status hps_setup(hps_ctx *c) {
  if (!c) return HPS_EINVAL;
  if (!c->have_h) return fail(c, HPS_ESTATE, "install an H-matrix first");
  return guarded(c, [&]() {
    const double t0 = now_ms();
    hps::Plan P;
    hps::make_plan(c->H, c->mesh, c->params.ordering, c->gseg, P);
    const double t1 = now_ms();
    const uint64_t need = plan_device_bytes(P, c->H, c->params);
    if (c->params.device_mem_cap && need > c->params.device_mem_cap)
      throw hps::Error{HPS_ENOMEM, "setup plan needs " + std::to_string(need) + " device bytes, over device_mem_cap " +
                                       std::to_string(c->params.device_mem_cap)};
    if (!c->dev) throw hps::Error{HPS_EDEVICE, "host-only context cannot run the setup"};
    c->dev->times.symbolic_ms = t1 - t0;
    c->have_setup = false;
    c->dev->setup(P, c->H);
    c->plan = std::move(P);
    c->symbolic_ms = t1 - t0;
    c->setup_ms = now_ms() - t0;
    c->dev->times.setup_ms = c->setup_ms;
    c->have_setup = true;
    return HPS_OK;
  });
}

static hps_status ratio_status(const hps_ctx *c, int64_t R, const double *ratio) {
  if (!ratio) return HPS_OK;
  for (int64_t r = 0; r < R; ++r)
    if (!(ratio[r] < c->params.ratio_warn)) return HPS_WRATIO;
  return HPS_OK;
}

hps_status hps_solve_planewaves(hps_ctx *c, int64_t R, const double *khat, const double *pol, void *X, double *rcs,
                                double *ratio) {
  if (!c) return HPS_EINVAL;
  if (!c->have_setup) return fail(c, HPS_ESTATE, "hps_setup first");
  if (R <= 0 || !khat || !pol) return fail(c, HPS_EINVAL, "bad plane-wave arguments");
  return guarded(c, [&]() {
    const int64_t RP = R * c->problems();
    std::vector<double> rt(RP);
    c->dev->solve_planewaves(R, khat, pol, X, rcs, rt.data());
    if (ratio) std::memcpy(ratio, rt.data(), RP * sizeof(double));
    return c->params.terms > 1 ? ratio_status(c, RP, rt.data()) : HPS_OK;
  });
}

hps_status hps_solve_rhs(hps_ctx *c, int64_t R, const void *B, void *X, double *ratio) {
  if (!c) return HPS_EINVAL;
  if (!c->have_setup) return fail(c, HPS_ESTATE, "hps_setup first");
  if (R <= 0 || !B || !X || B == X) return fail(c, HPS_EINVAL, "bad RHS arguments");
  return guarded(c, [&]() {
    const int64_t RP = R * c->problems();
    std::vector<double> rt(RP);
    c->dev->solve_rhs(R, B, X, rt.data());
    if (ratio) std::memcpy(ratio, rt.data(), RP * sizeof(double));
    return c->params.terms > 1 ? ratio_status(c, RP, rt.data()) : HPS_OK;
  });
}

hps_status hps_excitation(hps_ctx *c, int64_t R, const double *khat, const double *pol, void *B) {
  if (!c) return HPS_EINVAL;
  if (!c->have_setup) return fail(c, HPS_ESTATE, "hps_setup first");
  if (R <= 0 || !khat || !pol || !B) return fail(c, HPS_EINVAL, "bad plane-wave arguments");
  return guarded(c, [&]() {
    c->dev->excitation(R, khat, pol, B);
    return HPS_OK;
  });
}

hps_status hps_hmatvec(hps_ctx *c, int64_t R, const void *X, void *Y) {
  if (!c) return HPS_EINVAL;
  if (!c->have_setup) return fail(c, HPS_ESTATE, "hps_setup first");
  if (R <= 0 || !X || !Y || X == Y) return fail(c, HPS_EINVAL, "bad matvec arguments");
  return guarded(c, [&]() {
    c->dev->hmatvec(R, X, Y);
    return HPS_OK;
  });
}

hps_status hps_hmatvec_noalloc(hps_ctx *c, int64_t R, const void *X, void *Y) {
  if (!c) return HPS_EINVAL;
  if (!c->have_setup) return fail(c, HPS_ESTATE, "hps_setup first");
  if (R <= 0 || !X || !Y || X == Y) return fail(c, HPS_EINVAL, "bad matvec arguments");
  return guarded(c, [&]() {
    c->dev->hmatvec_noalloc(R, X, Y);
    return HPS_OK;
  });
}

hps_status hps_set_tuning(hps_ctx *c, const char *path) {
  if (!c) return HPS_EINVAL;
  return guarded(c, [&]() {
    // the file is read and checked first, so a bad table is reported as such
    hps::TuneTable t;
    if (path && *path) t = hps::read_tuning(path);
    if (!c->dev) return fail(c, HPS_EDEVICE, "host-only context");
    c->dev->set_tuning(t, (path && *path) ? std::string(path) : std::string("built-in (all 32 x 32)"));
    return HPS_OK;
  });
}

hps_status hps_profile(hps_ctx *c, int enable) {
  if (!c) return HPS_EINVAL;
  if (!c->dev) return fail(c, HPS_EDEVICE, "host-only context");
  return guarded(c, [&]() {
    c->dev->set_profiling(enable != 0);
    return HPS_OK;
  });
}

hps_status hps_stats(const hps_ctx *c, char *buf, size_t len) {
  if (!c || !buf || len == 0) return HPS_EINVAL;
  std::ostringstream o;
  o.precision(9);
  o << "{\"problems\": " << c->problems() << ", \"build_ms\": " << c->build_ms << ", \"setup_ms\": " << c->setup_ms << ", \"symbolic_ms\": " << c->symbolic_ms;
  if (c->have_h) {
    int64_t rsum = 0, rmax = 0;
    for (int32_t r : c->H.far_rank) { rsum += r; rmax = std::max<int64_t>(rmax, r); }
    o << ", \"hmatrix\": {\"N\": " << c->H.N << ", \"groups\": " << c->H.M << ", \"near_blocks\": " << c->H.n_near()
      << ", \"far_blocks\": " << c->H.n_far() << ", \"rank_mean\": "
      << (c->H.n_far() ? (double)rsum / c->H.n_far() : 0.0) << ", \"rank_max\": " << rmax
      << ", \"near_elems\": " << c->H.near_vals.size() << ", \"far_elems\": " << c->H.far_uv.size() << "}";
  }
  if (c->dev) o << ", \"device\": " << c->dev->stats_json();
  o << "}";
  const std::string s = o.str();
  const size_t n = std::min(len - 1, s.size());
  std::memcpy(buf, s.data(), n);
  buf[n] = 0;
  return HPS_OK;
}

}  // extern "C"
