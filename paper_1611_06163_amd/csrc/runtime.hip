// runtime.hip -- host runtime behind the C ABI of include/tdpd.h: parameter
// validation, device buffers, membrane topology, the per-step launch
// sequence, state readback.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "launch_list.h"

using namespace tdpd;

namespace {

struct HostMesh {
  int nv = 0, ntri = 0;
  std::vector<int32_t> tri;
  std::vector<int2> bond_ab;
  std::vector<float2> bond_par;
  std::vector<int32_t> bond_off, bond_inc;
  std::vector<int32_t> tri_off, dih_off;
  std::vector<int4> tri_inc, dih_inc;
  std::vector<uint8_t> dih_role;
  std::vector<float> A0t;
  std::vector<int32_t> ring_off, ring;  // 1-rings, counter-clockwise from the smallest index
  double ell = 0;                       // mean rest edge length
  std::vector<std::pair<int, int>> bfs;  // (vertex, parent) breadth-first order
  double A0 = 0, V0 = 0, theta0 = 0, max_radius = 0;
  tdpd_mesh_params mp{};
  MeshDev dev{};  // device pointers once uploaded
};

static double d_theta(const double *a, const double *b, const double *c, const double *d) {
  // signed angle between the outward normals of (a,b,c) and (d,c,b)
  double ba[3], ca[3], cd[3], bd[3], n1[3], n2[3], e[3], x[3];
  for (int q = 0; q < 3; ++q) {
    ba[q] = b[q] - a[q]; ca[q] = c[q] - a[q];
    cd[q] = c[q] - d[q]; bd[q] = b[q] - d[q];
    e[q] = c[q] - b[q];
  }
  auto cr = [](const double *u, const double *v, double *o) {
    o[0] = u[1] * v[2] - u[2] * v[1];
    o[1] = u[2] * v[0] - u[0] * v[2];
    o[2] = u[0] * v[1] - u[1] * v[0];
  };
  cr(ba, ca, n1);
  cr(cd, bd, n2);
  cr(n1, n2, x);
  const double le = std::sqrt(e[0] * e[0] + e[1] * e[1] + e[2] * e[2]);
  return std::atan2((x[0] * e[0] + x[1] * e[1] + x[2] * e[2]) / le,
                    n1[0] * n2[0] + n1[1] * n2[1] + n1[2] * n2[2]);
}

}  // namespace

struct HostBox {
  float L[3] = {0, 0, 0};
  int nc[3] = {0, 0, 0};
  int64_t ncell = 0, cell_base = 0;
  int64_t gid_base = 0, n = 0;
  uint64_t seed = 0;
  uint32_t box_id = 0;
  float shear = 0.f;  // Lees-Edwards shear rate
};

struct tdpd_sys {
  tdpd_params prm{};
  std::vector<HostBox> boxes;
  BoxDev *d_boxes = nullptr;
  PairConst pc{};
  MembraneConst mc{};
  hipStream_t st = nullptr;
  tdpd_alloc_fn alloc = nullptr;
  tdpd_free_fn free_fn = nullptr;
  void *user = nullptr;
  std::vector<void *> blocks;
  std::string err;

  int64_t n = 0;
  int S = 1;
  int64_t ncell = 0;
  int key_bits = 1;
  bool have_state = false, uploaded = false, forces_valid = false;
  int64_t step = 0;

  // host copies kept until upload
  std::vector<float> h_pos, h_vel, h_conc;
  std::vector<uint32_t> h_flags;
  std::vector<int32_t> h_box, h_body;

  State A{}, B{};
  bool cur_A = true;
  float *F = nullptr, *Q = nullptr;
  uint32_t *keys = nullptr, *vals = nullptr, *keys_tmp = nullptr, *vals_tmp = nullptr;
  uint32_t *keys_s = nullptr, *perm = nullptr, *hist = nullptr, *cell_start = nullptr;
  // gid -> slot of the membrane vertices, one map per state buffer (the
  // binning writes the other one, so kernels on the second stream can read
  // the current one while it runs)
  uint32_t *slot_of_gid = nullptr, *slot_of_gid_b = nullptr;
  unsigned long long *nzero = nullptr, *pair_count = nullptr;
  uint32_t *errw = nullptr;
  double *diag_partial = nullptr, *diag_out = nullptr;
  int device = -1;  // the HIP device current at creation (the stream's)

  std::vector<HostMesh> meshes;
  std::vector<int32_t> rbc_mesh, rbc_box;
  std::vector<int64_t> rbc_first, rbc_voff;
  MeshDev *d_meshes = nullptr;
  int32_t *d_rbc_mesh = nullptr, *d_rbc_box = nullptr;
  int64_t *d_rbc_first = nullptr, *d_rbc_voff = nullptr;
  double *d_av = nullptr, *d_centroid = nullptr;
  int64_t nvert = 0;
  size_t mem_lds = 0;  // dynamic LDS of the membrane kernel
  int pair_kernel = 1;  // 0: one thread per particle, 1: cell-tiled
  bool any_shear = false;  // a box has Lees-Edwards boundaries
  PairTile tile{4, 2, 1, 1};  // shape of the cell-tiled kernel
  int bin_mode = 0;     // 0: counting (one-digit stable) sort, 1: LSD radix sort
  bool use_graph = true;
  // membrane parts inside the scan's and the pair kernel's launches: 1
  // always, 0 never (a kernel of its own on the second stream), -1 by size
  int fuse_membrane = -1;
  int cu_count = 256;  // compute units of the device
  // Verlet neighbour lists (verlet_every > 0): rebuilt with the binning on
  // every verlet_every-th evaluation, pairs taken from them in between
  int verlet_every = 0;
  float verlet_skin = 0.f;
  bool list_valid = false;
  int list_age = 0;  // evaluations made with the current lists
  ListDev ld{};
  uint32_t *kdev = nullptr;       // device step counter read by the kernels
  uint32_t *kstep = nullptr;      // the counter of the current evaluation (second stream)
  uint32_t kdev_val = 0;          // host mirror of *kdev
  uint32_t *cell_count = nullptr, *bin_tmp = nullptr, *tile_sum = nullptr;
  float *Fm = nullptr;            // membrane forces by global vertex [nvert][3]
  float *Fb = nullptr;            // per-bond membrane forces [nrbc][3][bond_stride]
  int64_t bond_stride = 0;
  int max_nv = 0;
  // membrane surrogate (bending + local area from the network)
  bool surr_on = false;
  int surr_every = 0;             // fallback check interval (steps)
  SurrDev sd{};
  float *surr_params = nullptr, *surr_Ha = nullptr, *surr_Hb = nullptr;
  int32_t *d_vcell = nullptr;
  hipStream_t st2 = nullptr, gst = nullptr;  // membrane stream, capture stream
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  // captured steps: [0], [1] one step from buffer parity A / B; [2], [3]
  // kGraphSteps steps from parity A / B (an even count ends at the start parity)
  hipGraph_t graph[4] = {nullptr, nullptr, nullptr, nullptr};
  hipGraphExec_t gexec[4] = {nullptr, nullptr, nullptr, nullptr};
  // event timing per phase (index = log2 of TDPD_PHASE_*)
  int timing_mask = 0;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_pool[4];
  size_t ev_used[4] = {0, 0, 0, 0};

  State &cur() { return cur_A ? A : B; }
  State &nxt() { return cur_A ? B : A; }
  uint32_t *slot_cur() const { return cur_A ? slot_of_gid : slot_of_gid_b; }
  uint32_t *slot_nxt() const { return cur_A ? slot_of_gid_b : slot_of_gid; }

  int fail(int code, const std::string &m) {
    err = m;
    return code;
  }
  void *dalloc(size_t bytes) {
    if (bytes == 0) bytes = 16;
    bytes = (bytes + 255) & ~size_t(255);
    void *p = nullptr;
    if (alloc) {
      p = alloc(bytes, user);
    } else if (hipMalloc(&p, bytes) != hipSuccess) {
      p = nullptr;
    }
    if (p) blocks.push_back(p);
    return p;
  }
  void destroy_graphs() {
    for (int q = 0; q < 4; ++q) {
      if (gexec[q]) (void)hipGraphExecDestroy(gexec[q]);
      if (graph[q]) (void)hipGraphDestroy(graph[q]);
      gexec[q] = nullptr;
      graph[q] = nullptr;
    }
  }
  void destroy_streams() {
    if (ev_fork) (void)hipEventDestroy(ev_fork);
    if (ev_join) (void)hipEventDestroy(ev_join);
    if (st2) (void)hipStreamDestroy(st2);
    if (gst) (void)hipStreamDestroy(gst);
    ev_fork = ev_join = nullptr;
    st2 = gst = nullptr;
  }
  void destroy_events() {
    for (int q = 0; q < 4; ++q) {
      for (auto &e : ev_pool[q]) {
        (void)hipEventDestroy(e.first);
        (void)hipEventDestroy(e.second);
      }
      ev_pool[q].clear();
      ev_used[q] = 0;
    }
  }
  // start/stop a timed phase; returns false if timing is off for it
  bool phase_begin(int q, hipStream_t on) {
    if (!(timing_mask & (1 << q))) return false;
    if (ev_used[q] == ev_pool[q].size()) {
      hipEvent_t a, b;
      if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) return false;
      ev_pool[q].push_back({a, b});
    }
    (void)hipEventRecord(ev_pool[q][ev_used[q]].first, on);
    return true;
  }
  void phase_end(int q, bool enabled, hipStream_t on) {
    if (!enabled) return;
    (void)hipEventRecord(ev_pool[q][ev_used[q]].second, on);
    ++ev_used[q];
  }
  void release_all() {
    for (void *p : blocks) {
      if (free_fn) free_fn(p, user);
      else if (!alloc) (void)hipFree(p);
    }
    blocks.clear();
  }
};

#define HIPCHK(call)                                                                  \
  do {                                                                                \
    hipError_t e_ = (call);                                                           \
    if (e_ != hipSuccess)                                                             \
      return s->fail(TDPD_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

static bool is_finite_f(float v) { return std::isfinite(v); }

static float wrap_host(float x, float L) {
  if (x < 0.f) x += L;
  if (x >= L) x -= L;
  if (x >= L || x < 0.f) x = 0.f;
  return x;
}

// Checks of the parameters shared by every box.
static int check_common(const tdpd_params *p) {
  if (p->n_types < 1 || p->n_types > TDPD_MAX_TYPES || p->n_species < 1 ||
      p->n_species > TDPD_MAX_SPECIES)
    return TDPD_ERR_INVALID_ARG;
  if (!(p->rc > 0.f) || !(p->rcc > 0.f) || !(p->dt > 0.f) || !(p->kT >= 0.f) ||
      !(p->s_exp >= 0.f) || !(p->sc_exp >= 0.f) || !(p->m_s >= 0.f) || !(p->rho >= 0.f))
    return TDPD_ERR_INVALID_ARG;
  if (p->wall_axis < -1 || p->wall_axis > 3) return TDPD_ERR_INVALID_ARG;
  const int T = p->n_types;
  for (int e = 0; e < p->n_species * T; ++e)
    if (!std::isfinite(p->source[e]) || !std::isfinite(p->decay[e])) return TDPD_ERR_INVALID_ARG;
  for (int i = 0; i < T; ++i)
    for (int j = 0; j < T; ++j) {
      const float g = p->gamma[i * T + j], sg = p->sigma[i * T + j];
      if (p->alpha[i * T + j] != p->alpha[j * T + i] || g != p->gamma[j * T + i] ||
          sg != p->sigma[j * T + i] || g < 0.f)
        return TDPD_ERR_INVALID_ARG;
      // fluctuation-dissipation pairing, Eq. (6)
      const double lhs = double(sg) * sg, rhs = 2.0 * p->kT * g;
      if (std::fabs(lhs - rhs) > 1e-4 * std::max(1.0, std::max(lhs, rhs))) return TDPD_ERR_INVALID_ARG;
      for (int sp = 0; sp < p->n_species; ++sp) {
        const float k1 = p->kappa[(sp * T + i) * T + j], k2 = p->kappa[(sp * T + j) * T + i];
        if (k1 != k2 || k1 < 0.f) return TDPD_ERR_INVALID_ARG;
      }
    }
  return TDPD_OK;
}

// Geometry of one box; fails if it holds fewer than 3 cells of edge
// > max(rc, rcc) per axis.
static int make_box(const tdpd_params *p, const tdpd_box &in, HostBox &b) {
  if (in.box_id >= (1u << 24) || !std::isfinite(in.shear_rate)) return TDPD_ERR_INVALID_ARG;
  // sheared boundaries and frozen walls both act on the y faces
  if (in.shear_rate != 0.f && p->wall_axis >= 0) return TDPD_ERR_UNSUPPORTED;
  const float rmax = std::max(p->rc, p->rcc);
  for (int a = 0; a < 3; ++a) {
    if (!(in.box[a] > 0.f)) return TDPD_ERR_INVALID_ARG;
    b.L[a] = in.box[a];
    b.nc[a] = int(std::floor(double(in.box[a]) / (double(rmax) * (1.0 + 1e-4))));
    if (b.nc[a] < 3) return TDPD_ERR_BOX_TOO_SMALL;
  }
  if (p->wall_axis >= 0 && p->wall_axis <= 2 &&
      !(p->wall_w > 0.f && 2.f * p->wall_w < in.box[p->wall_axis]))
    return TDPD_ERR_INVALID_ARG;
  if (p->wall_axis == 3 &&
      !(p->wall_radius > 0.f && 2.f * p->wall_radius < std::min(in.box[1], in.box[2])))
    return TDPD_ERR_INVALID_ARG;
  b.ncell = int64_t(b.nc[0]) * b.nc[1] * b.nc[2];
  b.seed = in.seed;
  b.box_id = in.box_id;
  b.shear = in.shear_rate;
  return TDPD_OK;
}



// ------------------------------------------- allocation-free diagnostics
// Scratch of tdpd_diagnostics_noalloc: the per-workgroup partial sums of up
// to kNoAllocDiagBlocks workgroups, then the reduced totals.  One copy per
// device, alive until the process ends; host code never passes `scratch`
// itself to a kernel (on the host it only names the symbol), only the device
// address that hipGetSymbolAddress returned for the device.
constexpr int64_t kNoAllocMaxParticles = int64_t(1) << 23;
constexpr int64_t kNoAllocDiagBlocks = kNoAllocMaxParticles / kDiagSpan;
constexpr int64_t kNoAllocScratchDoubles = kNoAllocDiagBlocks * kDiagFields + 32;
static __device__ __align__(256) double scratch[kNoAllocScratchDoubles];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static double *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device, looked up once per
// device; records the device in *dev.  TDPD_ERR_HIP if the lookup fails.
static int scratch_for_current_device(int *dev) {
  int d = -1;
  if (hipGetDevice(&d) != hipSuccess || d < 0 || d >= kMaxDevices) return TDPD_ERR_HIP;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[d]) {
    void *ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return TDPD_ERR_HIP;
    g_scratch_ptr[d] = static_cast<double *>(ptr);
  }
  *dev = d;
  return TDPD_OK;
}

static int create_common(const tdpd_params *p, std::vector<HostBox> boxes, void *hip_stream,
                         tdpd_alloc_fn alloc, tdpd_free_fn free_fn, void *user, tdpd_sys **out) {
  tdpd_sys *s = new tdpd_sys();
  s->prm = *p;
  s->st = reinterpret_cast<hipStream_t>(hip_stream);
  s->alloc = alloc;
  s->free_fn = free_fn;
  s->user = user;
  s->S = p->n_species;
  s->boxes = std::move(boxes);
  for (auto &b : s->boxes) s->any_shear = s->any_shear || b.shear != 0.f;
  s->ncell = 0;
  for (auto &b : s->boxes) {
    b.cell_base = s->ncell;
    s->ncell += b.ncell;
  }
  s->key_bits = 1;
  while ((int64_t(1) << s->key_bits) < s->ncell) ++s->key_bits;
  PairConst &pc = s->pc;
  for (int a = 0; a < 3; ++a) pc.body_force[a] = p->body_force[a];
  pc.rc = p->rc;
  pc.rcc = p->rcc;
  pc.rc2 = p->rc * p->rc;
  pc.rcc2 = p->rcc * p->rcc;
  pc.rmax2 = std::max(pc.rc2, pc.rcc2);
  pc.inv_rc = 1.f / p->rc;
  pc.inv_rcc = 1.f / p->rcc;
  pc.s_half = 0.5f * p->s_exp;
  pc.sc_exp = p->sc_exp;
  pc.sc_half = 0.5f * p->sc_exp;
  pc.dt = p->dt;
  pc.half_dt = 0.5f * p->dt;
  pc.isdt = float(1.0 / std::sqrt(double(p->dt)));
  pc.ms_rho = p->m_s * p->m_s * p->rho;
  pc.n_types = p->n_types;
  pc.n_species = p->n_species;
  std::memcpy(pc.alpha, p->alpha, sizeof(pc.alpha));
  std::memcpy(pc.gamma, p->gamma, sizeof(pc.gamma));
  std::memcpy(pc.sigma, p->sigma, sizeof(pc.sigma));
  std::memcpy(pc.kappa, p->kappa, sizeof(pc.kappa));
  pc.wall_axis = p->wall_axis;
  pc.wall_w = p->wall_w;
  pc.wall_radius = p->wall_radius;
  pc.has_source = 0;
  for (int e = 0; e < kMaxS * kMaxT; ++e) {
    const bool used = e < p->n_species * p->n_types;
    pc.source[e] = used ? p->source[e] : 0.f;
    pc.decay[e] = used ? p->decay[e] : 0.f;
    if (pc.source[e] != 0.f || pc.decay[e] != 0.f) pc.has_source = 1;
  }
  pc.terms = p->terms;
  pc.n_boxes = int(s->boxes.size());
  s->mc.kT = p->kT;
  s->mc.dt = p->dt;
  s->mc.terms = p->terms;
  if (const char *e = std::getenv("TDPD_PAIR_KERNEL")) s->pair_kernel = std::atoi(e);
  if (const char *e = std::getenv("TDPD_BIN")) s->bin_mode = std::atoi(e);
  if (const char *e = std::getenv("TDPD_GRAPH")) s->use_graph = std::atoi(e) != 0;
  if (const char *e = std::getenv("TDPD_FUSE_MEMBRANE")) s->fuse_membrane = std::atoi(e) != 0 ? 1 : 0;
  {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
        cus > 0)
      s->cu_count = cus;
  }
  if (const char *e = std::getenv("TDPD_TILE")) {  // "waves,chunks,split,filter"
    PairTile t{};
    if (std::sscanf(e, "%d,%d,%d,%d", &t.waves, &t.chunks, &t.split, &t.filter) == 4 &&
        pair_tile_built(t, s->S))
      s->tile = t;
  }
  // set-up of the allocation-free diagnostics on this device; a failed
  // lookup only disables that entry point
  if (scratch_for_current_device(&s->device) != TDPD_OK) {
    s->device = -1;
    (void)hipGetLastError();
  }
  *out = s;
  return TDPD_OK;
}

extern "C" int tdpd_create(const tdpd_params *p, void *hip_stream, tdpd_alloc_fn alloc,
                           tdpd_free_fn free_fn, void *user, tdpd_sys **out) {
  if (!p || !out) return TDPD_ERR_INVALID_ARG;
  *out = nullptr;
  if ((alloc == nullptr) != (free_fn == nullptr)) return TDPD_ERR_INVALID_ARG;
  int rc = check_common(p);
  if (rc) return rc;
  tdpd_box in{};
  for (int a = 0; a < 3; ++a) in.box[a] = p->box[a];
  in.seed = p->seed;
  in.box_id = p->box_id;
  in.shear_rate = p->shear_rate;
  std::vector<HostBox> boxes(1);
  if ((rc = make_box(p, in, boxes[0]))) return rc;
  return create_common(p, std::move(boxes), hip_stream, alloc, free_fn, user, out);
}

extern "C" int tdpd_create_batch(const tdpd_params *p, int32_t n_boxes, const tdpd_box *in,
                                 void *hip_stream, tdpd_alloc_fn alloc, tdpd_free_fn free_fn,
                                 void *user, tdpd_sys **out) {
  if (!p || !out || !in || n_boxes < 1 || n_boxes > kMaxBoxes) return TDPD_ERR_INVALID_ARG;
  *out = nullptr;
  if ((alloc == nullptr) != (free_fn == nullptr)) return TDPD_ERR_INVALID_ARG;
  int rc = check_common(p);
  if (rc) return rc;
  std::vector<HostBox> boxes(n_boxes);
  for (int b = 0; b < n_boxes; ++b)
    if ((rc = make_box(p, in[b], boxes[b]))) return rc;
  return create_common(p, std::move(boxes), hip_stream, alloc, free_fn, user, out);
}

extern "C" void tdpd_destroy(tdpd_sys *s) {
  if (!s) return;
  if (s->uploaded) (void)hipStreamSynchronize(s->st);
  if (s->st2) (void)hipStreamSynchronize(s->st2);
  s->destroy_graphs();
  s->destroy_streams();
  s->destroy_events();
  s->release_all();
  delete s;
}

extern "C" const char *tdpd_last_error(const tdpd_sys *s) { return s ? s->err.c_str() : "null system"; }
extern "C" int64_t tdpd_num_particles(const tdpd_sys *s) { return s ? s->n : 0; }
extern "C" int64_t tdpd_step_counter(const tdpd_sys *s) { return s ? s->step : 0; }

extern "C" int tdpd_set_state_boxes(tdpd_sys *s, const int64_t *box_count, const float *pos,
                                    const float *vel, const float *conc, const uint32_t *flags) {
  if (!s || !box_count) return TDPD_ERR_INVALID_ARG;
  int64_t n = 0;
  for (size_t b = 0; b < s->boxes.size(); ++b) {
    if (box_count[b] < 0) return s->fail(TDPD_ERR_INVALID_ARG, "set_state: negative box count");
    n += box_count[b];
  }
  if (n >= (int64_t(1) << 31) || (n > 0 && (!pos || !vel || !conc || !flags)))
    return s->fail(TDPD_ERR_INVALID_ARG, "set_state: bad size or null pointer");
  const int S = s->S;
  for (int64_t i = 0; i < n; ++i) {
    if ((flags[i] & 0xffu) >= uint32_t(s->prm.n_types) || (flags[i] & ~0x1ffu))
      return s->fail(TDPD_ERR_INVALID_ARG, "set_state: bad flags word");
    for (int a = 0; a < 3; ++a)
      if (!is_finite_f(pos[3 * i + a]) || !is_finite_f(vel[3 * i + a]))
        return s->fail(TDPD_ERR_NONFINITE, "set_state: non-finite position or velocity");
    for (int sp = 0; sp < S; ++sp)
      if (!is_finite_f(conc[S * i + sp])) return s->fail(TDPD_ERR_NONFINITE, "set_state: non-finite concentration");
  }
  if (s->uploaded) (void)hipStreamSynchronize(s->st);
  if (s->st2) (void)hipStreamSynchronize(s->st2);
  s->destroy_graphs();
  s->release_all();
  s->uploaded = false;
  s->forces_valid = false;
  s->meshes.clear();
  s->rbc_mesh.clear();
  s->rbc_first.clear();
  s->rbc_box.clear();
  s->n = n;
  s->step = 0;
  s->mem_lds = 0;
  s->h_pos.assign(pos, pos + 3 * n);
  s->h_box.assign(n, 0);
  int64_t g = 0;
  for (size_t b = 0; b < s->boxes.size(); ++b) {
    HostBox &B = s->boxes[b];
    B.gid_base = g;
    B.n = box_count[b];
    for (int64_t i = g; i < g + B.n; ++i) {
      s->h_box[i] = int32_t(b);
      for (int a = 0; a < 3; ++a) {
        float x = s->h_pos[3 * i + a];
        const float L = B.L[a];
        if (x < -L || x >= 2.f * L) x = x - L * std::floor(x / L);  // far outside: fold first
        s->h_pos[3 * i + a] = wrap_host(x, L);
      }
    }
    g += B.n;
  }
  s->h_vel.assign(vel, vel + 3 * n);
  s->h_conc.assign(conc, conc + int64_t(S) * n);
  s->h_flags.assign(flags, flags + n);
  s->h_body.assign(n, -1);
  for (int64_t i = 0; i < n; ++i)
    if (s->h_flags[i] & TDPD_FLAG_FROZEN)
      for (int a = 0; a < 3; ++a) s->h_vel[3 * i + a] = 0.f;
  s->have_state = true;
  return TDPD_OK;
}

extern "C" int tdpd_set_state(tdpd_sys *s, int64_t n, const float *pos, const float *vel,
                              const float *conc, const uint32_t *flags) {
  if (!s) return TDPD_ERR_INVALID_ARG;
  if (s->boxes.size() != 1) return s->fail(TDPD_ERR_STATE, "set_state: a batch takes tdpd_set_state_boxes");
  if (n < 0) return s->fail(TDPD_ERR_INVALID_ARG, "set_state: negative count");
  return tdpd_set_state_boxes(s, &n, pos, vel, conc, flags);
}

extern "C" int32_t tdpd_num_boxes(const tdpd_sys *s) { return s ? int32_t(s->boxes.size()) : 0; }

extern "C" int tdpd_add_mesh(tdpd_sys *s, int32_t nv, const double *ref, int32_t ntri,
                             const int32_t *tri, const tdpd_mesh_params *mp, int32_t *mesh_id) {
  if (!s) return TDPD_ERR_INVALID_ARG;
  if (!s->have_state || s->uploaded) return s->fail(TDPD_ERR_STATE, "add_mesh: call after set_state, before stepping");
  if (nv < 4 || ntri < 4 || !ref || !tri || !mp || nv > 65535)
    return s->fail(TDPD_ERR_INVALID_ARG, "add_mesh: bad sizes");
  if (!(mp->p > 0.f) || !(mp->x0 > 0.f && mp->x0 < 1.f) || !(mp->m_pow > 0.f) ||
      mp->gamma_t < 0.f || 3.f * mp->gamma_c < mp->gamma_t)
    return s->fail(TDPD_ERR_INVALID_ARG, "add_mesh: bad membrane parameters");
  HostMesh M;
  M.nv = nv;
  M.ntri = ntri;
  M.mp = *mp;
  M.tri.assign(tri, tri + 3 * ntri);
  std::map<std::pair<int, int>, int> owner;  // directed edge -> triangle
  for (int t = 0; t < ntri; ++t)
    for (int e = 0; e < 3; ++e) {
      const int a = tri[3 * t + e], b = tri[3 * t + (e + 1) % 3];
      if (a < 0 || a >= nv || b < 0 || b >= nv || a == b || owner.count({a, b}))
        return s->fail(TDPD_ERR_INVALID_ARG, "add_mesh: not a consistently oriented manifold");
      owner[{a, b}] = t;
    }
  std::vector<std::vector<std::pair<int, int>>> bonds(nv);  // (nbr, edge index)
  std::vector<double> l0;
  std::vector<std::vector<int>> tris(nv);
  std::vector<int4> dihs;  // (a, b, c, d)
  for (auto &kv : owner) {
    const int a = kv.first.first, b = kv.first.second;
    if (a > b) continue;
    auto it = owner.find({b, a});
    if (it == owner.end()) return s->fail(TDPD_ERR_INVALID_ARG, "add_mesh: surface not closed");
    const int t1 = kv.second, t2 = it->second;
    int a0 = -1, d0 = -1;
    for (int e = 0; e < 3; ++e) {
      if (tri[3 * t1 + e] != a && tri[3 * t1 + e] != b) a0 = tri[3 * t1 + e];
      if (tri[3 * t2 + e] != a && tri[3 * t2 + e] != b) d0 = tri[3 * t2 + e];
    }
    const int ei = int(l0.size());
    double d[3];
    for (int q = 0; q < 3; ++q) d[q] = ref[3 * b + q] - ref[3 * a + q];
    l0.push_back(std::sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]));
    bonds[a].push_back({b, ei});
    bonds[b].push_back({a, ei});
    dihs.push_back(make_int4(a0, a, b, d0));  // t1 = (a0, a, b) holds a->b
  }
  // breadth-first order over bonds (for unwrapping at upload)
  {
    std::vector<char> seen(nv, 0);
    M.bfs.push_back({0, -1});
    seen[0] = 1;
    for (size_t q = 0; q < M.bfs.size(); ++q) {
      const int v = M.bfs[q].first;
      for (auto &nb : bonds[v])
        if (!seen[nb.first]) {
          seen[nb.first] = 1;
          M.bfs.push_back({nb.first, v});
        }
    }
    if (int(M.bfs.size()) != nv) return s->fail(TDPD_ERR_INVALID_ARG, "add_mesh: surface not connected");
  }
  const double kT = s->prm.kT, x0 = mp->x0;
  const double fwlc0 = kT / mp->p * (0.25 / ((1 - x0) * (1 - x0)) - 0.25 + x0);
  // bonds: endpoints (a < b), (l_m, k_p), and per-vertex signed incidences
  M.bond_ab.resize(l0.size());
  M.bond_par.resize(l0.size());
  for (int v = 0; v < nv; ++v)
    for (auto &nb : bonds[v])
      if (v < nb.first) M.bond_ab[nb.second] = make_int2(v, nb.first);
  for (size_t e = 0; e < l0.size(); ++e)
    M.bond_par[e] = make_float2(float(l0[e] / x0), float(fwlc0 * std::pow(l0[e], double(mp->m_pow))));
  M.bond_off.assign(nv + 1, 0);
  for (int v = 0; v < nv; ++v) {
    M.bond_off[v] = int(M.bond_inc.size());
    for (auto &nb : bonds[v]) M.bond_inc.push_back((nb.second << 1) | (v > nb.first ? 1 : 0));
  }
  M.bond_off[nv] = int(M.bond_inc.size());
  // triangles: per-vertex incidences (other two vertices, counter-clockwise)
  M.A0 = 0;
  M.V0 = 0;
  M.A0t.resize(ntri);
  for (int t = 0; t < ntri; ++t) {
    const double *a = ref + 3 * tri[3 * t], *b = ref + 3 * tri[3 * t + 1], *c = ref + 3 * tri[3 * t + 2];
    const double u[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
    const double w[3] = {c[0] - a[0], c[1] - a[1], c[2] - a[2]};
    const double nn[3] = {u[1] * w[2] - u[2] * w[1], u[2] * w[0] - u[0] * w[2], u[0] * w[1] - u[1] * w[0]};
    const double At = 0.5 * std::sqrt(nn[0] * nn[0] + nn[1] * nn[1] + nn[2] * nn[2]);
    M.A0t[t] = float(At);
    M.A0 += At;
    M.V0 += (a[0] * (b[1] * c[2] - b[2] * c[1]) + a[1] * (b[2] * c[0] - b[0] * c[2]) +
             a[2] * (b[0] * c[1] - b[1] * c[0])) / 6.0;
    for (int e = 0; e < 3; ++e) tris[tri[3 * t + e]].push_back(t);
  }
  M.tri_off.assign(nv + 1, 0);
  for (int v = 0; v < nv; ++v) {
    M.tri_off[v] = int(M.tri_inc.size());
    for (int t : tris[v]) {
      int e = 0;
      while (tri[3 * t + e] != v) ++e;
      M.tri_inc.push_back(make_int4(tri[3 * t + (e + 1) % 3], tri[3 * t + (e + 2) % 3], t, 0));
    }
  }
  M.tri_off[nv] = int(M.tri_inc.size());
  // dihedrals: per-vertex incidences with the vertex's role
  std::vector<std::vector<std::pair<int, int>>> dv(nv);  // (dihedral, role)
  double th_sum = 0;
  for (size_t q = 0; q < dihs.size(); ++q) {
    const int4 D = dihs[q];
    dv[D.x].push_back({int(q), 0});
    dv[D.y].push_back({int(q), 1});
    dv[D.z].push_back({int(q), 2});
    dv[D.w].push_back({int(q), 3});
    th_sum += d_theta(ref + 3 * D.x, ref + 3 * D.y, ref + 3 * D.z, ref + 3 * D.w);
  }
  M.theta0 = std::isnan(mp->theta0) ? th_sum / double(dihs.size()) : double(mp->theta0);
  M.dih_off.assign(nv + 1, 0);
  for (int v = 0; v < nv; ++v) {
    M.dih_off[v] = int(M.dih_inc.size());
    for (auto &pr : dv[v]) {
      M.dih_inc.push_back(dihs[pr.first]);
      M.dih_role.push_back(uint8_t(pr.second));
    }
  }
  M.dih_off[nv] = int(M.dih_inc.size());
  // 1-rings: next[v][p] = q for every triangle (v, p, q) in outward
  // counter-clockwise order; each ring starts at the smallest neighbour index
  {
    std::vector<std::map<int, int>> nxt(nv);
    for (int t = 0; t < ntri; ++t)
      for (int e = 0; e < 3; ++e)
        nxt[tri[3 * t + e]][tri[3 * t + (e + 1) % 3]] = tri[3 * t + (e + 2) % 3];
    M.ring_off.assign(nv + 1, 0);
    for (int v = 0; v < nv; ++v) {
      M.ring_off[v] = int(M.ring.size());
      const int start = nxt[v].begin()->first;
      int q = start;
      do {
        M.ring.push_back(q);
        q = nxt[v].at(q);
      } while (q != start && int(M.ring.size()) - M.ring_off[v] <= int(nxt[v].size()));
      if (q != start || int(M.ring.size()) - M.ring_off[v] != int(nxt[v].size()))
        return s->fail(TDPD_ERR_INVALID_ARG, "add_mesh: a vertex neighbourhood is not a disc");
    }
    M.ring_off[nv] = int(M.ring.size());
    double sl = 0;
    for (double l : l0) sl += l;
    M.ell = sl / double(l0.size());
  }
  // largest distance from the rest centroid (for the periodic-image limit)
  double cen[3] = {0, 0, 0};
  for (int v = 0; v < nv; ++v)
    for (int q = 0; q < 3; ++q) cen[q] += ref[3 * v + q] / nv;
  for (int v = 0; v < nv; ++v) {
    double r2 = 0;
    for (int q = 0; q < 3; ++q) r2 += (ref[3 * v + q] - cen[q]) * (ref[3 * v + q] - cen[q]);
    M.max_radius = std::max(M.max_radius, std::sqrt(r2));
  }
  if (membrane_lds_bytes(M.nv) > 60 * 1024)
    return s->fail(TDPD_ERR_UNSUPPORTED, "add_mesh: mesh too large for one workgroup's LDS");
  s->meshes.push_back(std::move(M));
  if (mesh_id) *mesh_id = int32_t(s->meshes.size() - 1);
  return TDPD_OK;
}

extern "C" int tdpd_add_rbc(tdpd_sys *s, int32_t mesh_id, int64_t first_gid, int32_t *rbc_id) {
  if (!s) return TDPD_ERR_INVALID_ARG;
  if (!s->have_state || s->uploaded) return s->fail(TDPD_ERR_STATE, "add_rbc: call after set_state, before stepping");
  if (mesh_id < 0 || mesh_id >= int(s->meshes.size())) return s->fail(TDPD_ERR_INVALID_ARG, "add_rbc: bad mesh id");
  const int nv = s->meshes[mesh_id].nv;
  if (first_gid < 0 || first_gid + nv > s->n) return s->fail(TDPD_ERR_INVALID_ARG, "add_rbc: gid range outside the state");
  if (s->rbc_mesh.size() >= size_t(kMaxBodies)) return s->fail(TDPD_ERR_UNSUPPORTED, "add_rbc: too many cells");
  const int32_t box = s->h_box[first_gid];
  if (s->h_box[first_gid + nv - 1] != box)
    return s->fail(TDPD_ERR_INVALID_ARG, "add_rbc: cell spans two boxes");
  const double rad = s->meshes[mesh_id].max_radius;
  for (int a = 0; a < 3; ++a)
    if (1.25 * rad + 1.0 > 0.5 * s->boxes[box].L[a])
      return s->fail(TDPD_ERR_UNSUPPORTED, "add_rbc: cell too large for its periodic box");
  for (int64_t g = first_gid; g < first_gid + nv; ++g)
    if (s->h_body[g] >= 0 || (s->h_flags[g] & TDPD_FLAG_FROZEN))
      return s->fail(TDPD_ERR_INVALID_ARG, "add_rbc: particle already bound or frozen");
  const int32_t body = int32_t(s->rbc_mesh.size());
  for (int64_t g = first_gid; g < first_gid + nv; ++g) s->h_body[g] = body;
  s->rbc_mesh.push_back(mesh_id);
  s->rbc_first.push_back(first_gid);
  s->rbc_box.push_back(box);
  if (rbc_id) *rbc_id = int32_t(s->rbc_mesh.size() - 1);
  return TDPD_OK;
}

template <class T>
static T *dallocT(tdpd_sys *s, size_t count) {
  return static_cast<T *>(s->dalloc(sizeof(T) * (count ? count : 1)));
}

template <class T>
static int upload(tdpd_sys *s, T **dst, const std::vector<T> &v) {
  *dst = dallocT<T>(s, v.size());
  if (!*dst) return s->fail(TDPD_ERR_OOM, "device allocation failed");
  if (!v.empty()) HIPCHK(hipMemcpyAsync(*dst, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice, s->st));
  return TDPD_OK;
}

static int alloc_state(tdpd_sys *s, State &st) {
  const int64_t n = s->n;
  float *blk = dallocT<float>(s, size_t(6 + s->S) * n);
  uint32_t *ib = dallocT<uint32_t>(s, size_t(2) * n);
  if (!blk || !ib) return s->fail(TDPD_ERR_OOM, "device allocation failed");
  st.x = blk;
  st.y = blk + n;
  st.z = blk + 2 * n;
  st.vx = blk + 3 * n;
  st.vy = blk + 4 * n;
  st.vz = blk + 5 * n;
  st.C = blk + 6 * n;
  st.gid = ib;
  st.info = ib + n;
  return TDPD_OK;
}

// Allocate device memory and upload state and membranes (once per set_state).
static int prepare(tdpd_sys *s) {
  if (!s->have_state) return s->fail(TDPD_ERR_STATE, "no state: call tdpd_set_state first");
  if (s->uploaded) return TDPD_OK;
  const int64_t n = s->n;
  const int S = s->S;
  int rc;
  if ((rc = alloc_state(s, s->A)) || (rc = alloc_state(s, s->B))) return rc;
  s->cur_A = true;
  s->F = dallocT<float>(s, 3 * size_t(n));
  s->Q = dallocT<float>(s, size_t(S) * n);
  s->keys = dallocT<uint32_t>(s, n);
  s->vals = dallocT<uint32_t>(s, n);
  s->keys_tmp = dallocT<uint32_t>(s, n);
  s->vals_tmp = dallocT<uint32_t>(s, n);
  s->keys_s = dallocT<uint32_t>(s, n);
  s->perm = dallocT<uint32_t>(s, n);
  s->hist = dallocT<uint32_t>(s, radix_hist_words(n));
  s->cell_start = dallocT<uint32_t>(s, size_t(s->ncell) + 1);
  s->slot_of_gid = dallocT<uint32_t>(s, n);
  s->slot_of_gid_b = dallocT<uint32_t>(s, n);
  s->nzero = dallocT<unsigned long long>(s, 2);
  s->pair_count = s->nzero + 1;
  s->errw = dallocT<uint32_t>(s, 1);
  s->kdev = dallocT<uint32_t>(s, 2);
  s->kstep = s->kdev ? s->kdev + 1 : nullptr;
  s->cell_count = dallocT<uint32_t>(s, size_t(s->ncell));
  s->bin_tmp = dallocT<uint32_t>(s, 2 * size_t(n));
  s->tile_sum = dallocT<uint32_t>(s, size_t(count_scan_tiles(s->ncell)));
  if (!s->kdev || !s->cell_count || !s->bin_tmp || !s->tile_sum)
    return s->fail(TDPD_ERR_OOM, "device allocation failed");
  s->list_valid = false;
  if (s->verlet_every > 0) {
    s->ld.nbr = dallocT<uint32_t>(s, size_t(s->ld.cap) * size_t(n));
    s->ld.lanes = n >= kFourLaneParticles ? 4 : 8;
    s->ld.ncnt = dallocT<uint32_t>(s, size_t(n) * s->ld.lanes);
    s->ld.xref = dallocT<float4>(s, n);
    s->ld.p4 = dallocT<float4>(s, n);
    s->ld.v4 = dallocT<float4>(s, n);
    s->ld.c4 = S <= 4 ? dallocT<float4>(s, n) : nullptr;
    if (!s->ld.nbr || !s->ld.ncnt || !s->ld.xref || !s->ld.p4 || !s->ld.v4 || (S <= 4 && !s->ld.c4))
      return s->fail(TDPD_ERR_OOM, "device allocation failed");
  }
  HIPCHK(hipMemsetAsync(s->kdev, 0, sizeof(uint32_t), s->st));
  HIPCHK(hipMemsetAsync(s->cell_count, 0, sizeof(uint32_t) * s->ncell, s->st));
  s->kdev_val = 0;
  s->diag_partial = dallocT<double>(s, size_t((n + kDiagSpan - 1) / kDiagSpan + 1) * kDiagFields);
  s->diag_out = dallocT<double>(s, kDiagFields);
  if (!s->F || !s->Q || !s->keys || !s->vals || !s->keys_tmp || !s->vals_tmp || !s->keys_s ||
      !s->perm || !s->hist || !s->cell_start || !s->slot_of_gid || !s->slot_of_gid_b ||
      !s->nzero || !s->errw ||
      !s->diag_partial || !s->diag_out)
    return s->fail(TDPD_ERR_OOM, "device allocation failed");
  // SoA planes in gid order
  std::vector<float> planes(size_t(6 + S) * n);
  std::vector<uint32_t> ints(2 * size_t(n));
  for (int64_t i = 0; i < n; ++i) {
    for (int a = 0; a < 3; ++a) {
      planes[a * n + i] = s->h_pos[3 * i + a];
      planes[(3 + a) * n + i] = s->h_vel[3 * i + a];
    }
    for (int sp = 0; sp < S; ++sp) planes[(6 + sp) * n + i] = s->h_conc[S * i + sp];
    ints[i] = uint32_t(i);
    ints[n + i] = make_info(int(s->h_flags[i] & 0xffu), (s->h_flags[i] & TDPD_FLAG_FROZEN) != 0,
                            s->h_box[i], s->h_body[i]);
  }
  if (n > 0) {
    HIPCHK(hipMemcpyAsync(s->A.x, planes.data(), sizeof(float) * planes.size(), hipMemcpyHostToDevice, s->st));
    HIPCHK(hipMemcpyAsync(s->A.gid, ints.data(), sizeof(uint32_t) * ints.size(), hipMemcpyHostToDevice, s->st));
    HIPCHK(hipMemcpyAsync(s->slot_of_gid, ints.data(), sizeof(uint32_t) * n, hipMemcpyHostToDevice, s->st));
    HIPCHK(hipMemcpyAsync(s->slot_of_gid_b, ints.data(), sizeof(uint32_t) * n, hipMemcpyHostToDevice, s->st));
    HIPCHK(hipMemsetAsync(s->F, 0, sizeof(float) * 3 * n, s->st));
    HIPCHK(hipMemsetAsync(s->Q, 0, sizeof(float) * S * n, s->st));
  }
  HIPCHK(hipMemsetAsync(s->nzero, 0, 2 * sizeof(unsigned long long), s->st));
  HIPCHK(hipMemsetAsync(s->errw, 0, sizeof(uint32_t), s->st));
  // membranes
  const int nrbc = int(s->rbc_mesh.size());
  s->nvert = 0;
  if (nrbc > 0) {
    std::vector<MeshDev> md(s->meshes.size());
    for (size_t m = 0; m < s->meshes.size(); ++m) {
      HostMesh &M = s->meshes[m];
      MeshDev &D = md[m];
      int32_t *tri, *bo, *bi, *to, *dof;
      int2 *bab;
      float2 *bp;
      int4 *ti, *di;
      uint8_t *dr;
      float *a0t;
      int32_t *rgo, *rg;
      if ((rc = upload(s, &tri, M.tri)) || (rc = upload(s, &bab, M.bond_ab)) ||
          (rc = upload(s, &bp, M.bond_par)) || (rc = upload(s, &bo, M.bond_off)) ||
          (rc = upload(s, &bi, M.bond_inc)) || (rc = upload(s, &to, M.tri_off)) ||
          (rc = upload(s, &ti, M.tri_inc)) || (rc = upload(s, &dof, M.dih_off)) ||
          (rc = upload(s, &di, M.dih_inc)) || (rc = upload(s, &dr, M.dih_role)) ||
          (rc = upload(s, &a0t, M.A0t)) || (rc = upload(s, &rgo, M.ring_off)) ||
          (rc = upload(s, &rg, M.ring)))
        return rc;
      D.ring_off = rgo;
      D.ring = rg;
      D.ell = float(M.ell);
      D.nv = M.nv;
      D.ntri = M.ntri;
      D.nbond = int(M.bond_ab.size());
      D.tri = tri;
      D.bond_ab = bab;
      D.bond_par = bp;
      D.bond_off = bo;
      D.bond_inc = bi;
      D.tri_off = to;
      D.tri_inc = ti;
      D.dih_off = dof;
      D.dih_inc = di;
      D.dih_role = dr;
      D.A0t = a0t;
      s->mem_lds = std::max(s->mem_lds, membrane_lds_bytes(M.nv));
      s->bond_stride = std::max<int64_t>(s->bond_stride, D.nbond);
      s->max_nv = std::max(s->max_nv, M.nv);
      D.A0 = M.A0;
      D.V0 = M.V0;
      D.theta0 = float(M.theta0);
      D.p = M.mp.p;
      D.m_pow = M.mp.m_pow;
      D.kb = M.mp.kb;
      D.kg = M.mp.kg;
      D.kl = M.mp.kl;
      D.kv = M.mp.kv;
      D.gamma_t = M.mp.gamma_t;
      D.gamma_c = M.mp.gamma_c;
      M.dev = D;
    }
    s->rbc_voff.assign(nrbc + 1, 0);
    std::vector<double> cen(3 * size_t(nrbc));
    for (int r = 0; r < nrbc; ++r) {
      const HostMesh &M = s->meshes[s->rbc_mesh[r]];
      s->rbc_voff[r + 1] = s->rbc_voff[r] + M.nv;
      // unwrapped centroid: breadth-first along bonds at nearest images
      std::vector<double> u(3 * size_t(M.nv));
      const int64_t g0 = s->rbc_first[r];
      for (auto &vp : M.bfs) {
        const int v = vp.first, par = vp.second;
        for (int a = 0; a < 3; ++a) {
          const double x = s->h_pos[3 * (g0 + v) + a];
          if (par < 0) {
            u[3 * v + a] = x;
          } else {
            const double L = s->boxes[s->rbc_box[r]].L[a];
            double d = x - s->h_pos[3 * (g0 + par) + a];
            d -= L * std::nearbyint(d / L);
            u[3 * v + a] = u[3 * par + a] + d;
          }
        }
      }
      for (int a = 0; a < 3; ++a) {
        double c = 0;
        for (int v = 0; v < M.nv; ++v) c += u[3 * v + a];
        c /= M.nv;
        const double L = s->boxes[s->rbc_box[r]].L[a];
        c -= L * std::floor(c / L);
        cen[3 * r + a] = c;
        for (int v = 0; v < M.nv; ++v)
          if (std::fabs(u[3 * v + a] - c - L * std::nearbyint((u[3 * v + a] - c) / L)) > 0.45 * L)
            return s->fail(TDPD_ERR_UNSUPPORTED, "add_rbc: cell spans half the box");
      }
    }
    s->nvert = s->rbc_voff[nrbc];
    if ((rc = upload(s, &s->d_meshes, md)) || (rc = upload(s, &s->d_rbc_mesh, s->rbc_mesh)) ||
        (rc = upload(s, &s->d_rbc_box, s->rbc_box)) ||
        (rc = upload(s, &s->d_rbc_first, s->rbc_first)) || (rc = upload(s, &s->d_rbc_voff, s->rbc_voff)) ||
        (rc = upload(s, &s->d_centroid, cen)))
      return rc;
    s->d_av = dallocT<double>(s, 2 * size_t(nrbc));
    s->Fm = dallocT<float>(s, 3 * size_t(s->nvert));
    s->Fb = dallocT<float>(s, 3 * size_t(nrbc) * size_t(s->bond_stride));
    if (!s->d_av || !s->Fm || !s->Fb) return s->fail(TDPD_ERR_OOM, "device allocation failed");
    if (!s->st2) {
      HIPCHK(hipStreamCreateWithFlags(&s->st2, hipStreamNonBlocking));
      HIPCHK(hipEventCreateWithFlags(&s->ev_fork, hipEventDisableTiming));
      HIPCHK(hipEventCreateWithFlags(&s->ev_join, hipEventDisableTiming));
    }
    HIPCHK(hipMemsetAsync(s->d_av, 0, sizeof(double) * 2 * nrbc, s->st));
  }
  // box table
  {
    std::vector<BoxDev> bd(s->boxes.size());
    for (size_t b = 0; b < s->boxes.size(); ++b) {
      const HostBox &H = s->boxes[b];
      BoxDev &D = bd[b];
      for (int a = 0; a < 3; ++a) {
        D.L[a] = H.L[a];
        D.invL[a] = 1.f / H.L[a];
        D.inv_h[a] = float(H.nc[a]) / H.L[a];
        D.nc[a] = H.nc[a];
      }
      D.cell_base = uint32_t(H.cell_base);
      D.ncell = uint32_t(H.ncell);
      D.gid_base = uint32_t(H.gid_base);
      D.seed_lo = uint32_t(H.seed & 0xffffffffu);
      D.seed_hi = uint32_t(H.seed >> 32);
      D.ctr3 = H.box_id << 8;
      D.shear = H.shear;
    }
    if ((rc = upload(s, &s->d_boxes, bd))) return rc;
  }
  HIPCHK(hipStreamSynchronize(s->st));  // host vectors may be released after this
  s->uploaded = true;
  return TDPD_OK;
}

// Membrane arguments of all cells (nrbc 0 when the system has none).
static MemArgs mem_args(const tdpd_sys *s, const MembraneConst &mc, float *Fm_out, SurrUse su) {
  MemArgs m{};
  m.mc = mc;
  m.meshes = s->d_meshes;
  m.rbc_mesh = s->d_rbc_mesh;
  m.rbc_box = s->d_rbc_box;
  m.rbc_first = s->d_rbc_first;
  m.rbc_voff = s->d_rbc_voff;
  m.slot_of_gid = s->slot_cur();
  m.av = s->d_av;
  m.centroid = s->d_centroid;
  m.Fm = Fm_out;
  m.Fb = s->Fb;
  m.bond_stride = s->bond_stride;
  m.su = su;
  m.nrbc = int(s->rbc_mesh.size());
  m.max_nv = s->max_nv;
  return m;
}

// Whether consecutive integrated steps may fold one step's closing kick
// into the next step's first kick (counting binning, which then advances
// the counter).
static bool can_fuse_kicks(const tdpd_sys *s) {
  return s->bin_mode == 0 && s->n > 0 && s->verlet_every == 0;
}

// Enqueue one force evaluation on stream `st`, optionally wrapped in the two
// velocity-Verlet half kicks.  The random-number counter is *kdev (set by the
// caller; each evaluation's last kernel advances it).  Host-side only swaps
// A/B.  Between integrated steps (can_fuse_kicks): fuse_prev does the
// previous evaluation's closing kick at the start of this one's first kick
// (the binning then advances the counter), and fuse_next leaves this
// evaluation's closing kick to the next one.
static int enqueue_evaluation(tdpd_sys *s, bool integrate, hipStream_t st, bool fuse_prev = false,
                              bool fuse_next = false) {
  const int64_t n = s->n;
  const int nrbc = int(s->rbc_mesh.size());
  const VertexMap vmap{nrbc > 0 ? s->Fm : nullptr, s->d_rbc_first, s->d_rbc_voff};
  // neighbour-list mode: the binning (and a list build) only on every
  // verlet_every-th evaluation
  const bool verlet = s->verlet_every > 0;
  const bool rebuild = !verlet || !s->list_valid || s->list_age >= s->verlet_every;
  const bool tb = s->phase_begin(1, st);
  if (rebuild) {
    launch_prekick(s->pc, s->d_boxes, s->cur(), s->F, s->Q, n, s->keys, s->vals, integrate,
                   s->bin_mode == 0 ? s->cell_count : nullptr, s->kdev, fuse_prev, vmap, s->kstep,
                   st);
  } else {
    launch_prekick_list(s->pc, s->d_boxes, s->cur(), s->F, s->Q, n, integrate, s->kdev, s->ld,
                        s->errw, s->kstep, st);
  }
  if (verlet) {
    s->list_age = rebuild ? 1 : s->list_age + 1;
    s->list_valid = true;
  }
  if (n == 0) {
    s->phase_end(1, tb, st);
    launch_postkick(s->pc, s->cur(), s->F, s->Q, 0, VertexMap{nullptr, nullptr, nullptr}, false,
                    s->kdev, st);  // advances the counter
    return TDPD_OK;
  }
  // (the tiled kernel packs a slot into 26 bits)
  const bool tiled = !(s->pair_kernel == 0 || n >= (int64_t(1) << 26));
  // The membrane terms normally ride along in two launches the step makes
  // anyway: the K-Gather and bond forces in the binning scan's launch, the
  // per-vertex part in the pair kernel's (no second stream, nothing
  // serialised).  The surrogate, the simple pair kernel, the radix binning,
  // a timed membrane phase or a mesh too large for either launch's LDS take
  // the membrane kernel on a second stream beside the pair kernel instead.
  // By size: the membrane workgroups of the scan's launch run after the
  // scan and before the pair kernel; beyond about four rounds of the chip
  // (many cells) a kernel of its own beside the pair kernel, where the pair
  // work hides it, costs less than the fork and join of the second stream.
  const bool fuse = s->fuse_membrane == 1 ||
                    (s->fuse_membrane < 0 &&
                     int64_t(nrbc) * membrane_element_parts(s->bond_stride) <= 4 * int64_t(s->cu_count));
  const bool split = nrbc > 0 && tiled && !verlet && s->bin_mode == 0 && fuse &&
                     !(s->timing_mask & (1 << 2)) && scan_takes_membrane(s->max_nv) &&
                     pair_tiled_takes_membrane(s->tile, s->S, s->any_shear, s->max_nv);
  MemArgs ma_split = mem_args(s, s->mc, s->Fm, SurrUse{nullptr, nullptr});
  if (!split) ma_split.nrbc = 0;
  // The membrane kernel on the second stream (when the membrane terms do not
  // ride in the binning and pair launches) starts right after the first
  // kick: it reads the drifted positions in the previous order through the
  // current id-to-slot map (the binning writes the other one) and the
  // evaluation's counter from the snapshot, so it runs beside the binning
  // and the pair kernel.
  if (nrbc > 0 && !split) {
    (void)hipEventRecord(s->ev_fork, st);
    (void)hipStreamWaitEvent(s->st2, s->ev_fork, 0);
    const bool tm = s->phase_begin(2, s->st2);
    SurrUse su{nullptr, nullptr};
    if (s->surr_on) {
      // network forces from the lagged cell totals, then (every surr_every
      // steps, gated on the device counter) the plain bending + local-area
      // forces and the per-vertex fallback decision
      launch_surr_features(s->sd, s->d_boxes, s->d_meshes, s->cur(), s->slot_cur(), s->d_av,
                           s->nvert, s->kstep, s->pc.dt, 0, s->st2);
      mlp_forward(s->surr_params, s->sd.X, s->nvert, s->sd.Y, s->st2);
      launch_surr_apply(s->sd, s->nvert, s->st2);
      MembraneConst ml = s->mc;
      ml.terms = s->mc.terms & (TDPD_TERM_AREA | TDPD_TERM_BENDING);
      ml.local_only = 1;
      ml.gate = s->surr_every;
      launch_membrane(mem_args(s, ml, s->sd.Fp, SurrUse{nullptr, nullptr}), s->d_boxes, s->cur(),
                      s->kstep, s->errw, s->mem_lds, s->st2);
      launch_surr_check(s->sd, nrbc, s->kstep, s->surr_every, s->st2);
      su = SurrUse{s->sd.flag, s->sd.Fs};
    }
    launch_membrane(mem_args(s, s->mc, s->Fm, su), s->d_boxes, s->cur(), s->kstep, s->errw,
                    s->mem_lds, s->st2);
    s->phase_end(2, tm, s->st2);
    (void)hipEventRecord(s->ev_join, s->st2);
  }
  // With the surrogate on the split path the network runs on the second
  // stream beside the binning, on the drifted positions in the previous
  // order (so its cell totals are those of the previous evaluation, which
  // the binning scan then updates); the check and the pair kernel's
  // per-vertex terms, which take its forces where the last check allows,
  // wait for it.
  const bool surr_split = split && s->surr_on;
  if (surr_split) {
    (void)hipEventRecord(s->ev_fork, st);
    (void)hipStreamWaitEvent(s->st2, s->ev_fork, 0);
    launch_surr_features(s->sd, s->d_boxes, s->d_meshes, s->cur(), s->slot_cur(), s->d_av,
                         s->nvert, s->kstep, s->pc.dt, 0, s->st2);
    mlp_forward(s->surr_params, s->sd.X, s->nvert, s->sd.Y, s->st2);
    launch_surr_apply(s->sd, s->nvert, s->st2);
    (void)hipEventRecord(s->ev_join, s->st2);
    ma_split.su = SurrUse{s->sd.flag, s->sd.Fs};
  }
  if (!rebuild) {
    // the particle order of the last rebuild stays
  } else if (s->bin_mode == 0) {
    launch_bin_counting(s->cur(), s->nxt(), s->keys, s->vals, s->cell_count, s->ncell,
                        s->cell_start, s->bin_tmp, s->tile_sum, n, s->S, s->slot_nxt(), s->keys_s,
                        fuse_prev ? s->kdev : nullptr, ma_split, s->d_boxes, s->kdev,
                        fuse_prev ? 1 : 0, s->errw, st);
  } else {
    radix_sort(s->keys, s->vals, s->keys_tmp, s->vals_tmp, s->keys_s, s->perm, s->hist, n,
               s->key_bits, st);
    launch_cell_bounds(s->keys_s, n, s->ncell, s->cell_start, st);
    launch_reorder(s->cur(), s->nxt(), s->perm, n, s->S, s->slot_nxt(), st);
  }
  if (rebuild) s->cur_A = !s->cur_A;
  // the pair kernel's per-vertex membrane terms read the new order
  ma_split.slot_of_gid = s->slot_cur();
  if (verlet && rebuild)
    launch_list_build(s->d_boxes, int(s->boxes.size()), s->cur(), s->S, s->cell_start, s->ncell,
                      n, s->ld, s->errw, st);
  if (surr_split) {
    // every surr_every steps (gated on the device counter): the plain
    // bending + local-area forces and the per-vertex fallback decision,
    // before the pair kernel's per-vertex terms read it
    (void)hipStreamWaitEvent(st, s->ev_join, 0);
    MembraneConst ml = s->mc;
    ml.terms = s->mc.terms & (TDPD_TERM_AREA | TDPD_TERM_BENDING);
    ml.local_only = 1;
    ml.gate = s->surr_every;
    launch_membrane(mem_args(s, ml, s->sd.Fp, SurrUse{nullptr, nullptr}), s->d_boxes, s->cur(),
                    s->kdev, s->errw, s->mem_lds, st);
    launch_surr_check(s->sd, nrbc, s->kdev, s->surr_every, st);
  }
  s->phase_end(1, tb, st);
  const bool tp = s->phase_begin(0, st);
  if (verlet) {
    launch_pair_list(s->pc, s->d_boxes, s->cur(), n, s->kdev, s->ld, s->F, s->Q, s->nzero,
                     s->errw, st);
  } else if (!tiled) {
    launch_pair_simple(s->pc, s->d_boxes, s->cur(), s->keys_s, s->cell_start, n, s->kdev, s->F,
                       s->Q, s->nzero, s->errw, st);
  } else {
    (void)launch_pair_tiled(s->pc, s->d_boxes, s->cur(), s->cell_start, s->ncell, n, s->kdev,
                            s->F, s->Q, s->nzero, s->errw, s->tile, s->any_shear, ma_split, st);
  }
  s->phase_end(0, tp, st);
  if (nrbc > 0 && !split) (void)hipStreamWaitEvent(st, s->ev_join, 0);
  if (!fuse_next) {
    const bool tk = s->phase_begin(3, st);
    launch_postkick(s->pc, s->cur(), s->F, s->Q, n, vmap, integrate, s->kdev, st);
    s->phase_end(3, tk, st);
  }
  return TDPD_OK;
}

static int check_launch(tdpd_sys *s) {
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return s->fail(TDPD_ERR_HIP, std::string("kernel launch: ") + hipGetErrorString(e));
  return TDPD_OK;
}

// Force evaluation at counter k without integration (the device counter is
// k + 1 afterwards, ready for the next step).
static int evaluate_at(tdpd_sys *s, uint32_t k) {
  launch_set_counter(s->kdev, k, s->st);
  s->kdev_val = k;
  int rc = enqueue_evaluation(s, false, s->st);
  if (rc) return rc;
  s->forces_valid = true;
  return check_launch(s);
}

// Capture, on a private stream, one integrated step and kGraphSteps
// integrated steps for each A/B parity (capturing runs nothing: only the
// host-side parity advances, and it is restored).
constexpr int kGraphSteps = 4;
static_assert(kGraphSteps % 2 == 0, "a multi-step graph must end at its start parity");
// Neighbour-list mode: one graph per buffer parity holding a whole rebuild
// period (a rebuilding step and verlet_every - 1 list steps), which flips
// the parity once; slots [0] and [1].
static int capture_list_graphs(tdpd_sys *s) {
  const bool start_A = s->cur_A;
  const int age = s->list_age;
  const bool valid = s->list_valid;
  for (int q = 0; q < 2; ++q) {
    const int slot = s->cur_A ? 0 : 1;
    s->list_valid = true;
    s->list_age = s->verlet_every;  // the first step of the period rebuilds
    HIPCHK(hipStreamBeginCapture(s->gst, hipStreamCaptureModeThreadLocal));
    int rc = TDPD_OK;
    for (int r = 0; r < s->verlet_every && !rc; ++r) rc = enqueue_evaluation(s, true, s->gst);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(s->gst, &g);
    if (rc) return rc;
    if (e != hipSuccess) return s->fail(TDPD_ERR_HIP, std::string("graph capture: ") + hipGetErrorString(e));
    s->graph[slot] = g;
    HIPCHK(hipGraphInstantiate(&s->gexec[slot], g, nullptr, nullptr, 0));
  }
  s->list_age = age;
  s->list_valid = valid;
  if (s->cur_A != start_A) return s->fail(TDPD_ERR_HIP, "graph capture: parity mismatch");
  return TDPD_OK;
}

static int capture_graphs(tdpd_sys *s) {
  if (!s->gst) HIPCHK(hipStreamCreateWithFlags(&s->gst, hipStreamNonBlocking));
  if (s->verlet_every > 0) return capture_list_graphs(s);
  const bool start_A = s->cur_A;
  for (int q = 0; q < 4; ++q) {
    const int slot = (q < 2 ? 0 : 2) + (s->cur_A ? 0 : 1);
    HIPCHK(hipStreamBeginCapture(s->gst, hipStreamCaptureModeThreadLocal));
    int rc = TDPD_OK;
    const int steps = q < 2 ? 1 : kGraphSteps;
    const bool fuse = can_fuse_kicks(s);
    for (int r = 0; r < steps && !rc; ++r)
      rc = enqueue_evaluation(s, true, s->gst, fuse && r > 0, fuse && r + 1 < steps);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(s->gst, &g);
    if (rc) return rc;
    if (e != hipSuccess) return s->fail(TDPD_ERR_HIP, std::string("graph capture: ") + hipGetErrorString(e));
    s->graph[slot] = g;
    HIPCHK(hipGraphInstantiate(&s->gexec[slot], g, nullptr, nullptr, 0));
    if (q == 2) s->cur_A = !s->cur_A;  // the multi-step graph of the other parity
  }
  s->cur_A = !s->cur_A;
  if (s->cur_A != start_A) return s->fail(TDPD_ERR_HIP, "graph capture: parity mismatch");
  return TDPD_OK;
}

extern "C" int tdpd_compute_forces(tdpd_sys *s, uint32_t k) {
  if (!s) return TDPD_ERR_INVALID_ARG;
  int rc = prepare(s);
  if (rc) return rc;
  return evaluate_at(s, k);
}

extern "C" int tdpd_step(tdpd_sys *s, int32_t n_steps) {
  if (!s) return TDPD_ERR_INVALID_ARG;
  if (n_steps < 0) return s->fail(TDPD_ERR_INVALID_ARG, "step: negative count");
  int rc = prepare(s);
  if (rc) return rc;
  if (!s->forces_valid && (rc = evaluate_at(s, 0))) return rc;
  if (s->step + n_steps > 0xffffffffLL) return s->fail(TDPD_ERR_UNSUPPORTED, "step counter exhausted");
  if (n_steps == 0) return TDPD_OK;
  // step n reads counter n from the device; each evaluation's last kernel
  // advances it (kdev_val is the counter of the last evaluation)
  if (s->kdev_val != uint32_t(s->step)) {
    launch_set_counter(s->kdev, uint32_t(s->step) + 1u, s->st);
    s->kdev_val = uint32_t(s->step);
  }
  const bool graphs = s->use_graph && s->timing_mask == 0 && s->n > 0;
  if (graphs && !s->gexec[0] && (rc = capture_graphs(s))) return rc;
  const bool verlet = s->verlet_every > 0;
  for (int i = 0; i < n_steps;) {
    if (graphs && verlet) {
      // whole rebuild periods from a rebuild on, single steps otherwise
      if (s->list_valid && s->list_age >= s->verlet_every && n_steps - i >= s->verlet_every) {
        HIPCHK(hipGraphLaunch(s->gexec[s->cur_A ? 0 : 1], s->st));
        s->cur_A = !s->cur_A;
        s->step += s->verlet_every;
        s->kdev_val += uint32_t(s->verlet_every);
        i += s->verlet_every;
        continue;
      }
      ++s->step;
      if ((rc = enqueue_evaluation(s, true, s->st))) return rc;
      ++s->kdev_val;
      ++i;
      continue;
    }
    if (graphs && n_steps - i >= kGraphSteps) {
      HIPCHK(hipGraphLaunch(s->gexec[2 + (s->cur_A ? 0 : 1)], s->st));  // parity unchanged
      s->step += kGraphSteps;
      s->kdev_val += kGraphSteps;
      i += kGraphSteps;
      continue;
    }
    ++s->step;
    if (graphs) {
      HIPCHK(hipGraphLaunch(s->gexec[s->cur_A ? 0 : 1], s->st));
      s->cur_A = !s->cur_A;
    } else if ((rc = enqueue_evaluation(s, true, s->st, can_fuse_kicks(s) && i > 0,
                                        can_fuse_kicks(s) && i + 1 < n_steps))) {
      return rc;
    }
    ++s->kdev_val;
    ++i;
  }
  return check_launch(s);
}

extern "C" int tdpd_sync(tdpd_sys *s) {
  if (!s) return TDPD_ERR_INVALID_ARG;
  if (!s->uploaded) return TDPD_OK;
  HIPCHK(hipStreamSynchronize(s->st));
  uint32_t e = 0;
  HIPCHK(hipMemcpy(&e, s->errw, sizeof(e), hipMemcpyDeviceToHost));
  if (e) {
    HIPCHK(hipMemset(s->errw, 0, sizeof(uint32_t)));
    if (e & kErrOverext) return s->fail(TDPD_ERR_BOND_OVEREXTENDED, "a membrane bond reached its maximum extension");
    if (e & kErrNonfinite) return s->fail(TDPD_ERR_NONFINITE, "a force became non-finite");
    if (e & kErrSkin)
      return s->fail(TDPD_ERR_LIST, "neighbour list: a particle moved more than half the skin "
                                    "between rebuilds (raise the skin or rebuild more often)");
    if (e & kErrListFull)
      return s->fail(TDPD_ERR_LIST, "neighbour list: a particle has more neighbours than the "
                                    "list capacity");
  }
  return TDPD_OK;
}

static int ensure_forces(tdpd_sys *s) {
  int rc = prepare(s);
  if (rc) return rc;
  if (!s->forces_valid && (rc = evaluate_at(s, 0))) return rc;
  return tdpd_sync(s);
}

static int readback(tdpd_sys *s, float *pos, float *vel, float *conc, float *F, float *Q) {
  int rc = ensure_forces(s);
  if (rc) return rc;
  const int64_t n = s->n;
  if (n == 0) return TDPD_OK;
  const int S = s->S;
  // temporary device AoS buffers, then one copy each
  float *buf = dallocT<float>(s, size_t(n) * (9 + 2 * S));
  if (!buf) return s->fail(TDPD_ERR_OOM, "device allocation failed");
  float *dp = buf, *dv = buf + 3 * n, *dc = buf + 6 * n, *dF = dc + S * n, *dQ = dF + 3 * n;
  launch_gid_order(s->cur(), n, S, s->F, s->Q, pos ? dp : nullptr, vel ? dv : nullptr,
                   conc ? dc : nullptr, F ? dF : nullptr, Q ? dQ : nullptr, s->st);
  hipError_t e = hipSuccess;
  if (pos && e == hipSuccess) e = hipMemcpyAsync(pos, dp, sizeof(float) * 3 * n, hipMemcpyDeviceToHost, s->st);
  if (vel && e == hipSuccess) e = hipMemcpyAsync(vel, dv, sizeof(float) * 3 * n, hipMemcpyDeviceToHost, s->st);
  if (conc && e == hipSuccess) e = hipMemcpyAsync(conc, dc, sizeof(float) * S * n, hipMemcpyDeviceToHost, s->st);
  if (F && e == hipSuccess) e = hipMemcpyAsync(F, dF, sizeof(float) * 3 * n, hipMemcpyDeviceToHost, s->st);
  if (Q && e == hipSuccess) e = hipMemcpyAsync(Q, dQ, sizeof(float) * S * n, hipMemcpyDeviceToHost, s->st);
  if (e == hipSuccess) e = hipStreamSynchronize(s->st);
  // release the temporary
  s->blocks.pop_back();
  if (s->free_fn) s->free_fn(buf, s->user);
  else if (!s->alloc) (void)hipFree(buf);
  if (e != hipSuccess) return s->fail(TDPD_ERR_HIP, std::string("readback: ") + hipGetErrorString(e));
  return TDPD_OK;
}

extern "C" int tdpd_get_state(tdpd_sys *s, float *pos, float *vel, float *conc) {
  if (!s) return TDPD_ERR_INVALID_ARG;
  return readback(s, pos, vel, conc, nullptr, nullptr);
}

extern "C" int tdpd_get_forces(tdpd_sys *s, float *F, float *Q) {
  if (!s) return TDPD_ERR_INVALID_ARG;
  return readback(s, nullptr, nullptr, nullptr, F, Q);
}

extern "C" int tdpd_get_pairs(tdpd_sys *s, int32_t which, int64_t cap, int32_t *ij, int64_t *n_out) {
  if (!s || !n_out || cap < 0 || (cap > 0 && !ij) || which < 0 || which > 3) return TDPD_ERR_INVALID_ARG;
  int rc = ensure_forces(s);
  if (rc) return rc;
  if (which >= 2 && s->verlet_every > 0)
    return s->fail(TDPD_ERR_STATE, "get_pairs: ordered pairs of the tiled kernel need cell mode");
  *n_out = 0;
  if (s->n == 0) return TDPD_OK;
  int32_t *dout = dallocT<int32_t>(s, 2 * size_t(cap > 0 ? cap : 1));
  if (!dout) return s->fail(TDPD_ERR_OOM, "device allocation failed");
  HIPCHK(hipMemsetAsync(s->pair_count, 0, sizeof(unsigned long long), s->st));
  const float rcut2 = (which & 1) ? s->pc.rcc2 : s->pc.rc2;
  if (which >= 2) {  // the tiled kernel's own candidate path at the current tile
    if (!launch_pair_tiled_emit(s->pc, s->d_boxes, s->cur(), s->cell_start, s->ncell, s->n,
                                s->kdev_val, rcut2, dout, cap, s->pair_count, s->nzero, s->errw,
                                s->tile, s->any_shear, s->st))
      return s->fail(TDPD_ERR_INVALID_ARG, "get_pairs: tile shape not built");
  } else if (s->verlet_every > 0) {  // the cells are those of the last rebuild: take the lists
    launch_list_emit(s->d_boxes, s->cur(), s->n, s->ld, rcut2, dout, cap, s->pair_count, s->st);
  } else {
    launch_pair_emit(s->pc, s->d_boxes, s->cur(), s->keys_s, s->cell_start, s->n, rcut2,
                     s->kdev_val, dout, cap, s->pair_count, s->st);
  }
  unsigned long long cnt = 0;
  hipError_t e = hipMemcpyAsync(&cnt, s->pair_count, sizeof(cnt), hipMemcpyDeviceToHost, s->st);
  if (e == hipSuccess) e = hipStreamSynchronize(s->st);
  const int64_t m = std::min<int64_t>(int64_t(cnt), cap);
  if (e == hipSuccess && m > 0) e = hipMemcpy(ij, dout, sizeof(int32_t) * 2 * m, hipMemcpyDeviceToHost);
  s->blocks.pop_back();
  if (s->free_fn) s->free_fn(dout, s->user);
  else if (!s->alloc) (void)hipFree(dout);
  if (e != hipSuccess) return s->fail(TDPD_ERR_HIP, std::string("get_pairs: ") + hipGetErrorString(e));
  *n_out = int64_t(cnt);
  if (int64_t(cnt) > cap) return s->fail(TDPD_ERR_CAPACITY, "get_pairs: buffer too small");
  return TDPD_OK;
}

extern "C" int tdpd_diagnostics(tdpd_sys *s, double *out, int64_t cap) {
  if (!s || !out) return TDPD_ERR_INVALID_ARG;
  const int S = s->S;
  const int nrbc = int(s->rbc_mesh.size());
  const int64_t need = 4 + S + 2 * int64_t(nrbc);
  if (cap < need) return s->fail(TDPD_ERR_CAPACITY, "diagnostics: buffer too small");
  int rc = ensure_forces(s);
  if (rc) return rc;
  double d[5 + kMaxS];
  launch_diag(s->cur(), s->n, S, s->diag_partial, s->diag_out, s->st);
  HIPCHK(hipMemcpyAsync(d, s->diag_out, sizeof(double) * (5 + S), hipMemcpyDeviceToHost, s->st));
  if (nrbc > 0)
    HIPCHK(hipMemcpyAsync(out + 4 + S, s->d_av, sizeof(double) * 2 * nrbc, hipMemcpyDeviceToHost, s->st));
  HIPCHK(hipStreamSynchronize(s->st));
  const double nm = d[4];
  out[0] = d[0];
  out[1] = d[1];
  out[2] = d[2];
  out[3] = nm > 1 ? (d[3] - (d[0] * d[0] + d[1] * d[1] + d[2] * d[2]) / nm) / (3.0 * (nm - 1)) : 0.0;
  for (int sp = 0; sp < S; ++sp) out[4 + sp] = d[5 + sp];
  return TDPD_OK;
}

extern "C" int tdpd_diagnostics_noalloc(tdpd_sys *s, double *out_dev, int64_t cap) {
  if (!s || !out_dev) return TDPD_ERR_INVALID_ARG;
  const int S = s->S;
  const int nrbc = int(s->rbc_mesh.size());
  const int64_t need = 4 + S + 2 * int64_t(nrbc);
  if (cap < need) return s->fail(TDPD_ERR_CAPACITY, "diagnostics_noalloc: buffer too small");
  if (!s->uploaded || !s->forces_valid)
    return s->fail(TDPD_ERR_STATE,
                   "diagnostics_noalloc: no evaluated state (call tdpd_compute_forces or tdpd_step)");
  if (s->n > kNoAllocMaxParticles)
    return s->fail(TDPD_ERR_CAPACITY,
                   "diagnostics_noalloc: more than 8,388,608 particles (the scratch limit)");
  if (s->device < 0 || !g_scratch_ptr[s->device])
    return s->fail(TDPD_ERR_HIP, "diagnostics_noalloc: device scratch unavailable");
  double *partial = g_scratch_ptr[s->device];
  double *sums = partial + kNoAllocDiagBlocks * kDiagFields;
  // every partial and total the kernels read is written first in this call,
  // so nothing is cleared
  launch_diag(s->cur(), s->n, S, partial, sums, s->st);
  launch_diag_finish(sums, S, out_dev, s->st);
  HIPCHK(hipGetLastError());
  if (nrbc > 0)
    HIPCHK(hipMemcpyAsync(out_dev + 4 + S, s->d_av, sizeof(double) * 2 * nrbc,
                          hipMemcpyDeviceToDevice, s->st));
  return TDPD_OK;
}

extern "C" int64_t tdpd_coincident_pairs(tdpd_sys *s) {
  if (!s || !s->uploaded) return 0;
  unsigned long long v = 0;
  if (hipStreamSynchronize(s->st) != hipSuccess) return -1;
  if (hipMemcpy(&v, s->nzero, sizeof(v), hipMemcpyDeviceToHost) != hipSuccess) return -1;
  return int64_t(v);
}

extern "C" int tdpd_set_timing(tdpd_sys *s, int32_t mask) {
  if (!s || mask < 0 || mask > 15) return TDPD_ERR_INVALID_ARG;
  s->timing_mask = mask;
  return TDPD_OK;
}

extern "C" int tdpd_get_timing(tdpd_sys *s, int32_t phase, double *total_ms, int64_t *launches) {
  if (!s || !total_ms || !launches) return TDPD_ERR_INVALID_ARG;
  int q = -1;
  for (int b = 0; b < 4; ++b)
    if (phase == (1 << b)) q = b;
  if (q < 0) return s->fail(TDPD_ERR_INVALID_ARG, "get_timing: phase must be one TDPD_PHASE_* bit");
  HIPCHK(hipStreamSynchronize(s->st));
  double tot = 0;
  for (size_t i = 0; i < s->ev_used[q]; ++i) {
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, s->ev_pool[q][i].first, s->ev_pool[q][i].second));
    tot += ms;
  }
  *total_ms = tot;
  *launches = int64_t(s->ev_used[q]);
  s->ev_used[q] = 0;
  return TDPD_OK;
}

// ------------------------------------------------------------ checkpoints
namespace {

constexpr char kCkptMagic[8] = {'T', 'D', 'P', 'D', 'C', 'K', 'P', '1'};

struct Fnv {
  uint64_t h = 1469598103934665603ull;
  void bytes(const void *p, size_t n) {
    const unsigned char *c = static_cast<const unsigned char *>(p);
    for (size_t i = 0; i < n; ++i) h = (h ^ c[i]) * 1099511628211ull;
  }
  template <class T>
  void val(const T &v) { bytes(&v, sizeof(T)); }
  template <class T>
  void vec(const std::vector<T> &v) {
    val(uint64_t(v.size()));
    if (!v.empty()) bytes(v.data(), sizeof(T) * v.size());
  }
};

// Fingerprint of everything a checkpoint must match: parameters field by
// field (no struct padding), boxes, sizes, meshes and cells.
uint64_t fingerprint(const tdpd_sys *s) {
  Fnv f;
  const tdpd_params &p = s->prm;
  f.val(p.rc); f.val(p.rcc); f.val(p.dt); f.val(p.kT); f.val(p.rho); f.val(p.m_s);
  f.val(p.s_exp); f.val(p.sc_exp); f.val(p.n_types); f.val(p.n_species);
  f.bytes(p.alpha, sizeof(p.alpha)); f.bytes(p.gamma, sizeof(p.gamma));
  f.bytes(p.sigma, sizeof(p.sigma)); f.bytes(p.kappa, sizeof(p.kappa));
  f.bytes(p.body_force, sizeof(p.body_force)); f.val(p.wall_axis); f.val(p.wall_w);
  f.bytes(p.source, sizeof(p.source)); f.bytes(p.decay, sizeof(p.decay)); f.val(p.wall_radius);
  f.val(p.terms);
  f.val(s->n); f.val(s->S); f.val(uint64_t(s->boxes.size()));
  f.val(s->verlet_every); f.val(s->verlet_skin); f.val(s->ld.cap);
  for (const HostBox &b : s->boxes) {
    f.bytes(b.L, sizeof(b.L)); f.val(b.n); f.val(b.seed); f.val(b.box_id);
  }
  for (const HostMesh &m : s->meshes) {
    f.val(m.nv); f.val(m.ntri); f.vec(m.tri); f.vec(m.A0t);
    const tdpd_mesh_params &q = m.mp;
    f.val(q.p); f.val(q.x0); f.val(q.m_pow); f.val(q.kb); f.val(q.kg); f.val(q.kl);
    f.val(q.kv); f.val(q.gamma_t); f.val(q.gamma_c); f.val(float(m.theta0));
  }
  f.vec(s->rbc_mesh); f.vec(s->rbc_first);
  return f.h;
}

struct CkptHeader {
  char magic[8];
  uint64_t fingerprint;
  int64_t n, step;
  int32_t S, nrbc;
  uint32_t kdev, forces_valid;
  int32_t list_age, list_valid;
};

// The device regions of a checkpoint, in file order.
std::vector<std::pair<void *, size_t>> ckpt_regions(tdpd_sys *s) {
  const size_t n = size_t(s->n), S = size_t(s->S), nrbc = s->rbc_mesh.size();
  State &c = s->cur();
  std::vector<std::pair<void *, size_t>> r = {
      {c.x, sizeof(float) * (6 + S) * n},   // x, y, z, vx, vy, vz, C planes (one block)
      {c.gid, sizeof(uint32_t) * 2 * n},    // gid, info
      {s->slot_cur(), sizeof(uint32_t) * n},
      {s->F, sizeof(float) * 3 * n},
      {s->Q, sizeof(float) * S * n},
      // the cells of the last binning (they hold the current positions),
      // which tdpd_get_pairs reads
      {s->keys_s, sizeof(uint32_t) * n},
      {s->cell_start, sizeof(uint32_t) * (size_t(s->ncell) + 1)}};
  if (nrbc) r.push_back({s->d_centroid, sizeof(double) * 3 * nrbc});
  if (s->verlet_every > 0) {  // the lists, so that a resumed run takes the same pairs in the same order
    r.push_back({s->ld.ncnt, sizeof(uint32_t) * n * s->ld.lanes});
    r.push_back({s->ld.nbr, sizeof(uint32_t) * n * s->ld.cap});
    r.push_back({s->ld.xref, sizeof(float4) * n});
    r.push_back({s->ld.p4, sizeof(float4) * n});
    r.push_back({s->ld.v4, sizeof(float4) * n});
    if (s->ld.c4) r.push_back({s->ld.c4, sizeof(float4) * n});
  }
  return r;
}

}  // namespace

extern "C" int tdpd_save(tdpd_sys *s, const char *path) {
  if (!s || !path) return TDPD_ERR_INVALID_ARG;
  int rc = ensure_forces(s);
  if (rc) return rc;
  CkptHeader h{};
  std::memcpy(h.magic, kCkptMagic, 8);
  h.fingerprint = fingerprint(s);
  h.n = s->n;
  h.step = s->step;
  h.S = s->S;
  h.nrbc = int32_t(s->rbc_mesh.size());
  h.kdev = s->kdev_val;
  h.forces_valid = s->forces_valid ? 1u : 0u;
  h.list_age = s->list_age;
  h.list_valid = s->list_valid ? 1 : 0;
  FILE *fp = std::fopen(path, "wb");
  if (!fp) return s->fail(TDPD_ERR_IO, std::string("save: cannot open ") + path);
  bool ok = std::fwrite(&h, sizeof(h), 1, fp) == 1;
  std::vector<char> buf;
  for (auto &reg : ckpt_regions(s)) {
    if (!ok || reg.second == 0) continue;
    buf.resize(reg.second);
    if (hipMemcpy(buf.data(), reg.first, reg.second, hipMemcpyDeviceToHost) != hipSuccess) {
      std::fclose(fp);
      return s->fail(TDPD_ERR_HIP, "save: device copy failed");
    }
    ok = std::fwrite(buf.data(), 1, reg.second, fp) == reg.second;
  }
  ok = (std::fclose(fp) == 0) && ok;
  if (!ok) return s->fail(TDPD_ERR_IO, std::string("save: write failed: ") + path);
  return TDPD_OK;
}

extern "C" int tdpd_load(tdpd_sys *s, const char *path) {
  if (!s || !path) return TDPD_ERR_INVALID_ARG;
  int rc = prepare(s);
  if (rc) return rc;
  HIPCHK(hipStreamSynchronize(s->st));
  FILE *fp = std::fopen(path, "rb");
  if (!fp) return s->fail(TDPD_ERR_IO, std::string("load: cannot open ") + path);
  CkptHeader h{};
  bool ok = std::fread(&h, sizeof(h), 1, fp) == 1 && std::memcmp(h.magic, kCkptMagic, 8) == 0;
  if (!ok || h.fingerprint != fingerprint(s) || h.n != s->n || h.S != s->S ||
      h.nrbc != int32_t(s->rbc_mesh.size()) || h.step < 0 || h.step > 0xffffffffLL) {
    std::fclose(fp);
    return s->fail(TDPD_ERR_IO, "load: not a checkpoint of this system");
  }
  // read everything before touching the device, so a short file changes nothing
  s->cur_A = true;
  auto regs = ckpt_regions(s);
  std::vector<std::vector<char>> data(regs.size());
  for (size_t i = 0; i < regs.size() && ok; ++i) {
    data[i].resize(regs[i].second);
    ok = std::fread(data[i].data(), 1, regs[i].second, fp) == regs[i].second;
  }
  std::fclose(fp);
  if (!ok) return s->fail(TDPD_ERR_IO, "load: truncated checkpoint");
  for (size_t i = 0; i < regs.size(); ++i)
    if (regs[i].second)
      HIPCHK(hipMemcpy(regs[i].first, data[i].data(), regs[i].second, hipMemcpyHostToDevice));
  launch_set_counter(s->kdev, h.kdev + 1u, s->st);  // the next step's counter
  HIPCHK(hipStreamSynchronize(s->st));
  s->kdev_val = h.kdev;
  s->step = h.step;
  s->forces_valid = h.forces_valid != 0;
  s->list_age = h.list_age;
  s->list_valid = s->verlet_every > 0 && h.list_valid != 0;
  // captured graphs hold the A/B parity they were recorded at; A is current now
  s->destroy_graphs();
  return check_launch(s);
}

// ------------------------------------------------------------- autotuning
namespace {

std::string tune_signature(const tdpd_sys *s) {
  hipDeviceProp_t prop{};
  int dev = 0;
  (void)hipGetDevice(&dev);
  (void)hipGetDeviceProperties(&prop, dev);
  char buf[256];
  std::snprintf(buf, sizeof(buf), "%s n=%lld S=%d boxes=%zu cells=%lld rbcs=%zu terms=%d q=%d",
                prop.gcnArchName, (long long)s->n, s->S, s->boxes.size(), (long long)s->ncell,
                s->rbc_mesh.size(), s->prm.terms, pair_tiled_queued(s->pc) ? 1 : 0);
  for (char *c = buf; *c; ++c)
    if (*c == ':' || *c == '\n') *c = '_';
  return buf;
}

bool cache_lookup(const char *path, const std::string &sig, int n_species, PairTile *t) {
  FILE *fp = path ? std::fopen(path, "r") : nullptr;
  if (!fp) return false;
  char line[512];
  bool found = false;
  while (std::fgets(line, sizeof(line), fp)) {
    const char *bar = std::strchr(line, '|');
    if (!bar || std::string(line, bar - line) != sig) continue;
    PairTile c{};
    if (std::sscanf(bar + 1, "%d %d %d %d", &c.waves, &c.chunks, &c.split, &c.filter) == 4 &&
        pair_tile_built(c, n_species)) {
      *t = c;
      found = true;  // the last matching line wins
    }
  }
  std::fclose(fp);
  return found;
}

}  // namespace

extern "C" int tdpd_autotune(tdpd_sys *s, const char *cache_path, int32_t reps,
                             double *best_ms) {
  if (!s || reps < 1) return TDPD_ERR_INVALID_ARG;
  int rc = ensure_forces(s);
  if (rc) return rc;
  const std::string sig = tune_signature(s);
  PairTile best = s->tile;
  double best_t = -1.0;
  if (s->n == 0 || s->pair_kernel == 0 || s->n >= (int64_t(1) << 26)) {
    if (best_ms) *best_ms = 0.0;
    return TDPD_OK;  // the tiled kernel is not used for this system
  }
  if (!cache_lookup(cache_path, sig, s->S, &best)) {
    // the pair kernel is a pure function of the binned state: time every
    // shape on the current state, keeping the coincident-pair counters
    unsigned long long saved[2] = {0, 0};
    HIPCHK(hipMemcpy(saved, s->nzero, sizeof(saved), hipMemcpyDeviceToHost));
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    for (int i = 0; i < kNumPairTiles; ++i) {
      const PairTile &t = kPairTiles[i];
      if (!pair_tile_built(t, s->S)) continue;
      auto launch = [&]() {
        MemArgs none{};  // the shapes are timed on the pair work alone
        (void)launch_pair_tiled(s->pc, s->d_boxes, s->cur(), s->cell_start, s->ncell, s->n,
                                s->kdev, s->F, s->Q, s->nzero, s->errw, t, s->any_shear, none,
                                s->st);
      };
      launch();  // warm-up
      (void)hipEventRecord(e0, s->st);
      for (int r = 0; r < reps; ++r) launch();
      (void)hipEventRecord(e1, s->st);
      if (hipEventSynchronize(e1) != hipSuccess) break;
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, e0, e1);
      const double avg = double(ms) / reps;
      if (best_t < 0.0 || avg < best_t) {
        best_t = avg;
        best = t;
      }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    rc = check_launch(s);
    if (rc) return rc;
    HIPCHK(hipMemcpy(s->nzero, saved, sizeof(saved), hipMemcpyHostToDevice));
    if (cache_path) {
      FILE *fp = std::fopen(cache_path, "a");
      if (!fp) return s->fail(TDPD_ERR_IO, std::string("autotune: cannot write ") + cache_path);
      std::fprintf(fp, "%s|%d %d %d %d %.6f\n", sig.c_str(), best.waves, best.chunks, best.split,
                   best.filter, best_t);
      std::fclose(fp);
    }
  }
  s->tile = best;
  if (best_ms) *best_ms = best_t;
  // graphs hold the previous shape; forces are re-evaluated with the chosen one
  s->destroy_graphs();
  rc = evaluate_at(s, s->kdev_val);
  if (rc) return rc;
  return tdpd_sync(s);
}

extern "C" int tdpd_set_tile(tdpd_sys *s, int32_t waves, int32_t chunks, int32_t split,
                             int32_t filter) {
  if (!s) return TDPD_ERR_INVALID_ARG;
  const PairTile t{waves, chunks, split, filter};
  if (!pair_tile_built(t, s->S)) return s->fail(TDPD_ERR_UNSUPPORTED, "set_tile: shape not built");
  s->tile = t;
  s->destroy_graphs();
  return TDPD_OK;
}

extern "C" int tdpd_get_tile(const tdpd_sys *s, int32_t *waves, int32_t *chunks, int32_t *split,
                             int32_t *filter) {
  if (!s || !waves || !chunks || !split || !filter) return TDPD_ERR_INVALID_ARG;
  *waves = s->tile.waves;
  *chunks = s->tile.chunks;
  *split = s->tile.split;
  *filter = s->tile.filter;
  return TDPD_OK;
}

// ------------------------------------------------------------- neighbour lists
constexpr int32_t kMaxListCap = 4096;

extern "C" int tdpd_set_verlet(tdpd_sys *s, float skin, int32_t every, int32_t capacity) {
  if (!s) return TDPD_ERR_INVALID_ARG;
  if (!std::isfinite(skin) || skin < 0.f || every < 0 || capacity < 0 || capacity > kMaxListCap)
    return s->fail(TDPD_ERR_INVALID_ARG, "set_verlet: bad skin, interval or capacity");
  if (s->uploaded)
    return s->fail(TDPD_ERR_STATE, "set_verlet: call after set_state, before the first step");
  const bool on = every > 0 && skin > 0.f;
  if (on && s->any_shear)
    return s->fail(TDPD_ERR_UNSUPPORTED, "set_verlet: not with Lees-Edwards boxes");
  if (on && s->prm.m_s > 0.f && (s->prm.terms & TDPD_TERM_FLUX_RANDOM))
    return s->fail(TDPD_ERR_UNSUPPORTED, "set_verlet: not with the random flux");
  const float rmax = std::max(s->prm.rc, s->prm.rcc);
  const float rl = on ? rmax + skin : rmax;
  // cells at least rl wide, so that the 27 around a particle hold its list
  std::vector<HostBox> boxes = s->boxes;
  int64_t ncell = 0;
  for (HostBox &b : boxes) {
    for (int a = 0; a < 3; ++a) {
      b.nc[a] = int(std::floor(double(b.L[a]) / (double(rl) * (1.0 + 1e-4))));
      if (b.nc[a] < 3)
        return s->fail(TDPD_ERR_BOX_TOO_SMALL, "set_verlet: fewer than 3 cells of the list radius");
    }
    b.ncell = int64_t(b.nc[0]) * b.nc[1] * b.nc[2];
    b.cell_base = ncell;
    ncell += b.ncell;
  }
  s->boxes = std::move(boxes);
  s->ncell = ncell;
  s->key_bits = 1;
  while ((int64_t(1) << s->key_bits) < s->ncell) ++s->key_bits;
  s->verlet_every = on ? every : 0;
  s->verlet_skin = on ? skin : 0.f;
  s->ld = ListDev{};
  if (on) {
    int64_t cap = capacity;
    if (cap == 0) {  // three times the mean count at the nominal density, with room
      // for membranes, whose vertices pack more densely than the solvent
      const double mean = 4.0 / 3.0 * M_PI * double(rl) * rl * rl * std::max(0.f, s->prm.rho);
      cap = std::min<int64_t>(kMaxListCap, (int64_t(3.0 * mean) + 128 + 31) / 32 * 32);
    }
    s->ld.cap = uint32_t((cap + kMaxListLanes - 1) / kMaxListLanes * kMaxListLanes);
    s->ld.rl2 = rl * rl;
    const float h = 0.5f * skin * (1.f - 1e-3f);  // half the skin, less a rounding margin
    s->ld.drift2 = h * h;
  }
  s->list_valid = false;
  s->list_age = 0;
  s->destroy_graphs();
  return TDPD_OK;
}

extern "C" int tdpd_get_verlet(const tdpd_sys *s, float *skin, int32_t *every, int32_t *capacity) {
  if (!s || !skin || !every || !capacity) return TDPD_ERR_INVALID_ARG;
  *skin = s->verlet_skin;
  *every = s->verlet_every;
  *capacity = int32_t(s->ld.cap);
  return TDPD_OK;
}

// ------------------------------------------------------------- surrogate
const float *mlp_device_params(const tdpd_mlp *m);

namespace {

// buffers of the surrogate path (once per system)
int surr_alloc(tdpd_sys *s) {
  if (s->sd.X) return TDPD_OK;
  const int64_t nv = s->nvert;
  const int nrbc = int(s->rbc_mesh.size());
  std::vector<int32_t> vcell(static_cast<size_t>(nv), 0);
  for (int r = 0; r < nrbc; ++r)
    for (int64_t v = s->rbc_voff[r]; v < s->rbc_voff[r + 1]; ++v) vcell[v] = r;
  int rc = upload(s, &s->d_vcell, vcell);
  if (rc) return rc;
  SurrDev &d = s->sd;
  d.vcell = s->d_vcell;
  d.rbc_mesh = s->d_rbc_mesh;
  d.rbc_box = s->d_rbc_box;
  d.rbc_voff = s->d_rbc_voff;
  d.rbc_first = s->d_rbc_first;
  d.X = dallocT<float>(s, size_t(nv) * kSurrIn);
  d.R = dallocT<float>(s, size_t(nv) * 9);
  d.Y = dallocT<float>(s, size_t(nv) * kSurrOut);
  d.Fs = dallocT<float>(s, size_t(nv) * 3);
  d.Fp = dallocT<float>(s, size_t(nv) * 3);
  d.stats = dallocT<float>(s, size_t(nrbc) * 3);
  d.ok = dallocT<uint8_t>(s, size_t(nv));
  d.flag = dallocT<uint8_t>(s, size_t(nv));
  s->surr_params = dallocT<float>(s, kSurrParams);
  s->surr_Ha = dallocT<float>(s, size_t(nv) * kSurrHid);
  s->surr_Hb = dallocT<float>(s, size_t(nv) * kSurrHid);
  if (!d.X || !d.R || !d.Y || !d.Fs || !d.Fp || !d.stats || !d.ok || !d.flag || !s->surr_params ||
      !s->surr_Ha || !s->surr_Hb) {
    d.X = nullptr;
    return s->fail(TDPD_ERR_OOM, "device allocation failed");
  }
  HIPCHK(hipMemsetAsync(d.flag, 0, size_t(nv), s->st));
  HIPCHK(hipMemsetAsync(d.ok, 0, size_t(nv), s->st));
  HIPCHK(hipMemsetAsync(d.stats, 0, sizeof(float) * 3 * nrbc, s->st));
  HIPCHK(hipMemsetAsync(d.Fs, 0, sizeof(float) * 3 * nv, s->st));
  return TDPD_OK;
}

}  // namespace

extern "C" int tdpd_surrogate_sample(tdpd_sys *s, float *X, float *T, uint8_t *ok) {
  if (!s) return TDPD_ERR_INVALID_ARG;
  int rc = ensure_forces(s);
  if (rc) return rc;
  if (s->rbc_mesh.empty()) return s->fail(TDPD_ERR_STATE, "surrogate_sample: no cells");
  if ((rc = surr_alloc(s))) return rc;
  const int64_t nv = s->nvert;
  // the state is that of the last evaluation (counter kdev_val); the device
  // counter already holds the next step's
  launch_set_counter(s->kdev, s->kdev_val, s->st);
  launch_surr_features(s->sd, s->d_boxes, s->d_meshes, s->cur(), s->slot_cur(), s->d_av, nv,
                       s->kdev, s->pc.dt, 0, s->st);
  MembraneConst ml = s->mc;
  ml.terms = s->mc.terms & (TDPD_TERM_AREA | TDPD_TERM_BENDING);
  ml.local_only = 1;
  ml.gate = 0;
  launch_membrane(mem_args(s, ml, s->sd.Fp, SurrUse{nullptr, nullptr}), s->d_boxes, s->cur(),
                  s->kdev, s->errw, s->mem_lds, s->st);
  // targets go through Fs, which the next step's surrogate pass rewrites
  launch_surr_targets(s->sd, s->sd.Fs, nv, s->st);
  launch_set_counter(s->kdev, s->kdev_val + 1u, s->st);
  if ((rc = check_launch(s))) return rc;
  if (X) HIPCHK(hipMemcpyAsync(X, s->sd.X, sizeof(float) * kSurrIn * nv, hipMemcpyDeviceToHost, s->st));
  if (T) HIPCHK(hipMemcpyAsync(T, s->sd.Fs, sizeof(float) * 3 * nv, hipMemcpyDeviceToHost, s->st));
  if (ok) HIPCHK(hipMemcpyAsync(ok, s->sd.ok, size_t(nv), hipMemcpyDeviceToHost, s->st));
  return tdpd_sync(s);
}

extern "C" int tdpd_surrogate_enable(tdpd_sys *s, const tdpd_mlp *mlp, float force_scale,
                                     float tol, int32_t check_every) {
  if (!s || !mlp || !(force_scale > 0.f) || !(tol >= 0.f) || check_every < 1)
    return TDPD_ERR_INVALID_ARG;
  int rc = prepare(s);
  if (rc) return rc;
  if (s->rbc_mesh.empty()) return s->fail(TDPD_ERR_STATE, "surrogate_enable: no cells");
  if ((rc = surr_alloc(s))) return rc;
  HIPCHK(hipStreamSynchronize(s->st));
  HIPCHK(hipMemcpy(s->surr_params, mlp_device_params(mlp), sizeof(float) * kSurrParams,
                   hipMemcpyDeviceToDevice));
  HIPCHK(hipMemset(s->sd.flag, 0, size_t(s->nvert)));
  s->sd.s_F = force_scale;
  s->sd.tol = tol;
  s->surr_every = check_every;
  s->surr_on = true;
  s->destroy_graphs();
  // forces at the current state with the network (a check runs when the
  // current counter is a multiple of check_every)
  if (s->forces_valid && (rc = evaluate_at(s, s->kdev_val))) return rc;
  return TDPD_OK;
}

extern "C" int tdpd_surrogate_disable(tdpd_sys *s) {
  if (!s) return TDPD_ERR_INVALID_ARG;
  if (!s->surr_on) return TDPD_OK;
  s->surr_on = false;
  s->destroy_graphs();
  return TDPD_OK;
}

extern "C" int tdpd_surrogate_stats(tdpd_sys *s, double *out) {
  if (!s || !out) return TDPD_ERR_INVALID_ARG;
  for (int q = 0; q < 4; ++q) out[q] = 0.0;
  if (!s->sd.X) return TDPD_OK;
  int rc = tdpd_sync(s);
  if (rc) return rc;
  const int nrbc = int(s->rbc_mesh.size());
  std::vector<float> st(3 * size_t(nrbc));
  std::vector<uint8_t> ok(size_t(s->nvert));
  HIPCHK(hipMemcpy(st.data(), s->sd.stats, sizeof(float) * st.size(), hipMemcpyDeviceToHost));
  HIPCHK(hipMemcpy(ok.data(), s->sd.ok, ok.size(), hipMemcpyDeviceToHost));
  double cnt = 0, mx = 0, sm = 0, nok = 0;
  for (int r = 0; r < nrbc; ++r) {
    cnt += st[3 * r];
    mx = std::max(mx, double(st[3 * r + 1]));
    sm += st[3 * r + 2];
  }
  for (uint8_t o : ok) nok += o ? 1.0 : 0.0;
  out[0] = cnt / double(s->nvert);
  out[1] = mx;
  out[2] = nok > 0 ? sm / nok : 0.0;
  out[3] = nok / double(s->nvert);
  return TDPD_OK;
}
