// extern "C" entry points of the QED step library: argument checks on the host,
// context memory, and the launches of the kernels in step.hip / tables.hip.
#include <hip/hip_runtime.h>
#include <string.h>

#include <mutex>
#include <new>
#include <string>

#include "internal.h"
#include "qed_device.h"

namespace {

int fail(qed_ctx *c, int code, const std::string &msg) {
  if (c) c->err = msg;
  return code;
}

int hip_fail(qed_ctx *c, hipError_t e, const char *where) {
  return fail(c, QED_ERR_HIP, std::string(where) + ": " + hipGetErrorString(e));
}

int check_species(qed_ctx *c, const qed_species_t *s, const char *name) {
  if (!s) return fail(c, QED_ERR_ARG, std::string(name) + " is null");
  if (s->dtype != QED_F32 && s->dtype != QED_F64)
    return fail(c, QED_ERR_ARG, std::string(name) + ": dtype must be QED_F32 or QED_F64");
  if (!s->x || !s->y || !s->z || !s->px || !s->py || !s->pz || !s->tau || !s->id || !s->count)
    return fail(c, QED_ERR_ARG, std::string(name) + ": null array");
  if (s->capacity <= 0 || s->capacity > (int64_t)INT32_MAX)
    return fail(c, QED_ERR_ARG, std::string(name) + ": capacity must be in [1, 2^31)");
  return QED_OK;
}

int check_fields(qed_ctx *c, const qed_fields_t *f) {
  if (!f) return fail(c, QED_ERR_ARG, "fields is null");
  if (f->kind == QED_FIELD_UNIFORM) return QED_OK;
  if (f->kind == QED_FIELD_GRID) {
    if (!f->grid || f->nx < 3 || f->ny < 3 || f->nz < 3 || !(f->dx > 0) || !(f->dy > 0) || !(f->dz > 0))
      return fail(c, QED_ERR_ARG, "grid fields: need grid pointer, n >= 3 and d > 0 on every axis");
    if (((uintptr_t)f->grid) % 8)
      return fail(c, QED_ERR_ARG, "grid fields: pointer must be 8-byte aligned");
    if ((int64_t)f->nx * f->ny * f->nz * 6 >= (int64_t)1 << 32)
      return fail(c, QED_ERR_ARG, "grid fields: nx ny nz 6 must be below 2^32 floats");
    return QED_OK;
  }
  if (f->kind == QED_FIELD_PER_PARTICLE) {
    for (int k = 0; k < 3; ++k)
      if (!f->pE[k] || !f->pB[k]) return fail(c, QED_ERR_ARG, "per-particle fields: null array");
    return QED_OK;
  }
  return fail(c, QED_ERR_ARG, "unknown field kind");
}

template <typename T> hipError_t dalloc(T **p, size_t n) {
  return hipMalloc((void **)p, n * sizeof(T) > 0 ? n * sizeof(T) : 1);
}

void free_emitters(qed_ctx *c) {
  (void)hipFree(c->em_idx); (void)hipFree(c->em_rec); (void)hipFree(c->em_mask);
  (void)hipFree(c->cont_idx); (void)hipFree(c->d_n_cont);
  c->em_idx = nullptr; c->em_rec = nullptr; c->em_mask = nullptr;
  c->cont_idx = nullptr; c->d_n_cont = nullptr;
  c->em_cap = 0;
}

void free_scan(qed_ctx *c) {
  (void)hipFree(c->d_status);
  c->d_status = nullptr;
  c->reserved = 0; c->status_len = 0;
}

// Scan state for species of up to n particles (one status word per tile of
// the smallest tile size, 256).  Allocates, so not under graph capture.
int ensure_scan(qed_ctx *c, int64_t n) {
  if (n <= c->reserved) return QED_OK;
  hipError_t e = hipDeviceSynchronize();
  if (e != hipSuccess) return hip_fail(c, e, "reserve");
  free_scan(c);
  const int64_t status_len = n / 256 + 64;
  if ((e = dalloc(&c->d_status, 2 * status_len)) != hipSuccess) {   // two regions (see qed_ctx)
    free_scan(c);
    return hip_fail(c, e, "reserve: hipMalloc");
  }
  c->reserved = n;
  c->status_len = status_len;
  return QED_OK;
}

// Emitter slots (one record per particle), ballot mask, ordered list and the
// list of the surrogate emission's second pass for lepton species of up to n
// particles.  Allocates, so not under graph capture.
int ensure_emitters(qed_ctx *c, int64_t n) {
  if (n <= c->em_cap) return QED_OK;
  hipError_t e = hipDeviceSynchronize();
  if (e != hipSuccess) return hip_fail(c, e, "reserve");
  free_emitters(c);
  if ((e = dalloc(&c->em_idx, n)) != hipSuccess || (e = dalloc(&c->em_rec, kEmRecMaxBytes * n)) != hipSuccess ||
      (e = dalloc(&c->em_mask, n / 64 + 1)) != hipSuccess || (e = dalloc(&c->cont_idx, n)) != hipSuccess ||
      (e = dalloc(&c->d_n_cont, 1)) != hipSuccess) {
    free_emitters(c);
    return hip_fail(c, e, "reserve: hipMalloc");
  }
  c->em_cap = n;
  c->em_owner = nullptr;
  return QED_OK;
}

void free_cands(qed_ctx *c) {
  (void)hipFree(c->cand_mask); (void)hipFree(c->cand_idx); (void)hipFree(c->d_n_cand);
  c->cand_mask = nullptr; c->cand_idx = nullptr; c->d_n_cand = nullptr;
  c->cand_cap = 0;
}

// Event (or, on the surrogate path, candidate) mask and list of the float32
// pair pass for photon species of up to n particles.  Allocates, so not under
// graph capture.
int ensure_cands(qed_ctx *c, int64_t n) {
  if (n <= c->cand_cap) return QED_OK;
  hipError_t e = hipDeviceSynchronize();
  if (e != hipSuccess) return hip_fail(c, e, "create_pairs");
  free_cands(c);
  if ((e = dalloc(&c->cand_mask, n / 64 + 1)) != hipSuccess || (e = dalloc(&c->cand_idx, n)) != hipSuccess ||
      (e = dalloc(&c->d_n_cand, 1)) != hipSuccess) {
    free_cands(c);
    return hip_fail(c, e, "create_pairs: hipMalloc");
  }
  c->cand_cap = n;
  return QED_OK;
}

hipStream_t S(void *s) { return (hipStream_t)s; }

// ------------------------------------------- static scratch (qed_compact_static)
// Scan state of qed_compact_static in a file-scope device array, so that the
// entry point needs no allocation: word 0 holds the tile ticket (low 32 bits),
// words 1 .. kStaticTiles + 1 the tile status words, for species of up to
// kStaticMaxParticles particles (513 KiB per device, held until the process
// ends).  In host code `scratch` only names the symbol; its device address on
// each GPU comes from hipGetSymbolAddress and is what the kernels are given.
constexpr int64_t kStaticMaxParticles = (int64_t)1 << 26;
constexpr int64_t kStaticTiles = kStaticMaxParticles / kCompactTile;
constexpr int64_t kStaticStatusWords = kStaticTiles + 1;
static __device__ __align__(256) uint64_t scratch[1 + kStaticStatusWords];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
uint64_t *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on `device` (the current device), looked up once
// per device.
hipError_t static_scratch_address(int device, uint64_t **out) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[device] = static_cast<uint64_t *>(ptr);
  }
  *out = g_scratch_ptr[device];
  return hipSuccess;
}

}  // namespace

extern "C" {

int qed_create(qed_ctx_t *out, const qed_params_t *p) {
  if (!out || !p) return QED_ERR_ARG;
  *out = nullptr;
  if (p->kmax < 1 || p->kmax > 4) return QED_ERR_ARG;
  qed_ctx *c = new (std::nothrow) qed_ctx();
  if (!c) return QED_ERR_ARG;
  c->params = *p;
  hipError_t e = hipGetDevice(&c->device);
  int ncu = 0;
  if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, c->device);
  if (e == hipSuccess) c->n_cu = ncu > 0 ? ncu : 256;
  if (e == hipSuccess) e = static_scratch_address(c->device, &c->static_scratch);
  if (e == hipSuccess) e = qed::mlp_set_attributes();
  if (e == hipSuccess) e = qed::step_set_attributes();
  if (e == hipSuccess) e = dalloc(&c->d_counters, qed::cNumCounters);
  if (e == hipSuccess) e = dalloc(&c->d_next_id, 1);
  if (e == hipSuccess) e = dalloc(&c->d_n_emit, 1);
  if (e == hipSuccess) e = dalloc(&c->d_ticket, 2);
  if (e == hipSuccess) e = dalloc(&c->d_killed, 1);
  if (e == hipSuccess) e = dalloc(&c->d_step, 1);
  if (e == hipSuccess) e = hipMemset(c->d_step, 0, sizeof(int64_t));
  if (e == hipSuccess) e = hipMemset(c->d_counters, 0, sizeof(unsigned long long) * qed::cNumCounters);
  if (e == hipSuccess) e = hipMemset(c->d_next_id, 0, sizeof(uint64_t));
  if (e == hipSuccess) e = hipMemset(c->d_n_emit, 0, sizeof(int64_t));
  if (e == hipSuccess) e = hipMemset(c->d_killed, 0, sizeof(int64_t));
  if (e != hipSuccess) {
    qed_destroy(c);
    return QED_ERR_HIP;
  }
  *out = c;
  return QED_OK;
}

void qed_destroy(qed_ctx_t c) {
  if (!c) return;
  (void)hipDeviceSynchronize();
  free_emitters(c);
  free_scan(c);
  free_cands(c);
  void *ptrs[] = {c->rad_lnh64, c->rad_S64, c->rad_lnh32, c->rad_s0sc, c->rad_q16, c->pair_L64,
                  c->pair_S64, c->pair_L32, c->pair_s0sc, c->pair_q16, c->tab_work, c->d_counters,
                  c->d_next_id, c->d_n_emit, c->d_ticket, c->rad_chk, c->mlp_theta[0], c->mlp_theta[1],
                  c->mlp_grad[0], c->mlp_grad[1], c->mlp_m[0], c->mlp_m[1], c->mlp_v[0], c->mlp_v[1],
                  c->sort_keys, c->sort_vals, c->sort_tmp, c->d_killed, c->d_step, c->d_tally};
  for (void *p : ptrs) (void)hipFree(p);
  delete c;
}

const char *qed_last_error(qed_ctx_t c) { return c ? c->err.c_str() : "null context"; }

int qed_reserve(qed_ctx_t c, int64_t n) {
  if (!c) return QED_ERR_ARG;
  if (n <= 0 || n > (int64_t)INT32_MAX) return fail(c, QED_ERR_ARG, "reserve: n must be in [1, 2^31)");
  int r = ensure_scan(c, n);
  return r ? r : ensure_emitters(c, n);
}

int qed_set_next_id(qed_ctx_t c, uint64_t v, void *st) {
  if (!c) return QED_ERR_ARG;
  // the value is copied from a host temporary, so wait for the copy
  hipError_t e = hipMemcpyAsync(c->d_next_id, &v, sizeof(v), hipMemcpyHostToDevice, S(st));
  if (e == hipSuccess) e = hipStreamSynchronize(S(st));
  return e == hipSuccess ? QED_OK : hip_fail(c, e, "set_next_id");
}

int qed_get_next_id(qed_ctx_t c, uint64_t *v, void *st) {
  if (!c || !v) return QED_ERR_ARG;
  hipError_t e = hipMemcpyAsync(v, c->d_next_id, sizeof(*v), hipMemcpyDeviceToHost, S(st));
  if (e == hipSuccess) e = hipStreamSynchronize(S(st));
  return e == hipSuccess ? QED_OK : hip_fail(c, e, "get_next_id");
}

// The surrogate nets cover chi in [1e-3, 1e2] and read the tables at the
// default node positions.
static bool default_range(const qed_ctx *c) {
  return c->range.rad_hi == qed::kRadChiMax && c->range.pair_hi == qed::kPairChiMax;
}

int qed_build_tables(qed_ctx_t c, int formula, void *st) {
  return qed_build_tables_range(c, formula, qed::kRadChiMax, qed::kPairChiMax, st);
}

int qed_build_tables_range(qed_ctx_t c, int formula, double rad_chi_max, double pair_chi_max, void *st) {
  if (!c) return QED_ERR_ARG;
  if (formula != QED_FORMULA_I && formula != QED_FORMULA_II && formula != QED_FORMULA_CLASSICAL)
    return fail(c, QED_ERR_ARG, "formula must be QED_FORMULA_I, QED_FORMULA_II or QED_FORMULA_CLASSICAL");
  using namespace qed;
  if (!(rad_chi_max >= kRadChiMaxLo && rad_chi_max <= kChiMaxHi) ||
      !(pair_chi_max >= kPairChiMaxLo && pair_chi_max <= kChiMaxHi))
    return fail(c, QED_ERR_ARG, "build_tables_range: need 1 <= rad_chi_max <= 1e6 and 10 <= pair_chi_max <= 1e6");
  hipError_t e = hipSuccess;
  if (!c->rad_lnh64) {
    const size_t work = (size_t)(kRadNChi + kPairNRate + kPairNCdf) * (4 * 1024 + 1);
    if ((e = dalloc(&c->rad_lnh64, kRadNChi)) != hipSuccess || (e = dalloc(&c->rad_S64, kRadNChi * kNU)) != hipSuccess ||
        (e = dalloc(&c->rad_lnh32, kRadNChi)) != hipSuccess || (e = dalloc(&c->rad_s0sc, 2 * kRadNChi)) != hipSuccess ||
        (e = dalloc(&c->rad_q16, kRadNChi * kNU)) != hipSuccess || (e = dalloc(&c->pair_L64, kPairNRate)) != hipSuccess ||
        (e = dalloc(&c->pair_S64, kPairNCdf * kNU)) != hipSuccess || (e = dalloc(&c->pair_L32, kPairNRate)) != hipSuccess ||
        (e = dalloc(&c->pair_s0sc, 2 * kPairNCdf)) != hipSuccess || (e = dalloc(&c->pair_q16, kPairNCdf * kNU)) != hipSuccess ||
        (e = dalloc(&c->rad_chk, kRadNChi * 82)) != hipSuccess || (e = dalloc(&c->tab_work, work)) != hipSuccess)
      return hip_fail(c, e, "build_tables: hipMalloc");
    c->tab_work_elems = work;
  }
  c->tables_ready = false;
  const TabRange rg = make_range(rad_chi_max, pair_chi_max);
  if ((e = launch_build_tables(c, formula, rg, S(st))) != hipSuccess) return hip_fail(c, e, "build_tables");
  c->tables_ready = true;
  c->formula = formula;
  c->range = rg;
  return QED_OK;
}

int qed_get_table(qed_ctx_t c, int which, void *host, size_t bytes) {
  if (!c || !host) return QED_ERR_ARG;
  if (!c->tables_ready) return fail(c, QED_ERR_STATE, "tables not built");
  using namespace qed;
  const void *src = nullptr;
  size_t need = 0;
  switch (which) {
    case 0: src = c->rad_lnh64; need = kRadNChi * 8; break;
    case 1: src = c->rad_S64; need = kRadNChi * kNU * 8; break;
    case 2: src = c->pair_L64; need = kPairNRate * 8; break;
    case 3: src = c->pair_S64; need = kPairNCdf * kNU * 8; break;
    case 4: src = c->rad_q16; need = kRadNChi * kNU * 2; break;
    case 5: src = c->rad_s0sc; need = 2 * kRadNChi * 4; break;
    case 6: src = c->pair_q16; need = kPairNCdf * kNU * 2; break;
    case 7: src = c->pair_s0sc; need = 2 * kPairNCdf * 4; break;
    default: return fail(c, QED_ERR_ARG, "get_table: unknown table");
  }
  if (bytes != need) return fail(c, QED_ERR_ARG, "get_table: wrong byte count, need " + std::to_string(need));
  hipError_t e = hipDeviceSynchronize();
  if (e == hipSuccess) e = hipMemcpy(host, src, need, hipMemcpyDeviceToHost);
  return e == hipSuccess ? QED_OK : hip_fail(c, e, "get_table");
}

int qed_init_optical_depth(qed_ctx_t c, qed_species_t *sp, int64_t step, void *st) {
  if (!c) return QED_ERR_ARG;
  int r = check_species(c, sp, "species");
  if (r) return r;
  if (step < 0 && step != QED_STEP_DEVICE) return fail(c, QED_ERR_ARG, "step must be >= 0 or QED_STEP_DEVICE");
  hipError_t e = qed::launch_init_tau(c, sp, step, S(st));
  return e == hipSuccess ? QED_OK : hip_fail(c, e, "init_optical_depth");
}

int qed_fill_standing_wave(qed_ctx_t c, float *grid, int n, double L, double a0, double t, void *st) {
  if (!c) return QED_ERR_ARG;
  if (!grid || n < 3 || n > kMaxWaveGrid || !(L > 0)) return fail(c, QED_ERR_ARG, "fill_standing_wave: bad grid");
  hipError_t e = qed::launch_standing_wave(grid, n, L, a0, t, 0.0, nullptr, S(st));
  return e == hipSuccess ? QED_OK : hip_fail(c, e, "fill_standing_wave");
}

int qed_fill_standing_wave_at_step(qed_ctx_t c, float *grid, int n, double L, double a0, double t0, double dt,
                                   void *st) {
  if (!c) return QED_ERR_ARG;
  if (!grid || n < 3 || n > kMaxWaveGrid || !(L > 0)) return fail(c, QED_ERR_ARG, "fill_standing_wave: bad grid");
  hipError_t e = qed::launch_standing_wave(grid, n, L, a0, t0, dt, c->d_step, S(st));
  return e == hipSuccess ? QED_OK : hip_fail(c, e, "fill_standing_wave_at_step");
}

int qed_set_step(qed_ctx_t c, int64_t step, void *st) {
  if (!c) return QED_ERR_ARG;
  if (step < 0) return fail(c, QED_ERR_ARG, "set_step: step must be >= 0");
  hipError_t e = qed::launch_set_step(c, step, 0, S(st));
  return e == hipSuccess ? QED_OK : hip_fail(c, e, "set_step");
}

int qed_advance_step(qed_ctx_t c, void *st) {
  if (!c) return QED_ERR_ARG;
  hipError_t e = qed::launch_set_step(c, 1, 1, S(st));
  return e == hipSuccess ? QED_OK : hip_fail(c, e, "advance_step");
}

int qed_gather_push(qed_ctx_t c, const qed_fields_t *f, qed_species_t *lep, int charge, double dt,
                    int64_t step, void *st) {
  if (!c) return QED_ERR_ARG;
  int r = check_species(c, lep, "leptons");
  if (r) return r;
  if ((r = check_fields(c, f))) return r;
  if (charge != -1 && charge != 1) return fail(c, QED_ERR_ARG, "charge must be -1 or +1");
  if (!(dt > 0)) return fail(c, QED_ERR_ARG, "dt must be > 0");
  if (!c->tables_ready) return fail(c, QED_ERR_STATE, "tables not built (call qed_build_tables)");
  if ((r = ensure_scan(c, lep->capacity)) || (r = ensure_emitters(c, lep->capacity))) return r;
  if ((c->params.flags & QED_FLAG_SURROGATE) && lep->dtype == QED_F32 && !c->mlp_ready)
    return fail(c, QED_ERR_STATE, "QED_FLAG_SURROGATE: surrogate not trained or loaded");
  if ((c->params.flags & QED_FLAG_SURROGATE) && (c->params.flags & QED_FLAG_METHOD_I))
    return fail(c, QED_ERR_ARG, "QED_FLAG_METHOD_I is not available with QED_FLAG_SURROGATE");
  if ((c->params.flags & QED_FLAG_SURROGATE) && lep->dtype == QED_F32 && !default_range(c))
    return fail(c, QED_ERR_STATE, "QED_FLAG_SURROGATE needs tables of the default chi range");
  if (step < 0 && step != QED_STEP_DEVICE) return fail(c, QED_ERR_ARG, "step must be >= 0 or QED_STEP_DEVICE");
  hipError_t e = qed::launch_gather_push(c, f, lep, charge, dt, step, S(st));
  if (e != hipSuccess) return hip_fail(c, e, "gather_push");
  c->em_owner = lep->x;
  c->em_dtype = lep->dtype;
  c->em_dt = dt;
  return QED_OK;
}

int qed_emit_photons(qed_ctx_t c, qed_species_t *lep, qed_species_t *ph, int64_t step, void *st) {
  if (!c) return QED_ERR_ARG;
  int r = check_species(c, lep, "leptons");
  if (r) return r;
  if ((r = check_species(c, ph, "photons"))) return r;
  if (lep->dtype != ph->dtype) return fail(c, QED_ERR_ARG, "leptons and photons must share dtype");
  if (step < 0 && step != QED_STEP_DEVICE) return fail(c, QED_ERR_ARG, "step must be >= 0 or QED_STEP_DEVICE");
  if (!c->tables_ready) return fail(c, QED_ERR_STATE, "tables not built");
  if (c->em_owner != lep->x || c->em_dtype != lep->dtype)
    return fail(c, QED_ERR_STATE, "emit_photons must follow qed_gather_push on the same leptons");
  hipError_t e = qed::launch_emit(c, lep, ph, step, S(st));
  if (e != hipSuccess) return hip_fail(c, e, "emit_photons");
  c->em_owner = nullptr;
  return QED_OK;
}

int qed_create_pairs(qed_ctx_t c, const qed_fields_t *f, qed_species_t *ph, qed_species_t *el,
                     qed_species_t *po, double dt, int64_t step, void *st) {
  if (!c) return QED_ERR_ARG;
  int r = check_species(c, ph, "photons");
  if (r) return r;
  if ((r = check_species(c, el, "electrons")) || (r = check_species(c, po, "positrons"))) return r;
  if ((r = check_fields(c, f))) return r;
  if (ph->dtype != el->dtype || ph->dtype != po->dtype)
    return fail(c, QED_ERR_ARG, "photons, electrons and positrons must share dtype");
  if (!(dt > 0)) return fail(c, QED_ERR_ARG, "dt must be > 0");
  if (step < 0 && step != QED_STEP_DEVICE) return fail(c, QED_ERR_ARG, "step must be >= 0 or QED_STEP_DEVICE");
  if (!c->tables_ready) return fail(c, QED_ERR_STATE, "tables not built");
  if ((r = ensure_scan(c, ph->capacity))) return r;
  if (ph->dtype == QED_F32 && (r = ensure_cands(c, ph->capacity))) return r;
  hipError_t e = qed::launch_pairs(c, f, ph, el, po, dt, step, S(st));
  return e == hipSuccess ? QED_OK : hip_fail(c, e, "create_pairs");
}

int qed_compact(qed_ctx_t c, qed_species_t *sp, void *st) {
  if (!c) return QED_ERR_ARG;
  int r = check_species(c, sp, "species");
  if (r) return r;
  if ((r = ensure_scan(c, sp->capacity))) return r;
  hipError_t e = qed::launch_compact(c, sp, S(st));
  return e == hipSuccess ? QED_OK : hip_fail(c, e, "compact");
}

int qed_compact_static(qed_ctx_t c, qed_species_t *sp, void *st) {
  if (!c) return QED_ERR_ARG;
  int r = check_species(c, sp, "species");
  if (r) return r;
  if (sp->capacity > kStaticMaxParticles)
    return fail(c, QED_ERR_RANGE, "compact_static: capacity above the static scan state's limit of 2^26 particles");
  uint64_t *w = c->static_scratch;   // this device's copy of `scratch`
  hipError_t e = qed::launch_compact_scan(c, sp, reinterpret_cast<uint32_t *>(w), w + 1, kStaticStatusWords, S(st));
  return e == hipSuccess ? QED_OK : hip_fail(c, e, "compact_static");
}

int qed_sort_by_cell(qed_ctx_t c, const qed_fields_t *f, qed_species_t *src, qed_species_t *dst, void *st) {
  if (!c) return QED_ERR_ARG;
  int r = check_species(c, src, "src");
  if (r) return r;
  if ((r = check_species(c, dst, "dst"))) return r;
  if ((r = check_fields(c, f))) return r;
  if (f->kind != QED_FIELD_GRID) return fail(c, QED_ERR_ARG, "sort_by_cell needs grid fields");
  if (src->dtype != dst->dtype || dst->capacity < src->capacity)
    return fail(c, QED_ERR_ARG, "sort_by_cell: dst must share dtype and hold src's capacity");
  if (src->x == dst->x) return fail(c, QED_ERR_ARG, "sort_by_cell: src and dst must differ");
  hipError_t e = qed::launch_sort_by_cell(c, f, src, dst, S(st));
  return e == hipSuccess ? QED_OK : hip_fail(c, e, "sort_by_cell");
}

int qed_set_retirement(qed_ctx_t c, double t_end, double field_bound) {
  if (!c) return QED_ERR_ARG;
  if (!(t_end >= 0.0) || (t_end > 0.0 && !(field_bound > 0.0)))
    return fail(c, QED_ERR_ARG, "set_retirement: need t_end >= 0 and field_bound > 0");
  if (t_end > 0.0 && !c->d_tally) {
    hipError_t e = dalloc(&c->d_tally, QED_TALLY_BINS);
    if (e == hipSuccess) e = hipMemset(c->d_tally, 0, QED_TALLY_BINS * sizeof(unsigned long long));
    if (e != hipSuccess) return hip_fail(c, e, "set_retirement");
  }
  c->ret_on = t_end > 0.0;
  c->ret_t_end = t_end;
  c->ret_field = field_bound;
  return QED_OK;
}

int qed_tally_species(qed_ctx_t c, const qed_species_t *sp, void *st) {
  if (!c) return QED_ERR_ARG;
  int r = check_species(c, sp, "photons");
  if (r) return r;
  if (!c->d_tally) return fail(c, QED_ERR_STATE, "tally_species: no tally (call qed_set_retirement first)");
  hipError_t e = qed::launch_tally_species(c, sp, S(st));
  return e == hipSuccess ? QED_OK : hip_fail(c, e, "tally_species");
}

int qed_get_tally(qed_ctx_t c, uint64_t *host, int64_t nbins, int clear, void *st) {
  if (!c || !host) return QED_ERR_ARG;
  if (nbins != QED_TALLY_BINS) return fail(c, QED_ERR_ARG, "get_tally: nbins must be QED_TALLY_BINS");
  if (!c->d_tally) return fail(c, QED_ERR_STATE, "get_tally: no tally (call qed_set_retirement first)");
  hipError_t e = hipStreamSynchronize(S(st));
  if (e == hipSuccess) e = hipMemcpy(host, c->d_tally, QED_TALLY_BINS * sizeof(uint64_t), hipMemcpyDeviceToHost);
  if (e == hipSuccess && clear) e = hipMemset(c->d_tally, 0, QED_TALLY_BINS * sizeof(uint64_t));
  return e == hipSuccess ? QED_OK : hip_fail(c, e, "get_tally");
}

int qed_eval_chi(qed_ctx_t c, const qed_fields_t *f, const qed_species_t *sp, int kind, double *chi, void *st) {
  if (!c) return QED_ERR_ARG;
  int r = check_species(c, sp, "species");
  if (r) return r;
  if ((r = check_fields(c, f))) return r;
  if (kind != QED_CHI_LEPTON && kind != QED_CHI_PHOTON) return fail(c, QED_ERR_ARG, "eval_chi: bad kind");
  if (!chi) return fail(c, QED_ERR_ARG, "eval_chi: chi is null");
  hipError_t e = qed::launch_eval_chi(c, f, sp, kind == QED_CHI_PHOTON, chi, S(st));
  return e == hipSuccess ? QED_OK : hip_fail(c, e, "eval_chi");
}

int qed_sample(qed_ctx_t c, const double *chi, const double *gamma, const uint64_t *id, int64_t n,
               int precision, int64_t step, float *lnw, float *xi, float *lnwp, void *st) {
  if (!c) return QED_ERR_ARG;
  if (!chi || !gamma || !id || !lnw || !xi || n < 0) return fail(c, QED_ERR_ARG, "sample: bad arguments");
  if (precision != QED_F32 && precision != QED_F64 && precision != QED_SAMPLER_MLP)
    return fail(c, QED_ERR_ARG, "sample: bad precision");
  if (!c->tables_ready) return fail(c, QED_ERR_STATE, "tables not built");
  if (precision == QED_SAMPLER_MLP && !c->mlp_ready)
    return fail(c, QED_ERR_STATE, "surrogate not trained or loaded");
  if (precision == QED_SAMPLER_MLP && !default_range(c))
    return fail(c, QED_ERR_STATE, "surrogate sampling needs tables of the default chi range");
  if (n == 0) return QED_OK;
  hipError_t e = precision == QED_SAMPLER_MLP
                     ? qed::launch_mlp_sample(c, chi, gamma, id, n, step, lnw, xi, lnwp, 2e-3f, S(st))
                     : qed::launch_sample(c, chi, gamma, id, n, precision, step, lnw, xi, lnwp, S(st));
  return e == hipSuccess ? QED_OK : hip_fail(c, e, "sample");
}

static int mlp_alloc(qed_ctx *c) {
  hipError_t e = hipSuccess;
  for (int k = 0; k < 2 && e == hipSuccess; ++k) {
    if (c->mlp_theta[k]) continue;
    const int n = qed::mlp_params(k);
    if ((e = dalloc(&c->mlp_theta[k], n)) == hipSuccess && (e = dalloc(&c->mlp_grad[k], n)) == hipSuccess &&
        (e = dalloc(&c->mlp_m[k], n)) == hipSuccess && (e = dalloc(&c->mlp_v[k], n)) == hipSuccess)
      e = hipMemset(c->mlp_grad[k], 0, n * sizeof(float));
  }
  return e == hipSuccess ? QED_OK : hip_fail(c, e, "surrogate: hipMalloc");
}

int qed_surrogate_params(int net) { return (net == 0 || net == 1) ? qed::mlp_params(net) : QED_ERR_ARG; }

int qed_surrogate_train(qed_ctx_t c, const qed_train_spec_t *spec, void *st) {
  if (!c || !spec) return QED_ERR_ARG;
  if (!c->tables_ready) return fail(c, QED_ERR_STATE, "tables not built");
  if (!default_range(c)) return fail(c, QED_ERR_STATE, "surrogate training needs tables of the default chi range");
  if (spec->steps < 0 || spec->batch < 16 || spec->batch > (1 << 22) || !(spec->lr > 0))
    return fail(c, QED_ERR_ARG, "train: need steps >= 0, 16 <= batch <= 2^22, lr > 0");
  int r = mlp_alloc(c);
  if (r) return r;
  hipStream_t s = S(st);
  for (int k = 0; k < 2; ++k) {
    if (!(spec->nets & (1 << k))) continue;
    const int n = qed::mlp_params(k);
    hipError_t e = qed::launch_mlp_init(c->mlp_theta[k], k, spec->seed + 977u * k, s);
    if (e == hipSuccess) e = hipMemsetAsync(c->mlp_m[k], 0, n * sizeof(float), s);
    if (e == hipSuccess) e = hipMemsetAsync(c->mlp_v[k], 0, n * sizeof(float), s);
    if (e == hipSuccess) e = hipMemsetAsync(c->mlp_grad[k], 0, n * sizeof(float), s);
    double b1t = 1.0, b2t = 1.0;
    for (int64_t it = 0; it < spec->steps && e == hipSuccess; ++it) {
      const double lr = spec->lr * 0.5 * (1.0 + cos(3.141592653589793 * (double)it / (double)spec->steps));
      b1t *= 0.9; b2t *= 0.999;
      e = qed::launch_mlp_grad(k, c->mlp_theta[k], c->mlp_grad[k], c->rad_S64, c->rad_lnh64, c->pair_L64, nullptr,
                               nullptr, nullptr, spec->batch, (uint64_t)it * (uint64_t)spec->batch, spec->seed, s);
      if (e == hipSuccess)
        e = qed::launch_adam(c->mlp_theta[k], c->mlp_grad[k], c->mlp_m[k], c->mlp_v[k], k, (float)lr,
                             (float)b1t, (float)b2t, s);
    }
    if (e != hipSuccess) return hip_fail(c, e, "surrogate_train");
  }
  for (int k = 0; k < 2; ++k)
    if (spec->nets & (1 << k)) c->mlp_have[k] = true;
  c->mlp_ready = c->mlp_have[0] && c->mlp_have[1];
  return QED_OK;
}

int qed_surrogate_io(qed_ctx_t c, int net, float *host, size_t bytes, int direction) {
  if (!c || !host || (net != 0 && net != 1) || (direction != 0 && direction != 1)) return QED_ERR_ARG;
  const size_t need = (size_t)qed::mlp_params(net) * sizeof(float);
  if (bytes != need) return fail(c, QED_ERR_ARG, "surrogate_io: wrong byte count, need " + std::to_string(need));
  int r = mlp_alloc(c);
  if (r) return r;
  hipError_t e = hipDeviceSynchronize();
  if (e == hipSuccess)
    e = direction == 0 ? hipMemcpy(host, c->mlp_theta[net], need, hipMemcpyDeviceToHost)
                       : hipMemcpy(c->mlp_theta[net], host, need, hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(c, e, "surrogate_io");
  if (direction == 1) {
    c->mlp_have[net] = true;
    c->mlp_ready = c->mlp_have[0] && c->mlp_have[1];
  }
  return QED_OK;
}

int qed_surrogate_forward(qed_ctx_t c, int net, const float *x, int64_t n, float *y, void *st) {
  if (!c || !x || !y || n < 0 || (net != 0 && net != 1)) return QED_ERR_ARG;
  if (!c->mlp_theta[net]) return fail(c, QED_ERR_STATE, "surrogate weights not set");
  if (n == 0) return QED_OK;
  hipError_t e = qed::launch_mlp_forward(c->mlp_theta[net], net, x, n, y, S(st));
  return e == hipSuccess ? QED_OK : hip_fail(c, e, "surrogate_forward");
}

int qed_surrogate_grad(qed_ctx_t c, int net, const float *x, const float *t, const float *mask, int64_t n,
                       float *grad, void *st) {
  if (!c || !x || !t || !grad || n < 1 || (net != 0 && net != 1)) return QED_ERR_ARG;
  if (!c->mlp_theta[net]) return fail(c, QED_ERR_STATE, "surrogate weights not set");
  hipError_t e = hipMemsetAsync(grad, 0, qed::mlp_params(net) * sizeof(float), S(st));
  if (e == hipSuccess)
    e = qed::launch_mlp_grad(net, c->mlp_theta[net], grad, nullptr, nullptr, nullptr, x, t, mask, n, 0, 0, S(st));
  return e == hipSuccess ? QED_OK : hip_fail(c, e, "surrogate_grad");
}

static_assert(sizeof(qed_counters_t) == sizeof(int64_t) * qed::cNumCounters, "counter layout");

int qed_get_status(qed_ctx_t c, qed_counters_t *out, void *st) {
  if (!c || !out) return QED_ERR_ARG;
  unsigned long long h[qed::cNumCounters];
  hipError_t e = hipStreamSynchronize(S(st));
  if (e == hipSuccess) e = hipMemcpy(h, c->d_counters, sizeof(h), hipMemcpyDeviceToHost);
  if (e == hipSuccess) e = hipMemset(c->d_counters, 0, sizeof(h));
  if (e != hipSuccess) return hip_fail(c, e, "get_status");
  int64_t *o = (int64_t *)out;
  for (int k = 0; k < qed::cNumCounters; ++k) o[k] = (int64_t)h[k];
  if (out->scan_timeouts) return fail(c, QED_ERR_STATE, "prefix scan timed out");
  if (out->dropped) return fail(c, QED_ERR_CAPACITY, "appends dropped: species capacity exceeded");
  return QED_OK;
}

}  // extern "C"
