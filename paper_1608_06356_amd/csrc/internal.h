// Host-side context of the QED step library and the launchers the entry points use.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string>

#include "../../include/qed.h"
#include "lookup.h"

// Bytes of one emitter record slot (the float64 record; the float32 one is smaller).
constexpr int64_t kEmRecMaxBytes = 128;
// Entry of the ordered emitter list: particle index and its record slot.
struct alignas(8) EmIdx {
  int32_t i, slot;
};

// Particles per tile of the compaction scan (one status word per tile).
constexpr int64_t kCompactTile = 1024;

// Largest node count per side of qed_fill_standing_wave grids.
constexpr int kMaxWaveGrid = 4096;

struct qed_ctx {
  int device = 0;
  qed_params_t params{};
  std::string err;

  // tables (library-owned device memory)
  bool tables_ready = false;
  int formula = 0;
  qed::TabRange range = qed::make_range(qed::kRadChiMax, qed::kPairChiMax);   // grids of the built tables
  double *rad_lnh64 = nullptr, *rad_S64 = nullptr;       // [256], [256*256]
  float *rad_lnh32 = nullptr, *rad_s0sc = nullptr;       // [256], [2*256]
  uint16_t *rad_q16 = nullptr;                           // [256*256]
  double *pair_L64 = nullptr, *pair_S64 = nullptr;       // [512], [256*256]
  float *pair_L32 = nullptr, *pair_s0sc = nullptr;       // [512], [2*256]
  uint16_t *pair_q16 = nullptr;
  float *rad_chk = nullptr;                              // [256 * 82] Hermite CDF check rows
  double *tab_work = nullptr;                            // quadrature scratch
  size_t tab_work_elems = 0;

  // counters and ids
  unsigned long long *d_counters = nullptr;              // qed_counters_t layout
  uint64_t *d_next_id = nullptr;
  int64_t *d_step = nullptr;     // device step index (QED_STEP_DEVICE)

  // emitter list produced by qed_gather_push
  int64_t reserved = 0;          // species size the scan state covers
  int64_t em_cap = 0;            // emitter slots (one per lepton of the largest lepton species)
  uint64_t *em_mask = nullptr;   // one bit per particle: optical depth ran out this step
  EmIdx *em_idx = nullptr;       // ordered emitter list
  unsigned char *em_rec = nullptr;   // em_cap records of up to kEmRecMaxBytes, slot = particle index
  int32_t *cont_idx = nullptr;   // surrogate emission: emitters with a further candidate (list positions)
  int64_t *d_n_cont = nullptr;
  int64_t *d_n_emit = nullptr;
  const void *em_owner = nullptr;   // species (x pointer) the list belongs to
  int em_dtype = -1;
  int em_charge = 0;
  double em_dt = 0.0;

  // photons of the float32 pair pass with an event (surrogate path: a
  // candidate event) this step: ballot mask and ordered list (sized for the
  // largest photon species)
  int64_t cand_cap = 0;
  uint64_t *cand_mask = nullptr;
  int32_t *cand_idx = nullptr;
  int64_t *d_n_cand = nullptr;

  // dead-particle count of the species compacted last (pairs add to it; compaction
  // skips its work when it is zero)
  int64_t *d_killed = nullptr;
  const void *killed_owner = nullptr;

  // decoupled look-back scan state: two tickets and two status regions of
  // status_len words; region 1 serves the emitter index so that one launch can
  // clear the state of both scans of qed_emit_photons
  uint32_t *d_ticket = nullptr;
  uint64_t *d_status = nullptr;
  int64_t status_len = 0;

  int n_cu = 256;

  // photon retirement (qed_set_retirement) and the tally of retired photons
  int ret_on = 0;
  double ret_t_end = 0.0, ret_field = 0.0;
  unsigned long long *d_tally = nullptr;

  // device address of the library's static scratch array on this context's
  // device (qed_compact_static)
  uint64_t *static_scratch = nullptr;

  // cell sort scratch
  uint32_t *sort_keys = nullptr, *sort_vals = nullptr;
  int64_t sort_cap = 0;
  void *sort_tmp = nullptr;
  size_t sort_tmp_bytes = 0;

  // surrogate networks (0: xi net, 1: rate net): float32 parameters, Adam state
  bool mlp_ready = false;
  bool mlp_have[2] = {false, false};   // parameters of net A / net B trained or loaded
  float *mlp_theta[2] = {nullptr, nullptr}, *mlp_grad[2] = {nullptr, nullptr};
  float *mlp_m[2] = {nullptr, nullptr}, *mlp_v[2] = {nullptr, nullptr};
};

namespace qed {
hipError_t mlp_set_attributes();
hipError_t step_set_attributes();
hipError_t launch_build_tables(qed_ctx *c, int formula, TabRange rg, hipStream_t s);
int mlp_params(int net);
hipError_t launch_sort_by_cell(qed_ctx *c, const qed_fields_t *f, const qed_species_t *s, qed_species_t *d,
                               hipStream_t st);
hipError_t launch_mlp_init(float *theta, int net, uint32_t seed, hipStream_t st);
hipError_t launch_mlp_grad(int net, const float *theta, float *grad, const double *S64, const double *lnh,
                           const double *L, const float *ext_x, const float *ext_t, const float *ext_m,
                           int64_t nbatch, uint64_t sample0, uint32_t seed, hipStream_t st);
hipError_t launch_adam(float *theta, float *grad, float *m, float *v, int net, float lr, float b1t, float b2t,
                       hipStream_t st);
hipError_t launch_mlp_forward(const float *theta, int net, const float *x, int64_t n, float *y, hipStream_t st);
hipError_t launch_mlp_sample(qed_ctx *c, const double *chi, const double *gamma, const uint64_t *id, int64_t n,
                             int64_t step, float *lnw, float *xi, float *lnwp, float tol, hipStream_t st);
}

namespace qed {
hipError_t launch_gather_push(qed_ctx *c, const qed_fields_t *f, const qed_species_t *sp, int charge,
                              double dt, int64_t step, hipStream_t st);
hipError_t launch_emit(qed_ctx *c, const qed_species_t *lep, const qed_species_t *ph, int64_t step,
                       hipStream_t st);
hipError_t launch_pairs(qed_ctx *c, const qed_fields_t *f, const qed_species_t *ph,
                        const qed_species_t *el, const qed_species_t *po, double dt, int64_t step,
                        hipStream_t st);
hipError_t launch_compact(qed_ctx *c, const qed_species_t *sp, hipStream_t st);
// The same with the scan state given by the caller: a ticket word and
// status_len status words (at least capacity / kCompactTile + 2).
hipError_t launch_compact_scan(qed_ctx *c, const qed_species_t *sp, uint32_t *ticket, uint64_t *status,
                               int64_t status_len, hipStream_t st);
hipError_t launch_init_tau(qed_ctx *c, const qed_species_t *sp, int64_t step, hipStream_t st);
hipError_t launch_standing_wave(float *grid, int n, double L, double a0, double t0, double dt_step,
                                const int64_t *d_step, hipStream_t st);
hipError_t launch_set_step(qed_ctx *c, int64_t v, int add, hipStream_t st);
hipError_t launch_tally_species(qed_ctx *c, const qed_species_t *sp, hipStream_t st);
hipError_t launch_eval_chi(qed_ctx *c, const qed_fields_t *f, const qed_species_t *sp, int photon, double *out,
                           hipStream_t st);
hipError_t launch_sample(qed_ctx *c, const double *chi, const double *gamma, const uint64_t *id,
                         int64_t n, int precision, int64_t step, float *lnw, float *xi, float *lnwp,
                         hipStream_t st);
}  // namespace qed
