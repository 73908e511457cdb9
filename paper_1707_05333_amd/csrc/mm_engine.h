// The engine behind both public front ends (one simulation per mm_ctx, many
// per mm_batch): the device memory of the internal (bucket-sorted) cell
// space, the segment table, the enqueue order of a tessellation and of a
// whole step, and the single status readback.  Host code only.
#pragma once

#include <hip/hip_runtime.h>

#include <string>

#include "../../include/mm.h"
#include "mm_internal.h"

namespace mm {

// Bytes of device memory the engine reserves per unit of capacity: per
// internal cell (faces at kFacesPerCell unique faces per cell included) and
// per slot of a caller-order pool.
constexpr int64_t kFacesPerCell = 12;
// Sliced-ELL list entries reserved per cell (a slice is as wide as its
// longest list: about 20 for jittered lattices, 30 for Poisson points).
constexpr int64_t kListPerCell = 40;
int64_t engine_bytes_per_cell(int precision);

// Bucket grid of a segment of n points in box p.box whose buckets start at
// `base` in the shared table.  Buckets are about one mean spacing wide
// whatever rfac, so the cell order (bucket, then slot) and with it every
// result do not depend on the candidate radius.
GridParams make_grid(const mm_params& p, int64_t n, double rfac, int64_t base);
HydroParams hydro_params(const mm_params& p);
bool params_ok(const mm_params* p, std::string& why);

struct Engine {
  int precision = MM_FP64;
  int64_t ncap = 0, slot_cap = 0, fcap = 0, nbcap = 0, sell_cap = 0;
  int segcap = 0;
  hipStream_t stream = nullptr;
  int device = 0;
  // Sort and tessellation.
  int32_t *key = nullptr, *perm = nullptr, *sseg = nullptr, *deferred = nullptr, *dcells = nullptr, *redo = nullptr;
  double *spos = nullptr, *geo = nullptr, *rmax2 = nullptr, *minv = nullptr;
  unsigned long long *bcount = nullptr, *boff = nullptr, *scan_tmp = nullptr, *counts = nullptr, *off = nullptr;
  unsigned long long* sbase = nullptr;   // sub-table base of each bucket (dense buckets)
  uint32_t* soffs = nullptr;             // sub-bucket offsets of the dense buckets
  unsigned long long *sw = nullptr, *soff = nullptr;   // slice widths and offsets of the per-cell lists
  StageNbr* stage_nb = nullptr;
  StageGeo* stage_geo = nullptr;
  Face* faces = nullptr;
  int32_t* csr = nullptr;
  void* nbr = nullptr;   // NbrEntry<R>[sell_cap]
  // State in internal order.
  void *U = nullptr, *G = nullptr, *Uh = nullptr, *rec = nullptr, *phi = nullptr;   // rec: FluxCell<R>[n]
  double *w = nullptr, *Qs = nullptr;
  double* pn = nullptr;   // positions after the drift, before they are committed
  // Half-step mesh (single simulations): positions r + w dt/2 and the
  // half-step states and mesh velocities parked in slot order while the
  // mesh is rebuilt.  Reserved only when init is asked for them.
  double* pos_half = nullptr;
  void* Uh_slots = nullptr;
  // Entropy column (single simulations): X and its half-step value per
  // cell, the face kernel's records, the face fluxes and Mach numbers, and
  // the gathered entropy charges.
  void *Xe = nullptr, *Xh = nullptr, *recx = nullptr, *phiX = nullptr;
  float* machF = nullptr;
  float* machs = nullptr;   // per cell, internal order
  double* Ss = nullptr;
  // Segment table and status.
  SegDesc* segs = nullptr;
  SegStatus* segst = nullptr;
  DevStatus* st = nullptr;
  SegDesc* segs_host = nullptr;       // pinned staging of the table
  SegStatus* segst_host = nullptr;    // pinned mirror
  DevStatus* st_host = nullptr;       // pinned mirror
  hipEvent_t upload_done = nullptr;
  int nseg = 0;
  // Mesh currently held.
  int64_t n = 0, n_faces = 0, nbt = 0;
  // List lengths of the last tessellation read back (none yet: -1); they
  // size the list passes' grids only.  last_dense_cap: the listed dense
  // cells the last two-cell dense pass took.
  TessHints hints;
  int64_t last_dense_cap = 0;
  // First-pass candidate radius in mean spacings.  It changes only the
  // work, never the cells (clipping is always in order of distance, ties
  // broken by neighbour and image).  With the first pass taking up to three
  // extra shells, 1.9 beat 1.5, 1.7, 2.2 and 2.4 on the Sod tube (early and
  // late), on uniform random points and on the two polytropes; an earlier
  // rule that widened it after many deferrals made those inputs slower.
  double rfac = 1.9;
  // Stage timing.
  bool timing = false;
  hipEvent_t ev[11] = {};   // 0-8 the step's stages, 9-10 around the half-step remesh
  double stage_ms[9] = {};  // sort, cells, mesh, cell_state, gradient_predict, gradient_half, flux, update, remesh
  bool remeshed = false;
  std::string err;

  // Reserves everything; returns MM_OK or MM_ENOMEM / MM_EHIP with err set.
  // single: also reserve the half-step mesh and entropy buffers.
  mm_status init(int precision, int64_t ncap, int64_t slot_cap, int64_t fcap, int segcap, hipStream_t stream,
                 bool single = false);
  // The same buffers (one segment, no half-step mesh or entropy column)
  // carved from the given device arena, with the given host memory as the
  // status mirrors: nothing is allocated, and no events exist (no stage
  // timing).  MM_ECAPACITY when they do not fit.
  mm_status init_arena(int precision, int64_t ncap, int64_t fcap, void* arena, size_t bytes, SegDesc* seg_host,
                       SegStatus* seg_status_host, DevStatus* status_host, hipStream_t stream);
  // Bytes init_arena needs (its alignment included).
  static size_t arena_bytes(int precision, int64_t ncap, int64_t fcap);
  void set_capacity(int precision, int64_t ncap, int64_t slot_cap, int64_t fcap, int segcap);
  void release();
  bool arena_mode = false;

  // Host staging of the segment table, safe to write once returned; then
  // upload(nseg) copies the first nseg descriptors (stream-ordered).
  SegDesc* staging();
  mm_status upload(int nseg);
  void reset_status();
  // Sort, cell construction and mesh assembly of n cells living in n_slots
  // caller-order slots (slot_seg: segment per slot, NULL for one segment).
  void enqueue_tessellation(const double* pos, int64_t n_slots, const int32_t* slot_seg, int64_t n, int64_t nbt);
  // One whole step: tessellation, charges of fresh segments, states, two
  // gradients with the predictor, fluxes, update and drift.  Q, pos and w
  // are slot-order arrays, updated in place.
  // half_step: rebuild the mesh at r + w dt/2 after the predictor and take
  // the second gradient, the fluxes and the update on it (single segment,
  // n_slots == n, buffers reserved at init).
  // S, mach (single segment, buffers reserved at init): the entropy
  // charges in/out and each cell's largest face Mach number out (Sec. 4.3).
  void enqueue_step(double* pos, double* w, double* Q, int64_t n_slots, const int32_t* slot_seg, int64_t n,
                    int64_t nbt, bool any_fresh, bool half_step = false, double* S = nullptr,
                    float* mach = nullptr);
  // Waits for the stream and copies the status of the launch set and of
  // the first nseg segments to the host mirrors.
  mm_status readback();
  void finish_timing();
  // Status code and message for failure bits (of the whole set or a segment).
  mm_status check_flags(int flags, int bad_cell, std::string& msg) const;
  mm_status fail(mm_status code, const std::string& msg) {
    err = msg;
    return code;
  }
  void mark(int k) {
    if (timing && !arena_mode) (void)hipEventRecord(ev[k], stream);
  }
};

double dt_from_bits(unsigned long long bits);

}  // namespace mm
