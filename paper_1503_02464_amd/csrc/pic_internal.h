// Internal declarations of the PIC library: the context, the workspace layout
// and the kernel launchers (one per phase, dispatching on precision, number of
// dimensions and shape order).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <utility>
#include <vector>

#include "pic.h"

namespace pic {

constexpr int kMaxSpecies = 8;         // species per diagnostics call
constexpr int kMaxSortLevels = 128;    // largest pic_params.sort_levels
constexpr int kDiagBlocks = 1024;      // partial sums per species / per grid pass
constexpr int kDiagSlots = PIC_NDIAG;  // UE UB K Q max|rho| max|G| max|dG| max|cont|
// Largest grid (nodes) of the allocation-free diagnostics, whose charge grid
// lives in a fixed device array, and the devices it keeps an address for.
constexpr int64_t kScratchCells = PIC_NOALLOC_MAX_CELLS;
constexpr int kMaxDevices = 64;
// Output extraction: grids per call, and the storage slots one workgroup of
// the particle selection scans (its count is one workspace entry).
constexpr int kMaxExtractGrids = PIC_MAX_EXTRACT_GRIDS;
constexpr int64_t kSelectChunk = 8192;
// Largest capacity of the fused kernel's list of particles that need the
// wide Esirkepov window (their nearest node changed), per precision; the
// context lowers it to what the LDS left by the field and current boxes holds.
constexpr int kCrossCapF32 = 512;
constexpr int kCrossCapF64 = 256;
constexpr size_t kLdsLimit = 160 * 1024;
// LDS bytes of a list of cap entries: old and new offsets, weight, v_z
// factor, packed cell; plus its length.
inline size_t cross_list_bytes(size_t elem, int cap) { return static_cast<size_t>(cap) * (8 * elem + 4) + 16; }

// Plane stride of the fused kernel's LDS current box (elements).  In 3D it
// is padded to the next value that is 7 mod 16: with the 15-element rows of
// an 8^3 tile's box, the window bases' element indices then fall evenly into
// the 16 residue classes that decide the LDS unit's 8-byte atomic replays.
__host__ __device__ constexpr int current_plane_stride(int jx, int jy, int dims) {
  return dims == 3 ? jx * jy + ((7 - jx * jy) % 16 + 16) % 16 : jx * jy;
}

// Byte offsets of the workspace regions (each 256-byte aligned).
struct Workspace {
  size_t flags = 0;       // int32[64]: sticky device flags
  size_t save_cell = 0;   // int32[max_particles]: packed cell at x^n (unfused path)
  size_t save_off = 0;    // T[3][max_particles]: offsets at x^n (unfused path)
  size_t sort_key = 0;    // int32[max_particles]
  size_t sort_rank = 0;   // int32[max_particles]
  size_t sort_src = 0;    // int32[max_particles]: the particle each sorted slot takes
  size_t stray_count = 0; // int32[2][16]: two banks of the tiled kernel's counters ([0] the particles it left
                          // outside their LDS box, [1..8] its tile queues)
  size_t stray_list = 0;  // int32[max_particles]: their indices
  size_t stay_count = 0;    // int32[ntiles * levels]: per (tile, level) bucket, particles that stayed in the tile
  size_t arrive_count = 0;  // int32[ntiles * levels]: per bucket, the others
  size_t bucket_start = 0;   // int32[kMaxSpecies][nbuckets + 1]: bucket starts of each species' last sort
  size_t scan_partials = 0;  // int64[scan blocks]
  size_t live_tiles = 0;     // int32[kMaxSpecies][ntiles + 1]: per species slot, the tiles its last sort
                             // left non-empty, in tile order, then their count
  size_t dense_tiles = 0;    // int32[kMaxSpecies][ntiles + 1]: of those, the ones with kSparseTile particles or more
  size_t sparse_tiles = 0;   // int32[kMaxSpecies][ntiles + 1]: and the others (3D; empty in 2D)
  size_t wmax_tiles = 0;     // uint32[kMaxSpecies][ntiles]: per tile, the bits of its largest |w| (FP32) as
                             // the first fused launch after the slot's last sort found it
  size_t partials = 0;    // double[kDiagSlots][kMaxSpecies * kDiagBlocks]
  size_t result = 0;      // double[16]
  size_t rho = 0;         // double[ncells]
  size_t rho_prev = 0;    // double[ncells]
  size_t gauss_prev = 0;  // double[ncells]
  size_t mur_old = 0;     // T[8][n1 * n2]: E_y, E_z^n of the planes next to the open x faces
  size_t select_base = 0; // int64[ceil(max_particles / kSelectChunk) + 1]: particle selection per chunk
  size_t total = 0;
};

enum Flag : int32_t { kFlagCross = 1, kFlagSort = 2 };

enum Phase { kPhaseSort = 0, kPhaseZero = 1, kPhasePush = 2, kPhaseYee = 3 };

}  // namespace pic

struct pic_ctx {
  pic_params p{};
  int64_t n[3] = {1, 1, 1};
  int64_t ncells = 0;
  int32_t bits[3] = {0, 0, 0};
  int32_t ntile[3] = {1, 1, 1};
  int64_t ntiles = 0;
  size_t elem = 4;  // sizeof(float) or sizeof(double)
  // LDS tile geometry of the fused kernel: field and current regions per
  // dimension, starting gf_lo / gj_lo cells below the tile origin.
  int32_t rf[3] = {1, 1, 1}, rj[3] = {1, 1, 1};
  int32_t jxy = 1;  // plane stride of the current box (current_plane_stride)
  int32_t gf_lo[3] = {0, 0, 0}, gj_lo[3] = {0, 0, 0};
  size_t lds_bytes = 0;
  bool acc64 = true;  // LDS current box 8 bytes per value (double or 64-bit fixed point)
  bool accfix = false;  // LDS current box in 64-bit fixed point (FP32 state)
  int32_t cross_cap = 0;  // capacity of the fused kernel's wide-window list
  int32_t levels = 32;  // rank levels per tile in the sort (particles sharing a node go to distinct levels)
  // (tile_start array, particle count) of every species this context sorted
  // (at most kMaxSpecies; entry i owns bucket-start slot i of the workspace):
  // the next sort of that species ranks by the runs tile_start describes
  std::vector<std::pair<const int32_t *, int64_t>> sorted_runs;
  // Open x faces: each sort's live count (tile_start[ntiles]) of species slot
  // i, copied to pinned host memory without waiting; the next sort of that
  // species drops the removed particles once the copy's event has completed.
  int32_t *live_host = nullptr;  // pinned, kMaxSpecies entries (allocated on first use)
  hipEvent_t live_event[pic::kMaxSpecies] = {};
  bool live_pending[pic::kMaxSpecies] = {};
  // The fixed-point current's per-tile weight bound: true once a fused launch
  // has stored it for slot i's current sort (cleared by every sort of the slot)
  mutable bool wmax_known[pic::kMaxSpecies] = {};  // set by the launch (which sees the context as const)
  // The fused launches alternate between the two counter banks: each launch's
  // straggler kernel clears the bank the next launch takes, so a launch needs
  // no clear of its own unless the chain broke (a failed call, a new workspace).
  mutable int stray_bank = 0;       // the bank the next fused launch takes
  mutable int stray_last = 0;       // the bank of the last fused launch
  mutable bool stray_clean = false; // the next bank is known to be zero
  bool has_laser = false;
  pic_laser laser{};
  double laser_j0 = 0.0;  // sheet amplitude radiating laser.e0 on the lattice
  pic::Workspace ws;
  char *wsptr = nullptr;
  size_t wsbytes = 0;
  // the species whose old positions the workspace holds (pic_gather_push -> pic_deposit)
  const void *pending_cell = nullptr;
  int64_t pending_np = -1;
  int64_t step = 0;
  int64_t diag_step = -1;  // step count at the previous pic_diagnostics call
  // per-phase timing
  bool timing = false;
  struct Ev {
    int phase;
    hipEvent_t a, b;
  };
  std::vector<Ev> events;
  std::vector<hipEvent_t> spare;
  double ms[PIC_NPHASE] = {0, 0, 0, 0};
  int64_t launches[PIC_NPHASE] = {0, 0, 0, 0};
  std::string err;

  template <typename X>
  X *wsp(size_t off) const { return reinterpret_cast<X *>(wsptr + off); }
};

namespace pic {

// Kernel launchers (device code in the .hip files).  Each returns the HIP
// error of its launches.
hipError_t launch_gather_push(const pic_ctx &c, const pic_species &sp, const pic_fields &f, hipStream_t s);
hipError_t launch_deposit(const pic_ctx &c, const pic_species &sp, const pic_fields &f, hipStream_t s);
// src: when not null, the slots of a sort whose copy was left to this launch
// (particle q of the sorted order is particle src[q] of the current set, which
// holds np_src particles: the sort may have dropped removed ones from np); the
// launch writes every particle into the second set and swaps the sets.
hipError_t launch_push_deposit_tiled(const pic_ctx &c, pic_species &sp, const pic_fields &f, hipStream_t s,
                                     const int32_t *src = nullptr, int64_t np_src = 0);
hipError_t launch_fill_zero(void *ptr, int64_t n, size_t elem, hipStream_t s);
// Zero count (1..kFillArrays) arrays of n elements each in one launch.
constexpr int kFillArrays = 4;
hipError_t launch_fill_zero_n(void *const *ptrs, int count, int64_t n, size_t elem, hipStream_t s);
// Open x faces: save = true keeps E_y, E_z^n next to the faces (before the E
// update), save = false applies the Mur update to the faces (after it).
hipError_t launch_mur(const pic_ctx &c, const pic_fields &f, bool save, hipStream_t s);
// J += the registered laser sheet at time t.
hipError_t launch_laser(const pic_ctx &c, const pic_fields &f, double t, hipStream_t s);
hipError_t launch_yee_b(const pic_ctx &c, const pic_fields &f, double frac, hipStream_t s);
// The one-pass Yee step into the second field set (3D; x and y divisible by
// its tile; f.E_alt and f.B_alt set), and whether it applies.
bool yee_fused_ok(const pic_ctx &c, const pic_fields &f);
hipError_t launch_yee_fused(const pic_ctx &c, const pic_fields &f, hipStream_t s);
// E += frac dt curl B (- dt J when with_j)
hipError_t launch_yee_e(const pic_ctx &c, const pic_fields &f, hipStream_t s, double frac = 1.0, bool with_j = true);
// Adjoint kernels.
hipError_t launch_scale_copy(const pic_ctx &c, void *const dst[3], const void *const src[3], double scale,
                             hipStream_t s);
hipError_t launch_particle_adjoint(const pic_ctx &c, const pic_species &sp, const pic_fields &f,
                                   const pic_fields &lam, const pic_species_adjoint &lsp, hipStream_t s);
// fold_src: when not null, the copy into the second set is left to the next
// fused push (*fold_src receives the slots; null if the sort copied anyway).
// With open x faces, wait = true drops the removed particles from np at once
// (synchronising); wait = false drops those of the previous sort of this
// species if its live count has reached the host, and starts the copy of
// this sort's count.
hipError_t launch_sort(pic_ctx &c, pic_species &sp, hipStream_t s, const int32_t **fold_src = nullptr,
                       bool wait = true);
void swap_sets(pic_species &sp);
// The non-empty tiles of a species' last sort (list, count at [ntiles]), or
// null when this context has not sorted that species.
const int32_t *live_tiles(const pic_ctx &c, const pic_species &sp);
// A 3D tile that its last sort left with fewer than kSparseTile particles is
// not staged by the in-place fused launches: the straggler kernel steps its
// particles against the fields and current in HBM.  These return the two
// parts of the live list (same layout), or null where live_tiles does.
constexpr int kSparseTile = 32;
const int32_t *dense_tiles(const pic_ctx &c, const pic_species &sp);
const int32_t *sparse_tiles(const pic_ctx &c, const pic_species &sp);
// The workspace slot of the species' last sort (as live_tiles finds it), or -1.
int sorted_slot(const pic_ctx &c, const pic_species &sp);

int64_t sort_scan_blocks(int64_t nbuckets);
int64_t sort_scan_capacity();
hipError_t launch_diagnostics(const pic_ctx &c, const pic_species *sp, int nspecies, const pic_fields &f,
                              bool have_prev, bool have_cont, hipStream_t s);
// rho (and, when gauss is not null, div E - rho) into caller-owned FP64 grids.
hipError_t launch_charge_density(const pic_ctx &c, const pic_species *sp, int nspecies, const pic_fields *f,
                                 double *rho, double *gauss, hipStream_t s);
// The device address of this device's copy of the allocation-free
// diagnostics' scratch array (looked up once per device).
hipError_t scratch_address(double **out);
// Diagnostics without history into that scratch; the result's 8 doubles sit
// at scratch_result_offset() doubles from its start.
hipError_t launch_diagnostics_noalloc(const pic_ctx &c, const pic_species *sp, int nspecies, const pic_fields &f,
                                      double *scratch, hipStream_t s);
size_t scratch_result_offset();

// Points of a box along dimension d (0 when hi <= lo).
inline int64_t box_points(const pic_box &b, int d) {
  return b.hi[d] > b.lo[d] ? (static_cast<int64_t>(b.hi[d]) - b.lo[d] + b.stride[d] - 1) / b.stride[d] : 0;
}
// Output extraction (callers validate the box against the grid).
hipError_t launch_extract_grid(const pic_ctx &c, const void *const *grids, int32_t ngrids, int32_t elem_bytes,
                               const pic_box &box, void *dst, hipStream_t s);
hipError_t launch_extract_particles(const pic_ctx &c, const pic_species &sp, const pic_box &cells, int64_t every,
                                    void *dst, int64_t capacity, int64_t *count, hipStream_t s);

}  // namespace pic
