// Host side of the C ABI declared in pic.h: parameter validation, workspace
// layout, phase ordering, per-phase timing and error reporting.  No call
// allocates device memory; every launch goes on the caller's stream.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <utility>

#include "pic_internal.h"

namespace {

size_t align256(size_t x) { return (x + 255) & ~static_cast<size_t>(255); }

int ceil_log2(int64_t n) {
  int b = 0;
  while ((int64_t(1) << b) < n) ++b;
  return b;
}

pic_status fail(pic_ctx *c, pic_status s, const char *msg) {
  if (c) c->err = msg;
  return s;
}

pic_status hip_fail(pic_ctx *c, hipError_t e, const char *where) {
  if (c) {
    c->err = std::string(where) + ": " + hipGetErrorString(e);
  }
  return PIC_EHIP;
}

bool fields_ok(const pic_fields *f) {
  if (!f) return false;
  for (int d = 0; d < 3; ++d)
    if (!f->E[d] || !f->B[d] || !f->J[d]) return false;
  return true;
}

bool species_ok(const pic_ctx *c, const pic_species *s, bool need_alt) {
  if (!s) return false;
  if (s->np < 0 || s->np > c->p.max_particles) return false;
  if (!(s->m > 0.0) || !std::isfinite(s->q)) return false;
  if (s->np == 0) return true;
  if (!s->cell || !s->w) return false;
  for (int d = 0; d < c->p.dims; ++d)
    if (!s->off[d]) return false;
  for (int d = 0; d < 3; ++d)
    if (!s->u[d]) return false;
  if (need_alt) {
    if (!s->cell_alt || !s->w_alt || !s->tile_start) return false;
    for (int d = 0; d < c->p.dims; ++d)
      if (!s->off_alt[d]) return false;
    for (int d = 0; d < 3; ++d)
      if (!s->u_alt[d]) return false;
  }
  return true;
}

// Record the start of a timed phase (no-op unless timing is on).
struct PhaseTimer {
  pic_ctx *c;
  hipStream_t s;
  int phase;
  hipEvent_t a = nullptr;
  PhaseTimer(pic_ctx *c_, hipStream_t s_, int ph) : c(c_), s(s_), phase(ph) {
    if (!c->timing) return;
    a = take();
    if (a && hipEventRecord(a, s) != hipSuccess) {
      c->spare.push_back(a);
      a = nullptr;
    }
  }
  // A recycled event, or a new one (null if it cannot be created: that
  // phase then goes untimed).
  hipEvent_t take() {
    hipEvent_t e = nullptr;
    if (!c->spare.empty()) {
      e = c->spare.back();
      c->spare.pop_back();
    } else if (hipEventCreate(&e) != hipSuccess) {
      e = nullptr;
    }
    return e;
  }
  ~PhaseTimer() {
    if (!c->timing || !a) return;
    hipEvent_t b = take();
    if (!b || hipEventRecord(b, s) != hipSuccess) {
      c->spare.push_back(a);
      if (b) c->spare.push_back(b);
      return;
    }
    c->events.push_back({phase, a, b});
  }
};

void collect_timing(pic_ctx *c) {
  for (auto &ev : c->events) {
    float ms = 0.f;
    if (hipEventSynchronize(ev.b) == hipSuccess && hipEventElapsedTime(&ms, ev.a, ev.b) == hipSuccess) {
      c->ms[ev.phase] += ms;
      c->launches[ev.phase] += 1;
    }
    c->spare.push_back(ev.a);
    c->spare.push_back(ev.b);
  }
  c->events.clear();
}

// B half step, E step (with the Mur faces when open_x), B half step: in one
// pass into the second field set, which then becomes the current one, when
// the caller gave one and the box suits; else in place in three passes.
hipError_t yee_step(pic_ctx *c, pic_fields &f, hipStream_t s) {
  if (pic::yee_fused_ok(*c, f)) {
    hipError_t e = pic::launch_yee_fused(*c, f, s);
    if (e != hipSuccess) return e;
    for (int d = 0; d < 3; ++d) {
      std::swap(f.E[d], f.E_alt[d]);
      std::swap(f.B[d], f.B_alt[d]);
    }
    return hipSuccess;
  }
  hipError_t e = pic::launch_yee_b(*c, f, 0.5, s);
  if (e == hipSuccess && c->p.open_x) e = pic::launch_mur(*c, f, true, s);
  if (e == hipSuccess) e = pic::launch_yee_e(*c, f, s);
  if (e == hipSuccess && c->p.open_x) e = pic::launch_mur(*c, f, false, s);
  if (e == hipSuccess) e = pic::launch_yee_b(*c, f, 0.5, s);
  return e;
}

pic_status check_ws(pic_ctx *c) {
  if (!c->wsptr) return fail(c, PIC_ENOMEM, "no workspace set (pic_set_workspace)");
  return PIC_OK;
}

}  // namespace

extern "C" {

const char *pic_status_string(pic_status s) {
  switch (s) {
    case PIC_OK: return "ok";
    case PIC_EINVAL: return "invalid argument";
    case PIC_ECFL: return "time step at or above the Yee stability limit";
    case PIC_EHIP: return "HIP runtime error";
    case PIC_ENOMEM: return "workspace missing or too small";
    case PIC_ECROSS: return "a particle moved a full cell or more in one step, or became non-finite";
    case PIC_ENAN: return "non-finite diagnostic";
    case PIC_ESTATE: return "call out of order";
  }
  return "unknown status";
}

pic_status pic_init(const pic_params *p, pic_ctx **out) {
  if (!p || !out) return PIC_EINVAL;
  *out = nullptr;
  if (p->dims != 2 && p->dims != 3) return PIC_EINVAL;
  if (p->shape_order != 1 && p->shape_order != 2) return PIC_EINVAL;
  if (p->precision != PIC_FP32 && p->precision != PIC_FP64) return PIC_EINVAL;
  if (p->max_particles < 0 || p->max_particles > (int64_t(1) << 31) - 1) return PIC_EINVAL;
  if (p->sort_every < 0 || p->slack < 0 || p->slack > 4) return PIC_EINVAL;
  if (p->current_accum != PIC_ACC_AUTO && p->current_accum != PIC_ACC_FP32 && p->current_accum != PIC_ACC_FP64 &&
      p->current_accum != PIC_ACC_FIX64)
    return PIC_EINVAL;
  if (p->precision == PIC_FP64 && (p->current_accum == PIC_ACC_FP32 || p->current_accum == PIC_ACC_FIX64))
    return PIC_EINVAL;
  if (p->open_x != 0 && p->open_x != 1) return PIC_EINVAL;
  if (p->sort_levels != 0 && (p->sort_levels < 2 || p->sort_levels > pic::kMaxSortLevels)) return PIC_EINVAL;
  if (p->open_x && (p->absorb < 2 * p->shape_order + 2 || p->n[0] < 2 * static_cast<int64_t>(p->absorb) + 2))
    return PIC_EINVAL;
  for (int d = 0; d < 3; ++d) {
    const bool used = d < p->dims;
    if (used) {
      if (p->n[d] < 4 || !(p->dx[d] > 0.0) || !std::isfinite(p->dx[d])) return PIC_EINVAL;
      if (p->tile[d] < 1 || p->n[d] % p->tile[d] != 0) return PIC_EINVAL;
      if (p->tile[d] + p->slack > 31) return PIC_EINVAL;  // local cells are packed in 6 bits
    } else {
      if (p->n[d] != 1 || p->tile[d] != 1) return PIC_EINVAL;
    }
  }
  int64_t ncells = 1;
  int bits = 0;
  for (int d = 0; d < p->dims; ++d) {
    ncells *= p->n[d];
    bits += ceil_log2(p->n[d]);
  }
  if (bits > 31) return PIC_EINVAL;
  if (!(p->dt > 0.0) || !std::isfinite(p->dt)) return PIC_EINVAL;
  double s = 0.0;
  for (int d = 0; d < p->dims; ++d) s += 1.0 / (p->dx[d] * p->dx[d]);
  if (p->dt >= 1.0 / std::sqrt(s)) return PIC_ECFL;

  pic_ctx *c = new (std::nothrow) pic_ctx();
  if (!c) return PIC_ENOMEM;
  c->p = *p;
  c->ncells = ncells;
  c->ntiles = 1;
  for (int d = 0; d < 3; ++d) {
    c->n[d] = p->n[d];
    c->bits[d] = d < p->dims ? ceil_log2(p->n[d]) : 0;
    c->ntile[d] = p->n[d] / p->tile[d];
    c->ntiles *= c->ntile[d];
  }
  c->elem = p->precision == PIC_FP64 ? 8 : 4;
  c->levels = p->sort_levels ? p->sort_levels : 32;
  c->acc64 = p->current_accum != PIC_ACC_FP32;
  c->accfix = p->precision == PIC_FP32 && (p->current_accum == PIC_ACC_FIX64 || p->current_accum == PIC_ACC_AUTO);
  const size_t jelem = c->acc64 ? 8 : 4;
  // LDS tile geometry: the gather reaches [c-1, c+M] around the particle's
  // cell, the Esirkepov window [c-M, c+M+1]; slack widens both on each side.
  const int M = p->shape_order;
  const int f_lo = 1, f_hi = M, j_lo = M, j_hi = M + 1;
  for (int d = 0; d < 3; ++d) {
    if (d < p->dims) {
      c->gf_lo[d] = f_lo + p->slack;
      c->rf[d] = p->tile[d] + f_lo + f_hi + 2 * p->slack;
      c->gj_lo[d] = j_lo + p->slack;
      c->rj[d] = p->tile[d] + j_lo + j_hi + 2 * p->slack;
    } else {
      c->gf_lo[d] = c->gj_lo[d] = 0;
      c->rf[d] = c->rj[d] = 1;
    }
  }
  c->jxy = pic::current_plane_stride(c->rj[0], c->rj[1], p->dims);
  const size_t jbox = 3 * static_cast<size_t>(c->jxy) * c->rj[2] * jelem;
  // The field box's rows are padded to an even length where it fits: the
  // gather then reads every run of three values as an aligned pair and a
  // single (the fixed-shape kernels assume it for their tile shapes).
  if ((c->rf[0] & 1) &&
      6 * static_cast<size_t>(c->rf[0] + 1) * c->rf[1] * c->rf[2] * c->elem + jbox + pic::cross_list_bytes(c->elem, 0) <=
          pic::kLdsLimit)
    c->rf[0] += 1;
  const size_t boxes = 6 * static_cast<size_t>(c->rf[0]) * c->rf[1] * c->rf[2] * c->elem + jbox;
  if (boxes + pic::cross_list_bytes(c->elem, 0) > pic::kLdsLimit) {
    delete c;
    return PIC_EINVAL;
  }
  // the wide-window list takes what is left, in multiples of 64 entries;
  // where the boxes are small (2D 8x8 tiles of a dense foil) it is twice as
  // long, for the many hot electrons such a tile holds
  const size_t entry = 8 * c->elem + 4;
  int cap = c->elem == 4 ? pic::kCrossCapF32 : pic::kCrossCapF64;
  if (boxes < 16 * 1024) cap *= 2;
  const size_t room = (pic::kLdsLimit - boxes - pic::cross_list_bytes(c->elem, 0)) / entry;
  if (static_cast<size_t>(cap) > room) cap = static_cast<int>(room / 64 * 64);
  c->cross_cap = cap;
  c->lds_bytes = boxes + pic::cross_list_bytes(c->elem, cap);
  // workspace layout
  pic::Workspace &w = c->ws;
  size_t off = 0;
  const size_t mp = static_cast<size_t>(p->max_particles);
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off = align256(off + bytes);
    return at;
  };
  w.flags = take(64 * sizeof(int32_t));
  w.save_cell = take(mp * 4);
  w.save_off = take(3 * mp * c->elem);
  w.sort_key = take(mp * 4);
  w.sort_rank = take(mp * 4);
  w.sort_src = take(mp * 4);
  w.stray_count = take(32 * 4);
  w.stray_list = take(mp * 4);
  // sort buckets: (tile, level) pairs plus one for particles removed at open faces
  const int64_t nbuckets = c->ntiles * c->levels + 1;
  if (pic::sort_scan_blocks(nbuckets) > pic::sort_scan_capacity() || nbuckets >= (int64_t(1) << 31) - 1) {
    delete c;
    return PIC_EINVAL;
  }
  w.stay_count = take(static_cast<size_t>(nbuckets) * 4);
  w.arrive_count = take(static_cast<size_t>(nbuckets) * 4);
  // bucket starts of the last sort, one slot per species (the next sort's hints)
  w.bucket_start = take(static_cast<size_t>(pic::kMaxSpecies) * (nbuckets + 1) * 4);
  w.scan_partials = take(static_cast<size_t>(pic::sort_scan_blocks(nbuckets)) * 8);
  w.live_tiles = take(static_cast<size_t>(pic::kMaxSpecies) * (c->ntiles + 1) * 4);
  w.dense_tiles = take(static_cast<size_t>(pic::kMaxSpecies) * (c->ntiles + 1) * 4);
  w.sparse_tiles = take(static_cast<size_t>(pic::kMaxSpecies) * (c->ntiles + 1) * 4);
  w.wmax_tiles = take(static_cast<size_t>(pic::kMaxSpecies) * c->ntiles * 4);
  w.partials = take(static_cast<size_t>(pic::kDiagSlots) * pic::kMaxSpecies * pic::kDiagBlocks * 8);
  w.result = take(16 * 8);
  w.rho = take(static_cast<size_t>(ncells) * 8);
  w.rho_prev = take(static_cast<size_t>(ncells) * 8);
  w.gauss_prev = take(static_cast<size_t>(ncells) * 8);
  w.mur_old = take(p->open_x ? static_cast<size_t>(8) * p->n[1] * p->n[2] * c->elem : 0);
  w.select_base = take(static_cast<size_t>((p->max_particles + pic::kSelectChunk - 1) / pic::kSelectChunk + 1) * 8);
  w.total = off;
  *out = c;
  return PIC_OK;
}

void pic_destroy(pic_ctx *c) {
  if (!c) return;
  for (auto &ev : c->events) {
    hipEventDestroy(ev.a);
    hipEventDestroy(ev.b);
  }
  for (auto e : c->spare) hipEventDestroy(e);
  for (auto e : c->live_event)
    if (e) hipEventDestroy(e);
  if (c->live_host) hipHostFree(c->live_host);
  delete c;
}

size_t pic_workspace_bytes(const pic_ctx *c) { return c ? c->ws.total : 0; }
int64_t pic_num_tiles(const pic_ctx *c) { return c ? c->ntiles : 0; }
size_t pic_tile_lds_bytes(const pic_ctx *c) { return c ? c->lds_bytes : 0; }
int64_t pic_step_count(const pic_ctx *c) { return c ? c->step : 0; }

void pic_cell_bits(const pic_ctx *c, int32_t bits[3]) {
  if (!c || !bits) return;
  for (int d = 0; d < 3; ++d) bits[d] = c->bits[d];
}

const char *pic_last_error(const pic_ctx *c) { return c ? c->err.c_str() : "null context"; }

pic_status pic_set_workspace(pic_ctx *c, void *ptr, size_t bytes) {
  if (!c) return PIC_EINVAL;
  if (!ptr) return fail(c, PIC_EINVAL, "workspace pointer is null");
  if ((reinterpret_cast<uintptr_t>(ptr) & 255) != 0) return fail(c, PIC_EINVAL, "workspace not 256-byte aligned");
  if (bytes < c->ws.total) return fail(c, PIC_ENOMEM, "workspace smaller than pic_workspace_bytes()");
  c->wsptr = static_cast<char *>(ptr);
  c->wsbytes = bytes;
  c->diag_step = -1;
  c->pending_cell = nullptr;
  // the tile lists, bucket starts and weight bounds of earlier sorts lived in
  // the previous workspace
  c->sorted_runs.clear();
  for (int i = 0; i < pic::kMaxSpecies; ++i) c->wmax_known[i] = false;
  c->stray_clean = false;  // the next fused launch clears its counters itself
  hipError_t e = hipMemset(c->wsptr + c->ws.flags, 0, 64 * sizeof(int32_t));
  if (e != hipSuccess) return hip_fail(c, e, "clearing workspace flags");
  return PIC_OK;
}

pic_status pic_gather_push(pic_ctx *c, pic_species *sp, const pic_fields *f, void *stream) {
  if (!c) return PIC_EINVAL;
  if (pic_status s = check_ws(c)) return s;
  if (!species_ok(c, sp, false)) return fail(c, PIC_EINVAL, "bad species");
  if (!fields_ok(f)) return fail(c, PIC_EINVAL, "bad fields");
  hipError_t e = pic::launch_gather_push(*c, *sp, *f, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(c, e, "gather_push");
  c->pending_cell = sp->cell;
  c->pending_np = sp->np;
  return PIC_OK;
}

pic_status pic_deposit(pic_ctx *c, const pic_species *sp, pic_fields *f, void *stream) {
  if (!c) return PIC_EINVAL;
  if (pic_status s = check_ws(c)) return s;
  if (!species_ok(c, sp, false)) return fail(c, PIC_EINVAL, "bad species");
  if (!fields_ok(f)) return fail(c, PIC_EINVAL, "bad fields");
  if (c->pending_cell != sp->cell || c->pending_np != sp->np)
    return fail(c, PIC_ESTATE, "pic_deposit must follow pic_gather_push of the same species");
  hipError_t e = pic::launch_deposit(*c, *sp, *f, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(c, e, "deposit");
  c->pending_cell = nullptr;
  return PIC_OK;
}

pic_status pic_zero_current(pic_ctx *c, pic_fields *f, void *stream) {
  if (!c) return PIC_EINVAL;
  if (!fields_ok(f)) return fail(c, PIC_EINVAL, "bad fields");
  hipError_t e = pic::launch_fill_zero_n(f->J, 3, c->ncells, c->elem, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(c, e, "zero_current");
  return PIC_OK;
}

pic_status pic_yee_step(pic_ctx *c, pic_fields *f, void *stream) {
  if (!c) return PIC_EINVAL;
  if (!fields_ok(f)) return fail(c, PIC_EINVAL, "bad fields");
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = yee_step(c, *f, s);
  if (e != hipSuccess) return hip_fail(c, e, "yee_step");
  c->step += 1;
  return PIC_OK;
}

pic_status pic_set_laser(pic_ctx *c, const pic_laser *L) {
  if (!c) return PIC_EINVAL;
  if (!L) {
    c->has_laser = false;
    return PIC_OK;
  }
  if (!c->p.open_x) return fail(c, PIC_EINVAL, "a laser needs open x faces");
  if (L->plane < 1 || L->plane > c->p.n[0] - 2) return fail(c, PIC_EINVAL, "laser plane outside (0, n0-1)");
  if (L->pol != 1 && !(L->pol == 2 && c->p.dims == 3)) return fail(c, PIC_EINVAL, "laser polarisation");
  if (!(L->e0 > 0) || !(L->w0 > 0) || !(L->tau > 0) || !(L->omega > 0) || !std::isfinite(L->t0) ||
      !std::isfinite(L->yc) || !std::isfinite(L->zc))
    return fail(c, PIC_EINVAL, "laser parameters");
  // lattice wavenumber of omega along x: sin(k dx/2) = (dx/dt) sin(omega dt/2)
  const double dx = c->p.dx[0], dt = c->p.dt;
  const double s = std::sin(0.5 * L->omega * dt);
  const double arg = dx / dt * s;
  if (!(arg < 1.0) || !(s > 0.0)) return fail(c, PIC_EINVAL, "laser frequency above the lattice cut-off");
  const double k = 2.0 * std::asin(arg) / dx;
  c->laser = *L;
  c->laser_j0 = -L->e0 * dt * std::sin(k * dx) / (dx * dx * s);
  c->has_laser = true;
  return PIC_OK;
}

pic_status pic_laser_current(pic_ctx *c, pic_fields *f, double t, void *stream) {
  if (!c) return PIC_EINVAL;
  if (!fields_ok(f)) return fail(c, PIC_EINVAL, "bad fields");
  if (!c->has_laser) return fail(c, PIC_ESTATE, "no laser registered (pic_set_laser)");
  hipError_t e = pic::launch_laser(*c, *f, t, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(c, e, "laser_current");
  return PIC_OK;
}

pic_status pic_sort(pic_ctx *c, pic_species *sp, void *stream) {
  if (!c) return PIC_EINVAL;
  if (pic_status s = check_ws(c)) return s;
  if (!species_ok(c, sp, true) || !sp->tile_start) return fail(c, PIC_EINVAL, "bad species (sort buffers)");
  hipError_t e = pic::launch_sort(*c, *sp, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(c, e, "sort");
  c->pending_cell = nullptr;
  return PIC_OK;
}

pic_status pic_step(pic_ctx *c, pic_species *sp, int32_t nspecies, pic_fields *f, int32_t nsteps, void *stream) {
  if (!c) return PIC_EINVAL;
  if (pic_status s = check_ws(c)) return s;
  if (nspecies < 0 || (nspecies > 0 && !sp) || nsteps < 0) return fail(c, PIC_EINVAL, "bad counts");
  if (!fields_ok(f)) return fail(c, PIC_EINVAL, "bad fields");
  for (int i = 0; i < nspecies; ++i)
    if (!species_ok(c, &sp[i], true)) return fail(c, PIC_EINVAL, "bad species (pic_step needs sort buffers)");
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = hipSuccess;
  for (int it = 0; it < nsteps; ++it) {
    const bool cadence = c->p.sort_every > 0 && (c->step % c->p.sort_every) == 0;
    {
      PhaseTimer t(c, s, pic::kPhaseZero);
      e = pic::launch_fill_zero_n(f->J, 3, c->ncells, c->elem, s);
      if (e == hipSuccess && c->has_laser) e = pic::launch_laser(*c, *f, (c->step + 0.5) * c->p.dt, s);
      if (e != hipSuccess) return hip_fail(c, e, "zero_current");
    }
    // Species by species.  In 3D a sort ranks the particles and leaves its
    // copy into the second array set to the push that follows it, which reads
    // each particle through the sort's slots and writes it in sorted order.
    // The 2D push has too little work per particle to hide the extra read, so
    // there the sort copies.
    const bool fold = c->p.dims == 3;
    for (int i = 0; i < nspecies; ++i) {
      if (sp[i].np == 0) continue;
      const int32_t *src = nullptr;
      const int64_t np_src = sp[i].np;  // a sort with open faces drops removed particles from np
      if (cadence || !sp[i].sorted) {
        PhaseTimer t(c, s, pic::kPhaseSort);
        e = pic::launch_sort(*c, sp[i], s, fold ? &src : nullptr, false);
        if (e != hipSuccess) return hip_fail(c, e, "sort");
      }
      if (sp[i].np == 0) continue;
      PhaseTimer t(c, s, pic::kPhasePush);
      e = pic::launch_push_deposit_tiled(*c, sp[i], *f, s, src, np_src);
      if (e != hipSuccess) {
        if (src) sp[i].sorted = 0;  // the sort's copy may not have happened: its order is not in the arrays
        return hip_fail(c, e, "push_deposit");
      }
    }
    {
      PhaseTimer t(c, s, pic::kPhaseYee);
      e = yee_step(c, *f, s);
      if (e != hipSuccess) return hip_fail(c, e, "yee");
    }
    c->step += 1;
  }
  c->pending_cell = nullptr;
  return PIC_OK;
}

pic_status pic_diagnostics(pic_ctx *c, const pic_species *sp, int32_t nspecies, const pic_fields *f, double *out,
                           void *stream) {
  if (!c) return PIC_EINVAL;
  if (pic_status s = check_ws(c)) return s;
  if (!out || nspecies < 0 || nspecies > pic::kMaxSpecies || (nspecies > 0 && !sp))
    return fail(c, PIC_EINVAL, "bad diagnostics arguments");
  if (!fields_ok(f)) return fail(c, PIC_EINVAL, "bad fields");
  for (int i = 0; i < nspecies; ++i)
    if (!species_ok(c, &sp[i], false)) return fail(c, PIC_EINVAL, "bad species");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const bool have_prev = c->diag_step >= 0;
  const bool have_cont = have_prev && c->diag_step + 1 == c->step;
  hipError_t e = pic::launch_diagnostics(*c, sp, nspecies, *f, have_prev, have_cont, s);
  if (e != hipSuccess) return hip_fail(c, e, "diagnostics");
  double res[16];
  e = hipMemcpyAsync(res, c->wsptr + c->ws.result, sizeof(double) * PIC_NDIAG, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(c, e, "diagnostics readback");
  if (!have_prev) res[6] = NAN;
  if (!have_cont) res[7] = NAN;
  for (int i = 0; i < PIC_NDIAG; ++i) out[i] = res[i];
  c->diag_step = c->step;
  for (int i = 0; i < 4; ++i)
    if (!std::isfinite(res[i])) return fail(c, PIC_ENAN, "non-finite energy or charge");
  return pic_check(c, stream);
}

pic_status pic_charge_density(pic_ctx *c, const pic_species *sp, int32_t nspecies, const pic_fields *f, double *rho,
                              double *gauss, void *stream) {
  if (!c) return PIC_EINVAL;
  if (!rho || nspecies < 0 || (nspecies > 0 && !sp)) return fail(c, PIC_EINVAL, "bad charge density arguments");
  if (gauss && !fields_ok(f)) return fail(c, PIC_EINVAL, "div E - rho needs the fields");
  for (int i = 0; i < nspecies; ++i)
    if (!species_ok(c, &sp[i], false)) return fail(c, PIC_EINVAL, "bad species");
  hipError_t e = pic::launch_charge_density(*c, sp, nspecies, f, rho, gauss, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(c, e, "charge_density");
  return PIC_OK;
}

pic_status pic_diagnostics_noalloc(pic_ctx *c, const pic_species *sp, int32_t nspecies, const pic_fields *f,
                                   double *out, void *stream) {
  if (!c) return PIC_EINVAL;
  if (!out || nspecies < 0 || nspecies > pic::kMaxSpecies || (nspecies > 0 && !sp))
    return fail(c, PIC_EINVAL, "bad diagnostics arguments");
  if (c->ncells > pic::kScratchCells)
    return fail(c, PIC_EINVAL, "grid larger than PIC_NOALLOC_MAX_CELLS nodes: use pic_diagnostics with a workspace");
  if (!fields_ok(f)) return fail(c, PIC_EINVAL, "bad fields");
  for (int i = 0; i < nspecies; ++i)
    if (!species_ok(c, &sp[i], false)) return fail(c, PIC_EINVAL, "bad species");
  hipStream_t s = static_cast<hipStream_t>(stream);
  double *scratch = nullptr;
  hipError_t e = pic::scratch_address(&scratch);
  if (e != hipSuccess) return hip_fail(c, e, "diagnostics_noalloc: scratch address");
  e = pic::launch_diagnostics_noalloc(*c, sp, nspecies, *f, scratch, s);
  if (e != hipSuccess) return hip_fail(c, e, "diagnostics_noalloc");
  double res[PIC_NDIAG];
  e = hipMemcpyAsync(res, scratch + pic::scratch_result_offset(), sizeof(double) * PIC_NDIAG, hipMemcpyDeviceToHost,
                     s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(c, e, "diagnostics_noalloc readback");
  res[6] = NAN;
  res[7] = NAN;
  for (int i = 0; i < PIC_NDIAG; ++i) out[i] = res[i];
  for (int i = 0; i < 4; ++i)
    if (!std::isfinite(res[i])) return fail(c, PIC_ENAN, "non-finite energy or charge");
  return PIC_OK;
}

namespace {
// A box inside the grid (points or cells): 0 <= lo <= hi <= n, and stride >= 1
// where the stride is used.
bool box_ok(const pic_ctx *c, const pic_box *b, bool strided) {
  if (!b) return false;
  for (int d = 0; d < 3; ++d)
    if (b->lo[d] < 0 || b->hi[d] < b->lo[d] || b->hi[d] > c->n[d] || (strided && b->stride[d] < 1)) return false;
  return true;
}
}  // namespace

pic_status pic_extract_grid(pic_ctx *c, const void *const *grids, int32_t ngrids, int32_t elem_bytes,
                            const pic_box *box, void *dst, void *stream) {
  if (!c) return PIC_EINVAL;
  if (!box_ok(c, box, true)) return fail(c, PIC_EINVAL, "bad box: need 0 <= lo <= hi <= n and stride >= 1");
  if (ngrids < 1 || ngrids > pic::kMaxExtractGrids || !grids)
    return fail(c, PIC_EINVAL, "between 1 and PIC_MAX_EXTRACT_GRIDS grids");
  if (elem_bytes != 4 && elem_bytes != 8) return fail(c, PIC_EINVAL, "elem_bytes must be 4 or 8");
  for (int g = 0; g < ngrids; ++g)
    if (!grids[g]) return fail(c, PIC_EINVAL, "null grid");
  const int64_t pts = pic::box_points(*box, 0) * pic::box_points(*box, 1) * pic::box_points(*box, 2);
  if (pts > 0 && !dst) return fail(c, PIC_EINVAL, "null dst");
  hipError_t e = pic::launch_extract_grid(*c, grids, ngrids, elem_bytes, *box, dst, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(c, e, "extract_grid");
  return PIC_OK;
}

pic_status pic_extract_particles(pic_ctx *c, const pic_species *sp, const pic_box *cells, int64_t every, void *dst,
                                 int64_t capacity, int64_t *count, void *stream) {
  if (!c) return PIC_EINVAL;
  if (pic_status s = check_ws(c)) return s;
  if (!box_ok(c, cells, false)) return fail(c, PIC_EINVAL, "bad cell box: need 0 <= lo <= hi <= n");
  if (every < 1 || capacity < 0 || !count || (capacity > 0 && !dst))
    return fail(c, PIC_EINVAL, "bad particle output arguments");
  if (!species_ok(c, sp, false)) return fail(c, PIC_EINVAL, "bad species");
  hipError_t e = pic::launch_extract_particles(*c, *sp, *cells, every, dst, capacity, count,
                                               static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(c, e, "extract_particles");
  return PIC_OK;
}

pic_status pic_energy_adjoint(pic_ctx *c, const pic_fields *f, pic_fields *lam, double scale, void *stream) {
  if (!c) return PIC_EINVAL;
  if (c->p.open_x) return fail(c, PIC_EINVAL, "the adjoint covers periodic boxes only");
  if (!fields_ok(f) || !fields_ok(lam)) return fail(c, PIC_EINVAL, "bad fields");
  double dV = 1.0;
  for (int d = 0; d < c->p.dims; ++d) dV *= c->p.dx[d];
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = pic::launch_scale_copy(*c, lam->E, f->E, scale * dV, s);
  if (e == hipSuccess) e = pic::launch_scale_copy(*c, lam->B, f->B, scale * dV, s);
  if (e != hipSuccess) return hip_fail(c, e, "energy_adjoint");
  return PIC_OK;
}

pic_status pic_yee_adjoint(pic_ctx *c, pic_fields *lam, void *stream) {
  if (!c) return PIC_EINVAL;
  if (c->p.open_x) return fail(c, PIC_EINVAL, "the adjoint covers periodic boxes only");
  if (!fields_ok(lam)) return fail(c, PIC_EINVAL, "bad fields");
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = pic::launch_yee_e(*c, *lam, s, -0.5, false);  // lamE -= dt/2 C_B lamB
  if (e == hipSuccess) e = pic::launch_scale_copy(*c, lam->J, lam->E, -c->p.dt, s);  // lamJ = -dt lamE
  if (e == hipSuccess) e = pic::launch_yee_b(*c, *lam, -1.0, s);  // lamB += dt C_E lamE
  if (e == hipSuccess) e = pic::launch_yee_e(*c, *lam, s, -0.5, false);  // lamE -= dt/2 C_B lamB
  if (e != hipSuccess) return hip_fail(c, e, "yee_adjoint");
  return PIC_OK;
}

pic_status pic_particle_adjoint(pic_ctx *c, const pic_species *sp, const pic_fields *f, pic_fields *lam,
                                pic_species_adjoint *lsp, void *stream) {
  if (!c) return PIC_EINVAL;
  if (c->p.open_x) return fail(c, PIC_EINVAL, "the adjoint covers periodic boxes only");
  if (pic_status s = check_ws(c)) return s;
  if (!species_ok(c, sp, false)) return fail(c, PIC_EINVAL, "bad species");
  if (!fields_ok(f) || !fields_ok(lam)) return fail(c, PIC_EINVAL, "bad fields");
  if (!lsp) return fail(c, PIC_EINVAL, "bad adjoint species");
  if (sp->np > 0) {
    for (int d = 0; d < 3; ++d)
      if (!lsp->u[d] || (d < c->p.dims && !lsp->x[d])) return fail(c, PIC_EINVAL, "bad adjoint species");
  }
  hipError_t e = pic::launch_particle_adjoint(*c, *sp, *f, *lam, *lsp, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(c, e, "particle_adjoint");
  return PIC_OK;
}

pic_status pic_check(pic_ctx *c, void *stream) {
  if (!c) return PIC_EINVAL;
  if (pic_status s = check_ws(c)) return s;
  hipStream_t s = static_cast<hipStream_t>(stream);
  int32_t flags = 0;
  hipError_t e = hipMemcpyAsync(&flags, c->wsptr + c->ws.flags, sizeof(int32_t), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(c, e, "check");
  if (flags != 0) {
    const int32_t zero = 0;
    e = hipMemcpyAsync(c->wsptr + c->ws.flags, &zero, sizeof(int32_t), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(c, e, "check reset");
    if (flags & pic::kFlagCross) return fail(c, PIC_ECROSS, pic_status_string(PIC_ECROSS));
    if (flags & pic::kFlagSort)
      return fail(c, PIC_ESTATE, "sort: the species' tile_start runs did not match its particles "
                                 "(edited without clearing sorted?)");
  }
  return PIC_OK;
}

pic_status pic_straggler_count(pic_ctx *c, int64_t *count, void *stream) {
  if (!c || !count) return PIC_EINVAL;
  if (pic_status s = check_ws(c)) return s;
  hipStream_t s = static_cast<hipStream_t>(stream);
  int32_t n = 0;
  // the last fused launch's bank
  const size_t at = c->ws.stray_count + static_cast<size_t>(c->stray_last) * 16 * sizeof(int32_t);
  hipError_t e = hipMemcpyAsync(&n, c->wsptr + at, sizeof(int32_t), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(c, e, "straggler count");
  *count = n;
  return PIC_OK;
}

pic_status pic_set_timing(pic_ctx *c, int32_t on) {
  if (!c) return PIC_EINVAL;
  c->timing = on != 0;
  return PIC_OK;
}

pic_status pic_get_timing(pic_ctx *c, double *ms, int64_t *launches, int32_t nphase) {
  if (!c || !ms || !launches || nphase < 1) return PIC_EINVAL;
  collect_timing(c);
  for (int i = 0; i < nphase && i < PIC_NPHASE; ++i) {
    ms[i] = c->ms[i];
    launches[i] = c->launches[i];
    c->ms[i] = 0.0;
    c->launches[i] = 0;
  }
  return PIC_OK;
}

}  // extern "C"
