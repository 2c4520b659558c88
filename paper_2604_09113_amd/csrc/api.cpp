// C ABI of the lbddc library: validation, state machine, device memory and the
// orchestration of the kernels of each phase.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>

#include "internal.h"

using namespace lbddc;

namespace lbddc {

bool dalloc(Ctx* c, void** p, size_t bytes) {
  *p = nullptr;
  if (bytes == 0) bytes = 8;
  if (hipMalloc(p, bytes) != hipSuccess) {
    *p = nullptr;
    hipGetLastError();
    char buf[128];
    snprintf(buf, sizeof buf, "device allocation of %zu bytes failed", bytes);
    c->err = buf;
    return false;
  }
  c->allocs.push_back(*p);
  c->dev_bytes += bytes;
  return true;
}

}  // namespace lbddc

// Free the device and pinned memory of a problem (not the ROMs, events,
// stream or the context-wide pinned buffers).
static void release_problem(Ctx* c) {
  if (c->h_red) hipHostFree(c->h_red);
  c->h_red = nullptr;
  for (void* p : c->allocs) hipFree(p);
  c->allocs.clear();
  c->dev_bytes = 0;
}

// A context holding only what outlives a problem: device, streams, ROMs,
// events, timing mask and the context-wide pinned buffers.  The ROM table is
// shared (shallow copy): only one of the two contexts ever frees it.
static void copy_persistent(const Ctx* c, Ctx* n) {
  n->device = c->device;
  n->stream = c->stream;
  n->own_stream = c->own_stream;
  n->roms = c->roms;
  for (int i = 0; i < Ctx::kNumEv; ++i) n->ev[i] = c->ev[i];
  n->side = c->side;
  n->side_fork = c->side_fork;
  n->side_join = c->side_join;
  for (int i = 0; i < Ctx::kRing; ++i)
    for (int k = 0; k < Ctx::kRingEv; ++k) n->pev[i][k] = c->pev[i][k];
  n->timing = c->timing;
  n->h_flags = c->h_flags;
  n->h_scal = c->h_scal;
}

static lbddc_status fail(Ctx* c, lbddc_status s, const char* msg) {
  c->err = msg;
  return s;
}

static lbddc_status hipfail(Ctx* c, hipError_t e, const char* where) {
  char buf[256];
  snprintf(buf, sizeof buf, "%s: %s", where, hipGetErrorString(e));
  c->err = buf;
  return LBDDC_E_HIP;
}

#define HIPCHK(expr, where)                  \
  do {                                       \
    hipError_t _e = (expr);                  \
    if (_e != hipSuccess) return hipfail(c, _e, where); \
  } while (0)

static lbddc_status check_flags(Ctx* c, const char* phase) {
  HIPCHK(hipMemcpyAsync(c->h_flags, c->d_flags, 8 * sizeof(int), hipMemcpyDeviceToHost, c->stream), phase);
  HIPCHK(hipStreamSynchronize(c->stream), phase);
  int f = c->h_flags[0];
  if (!f) return LBDDC_OK;
  char buf[256];
  lbddc_status s = LBDDC_E_NUMERIC;
  const char* what = "non-positive pivot in a local factorization";
  if (f & 1) { s = LBDDC_E_DEGENERATE_MAP; what = "det J <= 0 in a cell map"; }
  else if (f & 4) { s = LBDDC_E_ROM; what = "a cell's family has no ROM"; }
  else if (f & 2) { s = LBDDC_E_PARAM_RANGE; what = "a thickness parameter lies outside its ROM box"; }
  else if (f & 8) what = "non-positive pivot in K_II (local Schur complement)";
  else if (f & 16) what = "non-positive pivot in the constrained local factorization";
  else if (f & 32) what = "non-positive pivot in the coarse factorization";
  else if (f & 128) what = "root search along a trimmed cell edge ran out of room";
  snprintf(buf, sizeof buf, "%s: %s (flags 0x%x)", phase, what, f);
  c->err = buf;
  int zero[8] = {0};
  hipMemcpy(c->d_flags, zero, sizeof zero, hipMemcpyHostToDevice);
  return s;
}

extern "C" {

int lbddc_version(void) { return 2; }

lbddc_status lbddc_create(int device, void* stream, lbddc_ctx** out) {
  if (!out) return LBDDC_E_ARG;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return LBDDC_E_ARG;
  if (hipSetDevice(device) != hipSuccess) return LBDDC_E_HIP;
  // the device address of the static scratch of lbddc_assemble_fp32_noalloc,
  // taken once per device with that device current
  if (noalloc_scratch_init(device) != hipSuccess) return LBDDC_E_HIP;
  lbddc_ctx* x = new (std::nothrow) lbddc_ctx();
  if (!x) return LBDDC_E_NOMEM;
  Ctx* c = &x->c;
  c->device = device;
  if (stream) {
    c->stream = (hipStream_t)stream;
  } else {
    if (hipStreamCreate(&c->stream) != hipSuccess) { delete x; return LBDDC_E_HIP; }
    c->own_stream = true;
  }
  for (int i = 0; i < Ctx::kNumEv; ++i)
    if (hipEventCreate(&c->ev[i]) != hipSuccess) { delete x; return LBDDC_E_HIP; }
  if (hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&c->side_fork, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&c->side_join, hipEventDisableTiming) != hipSuccess) {
    delete x;
    return LBDDC_E_HIP;
  }
  for (int i = 0; i < Ctx::kRing; ++i)
    for (int k = 0; k < Ctx::kRingEv; ++k)
      if (hipEventCreate(&c->pev[i][k]) != hipSuccess) { delete x; return LBDDC_E_HIP; }
  if (hipHostMalloc((void**)&c->h_flags, 128 * sizeof(int)) != hipSuccess ||
      hipHostMalloc((void**)&c->h_scal, 32 * sizeof(double)) != hipSuccess) {
    delete x;
    return LBDDC_E_NOMEM;
  }
  *out = x;
  return LBDDC_OK;
}

void lbddc_destroy(lbddc_ctx* x) {
  if (!x) return;
  Ctx* c = &x->c;
  hipSetDevice(c->device);
  hipStreamSynchronize(c->stream);
  for (void* p : c->allocs) hipFree(p);
  for (auto& kv : c->roms) {
    for (auto p : kv.second.ut64) hipFree(p);
    for (auto p : kv.second.ut32) hipFree(p);
    for (auto p : kv.second.ucol64) hipFree(p);
    if (kv.second.coeff) hipFree(kv.second.coeff);
  }
  for (int i = 0; i < Ctx::kNumEv; ++i)
    if (c->ev[i]) hipEventDestroy(c->ev[i]);
  for (int i = 0; i < Ctx::kRing; ++i)
    for (int k = 0; k < Ctx::kRingEv; ++k)
      if (c->pev[i][k]) hipEventDestroy(c->pev[i][k]);
  if (c->h_flags) hipHostFree(c->h_flags);
  if (c->h_scal) hipHostFree(c->h_scal);
  if (c->h_red) hipHostFree(c->h_red);
  if (c->side_fork) hipEventDestroy(c->side_fork);
  if (c->side_join) hipEventDestroy(c->side_join);
  if (c->side) hipStreamDestroy(c->side);
  if (c->own_stream) hipStreamDestroy(c->stream);
  delete x;
}

const char* lbddc_last_error(const lbddc_ctx* x) { return x ? x->c.err.c_str() : "null context"; }

// Tile the reduced basis for the contraction kernel: per 16-pair tile, per s,
// per k-chunk, the 64 MFMA A-operand values (row = lane % 16, k = lane / 16).
// FP64 MFMA 16x16x4 returns rows lane/16 + 4v, so the FP64 rows are permuted to
// hand each lane four consecutive pairs.
lbddc_status lbddc_load_rom(lbddc_ctx* x, const lbddc_rom_desc* d) {
  if (!x) return LBDDC_E_ARG;
  Ctx* c = &x->c;
  if (!d || !d->U || !d->coeff || !d->I_pi) return fail(c, LBDDC_E_ARG, "load_rom: null pointer");
  if (d->p < 2 || d->p > kMaxP || d->q < 1 || d->q > 3) return fail(c, LBDDC_E_UNSUPPORTED, "load_rom: p or q out of range");
  const int dim = d->dim == 0 ? 1 : d->dim;
  if (dim != 1 && dim != 4) return fail(c, LBDDC_E_UNSUPPORTED, "load_rom: dim must be 1 or 4");
  if (d->n_r < 1 || d->n_r > 43 || d->r < 1 || d->r > (dim == 1 ? 16 : 8) || d->n_k < 1 ||
      d->n_k > (dim == 1 ? 16 : 2))
    return fail(c, LBDDC_E_UNSUPPORTED, "load_rom: n_r, r or n_k out of range");
  int ncl = 1, nnode = 1;
  for (int i = 0; i < dim; ++i) { ncl *= d->n_k; nnode *= d->r + 1; }
  if (d->family < 0 || d->family >= 64) return fail(c, LBDDC_E_ARG, "load_rom: family id must be in [0, 64)");
  if (!(d->hi > d->lo) || !std::isfinite(d->lo) || !std::isfinite(d->hi)) return fail(c, LBDDC_E_ARG, "load_rom: bad box");
  hipSetDevice(c->device);
  const int p = d->p, q = d->q, nB = (p + 1) * (p + 1), nL = (q + 1) * (q + 1), ns = 4 * nL;
  const int nN = nB, npair = nN * (nN + 1) / 2, NPT = (npair + 15) / 16;
  const long long n_i = (long long)nB * nB * ns;
  const int KC = (d->n_r + 1 + 3) / 4;
  // permuted node order (interior nodes, then skeleton slots) -> natural index
  std::vector<int> perm;
  for (int b = 1; b < p; ++b)
    for (int a = 1; a < p; ++a) perm.push_back(a + (p + 1) * b);
  {
    int corners[4][2] = {{0, 0}, {p, 0}, {0, p}, {p, p}};
    for (auto& cc : corners) perm.push_back(cc[0] + (p + 1) * cc[1]);
    for (int b = 1; b < p; ++b) perm.push_back(0 + (p + 1) * b);
    for (int b = 1; b < p; ++b) perm.push_back(p + (p + 1) * b);
    for (int a = 1; a < p; ++a) perm.push_back(a);
    for (int a = 1; a < p; ++a) perm.push_back(a + (p + 1) * p);
  }
  std::vector<int> pn1(npair), pn2(npair);
  for (int n1 = 0, P = 0; n1 < nN; ++n1)
    for (int n2 = 0; n2 <= n1; ++n2, ++P) { pn1[P] = n1; pn2[P] = n2; }
  RomDev R;
  R.family = d->family; R.p = p; R.q = q; R.n_k = d->n_k; R.n_r = d->n_r; R.r = d->r;
  R.dim = dim; R.ncl = ncl;
  R.lo = d->lo; R.hi = d->hi; R.KC = KC;
  const size_t tile_n = (size_t)NPT * ns * KC * 64;
  const int RB = (4 * KC + 15) / 16;
  const size_t tile2_n = (size_t)NPT * ns * RB * 4 * 64;
  std::vector<double> h64(tile_n), h2(tile2_n);
  std::vector<float> h32(tile_n);
  for (int k = 0; k < ncl; ++k) {
    const double* U = d->U + (size_t)k * n_i * d->n_r;
    for (int pt = 0; pt < NPT; ++pt)
      for (int s = 0; s < ns; ++s)
        for (int kc = 0; kc < KC; ++kc)
          for (int lane = 0; lane < 64; ++lane) {
            const int row = lane & 15, r = 4 * kc + (lane >> 4);
            const int off64 = 4 * (row & 3) + (row >> 2);  // FP64 row permutation
            double v64 = 0.0, v32 = 0.0;
            for (int which = 0; which < 2; ++which) {
              const int P = pt * 16 + (which == 0 ? off64 : row);
              double v = 0.0;
              if (P < npair) {
                const long long idx = ((long long)perm[pn1[P]] * nB + perm[pn2[P]]) * ns + s;
                if (r < d->n_r) v = U[(size_t)idx * d->n_r + r];
                else if (r == d->n_r) v = d->I_pi[idx];
              }
              if (which == 0) v64 = v; else v32 = v;
            }
            const size_t o = (((size_t)pt * ns + s) * KC + kc) * 64 + lane;
            h64[o] = v64;
            h32[o] = (float)v32;
          }
    // transposed tiles of the adjoint: [pt][s][rb][kk][lane], row = r, k = pair 4*(lane/16) + kk
    for (int pt = 0; pt < NPT; ++pt)
      for (int s = 0; s < ns; ++s)
        for (int rb = 0; rb < RB; ++rb)
          for (int kk = 0; kk < 4; ++kk)
            for (int lane = 0; lane < 64; ++lane) {
              const int r = 16 * rb + (lane & 15), P = pt * 16 + 4 * (lane >> 4) + kk;
              double v = 0.0;
              if (P < npair) {
                const long long idx = ((long long)perm[pn1[P]] * nB + perm[pn2[P]]) * ns + s;
                if (r < d->n_r) v = U[(size_t)idx * d->n_r + r];
                else if (r == d->n_r) v = d->I_pi[idx];
              }
              h2[((((size_t)pt * ns + s) * RB + rb) * 4 + kk) * 64 + lane] = v;
            }
    double* d64 = nullptr;
    double* d2 = nullptr;
    float* d32 = nullptr;
    if (hipMalloc(&d64, tile_n * 8) != hipSuccess || hipMalloc(&d32, tile_n * 4) != hipSuccess ||
        hipMalloc(&d2, tile2_n * 8) != hipSuccess)
      return fail(c, LBDDC_E_NOMEM, "load_rom: device allocation failed");
    if (hipMemcpy(d64, h64.data(), tile_n * 8, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(d32, h32.data(), tile_n * 4, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(d2, h2.data(), tile2_n * 8, hipMemcpyHostToDevice) != hipSuccess)
      return fail(c, LBDDC_E_HIP, "load_rom: copy failed");
    R.ut64.push_back(d64);
    R.ut32.push_back(d32);
    R.ucol64.push_back(d2);
  }
  const size_t nco = (size_t)ncl * nnode * d->n_r;
  if (hipMalloc(&R.coeff, nco * 8) != hipSuccess) return fail(c, LBDDC_E_NOMEM, "load_rom: allocation failed");
  if (hipMemcpy(R.coeff, d->coeff, nco * 8, hipMemcpyHostToDevice) != hipSuccess)
    return fail(c, LBDDC_E_HIP, "load_rom: copy failed");
  auto it = c->roms.find(d->family);
  if (it != c->roms.end()) {
    for (auto p2 : it->second.ut64) hipFree(p2);
    for (auto p2 : it->second.ut32) hipFree(p2);
    for (auto p2 : it->second.ucol64) hipFree(p2);
    if (it->second.coeff) hipFree(it->second.coeff);
  }
  c->roms[d->family] = R;
  c->have_problem = c->assembled = c->setup_done = c->solved = false;
  return LBDDC_OK;
}

// Build a problem into a context that holds only the persistent parts
// (copy_persistent).  On failure the caller releases what was allocated.
static lbddc_status build_problem(Ctx* c, const lbddc_problem_desc* d, const std::vector<int>& fam_ids) {
  const int ncell = d->nx * d->ny;
  const int netx = d->map_order * d->nx + 1, nety = d->map_order * d->ny + 1;
  c->fam_ids = fam_ids;
  c->nx = d->nx; c->ny = d->ny; c->p = d->p; c->q = d->q; c->m = d->map_order; c->nrhs = d->nrhs;
  c->E = d->E; c->nu = d->nu; c->rho = d->rho;
  c->moments = (d->constraints & LBDDC_CON_EDGE_MOMENT) != 0;
  c->clamped = d->clamped_sides;
  c->load_edge = d->loaded_side == LBDDC_SIDE_LEFT ? 0 : d->loaded_side == LBDDC_SIDE_RIGHT ? 1
               : d->loaded_side == LBDDC_SIDE_BOTTOM ? 2 : 3;
  c->n_side = c->load_edge < 2 ? d->ny : d->nx;
  c->ncell = ncell; c->nB = (c->p + 1) * (c->p + 1); c->ndof = 2 * c->nB; c->nN = c->nB;
  c->nIn = (c->p - 1) * (c->p - 1); c->nI = 2 * c->nIn; c->nU = 8 * c->p; c->nE = c->nU - 8;
  c->nce = c->moments ? 3 : 2; c->nC = 8 + 4 * c->nce; c->nL = (c->q + 1) * (c->q + 1); c->ns = 4 * c->nL;
  c->npair = c->nN * (c->nN + 1) / 2; c->NPT = (c->npair + 15) / 16;
  c->n_i = (long long)c->nB * c->nB * c->ns;
  c->Gx = c->p * c->nx + 1; c->Gy = c->p * c->ny + 1; c->netx = netx; c->nety = nety;
  c->KC = 0;
  for (int f : fam_ids) c->KC = std::max(c->KC, c->roms[f].KC);
  c->NI = c->nI * ncell;
  {
    const int kx = ((c->clamped & LBDDC_SIDE_LEFT) != 0) + ((c->clamped & LBDDC_SIDE_RIGHT) != 0);
    const int ky = ((c->clamped & LBDDC_SIDE_BOTTOM) != 0) + ((c->clamped & LBDDC_SIDE_TOP) != 0);
    c->Nfree = 2 * (c->Gx - kx) * (c->Gy - ky);
  }
  if (!build_topology(c)) return LBDDC_E_NOMEM;
  std::vector<double> tab;
  build_tables(c, tab);
  const size_t nU = c->nU, nC = c->nC, NU = c->NU, NC = c->NC;
  c->nblk = std::min(c->nrhs, kBlockRhs);
  const size_t nbk = c->nblk;
  bool ok = dalloc_t(c, &c->d_tab, tab.size()) && dalloc_t(c, &c->d_ctrl, (size_t)netx * nety * 2) &&
            dalloc_t(c, &c->d_ctrl_bak, (size_t)netx * nety * 2) && dalloc_t(c, &c->d_t_bak, ncell) &&
            dalloc_t(c, &c->d_family, ncell) && dalloc_t(c, &c->d_t, ncell) &&
            dalloc_t(c, &c->d_mu, (size_t)ncell * 4) && dalloc_t(c, &c->d_mu_bak, (size_t)ncell * 4) &&
            dalloc_t(c, &c->d_trac, (size_t)c->nrhs * c->n_side * 2) && dalloc_t(c, &c->d_flags, 128) &&
            dalloc_t(c, &c->d_theta, (size_t)ncell * c->ns * 4) && dalloc_t(c, &c->d_theta32, (size_t)ncell * c->ns * 4) &&
            dalloc_t(c, &c->d_itil, (size_t)ncell * 4 * c->KC) && dalloc_t(c, &c->d_itil32, (size_t)ncell * 4 * c->KC) &&
            dalloc_t(c, &c->d_cluster, ncell) && dalloc_t(c, &c->d_sorted, ncell) &&
            dalloc_t(c, &c->d_tiles, (size_t)4 * (ncell / 16 + 64) + 64) &&
            dalloc_t(c, &c->d_theta_t, (size_t)(ncell / 128 + 17) * c->ns * 512) &&
            dalloc_t(c, &c->d_theta_t32, (size_t)(ncell / 128 + 17) * c->ns * 512) &&
            dalloc_t(c, &c->d_K, (size_t)ncell * c->npair * 4) &&
            dalloc_t(c, &c->d_load, (size_t)c->nrhs * ncell * nU) &&
            dalloc_t(c, &c->d_cons, (size_t)ncell * 4 * c->nce * (c->p + 1) * 2) &&
            dalloc_t(c, &c->d_S, (size_t)ncell * nU * (nU + 1) / 2) &&
            dalloc_t(c, &c->d_W, (size_t)ncell * schur_w_count(c->p)) && dalloc_t(c, &c->d_diagK, (size_t)ncell * nU) &&
            dalloc_t(c, &c->d_Ktot, NU) && dalloc(c, &c->d_P, (size_t)ncell * c->nE * (c->nE + 1) / 2 * 8) &&
            dalloc(c, &c->d_Psi, (size_t)ncell * nU * nC * 8) && dalloc_t(c, &c->d_D, (size_t)ncell * nU) &&
            dalloc_t(c, &c->d_ScLoc, (size_t)ncell * nC * (nC + 1) / 2) &&
            dalloc_t(c, &c->d_coarse, (size_t)c->co.nd_front_total) &&
            dalloc_t(c, &c->d_up, ((size_t)c->co.nd_up_total + 1) * nbk) &&
            dalloc_t(c, &c->d_beff, ((size_t)c->co.nd_beff_total + 1) * nbk) &&
            dalloc_t(c, &c->d_gjC, (size_t)c->co.nd_cp_total + 1) &&
            dalloc_t(c, &c->d_f_blk, (size_t)c->co.f_blk_total + 2) &&
            dalloc_t(c, &c->d_f, (size_t)c->nrhs * NU) && dalloc_t(c, &c->d_x, (size_t)c->nrhs * NU) &&
            dalloc_t(c, &c->d_r, NU * nbk) && dalloc_t(c, &c->d_z, NU * nbk) && dalloc_t(c, &c->d_p, NU * nbk) &&
            dalloc_t(c, &c->d_q, NU * nbk) &&
            dalloc_t(c, &c->d_partU, (size_t)ncell * nU * nbk) && dalloc_t(c, &c->d_partC, (size_t)ncell * nC * nbk) &&
            dalloc_t(c, &c->d_zc, NC * nbk) && dalloc_t(c, &c->d_tc, NC) && dalloc_t(c, &c->d_xc, NC * nbk) &&
            dalloc_t(c, &c->d_red, (size_t)(std::max(NU, NC) / 256 + 272)) && dalloc_t(c, &c->d_scal, c->scal_stride() * nbk) &&
            dalloc_t(c, &c->d_vred, c->vred_stride() * nbk) &&
            dalloc_t(c, &c->d_u, (size_t)c->nrhs * c->Gx * c->Gy * 2) &&
            dalloc_t(c, &c->d_ucell, (size_t)c->nrhs * ncell * c->ndof) &&
            dalloc_t(c, &c->d_H, (size_t)ncell * 4 * c->KC) && dalloc_t(c, &c->d_G, (size_t)ncell * c->ns * 4) &&
            dalloc_t(c, &c->d_gcell, (size_t)ncell * (c->m + 1) * (c->m + 1) * 2) &&
            dalloc_t(c, &c->d_edge_br, (size_t)ncell * 4 * kEdgeBreaks) && dalloc_t(c, &c->d_edge_nm, (size_t)ncell * 8) &&
            dalloc_t(c, &c->d_gt, (size_t)c->nrhs * ncell) && dalloc_t(c, &c->d_gmu, (size_t)c->nrhs * ncell * 4) &&
            dalloc_t(c, &c->d_gX, (size_t)c->nrhs * netx * nety * 2) && dalloc_t(c, &c->d_J, c->nrhs) &&
            dalloc_t(c, &c->d_adj_tiles, (size_t)4 * (ncell / 16 + 64)) && dalloc(c, &c->d_adj_ptrs, 64 * 8);
  if (ok && hipHostMalloc((void**)&c->h_red, c->scal_stride() * nbk * sizeof(double),
                      hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess) {
    c->h_red = nullptr;
    c->err = "pinned host allocation failed";
    ok = false;
  }
  if (ok && hipHostGetDevicePointer((void**)&c->d_hred, c->h_red, 0) != hipSuccess) {
    c->err = "pinned host buffer has no device address";
    ok = false;
  }
  if (!ok) return LBDDC_E_NOMEM;
  // family -> slot table after the 8 flag words
  std::vector<int> flags(128, 0);
  for (int f = 0; f < 64; ++f) flags[8 + f] = -1;
  for (size_t s = 0; s < fam_ids.size(); ++s) flags[8 + fam_ids[s]] = (int)s;
  hipError_t e = hipSuccess;
  if (e == hipSuccess) e = hipMemcpy(c->d_flags, flags.data(), 128 * sizeof(int), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(c->d_tab, tab.data(), tab.size() * 8, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(c->d_ctrl, d->ctrl, (size_t)netx * nety * 2 * 8, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(c->d_family, d->family, ncell * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(c->d_t, d->t, ncell * 8, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = d->mu ? hipMemcpy(c->d_mu, d->mu, (size_t)ncell * 4 * 8, hipMemcpyHostToDevice)
                                 : hipMemset(c->d_mu, 0, (size_t)ncell * 4 * 8);
  // dJ/dmu stays zero for problems without four-parameter families
  if (e == hipSuccess) e = hipMemset(c->d_gmu, 0, (size_t)c->nrhs * ncell * 4 * 8);
  if (e == hipSuccess) e = hipMemcpy(c->d_trac, d->traction, (size_t)c->nrhs * c->n_side * 2 * 8, hipMemcpyHostToDevice);
  if (e != hipSuccess) return hipfail(c, e, "set_problem upload");
  c->fam_host.assign(d->family, d->family + ncell);
  c->t_host.assign(d->t, d->t + ncell);
  c->any_dim4 = false;
  for (int f : fam_ids) c->any_dim4 |= c->roms[f].dim == 4;
  // validate the maps on the device (det J) right away
  e = launch_geometry(c);
  if (e != hipSuccess) return hipfail(c, e, "set_problem geometry");
  return check_flags(c, "set_problem");
}

lbddc_status lbddc_set_problem(lbddc_ctx* x, const lbddc_problem_desc* d) {
  if (!x) return LBDDC_E_ARG;
  Ctx* c = &x->c;
  if (!d || !d->ctrl || !d->family || !d->t || !d->traction) return fail(c, LBDDC_E_ARG, "set_problem: null pointer");
  if (d->nx < 1 || d->ny < 1 || (long long)d->nx * d->ny > (1LL << 22)) return fail(c, LBDDC_E_ARG, "set_problem: bad grid size");
  if (d->p < 2 || d->p > 8) return fail(c, LBDDC_E_UNSUPPORTED, "set_problem: 2 <= p <= 8 supported");
  if (d->q < 1 || d->q > 3 || d->map_order < 1 || d->map_order > 4) return fail(c, LBDDC_E_UNSUPPORTED, "set_problem: q or map order out of range");
  if (d->nrhs < 1 || d->nrhs > 16) return fail(c, LBDDC_E_ARG, "set_problem: 1 <= nrhs <= 16");
  if (!(d->E > 0) || !(d->nu > -1 && d->nu < 0.5) || !(d->rho >= 0 && d->rho < 1))
    return fail(c, LBDDC_E_ARG, "set_problem: material or rho out of range");
  if (d->constraints & ~7u) return fail(c, LBDDC_E_ARG, "set_problem: unknown constraint bits");
  if (d->constraints != (LBDDC_CON_CORNERS | LBDDC_CON_EDGE_AVG) &&
      d->constraints != (LBDDC_CON_CORNERS | LBDDC_CON_EDGE_AVG | LBDDC_CON_EDGE_MOMENT))
    return fail(c, LBDDC_E_UNSUPPORTED, "set_problem: constraint sets CORNERS|EDGE_AVG and CORNERS|EDGE_AVG|EDGE_MOMENT are supported");
  if (d->p < 3 && (d->constraints & LBDDC_CON_EDGE_MOMENT))
    return fail(c, LBDDC_E_UNSUPPORTED,
                "set_problem: edge moments need p >= 3 (at p = 2 an edge has 2 interior dofs for 3 edge constraints)");
  if (d->clamped_sides == 0 || (d->clamped_sides & ~15u))
    return fail(c, LBDDC_E_ARG, "set_problem: clamped_sides must be a nonempty set of LBDDC_SIDE_* bits");
  if (d->loaded_side != LBDDC_SIDE_LEFT && d->loaded_side != LBDDC_SIDE_RIGHT && d->loaded_side != LBDDC_SIDE_BOTTOM &&
      d->loaded_side != LBDDC_SIDE_TOP)
    return fail(c, LBDDC_E_ARG, "set_problem: loaded_side must be one LBDDC_SIDE_* value");
  if ((uint32_t)d->loaded_side & d->clamped_sides) return fail(c, LBDDC_E_ARG, "set_problem: the loaded side is clamped");
  const int ncell = d->nx * d->ny;
  const int netx = d->map_order * d->nx + 1, nety = d->map_order * d->ny + 1;
  const int n_side = (d->loaded_side == LBDDC_SIDE_LEFT || d->loaded_side == LBDDC_SIDE_RIGHT) ? d->ny : d->nx;
  for (size_t i = 0; i < (size_t)netx * nety * 2; ++i)
    if (!std::isfinite(d->ctrl[i])) return fail(c, LBDDC_E_ARG, "set_problem: non-finite control point");
  for (size_t i = 0; i < (size_t)d->nrhs * n_side * 2; ++i)
    if (!std::isfinite(d->traction[i])) return fail(c, LBDDC_E_ARG, "set_problem: non-finite traction");
  std::vector<int> fam_ids;
  for (int i = 0; i < ncell; ++i) {
    int f = d->family[i];
    auto it = c->roms.find(f);
    if (it == c->roms.end()) return fail(c, LBDDC_E_ROM, "set_problem: a cell's family has no loaded ROM");
    if (it->second.p != d->p || it->second.q != d->q) return fail(c, LBDDC_E_ROM, "set_problem: ROM degrees differ from the problem's");
    if (it->second.dim == 4) {
      if (!d->mu) return fail(c, LBDDC_E_ARG, "set_problem: a family has four parameters per cell and mu is NULL");
      for (int k = 0; k < 4; ++k) {
        const double v = d->mu[(size_t)i * 4 + k];
        if (!std::isfinite(v)) return fail(c, LBDDC_E_ARG, "set_problem: non-finite threshold");
        if (!(v >= it->second.lo && v <= it->second.hi))
          return fail(c, LBDDC_E_PARAM_RANGE, "set_problem: a corner threshold lies outside its ROM box");
      }
    } else {
      double t = d->t[i];
      if (!std::isfinite(t)) return fail(c, LBDDC_E_ARG, "set_problem: non-finite thickness");
      if (!(t >= it->second.lo && t <= it->second.hi))
        return fail(c, LBDDC_E_PARAM_RANGE, "set_problem: a thickness parameter lies outside its ROM box");
    }
    if (std::find(fam_ids.begin(), fam_ids.end(), f) == fam_ids.end()) fam_ids.push_back(f);
  }
  if (fam_ids.size() > 4) return fail(c, LBDDC_E_UNSUPPORTED, "set_problem: at most 4 families per problem");
  std::sort(fam_ids.begin(), fam_ids.end());
  int G = 0;
  for (int f : fam_ids) G += c->roms[f].ncl;
  if (G > 16) return fail(c, LBDDC_E_UNSUPPORTED, "set_problem: at most 16 (family, cluster) groups");
  hipSetDevice(c->device);
  hipStreamSynchronize(c->stream);
  // the new problem is built beside the current one, which stays in place
  // (with all its stages) until the new one is complete and valid
  Ctx* n = new (std::nothrow) Ctx();
  if (!n) return fail(c, LBDDC_E_NOMEM, "set_problem: host allocation failed");
  copy_persistent(c, n);
  lbddc_status s = build_problem(n, d, fam_ids);
  if (s != LBDDC_OK) {
    hipStreamSynchronize(c->stream);
    c->err = n->err;
    release_problem(n);
    delete n;
    return s;
  }
  release_problem(c);
  n->roms = std::move(c->roms);
  n->have_problem = true;
  *c = std::move(*n);
  delete n;
  return LBDDC_OK;
}

lbddc_status lbddc_set_geometry_device(lbddc_ctx* x, const double* d_ctrl, const double* d_t, const double* d_mu) {
  if (!x) return LBDDC_E_ARG;
  Ctx* c = &x->c;
  if (!c->have_problem) return fail(c, LBDDC_E_STATE, "set_geometry_device: no problem");
  if (!d_ctrl && !d_t && !d_mu) return fail(c, LBDDC_E_ARG, "set_geometry_device: null pointers");
  hipSetDevice(c->device);
  const size_t nctrl = (size_t)c->netx * c->nety * 2 * 8, nt = (size_t)c->ncell * 8, nmu = 4 * nt;
  // keep the current geometry aside, validate the new one in its place, and
  // put the old one back if it is rejected
  HIPCHK(hipMemcpyAsync(c->d_ctrl_bak, c->d_ctrl, nctrl, hipMemcpyDeviceToDevice, c->stream), "set_geometry_device");
  HIPCHK(hipMemcpyAsync(c->d_t_bak, c->d_t, nt, hipMemcpyDeviceToDevice, c->stream), "set_geometry_device");
  HIPCHK(hipMemcpyAsync(c->d_mu_bak, c->d_mu, nmu, hipMemcpyDeviceToDevice, c->stream), "set_geometry_device");
  if (d_ctrl) HIPCHK(hipMemcpyAsync(c->d_ctrl, d_ctrl, nctrl, hipMemcpyDeviceToDevice, c->stream), "set_geometry_device");
  if (d_t) HIPCHK(hipMemcpyAsync(c->d_t, d_t, nt, hipMemcpyDeviceToDevice, c->stream), "set_geometry_device");
  if (d_mu) HIPCHK(hipMemcpyAsync(c->d_mu, d_mu, nmu, hipMemcpyDeviceToDevice, c->stream), "set_geometry_device");
  c->geom_gen++;  // (also when the new geometry is rejected and the old one restored: harmless)
  HIPCHK(launch_geometry(c), "set_geometry_device");
  lbddc_status s = check_flags(c, "set_geometry_device");
  if (s != LBDDC_OK) {
    const std::string msg = c->err;
    // the previous geometry and the coefficients computed from it (the
    // geometry pass is deterministic, so they are restored bit for bit)
    HIPCHK(hipMemcpyAsync(c->d_ctrl, c->d_ctrl_bak, nctrl, hipMemcpyDeviceToDevice, c->stream), "set_geometry_device restore");
    HIPCHK(hipMemcpyAsync(c->d_t, c->d_t_bak, nt, hipMemcpyDeviceToDevice, c->stream), "set_geometry_device restore");
    HIPCHK(hipMemcpyAsync(c->d_mu, c->d_mu_bak, nmu, hipMemcpyDeviceToDevice, c->stream), "set_geometry_device restore");
    HIPCHK(launch_geometry(c), "set_geometry_device restore");
    lbddc_status s2 = check_flags(c, "set_geometry_device restore");
    if (s2 != LBDDC_OK) return s2;
    c->err = msg;
    return s;
  }
  c->assembled = c->setup_done = c->solved = false;
  c->k32_valid = false;
  return LBDDC_OK;
}

lbddc_status lbddc_assemble(lbddc_ctx* x, lbddc_precision prec) {
  if (!x) return LBDDC_E_ARG;
  Ctx* c = &x->c;
  if (!c->have_problem) return fail(c, LBDDC_E_STATE, "assemble: no problem set");
  if (prec != LBDDC_FP64 && prec != LBDDC_MIXED && prec != LBDDC_FP32_CONTRACTION)
    return fail(c, LBDDC_E_ARG, "assemble: bad precision");
  hipSetDevice(c->device);
  const bool fp32 = prec == LBDDC_FP32_CONTRACTION;
  if (fp32 && !c->d_K32) {
    if (!dalloc_t(c, &c->d_K32, (size_t)c->ncell * c->npair * 4)) return LBDDC_E_NOMEM;
  }
  c->assembled = c->setup_done = c->solved = false;
  c->k32_valid = false;
  HIPCHK(hipEventRecord(c->ev[6], c->stream), "assemble");
  // The edge rows and loads depend on the control net and the thresholds
  // only.  On four-parameter lattices their root searches take about half a
  // millisecond, so they run on the second stream beside the geometry pass and
  // the contraction, joined before the end of the call.
  const bool side = c->any_dim4;
  if (side) {
    HIPCHK(hipEventRecord(c->side_fork, c->stream), "assemble");
    HIPCHK(hipStreamWaitEvent(c->side, c->side_fork, 0), "assemble");
    HIPCHK(launch_constraints_loads(c, c->side), "assemble constraints");
    HIPCHK(hipEventRecord(c->side_join, c->side), "assemble");
  }
  HIPCHK(launch_geometry(c), "assemble geometry");
  HIPCHK(hipEventRecord(c->ev[2], c->stream), "assemble");
  if (!side) HIPCHK(launch_constraints_loads(c, c->stream), "assemble constraints");
  HIPCHK(launch_assembly(c, fp32, c->ev[0], c->ev[1]), "assemble contraction");
  if (side) HIPCHK(hipStreamWaitEvent(c->stream, c->side_join, 0), "assemble");
  HIPCHK(hipEventRecord(c->ev[7], c->stream), "assemble");
  lbddc_status s = check_flags(c, "assemble");
  if (s != LBDDC_OK) return s;
  float ms = 0;
  if (hipEventElapsedTime(&ms, c->ev[0], c->ev[1]) == hipSuccess) c->phase_ms[0] = ms;
  if (hipEventElapsedTime(&ms, c->ev[6], c->ev[7]) == hipSuccess) c->phase_ms[1] = ms;
  if (hipEventElapsedTime(&ms, c->ev[6], c->ev[2]) == hipSuccess) c->phase_ms[14] = ms;
  c->asm_prec = prec;
  c->assembled = !fp32;  // the FP32 contraction alone feeds no later stage
  c->k32_valid = fp32;
  return LBDDC_OK;
}

lbddc_status lbddc_assemble_fp32_noalloc(lbddc_ctx* x, float* d_K) {
  if (!x) return LBDDC_E_ARG;
  Ctx* c = &x->c;
  if (!c->have_problem) return fail(c, LBDDC_E_STATE, "assemble_fp32_noalloc: no problem set");
  if (!d_K) return fail(c, LBDDC_E_ARG, "assemble_fp32_noalloc: null output");
  hipSetDevice(c->device);
  lbddc_status s = assemble_fp32_noalloc(c, d_K);
  if (s != LBDDC_OK) return s;
  return check_flags(c, "assemble_fp32_noalloc");
}

lbddc_status lbddc_coarse_solve(lbddc_ctx* x, const double* z, double* g) {
  if (!x) return LBDDC_E_ARG;
  Ctx* c = &x->c;
  if (!c->setup_done) return fail(c, LBDDC_E_STATE, "coarse_solve: setup first");
  if (!z || !g) return fail(c, LBDDC_E_ARG, "coarse_solve: null vector");
  hipSetDevice(c->device);
  const size_t n = (size_t)c->NC * 8;
  HIPCHK(hipMemcpyAsync(c->d_zc, z, n, hipMemcpyHostToDevice, c->stream), "coarse_solve");
  HIPCHK(launch_coarse_solve(c, c->d_zc, c->d_xc), "coarse_solve");
  HIPCHK(hipMemcpyAsync(g, c->d_xc, n, hipMemcpyDeviceToHost, c->stream), "coarse_solve");
  HIPCHK(hipStreamSynchronize(c->stream), "coarse_solve");
  return LBDDC_OK;
}

lbddc_status lbddc_setup(lbddc_ctx* x, lbddc_precision prec) {
  if (!x) return LBDDC_E_ARG;
  Ctx* c = &x->c;
  if (!c->assembled) return fail(c, LBDDC_E_STATE, "setup: assemble (FP64 or mixed) first");
  if (prec != LBDDC_FP64 && prec != LBDDC_MIXED) return fail(c, LBDDC_E_ARG, "setup: bad precision");
  hipSetDevice(c->device);
  c->setup_done = c->solved = false;
  const bool fp32 = prec == LBDDC_MIXED;
  HIPCHK(hipEventRecord(c->ev[6], c->stream), "setup");
  HIPCHK(hipEventRecord(c->ev[0], c->stream), "setup");
  HIPCHK(launch_schur(c), "setup schur");
  HIPCHK(hipEventRecord(c->ev[1], c->stream), "setup");
  HIPCHK(launch_weights(c), "setup weights");
  HIPCHK(launch_precond(c, fp32), "setup precond");
  HIPCHK(launch_coarse_assemble(c), "setup coarse assembly");
  HIPCHK(hipEventRecord(c->ev[2], c->stream), "setup");
  HIPCHK(launch_coarse_factor(c), "setup coarse factor");
  HIPCHK(hipEventRecord(c->ev[3], c->stream), "setup");
  HIPCHK(hipEventRecord(c->ev[7], c->stream), "setup");
  lbddc_status s = check_flags(c, "setup");
  if (s != LBDDC_OK) return s;
  float ms = 0;
  if (hipEventElapsedTime(&ms, c->ev[0], c->ev[1]) == hipSuccess) c->phase_ms[2] = ms;
  if (hipEventElapsedTime(&ms, c->ev[6], c->ev[7]) == hipSuccess) c->phase_ms[3] = ms;
  if (hipEventElapsedTime(&ms, c->ev[2], c->ev[3]) == hipSuccess) c->phase_ms[4] = ms;
  c->setup_prec = prec;
  c->setup_done = true;
  return LBDDC_OK;
}

// Both solve entries: the load cases one PCG at a time (block = false), or in
// blocks of up to kBlockRhs cases (block = true, the default for several).
static lbddc_status solve_cases(lbddc_ctx* x, double rtol, int32_t max_iter, lbddc_solve_info* info, bool block) {
  if (!x) return LBDDC_E_ARG;
  Ctx* c = &x->c;
  if (!c->setup_done) return fail(c, LBDDC_E_STATE, "solve: setup first");
  if (!(rtol > 0) || max_iter < 1) return fail(c, LBDDC_E_ARG, "solve: rtol > 0 and max_iter >= 1 required");
  hipSetDevice(c->device);
  c->solved = false;
  const bool fp32 = c->setup_prec == LBDDC_MIXED;
  c->info.assign(c->nrhs, lbddc_solve_info{0, 0, 0});
  double t_op = 0, t_pre = 0, t_coarse = 0, t_cf = 0, t_cb = 0;
  int napp = 0, nop = 0;
  float ms = 0;
  double t_rec = 0;
  HIPCHK(hipEventRecord(c->ev[7], c->stream), "solve");
  hipEvent_t e_start;
  HIPCHK(hipEventCreate(&e_start), "solve");
  HIPCHK(hipEventRecord(e_start, c->stream), "solve");
  lbddc_status status = LBDDC_OK;
  const int step = block && c->nrhs > 1 ? c->nblk : 1;
  for (int r0 = 0; r0 < c->nrhs; r0 += step) {
    const int nr = std::min(step, c->nrhs - r0);
    // right-hand sides: gather-sum of the cell loads (f_I = 0 for edge tractions)
    for (int r = r0; r < r0 + nr; ++r) HIPCHK(gather_rhs(c, r), "solve rhs");
    lbddc_solve_info* inf = c->info.data() + r0;
    hipError_t e;
    if (nr == 1) {
      e = pcg_solve(c, r0, rtol, max_iter, inf, fp32, &t_op, &t_pre, &t_coarse, &t_cf, &t_cb, &napp);
      nop += inf->iters;
    } else {
      e = pcg_solve_block(c, r0, nr, rtol, max_iter, inf, fp32, &t_op, &t_pre, &t_coarse, &t_cf, &t_cb, &napp,
                          &nop);
    }
    if (e == hipErrorUnknown) {
      if (info)
        for (int r = r0; r < r0 + nr; ++r) info[r] = c->info[r];
      hipStreamSynchronize(c->stream);
      return fail(c, LBDDC_E_BREAKDOWN, "solve: PCG breakdown (p^T S p <= 0 or r^T z <= 0)");
    }
    if (e != hipSuccess) return hipfail(c, e, "solve pcg");
    for (int r = r0; r < r0 + nr; ++r) {
      HIPCHK(pcg_true_residual(c, r, &c->info[r].true_rel_res), "solve residual");
      hipEvent_t a, b;
      hipEventCreate(&a);
      hipEventCreate(&b);
      hipEventRecord(a, c->stream);
      HIPCHK(launch_recover(c, r), "solve recovery");
      hipEventRecord(b, c->stream);
      hipEventSynchronize(b);
      if (hipEventElapsedTime(&ms, a, b) == hipSuccess) t_rec += ms;
      hipEventDestroy(a);
      hipEventDestroy(b);
      if (info) info[r] = c->info[r];
      if (c->info[r].rel_res > rtol) status = LBDDC_E_NOT_CONVERGED;
    }
  }
  HIPCHK(hipEventRecord(c->ev[6], c->stream), "solve");
  HIPCHK(hipEventSynchronize(c->ev[6]), "solve");
  if (hipEventElapsedTime(&ms, e_start, c->ev[6]) == hipSuccess) c->phase_ms[5] = ms;
  hipEventDestroy(e_start);
  c->phase_ms[6] = nop ? t_op / nop : 0;
  c->phase_ms[7] = napp ? t_pre / napp : 0;
  c->phase_ms[8] = napp ? t_coarse / napp : 0;
  c->phase_ms[12] = napp ? t_cf / napp : 0;
  c->phase_ms[13] = napp ? t_cb / napp : 0;
  c->phase_ms[9] = t_rec;
  {
    lbddc_status fs = check_flags(c, "solve");
    if (fs != LBDDC_OK) return fs;
  }
  c->solved = true;
  if (status != LBDDC_OK) c->err = "solve: PCG reached max_iter before rtol";
  return status;
}

lbddc_status lbddc_solve(lbddc_ctx* x, double rtol, int32_t max_iter, lbddc_solve_info* info) {
  return solve_cases(x, rtol, max_iter, info, true);
}

lbddc_status lbddc_solve_sequential(lbddc_ctx* x, double rtol, int32_t max_iter, lbddc_solve_info* info) {
  return solve_cases(x, rtol, max_iter, info, false);
}

lbddc_status lbddc_set_timing(lbddc_ctx* x, int32_t mask) {
  if (!x) return LBDDC_E_ARG;
  if (mask & ~(LBDDC_TIME_ALL | LBDDC_TIME_SAMPLE)) return fail(&x->c, LBDDC_E_ARG, "set_timing: unknown phase bits");
  x->c.timing = mask;
  return LBDDC_OK;
}

lbddc_status lbddc_get_displacement(lbddc_ctx* x, int32_t rhs, double* u) {
  if (!x) return LBDDC_E_ARG;
  Ctx* c = &x->c;
  if (!c->solved) return fail(c, LBDDC_E_STATE, "get_displacement: solve first");
  if (rhs < 0 || rhs >= c->nrhs || !u) return fail(c, LBDDC_E_ARG, "get_displacement: bad arguments");
  hipSetDevice(c->device);
  const size_t n = (size_t)c->Gx * c->Gy * 2;
  HIPCHK(hipMemcpyAsync(u, c->d_u + rhs * n, n * 8, hipMemcpyDeviceToHost, c->stream), "get_displacement");
  HIPCHK(hipStreamSynchronize(c->stream), "get_displacement");
  return LBDDC_OK;
}

lbddc_status lbddc_get_displacement_device(lbddc_ctx* x, int32_t rhs, double* d_u) {
  if (!x) return LBDDC_E_ARG;
  Ctx* c = &x->c;
  if (!c->solved) return fail(c, LBDDC_E_STATE, "get_displacement_device: solve first");
  if (rhs < 0 || rhs >= c->nrhs || !d_u) return fail(c, LBDDC_E_ARG, "get_displacement_device: bad arguments");
  hipSetDevice(c->device);
  const size_t n = (size_t)c->Gx * c->Gy * 2;
  HIPCHK(hipMemcpyAsync(d_u, c->d_u + rhs * n, n * 8, hipMemcpyDeviceToDevice, c->stream), "get_displacement_device");
  return LBDDC_OK;
}

lbddc_status lbddc_query(const lbddc_ctx* x, int32_t what, int64_t* v) {
  if (!x || !v) return LBDDC_E_ARG;
  const Ctx* c = &x->c;
  if (!c->have_problem && what != LBDDC_Q_DEVICE_BYTES) return LBDDC_E_STATE;
  switch (what) {
    case LBDDC_Q_NCELL: *v = c->ncell; break;
    case LBDDC_Q_NDOF_FREE: *v = c->Nfree; break;
    case LBDDC_Q_N_SKELETON: *v = c->NU; break;
    case LBDDC_Q_N_INTERIOR: *v = c->NI; break;
    case LBDDC_Q_N_COARSE: *v = c->NC; break;
    case LBDDC_Q_N_I_ROM: *v = c->n_i; break;
    case LBDDC_Q_NU_CELL: *v = c->nU; break;
    case LBDDC_Q_NC_CELL: *v = c->nC; break;
    case LBDDC_Q_NRHS: *v = c->nrhs; break;
    case LBDDC_Q_NR_MAX: *v = 4 * c->KC; break;
    case LBDDC_Q_NPAIR: *v = c->npair; break;
    case LBDDC_Q_DEVICE_BYTES: *v = (int64_t)c->dev_bytes; break;
    case LBDDC_Q_COARSE_SOLVE_BYTES: {
      int64_t b = 0;
      for (const NDNodeH& d : c->co.nd_nodes) b += 8LL * d.ns * (d.ns + 2LL * d.nb);
      *v = b;
      break;
    }
    case LBDDC_Q_COARSE_LEVELS: *v = (int64_t)c->co.nd_levels.size(); break;
    case LBDDC_Q_COARSE_FWD_BYTES: {
      int64_t b = 0;
      for (const NDNodeH& d : c->co.nd_nodes) b += 8LL * d.ns * d.nb;
      *v = b;
      break;
    }
    case LBDDC_Q_COARSE_SWEEP_LAUNCHES: {
      // levels above the subtree levels one launch each, the subtrees one
      const int L = (int)c->co.nd_levels.size();
      *v = c->co.fused ? c->co.fused_level + 1 : c->co.sub_level < L ? c->co.sub_level + 1 : L;
      break;
    }
    default: return LBDDC_E_ARG;
  }
  return LBDDC_OK;
}

lbddc_status lbddc_phase_times(lbddc_ctx* x, double* ms, int32_t n) {
  if (!x || !ms || n < 0 || n > 15) return LBDDC_E_ARG;
  for (int i = 0; i < n; ++i) ms[i] = x->c.phase_ms[i];
  return LBDDC_OK;
}

lbddc_status lbddc_export_cells(lbddc_ctx* x, int32_t which, int32_t first, int32_t count, double* out) {
  if (!x) return LBDDC_E_ARG;
  Ctx* c = &x->c;
  if (!c->have_problem) return fail(c, LBDDC_E_STATE, "export: no problem");
  if (!out || first < 0 || count < 0 || first + count > c->ncell) return fail(c, LBDDC_E_ARG, "export: bad range");
  const bool need_asm = which == LBDDC_X_K || which == LBDDC_X_LOAD || which == LBDDC_X_CONS;
  const bool need_setup = which == LBDDC_X_S || which == LBDDC_X_D || which == LBDDC_X_PSI || which == LBDDC_X_SC || which == LBDDC_X_FINE;
  if (need_asm && !c->assembled && !(which == LBDDC_X_K && c->k32_valid)) return fail(c, LBDDC_E_STATE, "export: assemble first");
  if (need_setup && !c->setup_done) return fail(c, LBDDC_E_STATE, "export: setup first");
  hipSetDevice(c->device);
  HIPCHK(hipStreamSynchronize(c->stream), "export");
  const int nU = c->nU, nC = c->nC, nB = c->nB, nE = c->nE;
  auto fetch = [&](const void* base, size_t per, size_t elem) -> std::vector<char> {
    std::vector<char> h(per * count * elem);
    hipMemcpy(h.data(), (const char*)base + (size_t)first * per * elem, h.size(), hipMemcpyDeviceToHost);
    return h;
  };
  const bool p32 = c->setup_prec == LBDDC_MIXED;
  switch (which) {
    case LBDDC_X_K: {
      const bool use32 = c->k32_valid;
      const size_t per = (size_t)c->npair * 4;
      auto h = use32 ? fetch(c->d_K32, per, 4) : fetch(c->d_K, per, 8);
      for (int k = 0; k < count; ++k) {
        double* o = out + (size_t)k * 4 * nB * nB;
        for (int n1 = 0, P = 0; n1 < c->nN; ++n1)
          for (int n2 = 0; n2 <= n1; ++n2, ++P)
            for (int i1 = 0; i1 < 2; ++i1)
              for (int i2 = 0; i2 < 2; ++i2) {
                size_t src = ((size_t)k * c->npair + P) * 4 + 2 * i1 + i2;
                double v = use32 ? (double)((float*)h.data())[src] : ((double*)h.data())[src];
                int row = i1 * nB + c->perm_nat[n1], col = i2 * nB + c->perm_nat[n2];
                o[(size_t)row * 2 * nB + col] = v;
                o[(size_t)col * 2 * nB + row] = v;
              }
      }
      break;
    }
    case LBDDC_X_THETA: {
      auto h = fetch(c->d_theta, (size_t)c->ns * 4, 8);
      const double* src = (const double*)h.data();
      for (int k = 0; k < count; ++k)
        for (int i1 = 0; i1 < 2; ++i1)
          for (int j1 = 0; j1 < 2; ++j1)
            for (int i2 = 0; i2 < 2; ++i2)
              for (int j2 = 0; j2 < 2; ++j2)
                for (int k3 = 0; k3 < c->nL; ++k3) {
                  int s = (j1 * 2 + j2) * c->nL + k3;
                  out[(size_t)k * 16 * c->nL + ((((i1 * 2 + j1) * 2 + i2) * 2 + j2) * c->nL + k3)] =
                      src[((size_t)k * c->ns + s) * 4 + 2 * i1 + i2];
                }
      break;
    }
    case LBDDC_X_ITIL: {
      auto h = fetch(c->d_itil, (size_t)4 * c->KC, 8);
      memcpy(out, h.data(), h.size());
      break;
    }
    case LBDDC_X_S: {
      auto h = fetch(c->d_S, (size_t)nU * (nU + 1) / 2, 8);
      const double* src = (const double*)h.data();
      for (int k = 0; k < count; ++k)
        for (int i = 0; i < nU; ++i)
          for (int j = 0; j <= i; ++j) {
            double v = src[(size_t)k * nU * (nU + 1) / 2 + i * (i + 1) / 2 + j];
            out[(size_t)k * nU * nU + i * nU + j] = v;
            out[(size_t)k * nU * nU + j * nU + i] = v;
          }
      break;
    }
    case LBDDC_X_D: {
      auto h = fetch(c->d_D, nU, 8);
      memcpy(out, h.data(), h.size());
      break;
    }
    case LBDDC_X_PSI: {
      // stored [cell][nC][nU]; exported [cell][nU][nC]
      auto h = fetch(c->d_Psi, (size_t)nU * nC, p32 ? 4 : 8);
      for (size_t k = 0; k < (size_t)count; ++k)
        for (int i = 0; i < nU; ++i)
          for (int j = 0; j < nC; ++j) {
            const size_t src = (k * nC + j) * nU + i;
            out[(k * nU + i) * nC + j] = p32 ? (double)((float*)h.data())[src] : ((double*)h.data())[src];
          }
      break;
    }
    case LBDDC_X_SC: {
      auto h = fetch(c->d_ScLoc, (size_t)nC * (nC + 1) / 2, 8);
      const double* src = (const double*)h.data();
      for (int k = 0; k < count; ++k)
        for (int i = 0; i < nC; ++i)
          for (int j = 0; j <= i; ++j) {
            double v = src[(size_t)k * nC * (nC + 1) / 2 + i * (i + 1) / 2 + j];
            out[(size_t)k * nC * nC + i * nC + j] = v;
            out[(size_t)k * nC * nC + j * nC + i] = v;
          }
      break;
    }
    case LBDDC_X_LOAD: {
      for (int r = 0; r < c->nrhs; ++r) {
        std::vector<double> h((size_t)count * nU);
        hipMemcpy(h.data(), c->d_load + ((size_t)r * c->ncell + first) * nU, h.size() * 8, hipMemcpyDeviceToHost);
        for (int k = 0; k < count; ++k)
          memcpy(out + ((size_t)k * c->nrhs + r) * nU, h.data() + (size_t)k * nU, nU * 8);
      }
      break;
    }
    case LBDDC_X_FINE: {
      const size_t per = (size_t)nE * (nE + 1) / 2;
      auto h = fetch(c->d_P, per, p32 ? 4 : 8);
      for (int k = 0; k < count; ++k) {
        double* o = out + (size_t)k * nU * nU;
        for (int i = 0; i < nU * nU; ++i) o[i] = 0.0;
        for (int i = 0; i < nE; ++i)
          for (int j = 0; j <= i; ++j) {
            size_t src = (size_t)k * per + i * (i + 1) / 2 + j;
            double v = p32 ? (double)((float*)h.data())[src] : ((double*)h.data())[src];
            o[(size_t)(8 + i) * nU + 8 + j] = v;
            o[(size_t)(8 + j) * nU + 8 + i] = v;
          }
      }
      break;
    }
    case LBDDC_X_CONS: {
      auto h = fetch(c->d_cons, (size_t)4 * c->nce * (c->p + 1) * 2, 8);
      memcpy(out, h.data(), h.size());
      break;
    }
    case LBDDC_X_RU:
    case LBDDC_X_RC: {
      const std::vector<int>& R = which == LBDDC_X_RU ? c->RU : c->RC;
      const int w = which == LBDDC_X_RU ? nU : nC;
      for (size_t i = 0; i < (size_t)count * w; ++i) out[i] = (double)R[(size_t)first * w + i];
      break;
    }
    default:
      return fail(c, LBDDC_E_ARG, "export: unknown field");
  }
  return LBDDC_OK;
}

}  // extern "C"
