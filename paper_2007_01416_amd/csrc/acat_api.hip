// C ABI of the ACAT library: argument checks, workspace layout, launches.
#include <hip/hip_runtime.h>

#include <atomic>
#include <cstring>
#include <vector>

#include "../../include/acat.h"
#include "acat_internal.hpp"

namespace acat {
void copy_tables(int p, double* g1, double* gt, double* eta, double* tau);

namespace {

constexpr size_t ALIGN = 256;
inline size_t align_up(size_t x) { return (x + ALIGN - 1) / ALIGN * ALIGN; }

acat_status check_problem(const acat_problem* pb) {
  if (!pb) return ACAT_ERR_NULL;
  if (pb->dim != 1 && pb->dim != 2) return ACAT_ERR_ARG;
  if (pb->flags & ~(ACAT_FLAG_FLO_LF | ACAT_FLAG_FLO_HLL | ACAT_FLAG_PSI2_MODIFIED | ACAT_FLAG_PSI1_ROE |
                    ACAT_FLAG_SQUARE_2D))
    return ACAT_ERR_ARG;
  if ((pb->flags & ACAT_FLAG_SQUARE_2D) && pb->dim != 2) return ACAT_ERR_ARG;
  if ((pb->flags & ACAT_FLAG_FLO_LF) && (pb->flags & ACAT_FLAG_FLO_HLL)) return ACAT_ERR_ARG;
  if ((pb->flags & ACAT_FLAG_PSI1_ROE) && pb->flux == ACAT_FLUX_EULER) return ACAT_ERR_UNSUPPORTED;
  if (pb->bc != ACAT_BC_PERIODIC && pb->bc != ACAT_BC_TRANSMISSIVE) return ACAT_ERR_ARG;
  if (pb->flux < ACAT_FLUX_ADVECTION || pb->flux > ACAT_FLUX_EULER) return ACAT_ERR_ARG;
  if (pb->P < 1 || pb->P > PMAX) return ACAT_ERR_ARG;
  const int64_t G = pb->P > 2 ? pb->P : 2;
  if (pb->nx < 2 * G || pb->nx > (int64_t)1 << 31) return ACAT_ERR_ARG;
  if (pb->dim == 2 && (pb->ny < 2 * G || pb->ny > (int64_t)1 << 31)) return ACAT_ERR_ARG;
  if (!(pb->dx > 0.0) || (pb->dim == 2 && !(pb->dy > 0.0))) return ACAT_ERR_ARG;
  if (!(pb->eps >= 0.0) || !(pb->theta > 0.0 && pb->theta <= 1.0)) return ACAT_ERR_ARG;
  if (pb->flux == ACAT_FLUX_EULER && pb->nvar != (pb->dim == 1 ? 3 : 4)) return ACAT_ERR_ARG;
  if (pb->flux == ACAT_FLUX_EULER && !(pb->gamma > 1.0)) return ACAT_ERR_ARG;
  if (pb->flux == ACAT_FLUX_BURGERS && (pb->nvar != 1 || pb->dim != 1)) return ACAT_ERR_ARG;
  if (pb->flux == ACAT_FLUX_ADVECTION && pb->nvar < 1) return ACAT_ERR_ARG;
  // valid problems without kernels
  if (pb->flux == ACAT_FLUX_ADVECTION && pb->nvar != 1) return ACAT_ERR_UNSUPPORTED;
  if (pb->dim == 2 && pb->P > PMAX_2D) return ACAT_ERR_UNSUPPORTED;
  const int64_t cells = pb->nx * (pb->dim == 2 ? pb->ny : 1);
  const int64_t items = (pb->dim == 2) ? (pb->nx + 1) * (pb->ny + 1) : pb->nx + 1;
  if (cells * pb->nvar >= ((int64_t)1 << 40) || items >= ((int64_t)1 << 31) - 1) return ACAT_ERR_UNSUPPORTED;
  // the square-stencil variant tags list entries in bits 29 and 30
  if ((pb->flags & ACAT_FLAG_SQUARE_2D) && items >= ((int64_t)1 << LIST_TAG_SHIFT)) return ACAT_ERR_UNSUPPORTED;
  return ACAT_OK;
}

KProb make_kprob(const acat_problem* p) {
  KProb k{};
  k.dim = p->dim;
  k.nvar = p->nvar;
  k.flux = p->flux;
  k.P = p->P;
  k.bc = p->bc;
  k.flags = p->flags;
  k.nx = p->nx;
  k.ny = p->dim == 2 ? p->ny : 1;
  const int64_t ext = p->bc == ACAT_BC_PERIODIC ? 0 : 1;
  k.nIx = k.nx + ext;
  k.nIy = p->dim == 2 ? k.ny + ext : 0;
  k.ioff = -ext;
  k.n1 = k.nx + ext;
  k.n2 = p->dim == 2 ? k.ny + ext : 1;
  k.ph.gamma = p->gamma;
  k.ph.gm1 = p->gamma - 1.0;
  k.ph.ax = p->ax;
  k.ph.ay = p->ay;
  k.dx = p->dx;
  k.dy = p->dim == 2 ? p->dy : 1.0;
  k.eps = p->eps;
  k.theta = p->theta;
  return k;
}

// Workspace layout (each part 256-byte aligned):
//   counts  int32[MAX_CLASSES] + status uint32 (one 256-byte header)
//   ordx, ordy    int8 decision maps     (used when the caller records none)
//   psix, psiy    double
//   alx, aly      double
//   Fx, Gy        double interface fluxes
//   cls           int8 order class of every item (1D interface, 2D corner)
//   hist          int32[tiles][MAX_CLASSES]
//   offs          int32[MAX_CLASSES][tiles + 1]
//   list          int32[items]
//   part          double[tiles][dim] partial wave-speed maxima (acat_step_cfl)
struct Layout {
  size_t hdr, ordx, ordy, psix, psiy, alx, aly, Fx, Gy, cls, hist, offs, list, part, total;
  int64_t nItems;
};

Layout layout(const KProb& k) {
  Layout L{};
  const int64_t nx_if = k.ny * k.nIx;             // 1D: nI
  const int64_t ny_if = k.dim == 2 ? k.nIy * k.nx : 0;
  L.nItems = k.dim == 2 ? k.n1 * k.n2 : k.nIx;
  const int64_t cblocks = class_tiles(k);
  size_t o = 0;
  L.hdr = o;   o += align_up(sizeof(int32_t) * MAX_CLASSES + sizeof(uint32_t) * 4);
  L.ordx = o;  o += align_up((size_t)nx_if);
  L.ordy = o;  o += align_up((size_t)ny_if);
  L.psix = o;  o += align_up(sizeof(double) * nx_if);
  L.psiy = o;  o += align_up(sizeof(double) * ny_if);
  L.alx = o;   o += align_up(sizeof(double) * nx_if);
  L.aly = o;   o += align_up(sizeof(double) * ny_if);
  L.Fx = o;    o += align_up(sizeof(double) * k.nvar * nx_if);
  L.Gy = o;    o += align_up(sizeof(double) * k.nvar * ny_if);
  L.cls = o;   o += align_up((size_t)L.nItems);
  L.hist = o;  o += align_up(sizeof(int32_t) * MAX_CLASSES * (size_t)cblocks);
  L.offs = o;  o += align_up(sizeof(int32_t) * MAX_CLASSES * (size_t)(cblocks + 1));
  // a corner with q1 != q2 has two entries under the square-stencil variant
  L.list = o;  o += align_up(sizeof(int32_t) * (size_t)L.nItems * ((k.flags & FLAG_SQUARE_2D) ? 2 : 1));
  L.part = o;  o += align_up(sizeof(double) * 2 * (size_t)cblocks);
  L.total = o;
  return L;
}

// Device status word: one per device, in the library's own static memory.
__device__ uint32_t g_status;

uint32_t* status_ptr() {
  static uint32_t* ptrs[64] = {};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return nullptr;
  if (!ptrs[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(g_status)) != hipSuccess) return nullptr;
    ptrs[dev] = static_cast<uint32_t*>(p);
  }
  return ptrs[dev];
}

// Workspace of acat_step_noalloc: one fixed array per device, in the
// library's own static memory, held until the process ends.  Host code uses
// the device address obtained from the runtime, never the array's name.
__device__ __align__(256) unsigned char scratch[ACAT_NOALLOC_SCRATCH_BYTES];

void* noalloc_scratch_ptr() {
  static std::atomic<void*> ptrs[64] = {};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return nullptr;
  void* p = ptrs[dev].load(std::memory_order_acquire);
  if (!p) {
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return nullptr;
    ptrs[dev].store(p, std::memory_order_release);
  }
  return p;
}

bool overlaps(const void* a, const void* b, size_t n) {
  const char* x = static_cast<const char*>(a);
  const char* y = static_cast<const char*>(b);
  return x < y + n && y < x + n;
}

struct CflArgs {
  double cfl, t_final;
  double* t_dev;
  double* dt_out;
};

acat_status do_step(const acat_problem* prob, const double* u_in, double* u_out, double dt, const double* dt_dev,
                    void* ws, size_t ws_bytes, const acat_decisions* dec, bool replay, void* stream,
                    const CflArgs* cfl = nullptr) {
  acat_status rc = check_problem(prob);
  if (rc != ACAT_OK) return rc;
  if (!u_in || !u_out) return ACAT_ERR_NULL;
  if (cfl) {
    if (!cfl->dt_out) return ACAT_ERR_NULL;
    if (!(cfl->cfl > 0.0)) return ACAT_ERR_ARG;
  } else if (!dt_dev && !(dt >= 0.0)) {
    return ACAT_ERR_ARG;
  }
  const KProb k = make_kprob(prob);
  const size_t state_bytes = sizeof(double) * (size_t)k.nvar * k.nx * k.ny;
  if (overlaps(u_in, u_out, state_bytes)) return ACAT_ERR_ALIAS;
  const Layout L = layout(k);
  if (!ws || ws_bytes < L.total) return ACAT_ERR_WORKSPACE;
  if (replay) {
    if (!dec || !dec->order_x || !dec->psi1_x || !dec->alpha_x) return ACAT_ERR_NULL;
    if (k.dim == 2 && (!dec->order_y || !dec->psi1_y || !dec->alpha_y)) return ACAT_ERR_NULL;
  }
  char* w = static_cast<char*>(ws);
  KStep st{};
  st.u = u_in;
  st.uout = u_out;
  st.dt = dt;
  st.dt_dev = dt_dev;
  st.ordx = (dec && dec->order_x) ? dec->order_x : reinterpret_cast<int8_t*>(w + L.ordx);
  st.psix = (dec && dec->psi1_x) ? dec->psi1_x : reinterpret_cast<double*>(w + L.psix);
  st.alx = (dec && dec->alpha_x) ? dec->alpha_x : reinterpret_cast<double*>(w + L.alx);
  st.ordy = (dec && dec->order_y) ? dec->order_y : reinterpret_cast<int8_t*>(w + L.ordy);
  st.psiy = (dec && dec->psi1_y) ? dec->psi1_y : reinterpret_cast<double*>(w + L.psiy);
  st.aly = (dec && dec->alpha_y) ? dec->alpha_y : reinterpret_cast<double*>(w + L.aly);
  st.Fx = reinterpret_cast<double*>(w + L.Fx);
  st.Gy = reinterpret_cast<double*>(w + L.Gy);
  st.counts = reinterpret_cast<int32_t*>(w + L.hdr);
  st.cls = reinterpret_cast<int8_t*>(w + L.cls);
  st.hist = reinterpret_cast<int32_t*>(w + L.hist);
  st.offs = reinterpret_cast<int32_t*>(w + L.offs);
  st.list = reinterpret_cast<int32_t*>(w + L.list);
  st.status = status_ptr();
  if (!st.status) return ACAT_ERR_DEVICE;
  st.replay = replay ? 1 : 0;
  if (cfl) {
    st.cfl_mode = 1;
    st.cfl = cfl->cfl;
    st.t_final = cfl->t_final;
    st.t_dev = cfl->t_dev;
    st.dt_out = cfl->dt_out;
    st.dt_dev = cfl->dt_out;   // the flux and update kernels read the time step computed in the step
    st.part = reinterpret_cast<double*>(w + L.part);
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = k.dim == 1 ? launch_step_1d(k, st, 0, s) : launch_step_2d(k, st, 0, s);
  return e == hipSuccess ? ACAT_OK : ACAT_ERR_DEVICE;
}

// Adjoint workspace: header, class map, tile histograms, prefix, item lists
// and the per-item contribution buffer C[nvar][items][LMAX].
struct ALayout {
  size_t hdr, cls, hist, offs, list, C, total;
  int64_t nItems;
  int lmax;
};

ALayout alayout(const KProb& k) {
  ALayout L{};
  L.nItems = k.dim == 2 ? k.n1 * k.n2 : k.nIx;
  L.lmax = k.dim == 2 ? 4 * k.P * k.P : 2 * k.P;
  const int64_t cblocks = class_tiles(k);
  size_t o = 0;
  L.hdr = o;   o += align_up(sizeof(int32_t) * MAX_CLASSES + sizeof(uint32_t) * 4);
  L.cls = o;   o += align_up((size_t)L.nItems);
  L.hist = o;  o += align_up(sizeof(int32_t) * MAX_CLASSES * (size_t)cblocks);
  L.offs = o;  o += align_up(sizeof(int32_t) * MAX_CLASSES * (size_t)(cblocks + 1));
  L.list = o;  o += align_up(sizeof(int32_t) * (size_t)L.nItems);
  L.C = o;     o += align_up(sizeof(double) * (size_t)k.nvar * (size_t)L.nItems * (size_t)L.lmax);
  L.total = o;
  return L;
}

acat_status check_adjoint(const acat_problem* prob) {
  acat_status rc = check_problem(prob);
  if (rc != ACAT_OK) return rc;
  if (prob->flags & (ACAT_FLAG_FLO_HLL | ACAT_FLAG_SQUARE_2D)) return ACAT_ERR_UNSUPPORTED;
  return ACAT_OK;
}

// ------------------------------------------------------------------ batch
acat_status check_batch(const acat_batch* bt) {
  if (!bt) return ACAT_ERR_NULL;
  if (bt->nprob < 1) return ACAT_ERR_ARG;
  if (!bt->n || !bt->P || !bt->bc || !bt->dx) return ACAT_ERR_NULL;
  if (bt->flux < ACAT_FLUX_ADVECTION || bt->flux > ACAT_FLUX_EULER) return ACAT_ERR_ARG;
  if (bt->flux == ACAT_FLUX_EULER && (bt->nvar != 3 || !(bt->gamma > 1.0))) return ACAT_ERR_ARG;
  if (bt->flux != ACAT_FLUX_EULER && bt->nvar != 1) return bt->nvar < 1 ? ACAT_ERR_ARG : ACAT_ERR_UNSUPPORTED;
  if (!(bt->eps >= 0.0) || !(bt->theta > 0.0 && bt->theta <= 1.0)) return ACAT_ERR_ARG;
  if (bt->launch) {
    for (int p = 0; p < BATCH_PMAX; ++p) {
      const int w = bt->launch[2 * p], c = bt->launch[2 * p + 1];
      if (!(w == 0 || w == 1 || w == 2 || w == 4) || c < 0 || c > 32) return ACAT_ERR_ARG;
    }
  }
  int64_t cells = 0, ifs = 0;
  for (int b = 0; b < bt->nprob; ++b) {
    const int P = bt->P[b];
    if (P < 1 || P > 4) return ACAT_ERR_ARG;
    const int64_t G = P > 2 ? P : 2;
    if (bt->n[b] < 8 || bt->n[b] < 2 * G) return ACAT_ERR_ARG;
    if (bt->bc[b] != ACAT_BC_PERIODIC && bt->bc[b] != ACAT_BC_TRANSMISSIVE) return ACAT_ERR_ARG;
    if (!(bt->dx[b] > 0.0)) return ACAT_ERR_ARG;
    cells += bt->n[b];
    ifs += bt->n[b] + (bt->bc[b] == ACAT_BC_PERIODIC ? 0 : 1);
    if (ifs >= ((int64_t)1 << 31) - 1) return ACAT_ERR_UNSUPPORTED;
  }
  return ACAT_OK;
}

struct BLayout {
  size_t hdr, coff, ioffs, N, P, bc, dx, pif, pcell, smax, ord, psi, al, wmax, F, hist, offs, list, total;
  int64_t ncell, nif;
  int Pmax;
};

BLayout blayout(const acat_batch* bt) {
  BLayout L{};
  const int np = bt->nprob;
  L.Pmax = 1;
  for (int b = 0; b < np; ++b) {
    L.ncell += bt->n[b];
    L.nif += bt->n[b] + (bt->bc[b] == ACAT_BC_PERIODIC ? 0 : 1);
    if (bt->P[b] > L.Pmax) L.Pmax = bt->P[b];
  }
  const int64_t tiles = (L.nif + BLOCK - 1) / BLOCK;
  size_t o = 0;
  L.hdr = o;   o += align_up(sizeof(int32_t) * MAX_CLASSES);
  L.coff = o;  o += align_up(sizeof(int64_t) * (np + 1));
  L.ioffs = o; o += align_up(sizeof(int64_t) * (np + 1));
  L.N = o;     o += align_up(sizeof(int32_t) * np);
  L.P = o;     o += align_up(sizeof(int32_t) * np);
  L.bc = o;    o += align_up(sizeof(int32_t) * np);
  L.dx = o;    o += align_up(sizeof(double) * np);
  L.pif = o;   o += align_up(sizeof(int32_t) * L.nif);
  L.pcell = o; o += align_up(sizeof(int32_t) * L.ncell);
  L.smax = o;  o += align_up(sizeof(double) * np);
  L.ord = o;   o += align_up((size_t)L.nif);
  L.psi = o;   o += align_up(sizeof(double) * L.nif);
  L.al = o;    o += align_up(sizeof(double) * L.nif);
  L.wmax = o;  o += align_up(sizeof(double) * ((L.ncell + 63) / 64));
  L.F = o;     o += align_up(sizeof(double) * bt->nvar * L.nif);
  L.hist = o;  o += align_up(sizeof(int32_t) * MAX_CLASSES * tiles);
  L.offs = o;  o += align_up(sizeof(int32_t) * MAX_CLASSES * (tiles + 1));
  L.list = o;  o += align_up(sizeof(int32_t) * L.nif);
  L.total = o;
  return L;
}

KBatch make_kbatch(const acat_batch* bt, const BLayout& L, char* w) {
  KBatch k{};
  k.nvar = bt->nvar;
  k.flux = bt->flux;
  k.nprob = bt->nprob;
  k.Pmax = L.Pmax;
  k.ph.gamma = bt->gamma;
  k.ph.gm1 = bt->gamma - 1.0;
  k.ph.ax = bt->ax;
  k.ph.ay = 0.0;
  k.eps = bt->eps;
  k.theta = bt->theta;
  k.ncell = L.ncell;
  k.nif = L.nif;
  k.coff = reinterpret_cast<const int64_t*>(w + L.coff);
  k.ioffs = reinterpret_cast<const int64_t*>(w + L.ioffs);
  k.N = reinterpret_cast<const int32_t*>(w + L.N);
  k.P = reinterpret_cast<const int32_t*>(w + L.P);
  k.bc = reinterpret_cast<const int32_t*>(w + L.bc);
  k.dx = reinterpret_cast<const double*>(w + L.dx);
  k.pif = reinterpret_cast<const int32_t*>(w + L.pif);
  k.pcell = reinterpret_cast<const int32_t*>(w + L.pcell);
  for (int p = 1; p <= BATCH_PMAX; ++p) {
    k.waves[p] = bt->launch && bt->launch[2 * (p - 1)] > 0 ? bt->launch[2 * (p - 1)] : 4;
    k.per_cu[p] = bt->launch ? bt->launch[2 * (p - 1) + 1] : 0;
  }
  k.fused_flux = bt->launch ? 0 : 1;
  k.waves[0] = 4;
  k.per_cu[0] = 0;
  return k;
}

}  // namespace
}  // namespace acat

using namespace acat;

extern "C" {

acat_status acat_workspace_size(const acat_problem* prob, size_t* bytes) {
  acat_status rc = check_problem(prob);
  if (rc != ACAT_OK) return rc;
  if (!bytes) return ACAT_ERR_NULL;
  *bytes = layout(make_kprob(prob)).total;
  return ACAT_OK;
}

acat_status acat_step(const acat_problem* prob, const double* u_in, double* u_out, double dt,
                      const double* dt_dev, void* workspace, size_t workspace_bytes, const acat_decisions* dec,
                      void* stream) {
  return do_step(prob, u_in, u_out, dt, dt_dev, workspace, workspace_bytes, dec, false, stream);
}

acat_status acat_step_noalloc(const acat_problem* prob, const double* u_in, double* u_out, double dt,
                              const double* dt_dev, const acat_decisions* dec, void* stream) {
  acat_status rc = check_problem(prob);
  if (rc != ACAT_OK) return rc;
  if (layout(make_kprob(prob)).total > ACAT_NOALLOC_SCRATCH_BYTES) return ACAT_ERR_WORKSPACE;
  void* ws = noalloc_scratch_ptr();
  if (!ws) return ACAT_ERR_DEVICE;
  return do_step(prob, u_in, u_out, dt, dt_dev, ws, ACAT_NOALLOC_SCRATCH_BYTES, dec, false, stream);
}

acat_status acat_step_cfl(const acat_problem* prob, const double* u_in, double* u_out, double cfl, double t_final,
                          double* t_dev, double* dt_dev, void* workspace, size_t workspace_bytes,
                          const acat_decisions* dec, void* stream) {
  CflArgs c{cfl, t_final, t_dev, dt_dev};
  return do_step(prob, u_in, u_out, 0.0, nullptr, workspace, workspace_bytes, dec, false, stream, &c);
}

acat_status acat_step_replay(const acat_problem* prob, const double* u_in, double* u_out, double dt,
                             const double* dt_dev, void* workspace, size_t workspace_bytes,
                             const acat_decisions* dec, void* stream) {
  return do_step(prob, u_in, u_out, dt, dt_dev, workspace, workspace_bytes, dec, true, stream);
}

acat_status acat_adjoint_workspace_size(const acat_problem* prob, size_t* bytes) {
  acat_status rc = check_adjoint(prob);
  if (rc != ACAT_OK) return rc;
  if (!bytes) return ACAT_ERR_NULL;
  *bytes = alayout(make_kprob(prob)).total;
  return ACAT_OK;
}

// lists_ws: the workspace of the forward step whose class lists the adjoint
// reuses (acat_step_adjoint_lists), or NULL to build them here
acat_status do_adjoint(const acat_problem* prob, const double* u_in, double dt, const double* dt_dev,
                       const acat_decisions* dec, const double* ubar_out, double* ubar_in, void* workspace,
                       size_t workspace_bytes, const void* lists_ws, size_t lists_ws_bytes, void* stream) {
  acat_status rc = check_adjoint(prob);
  if (rc != ACAT_OK) return rc;
  if (!u_in || !ubar_out || !ubar_in || !dec) return ACAT_ERR_NULL;
  if (!dec->order_x || !dec->psi1_x || !dec->alpha_x) return ACAT_ERR_NULL;
  if (prob->dim == 2 && (!dec->order_y || !dec->psi1_y || !dec->alpha_y)) return ACAT_ERR_NULL;
  if (!dt_dev && !(dt >= 0.0)) return ACAT_ERR_ARG;
  const KProb k = make_kprob(prob);
  const size_t state_bytes = sizeof(double) * (size_t)k.nvar * k.nx * k.ny;
  if (overlaps(u_in, ubar_in, state_bytes)) return ACAT_ERR_ALIAS;
  if (ubar_in != ubar_out && overlaps(ubar_in, ubar_out, state_bytes)) return ACAT_ERR_ALIAS;
  const ALayout L = alayout(k);
  if (!workspace || workspace_bytes < L.total) return ACAT_ERR_WORKSPACE;
  char* w = static_cast<char*>(workspace);
  KStep st{};
  st.u = u_in;
  st.dt = dt;
  st.dt_dev = dt_dev;
  st.ordx = dec->order_x;
  st.psix = dec->psi1_x;
  st.alx = dec->alpha_x;
  st.ordy = dec->order_y;
  st.psiy = dec->psi1_y;
  st.aly = dec->alpha_y;
  st.counts = reinterpret_cast<int32_t*>(w + L.hdr);
  st.cls = reinterpret_cast<int8_t*>(w + L.cls);
  st.hist = reinterpret_cast<int32_t*>(w + L.hist);
  st.offs = reinterpret_cast<int32_t*>(w + L.offs);
  st.list = reinterpret_cast<int32_t*>(w + L.list);
  if (lists_ws) {
    // the forward step's class map, per-class counts and lists
    const Layout F = layout(k);
    if (lists_ws_bytes < F.total) return ACAT_ERR_WORKSPACE;
    char* fw = const_cast<char*>(static_cast<const char*>(lists_ws));
    st.counts = reinterpret_cast<int32_t*>(fw + F.hdr);
    st.cls = reinterpret_cast<int8_t*>(fw + F.cls);
    st.list = reinterpret_cast<int32_t*>(fw + F.list);
  }
  st.status = status_ptr();
  if (!st.status) return ACAT_ERR_DEVICE;
  st.replay = 1;
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = lists_ws ? hipSuccess : launch_lists(k, st, s);
  if (e == hipSuccess) e = launch_adjoint(k, st, ubar_out, ubar_in, reinterpret_cast<double*>(w + L.C), s);
  return e == hipSuccess ? ACAT_OK : ACAT_ERR_DEVICE;
}

acat_status acat_step_adjoint(const acat_problem* prob, const double* u_in, double dt, const double* dt_dev,
                              const acat_decisions* dec, const double* ubar_out, double* ubar_in, void* workspace,
                              size_t workspace_bytes, void* stream) {
  return do_adjoint(prob, u_in, dt, dt_dev, dec, ubar_out, ubar_in, workspace, workspace_bytes, nullptr, 0,
                    stream);
}

acat_status acat_step_adjoint_lists(const acat_problem* prob, const double* u_in, double dt, const double* dt_dev,
                                    const acat_decisions* dec, const double* ubar_out, double* ubar_in,
                                    const void* step_workspace, size_t step_workspace_bytes, void* workspace,
                                    size_t workspace_bytes, void* stream) {
  if (!step_workspace) return ACAT_ERR_NULL;
  return do_adjoint(prob, u_in, dt, dt_dev, dec, ubar_out, ubar_in, workspace, workspace_bytes, step_workspace,
                    step_workspace_bytes, stream);
}

acat_status acat_max_wave_speed(const acat_problem* prob, const double* u, double* smax_dev, void* stream) {
  acat_status rc = check_problem(prob);
  if (rc != ACAT_OK) return rc;
  if (!u || !smax_dev) return ACAT_ERR_NULL;
  hipError_t e = launch_max_speed(make_kprob(prob), u, smax_dev, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? ACAT_OK : ACAT_ERR_DEVICE;
}

acat_status acat_cfl_dt(const acat_problem* prob, const double* smax_dev, double cfl, double t_final,
                        double* t_dev, double* dt_dev, void* stream) {
  acat_status rc = check_problem(prob);
  if (rc != ACAT_OK) return rc;
  if (!smax_dev || !dt_dev) return ACAT_ERR_NULL;
  if (!(cfl > 0.0)) return ACAT_ERR_ARG;
  hipError_t e = launch_cfl_dt(make_kprob(prob), smax_dev, cfl, t_final, t_dev, dt_dev,
                               static_cast<hipStream_t>(stream));
  return e == hipSuccess ? ACAT_OK : ACAT_ERR_DEVICE;
}

acat_status acat_batch_workspace_size(const acat_batch* batch, size_t* bytes) {
  acat_status rc = check_batch(batch);
  if (rc != ACAT_OK) return rc;
  if (!bytes) return ACAT_ERR_NULL;
  *bytes = blayout(batch).total;
  return ACAT_OK;
}

acat_status acat_batch_init(const acat_batch* batch, void* workspace, size_t workspace_bytes) {
  acat_status rc = check_batch(batch);
  if (rc != ACAT_OK) return rc;
  const BLayout L = blayout(batch);
  if (!workspace || workspace_bytes < L.total) return ACAT_ERR_WORKSPACE;
  const int np = batch->nprob;
  std::vector<char> host(L.ord - L.coff, 0);   // the static tables, and smax cleared
  auto put = [&](size_t off, const void* src, size_t n) { std::memcpy(host.data() + (off - L.coff), src, n); };
  std::vector<int64_t> coff(np + 1, 0), ioffs(np + 1, 0);
  std::vector<int32_t> N(np), P(np), bc(np);
  for (int b = 0; b < np; ++b) {
    coff[b + 1] = coff[b] + batch->n[b];
    ioffs[b + 1] = ioffs[b] + batch->n[b] + (batch->bc[b] == ACAT_BC_PERIODIC ? 0 : 1);
    N[b] = (int32_t)batch->n[b];
    P[b] = batch->P[b];
    bc[b] = batch->bc[b];
  }
  put(L.coff, coff.data(), sizeof(int64_t) * (np + 1));
  put(L.ioffs, ioffs.data(), sizeof(int64_t) * (np + 1));
  put(L.N, N.data(), sizeof(int32_t) * np);
  put(L.P, P.data(), sizeof(int32_t) * np);
  put(L.bc, bc.data(), sizeof(int32_t) * np);
  put(L.dx, batch->dx, sizeof(double) * np);
  // problem of every interface and of every cell (the layout is fixed for the batch)
  int32_t* pif = reinterpret_cast<int32_t*>(host.data() + (L.pif - L.coff));
  int32_t* pcell = reinterpret_cast<int32_t*>(host.data() + (L.pcell - L.coff));
  for (int b = 0; b < np; ++b) {
    for (int64_t k = ioffs[b]; k < ioffs[b + 1]; ++k) pif[k] = b;
    for (int64_t e = coff[b]; e < coff[b + 1]; ++e) pcell[e] = b;
  }
  char* w = static_cast<char*>(workspace);
  if (hipMemcpy(w + L.coff, host.data(), host.size(), hipMemcpyHostToDevice) != hipSuccess) return ACAT_ERR_DEVICE;
  return ACAT_OK;
}

namespace acat {
namespace {
acat_status step_batched(const acat_batch* batch, const double* u_in, double* u_out, double* dt_dev, double cfl,
                         bool fused_cfl, void* workspace, size_t workspace_bytes, void* stream) {
  acat_status rc = check_batch(batch);
  if (rc != ACAT_OK) return rc;
  if (!u_in || !u_out || !dt_dev) return ACAT_ERR_NULL;
  if (fused_cfl && !(cfl > 0.0)) return ACAT_ERR_ARG;
  const BLayout L = blayout(batch);
  if (!workspace || workspace_bytes < L.total) return ACAT_ERR_WORKSPACE;
  if (overlaps(u_in, u_out, sizeof(double) * batch->nvar * (size_t)L.ncell)) return ACAT_ERR_ALIAS;
  char* w = static_cast<char*>(workspace);
  const KBatch bt = make_kbatch(batch, L, w);
  KBStep st{};
  st.u = u_in;
  st.uout = u_out;
  st.dt = dt_dev;
  st.ord = reinterpret_cast<int8_t*>(w + L.ord);
  st.psi = reinterpret_cast<double*>(w + L.psi);
  st.al = reinterpret_cast<double*>(w + L.al);
  st.F = reinterpret_cast<double*>(w + L.F);
  st.hist = reinterpret_cast<int32_t*>(w + L.hist);
  st.offs = reinterpret_cast<int32_t*>(w + L.offs);
  st.counts = reinterpret_cast<int32_t*>(w + L.hdr);
  st.list = reinterpret_cast<int32_t*>(w + L.list);
  st.status = status_ptr();
  if (!st.status) return ACAT_ERR_DEVICE;
  if (fused_cfl) {
    st.smax = reinterpret_cast<unsigned long long*>(w + L.smax);
    st.wmax = reinterpret_cast<double*>(w + L.wmax);
    st.dt_next = dt_dev;
    st.cfl = cfl;
  }
  hipError_t e = launch_step_batched(bt, st, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? ACAT_OK : ACAT_ERR_DEVICE;
}
}  // namespace
}  // namespace acat

acat_status acat_step_batched(const acat_batch* batch, const double* u_in, double* u_out, const double* dt_dev,
                              void* workspace, size_t workspace_bytes, void* stream) {
  return step_batched(batch, u_in, u_out, const_cast<double*>(dt_dev), 0.0, false, workspace, workspace_bytes,
                      stream);
}

acat_status acat_step_batched_cfl(const acat_batch* batch, const double* u_in, double* u_out, double* dt_dev,
                                  double cfl, void* workspace, size_t workspace_bytes, void* stream) {
  return step_batched(batch, u_in, u_out, dt_dev, cfl, true, workspace, workspace_bytes, stream);
}

acat_status acat_batched_cfl_dt(const acat_batch* batch, const double* u, double cfl, double* dt_dev,
                                void* workspace, size_t workspace_bytes, void* stream) {
  acat_status rc = check_batch(batch);
  if (rc != ACAT_OK) return rc;
  if (!u || !dt_dev) return ACAT_ERR_NULL;
  if (!(cfl > 0.0)) return ACAT_ERR_ARG;
  const BLayout L = blayout(batch);
  if (!workspace || workspace_bytes < L.total) return ACAT_ERR_WORKSPACE;
  char* w = static_cast<char*>(workspace);
  const KBatch bt = make_kbatch(batch, L, w);
  hipError_t e = launch_cfl_batched(bt, u, cfl, reinterpret_cast<unsigned long long*>(w + L.smax), dt_dev,
                                    static_cast<hipStream_t>(stream));
  return e == hipSuccess ? ACAT_OK : ACAT_ERR_DEVICE;
}

acat_status acat_device_status(int32_t* flags_host, void* stream) {
  if (!flags_host) return ACAT_ERR_NULL;
  uint32_t* p = status_ptr();
  if (!p) return ACAT_ERR_DEVICE;
  hipStream_t s = static_cast<hipStream_t>(stream);
  uint32_t v = 0;
  if (hipMemcpyAsync(&v, p, sizeof(v), hipMemcpyDeviceToHost, s) != hipSuccess) return ACAT_ERR_DEVICE;
  if (hipStreamSynchronize(s) != hipSuccess) return ACAT_ERR_DEVICE;
  const uint32_t zero = 0;
  if (hipMemcpyAsync(p, &zero, sizeof(zero), hipMemcpyHostToDevice, s) != hipSuccess) return ACAT_ERR_DEVICE;
  if (hipStreamSynchronize(s) != hipSuccess) return ACAT_ERR_DEVICE;
  *flags_host = (int32_t)v;
  return ACAT_OK;
}

const char* acat_status_string(acat_status s) {
  switch (s) {
    case ACAT_OK: return "ok";
    case ACAT_ERR_NULL: return "required pointer is NULL";
    case ACAT_ERR_ARG: return "invalid argument";
    case ACAT_ERR_ALIAS: return "input and output states overlap";
    case ACAT_ERR_UNSUPPORTED: return "problem not supported by the GPU kernels";
    case ACAT_ERR_DEVICE: return "HIP runtime error";
    case ACAT_ERR_WORKSPACE: return "workspace missing or too small";
  }
  return "unknown status";
}

acat_status acat_coefficients(int32_t p, double* g1, double* gt, double* eta, double* tau) {
  if (p < 1 || p > PMAX) return ACAT_ERR_ARG;
  copy_tables(p, g1, gt, eta, tau);
  return ACAT_OK;
}

}  // extern "C"
