// Internal structures shared by the ABI layer and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "coeffs.hpp"
#include "physics.hpp"

namespace acat {

constexpr int BLOCK = 256;        // threads per block of every step kernel
constexpr int MAX_CLASSES = 16;   // order classes: P in 1D, P*P in 2D
constexpr int BATCH_PMAX = 4;     // largest half-width of a batched problem

// Problem geometry and parameters as the kernels see them.
struct KProb {
  int dim, nvar, flux, P, bc;
  int flags;          // FLAG_* variants
  int64_t nx, ny;
  int64_t nIx, nIy;   // x-interfaces per row, y-interfaces per column
  int64_t ioff;       // interface entry k <-> cell i = k + ioff (0 or -1)
  int64_t n1, n2;     // 2D corner grid extents: i1 in [ioff, nx), i2 in [ioff, ny)
  Phys ph;
  double dx, dy, eps, theta;
};

// Tiles of the classification and of the class lists.  1D: 256 consecutive
// interfaces.  2D: 16 x 16 corners, tiles numbered row by row; the class
// lists are therefore tile-major (row-major inside a tile), so a block
// walking a stretch of a list works on a compact patch of the grid whose
// stencil cells stay in cache.
constexpr int TILE_X = 16, TILE_Y = 16;
static_assert(TILE_X * TILE_Y == BLOCK, "one classification thread per item of a tile");
// List entries under the square-stencil variant: item | tag << LIST_TAG_SHIFT,
// tag 1 = store F only, 2 = store G only, 0 = both.
constexpr int LIST_TAG_SHIFT = 29;
inline int64_t class_tiles(const KProb& k) {
  if (k.dim == 2) return ((k.n1 + TILE_X - 1) / TILE_X) * ((k.n2 + TILE_Y - 1) / TILE_Y);
  return (k.nIx + BLOCK - 1) / BLOCK;
}

// Everything one step's kernels read and write.
struct KStep {
  const double* u;
  double* uout;
  double dt;
  const double* dt_dev;   // device time step (overrides dt when not null)
  int8_t* ordx;
  double* psix;
  double* alx;
  int8_t* ordy;
  double* psiy;
  double* aly;
  double* Fx;             // x-interface fluxes [nvar][ny][nIx] (1D: [nvar][nI])
  double* Gy;             // y-interface fluxes [nvar][nIy][nx]
  int8_t* cls;            // order class of every item: 1D p-1 per interface; 2D (q1-1)*P + (q2-1) per corner [n2][n1]
  int32_t* hist;          // per-tile class histograms of the classification kernel [tiles][MAX_CLASSES]
  int32_t* offs;          // per-class exclusive prefix of hist over tiles [MAX_CLASSES][tiles + 1]
  int32_t* counts;        // [MAX_CLASSES] items per order class
  int32_t* list;          // item ids grouped by class, tile order within a class [items]
  uint32_t* status;       // device status bits
  int replay;             // decisions given in ord/psi/al
  // CFL mode: the classification also reduces the cells' spectral radii into
  // per-block partial maxima `part`, from which one block computes the time
  // step into dt_out (and advances t_dev) before the flux kernels read it
  int cfl_mode;
  double cfl, t_final;
  double* t_dev;
  double* dt_out;
  double* part;           // [tiles][dim]
};

__device__ __forceinline__ double step_dt(const KStep& s) { return s.dt_dev ? *s.dt_dev : s.dt; }

// Kernel timer: when enabled, every launch of the library is bracketed by
// two HIP events on its own stream (not while the stream is being captured
// into a graph).  acat_profile_read() reports per-kernel totals.
struct ProfScope {
  int slot;
  hipStream_t stream;
  ProfScope(const char* name, hipStream_t s);
  ~ProfScope();
};

// Launchers (return the first HIP error).
hipError_t launch_step_1d(const KProb& pb, const KStep& st, int grid_blocks, hipStream_t stream);
hipError_t launch_step_2d(const KProb& pb, const KStep& st, int grid_blocks, hipStream_t stream);
hipError_t launch_max_speed(const KProb& pb, const double* u, double* smax, hipStream_t stream);
// classification (replay: recorded orders) and per-class item lists only
hipError_t launch_lists(const KProb& pb, const KStep& st, hipStream_t stream);
// adjoint of one step with the decisions and lists in st: ubi = ubo + (dF/du)^T Fbar;
// C is the per-item contribution buffer [nvar][items][LMAX] (LMAX = 2P in 1D, 4P^2 in 2D)
hipError_t launch_adjoint(const KProb& pb, const KStep& st, const double* ubo, double* ubi, double* C,
                          hipStream_t stream);
hipError_t launch_cfl_dt(const KProb& pb, const double* smax, double cfl, double t_final, double* t_dev,
                         double* dt_dev, hipStream_t stream);

struct KBatch {
  int nvar, flux, nprob, Pmax;
  Phys ph;
  double eps, theta;
  int64_t ncell, nif;       // total cells and interfaces
  const int64_t* coff;      // [nprob + 1] first cell of each problem
  const int64_t* ioffs;     // [nprob + 1] first interface of each problem
  const int32_t* N;         // [nprob] cells
  const int32_t* P;         // [nprob] largest half-width
  const int32_t* bc;        // [nprob] boundary
  const double* dx;         // [nprob]
  const int32_t* pif;       // [nif] problem of each interface
  const int32_t* pcell;     // [ncell] problem of each cell
  int waves[BATCH_PMAX + 1];    // per order class p: waves per block of the flux kernel (1, 2 or 4)
  int per_cu[BATCH_PMAX + 1];   // per order class p: persistent blocks per CU (0: occupancy limit)
  int fused_flux;               // every order class in one launch (k_flux_b_all) instead of one per class
};

struct KBStep {
  const double* u;
  double* uout;
  const double* dt;         // [nprob]
  int8_t* ord;
  double* psi;
  double* al;
  double* F;                // [nvar][nif]
  int32_t* hist;
  int32_t* offs;
  int32_t* counts;
  int32_t* list;
  uint32_t* status;
  // with smax set: the update also reduces the spectral radius of the new
  // state, one maximum per wave that lies whole inside one problem into
  // wmax[wave] and the rest into smax[problem] (bit patterns of non-negative
  // doubles, atomic maxima; zero on entry); a last kernel folds both into
  // the next time steps dt_next[b] = cfl dx[b] / max and clears smax
  unsigned long long* smax;
  double* wmax;             // [ceil(ncell / 64)]
  double* dt_next;
  double cfl;
};

hipError_t launch_step_batched(const KBatch& bt, const KBStep& st, hipStream_t stream);
hipError_t launch_cfl_batched(const KBatch& bt, const double* u, double cfl, unsigned long long* smax, double* dt,
                              hipStream_t stream);

}  // namespace acat
