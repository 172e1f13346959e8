// Host run of the library's 2D adjoint kernel templates (the kernels of
// acat_adjoint.hip, compiled for the CPU with the host execution model in
// hip/hip_runtime.h), for sanitizer builds: chosen corner classes of P = 4,
// each in its one-kernel form (PASSES = 3) and split into two launches
// (PASSES = 1 then 2), on a 10 x 9 2D Euler grid with forced decisions
// (psi^1 = 0.6, alpha = 2 where an order is 1), periodic or transmissive.
// Mirror pairs: the corners split between classes (qa, qb) and (qb, qa) by a
// fixed pattern, run by the pair kernel (one launch, blocks divided between
// the classes) and by the two one-class kernels.
// Usage: adjoint2d_host OUT.bin bc:q1:q2 ... pair:bc:qa:qb ...  writes, per
// case, the gathered adjoint of the one-kernel form, of the split form, and
// the seed ubar; per pair case, that of the pair kernel and of the two
// one-class kernels.
#include <hip/hip_runtime.h>
#include <cstring>
#include <vector>
thread_local dim3s threadIdx, blockIdx;
dim3s gridDim, blockDim;
pthread_barrier_t g_block_barrier;
#include "adjoint_kernels.inc"
using namespace acat;

template <class F>
void launch(int grid, F f) {
  gridDim = dim3s{(unsigned)grid, 1, 1};
  blockDim = dim3s{BLOCK, 1, 1};
  for (int b = 0; b < grid; ++b) {
    pthread_barrier_init(&g_block_barrier, nullptr, BLOCK);
    std::vector<pthread_t> th(BLOCK);
    struct Arg { F* f; int t, b; };
    std::vector<Arg> args(BLOCK);
    for (int t = 0; t < BLOCK; ++t) {
      args[t] = Arg{&f, t, b};
      pthread_create(&th[t], nullptr, [](void* p) -> void* {
        Arg* a = static_cast<Arg*>(p);
        threadIdx = dim3s{(unsigned)a->t, 0, 0};
        blockIdx = dim3s{(unsigned)a->b, 0, 0};
        (*a->f)();
        return nullptr;
      }, &args[t]);
    }
    for (int t = 0; t < BLOCK; ++t) pthread_join(th[t], nullptr);
    pthread_barrier_destroy(&g_block_barrier);
  }
}

const int NX = 10, NY = 9, P = 4, NV = 4;

struct Case {
  KProb pb;
  KStep st;
  std::vector<double> u, ubo, psix, alx, psiy, aly, C, ubi;
  std::vector<int8_t> ordx, ordy, cls;
  std::vector<int32_t> counts, list;
};

void setup(Case& cs, int bc, int q1, int q2, unsigned seed) {
  KProb& k = cs.pb;
  std::memset(&k, 0, sizeof(k));
  k.dim = 2; k.nvar = NV; k.flux = EUL; k.P = P; k.bc = bc; k.flags = 0;
  k.nx = NX; k.ny = NY;
  const int ext = bc == PERIODIC ? 0 : 1;
  k.nIx = NX + ext; k.nIy = NY + ext; k.ioff = -ext; k.n1 = NX + ext; k.n2 = NY + ext;
  k.ph.gamma = 1.4; k.ph.gm1 = 0.4; k.ph.ax = 1; k.ph.ay = 1;
  k.dx = 1.0 / NX; k.dy = 1.0 / NY; k.eps = 1e-12; k.theta = 0.5;
  const int plane = NX * NY;
  cs.u.resize(NV * plane); cs.ubo.resize(NV * plane); cs.ubi.assign(NV * plane, 0.0);
  for (int j = 0; j < NY; ++j)
    for (int i = 0; i < NX; ++i) {
      const double X = (i + 0.5) / NX, Y = (j + 0.5) / NY, tp = 2 * M_PI;
      const double rho = 1 + 0.1 * std::sin(tp * X) * std::cos(tp * Y);
      const double v = 0.3 + 0.05 * std::sin(tp * Y), w = -0.2 + 0.05 * std::cos(tp * X);
      const double p = 1 + 0.05 * std::sin(tp * (X + Y));
      const int e = j * NX + i;
      cs.u[e] = rho; cs.u[plane + e] = rho * v; cs.u[2 * plane + e] = rho * w;
      cs.u[3 * plane + e] = p / 0.4 + 0.5 * rho * (v * v + w * w);
    }
  unsigned s = seed;
  for (auto& x : cs.ubo) { s = s * 1664525u + 1013904223u; x = (s >> 8) * (1.0 / 16777216.0) - 0.5; }
  cs.ordx.assign(k.ny * k.nIx, (int8_t)q1); cs.ordy.assign(k.nIy * k.nx, (int8_t)q2);
  cs.psix.assign(k.ny * k.nIx, 0.6); cs.psiy.assign(k.nIy * k.nx, 0.6);
  cs.alx.assign(k.ny * k.nIx, 2.0); cs.aly.assign(k.nIy * k.nx, 2.0);
  const int items = k.n1 * k.n2;
  cs.cls.assign(items, (int8_t)((q1 - 1) * P + (q2 - 1)));
  cs.counts.assign(MAX_CLASSES, 0);
  cs.counts[(q1 - 1) * P + (q2 - 1)] = items;
  cs.list.resize(items);
  for (int e = 0; e < items; ++e) cs.list[e] = e;
  cs.C.assign((size_t)NV * items * 4 * P * P, 0.0);
  KStep& st = cs.st;
  std::memset(&st, 0, sizeof(st));
  st.u = cs.u.data(); st.dt = 0.002; st.dt_dev = nullptr;
  st.ordx = cs.ordx.data(); st.psix = cs.psix.data(); st.alx = cs.alx.data();
  st.ordy = cs.ordy.data(); st.psiy = cs.psiy.data(); st.aly = cs.aly.data();
  st.cls = cs.cls.data(); st.counts = cs.counts.data(); st.list = cs.list.data(); st.replay = 1;
}

template <int Q1, int Q2, int PASSES>
void run_adj(Case& cs) {
  KProb pb = cs.pb; KStep st = cs.st;
  const double* ubo = cs.ubo.data();
  double* C = cs.C.data();
  launch(8, [=]() { k_adj2d<EUL, NV, Q1, Q2, PASSES>(pb, st, ubo, C, 4 * P * P); });
}

void gather(Case& cs) {
  KProb pb = cs.pb; KStep st = cs.st;
  const double* ubo = cs.ubo.data();
  const double* C = cs.C.data();
  double* ubi = cs.ubi.data();
  const int grid = (NX * NY + BLOCK - 1) / BLOCK;
  if (pb.bc == PERIODIC) launch(grid, [=]() { k_gather2d<NV, true, P>(pb, st, ubo, C, 4 * P * P, ubi); });
  else launch(grid, [=]() { k_gather2d<NV, false, P>(pb, st, ubo, C, 4 * P * P, ubi); });
}

template <int Q1, int Q2>
void run_class(FILE* out, int bc) {
  Case one, split;
  setup(one, bc, Q1, Q2, 10 * Q1 + Q2);
  setup(split, bc, Q1, Q2, 10 * Q1 + Q2);
  run_adj<Q1, Q2, 3>(one);
  gather(one);
  if (Q1 != Q2) {
    run_adj<Q1, Q2, 1>(split);
    run_adj<Q1, Q2, 2>(split);
  } else {
    run_adj<Q1, Q2, 3>(split);
  }
  gather(split);
  double maxd = 0, scale = 0;
  for (size_t a = 0; a < one.ubi.size(); ++a) {
    maxd = std::fmax(maxd, std::fabs(one.ubi[a] - split.ubi[a]));
    scale = std::fmax(scale, std::fabs(split.ubi[a]));
  }
  std::printf("bc=%d class (%d,%d): max |one-kernel - split| = %.3e (scale %.3e)\n", bc, Q1, Q2, maxd, scale);
  std::fflush(stdout);
  std::fwrite(one.ubi.data(), sizeof(double), one.ubi.size(), out);
  std::fwrite(split.ubi.data(), sizeof(double), split.ubi.size(), out);
  std::fwrite(one.ubo.data(), sizeof(double), one.ubo.size(), out);
}

// corners of class (qb, qa) where (i1 + 2 i2) % 3 == 0, (qa, qb) elsewhere
void setup_pair(Case& cs, int bc, int qa, int qb, unsigned seed) {
  setup(cs, bc, qa, qb, seed);
  const int ca = (qa - 1) * P + (qb - 1), cb = (qb - 1) * P + (qa - 1);
  const int items = cs.pb.n1 * cs.pb.n2;
  std::vector<int32_t> la, lb;
  for (int e = 0; e < items; ++e) {
    const int i1 = e % cs.pb.n1, i2 = e / cs.pb.n1;
    const bool b = (i1 + 2 * i2) % 3 == 0;
    cs.cls[e] = (int8_t)(b ? cb : ca);
    (b ? lb : la).push_back(e);
  }
  cs.counts[ca] = (int32_t)la.size();
  cs.counts[cb] = (int32_t)lb.size();
  cs.list = la;
  cs.list.insert(cs.list.end(), lb.begin(), lb.end());
  cs.st.cls = cs.cls.data();
  cs.st.counts = cs.counts.data();
  cs.st.list = cs.list.data();
}

template <int QA, int QB>
void run_pair(FILE* out, int bc) {
  Case pair, sep;
  setup_pair(pair, bc, QA, QB, 10 * QA + QB);
  setup_pair(sep, bc, QA, QB, 10 * QA + QB);
  {
    KProb pb = pair.pb; KStep st = pair.st;
    const double* ubo = pair.ubo.data();
    double* C = pair.C.data();
    launch(2 * NXCD, [=]() { k_adj2d_pair<EUL, NV, QA, QB>(pb, st, ubo, C, 4 * P * P); });
  }
  gather(pair);
  run_adj<QA, QB, 3>(sep);
  run_adj<QB, QA, 3>(sep);
  gather(sep);
  double maxd = 0;
  for (size_t a = 0; a < pair.ubi.size(); ++a) maxd = std::fmax(maxd, std::fabs(pair.ubi[a] - sep.ubi[a]));
  std::printf("bc=%d pair (%d,%d)+(%d,%d): max |pair - one-class kernels| = %.3e\n", bc, QA, QB, QB, QA, maxd);
  std::fflush(stdout);
  std::fwrite(pair.ubi.data(), sizeof(double), pair.ubi.size(), out);
  std::fwrite(sep.ubi.data(), sizeof(double), sep.ubi.size(), out);
}

typedef void (*ClassFn)(FILE*, int);
struct Entry { int q1, q2; ClassFn fn; };
const Entry kClasses[] = {{2, 4, run_class<2, 4>}, {4, 2, run_class<4, 2>}, {3, 4, run_class<3, 4>},
                          {4, 3, run_class<4, 3>}, {3, 3, run_class<3, 3>}, {1, 4, run_class<1, 4>}};

const Entry kPairs[] = {{1, 2, run_pair<1, 2>}, {1, 3, run_pair<1, 3>}, {2, 3, run_pair<2, 3>},
                        {1, 4, run_pair<1, 4>}};

int main(int argc, char** argv) {
  if (argc < 3) return 2;
  FILE* out = std::fopen(argv[1], "wb");
  if (!out) return 2;
  for (int a = 2; a < argc; ++a) {
    int bc = 0, q1 = 0, q2 = 0;
    const bool pair = std::strncmp(argv[a], "pair:", 5) == 0;
    if (std::sscanf(argv[a] + (pair ? 5 : 0), "%d:%d:%d", &bc, &q1, &q2) != 3) return 2;
    bool found = false;
    const Entry* tab = pair ? kPairs : kClasses;
    const size_t ntab = pair ? sizeof(kPairs) / sizeof(Entry) : sizeof(kClasses) / sizeof(Entry);
    for (const Entry& e : std::vector<Entry>(tab, tab + ntab))
      if (e.q1 == q1 && e.q2 == q2) {
        e.fn(out, bc);
        found = true;
      }
    if (!found) return 3;
  }
  std::fclose(out);
  return 0;
}
