// gpf_runtime.hip -- host runtime and C ABI (include/gpf.h) of the coupled
// GP phase-field / lattice-Boltzmann step on gfx950.
//
// Context = validated parameters + A-B device buffers of the state
// (phi [N], mu [nc], U [dim], f* [Q], structure-of-arrays, x fastest) +
// the stream work is launched on.  Kernels are instantiated per
// (dim, N, nc, precision); gpf_init picks one and keeps its launchers.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <algorithm>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/gpf.h"
#include "gpf_adjoint.hpp"

namespace {

// message of the last gpf_init that failed on this thread (no context exists then)
thread_local std::string g_init_error;

const double kPi = 3.14159265358979323846;

struct Ops;

struct DevBuf {
  void* ptr = nullptr;
  size_t bytes = 0;
};

// one full state: phi [N], mu [nc], U [dim], stored populations f* [Q];
// tape states of the adjoint sweep also keep rho - rho0 of the step that
// produced them and share two population buffers
struct StateBuf {
  DevBuf phi, mu, u, f, dr;
};

}  // namespace

struct gpf_ctx {
  gpf_grid grid;
  gpf_params prm;
  int N = 0, nc = 0, Q = 0, dim = 0;
  int64_t n[3] = {1, 1, 1};
  int64_t cells = 0;
  size_t esize = 8;  // bytes per stored value
  hipStream_t stream = nullptr;
  DevBuf phi[2], mu[2], u[2], f[2];
  int cur = 0;  // index of the buffers holding step `step`
  int64_t step = 0;
  DevBuf scratch;   // FP64 staging for read / write (components * cells doubles)
  DevBuf partial;   // reduction partials
  DevBuf redout;    // final reduction values
  DevBuf badstep;   // health: smallest failing step
  DevBuf frontbuf;  // moving frame: front position found on the device
  // per k_phi_z block: the step that produced state buffer i left phi
  // unchanged on the block's cells (valid while bulk_ok[i])
  DevBuf bulkf[2];
  bool bulk_ok[2] = {false, false};
  // tiles that k_phi_zl walks (3D grids, bulk history on) and their
  // number, which starts at zero; zl_grid: its blocks per launch, the
  // device's resident blocks of it
  DevBuf tlist, tcount;
  unsigned zl_grid = 0;
  int64_t frame_off = 0;  // moving frame: cells shifted so far along the pull axis
  const double* target = nullptr;  // loss target (caller's device memory, N * cells FP64)
  int device = 0;                    // HIP device current at gpf_init
  double* noalloc_partial = nullptr; // this device's address of the static scratch array
  const Ops* ops = nullptr;
  std::string err;
  // adjoint: checkpoints every rec_every steps from step rec_start
  int64_t rec_every = 0, rec_start = 0;
  std::vector<StateBuf> ckpt;
  // two tapes of recomputed segment states (no f of their own): the segment
  // being reversed reads one while the previous segment is recomputed into
  // the other on a second stream (default priority)
  std::vector<StateBuf> tape[2];
  DevBuf tape_f[2][2];             // populations of each tape's states, alternating
  DevBuf tape_act[2];              // active set of phi per cell of each recomputed step (bytes)
  hipStream_t side = nullptr;
  hipEvent_t ev_free[2] = {nullptr, nullptr}, ev_done[2] = {nullptr, nullptr};
  StateBuf lam[2];                 // adjoint state (phi, mu, U, post-streaming f)
  DevBuf t_phil, t_w, t_rbar, t_part, t_acc, t_slices, t_rflag, t_fflag, t_fbuf, t_cbuf;
  DevBuf t_rowflag;                // per (y, z) row seed flags, two step parities
  int lam_cur = 0;                 // lam[lam_cur] holds the adjoint of the earliest state reached
  bool have_adjoint = false;
  // graph replay of kGraphSteps steps on small grids, one per starting buffer
  // set, valid while the kernel parameter block and shift it was captured
  // with are unchanged; captured on a stream of the library's own
  hipStream_t gstream = nullptr;
  hipGraphExec_t gexec[2] = {nullptr, nullptr};
  std::string gkey[2];
};

namespace {

int fail(gpf_ctx* c, int code, const char* fmt, ...) {
  if (c) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    c->err = buf;
  }
  return code;
}

#define HIP_OR_FAIL(ctx, call)                                                         \
  do {                                                                                 \
    hipError_t e_ = (call);                                                            \
    if (e_ != hipSuccess)                                                              \
      return fail(ctx, GPF_ERR_DEVICE, "%s failed: %s", #call, hipGetErrorString(e_)); \
  } while (0)

int dev_alloc(gpf_ctx* c, DevBuf& b, size_t bytes) {
  if (bytes == 0) bytes = 16;
  void* p = nullptr;
  if (c->prm.dev_alloc) {
    p = c->prm.dev_alloc(bytes, c->prm.alloc_user);
    if (!p) return fail(c, GPF_ERR_NOMEM, "dev_alloc callback returned NULL for %zu bytes", bytes);
  } else {
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess)
      return fail(c, GPF_ERR_NOMEM, "hipMalloc of %zu bytes failed: %s", bytes, hipGetErrorString(e));
  }
  b.ptr = p;
  b.bytes = bytes;
  return GPF_OK;
}

void dev_release(gpf_ctx* c, DevBuf& b) {
  if (!b.ptr) return;
  if (c->prm.dev_alloc) {
    if (c->prm.dev_free) c->prm.dev_free(b.ptr, c->prm.alloc_user);
  } else {
    (void)hipFree(b.ptr);
  }
  b.ptr = nullptr;
  b.bytes = 0;
}

// ---------------------------------------------------------------------------
// kernel parameter block
// ---------------------------------------------------------------------------
// lattice weight w_k of D2Q9 (Q = 9), D3Q19 or D3Q27
double lattice_w(int Q, int k) {
  return Q == 9 ? gpf::Lat<9>::w(k) : (Q == 19 ? gpf::Lat<19>::w(k) : gpf::Lat<27>::w(k));
}

template <class R>
gpf::KP<R> make_kp(const gpf_ctx* c) {
  const gpf_params& p = c->prm;
  gpf::KP<R> k;
  std::memset(&k, 0, sizeof(k));
  for (int a = 0; a < 3; ++a) {
    k.n[a] = (int)c->n[a];
    k.per[a] = (a < c->dim) ? (int)((c->grid.periodic_mask >> a) & 1u) : 1;
  }
  k.sy = c->n[0];
  k.sz = c->n[0] * c->n[1];
  k.cells = c->cells;
  k.potential = p.potential;
  k.pull_axis = p.pull_axis;
  k.grav_axis = p.grav_axis;
  k.dx = (R)c->grid.dx;
  k.dt = (R)p.dt;
  k.eps = (R)p.eps;
  k.rate = (R)(p.dt / (p.tau_pf * p.eps));
  k.tau_pf = (R)p.tau_pf;
  for (int a = 0; a < 4; ++a)
    for (int b = 0; b < 4; ++b) {
      k.gamma[a][b] = (R)p.gamma[a][b];
      k.delta[a][b] = (R)p.delta[a][b];
    }
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) k.chi[i][j] = (R)p.chi[i][j];
  for (int a = 0; a < 4; ++a) {
    for (int i = 0; i < 2; ++i) {
      k.c0[a][i] = (R)p.c0[a][i];
      k.D[a][i] = (R)p.D[a][i];
    }
    k.dS[a] = (R)p.dS[a];
  }
  for (int i = 0; i < 2; ++i) {
    k.mu_ref_d[i] = (p.precision == GPF_FP32 && i < c->nc) ? p.mu_inf[i] : 0.0;
    k.mu_ref[i] = (R)k.mu_ref_d[i];
  }
  for (int a = 0; a < 4; ++a)
    for (int i = 0; i < 2; ++i) {
      double s = p.c0[a][i];
      for (int j = 0; j < c->nc; ++j) s += p.chi[i][j] * k.mu_ref_d[j];
      k.c0s_d[a][i] = s;
      k.c0s[a][i] = (R)s;
    }
  k.G = (R)p.G;
  k.tdev_iso = (R)(p.T_iso - p.T_E);
  k.tdep = 0;
  for (int a = 0; a < 4; ++a)
    for (int i = 0; i < 2; ++i) {
      k.mT[a][i] = (a < c->N && i < c->nc) ? (R)p.mT[a][i] : R(0);
      if (k.mT[a][i] != R(0)) k.tdep = 1;
    }
  k.dtdev = (R)(p.G != 0.0 ? -p.G * p.V : 0.0);
  k.T_E = (R)p.T_E;
  k.tau_lb = (R)p.tau_lb;
  k.omega = (R)(1.0 / p.tau_lb);
  k.guo = (R)(1.0 - 0.5 / p.tau_lb);
  k.idx = (R)(1.0 / c->grid.dx);
  k.conv = (R)(c->grid.dx / p.dt);
  k.ieps = (R)(1.0 / p.eps);
  k.rho0 = (R)p.rho0;
  for (int i = 0; i < 2; ++i) {
    k.gbeta[i] = (R)p.gbeta[i];
    k.c_ref[i] = (R)p.c_ref[i];
  }
  k.grav_sign = (R)p.grav_sign;
  const double nu = (p.tau_lb - 0.5) / 3.0;
  k.kappa = (R)(2.0 * nu * p.h_drag / p.W0);
  k.lid_u = (R)p.lid_u;
  k.shrink = 0;
  for (int a = 0; a < 4; ++a) {
    k.eta[a] = (a < c->N) ? (R)p.eta[a] : R(0);
    if (k.eta[a] != R(0)) k.shrink = 1;
  }
  k.qmin2 = (sizeof(R) == 8) ? (R)1e-24 : (R)1e-12;
  for (int q = 0; q < c->Q; ++q)
    k.w[q] = (R)lattice_w(c->Q, q);
  return k;
}

// the pulled temperature's moving origin y0 + V n
// T - T_E = G (x_pull - tshift): x_pull + frame_off is the laboratory coordinate
double tshift(const gpf_ctx* c, int64_t step) {
  return c->prm.y0 + c->prm.V * (double)step - (double)c->frame_off;
}

// ---------------------------------------------------------------------------
// per-instance launchers
// ---------------------------------------------------------------------------
struct Ops {
  int (*step)(gpf_ctx*, int64_t, double*, int);
  int (*frame)(gpf_ctx*);
  int (*read)(gpf_ctx*, int, double*);  // to scratch (device FP64), returns components
  int (*write)(gpf_ctx*, int);          // from scratch
  int (*reduce)(gpf_ctx*, int, double*);
  int (*reduce_dev)(gpf_ctx*, int, double*, double*);  // which, partials, device output
  int (*loss_seed)(gpf_ctx*, double*);
  int (*read_native)(gpf_ctx*, int, void*);
  int (*adjoint)(gpf_ctx*, const double*, bool, double*);  // seed, seed in device memory, grads
  int (*copy_state)(gpf_ctx*, const StateBuf&, const StateBuf&);
  int (*lam_read)(gpf_ctx*, int, double*);
};

inline unsigned lin_blocks(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }
// blocks of the partial-sum kernel of the FP64 totals: at most kRedBlocks
constexpr int kRedBlocks = 2048;
inline int reduce_blocks(const gpf_ctx* c) {
  return (int)std::min<int64_t>(kRedBlocks, lin_blocks(c->cells, gpf::RED_BLOCK));
}

// gpf_reduce_noalloc keeps its partial sums in this file-scope array instead
// of the context's buffer: kRedBlocks blocks x 2 components, 32 KiB per GPU,
// held until the process ends.  Host code never passes the array's name to a
// kernel (on the host it is only a stand-in symbol): it uses the device
// address that hipGetSymbolAddress returns, resolved once per device.
constexpr int kNoAllocDoubles = kRedBlocks * 2;
__device__ __align__(256) double scratch[kNoAllocDoubles];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_dev[kMaxDevices] = {};

// the current device's address of `scratch` into c (called by gpf_init with
// the context's device current)
int resolve_scratch(gpf_ctx* c) {
  int dev = 0;
  HIP_OR_FAIL(c, hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(c, GPF_ERR_DEVICE, "device %d beyond %d", dev, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(c, GPF_ERR_DEVICE, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
    g_scratch_dev[dev] = static_cast<double*>(ptr);
  }
  c->device = dev;
  c->noalloc_partial = g_scratch_dev[dev];
  return GPF_OK;
}
// grid of the adjoint kernels: one slab of ceil(ny / 8) rows per XCD (gpf::adj_cell)
inline unsigned adj_blocks(const int64_t (&n)[3]) {
  return 8u * lin_blocks(n[0] * ((n[1] + 7) / 8) * n[2], gpf::ADJ_BLOCK);
}

// z-marching launch shape: 64 x GPF_TILE_Y tiles; each block of k_phi_z walks
// GPF_ZCHUNK_PHI planes, each of k_mulbm_z GPF_ZCHUNK_MU (best measured of
// 64 x {2, 4, 8} x {4, 8, 16, 32} on the 256^3 dendrite)
#ifndef GPF_TILE_Y
#define GPF_TILE_Y 4
#endif
#ifndef GPF_ZCHUNK_PHI2
#define GPF_ZCHUNK_PHI2 4
#endif
#ifndef GPF_ZCHUNK_PHI
#define GPF_ZCHUNK_PHI 16
#endif
#ifndef GPF_ZCHUNK_MU
#define GPF_ZCHUNK_MU 4
#endif
constexpr int kTileY = GPF_TILE_Y, kZChunkMu = GPF_ZCHUNK_MU;
// planes per phase-field block: a two-phase step spends its phase-field time
// in the few tiles near the interface (3D: the tiles k_phi_zl walks), whose
// plane walk a shorter chunk shortens; three and four phases have interface
// throughout the solid, where a longer chunk re-reads fewer halo planes
constexpr int zchunk_phi(int N) { return N == 2 ? GPF_ZCHUNK_PHI2 : GPF_ZCHUNK_PHI; }
// a k_mulbm_z block's planes lie within one k_phi_z block's (its bulk flag applies)
static_assert(zchunk_phi(2) % kZChunkMu == 0 && zchunk_phi(3) % kZChunkMu == 0,
              "the phase-field plane chunk must be a multiple of the LBM's");
// blocks of one k_phi_z launch (64 x kTileY tiles, zchunk_phi(N) planes each in 3D)
inline int64_t phi_blocks(const gpf_ctx* c) {
  const int64_t tx = (c->n[0] + 63) / 64, ty = (c->n[1] + kTileY - 1) / kTileY;
  const int zc = zchunk_phi(c->N);
  const int64_t tz = (c->dim == 3) ? (c->n[2] + zc - 1) / zc : 1;
  return tx * ty * tz;
}

template <int D, int Q, int N, int NC, class R>
struct Impl {
  static R* P(DevBuf& b) { return static_cast<R*>(b.ptr); }

  static int health(gpf_ctx* c) {
    gpf::KP<R> k = make_kp<R>(c);
    const int s = c->cur;
    hipLaunchKernelGGL((gpf::k_health<D, Q, N, NC, R>), dim3(lin_blocks(c->cells, 256)), dim3(256), 0,
                       c->stream, k, P(c->phi[s]), P(c->mu[s]), P(c->f[s]),
                       (unsigned long long)c->step,
                       static_cast<unsigned long long*>(c->badstep.ptr));
    HIP_OR_FAIL(c, hipGetLastError());
    return GPF_OK;
  }

  struct SP {
    R *phi, *mu, *u, *f, *dr;
  };
  static SP sp(StateBuf& s) { return SP{P(s.phi), P(s.mu), P(s.u), P(s.f), P(s.dr)}; }
  static SP cur(gpf_ctx* c, int s) {
    return SP{P(c->phi[s]), P(c->mu[s]), P(c->u[s]), P(c->f[s]), nullptr};
  }

  // bulk_in / bulk_out: k_phi_z's bulk history, only for a step from one
  // state buffer into the other (null elsewhere)
  static void launch_step(gpf_ctx* c, const gpf::KP<R>& k, const SP& in, const SP& out, R ts,
                          hipStream_t st, hipEvent_t* ev, const uint8_t* bulk_in = nullptr,
                          uint8_t* bulk_out = nullptr, uint8_t* act_out = nullptr) {
    constexpr int TX = 64, TY = kTileY, ZP = zchunk_phi(N);
    const int tiles_x = (int)((c->n[0] + TX - 1) / TX), tiles_y = (int)((c->n[1] + TY - 1) / TY);
    auto grid = [&](int zc) {
      const int tiles_z = (D == 3) ? (int)((c->n[2] + zc - 1) / zc) : 1;
      return dim3((unsigned)tiles_x * (unsigned)tiles_y * (unsigned)tiles_z);
    };
    const dim3 block(TX * TY);
    if (ev) (void)hipEventRecord(ev[0], st);
    unsigned* counts = nullptr;  // set when the listed phase-field kernels ran
    if constexpr (D == 3) {
      if (bulk_in && !act_out && c->zl_grid) {
        // the tiles whose neighbourhood changed, then a walk over them only
        const int tiles_z = (int)((c->n[2] + ZP - 1) / ZP);
        const unsigned nb = (unsigned)tiles_x * (unsigned)tiles_y * (unsigned)tiles_z;
        unsigned* list = static_cast<unsigned*>(c->tlist.ptr);
        counts = static_cast<unsigned*>(c->tcount.ptr);
        hipLaunchKernelGGL((gpf::k_phi_todo<D>), dim3((nb + 255u) / 256u), dim3(256), 0, st, bulk_in, bulk_out, list,
                           counts, tiles_x, tiles_y, tiles_z, k.per[0], k.per[1], k.per[2]);
        const unsigned g = std::max(8u, std::min(c->zl_grid, (nb + 7u) / 8u * 8u));
        hipLaunchKernelGGL((gpf::k_phi_zl<D, N, NC, R, TX, TY>), dim3(g), block, 0, st, k, in.phi, in.mu, out.phi,
                           bulk_in, bulk_out, list, counts, ts, tiles_x, tiles_y, ZP);
      }
    }
    if (!counts) {
      if (act_out)
        hipLaunchKernelGGL((gpf::k_phi_z<D, N, NC, R, TX, TY, true>), grid(ZP), block, 0, st, k, in.phi, in.mu,
                           out.phi, bulk_in, bulk_out, act_out, ts, tiles_x, tiles_y, ZP);
      else
        hipLaunchKernelGGL((gpf::k_phi_z<D, N, NC, R, TX, TY, false>), grid(ZP), block, 0, st, k, in.phi, in.mu,
                           out.phi, bulk_in, bulk_out, act_out, ts, tiles_x, tiles_y, ZP);
    }
    if (ev) (void)hipEventRecord(ev[1], st);
#define GPF_MULBM(SH, MT)                                                                                     \
  hipLaunchKernelGGL((gpf::k_mulbm_z<D, Q, N, NC, R, TX, TY, SH, MT>), grid(kZChunkMu), block, 0, st, k, in.phi, \
                     out.phi, in.mu, in.u, in.f, out.mu, out.u, out.f, out.dr, bulk_out, ZP, ts, tiles_x,            \
                     tiles_y, kZChunkMu, counts)
    if (k.shrink) {
      if (k.tdep)
        GPF_MULBM(true, true);
      else
        GPF_MULBM(true, false);
    } else if (k.tdep) {
      GPF_MULBM(false, true);
    } else {
      GPF_MULBM(false, false);
    }
#undef GPF_MULBM
    if (ev) (void)hipEventRecord(ev[2], st);
  }

  // Moving frame.  Reading (the paper names the approach only): every
  // frame_every steps the front is the largest pull-axis index of a cell with
  // liquid fraction <= 1/2; beyond frame_front, every field of the state
  // (phi, mu, U, the streamed populations f^n) moves down the pull axis by the
  // excess d into the other buffer set, the d new far planes repeat the last
  // plane (zero gradient into the melt) and the frame origin grows by d.
  static int frame(gpf_ctx* c) {
    gpf::KP<R> k = make_kp<R>(c);
    int* fb = static_cast<int*>(c->frontbuf.ptr);
    hipLaunchKernelGGL((gpf::k_fill<int>), dim3(1), dim3(64), 0, c->stream, fb, (int64_t)1, -1);
    hipLaunchKernelGGL((gpf::k_front<N, R>), dim3(lin_blocks(c->cells, 256)), dim3(256), 0, c->stream, k,
                       P(c->phi[c->cur]), fb);
    HIP_OR_FAIL(c, hipGetLastError());
    int front = -1;
    HIP_OR_FAIL(c, hipMemcpyAsync(&front, fb, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
    const int64_t d = (int64_t)front - c->prm.frame_front;
    if (front < 0 || d <= 0) return GPF_OK;
    const int ax = c->prm.pull_axis;
    const int64_t stride = ax == 0 ? 1 : (ax == 1 ? c->n[0] : c->n[0] * c->n[1]);
    const int s = c->cur, t = 1 - c->cur;
    auto mv = [&](DevBuf& in, DevBuf& out, int ncomp) {
      const int64_t count = (int64_t)ncomp * c->cells;
      hipLaunchKernelGGL((gpf::k_shift<R>), dim3(lin_blocks(count, 256)), dim3(256), 0, c->stream, P(in), P(out),
                         count, c->cells, stride, c->n[ax], d);
    };
    mv(c->phi[s], c->phi[t], N);
    mv(c->mu[s], c->mu[t], NC);
    mv(c->u[s], c->u[t], D);
    // the populations move as the streamed f^n of the state: pull them into
    // FP64 staging, then store the f* whose pull gives f^n moved by d
    double* fs = static_cast<double*>(c->scratch.ptr);
    hipLaunchKernelGGL((gpf::k_gather_f<D, Q, R>), dim3(lin_blocks(c->cells, 256)), dim3(256), 0, c->stream, k,
                       P(c->f[s]), fs);
    hipLaunchKernelGGL((gpf::k_scatter_f<D, Q, R>), dim3(lin_blocks(c->cells, 256)), dim3(256), 0, c->stream, k,
                       fs, P(c->f[t]), ax, (int)d);
    HIP_OR_FAIL(c, hipGetLastError());
    c->cur = t;
    c->frame_off += d;
    c->bulk_ok[0] = c->bulk_ok[1] = false;
    return GPF_OK;
  }

  // Small grids: a step is two launches of a few microseconds, and the gaps
  // between launches are a sizeable part of it.  Runs of kGraphSteps steps
  // whose kernels see the same arguments every step (no pulled temperature in
  // motion, no moving frame, health check or recording) replay one captured
  // graph of them instead; its first step does not use the bulk history, so
  // the graph holds whatever state the buffers hold.
  static constexpr int64_t kGraphSteps = 64;
  static bool graph_eligible(const gpf_ctx* c, bool timed) {
    return small_grid(c) && !timed && c->prm.frame_every == 0 && c->prm.health_every == 0 && c->rec_every == 0 &&
           (c->prm.G == 0.0 || c->prm.V == 0.0);
  }
  // kGraphSteps steps from the current state by graph replay; *done false when
  // no graph could be used (nothing was queued then)
  static int graph_steps(gpf_ctx* c, const gpf::KP<R>& k, int64_t remaining, bool* done) {
    *done = false;
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    if (c->stream && hipStreamIsCapturing(c->stream, &cap) == hipSuccess && cap != hipStreamCaptureStatusNone)
      return GPF_OK;  // the caller is capturing: its graph records the plain launches
    const int s = c->cur, t = 1 - c->cur;
    const R ts = (R)tshift(c, c->step);
    std::string key(reinterpret_cast<const char*>(&k), sizeof(k));
    if (k.G != R(0)) key.append(reinterpret_cast<const char*>(&ts), sizeof(ts));
    if (!c->gexec[s] || c->gkey[s] != key) {
      if (remaining < 2 * kGraphSteps) return GPF_OK;  // not worth a capture
      if (c->gexec[s]) {
        (void)hipGraphExecDestroy(c->gexec[s]);
        c->gexec[s] = nullptr;
      }
      if (!c->gstream) HIP_OR_FAIL(c, hipStreamCreateWithFlags(&c->gstream, hipStreamNonBlocking));
      HIP_OR_FAIL(c, hipStreamBeginCapture(c->gstream, hipStreamCaptureModeThreadLocal));
      for (int64_t j = 0; j < kGraphSteps; ++j) {
        const int a = (s + (int)j) & 1, b = 1 - a;
        launch_step(c, k, cur(c, a), cur(c, b), ts, c->gstream, nullptr,
                    j ? static_cast<const uint8_t*>(c->bulkf[a].ptr) : nullptr, static_cast<uint8_t*>(c->bulkf[b].ptr));
      }
      hipGraph_t g = nullptr;
      HIP_OR_FAIL(c, hipStreamEndCapture(c->gstream, &g));
      const hipError_t e = hipGraphInstantiate(&c->gexec[s], g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (e != hipSuccess) {
        c->gexec[s] = nullptr;
        return fail(c, GPF_ERR_DEVICE, "hipGraphInstantiate failed: %s", hipGetErrorString(e));
      }
      c->gkey[s] = key;
    }
    HIP_OR_FAIL(c, hipGraphLaunch(c->gexec[s], c->stream));
    c->bulk_ok[s] = c->bulk_ok[t] = true;
    c->step += kGraphSteps;  // an even count: the state is back in buffer set s
    *done = true;
    return GPF_OK;
  }

  static int step(gpf_ctx* c, int64_t nsteps, double* kernel_ms, int nk) {
    gpf::KP<R> k = make_kp<R>(c);
    if constexpr (D == 3) {
      if (!c->zl_grid) {  // once, outside any capture: k_phi_zl's grid (a multiple of 8)
        int per_cu = 0, cus = 0;
        HIP_OR_FAIL(c, hipOccupancyMaxActiveBlocksPerMultiprocessor(
                           &per_cu, gpf::k_phi_zl<D, N, NC, R, 64, kTileY>, 64 * kTileY, 0));
        HIP_OR_FAIL(c, hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c->device));
        c->zl_grid = std::max(8u, (unsigned)(std::max(per_cu, 1) * cus) / 8u * 8u);
      }
    }
    hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
    if (kernel_ms) {
      for (int i = 0; i < 3; ++i) HIP_OR_FAIL(c, hipEventCreate(&ev[i]));
      for (int i = 0; i < nk; ++i) kernel_ms[i] = 0.0;
    }
    const int64_t H = c->prm.health_every;
    const bool graphs = graph_eligible(c, kernel_ms != nullptr);
    for (int64_t it = 0; it < nsteps; ++it) {
      if (graphs && nsteps - it >= kGraphSteps) {
        bool done = false;
        if (int rc = graph_steps(c, k, nsteps - it, &done)) return rc;
        if (done) {
          it += kGraphSteps - 1;
          continue;
        }
      }
      const int s = c->cur, t = 1 - c->cur;
      const R ts = (R)tshift(c, c->step);
      launch_step(c, k, cur(c, s), cur(c, t), ts, c->stream, kernel_ms ? ev : nullptr,
                  c->bulk_ok[s] ? static_cast<const uint8_t*>(c->bulkf[s].ptr) : nullptr,
                  static_cast<uint8_t*>(c->bulkf[t].ptr));
      HIP_OR_FAIL(c, hipGetLastError());
      c->bulk_ok[t] = true;
      if (kernel_ms) {
        HIP_OR_FAIL(c, hipEventSynchronize(ev[2]));
        float a = 0.f, b = 0.f;
        HIP_OR_FAIL(c, hipEventElapsedTime(&a, ev[0], ev[1]));
        HIP_OR_FAIL(c, hipEventElapsedTime(&b, ev[1], ev[2]));
        if (nk > 0) kernel_ms[0] += a;
        if (nk > 1) kernel_ms[1] += b;
      }
      c->cur = t;
      c->step += 1;
      if (c->prm.frame_every > 0 && c->step % c->prm.frame_every == 0) {
        int rc = frame(c);
        if (rc) return rc;
      }
      if (H > 0 && (c->step % H == 0 || it == nsteps - 1)) {
        int rc = health(c);
        if (rc) return rc;
      }
      if (c->rec_every > 0 && (c->step - c->rec_start) % c->rec_every == 0) {
        int rc = save_ckpt(c);
        if (rc) return rc;
      }
    }
    if (kernel_ms)
      for (int i = 0; i < 3; ++i) (void)hipEventDestroy(ev[i]);
    return GPF_OK;
  }

  // field -> scratch (FP64 on the device); returns the component count
  static int read(gpf_ctx* c, int field, double* comps) {
    gpf::KP<R> k = make_kp<R>(c);
    const int s = c->cur;
    double* out = static_cast<double*>(c->scratch.ptr);
    const unsigned nb = lin_blocks(c->cells, 256);
    int ncomp = 0;
    switch (field) {
      case GPF_PHI: ncomp = N; break;
      case GPF_MU: ncomp = NC; break;
      case GPF_U: ncomp = D; break;
      default: break;
    }
    if (field == GPF_MU) {
      const int64_t cnt = ncomp * c->cells;
      hipLaunchKernelGGL((gpf::k_mu_to_double<R>), dim3(lin_blocks(cnt, 256)), dim3(256), 0, c->stream,
                         P(c->mu[s]), out, c->cells, NC, k.mu_ref_d[0], k.mu_ref_d[1]);
    } else if (ncomp) {
      const R* src = field == GPF_PHI ? P(c->phi[s]) : P(c->u[s]);
      const int64_t cnt = ncomp * c->cells;
      hipLaunchKernelGGL((gpf::k_to_double<R>), dim3(lin_blocks(cnt, 256)), dim3(256), 0, c->stream, src,
                         out, cnt);
    } else if (field == GPF_FPOST) {
      ncomp = Q;
      const int64_t cnt = ncomp * c->cells;
      hipLaunchKernelGGL((gpf::k_to_double<R>), dim3(lin_blocks(cnt, 256)), dim3(256), 0, c->stream,
                         P(c->f[s]), out, cnt);
    } else if (field == GPF_F || field == GPF_RHO) {
      ncomp = (field == GPF_F) ? Q : 1;
      hipLaunchKernelGGL((gpf::k_gather_f<D, Q, R>), dim3(nb), dim3(256), 0, c->stream, k, P(c->f[s]),
                         out);
      if (field == GPF_RHO) {
        // rho into the slot after the Q populations, then move to the front
        double* rho = out + (int64_t)Q * c->cells;
        hipLaunchKernelGGL((gpf::k_derived<D, Q, N, NC, R>), dim3(nb), dim3(256), 0, c->stream, k, 0,
                           P(c->phi[s]), P(c->mu[s]), out, 0.0, rho);
        HIP_OR_FAIL(c, hipMemcpyAsync(out, rho, c->cells * sizeof(double), hipMemcpyDeviceToDevice,
                                      c->stream));
      }
    } else if (field == GPF_C || field == GPF_T || field == GPF_FLAGS) {
      const int which = field == GPF_C ? 1 : field == GPF_T ? 2 : 3;
      ncomp = field == GPF_C ? NC : 1;
      hipLaunchKernelGGL((gpf::k_derived<D, Q, N, NC, R>), dim3(nb), dim3(256), 0, c->stream, k, which,
                         P(c->phi[s]), P(c->mu[s]), out, tshift(c, c->step), out);
    } else {
      return fail(c, GPF_ERR_ARG, "unknown field %d", field);
    }
    HIP_OR_FAIL(c, hipGetLastError());
    *comps = ncomp;
    return GPF_OK;
  }

  static int read_native(gpf_ctx* c, int field, void* dst) {
    const int s = c->cur;
    size_t bytes = 0;
    const void* src = nullptr;
    switch (field) {
      case GPF_PHI: src = c->phi[s].ptr; bytes = N * c->cells * sizeof(R); break;
      case GPF_MU: {
        gpf::KP<R> k = make_kp<R>(c);
        const int64_t cnt = NC * c->cells;
        hipLaunchKernelGGL((gpf::k_mu_native<R>), dim3(lin_blocks(cnt, 256)), dim3(256), 0, c->stream,
                           P(c->mu[s]), static_cast<R*>(dst), c->cells, NC, k.mu_ref[0], k.mu_ref[1]);
        HIP_OR_FAIL(c, hipGetLastError());
        return GPF_OK;
      }
      case GPF_U: src = c->u[s].ptr; bytes = D * c->cells * sizeof(R); break;
      case GPF_F: {
        double comps = 0;
        int rc = read(c, GPF_F, &comps);
        if (rc) return rc;
        const int64_t cnt = Q * c->cells;
        hipLaunchKernelGGL((gpf::k_from_double<R>), dim3(lin_blocks(cnt, 256)), dim3(256), 0,
                           c->stream, static_cast<const double*>(c->scratch.ptr), static_cast<R*>(dst), cnt);
        HIP_OR_FAIL(c, hipGetLastError());
        return GPF_OK;
      }
      default: return fail(c, GPF_ERR_ARG, "field %d has no native device copy", field);
    }
    HIP_OR_FAIL(c, hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, c->stream));
    return GPF_OK;
  }

  // scratch (FP64) -> field of the current buffers
  static int write(gpf_ctx* c, int field) {
    gpf::KP<R> k = make_kp<R>(c);
    const int s = c->cur;
    const double* in = static_cast<const double*>(c->scratch.ptr);
    if (field == GPF_FPOST) {
      const int64_t cnt = Q * c->cells;
      hipLaunchKernelGGL((gpf::k_from_double<R>), dim3(lin_blocks(cnt, 256)), dim3(256), 0, c->stream, in,
                         P(c->f[s]), cnt);
    } else if (field == GPF_F) {
      hipLaunchKernelGGL((gpf::k_scatter_f<D, Q, R>), dim3(lin_blocks(c->cells, 256)), dim3(256), 0,
                         c->stream, k, in, P(c->f[s]), 0, 0);
    } else if (field == GPF_MU) {
      const int64_t cnt = NC * c->cells;
      hipLaunchKernelGGL((gpf::k_mu_from_double<R>), dim3(lin_blocks(cnt, 256)), dim3(256), 0, c->stream, in,
                         P(c->mu[s]), c->cells, NC, k.mu_ref_d[0], k.mu_ref_d[1]);
    } else {
      int ncomp = field == GPF_PHI ? N : D;
      R* dst = field == GPF_PHI ? P(c->phi[s]) : P(c->u[s]);
      const int64_t cnt = ncomp * c->cells;
      hipLaunchKernelGGL((gpf::k_from_double<R>), dim3(lin_blocks(cnt, 256)), dim3(256), 0, c->stream, in,
                         dst, cnt);
    }
    HIP_OR_FAIL(c, hipGetLastError());
    return GPF_OK;
  }

  // the fixed-order FP64 total `which` into dev_out (device memory) through
  // the partial sums in `partial` (reduce_blocks(c) * 2 doubles); asynchronous
  static int reduce_dev(gpf_ctx* c, int which, double* partial, double* dev_out) {
    gpf::KP<R> k = make_kp<R>(c);
    const int s = c->cur;
    const int nblk = reduce_blocks(c);
    const int ncomp = which == GPF_SUM_SOLUTE ? NC : 1;
    hipLaunchKernelGGL((gpf::k_partial<D, Q, N, NC, R>), dim3(nblk), dim3(gpf::RED_BLOCK), 0, c->stream, k,
                       which, P(c->phi[s]), P(c->mu[s]), P(c->f[s]), c->target, tshift(c, c->step), partial);
    hipLaunchKernelGGL(gpf::k_final_sum, dim3(1), dim3(gpf::RED_BLOCK), 0, c->stream, partial, nblk, ncomp,
                       dev_out);
    HIP_OR_FAIL(c, hipGetLastError());
    return GPF_OK;
  }

  static int reduce(gpf_ctx* c, int which, double* host_out) {
    const int ncomp = which == GPF_SUM_SOLUTE ? NC : 1;
    int rc = reduce_dev(c, which, static_cast<double*>(c->partial.ptr), static_cast<double*>(c->redout.ptr));
    if (rc) return rc;
    HIP_OR_FAIL(c, hipMemcpyAsync(host_out, c->redout.ptr, ncomp * sizeof(double), hipMemcpyDeviceToHost,
                                  c->stream));
    HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
    return GPF_OK;
  }

  static int loss_seed(gpf_ctx* c, double* dev_seed) {
    const int64_t cnt = (int64_t)N * c->cells;
    hipLaunchKernelGGL((gpf::k_loss_seed<R>), dim3(lin_blocks(cnt, 256)), dim3(256), 0, c->stream,
                       P(c->phi[c->cur]), c->target, dev_seed, cnt);
    HIP_OR_FAIL(c, hipGetLastError());
    return GPF_OK;
  }

  // ---------------- adjoint ----------------
  static int alloc_state(gpf_ctx* c, StateBuf& s) {
    const size_t cs = (size_t)c->cells * sizeof(R);
    int rc = dev_alloc(c, s.phi, N * cs);
    if (!rc) rc = dev_alloc(c, s.mu, NC * cs);
    if (!rc) rc = dev_alloc(c, s.u, D * cs);
    if (!rc) rc = dev_alloc(c, s.f, Q * cs);
    return rc;
  }
  static int copy_state(gpf_ctx* c, const StateBuf& dst, const StateBuf& src) {
    HIP_OR_FAIL(c, hipMemcpyAsync(dst.phi.ptr, src.phi.ptr, dst.phi.bytes, hipMemcpyDeviceToDevice, c->stream));
    HIP_OR_FAIL(c, hipMemcpyAsync(dst.mu.ptr, src.mu.ptr, dst.mu.bytes, hipMemcpyDeviceToDevice, c->stream));
    HIP_OR_FAIL(c, hipMemcpyAsync(dst.u.ptr, src.u.ptr, dst.u.bytes, hipMemcpyDeviceToDevice, c->stream));
    HIP_OR_FAIL(c, hipMemcpyAsync(dst.f.ptr, src.f.ptr, dst.f.bytes, hipMemcpyDeviceToDevice, c->stream));
    return GPF_OK;
  }
  // checkpoint m = (step - rec_start) / rec_every of the recording; a state
  // restored to an earlier step and stepped again overwrites the later ones
  static int save_ckpt(gpf_ctx* c) {
    const int64_t m = (c->step - c->rec_start) / c->rec_every;
    if (c->step < c->rec_start || m > (int64_t)c->ckpt.size())
      return fail(c, GPF_ERR_STATE, "step %lld is outside the recording started at step %lld",
                  (long long)c->step, (long long)c->rec_start);
    if (m == (int64_t)c->ckpt.size()) {
      StateBuf s;
      int rc = alloc_state(c, s);
      if (rc) return rc;
      c->ckpt.push_back(s);
    }
    StateBuf& s = c->ckpt[m];
    StateBuf cur_s;
    cur_s.phi = c->phi[c->cur];
    cur_s.mu = c->mu[c->cur];
    cur_s.u = c->u[c->cur];
    cur_s.f = c->f[c->cur];
    return copy_state(c, s, cur_s);
  }
  static void fill(gpf_ctx* c, DevBuf& b, int64_t n) {
    hipLaunchKernelGGL((gpf::k_fill<R>), dim3(lin_blocks(n, 256)), dim3(256), 0, c->stream, P(b), n, R(0));
  }

  // Reverse of step n (X^n -> X^{n+1}): lam_in = adjoint of X^{n+1}, lam_out =
  // adjoint of X^n.  Four stages, each a kernel boundary: the LBM reverse,
  // the mu / phi-local reverse, the flux VJPs, their gather.  On small grids
  // the gather of step n and the LBM reverse of step n - 1 share a launch.
  struct AdjLaunch {
    dim3 g, b;
    double* part;
    int64_t pstride;
    uint8_t *rflag, *fflag;
  };
  // Grids that do not fill the chip even at four waves per SIMD (256 CUs x
  // 4 SIMDs x 4 x 64 cells): there every adjoint kernel is latency-bound, so
  // the sweep trades work per thread for waves in flight and launches.
  static bool small_grid(const gpf_ctx* c) { return c->cells <= (int64_t)256 * 4 * 4 * 64; }
  static AdjLaunch adj_launch(gpf_ctx* c) {
    const unsigned nb = adj_blocks(c->n);
    return {dim3(nb), dim3(gpf::ADJ_BLOCK), static_cast<double*>(c->t_part.ptr), (int64_t)nb * gpf::NG,
            static_cast<uint8_t*>(c->t_rflag.ptr), static_cast<uint8_t*>(c->t_fflag.ptr)};
  }
  // row seed flags of reverse step n (parity n mod 2)
  static uint8_t* rowflags(gpf_ctx* c, int64_t n) {
    return static_cast<uint8_t*>(c->t_rowflag.ptr) + (n & 1) * c->n[1] * c->n[2];
  }
  // LBM reverse of step n (X^n -> X^{n+1}); its forces used T^{n+1}
  static void adj_lbm(gpf_ctx* c, const gpf::KP<R>& k, int64_t n, const SP& x0, const SP& x1, StateBuf& li,
                      StateBuf& lo) {
    const AdjLaunch a = adj_launch(c);
    const R ts1 = (R)tshift(c, n + 1);
    if (x1.dr)
      hipLaunchKernelGGL((gpf::k_adj_lbm<D, Q, N, NC, R, true>), a.g, a.b, 0, c->stream, k, x0.f, x1.dr, x1.u,
                         x1.phi, x1.mu, P(li.f), P(li.u), P(li.mu), P(lo.f), P(c->t_phil), P(c->t_w), P(lo.mu),
                         ts1, a.part);
    else
      hipLaunchKernelGGL((gpf::k_adj_lbm<D, Q, N, NC, R, false>), a.g, a.b, 0, c->stream, k, x0.f, x1.dr, x1.u,
                         x1.phi, x1.mu, P(li.f), P(li.u), P(li.mu), P(lo.f), P(c->t_phil), P(c->t_w), P(lo.mu),
                         ts1, a.part);
  }
  // act: the active sets of phi^n recorded by the recomputation of step n, or null
  static void adj_muphi_vjp(gpf_ctx* c, const gpf::KP<R>& k, const SP& x0, const SP& x1, int64_t n,
                            StateBuf& li, StateBuf& lo, const uint8_t* act) {
    const AdjLaunch a = adj_launch(c);
    if (act)
      hipLaunchKernelGGL((gpf::k_adj_muphi<D, N, NC, R, true>), a.g, a.b, 0, c->stream, k, x0.phi, x1.phi,
                         x0.mu, x1.mu, x0.u, P(c->t_w), P(li.phi), P(c->t_phil), P(lo.phi),
                         P(lo.mu), P(lo.u), P(c->t_rbar), a.rflag, rowflags(c, n), act, (R)tshift(c, n),
                         a.part + a.pstride);
    else
      hipLaunchKernelGGL((gpf::k_adj_muphi<D, N, NC, R, false>), a.g, a.b, 0, c->stream, k, x0.phi, x1.phi,
                         x0.mu, x1.mu, x0.u, P(c->t_w), P(li.phi), P(c->t_phil), P(lo.phi),
                         P(lo.mu), P(lo.u), P(c->t_rbar), a.rflag, rowflags(c, n), act, (R)tshift(c, n),
                         a.part + a.pstride);
    const int split = small_grid(c) ? 1 : 0;
    hipLaunchKernelGGL((gpf::k_adj_vjp<D, N, NC, R>), dim3(a.g.x * (split ? D + 1 : 1)), a.b, 0, c->stream, k,
                       x0.phi, P(c->t_rbar), a.rflag, P(c->t_fbuf), a.fflag, P(c->t_cbuf), a.part + 2 * a.pstride,
                       rowflags(c, n), split);
  }
  // gather of step n into lo.phi alone
  static void adj_phi2(gpf_ctx* c, const gpf::KP<R>& k, int64_t n, StateBuf& lo) {
    const AdjLaunch a = adj_launch(c);
    hipLaunchKernelGGL((gpf::k_adj_phi2<D, N, NC, R>), a.g, a.b, 0, c->stream, k, a.rflag, P(c->t_fbuf), a.fflag,
                       P(c->t_cbuf), P(lo.phi), rowflags(c, n), rowflags(c, n + 1));
  }
  // gather of step n into lo.phi, and the LBM reverse of step n - 1 (states
  // x0 = X^{n-1}, x1 = X^n) from lo (the adjoint of X^n) into li
  static void adj_phi2_lbm(gpf_ctx* c, const gpf::KP<R>& k, int64_t n, const SP& x0, const SP& x1,
                           StateBuf& lo, StateBuf& li) {
    const AdjLaunch a = adj_launch(c);
    if (x1.dr)
      hipLaunchKernelGGL((gpf::k_adj_phi2_lbm<D, Q, N, NC, R, true>), dim3(2 * a.g.x), a.b, 0, c->stream, k,
                         a.rflag,
                         P(c->t_fbuf), a.fflag, P(c->t_cbuf), P(lo.phi), rowflags(c, n), rowflags(c, n + 1), x0.f,
                         x1.dr, x1.u, x1.phi, x1.mu, P(lo.f),
                         P(lo.u), P(lo.mu), P(li.f), P(c->t_phil), P(c->t_w), P(li.mu), (R)tshift(c, n), a.part);
    else
      hipLaunchKernelGGL((gpf::k_adj_phi2_lbm<D, Q, N, NC, R, false>), dim3(2 * a.g.x), a.b, 0, c->stream, k,
                         a.rflag,
                         P(c->t_fbuf), a.fflag, P(c->t_cbuf), P(lo.phi), rowflags(c, n), rowflags(c, n + 1), x0.f,
                         x1.dr, x1.u, x1.phi, x1.mu, P(lo.f),
                         P(lo.u), P(lo.mu), P(li.f), P(c->t_phil), P(c->t_w), P(li.mu), (R)tshift(c, n), a.part);
  }

  // seed: dL/dphi at the current (final) state, FP64, N * cells values, in
  // host memory or (seed_on_device) device memory
  static int adjoint(gpf_ctx* c, const double* seed, bool seed_on_device, double* grads) {
    const int64_t K = c->rec_every;
    const int64_t total = c->step - c->rec_start;
    if (K <= 0 || total <= 0 || c->ckpt.empty())
      return fail(c, GPF_ERR_STATE, "nothing recorded: call gpf_record before stepping");
    if (c->n[0] * ((c->n[1] + 7) / 8) * c->n[2] >= ((int64_t)1 << 31))
      return fail(c, GPF_ERR_UNSUPPORTED, "grid too large for the adjoint's 32-bit cell slots");
    const size_t cs = (size_t)c->cells * sizeof(R);
    int rc = GPF_OK;
    if (!c->lam[0].phi.ptr) {
      for (int i = 0; i < 2 && !rc; ++i) rc = alloc_state(c, c->lam[i]);
      const unsigned nb = adj_blocks(c->n);
      if (!rc) rc = dev_alloc(c, c->t_phil, cs);
      if (!rc) rc = dev_alloc(c, c->t_w, NC * cs);
      if (!rc) rc = dev_alloc(c, c->t_rbar, N * cs);
      // running sums: the LBM, mu / phi-local and (up to D + 1 grids) VJP reverses
      if (!rc) rc = dev_alloc(c, c->t_part, (size_t)(D + 3) * nb * gpf::NG * sizeof(double));
      if (!rc) rc = dev_alloc(c, c->t_acc, gpf::NG * sizeof(double));
      if (!rc) rc = dev_alloc(c, c->t_slices, (size_t)gpf::GA * gpf::NG * sizeof(double));
      if (!rc) rc = dev_alloc(c, c->t_rflag, (size_t)c->cells);
      if (!rc) rc = dev_alloc(c, c->t_rowflag, (size_t)2 * c->n[1] * c->n[2]);
      if (!rc) rc = dev_alloc(c, c->t_fflag, (size_t)D * c->cells);
      // reverse of the face fluxes and cell terms: N (1 + D) values per face / cell
      if (!rc) rc = dev_alloc(c, c->t_fbuf, (size_t)D * N * (1 + D) * cs);
      if (!rc) rc = dev_alloc(c, c->t_cbuf, (size_t)N * (1 + D) * cs);
      if (rc) return rc;
    }
    const int64_t nseg = (total + K - 1) / K;
    auto alloc_tape = [&](int b) -> int {
      while ((int64_t)c->tape[b].size() < K - 1) {
        StateBuf s;
        int r = dev_alloc(c, s.phi, N * cs);
        if (!r) r = dev_alloc(c, s.mu, NC * cs);
        if (!r) r = dev_alloc(c, s.u, D * cs);
        if (!r) r = dev_alloc(c, s.dr, cs);
        if (r) {
          dev_release(c, s.phi);
          dev_release(c, s.mu);
          dev_release(c, s.u);
          return r;
        }
        c->tape[b].push_back(s);
      }
      for (int i = 0; i < 2 && K > 1; ++i) {
        int r;
        if (!c->tape_f[b][i].ptr && (r = dev_alloc(c, c->tape_f[b][i], Q * cs))) return r;
      }
      const size_t act_bytes = (size_t)(K - 1) * (size_t)c->cells;
      if (K > 1 && c->tape_act[b].bytes < act_bytes) {
        dev_release(c, c->tape_act[b]);
        if (int r = dev_alloc(c, c->tape_act[b], act_bytes)) return r;
      }
      return GPF_OK;
    };
    // tape 0; with several segments, tape 1 for recomputing the previous
    // segment on the second stream.  If tape 1 does not fit, each segment is
    // recomputed into tape 0 on the library's stream before its reverse.
    if ((rc = alloc_tape(0))) return rc;
    int ntape = 1;
    if (nseg > 1) {
      if (alloc_tape(1) == GPF_OK) {
        ntape = 2;
      } else {
        for (auto& st : c->tape[1]) {
          dev_release(c, st.phi);
          dev_release(c, st.mu);
          dev_release(c, st.u);
          dev_release(c, st.dr);
        }
        c->tape[1].clear();
        dev_release(c, c->tape_f[1][0]);
        dev_release(c, c->tape_f[1][1]);
        dev_release(c, c->tape_act[1]);
        (void)hipGetLastError();  // a failed hipMalloc leaves its error behind
        c->err.clear();
      }
    }
    if (ntape > 1 && !c->side) {
      HIP_OR_FAIL(c, hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking));
      for (int b = 0; b < 2; ++b) {
        HIP_OR_FAIL(c, hipEventCreateWithFlags(&c->ev_free[b], hipEventDisableTiming));
        HIP_OR_FAIL(c, hipEventCreateWithFlags(&c->ev_done[b], hipEventDisableTiming));
      }
    }
    gpf::KP<R> k = make_kp<R>(c);
    // lam^N = (seed, 0, 0, 0)
    StateBuf* li = &c->lam[0];
    StateBuf* lo = &c->lam[1];
    if (!seed_on_device)
      HIP_OR_FAIL(c, hipMemcpyAsync(c->scratch.ptr, seed, (size_t)N * c->cells * sizeof(double),
                                    hipMemcpyHostToDevice, c->stream));
    hipLaunchKernelGGL((gpf::k_from_double<R>), dim3(lin_blocks(N * c->cells, 256)), dim3(256), 0,
                       c->stream, seed_on_device ? seed : static_cast<const double*>(c->scratch.ptr), P(li->phi),
                       N * c->cells);
    fill(c, li->mu, NC * c->cells);
    fill(c, li->u, D * c->cells);
    fill(c, li->f, Q * c->cells);
    hipLaunchKernelGGL((gpf::k_fill<double>), dim3(1), dim3(gpf::NG), 0, c->stream,
                       static_cast<double*>(c->t_acc.ptr), (int64_t)gpf::NG, 0.0);
    // per-block running sums of the parameter derivatives over the sweep
    hipLaunchKernelGGL((gpf::k_fill<uint8_t>), dim3(lin_blocks(2 * c->n[1] * c->n[2], 256)), dim3(256), 0,
                       c->stream, static_cast<uint8_t*>(c->t_rowflag.ptr), 2 * c->n[1] * c->n[2], (uint8_t)0);
    const int64_t nparts = (int64_t)(D + 3) * adj_blocks(c->n);
    hipLaunchKernelGGL((gpf::k_fill<double>), dim3(lin_blocks(nparts * gpf::NG, 256)), dim3(256), 0, c->stream,
                       static_cast<double*>(c->t_part.ptr), nparts * gpf::NG, 0.0);
    // slot j of segment sg in tape b holds X^{n0 + j} (slot 0 is the
    // checkpoint) and rho - rho0 of step n0 + j - 1; the tape's populations
    // alternate between its two buffers
    auto slot = [&](int b, int64_t sg, int64_t j) -> SP {
      if (j == 0) return sp(c->ckpt[sg]);
      SP s = sp(c->tape[b][j - 1]);
      s.f = P(c->tape_f[b][j % 2]);
      return s;
    };
    auto seg_len = [&](int64_t sg) { return std::min<int64_t>(K, total - sg * K); };
    // step j of the recomputation of segment sg into tape b; it also records
    // the active sets of phi^{n0 + j} (j < K - 1)
    auto act_of = [&](int b, int64_t j) { return static_cast<uint8_t*>(c->tape_act[b].ptr) + j * c->cells; };
    auto recompute_step = [&](int b, int64_t sg, int64_t j, hipStream_t st) {
      launch_step(c, k, slot(b, sg, j), slot(b, sg, j + 1), (R)tshift(c, c->rec_start + sg * K + j), st, nullptr,
                  nullptr, nullptr, act_of(b, j));
    };
    auto tape_of = [&](int64_t sg) { return ntape == 2 ? (int)((nseg - 1 - sg) & 1) : 0; };
    // X^{rec_start + m}, m in [0, total]: the checkpoints every K steps, the
    // current state at m = total (neither holds rho - rho0, so the LBM reverse
    // of the step that ends there reads its populations), else slot m mod K
    // of its segment's tape
    auto state = [&](int64_t m) -> SP {
      const int64_t sg = m / K, j = m % K;
      if (j == 0 && sg < (int64_t)c->ckpt.size()) return sp(c->ckpt[sg]);
      if (m == total) return cur(c, c->cur);
      return slot(tape_of(sg), sg, j);
    };
    // On small grids the gather and the next LBM reverse share a launch, as
    // two grids side by side (one kernel boundary less per step); on larger
    // ones the combined kernel's registers (121, against 67 for the gather
    // alone) cost more than the boundary.
    const bool fuse = small_grid(c);
    for (int64_t j = 0; j < seg_len(nseg - 1) - 1; ++j) recompute_step(0, nseg - 1, j, c->stream);
    adj_lbm(c, k, c->rec_start + total - 1, state(total - 1), state(total), *li, *lo);
    int64_t nrec = 0, jr = 0;
    for (int64_t m = total - 1; m >= 0; --m) {
      const int64_t sg = m / K, j = m % K;
      const int b = tape_of(sg);
      if (m == total - 1 || j == K - 1) {
        // first reverse step of segment sg: the previous segment goes into the
        // other tape once everything that read that tape (already queued) is
        // done; its steps are queued alternately with the reverse steps, so
        // neither stream waits for the host to queue the other's work
        nrec = (sg > 0 && ntape == 2) ? K - 1 : 0;
        jr = 0;
        if (sg > 0 && ntape == 2) {
          HIP_OR_FAIL(c, hipEventRecord(c->ev_free[1 - b], c->stream));
          HIP_OR_FAIL(c, hipStreamWaitEvent(c->side, c->ev_free[1 - b], 0));
        }
      }
      // the active sets of step m were recorded unless its successor is a
      // checkpoint or the final state (the step was not recomputed)
      const uint8_t* act = (j < seg_len(sg) - 1) ? act_of(b, j) : nullptr;
      adj_muphi_vjp(c, k, state(m), state(m + 1), c->rec_start + m, *li, *lo, act);
      if (jr < nrec) recompute_step(1 - b, sg - 1, jr++, c->side);
      if (m > 0) {
        if (j == 0 && ntape == 2) {
          // step m - 1 lies in the previous segment: its tape must be complete
          while (jr < nrec) recompute_step(1 - b, sg - 1, jr++, c->side);
          HIP_OR_FAIL(c, hipEventRecord(c->ev_done[1 - b], c->side));
          HIP_OR_FAIL(c, hipStreamWaitEvent(c->stream, c->ev_done[1 - b], 0));
        } else if (j == 0) {
          // one tape: the previous segment replaces this one, whose last
          // reader (the reverse of step m) is already queued
          for (int64_t jj = 0; jj < K - 1; ++jj) recompute_step(0, sg - 1, jj, c->stream);
        }
        if (fuse) {
          adj_phi2_lbm(c, k, c->rec_start + m, state(m - 1), state(m), *lo, *li);
        } else {
          adj_phi2(c, k, c->rec_start + m, *lo);
          adj_lbm(c, k, c->rec_start + m - 1, state(m - 1), state(m), *lo, *li);
        }
      } else {
        adj_phi2(c, k, c->rec_start + m, *lo);
      }
      HIP_OR_FAIL(c, hipGetLastError());
      std::swap(li, lo);
    }
    hipLaunchKernelGGL(gpf::k_grad_slices, dim3(gpf::GA), dim3(gpf::ADJ_BLOCK), 0, c->stream,
                       static_cast<const double*>(c->t_part.ptr), nparts, static_cast<double*>(c->t_slices.ptr));
    hipLaunchKernelGGL(gpf::k_grad_accum, dim3(1), dim3(gpf::GA), 0, c->stream,
                       static_cast<const double*>(c->t_slices.ptr), static_cast<double*>(c->t_acc.ptr));
    HIP_OR_FAIL(c, hipGetLastError());
    c->lam_cur = (li == &c->lam[0]) ? 0 : 1;
    c->have_adjoint = true;
    HIP_OR_FAIL(c, hipMemcpyAsync(grads, c->t_acc.ptr, gpf::NG * sizeof(double), hipMemcpyDeviceToHost,
                                  c->stream));
    HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
    return GPF_OK;
  }

  // adjoint of the recorded initial state, field by field, as FP64
  static int lam_read(gpf_ctx* c, int field, double* host) {
    StateBuf& l = c->lam[c->lam_cur];
    const R* src = nullptr;
    int64_t cnt = 0;
    switch (field) {
      case GPF_PHI: src = P(l.phi); cnt = N * c->cells; break;
      case GPF_MU: src = P(l.mu); cnt = NC * c->cells; break;
      case GPF_U: src = P(l.u); cnt = D * c->cells; break;
      case GPF_F: src = P(l.f); cnt = Q * c->cells; break;
      default: return fail(c, GPF_ERR_ARG, "field %d has no adjoint", field);
    }
    hipLaunchKernelGGL((gpf::k_to_double<R>), dim3(lin_blocks(cnt, 256)), dim3(256), 0, c->stream, src,
                       static_cast<double*>(c->scratch.ptr), cnt);
    HIP_OR_FAIL(c, hipMemcpyAsync(host, c->scratch.ptr, cnt * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
    return GPF_OK;
  }

  static const Ops* ops() {
    static const Ops o = {&step,      &frame,   &read,       &write,      &reduce,  &reduce_dev,
                          &loss_seed, &read_native, &adjoint, &copy_state, &lam_read};
    return &o;
  }
};

template <int D, int Q, int N, class R>
const Ops* pick_nc(int nc) {
  return nc == 1 ? Impl<D, Q, N, 1, R>::ops() : Impl<D, Q, N, 2, R>::ops();
}
template <int D, int Q, class R>
const Ops* pick_n(int N, int nc) {
  // four phases only with two solutes (three components), as Case 3
  return N == 2 ? pick_nc<D, Q, 2, R>(nc) : (N == 3 ? pick_nc<D, Q, 3, R>(nc) : Impl<D, Q, 4, 2, R>::ops());
}
template <class R>
const Ops* pick_d(int Q, int N, int nc) {
  return Q == 9 ? pick_n<2, 9, R>(N, nc) : (Q == 19 ? pick_n<3, 19, R>(N, nc) : pick_n<3, 27, R>(N, nc));
}
const Ops* pick(int Q, int N, int nc, int prec) {
  return prec == GPF_FP64 ? pick_d<double>(Q, N, nc) : pick_d<float>(Q, N, nc);
}

// ---------------------------------------------------------------------------
// validation
// ---------------------------------------------------------------------------
int validate(gpf_ctx* c, const gpf_grid* g, int N, int K, const gpf_params* p) {
  if (g->dim != 2 && g->dim != 3) return fail(c, GPF_ERR_UNSUPPORTED, "dim must be 2 or 3, got %d", g->dim);
  if ((g->dim == 2 && p->lattice != GPF_D2Q9) ||
      (g->dim == 3 && p->lattice != GPF_D3Q19 && p->lattice != GPF_D3Q27))
    return fail(c, GPF_ERR_PARAM, "lattice %d does not match dim %d (D2Q9 in 2D, D3Q19 or D3Q27 in 3D)",
                p->lattice, g->dim);
  if (N < 2 || N > 4) return fail(c, GPF_ERR_UNSUPPORTED, "n_phases must be 2, 3 or 4, got %d", N);
  if (N == 4 && K != 3)
    return fail(c, GPF_ERR_UNSUPPORTED, "four phases are built for three components (n_components = 3)");
  if (K < 2 || K > 3) return fail(c, GPF_ERR_UNSUPPORTED, "n_components must be 2 or 3, got %d", K);
  for (int a = 0; a < 4; ++a)
    if (!std::isfinite(p->eta[a])) return fail(c, GPF_ERR_PARAM, "eta[%d] is not finite", a);
  if (p->frame_every < 0) return fail(c, GPF_ERR_PARAM, "frame_every must be >= 0");
  if (p->frame_every > 0) {
    const int ax = p->pull_axis;
    if (ax < 0 || ax >= g->dim || (g->periodic_mask >> ax) & 1u)
      return fail(c, GPF_ERR_PARAM, "the moving frame needs walls on the pull axis");
    if (p->frame_front < 0 || p->frame_front >= g->n[ax])
      return fail(c, GPF_ERR_PARAM, "frame_front %lld outside [0, %lld)", (long long)p->frame_front,
                  (long long)g->n[ax]);
  }
  if (p->precision != GPF_FP64 && p->precision != GPF_FP32)
    return fail(c, GPF_ERR_ARG, "unknown precision %d", p->precision);
  if (p->potential != GPF_OBSTACLE && p->potential != GPF_WELL)
    return fail(c, GPF_ERR_ARG, "unknown potential %d", p->potential);
  for (int a = 0; a < g->dim; ++a)
    if (g->n[a] < 1 || g->n[a] > (1 << 20)) return fail(c, GPF_ERR_PARAM, "n[%d] = %lld out of range", a, (long long)g->n[a]);
  if (g->dim == 3 && g->n[2] > 65535) return fail(c, GPF_ERR_PARAM, "n[2] above 65535");
  if (!(g->dx > 0)) return fail(c, GPF_ERR_PARAM, "dx must be > 0");
  if (!(p->dt > 0) || !(p->eps > 0) || !(p->tau_pf > 0))
    return fail(c, GPF_ERR_PARAM, "dt, eps and tau_pf must be > 0");
  if (!(p->tau_lb > 0.5)) return fail(c, GPF_ERR_PARAM, "tau_lb must exceed 1/2 (got %g)", p->tau_lb);
  if (!(p->rho0 > 0)) return fail(c, GPF_ERR_PARAM, "rho0 must be > 0");
  if (!(p->W0 > 0) || !(p->h_drag >= 0)) return fail(c, GPF_ERR_PARAM, "W0 > 0 and h_drag >= 0 required");
  const int nc = K - 1;
  if (nc == 1) {
    if (!(p->chi[0][0] > 0)) return fail(c, GPF_ERR_PARAM, "chi must be positive");
  } else {
    const double det = p->chi[0][0] * p->chi[1][1] - p->chi[0][1] * p->chi[1][0];
    if (!(p->chi[0][0] > 0) || !(det > 0) || p->chi[0][1] != p->chi[1][0])
      return fail(c, GPF_ERR_PARAM, "chi must be symmetric positive definite");
  }
  if (p->pull_axis < 0 || p->pull_axis >= g->dim || p->grav_axis < 0 || p->grav_axis >= g->dim)
    return fail(c, GPF_ERR_PARAM, "pull_axis / grav_axis out of range");
  if (p->grav_sign != 1 && p->grav_sign != -1) return fail(c, GPF_ERR_PARAM, "grav_sign must be +1 or -1");
  // explicit (forward Euler) stability of the two diffusive updates
  const double lim = 1.0 / (2.0 * g->dim);
  double dmax = 0, gmax = 0, dlt = 0;
  for (int a = 0; a < N; ++a)
    for (int i = 0; i < nc; ++i) dmax = std::fmax(dmax, p->D[a][i]);
  for (int a = 0; a < N; ++a)
    for (int b = 0; b < N; ++b) {
      if (a == b) continue;
      gmax = std::fmax(gmax, p->gamma[a][b]);
      dlt = std::fmax(dlt, std::fabs(p->delta[a][b]));
      if (p->gamma[a][b] != p->gamma[b][a] || p->delta[a][b] != p->delta[b][a])
        return fail(c, GPF_ERR_PARAM, "gamma and delta must be symmetric");
      if (!(p->gamma[a][b] > 0)) return fail(c, GPF_ERR_PARAM, "gamma must be > 0");
    }
  if (dmax * p->dt / (g->dx * g->dx) > lim)
    return fail(c, GPF_ERR_PARAM, "D dt / dx^2 = %g exceeds the explicit bound %g", dmax * p->dt / (g->dx * g->dx), lim);
  const double pf = gmax * (1 + 3 * dlt) * (1 + 3 * dlt) * p->dt / (p->tau_pf * g->dx * g->dx);
  if (pf > lim) return fail(c, GPF_ERR_PARAM, "gamma dt / (tau dx^2) = %g exceeds the explicit bound %g", pf, lim);
  if (dlt >= 1.0 / 15.0) return fail(c, GPF_ERR_PARAM, "|delta| >= 1/15 makes the cubic stiffness negative");
  if (p->health_every < 0) return fail(c, GPF_ERR_PARAM, "health_every must be >= 0");
  if ((p->dev_alloc == nullptr) != (p->dev_free == nullptr))
    return fail(c, GPF_ERR_ARG, "dev_alloc and dev_free must be given together");
  return GPF_OK;
}

// ---------------------------------------------------------------------------
// initial state on the host (FP64), written through the same path as gpf_write
// ---------------------------------------------------------------------------

// counter-based SplitMix64 (Steele, Lea and Flood 2014): output j of the
// stream keyed by seed is the mix of seed + (j + 1) * golden gamma
uint64_t mix64(uint64_t seed, uint64_t j) {
  uint64_t z = seed + (j + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
// standard normal number j: Box-Muller on the 53-bit uniforms of counters 2j, 2j+1
double gauss(uint64_t seed, uint64_t j) {
  const double u1 = ((double)(mix64(seed, 2 * j) >> 11) + 1.0) * 0x1.0p-53;
  const double u2 = (double)(mix64(seed, 2 * j + 1) >> 11) * 0x1.0p-53;
  return std::sqrt(-2.0 * std::log(u1)) * std::cos(2.0 * kPi * u2);
}
// solid fraction of the double-obstacle equilibrium profile at signed distance s
double solid_fraction(double s, double eps) {
  const double half = kPi * kPi * eps / 8.0;
  if (s <= -half) return 1.0;
  if (s >= half) return 0.0;
  return 0.5 - 0.5 * std::sin(4.0 * s / (kPi * eps));
}

int write_host(gpf_ctx* c, int field, const double* src, size_t count);

int init_state(gpf_ctx* c, uint64_t seed) {
  const gpf_params& p = c->prm;
  const int64_t cells = c->cells;
  std::vector<double> phi((size_t)c->N * cells, 0.0), mu((size_t)c->nc * cells, 0.0),
      f((size_t)c->Q * cells, 0.0), u((size_t)c->dim * cells, 0.0);
  const double dx = c->grid.dx;
  for (int64_t P = 0; P < cells; ++P) {
    const int64_t x[3] = {P % c->n[0], (P / c->n[0]) % c->n[1], P / (c->n[0] * c->n[1])};
    double sol = 0.0;
    int solid = 0;
    if (p.init_kind == GPF_INIT_SEED) {
      double r2 = 0.0;
      for (int a = 0; a < c->dim; ++a) {
        const double d = ((double)x[a] - p.init_center[a]) * dx;
        r2 += d * d;
      }
      sol = solid_fraction(std::sqrt(r2) - p.init_radius * dx, p.eps);
    } else if (p.init_kind == GPF_INIT_LAMELLAE) {
      sol = solid_fraction(((double)x[p.pull_axis] - p.lam_height) * dx, p.eps);
      // the N - 1 solids take turns along x, lam_width cells each
      if (c->N >= 3 && p.lam_width > 0)
        solid = (int)(((int64_t)std::floor((double)x[0] / p.lam_width)) % (c->N - 1));
    }
    phi[(size_t)solid * cells + P] = sol;
    phi[(size_t)(c->N - 1) * cells + P] = 1.0 - sol;
    for (int i = 0; i < c->nc; ++i)
      mu[(size_t)i * cells + P] = p.mu_inf[i] + p.noise_sigma * gauss(seed, (uint64_t)P * c->nc + i);
    for (int k = 0; k < c->Q; ++k)
      f[(size_t)k * cells + P] = lattice_w(c->Q, k) * p.rho0;
  }
  int rc;
  if ((rc = write_host(c, GPF_PHI, phi.data(), phi.size()))) return rc;
  if ((rc = write_host(c, GPF_MU, mu.data(), mu.size()))) return rc;
  if ((rc = write_host(c, GPF_F, f.data(), f.size()))) return rc;
  if ((rc = write_host(c, GPF_U, u.data(), u.size()))) return rc;
  return GPF_OK;
}

int components(const gpf_ctx* c, int field) {
  switch (field) {
    case GPF_PHI: return c->N;
    case GPF_MU: return c->nc;
    case GPF_F: return c->Q;
    case GPF_RHO: return 1;
    case GPF_U: return c->dim;
    case GPF_C: return c->nc;
    case GPF_T: return 1;
    case GPF_FLAGS: return 1;
    case GPF_FPOST: return c->Q;
  }
  return -1;
}

int write_host(gpf_ctx* c, int field, const double* src, size_t count) {
  if (field != GPF_PHI && field != GPF_MU && field != GPF_F && field != GPF_U && field != GPF_FPOST)
    return fail(c, GPF_ERR_ARG, "field %d is not writable", field);
  const size_t want = (size_t)components(c, field) * (size_t)c->cells;
  if (count != want) return fail(c, GPF_ERR_ARG, "count %zu, expected %zu", count, want);
  HIP_OR_FAIL(c, hipMemcpyAsync(c->scratch.ptr, src, want * sizeof(double), hipMemcpyHostToDevice, c->stream));
  int rc = c->ops->write(c, field);
  if (rc) return rc;
  HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
  return GPF_OK;
}

void free_all(gpf_ctx* c) {
  for (int s = 0; s < 2; ++s) {
    dev_release(c, c->phi[s]);
    dev_release(c, c->mu[s]);
    dev_release(c, c->u[s]);
    dev_release(c, c->f[s]);
  }
  dev_release(c, c->scratch);
  dev_release(c, c->partial);
  dev_release(c, c->redout);
  dev_release(c, c->badstep);
  dev_release(c, c->frontbuf);
  dev_release(c, c->bulkf[0]);
  dev_release(c, c->bulkf[1]);
  dev_release(c, c->tlist);
  dev_release(c, c->tcount);
  auto rel = [&](StateBuf& s) {
    dev_release(c, s.phi);
    dev_release(c, s.mu);
    dev_release(c, s.u);
    dev_release(c, s.f);
    dev_release(c, s.dr);
  };
  if (c->side) {
    (void)hipStreamSynchronize(c->side);
    (void)hipStreamDestroy(c->side);
    c->side = nullptr;
  }
  for (auto& s : c->ckpt) rel(s);
  c->ckpt.clear();
  for (int b = 0; b < 2; ++b) {
    for (auto& s : c->tape[b]) rel(s);
    c->tape[b].clear();
    dev_release(c, c->tape_f[b][0]);
    dev_release(c, c->tape_f[b][1]);
    dev_release(c, c->tape_act[b]);
  }
  for (int b = 0; b < 2; ++b) {
    if (c->ev_free[b]) (void)hipEventDestroy(c->ev_free[b]);
    if (c->ev_done[b]) (void)hipEventDestroy(c->ev_done[b]);
    c->ev_free[b] = c->ev_done[b] = nullptr;
  }
  rel(c->lam[0]);
  rel(c->lam[1]);
  dev_release(c, c->t_phil);
  dev_release(c, c->t_w);
  dev_release(c, c->t_rbar);
  dev_release(c, c->t_part);
  dev_release(c, c->t_acc);
  dev_release(c, c->t_slices);
  dev_release(c, c->t_rflag);
  dev_release(c, c->t_rowflag);
  dev_release(c, c->t_fflag);
  dev_release(c, c->t_fbuf);
  dev_release(c, c->t_cbuf);
  for (int b = 0; b < 2; ++b) {
    if (c->gexec[b]) (void)hipGraphExecDestroy(c->gexec[b]);
    c->gexec[b] = nullptr;
  }
  if (c->gstream) {
    (void)hipStreamDestroy(c->gstream);
    c->gstream = nullptr;
  }
}

int set_named(gpf_ctx* c, gpf_params& p, const char* name, double v) {
  const int l = c->N - 1;
  if (!std::strcmp(name, "delta")) {
    for (int a = 0; a < 4; ++a)
      for (int b = 0; b < 4; ++b)
        if (p.delta[a][b] != 0.0) p.delta[a][b] = v;
  } else if (!std::strcmp(name, "tau_pf")) {
    p.tau_pf = v;
  } else if (!std::strcmp(name, "D")) {
    p.D[l][0] = v;
  } else if (!std::strcmp(name, "D1")) {
    p.D[l][1] = v;
  } else if (!std::strcmp(name, "gbeta")) {
    p.gbeta[0] = v;
  } else if (!std::strcmp(name, "gbeta1")) {
    p.gbeta[1] = v;
  } else {
    return fail(c, GPF_ERR_ARG, "unknown parameter '%s'", name);
  }
  return GPF_OK;
}

}  // namespace

// ============================ C ABI ==========================================

extern "C" {

int gpf_init(gpf_ctx** out, const gpf_grid* grid, int32_t n_phases, int32_t n_components,
             const gpf_params* params, uint64_t seed) {
  if (!out) return GPF_ERR_ARG;
  *out = nullptr;
  if (!grid || !params) return GPF_ERR_ARG;
  gpf_ctx* c = new (std::nothrow) gpf_ctx;
  if (!c) return GPF_ERR_NOMEM;
  int rc = validate(c, grid, n_phases, n_components, params);
  if (rc) {
    g_init_error = c->err;
    delete c;
    return rc;
  }
  c->grid = *grid;
  c->prm = *params;
  c->dim = grid->dim;
  c->N = n_phases;
  c->nc = n_components - 1;
  c->Q = (c->dim == 2) ? 9 : (params->lattice == GPF_D3Q27 ? 27 : 19);
  for (int a = 0; a < 3; ++a) c->n[a] = (a < c->dim) ? grid->n[a] : 1;
  c->cells = c->n[0] * c->n[1] * c->n[2];
  c->esize = (params->precision == GPF_FP64) ? 8 : 4;
  c->ops = pick(c->Q, c->N, c->nc, params->precision);
  rc = resolve_scratch(c);
  const size_t cs = (size_t)c->cells * c->esize;
  for (int s = 0; s < 2 && !rc; ++s) {
    if (!rc) rc = dev_alloc(c, c->phi[s], c->N * cs);
    if (!rc) rc = dev_alloc(c, c->mu[s], c->nc * cs);
    if (!rc) rc = dev_alloc(c, c->u[s], c->dim * cs);
    if (!rc) rc = dev_alloc(c, c->f[s], c->Q * cs);
  }
  if (!rc) rc = dev_alloc(c, c->scratch, (size_t)(c->Q + 1) * c->cells * sizeof(double));
  if (!rc) rc = dev_alloc(c, c->partial, kRedBlocks * 2 * sizeof(double));
  if (!rc) rc = dev_alloc(c, c->redout, 4 * sizeof(double));
  if (!rc) rc = dev_alloc(c, c->badstep, sizeof(unsigned long long));
  if (!rc) rc = dev_alloc(c, c->frontbuf, sizeof(int));
  for (int i = 0; i < 2 && !rc; ++i) rc = dev_alloc(c, c->bulkf[i], (size_t)phi_blocks(c));
  if (!rc) rc = dev_alloc(c, c->tlist, (size_t)phi_blocks(c) * sizeof(unsigned));
  if (!rc) rc = dev_alloc(c, c->tcount, sizeof(unsigned));
  if (!rc) {
    hipError_t e = hipMemsetAsync(c->badstep.ptr, 0xff, sizeof(unsigned long long), c->stream);
    if (e == hipSuccess) e = hipMemsetAsync(c->tcount.ptr, 0, sizeof(unsigned), c->stream);
    if (e == hipSuccess) e = hipMemsetAsync(c->tlist.ptr, 0, c->tlist.bytes, c->stream);
    if (e != hipSuccess) rc = fail(c, GPF_ERR_DEVICE, "hipMemsetAsync: %s", hipGetErrorString(e));
  }
  if (!rc) rc = init_state(c, seed);
  if (rc) {
    g_init_error = c->err;
    free_all(c);
    delete c;
    return rc;
  }
  g_init_error.clear();
  *out = c;
  return GPF_OK;
}

int gpf_set_stream(gpf_ctx* c, void* s) {
  if (!c) return GPF_ERR_ARG;
  c->stream = static_cast<hipStream_t>(s);
  return GPF_OK;
}

static int check_health_result(gpf_ctx* c) {
  unsigned long long bad = 0;
  HIP_OR_FAIL(c, hipMemcpyAsync(&bad, c->badstep.ptr, sizeof(bad), hipMemcpyDeviceToHost, c->stream));
  HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
  if (bad != ~0ull)
    return fail(c, GPF_ERR_NONFINITE, "non-finite phi/mu or rho <= 0 detected at step %llu", bad);
  return GPF_OK;
}

int gpf_step(gpf_ctx* c, int64_t n) {
  if (!c) return GPF_ERR_ARG;
  if (n < 0) return fail(c, GPF_ERR_ARG, "negative step count");
  int rc = c->ops->step(c, n, nullptr, 0);
  if (rc) return rc;
  if (c->prm.health_every > 0) return check_health_result(c);
  return GPF_OK;
}

int gpf_step_timed(gpf_ctx* c, int64_t n, double* kernel_ms, int32_t n_kernels) {
  if (!c || !kernel_ms || n_kernels < 1) return GPF_ERR_ARG;
  if (n < 0) return fail(c, GPF_ERR_ARG, "negative step count");
  int rc = c->ops->step(c, n, kernel_ms, n_kernels);
  if (rc) return rc;
  if (c->prm.health_every > 0) return check_health_result(c);
  HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
  return GPF_OK;
}

int gpf_read(gpf_ctx* c, int32_t field, double* dst, size_t count) {
  if (!c || !dst) return GPF_ERR_ARG;
  const int comps = components(c, field);
  if (comps < 0) return fail(c, GPF_ERR_ARG, "unknown field %d", field);
  if (count != (size_t)comps * (size_t)c->cells)
    return fail(c, GPF_ERR_ARG, "count %zu, expected %zu", count, (size_t)comps * (size_t)c->cells);
  double got = 0;
  int rc = c->ops->read(c, field, &got);
  if (rc) return rc;
  HIP_OR_FAIL(c, hipMemcpyAsync(dst, c->scratch.ptr, count * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
  return GPF_OK;
}

int gpf_read_device(gpf_ctx* c, int32_t field, void* dst, size_t bytes) {
  if (!c || !dst) return GPF_ERR_ARG;
  const int comps = components(c, field);
  if (field != GPF_PHI && field != GPF_MU && field != GPF_U && field != GPF_F)
    return fail(c, GPF_ERR_ARG, "field %d has no native device copy", field);
  if (bytes != (size_t)comps * (size_t)c->cells * c->esize)
    return fail(c, GPF_ERR_ARG, "bytes %zu, expected %zu", bytes, (size_t)comps * (size_t)c->cells * c->esize);
  return c->ops->read_native(c, field, dst);
}

int gpf_write(gpf_ctx* c, int32_t field, const double* src, size_t count) {
  if (!c || !src) return GPF_ERR_ARG;
  int rc = write_host(c, field, src, count);
  if (rc) return rc;
  c->bulk_ok[0] = c->bulk_ok[1] = false;  // the buffers no longer hold consecutive states
  // a written state starts a fresh health record
  HIP_OR_FAIL(c, hipMemsetAsync(c->badstep.ptr, 0xff, sizeof(unsigned long long), c->stream));
  HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
  return GPF_OK;
}

int gpf_reduce(gpf_ctx* c, int32_t which, double* out) {
  if (!c || !out) return GPF_ERR_ARG;
  if (which != GPF_SUM_SOLUTE && which != GPF_SUM_MASS && which != GPF_LOSS)
    return fail(c, GPF_ERR_ARG, "unknown reduction %d", which);
  if (which == GPF_LOSS && !c->target) return fail(c, GPF_ERR_STATE, "GPF_LOSS needs a target (gpf_set_target)");
  return c->ops->reduce(c, which, out);
}

int gpf_reduce_noalloc(gpf_ctx* c, int32_t which, double* dev_out) {
  if (!c || !dev_out) return GPF_ERR_ARG;
  if (which != GPF_SUM_SOLUTE && which != GPF_SUM_MASS && which != GPF_LOSS)
    return fail(c, GPF_ERR_ARG, "unknown reduction %d", which);
  if (which == GPF_LOSS && !c->target) return fail(c, GPF_ERR_STATE, "GPF_LOSS needs a target (gpf_set_target)");
  const int64_t need = (int64_t)reduce_blocks(c) * (which == GPF_SUM_SOLUTE ? c->nc : 1);
  if (need > kNoAllocDoubles)
    return fail(c, GPF_ERR_ARG, "%lld partial sums exceed the static scratch of %d doubles", (long long)need,
                kNoAllocDoubles);
  int dev = -1;
  HIP_OR_FAIL(c, hipGetDevice(&dev));
  if (dev != c->device)
    return fail(c, GPF_ERR_STATE, "device %d is current, the context lives on device %d", dev, c->device);
  return c->ops->reduce_dev(c, which, c->noalloc_partial, dev_out);
}

int gpf_bandwidth_probe(int32_t pattern, const void* dev_in, void* dev_out, const int64_t* n, int32_t reps,
                        void* stream, double* gbps) {
  if (!dev_in || !dev_out || !n || !gbps || reps < 1 || pattern < 0 || pattern > 2) return GPF_ERR_ARG;
  if (n[0] < 64 || n[0] % 64 || n[1] < kTileY || n[1] % kTileY || n[2] < kZChunkMu || n[2] % kZChunkMu ||
      n[0] > (1 << 20) || n[1] > (1 << 20) || n[2] > 65535)
    return GPF_ERR_ARG;
  const int64_t cells = n[0] * n[1] * n[2];
  if (19 * cells >= ((int64_t)1 << 31) * 8) return GPF_ERR_ARG;
  const float* in = static_cast<const float*>(dev_in);
  float* out = static_cast<float*>(dev_out);
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int n0 = (int)n[0], n1 = (int)n[1], n2 = (int)n[2];
  const unsigned zblocks = (unsigned)((n0 / 64) * (n1 / kTileY) * (n2 / kZChunkMu));
  auto launch = [&]() {
    if (pattern == 0)
      hipLaunchKernelGGL(gpf::k_probe_copy19, dim3(lin_blocks(cells, 256)), dim3(256), 0, st, in, out, cells);
    else if (pattern == 1)
      hipLaunchKernelGGL(gpf::k_probe_pull19, dim3(lin_blocks(cells, 256)), dim3(256), 0, st, in, out, n0, n1, n2);
    else
      hipLaunchKernelGGL((gpf::k_probe_pull19_z<kTileY>), dim3(zblocks), dim3(64 * kTileY), 0, st, in, out, n0, n1,
                         n2, kZChunkMu);
  };
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return GPF_ERR_DEVICE;
  launch();
  launch();
  (void)hipEventRecord(e0, st);
  for (int r = 0; r < reps; ++r) launch();
  (void)hipEventRecord(e1, st);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float ms = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (e != hipSuccess || !(ms > 0.f)) return GPF_ERR_DEVICE;
  *gbps = 2.0 * 19.0 * 4.0 * (double)cells * reps / (ms * 1e-3) / 1e9;
  return GPF_OK;
}

int gpf_set_target(gpf_ctx* c, const void* dev_target, size_t count) {
  if (!c) return GPF_ERR_ARG;
  if (!dev_target) {
    if (count != 0) return fail(c, GPF_ERR_ARG, "a NULL target clears it and takes count 0");
    c->target = nullptr;
    return GPF_OK;
  }
  if (count != (size_t)c->N * (size_t)c->cells)
    return fail(c, GPF_ERR_ARG, "count %zu, expected %zu", count, (size_t)c->N * (size_t)c->cells);
  c->target = static_cast<const double*>(dev_target);
  return GPF_OK;
}

int gpf_loss_seed_device(gpf_ctx* c, void* dev_seed, size_t count) {
  if (!c || !dev_seed) return GPF_ERR_ARG;
  if (count != (size_t)c->N * (size_t)c->cells)
    return fail(c, GPF_ERR_ARG, "count %zu, expected %zu", count, (size_t)c->N * (size_t)c->cells);
  if (!c->target) return fail(c, GPF_ERR_STATE, "no loss target (gpf_set_target)");
  return c->ops->loss_seed(c, static_cast<double*>(dev_seed));
}

int gpf_set_param(gpf_ctx* c, const char* name, double value) {
  if (!c || !name) return GPF_ERR_ARG;
  gpf_params p = c->prm;
  int rc = set_named(c, p, name, value);
  if (rc) return rc;
  rc = validate(c, &c->grid, c->N, c->nc + 1, &p);
  if (rc) return rc;
  c->prm = p;
  return GPF_OK;
}

int gpf_record(gpf_ctx* c, int64_t checkpoint_every) {
  if (!c) return GPF_ERR_ARG;
  if (checkpoint_every < 1) return fail(c, GPF_ERR_ARG, "checkpoint_every must be >= 1");
  (void)hipStreamSynchronize(c->stream);
  auto rel = [&](StateBuf& s) {
    dev_release(c, s.phi);
    dev_release(c, s.mu);
    dev_release(c, s.u);
    dev_release(c, s.f);
    dev_release(c, s.dr);
  };
  for (auto& s : c->ckpt) rel(s);
  c->ckpt.clear();
  for (int b = 0; b < 2; ++b)
    if ((int64_t)c->tape[b].size() > checkpoint_every) {
      for (auto& s : c->tape[b]) rel(s);
      c->tape[b].clear();
    }
  c->rec_every = checkpoint_every;
  c->rec_start = c->step;
  c->have_adjoint = false;
  StateBuf s;
  const size_t cs = (size_t)c->cells * c->esize;
  int rc = dev_alloc(c, s.phi, c->N * cs);
  if (!rc) rc = dev_alloc(c, s.mu, c->nc * cs);
  if (!rc) rc = dev_alloc(c, s.u, c->dim * cs);
  if (!rc) rc = dev_alloc(c, s.f, c->Q * cs);
  if (rc) return rc;
  c->ckpt.push_back(s);
  StateBuf cur_s;
  cur_s.phi = c->phi[c->cur];
  cur_s.mu = c->mu[c->cur];
  cur_s.u = c->u[c->cur];
  cur_s.f = c->f[c->cur];
  rc = c->ops->copy_state(c, s, cur_s);
  if (rc) return rc;
  HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
  return GPF_OK;
}

static int grad_slot(const char* name) {
  if (!std::strcmp(name, "delta")) return gpf::G_DELTA;
  if (!std::strcmp(name, "tau_pf")) return gpf::G_TAU;
  if (!std::strcmp(name, "D")) return gpf::G_D0;
  if (!std::strcmp(name, "D1")) return gpf::G_D1;
  if (!std::strcmp(name, "gbeta")) return gpf::G_GB0;
  if (!std::strcmp(name, "gbeta1")) return gpf::G_GB1;
  return -1;
}

namespace {
int adjoint_entry(gpf_ctx* c, const double* dL_dphi, bool on_device, size_t count, const char* const* names,
                  int32_t n_names, double* grads_out) {
  if (!c || !dL_dphi || (n_names > 0 && (!names || !grads_out)) || n_names < 0) return GPF_ERR_ARG;
  if (count != (size_t)c->N * (size_t)c->cells)
    return fail(c, GPF_ERR_ARG, "count %zu, expected %zu", count, (size_t)c->N * (size_t)c->cells);
  if (n_names > gpf::NG) return fail(c, GPF_ERR_ARG, "at most %d parameters", gpf::NG);
  for (int a = 0; a < 4; ++a)
    if (c->prm.eta[a] != 0.0)
      return fail(c, GPF_ERR_UNSUPPORTED, "the adjoint does not include the shrinkage force (eta != 0)");
  if (c->prm.frame_every > 0)
    return fail(c, GPF_ERR_UNSUPPORTED, "the adjoint does not include the moving frame (frame_every > 0)");
  int slots[gpf::NG];
  for (int i = 0; i < n_names; ++i) {
    slots[i] = names[i] ? grad_slot(names[i]) : -1;
    if (slots[i] < 0) return fail(c, GPF_ERR_ARG, "unknown parameter '%s'", names[i] ? names[i] : "(null)");
  }
  double g[gpf::NG];
  int rc = c->ops->adjoint(c, dL_dphi, on_device, g);
  if (rc) return rc;
  for (int i = 0; i < n_names; ++i) grads_out[i] = g[slots[i]];
  return GPF_OK;
}
}  // namespace

int gpf_adjoint(gpf_ctx* c, const double* dL_dphi, size_t count, const char* const* names,
                int32_t n_names, double* grads_out) {
  return adjoint_entry(c, dL_dphi, false, count, names, n_names, grads_out);
}

int gpf_adjoint_device(gpf_ctx* c, const void* dev_dL_dphi, size_t count, const char* const* names,
                       int32_t n_names, double* grads_out) {
  return adjoint_entry(c, static_cast<const double*>(dev_dL_dphi), true, count, names, n_names, grads_out);
}

int gpf_adjoint_state(gpf_ctx* c, int32_t field, double* host_dst, size_t count) {
  if (!c || !host_dst) return GPF_ERR_ARG;
  if (!c->have_adjoint) return fail(c, GPF_ERR_STATE, "no adjoint computed yet");
  const int comps = field == GPF_PHI ? c->N : field == GPF_MU ? c->nc : field == GPF_U ? c->dim
                  : field == GPF_F ? c->Q : -1;
  if (comps < 0) return fail(c, GPF_ERR_ARG, "field %d has no adjoint", field);
  if (count != (size_t)comps * (size_t)c->cells)
    return fail(c, GPF_ERR_ARG, "count %zu, expected %zu", count, (size_t)comps * (size_t)c->cells);
  return c->ops->lam_read(c, field, host_dst);
}

int64_t gpf_step_index(const gpf_ctx* c) { return c ? c->step : -1; }

int gpf_set_step_index(gpf_ctx* c, int64_t n) {
  if (!c) return GPF_ERR_ARG;
  if (n < 0) return fail(c, GPF_ERR_ARG, "negative step index");
  c->step = n;
  return GPF_OK;
}

int64_t gpf_frame_offset(const gpf_ctx* c) { return c ? c->frame_off : -1; }

int gpf_set_frame_offset(gpf_ctx* c, int64_t offset) {
  if (!c) return GPF_ERR_ARG;
  if (offset < 0) return fail(c, GPF_ERR_ARG, "negative frame offset");
  c->frame_off = offset;
  return GPF_OK;
}

const char* gpf_last_error(const gpf_ctx* c) { return c ? c->err.c_str() : g_init_error.c_str(); }

const char* gpf_status_string(int s) {
  switch (s) {
    case GPF_OK: return "ok";
    case GPF_ERR_ARG: return "invalid argument";
    case GPF_ERR_PARAM: return "invalid parameter";
    case GPF_ERR_NOMEM: return "out of device memory";
    case GPF_ERR_DEVICE: return "HIP error";
    case GPF_ERR_NONFINITE: return "non-finite state";
    case GPF_ERR_STATE: return "invalid state";
    case GPF_ERR_UNSUPPORTED: return "unsupported configuration";
  }
  return "unknown status";
}

void gpf_destroy(gpf_ctx* c) {
  if (!c) return;
  (void)hipStreamSynchronize(c->stream);
  free_all(c);
  delete c;
}

}  // extern "C"
