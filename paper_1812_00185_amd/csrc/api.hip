// C-ABI entry points of the CGP library (declared in include/cgp.h).
//
// Orchestration only: argument checks, workspace carving, uploads, and the
// host loops that queue solver iterations.  Krylov loops queue iterations in
// chunks and poll the device-side stopping flags one chunk behind (a copy of
// the solver scalars into pinned memory plus an event), so the GPU never
// idles waiting for the host while a solve is running.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "capcg.hpp"
#include "cgp.h"
#include "cheb2.hpp"
#include "corrlat.hpp"
#include "momlat.hpp"
#include "device.hpp"
#include "mesh.hpp"
#include "mpnn.hpp"
#include "ndchol.hpp"

using cgp::DLevel;
using cgp::Scal;

// The no-alloc scratch (see cgp_pcg_solve_noalloc): 7.5 MB per GPU.
constexpr size_t kScratchDoubles = 128 + 8 * 2 * 1280 + 7 * 131072;
static __device__ __align__(256) double scratch[kScratchDoubles];

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

#define HIPCHK(x)                                                                        \
  do {                                                                                   \
    hipError_t e_ = (x);                                                                 \
    if (e_ != hipSuccess) return fail(CGP_ERR_HIP, std::string(#x) + ": " + hipGetErrorString(e_)); \
  } while (0)

// Bump allocator over the caller's workspace (256-byte aligned pieces).  With
// base == nullptr it only measures.
struct Carver {
  char* base;
  size_t off = 0;
  explicit Carver(void* b) : base((char*)b) {}
  template <class T>
  T* take(size_t count) {
    off = (off + 255) & ~(size_t)255;
    T* p = base ? (T*)(base + off) : nullptr;
    off += count * sizeof(T);
    return p;
  }
};

// page-locked host buffer the caller provides to cgp_assemble: two chunks of
// eight mirrored solver-scalar records
constexpr size_t kHostBytes = sizeof(cgp::Scal) * 16;

// ---- device scratch of cgp_pcg_solve_noalloc ----------------------------
// The FP64 Jacobi-PCG's Krylov vectors (p and the alternating r, w, s),
// partial sums and solver scalars for callers that cannot allocate: one
// file-scope array per GPU, alive until the process ends.  Layout in
// doubles: scalars [0, 128), partial sums [128, 128 + kSlots * 2 * kNbMax),
// then seven vectors of kNoAllocMaxRows entries (every piece 256-byte
// aligned).  In host code the array's name is only a stand-in: kernels get
// the device address that hipGetSymbolAddress returns for the current GPU.
constexpr int32_t kNoAllocMaxRows = 131072;
constexpr size_t kScrScal = 0;
constexpr size_t kScrPart = 128;
constexpr size_t kScrVec = kScrPart + (size_t)cgp::kSlots * 2 * cgp::kNbMax;
constexpr size_t kScrDoubles = kScrVec + 7 * (size_t)kNoAllocMaxRows;
static_assert(sizeof(cgp::Scal) * 8 <= kScrPart * sizeof(double), "scalar slots");
static_assert((kScrVec * sizeof(double)) % 256 == 0, "vector alignment");
static_assert((kNoAllocMaxRows * sizeof(double)) % 256 == 0, "vector alignment");
static_assert(kScrDoubles == kScratchDoubles, "scratch size");

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_dev[kMaxDevices] = {};

// Device address of `scratch` on the current GPU (looked up once per device).
int scratch_address(double** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail(CGP_ERR_HIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices) return fail(CGP_ERR_INVALID, "device ordinal out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(CGP_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") +
                                   hipGetErrorString(e));
    g_scratch_dev[dev] = static_cast<double*>(ptr);
  }
  *out = g_scratch_dev[dev];
  return CGP_OK;
}

}  // namespace

struct cgp_ctx {
  cgp_problem prob;
  cgp::Hierarchy h;
  size_t ws_bytes = 0;
  bool assembled = false;
  int32_t nf = 0, nc = 0, tf = 0, tc = 0, ndir = 0;
  int nb_f = 1, nb_c = 1;

  DLevel F{}, C{};
  int32_t *tri_f = nullptr, *tri_c = nullptr, *pcode = nullptr, *cn_ptr = nullptr,
          *cn_tri = nullptr, *dir_index = nullptr;
  uint8_t* nat_c = nullptr;
  double *Mval = nullptr, *Aval = nullptr, *invdA = nullptr;
  double *Kc = nullptr, *Dxc = nullptr, *Dyc = nullptr, *invdKc = nullptr, *lumped_c = nullptr;
  float *Kc32 = nullptr, *invdKc32 = nullptr;
  // ELL copy of K_c for the PCG iteration kernel (width = longest row)
  int ell_w = 0;
  int mom_expect = 0;  // iterations of the last momentum solve (0: unknown)
  int32_t* ell_col = nullptr;
  double* ell_val = nullptr;    // K (factor-preconditioned PCG)
  double* ell_sval = nullptr;   // K D^-1 (Jacobi PCG, FP64)
  float* ell_sval32 = nullptr;  // K D^-1 (Jacobi PCG, FP32)
  double *ut = nullptr, *rhs = nullptr, *r = nullptr, *rhat = nullptr, *p = nullptr,
         *v = nullptr, *phat = nullptr, *shat = nullptr, *t = nullptr;
  double* phi_f = nullptr;
  int32_t* vpos = nullptr;              // lattice vertex rows: CSR positions
  int32_t* node_of = nullptr;           // [N_f] lattice node -> mesh node
  double* corr_v4 = nullptr;            // [N_f][4] correction inputs in lattice order
  uint8_t* mslot = nullptr;             // [N_f][8] lattice momentum rows: CSR offsets
  cgp::MomRow* mrow = nullptr;          // [N_f] their neighbour and triangle records
  cgp::MomTri* mtri = nullptr;          // [nT] coarse-triangle coefficients
  std::vector<cgp::MomRow> mrow_h;      // host copies (set-up)
  std::vector<cgp::MomTri> mtri_h;
  cgp::MomLattice mlat{};               // their launch description
  double* mrhs = nullptr;               // [3][N_f] mass-solve right-hand sides
  double* mx[3] = {nullptr, nullptr, nullptr};  // [3][N_f] Chebyshev iterates
  float* my[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};  // mixed form: [5][N_f][3]
  int cheb_iters = 0;
  // lattice layout of the mass solves (host structure and device view)
  cgp::Lattice lat;
  cgp::LatDev latd{};
  // coarse vectors: b_c, the PCG direction and alternating r, w, s (FP64 and
  // FP32), the refinement residual and a saved iterate
  double *bc = nullptr, *cr = nullptr, *cxsave = nullptr, *cp = nullptr;
  double *cr2[2] = {}, *cw2[2] = {}, *cs2[2] = {};
  float *cb32 = nullptr, *cx32 = nullptr, *cp32 = nullptr;
  float *cr32[2] = {}, *cw32[2] = {}, *cs32[2] = {};
  double* tripart = nullptr;
  double* part = nullptr;
  Scal* scal = nullptr;

  Scal* pinned = nullptr;  // [2][8] host-pinned copies of the solver scalars (caller's buffer)
  hipEvent_t ev[2] = {nullptr, nullptr};

  // learned initial guess
  cgp::net::Buffers net;
  __bf16* net_wb = nullptr;
  double* net_scal = nullptr;   // (s_b, s, s_1, s_2)
  double* net_dpart = nullptr;  // reduction scratch
  double* net_lpart = nullptr;
  float* net_loss = nullptr;
  int32_t* chose = nullptr;     // guard decision
  double* guess_tmp = nullptr;  // [N_c]
  double hbar = 1.0;

  // nested-dissection factor preconditioner (CGP_PRECOND_NDCHOL): host
  // structure, device view, and the PCG vectors z, p (alternating) and q
  cgp::NdFactor nd;
  cgp::NdDev ndd{};     // FP64 factor (precision CGP_FP64)
  cgp::NdDev32 ndd32{}; // FP32 factor (CGP_MIXED: the solve inside the refinement)
  float* nd_z32 = nullptr;
  double* nd_z = nullptr;
  double* nd_p[2] = {nullptr, nullptr};
  double* nd_q = nullptr;

  // s-step Jacobi-PCG (CGP_PRECOND_JACOBI_S4): host plan and device view
  cgp::CaPlan ca;
  cgp::CaDev cad{};

  // device address of the no-alloc scratch on the context's GPU (set by
  // cgp_assemble)
  double* scratch_dev = nullptr;

  // measurement hook (cgp_timing_enable)
  int timed_id = 0;
  std::vector<hipEvent_t> tev;
  size_t tev_used = 0;
};

namespace {

// Lays out the workspace; with base == nullptr it measures.
size_t carve(cgp_ctx* c, void* base) {
  Carver w(base);
  const size_t nf = c->nf, nc = c->nc;
  const size_t nnzf = c->h.gf.nnz(), nnzc = c->h.gc.nnz();
  int32_t* rp_f = w.take<int32_t>(nf + 1);
  int32_t* col_f = w.take<int32_t>(nnzf);
  int32_t* side_f = w.take<int32_t>(2 * nnzf);
  double2* xy_f = w.take<double2>(nf);
  c->tri_f = w.take<int32_t>(3 * (size_t)c->tf);
  c->pcode = w.take<int32_t>(2 * nf);
  c->dir_index = w.take<int32_t>(nf);
  c->Mval = w.take<double>(nnzf);
  c->Aval = w.take<double>(nnzf);
  c->invdA = w.take<double>(nf);
  int32_t* tile_f = w.take<int32_t>(c->h.gf.tile.size());
  double** vec2[] = {&c->ut, &c->rhs, &c->r, &c->rhat, &c->p, &c->v, &c->phat, &c->shat, &c->t};
  for (double** q : vec2) *q = w.take<double>(2 * nf);
  c->phi_f = w.take<double>(nf);
  {
    const cgp::Lattice& L = c->lat;
    cgp::LatDev& d = c->latd;
    d.m = L.m;
    d.nI = L.nI;
    d.nT = L.nT;
    d.nE = L.nE;
    d.nV = L.nV;
    d.EB = L.EB;
    d.VB = L.VB;
    d.tri_e = w.take<int32_t>(L.tri_e.size());
    d.edge_v = w.take<int32_t>(L.edge_v.size());
    d.edge_t = w.take<int32_t>(L.edge_t.size());
    d.af = w.take<double>(L.af.size());
    d.ldir = w.take<uint8_t>(L.ldir.size());
    d.lat_of = w.take<int32_t>(L.lat_of.size());
    d.vw = L.vw;
    d.vcol = w.take<int32_t>(L.vcol.size());
    d.vval = w.take<double>(L.vcol.size());
    d.erec = L.erec.empty() ? nullptr : w.take<cgp::LatEdgeRec>(L.erec.size());
    c->vpos = w.take<int32_t>(L.vpos.size());
    c->node_of = w.take<int32_t>(L.node_of.size());
    c->corr_v4 = w.take<double>(4 * L.node_of.size());
    c->mslot = w.take<uint8_t>(L.mslot.size());
    c->mrow = w.take<cgp::MomRow>(c->mrow_h.size());
    c->mtri = w.take<cgp::MomTri>(c->mtri_h.size());
  }
  c->mrhs = w.take<double>(3 * nf);
  if (c->prob.mass_mode == CGP_MASS_CONSISTENT_MIXED) {
    for (int k = 0; k < 5; ++k) c->my[k] = w.take<float>(3 * nf);
  } else {
    for (int k = 0; k < 3; ++k) c->mx[k] = w.take<double>(3 * nf);
  }

  int32_t* rp_c = w.take<int32_t>(nc + 1);
  int32_t* col_c = w.take<int32_t>(nnzc);
  int32_t* side_c = w.take<int32_t>(2 * nnzc);
  double2* xy_c = w.take<double2>(nc);
  c->tri_c = w.take<int32_t>(3 * (size_t)c->tc);
  c->cn_ptr = w.take<int32_t>(nc + 1);
  c->cn_tri = w.take<int32_t>(3 * (size_t)c->tc);
  c->nat_c = w.take<uint8_t>(nc);
  c->Kc = w.take<double>(nnzc);
  c->Kc32 = w.take<float>(nnzc);
  {
    int wmax = 1;
    const auto& rp = c->h.gc.rowptr;
    for (size_t i = 0; i + 1 < rp.size(); ++i) wmax = std::max(wmax, rp[i + 1] - rp[i]);
    c->ell_w = (wmax + cgp::kEllPad - 1) / cgp::kEllPad * cgp::kEllPad;
  }
  c->ell_col = w.take<int32_t>((size_t)c->ell_w * nc);
  c->ell_val = w.take<double>((size_t)c->ell_w * nc);
  c->ell_sval = w.take<double>((size_t)c->ell_w * nc);
  c->ell_sval32 = w.take<float>((size_t)c->ell_w * nc);
  c->Dxc = w.take<double>(nnzc);
  c->Dyc = w.take<double>(nnzc);
  c->invdKc = w.take<double>(nc);
  c->invdKc32 = w.take<float>(nc);
  c->lumped_c = w.take<double>(nc);
  int32_t* tile_c = w.take<int32_t>(c->h.gc.tile.size());
  double** cvec[] = {&c->bc,     &c->cr,     &c->cxsave, &c->cp,    &c->cr2[0],
                     &c->cr2[1], &c->cw2[0], &c->cw2[1], &c->cs2[0], &c->cs2[1]};
  for (double** q : cvec) *q = w.take<double>(nc);
  float** cvec32[] = {&c->cb32,     &c->cx32,     &c->cp32,     &c->cr32[0], &c->cr32[1],
                      &c->cw32[0], &c->cw32[1], &c->cs32[0], &c->cs32[1]};
  for (float** q : cvec32) *q = w.take<float>(nc);
  c->tripart = w.take<double>(3 * (size_t)c->tc);
  c->part = w.take<double>((size_t)cgp::kSlots * 2 * cgp::kNbMax);
  c->scal = w.take<Scal>(8);
  float* netf = w.take<float>(cgp::net::workspace_floats(c->nc, (int)nnzc));
  if (base) c->net.carve(netf, c->nc, (int)nnzc);
  c->net_wb = w.take<__bf16>(cgp::net::kWeightsB);
  c->net_scal = w.take<double>(4);
  c->net_dpart = w.take<double>(5 * cgp::kNbMax);
  c->net_lpart = w.take<double>(2 * cgp::kNbMax);
  c->net_loss = w.take<float>(4);
  c->chose = w.take<int32_t>(4);
  c->guess_tmp = w.take<double>(nc);
  if (c->prob.coarse_precond == CGP_PRECOND_NDCHOL) {
    const cgp::NdFactor& f = c->nd;
    cgp::NdDev& d = c->ndd;
    d.nfac = f.nfac;
    d.perm = w.take<int32_t>(f.perm.size());
    d.sn = w.take<cgp::NdSuper>(f.sn.size());
    d.rows = w.take<int32_t>(f.rows.size());
    d.gptr = w.take<int32_t>(f.gptr.size());
    d.gidx = w.take<int32_t>(f.gidx.size());
    d.fwd = w.take<cgp::NdItem>(f.fwd.size());
    d.bwd = w.take<cgp::NdItem>(f.bwd.size());
    if (c->prob.precision == CGP_FP64) {
      d.G = w.take<double>((size_t)f.g_entries);
      d.GT = w.take<double>((size_t)f.g_entries);
      d.Y = w.take<double>(f.nfac);
      d.X = w.take<double>(f.nfac);
      d.U = w.take<double>(f.n_upd);
      c->nd_z = w.take<double>(nc);
      c->nd_p[0] = w.take<double>(nc);
      c->nd_p[1] = w.take<double>(nc);
      c->nd_q = w.take<double>(nc);
    } else {
      // the same structure with FP32 values
      cgp::NdDev32& e = c->ndd32;
      e.nfac = d.nfac;
      e.perm = d.perm;
      e.sn = d.sn;
      e.rows = d.rows;
      e.gptr = d.gptr;
      e.gidx = d.gidx;
      e.fwd = d.fwd;
      e.bwd = d.bwd;
      e.G = w.take<float>((size_t)f.g_entries);
      e.GT = w.take<float>((size_t)f.g_entries);
      e.Y = w.take<float>(f.nfac);
      e.X = w.take<float>(f.nfac);
      e.U = w.take<float>(f.n_upd);
      c->nd_z32 = w.take<float>(nc);
    }
  }
  if (c->prob.coarse_precond == CGP_PRECOND_JACOBI_S4) {
    const cgp::CaPlan& pl = c->ca;
    cgp::CaDev& d = c->cad;
    d.n = c->nc;
    d.ntiles = pl.ntiles;
    d.ntiles_pad = pl.ntiles_pad;
    d.width = pl.width;
    d.perm = w.take<int32_t>(pl.perm.size());
    d.own_off = w.take<int32_t>(pl.own_off.size());
    d.ext_off = w.take<int32_t>(pl.ext_off.size());
    d.ext = w.take<int32_t>(pl.ext.size());
    d.layer = w.take<int32_t>(pl.layer.size());
    d.ell_off = w.take<int32_t>(pl.ell_off.size());
    d.ell_col = w.take<uint16_t>(pl.ell_col.size());
    d.ell_slot = w.take<int32_t>(pl.ell_slot.size());
    d.ell_val = w.take<double>(pl.ell_col.size());
    d.sq = w.take<double>(nc);
    d.xh = w.take<double>(nc);
    d.r0 = w.take<double>(nc);
    d.V[0] = w.take<double>((size_t)cgp::kCaM * nc);
    d.V[1] = w.take<double>((size_t)cgp::kCaM * nc);
    d.gpart = w.take<double>((size_t)2 * cgp::kCaNG * pl.ntiles_pad);
    d.spart = w.take<double>((size_t)2 * pl.ntiles_pad);
  }

  c->F = DLevel{c->nf, (int32_t)nnzf, rp_f, col_f, side_f, xy_f, tile_f, c->h.gf.ntiles()};
  c->latd.tri_v = c->tri_c;
  c->mlat = cgp::MomLattice{c->mslot, c->mrow, c->mtri, c->lat.nV};
  c->C = DLevel{c->nc, (int32_t)nnzc, rp_c, col_c, side_c, xy_c, tile_c, c->h.gc.ntiles()};
  return w.off + 256;
}

int check_ready(cgp_ctx* c) {
  if (!c) return fail(CGP_ERR_INVALID, "null context");
  if (!c->assembled) return fail(CGP_ERR_INVALID, "cgp_assemble has not been called");
  return CGP_OK;
}

hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

// Event pair for one launch of kernel `id` when it is the timed kernel.
hipEvent_t* timer(cgp_ctx* c, int id) {
  if (c->timed_id != id) return nullptr;
  while (c->tev.size() < c->tev_used + 2) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    c->tev.push_back(e);
  }
  hipEvent_t* p = c->tev.data() + c->tev_used;
  c->tev_used += 2;
  return p;
}

struct NoStop {
  bool operator()(const Scal*) const { return false; }
};

// Queues iterations 1..last of a Krylov solve through `launch(it, check_only)`
// in chunks, polling the stopping flags of the first `nrhs` scalars one chunk
// behind.  `last` = max_iter for PCG, max_iter + 1 for BiCGSTAB (whose final
// test runs at the start of the next iteration).  Copies the final scalars to
// `out`.  `stop(polled)` may end an unfinished solve early (the chunk already
// queued still runs); *launched receives the number of iterations queued.
template <class Launch, class Stop = NoStop>
int drive(cgp_ctx* c, Scal* sc, int nrhs, int last, int chunk, bool trailing_check,
          Launch launch, hipStream_t s, Scal* out, Stop stop = Stop(),
          int* launched = nullptr, int first = 0) {
  int it = 1, k = 0;
  bool have_prev = false;
  auto all_done = [&](int slot) {
    for (int d = 0; d < nrhs; ++d)
      if (c->pinned[8 * slot + d].done_stamp == 0) return false;
    return true;
  };
  if (first > 0) {
    // a first chunk of the expected length, polled before anything else is
    // queued (no speculative iterations when the expectation holds)
    const int hi = std::min(first, last);
    for (; it <= hi; ++it) launch(it, trailing_check && it == last);
    if (launched) *launched = it - 1;
    cgp::launch_mirror(sc, c->pinned, nrhs, s);
    HIPCHK(hipEventRecord(c->ev[0], s));
    HIPCHK(hipEventSynchronize(c->ev[0]));
    if (all_done(0) || it > last || stop(c->pinned)) {
      std::memcpy(out, c->pinned, sizeof(Scal) * nrhs);
      return CGP_OK;
    }
  }
  while (true) {
    const int hi = std::min(it + chunk - 1, last);
    for (; it <= hi; ++it) launch(it, trailing_check && it == last);
    if (launched) *launched = it - 1;
    cgp::launch_mirror(sc, c->pinned + 8 * k, nrhs, s);
    HIPCHK(hipEventRecord(c->ev[k], s));
    if (have_prev) {
      HIPCHK(hipEventSynchronize(c->ev[k ^ 1]));
      if (all_done(k ^ 1)) {
        std::memcpy(out, c->pinned + 8 * (k ^ 1), sizeof(Scal) * nrhs);
        return CGP_OK;
      }
      if (stop(c->pinned + 8 * (k ^ 1))) {
        HIPCHK(hipEventSynchronize(c->ev[k]));
        std::memcpy(out, c->pinned + 8 * k, sizeof(Scal) * nrhs);
        return CGP_OK;
      }
    }
    if (it > last) {
      HIPCHK(hipEventSynchronize(c->ev[k]));
      std::memcpy(out, c->pinned + 8 * k, sizeof(Scal) * nrhs);
      return CGP_OK;
    }
    have_prev = true;
    k ^= 1;
  }
}

int stats_status(const Scal* s, int nrhs, int max_iter, cgp_solve_stats* st) {
  int code = CGP_OK;
  for (int d = 0; d < nrhs; ++d) {
    const bool done = s[d].done_stamp != 0;
    if (s[d].status == 2) code = CGP_ERR_NAN;
    else if (!done && code == CGP_OK) code = CGP_NOT_CONVERGED;
    if (st) {
      st[d].iters = done ? s[d].iters : max_iter;
      st[d].outer_iters = 0;
      st[d].converged = done && s[d].status == 0;
      st[d].rel_res = s[d].rel;
    }
  }
  if (code == CGP_ERR_NAN) g_err = "solver produced NaN/Inf";
  if (code == CGP_NOT_CONVERGED) g_err = "iteration limit reached";
  return code;
}

int worst(int a, int b) {
  if (a < 0 || b < 0) return std::min(a, b);
  return std::max(a, b);
}

int run_momentum(cgp_ctx* c, const double* u_prev, const double* u, const double* p,
                 const double* u_dir, const double* f, const double* t_nat, double* ut,
                 cgp_solve_stats* st, hipStream_t s) {
  const cgp_problem& P = c->prob;
  // the assembly also forms the initial residual r = b - A x0 (x0 = W, the
  // boundary values on Dirichlet rows), so the solve starts without a product
  cgp::launch_momentum_assemble(c->F, c->dir_index, P.dt, P.nu, u_prev, u, p, u_dir, c->ndir,
                                f, t_nat, c->Aval, c->invdA, c->rhs, ut, c->r,
                                c->phat, c->shat, s, timer(c, CGP_K_MOM_ASSEMBLE),
                                c->lat.mom_ok ? &c->mlat : nullptr);
  cgp::BicgVecs V{ut, c->r, c->rhat, c->p, c->v, c->phat, c->shat, c->t, c->rhs, c->invdA};
  cgp::launch_bicg_start(c->nf, V, c->scal, c->part, c->nb_f, s);
  Scal out[2];
  const int last = P.mom_max_iter + 1;
  // the first chunk covers the previous solve's iterations plus the launch
  // that runs the final test
  const int first = c->mom_expect > 0 ? c->mom_expect + 1 : 0;
  int rc = drive(c, c->scal, 2, last, 4, true,
                 [&](int it, bool chk) {
                   cgp::launch_bicg_iter(c->F, c->Aval, V, c->scal, c->part, c->nb_f, it,
                                         P.mom_tol, chk, s, chk ? nullptr : timer(c, CGP_K_MOM_SPMV));
                 },
                 s, out, NoStop(), nullptr, first);
  if (rc) return rc;
  c->mom_expect = (out[0].done_stamp && out[1].done_stamp) ? std::max(out[0].iters, out[1].iters) : 0;
  return stats_status(out, 2, P.mom_max_iter, st);
}

int run_restrict(cgp_ctx* c, const double* ut, double* b, hipStream_t s) {
  // The restriction evaluates a divergence: for a nearly solenoidal U~ a sum of
  // nearly cancelling terms, so it runs in FP64 on both precision paths.
  const cgp_problem& P = c->prob;
  const double scale = -1.5 / P.dt;
  if (P.restrict_mode == CGP_RESTRICT_GALERKIN) {
    cgp::launch_restrict_galerkin(c->tri_f, c->tf, c->F.xy, P.levels, ut, c->nf, c->tripart, s);
    cgp::launch_restrict_nodes(c->nc, c->cn_ptr, c->cn_tri, c->tripart, c->nat_c, scale, b,
                               c->part, c->nb_c, s);
  } else {
    cgp::launch_restrict_inject(c->C, c->nat_c, ut, c->nf, scale, b, c->part, c->nb_c, s);
  }
  if (c->h.n_nat_c == 0) cgp::launch_remove_mean(c->nc, b, c->part, c->nb_c, nullptr, s);
  return CGP_OK;
}

// PCG preconditioned by the nested-dissection factor.  The FP64 residual is
// tested before the first iteration and after each one.  The first test and
// the first iteration are queued together (the iteration's kernels return at
// once if the test found the guess converged), so a solve that one iteration
// finishes, the usual case with the exact factor, costs one host poll.
int run_pcg_nd(cgp_ctx* c, const double* b, double* x, cgp_solve_stats* st, hipStream_t s) {
  const cgp_problem& P = c->prob;
  double* const pbuf[2] = {c->nd_p[0], c->nd_p[1]};
  Scal* const first = c->scal + 4;  // test of the guess
  Scal* const later = c->scal + 6;  // test after each iteration
  cgp::launch_residual64(c->C, c->Kc, b, x, c->cr, c->cb32, c->part, c->nb_c, s);
  cgp::launch_reduce_check(c->part, c->nb_c, P.pcg_tol, first, 0, s);
  cgp::launch_nd_solve(c->ndd, c->nd, c->cr, c->nd_z, s, first);
  cgp::launch_fpcg_iter(c->nc, c->ell_col, c->ell_val, c->ell_w, c->nd_z, pbuf, c->nd_q, x,
                        c->cr, c->scal + 5, c->part, c->nb_c, 1, s, first);
  cgp::launch_reduce_check(c->part, c->nb_c, P.pcg_tol, later, 1, s);
  cgp::launch_mirror(first, c->pinned, 3, s);
  HIPCHK(hipStreamSynchronize(s));
  int it = 0, rc = CGP_OK;
  Scal chk = c->pinned[0];
  if (chk.status != 2 && chk.bb != 0.0 && !chk.done_stamp) {
    it = 1;
    chk = c->pinned[2];
  }
  for (;;) {
    if (chk.status == 2) {
      rc = fail(CGP_ERR_NAN, "coarse PCG produced NaN/Inf");
      break;
    }
    if (chk.bb == 0.0) {  // zero right-hand side: the solution is zero
      cgp::launch_fill(x, 0.0, c->nc, s);
      break;
    }
    if (chk.done_stamp) break;
    if (it >= P.max_iter) {
      rc = fail(CGP_NOT_CONVERGED, "iteration limit reached");
      break;
    }
    ++it;
    cgp::launch_nd_solve(c->ndd, c->nd, c->cr, c->nd_z, s);
    cgp::launch_fpcg_iter(c->nc, c->ell_col, c->ell_val, c->ell_w, c->nd_z, pbuf, c->nd_q, x,
                          c->cr, c->scal + 5, c->part, c->nb_c, it, s);
    cgp::launch_reduce_check(c->part, c->nb_c, P.pcg_tol, later, it, s);
    cgp::launch_mirror(later, c->pinned, 1, s);
    HIPCHK(hipStreamSynchronize(s));
    chk = c->pinned[0];
  }
  if (st) {
    st->iters = it;
    st->outer_iters = 0;
    st->converged = rc == CGP_OK;
    st->rel_res = chk.rel;
  }
  return rc;
}

// Krylov vectors, partial sums and scalars of the FP64 Jacobi-PCG: the
// context's workspace, or the file-scope scratch of cgp_pcg_solve_noalloc.
struct JacobiBufs {
  double* p;
  double* r[2];
  double* w[2];
  double* s[2];
  double* part;
  Scal* scal;
  bool timed;  // honour cgp_timing_enable (its events are created on demand)
};

// FP64 Jacobi-PCG in the single-reduction form from the guess in x, one
// launch per iteration, the stopping flags polled one chunk behind.
int jacobi_pcg64(cgp_ctx* c, const double* b, double* x, cgp_solve_stats* st, hipStream_t s,
                 const JacobiBufs& B) {
  const cgp_problem& P = c->prob;
  cgp::PcgVecs<double> V{x,          B.p,         {B.r[0], B.r[1]},
                         {B.w[0], B.w[1]},        {B.s[0], B.s[1]},
                         b,          c->invdKc,   c->Kc,
                         c->ell_col, c->ell_sval, c->ell_w};
  cgp::launch_pcg_init<double>(c->C, V, false, B.scal, B.part, c->nb_c, s);
  Scal out[1];
  int rc = drive(c, B.scal, 1, P.max_iter + 1, 32, true,
                 [&](int it, bool chk) {
                   cgp::launch_pcg_iter<double>(
                       c->C, V, B.scal, B.part, c->nb_c, it, P.pcg_tol, chk, s,
                       (chk || !B.timed) ? nullptr : timer(c, CGP_K_COARSE_SPMV));
                 },
                 s, out);
  if (rc) return rc;
  return stats_status(out, 1, P.max_iter, st);
}

// Mixed precision with the factor: FP64 iterative refinement whose
// correction is the FP32 factor solve, x += L^-T L^-1 (float) r, r = b - K x
// in FP64 (each correction removes all but about kappa eps_32 of the error).
// The FP64 residual is tested before every correction.  Corrections are
// queued two at a time between host polls; a correction whose test found the
// solve done returns at once.
int run_pcg_nd_mixed(cgp_ctx* c, const double* b, double* x, cgp_solve_stats* st,
                     hipStream_t s) {
  const cgp_problem& P = c->prob;
  Scal* const chk = c->scal + 4;
  int queued = 0, rc = CGP_OK;
  Scal last{};
  const int cap = std::min(P.max_outer, P.max_iter);
  for (;;) {
    const int burst = queued == 0 ? 2 : 1;
    for (int k = 0; k < burst && queued < cap; ++k, ++queued) {
      cgp::launch_residual64(c->C, c->Kc, b, x, c->cr, c->cb32, c->part, c->nb_c, s);
      cgp::launch_reduce_check(c->part, c->nb_c, P.pcg_tol, chk, queued, s);
      cgp::launch_nd_solve<float>(c->ndd32, c->nd, c->cb32, c->nd_z32, s, chk);
      cgp::launch_axpy_f32(c->nd_z32, x, c->nc, s, chk);
    }
    cgp::launch_residual64(c->C, c->Kc, b, x, c->cr, c->cb32, c->part, c->nb_c, s);
    cgp::launch_reduce_check(c->part, c->nb_c, P.pcg_tol, chk, queued, s);
    cgp::launch_mirror(chk, c->pinned, 1, s);
    HIPCHK(hipStreamSynchronize(s));
    last = c->pinned[0];
    if (last.status == 2) {
      rc = fail(CGP_ERR_NAN, "mixed-precision refinement produced NaN/Inf");
      break;
    }
    if (last.done_stamp) break;
    if (queued >= cap) {
      rc = fail(CGP_NOT_CONVERGED, "refinement limit reached");
      break;
    }
  }
  // a check that finds the solve done stores (its index + 1); the
  // corrections before it were applied
  const int applied = last.done_stamp ? last.done_stamp - 1 : queued;
  if (st) {
    st->iters = applied;
    st->outer_iters = applied;
    st->converged = rc == CGP_OK;
    st->rel_res = last.rel;
  }
  return rc;
}

int run_pcg(cgp_ctx* c, const double* b, double* x, cgp_solve_stats* st, hipStream_t s) {
  const cgp_problem& P = c->prob;
  int rc = CGP_OK;
  if (c->h.n_nat_c) cgp::launch_zero_masked(x, c->nat_c, c->nc, s);
  if (P.coarse_precond == CGP_PRECOND_NDCHOL && P.precision == CGP_MIXED) {
    rc = run_pcg_nd_mixed(c, b, x, st, s);
    if (rc == CGP_ERR_HIP) return rc;
  } else if (P.coarse_precond == CGP_PRECOND_NDCHOL) {
    rc = run_pcg_nd(c, b, x, st, s);
  } else if (P.coarse_precond == CGP_PRECOND_JACOBI_S4) {
    // one launch per kCaS iterations (launch 1 tests the guess); the scalars
    // are polled every 8 launches, one chunk behind
    const cgp::CaDev& d = c->cad;
    cgp::launch_ca_start(d, c->ell_col, c->ell_val, c->ell_w, b, x, c->scal, s);
    Scal out[1];
    const int last = 1 + (P.max_iter + cgp::kCaS - 1) / cgp::kCaS;
    rc = drive(c, c->scal, 1, last, 8, false,
               [&](int o, bool) {
                 cgp::launch_ca_outer(d, c->scal, o, P.pcg_tol, P.max_iter, cgp::stamp(o, 1), s,
                                      timer(c, CGP_K_COARSE_SPMV));
               },
               s, out);
    if (rc) return rc;
    cgp::launch_ca_final(d, x, s);
    rc = stats_status(out, 1, P.max_iter, st);
  } else if (P.precision == CGP_FP64) {
    const JacobiBufs B{c->cp,    {c->cr2[0], c->cr2[1]}, {c->cw2[0], c->cw2[1]},
                       {c->cs2[0], c->cs2[1]}, c->part, c->scal, true};
    rc = jacobi_pcg64(c, b, x, st, s, B);
    if (rc == CGP_ERR_HIP) return rc;
  } else {
    // FP64 iterative refinement around FP32-inner Jacobi-PCG.  A correction
    // that does not halve the FP64 residual (the inner solve went below what
    // FP32 resolves on this operator) is undone and the inner tolerance floor
    // raised; the iterate is never left worse than the best one seen.
    int inner_total = 0, outer = 0;
    Scal chk{};
    bool converged = false, undone = false;
    double prev_rel = 0.0, eta_floor = P.inner_tol;
    double* xsave = c->cxsave;
    for (;;) {
      cgp::launch_residual64(c->C, c->Kc, b, x, c->cr, c->cb32, c->part, c->nb_c, s);
      cgp::launch_reduce_check(c->part, c->nb_c, P.pcg_tol, c->scal + 4, outer, s);
      cgp::launch_mirror(c->scal + 4, c->pinned, 1, s);
      HIPCHK(hipStreamSynchronize(s));
      chk = c->pinned[0];
      if (chk.status == 2 && outer == 0) {
        rc = fail(CGP_ERR_NAN, "mixed-precision refinement produced NaN/Inf");
        break;
      }
      if (chk.done_stamp) {
        converged = true;
        break;
      }
      if (outer > 0 && !undone && !(chk.rel <= 0.5 * prev_rel)) {
        cgp::launch_copy(xsave, x, c->nc, s);
        eta_floor *= 100.0;
        undone = true;
        if (eta_floor >= 0.1) {
          chk.rel = prev_rel;
          break;
        }
        continue;  // recompute the residual of the restored iterate
      }
      undone = false;
      prev_rel = chk.rel;
      if (outer >= P.max_outer || inner_total >= P.max_iter) break;
      cgp::launch_copy(x, xsave, c->nc, s);
      cgp::PcgVecs<float> V{c->cx32,     c->cp32,       {c->cr32[0], c->cr32[1]},
                            {c->cw32[0], c->cw32[1]}, {c->cs32[0], c->cs32[1]},
                            c->cb32,     c->invdKc32,   c->Kc32,
                            c->ell_col,  c->ell_sval32, c->ell_w};
      cgp::launch_pcg_init<float>(c->C, V, true, c->scal, c->part, c->nb_c, s);
      Scal out[1];
      const int budget = std::max(1, P.max_iter - inner_total);
      // reduce the residual just enough to reach pcg_tol (with margin), but
      // not below the floor
      const double eta = std::max(eta_floor, 0.3 * P.pcg_tol / std::max(chk.rel, 1e-300));
      // FP32 stagnation: once the recursive residual is below 1e-3 of the
      // inner right-hand side (where FP32's attainable accuracy can bind), it
      // has not halved in 8 polls.  Above that, long plateaus are ordinary CG
      // behaviour (the full channel mesh sits near 1 for ~300 iterations
      // before converging) and are not stopped.
      double best = 1e300;
      int since = 0, launched = 0;
      auto stalled = [&](const Scal* p) {
        if (p->rel < 0.5 * best) {
          best = p->rel;
          since = 0;
          return false;
        }
        return best <= 1e-3 && ++since >= 8;
      };
      int r2 = drive(c, c->scal, 1, budget + 1, 32, true,
                     [&](int it, bool chk2) {
                       cgp::launch_pcg_iter<float>(c->C, V, c->scal, c->part, c->nb_c, it, eta,
                                                   chk2, s);
                     },
                     s, out, stalled, &launched);
      if (r2) return r2;
      inner_total += out[0].done_stamp ? out[0].iters : std::min(launched, budget);
      ++outer;
      if (out[0].status == 2) {
        // no correction from a failed inner solve: demand less of FP32
        eta_floor *= 100.0;
        undone = true;
        if (eta_floor >= 0.1) {
          rc = fail(CGP_ERR_NAN, "inner FP32 solve produced NaN/Inf");
          break;
        }
        continue;
      }
      cgp::launch_axpy_f32(c->cx32, x, c->nc, s);
    }
    if (st) {
      st->iters = inner_total;
      st->outer_iters = outer;
      st->converged = converged;
      st->rel_res = chk.rel;
    }
    if (rc == CGP_OK && !converged) rc = fail(CGP_NOT_CONVERGED, "refinement limit reached");
  }
  if (c->h.n_nat_c == 0) {
    cgp::launch_weighted_sums(c->nc, x, c->lumped_c, c->part, c->nb_c, s);
    cgp::launch_remove_mean(c->nc, x, c->part, c->nb_c, c->lumped_c, s);
  }
  return rc;
}

hipEvent_t* cheb_timer(void* c, int which) {
  return timer(static_cast<cgp_ctx*>(c),
               which == cgp::kChebTimedPair ? CGP_K_MASS_PAIR : CGP_K_MASS_SPMV);
}

// phi_c: the coarse increment phi_f was prolonged from (Eq. 24), or nullptr
int run_correct(cgp_ctx* c, const double* ut, const double* phi_f, const double* p_in,
                double* u_out, double* p_out, cgp_solve_stats* st, hipStream_t s,
                const double* phi_c = nullptr) {
  const cgp_problem& P = c->prob;
  const int chi = P.chi;
  const int mode = P.mass_mode;
  // velocity: M dU = -(2/3) dt G phi_f on the non-Dirichlet nodes; rotational
  // form: M dp = -nu D U~ on all nodes.  Consistent M: one fused Chebyshev
  // solve; lumped M (Eq. 27 for p, and for U in mode LUMPED): a division by
  // the row sum 2 M_ii, fused into the right-hand-side kernel
  const bool mixed = mode == CGP_MASS_CONSISTENT_MIXED;
  const bool consistent = mode == CGP_MASS_CONSISTENT || mixed;
  const bool cheb_u = mode != CGP_MASS_LUMPED;
  const bool cheb_p = chi && consistent;
  const int nr = cheb_u ? (cheb_p ? 3 : 2) : 0;
  if (consistent) {
    // right-hand sides on the lattice layout, geometry from the coarse mesh
    const cgp::CorrLatArgs A{c->nf,      reinterpret_cast<const double*>(c->C.xy), c->cn_ptr,
                             c->cn_tri, c->corr_v4, phi_c, P.dt, P.nu, chi};
    if (!cgp::launch_correct_rhs_lattice(c->latd, c->node_of, phi_f, ut, A, c->mrhs,
                                         mixed ? c->my[3] : nullptr, s))
      return fail(CGP_ERR_INVALID, "correction right-hand side: misaligned buffer or unsupported lattice size");
  } else {
    cgp::launch_correct_rhs(c->F, c->dir_index, c->Mval, P.dt, P.nu, chi, mode, phi_f, ut, p_in,
                            c->mrhs, u_out, p_out, c->latd.lat_of, s);
  }
  if (st) {
    // a-priori bound of the Chebyshev iteration on [1/2, 2]; lumped: exact.
    // Mixed: two refinement steps, each reducing the error by the inner
    // bound plus an allowance of 8 float ulps for the float storage
    const double inner = 4.0 * std::pow(1.0 / 3.0, c->cheb_iters);
    const double bound = mixed ? std::pow(inner + 8.0 * 0x1p-24, 2) : inner;
    const int steps = mixed ? 2 * c->cheb_iters : c->cheb_iters;
    for (int d = 0; d < 3; ++d) {
      const bool solved = d < 2 ? cheb_u : cheb_p;
      st[d] = cgp_solve_stats{solved ? steps : 0, mixed && solved ? 2 : 0, 1, 0,
                              solved ? bound : 0.0};
    }
  }
  if (nr == 0) return CGP_OK;  // the kernel wrote U and P
  if (mixed) {
    const float* d1 = nullptr;
    const float* d2 = nullptr;
    if (!cgp::launch_cheb_mixed(c->latd, c->nf, c->mrhs, nr, c->my, c->cheb_iters, s,
                                (c->timed_id == CGP_K_MASS_SPMV || c->timed_id == CGP_K_MASS_PAIR)
                                    ? cheb_timer
                                    : nullptr,
                                c, &d1, &d2))
      return fail(CGP_ERR_INVALID, "mass solve: misaligned vectors or unsupported lattice size");
    cgp::launch_final_update2(c->nf, ut, d1, d2, p_in, phi_f, nr, true, u_out, p_out,
                              c->latd.lat_of, s);
    return CGP_OK;
  }
  const double* du = cgp::launch_cheb(c->latd, c->nf, c->mrhs, nr, c->mx, c->cheb_iters, s,
                                      (c->timed_id == CGP_K_MASS_SPMV || c->timed_id == CGP_K_MASS_PAIR) ? cheb_timer : nullptr, c);
  if (!du) return fail(CGP_ERR_INVALID, "mass solve: misaligned vectors or unsupported lattice size");
  // with the lumped pressure update the kernel above wrote P already
  cgp::launch_final_update(c->nf, ut, du, p_in, phi_f, nr, cheb_p || !chi, u_out, p_out,
                           c->latd.lat_of, s);
  return CGP_OK;
}

}  // namespace

extern "C" {

const char* cgp_last_error(void) { return g_err.c_str(); }

int cgp_create(const cgp_problem* prob, cgp_ctx** out) {
  if (!prob || !out) return fail(CGP_ERR_INVALID, "null argument");
  *out = nullptr;
  const cgp_mesh& m = prob->coarse;
  if (!m.xy || !m.tri || (m.n_bedges > 0 && (!m.bedge || !m.btag)) || m.n_nodes < 3 ||
      m.n_tris < 1 || m.n_bedges < 0)
    return fail(CGP_ERR_INVALID, "coarse mesh arrays missing or empty");
  if (prob->levels < 0 || prob->levels > 3) return fail(CGP_ERR_INVALID, "levels must be 0..3");
  if (prob->chi != 0 && prob->chi != 1) return fail(CGP_ERR_INVALID, "chi must be 0 or 1");
  if (prob->precision != CGP_FP64 && prob->precision != CGP_MIXED)
    return fail(CGP_ERR_INVALID, "precision must be CGP_FP64 or CGP_MIXED");
  if (prob->restrict_mode != CGP_RESTRICT_GALERKIN && prob->restrict_mode != CGP_RESTRICT_INJECT)
    return fail(CGP_ERR_INVALID, "unknown restrict_mode");
  if (!(prob->dt > 0) || !(prob->nu > 0) || !(prob->pcg_tol > 0) || !(prob->mom_tol > 0) ||
      !(prob->mass_tol > 0) || !(prob->inner_tol > 0) || prob->max_iter < 1 ||
      prob->mom_max_iter < 1 || prob->mass_max_iter < 1 || prob->max_outer < 1)
    return fail(CGP_ERR_INVALID, "dt, nu, tolerances and iteration caps must be positive");
  if (prob->mass_mode < CGP_MASS_CONSISTENT || prob->mass_mode > CGP_MASS_CONSISTENT_MIXED)
    return fail(CGP_ERR_INVALID, "unknown mass_mode");
  if (prob->coarse_precond != CGP_PRECOND_JACOBI && prob->coarse_precond != CGP_PRECOND_NDCHOL &&
      prob->coarse_precond != CGP_PRECOND_JACOBI_S4)
    return fail(CGP_ERR_INVALID, "unknown coarse_precond");
  if (prob->scheme != CGP_SCHEME_INCREMENTAL && prob->scheme != CGP_SCHEME_NONINCREMENTAL)
    return fail(CGP_ERR_INVALID, "unknown scheme");
  if (prob->scheme == CGP_SCHEME_NONINCREMENTAL && prob->chi != 0)
    return fail(CGP_ERR_INVALID, "the non-incremental scheme has no rotational form (chi = 0)");
  if (prob->coarse_precond == CGP_PRECOND_JACOBI_S4 && prob->precision != CGP_FP64)
    return fail(CGP_ERR_INVALID, "CGP_PRECOND_JACOBI_S4 requires precision CGP_FP64");
  cgp::Mesh cm;
  cm.n_nodes = m.n_nodes;
  cm.n_tris = m.n_tris;
  cm.xy.assign(m.xy, m.xy + 2 * (size_t)m.n_nodes);
  cm.tri.assign(m.tri, m.tri + 3 * (size_t)m.n_tris);
  if (m.n_bedges) {
    cm.bedge.assign(m.bedge, m.bedge + 2 * (size_t)m.n_bedges);
    cm.btag.assign(m.btag, m.btag + m.n_bedges);
  }
  cgp_ctx* c = new (std::nothrow) cgp_ctx();
  if (!c) return fail(CGP_ERR_INVALID, "out of host memory");
  c->prob = *prob;
  c->prob.coarse = cgp_mesh{};  // host pointers are not kept
  std::string err;
  try {
    err = cgp::build_hierarchy(cm, prob->levels, c->h);
  } catch (const std::exception& e) {
    err = std::string("host set-up failed: ") + e.what();
  }
  if (!err.empty()) {
    delete c;
    return fail(CGP_ERR_MESH, err);
  }
  try {
    err = cgp::build_lattice(c->h, c->lat);
    if (err.empty()) cgp::build_mom_slots(c->h, c->lat);
    if (err.empty() && c->lat.mom_ok) {
      // row records (mesh numbering) and coarse-triangle coefficients
      const cgp::Lattice& L = c->lat;
      const cgp::LatDev v = L.host_view();
      c->mrow_h.assign(L.lat_of.size(), cgp::MomRow{{-1, -1, -1, -1, -1, -1}, {-1, -1}});
      c->mtri_h.resize(L.nT);
      cgp::lat_dispatch(v.m, [&](auto lat) {
        constexpr int M = decltype(lat)::kM;
        for (int32_t i = L.nV; i < (int32_t)L.lat_of.size(); ++i)
          c->mrow_h[i] = cgp::mom_row_record<M>(v, L.node_of.data(), L.lat_of[i]);
        for (int32_t T = 0; T < L.nT; ++T)
          c->mtri_h[T] = cgp::mom_tri_coef<M>(v, c->h.coarse.xy.data(), T);
      });
    }
  } catch (const std::exception& e) {
    err = std::string("lattice set-up failed: ") + e.what();
  }
  if (!err.empty()) {
    delete c;
    return fail(CGP_ERR_MESH, err);
  }
  c->nf = c->h.fine.n_nodes;
  c->nc = c->h.coarse.n_nodes;
  c->tf = c->h.fine.n_tris;
  c->tc = c->h.coarse.n_tris;
  c->ndir = (int32_t)c->h.dir_nodes.size();
  c->nb_f = std::min(cgp::kNbMax, std::max(1, (c->nf + cgp::kBlock - 1) / cgp::kBlock));
  // the coarse PCG product kernel requires every block to own a tile
  // one row per thread in the PCG iteration kernel; the tiled kernels loop
  c->nb_c = std::min(cgp::kNbCoarse, std::max({1, c->h.gc.ntiles(),
                                            (c->nc + cgp::kBlock - 1) / cgp::kBlock}));
  {  // mean coarse edge length (scale of the learned guess's edge features)
    const cgp::Graph& g = c->h.gc;
    double sum = 0.0;
    int64_t cnt = 0;
    for (int32_t i = 0; i < c->nc; ++i)
      for (int32_t k = g.rowptr[i] + 1; k < g.rowptr[i + 1]; ++k) {
        const int32_t j = g.col[k];
        sum += std::hypot(c->h.coarse.xy[2 * j] - c->h.coarse.xy[2 * i],
                          c->h.coarse.xy[2 * j + 1] - c->h.coarse.xy[2 * i + 1]);
        ++cnt;
      }
    c->hbar = cnt ? sum / cnt : 1.0;
  }
  // mixed: each of the two float solves reduces the error to the square
  // root of mass_tol, with one step more for the float storage
  c->cheb_iters = prob->mass_mode == CGP_MASS_CONSISTENT_MIXED
                      ? cgp::cheb_iterations(std::sqrt(prob->mass_tol)) + 1
                      : cgp::cheb_iterations(prob->mass_tol);
  if (c->cheb_iters > prob->mass_max_iter) {
    delete c;
    return fail(CGP_ERR_INVALID, "mass_max_iter is below the Chebyshev count for mass_tol");
  }
  if (prob->coarse_precond == CGP_PRECOND_NDCHOL) {
    // phi = 0 nodes are not unknowns; without any, K_c is singular (constant
    // null space) and the last coarse node is pinned
    std::vector<uint8_t> skip(c->h.nat_c.begin(), c->h.nat_c.end());
    if (c->h.n_nat_c == 0) skip[c->nc - 1] = 1;
    try {
      err = cgp::nd_symbolic(c->nc, c->h.gc.rowptr, c->h.gc.col, c->h.coarse.xy.data(), skip,
                             c->nd);
    } catch (const std::exception& e) {
      err = std::string("coarse factor set-up failed: ") + e.what();
    }
    if (!err.empty()) {
      delete c;
      return fail(CGP_ERR_INVALID, err);
    }
  }
  if (prob->coarse_precond == CGP_PRECOND_JACOBI_S4) {
    try {
      err = cgp::ca_plan(c->nc, c->h.gc.rowptr, c->h.gc.col, c->h.coarse.xy.data(), cgp::kCaS,
                         cgp::kCaThreads, cgp::kCaExtMax, cgp::kCaEllMax, c->ca);
    } catch (const std::exception& e) {
      err = std::string("s-step plan failed: ") + e.what();
    }
    if (!err.empty()) {
      delete c;
      return fail(CGP_ERR_INVALID, "CGP_PRECOND_JACOBI_S4: " + err);
    }
  }
  c->ws_bytes = carve(c, nullptr);
  *out = c;
  return CGP_OK;
}

int cgp_query(const cgp_ctx* c, cgp_sizes* out) {
  if (!c || !out) return fail(CGP_ERR_INVALID, "null argument");
  out->n_fine = c->nf;
  out->n_coarse = c->nc;
  out->n_fine_tris = c->tf;
  out->n_coarse_tris = c->tc;
  out->nnz_fine = c->h.gf.nnz();
  out->nnz_coarse = c->h.gc.nnz();
  out->n_dirichlet = c->ndir;
  out->n_natural_coarse = c->h.n_nat_c;
  out->workspace_bytes = c->ws_bytes;
  out->host_bytes = kHostBytes;
  return CGP_OK;
}

int cgp_fine_nodes(const cgp_ctx* c, double* xy) {
  if (!c || !xy) return fail(CGP_ERR_INVALID, "null argument");
  std::memcpy(xy, c->h.fine.xy.data(), sizeof(double) * c->h.fine.xy.size());
  return CGP_OK;
}

int cgp_dirichlet_nodes(const cgp_ctx* c, int32_t* nodes) {
  if (!c || (!nodes && c->ndir)) return fail(CGP_ERR_INVALID, "null argument");
  if (c->ndir) std::memcpy(nodes, c->h.dir_nodes.data(), sizeof(int32_t) * c->ndir);
  return CGP_OK;
}

int cgp_assemble(cgp_ctx* c, void* ws, size_t bytes, void* host, size_t host_bytes,
                 void* stream) {
  if (!c) return fail(CGP_ERR_INVALID, "null context");
  if (!ws || bytes < c->ws_bytes)
    return fail(CGP_ERR_WORKSPACE, "workspace missing or smaller than cgp_query().workspace_bytes");
  if (reinterpret_cast<uintptr_t>(ws) & 255) return fail(CGP_ERR_WORKSPACE, "workspace must be 256-byte aligned");
  if (!host || host_bytes < kHostBytes)
    return fail(CGP_ERR_WORKSPACE, "host buffer missing or smaller than cgp_query().host_bytes");
  if (reinterpret_cast<uintptr_t>(host) & 63) return fail(CGP_ERR_WORKSPACE, "host buffer must be 64-byte aligned");
  hipStream_t s = as_stream(stream);
  carve(c, ws);
  auto up = [&](void* dst, const void* src, size_t n) -> hipError_t {
    return n ? hipMemcpyAsync(dst, src, n, hipMemcpyHostToDevice, s) : hipSuccess;
  };
  const cgp::Hierarchy& h = c->h;
  HIPCHK(up((void*)c->F.rowptr, h.gf.rowptr.data(), 4 * h.gf.rowptr.size()));
  HIPCHK(up((void*)c->F.col, h.gf.col.data(), 4 * h.gf.col.size()));
  HIPCHK(up((void*)c->F.side, h.gf.side.data(), 4 * h.gf.side.size()));
  HIPCHK(up((void*)c->F.xy, h.fine.xy.data(), 8 * h.fine.xy.size()));
  HIPCHK(up((void*)c->F.tile, h.gf.tile.data(), 4 * h.gf.tile.size()));
  HIPCHK(up((void*)c->C.tile, h.gc.tile.data(), 4 * h.gc.tile.size()));
  HIPCHK(up(c->tri_f, h.fine.tri.data(), 4 * h.fine.tri.size()));
  HIPCHK(up(c->pcode, h.pcode.data(), 4 * h.pcode.size()));
  HIPCHK(up(c->dir_index, h.dir_index.data(), 4 * h.dir_index.size()));
  HIPCHK(up((void*)c->C.rowptr, h.gc.rowptr.data(), 4 * h.gc.rowptr.size()));
  HIPCHK(up((void*)c->C.col, h.gc.col.data(), 4 * h.gc.col.size()));
  HIPCHK(up((void*)c->C.side, h.gc.side.data(), 4 * h.gc.side.size()));
  HIPCHK(up((void*)c->C.xy, h.coarse.xy.data(), 8 * h.coarse.xy.size()));
  HIPCHK(up(c->tri_c, h.coarse.tri.data(), 4 * h.coarse.tri.size()));
  HIPCHK(up(c->cn_ptr, h.cn_ptr.data(), 4 * h.cn_ptr.size()));
  HIPCHK(up(c->cn_tri, h.cn_tri.data(), 4 * h.cn_tri.size()));
  HIPCHK(up(c->nat_c, h.nat_c.data(), h.nat_c.size()));
  {
    const cgp::Lattice& L = c->lat;
    const cgp::LatDev& d = c->latd;
    HIPCHK(up((void*)d.tri_e, L.tri_e.data(), 4 * L.tri_e.size()));
    HIPCHK(up((void*)d.edge_v, L.edge_v.data(), 4 * L.edge_v.size()));
    HIPCHK(up((void*)d.edge_t, L.edge_t.data(), 4 * L.edge_t.size()));
    HIPCHK(up((void*)d.af, L.af.data(), 8 * L.af.size()));
    HIPCHK(up((void*)d.ldir, L.ldir.data(), L.ldir.size()));
    HIPCHK(up((void*)d.lat_of, L.lat_of.data(), 4 * L.lat_of.size()));
    HIPCHK(up((void*)d.vcol, L.vcol.data(), 4 * L.vcol.size()));
    if (d.erec)
      HIPCHK(up((void*)d.erec, L.erec.data(), sizeof(cgp::LatEdgeRec) * L.erec.size()));
    HIPCHK(up((void*)c->vpos, L.vpos.data(), 4 * L.vpos.size()));
    HIPCHK(up((void*)c->node_of, L.node_of.data(), 4 * L.node_of.size()));
    HIPCHK(up((void*)c->mslot, L.mslot.data(), L.mslot.size()));
    HIPCHK(up((void*)c->mrow, c->mrow_h.data(), sizeof(cgp::MomRow) * c->mrow_h.size()));
    HIPCHK(up((void*)c->mtri, c->mtri_h.data(), sizeof(cgp::MomTri) * c->mtri_h.size()));
  }
  c->pinned = static_cast<Scal*>(host);
  std::memset(c->pinned, 0, kHostBytes);
  if (int rc = scratch_address(&c->scratch_dev)) return rc;
  for (int k = 0; k < 2; ++k)
    if (!c->ev[k]) HIPCHK(hipEventCreateWithFlags(&c->ev[k], hipEventDisableTiming));
  HIPCHK(hipMemsetAsync(c->scal, 0, sizeof(Scal) * 8, s));
  cgp::launch_mass_assemble(c->F, c->Mval, s);
  cgp::launch_vertex_rows((int64_t)c->lat.vpos.size(), c->vpos, c->Mval,
                          const_cast<double*>(c->latd.vval), s);
  cgp::launch_coarse_assemble(c->C, c->nat_c, c->Kc, c->Kc32, c->Dxc, c->Dyc, c->invdKc,
                              c->invdKc32, c->lumped_c, s);
  cgp::launch_make_ell(c->C, c->Kc, c->invdKc, c->ell_w, c->ell_col, c->ell_val, c->ell_sval,
                       c->ell_sval32, s);
  cgp::net::launch_edge_features(c->C, c->hbar, c->net, s);
  if (c->prob.coarse_precond == CGP_PRECOND_JACOBI_S4) {
    const cgp::CaPlan& pl = c->ca;
    const cgp::CaDev& d = c->cad;
    HIPCHK(up((void*)d.perm, pl.perm.data(), 4 * pl.perm.size()));
    HIPCHK(up((void*)d.own_off, pl.own_off.data(), 4 * pl.own_off.size()));
    HIPCHK(up((void*)d.ext_off, pl.ext_off.data(), 4 * pl.ext_off.size()));
    HIPCHK(up((void*)d.ext, pl.ext.data(), 4 * pl.ext.size()));
    HIPCHK(up((void*)d.layer, pl.layer.data(), 4 * pl.layer.size()));
    HIPCHK(up((void*)d.ell_off, pl.ell_off.data(), 4 * pl.ell_off.size()));
    HIPCHK(up((void*)d.ell_col, pl.ell_col.data(), 2 * pl.ell_col.size()));
    HIPCHK(up((void*)d.ell_slot, pl.ell_slot.data(), 4 * pl.ell_slot.size()));
    cgp::launch_ca_setup(d, c->C.rowptr, c->Kc, s);
  }
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(s));
  if (c->prob.coarse_precond == CGP_PRECOND_NDCHOL) {
    // factor the K_c just assembled (its own rounding), upload the factor
    cgp::NdFactor& f = c->nd;
    std::vector<double> kc(h.gc.nnz());
    HIPCHK(hipMemcpyAsync(kc.data(), c->Kc, sizeof(double) * kc.size(), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    std::string err;
    try {
      err = cgp::nd_numeric(h.gc.rowptr, h.gc.col, kc.data(), f);
    } catch (const std::exception& e) {
      err = std::string("coarse factorisation failed: ") + e.what();
    }
    if (!err.empty()) return fail(CGP_ERR_INVALID, err);
    const cgp::NdDev& d = c->ndd;
    HIPCHK(up((void*)d.perm, f.perm.data(), sizeof(int32_t) * f.perm.size()));
    HIPCHK(up((void*)d.sn, f.sn.data(), sizeof(cgp::NdSuper) * f.sn.size()));
    HIPCHK(up((void*)d.rows, f.rows.data(), sizeof(int32_t) * f.rows.size()));
    HIPCHK(up((void*)d.gptr, f.gptr.data(), sizeof(int32_t) * f.gptr.size()));
    HIPCHK(up((void*)d.gidx, f.gidx.data(), sizeof(int32_t) * f.gidx.size()));
    HIPCHK(up((void*)d.fwd, f.fwd.data(), sizeof(cgp::NdItem) * f.fwd.size()));
    HIPCHK(up((void*)d.bwd, f.bwd.data(), sizeof(cgp::NdItem) * f.bwd.size()));
    if (c->prob.precision == CGP_FP64) {
      HIPCHK(up((void*)d.G, f.G.data(), sizeof(double) * f.G.size()));
      HIPCHK(up((void*)d.GT, f.GT.data(), sizeof(double) * f.GT.size()));
      // z is written at the factored unknowns only: zero once
      cgp::launch_fill(c->nd_z, 0.0, c->nc, s);
      HIPCHK(hipGetLastError());
      HIPCHK(hipStreamSynchronize(s));
    } else {
      // the FP64 factor rounded to FP32 for the solve inside the refinement
      const cgp::NdDev32& e = c->ndd32;
      std::vector<float> g32(f.G.begin(), f.G.end()), gt32(f.GT.begin(), f.GT.end());
      HIPCHK(up((void*)e.G, g32.data(), sizeof(float) * g32.size()));
      HIPCHK(up((void*)e.GT, gt32.data(), sizeof(float) * gt32.size()));
      cgp::launch_fill32(c->nd_z32, 0.0f, c->nc, s);
      HIPCHK(hipGetLastError());
      HIPCHK(hipStreamSynchronize(s));
    }
    std::vector<double>().swap(f.G);
    std::vector<double>().swap(f.GT);
  }
  c->assembled = true;
  return CGP_OK;
}

int cgp_momentum(cgp_ctx* c, const double* u_prev, const double* u, const double* p,
                 const double* u_dir, const double* f, const double* t_nat, double* u_tilde,
                 cgp_solve_stats st[2], void* stream) {
  if (int rc = check_ready(c)) return rc;
  const bool noninc = c->prob.scheme == CGP_SCHEME_NONINCREMENTAL;
  if (!u_prev || !u || (!p && !noninc) || !u_tilde || (c->ndir && !u_dir))
    return fail(CGP_ERR_INVALID, "null device pointer");
  if (u_tilde == u || u_tilde == u_prev) return fail(CGP_ERR_INVALID, "u_tilde aliases an input");
  hipStream_t s = as_stream(stream);
  if (t_nat && c->h.n_nat_c == 0) return fail(CGP_ERR_INVALID, "traction given but no boundary is natural");
  int rc = run_momentum(c, u_prev, u, noninc ? nullptr : p, u_dir, f, t_nat, u_tilde, st, s);
  HIPCHK(hipGetLastError());
  return rc;
}

int cgp_restrict(cgp_ctx* c, const double* ut, double* b, void* stream) {
  if (int rc = check_ready(c)) return rc;
  if (!ut || !b) return fail(CGP_ERR_INVALID, "null device pointer");
  run_restrict(c, ut, b, as_stream(stream));
  HIPCHK(hipGetLastError());
  return CGP_OK;
}

int cgp_pcg_solve(cgp_ctx* c, const double* b, double* phi, cgp_solve_stats* st, void* stream) {
  if (int rc = check_ready(c)) return rc;
  if (!b || !phi) return fail(CGP_ERR_INVALID, "null device pointer");
  if (b == phi) return fail(CGP_ERR_INVALID, "b_c and phi_c alias");
  int rc = run_pcg(c, b, phi, st, as_stream(stream));
  HIPCHK(hipGetLastError());
  return rc;
}

int cgp_pcg_solve_noalloc(cgp_ctx* c, const double* b, double* phi, cgp_solve_stats* st,
                          void* stream) {
  if (int rc = check_ready(c)) return rc;
  if (!b || !phi) return fail(CGP_ERR_INVALID, "null device pointer");
  if (b == phi) return fail(CGP_ERR_INVALID, "b_c and phi_c alias");
  if (c->prob.coarse_precond != CGP_PRECOND_JACOBI || c->prob.precision != CGP_FP64)
    return fail(CGP_ERR_INVALID,
                "cgp_pcg_solve_noalloc: needs coarse_precond CGP_PRECOND_JACOBI and CGP_FP64");
  if (c->nc > kNoAllocMaxRows)
    return fail(CGP_ERR_WORKSPACE, "cgp_pcg_solve_noalloc: " + std::to_string(c->nc) +
                                       " coarse unknowns exceed the scratch maximum of " +
                                       std::to_string(kNoAllocMaxRows));
  if (!c->scratch_dev) return fail(CGP_ERR_INVALID, "no scratch address (cgp_assemble)");
  hipStream_t s = as_stream(stream);
  double* base = c->scratch_dev;
  const size_t n = kNoAllocMaxRows;
  double* v = base + kScrVec;
  // every vector entry read is written first in the same solve, the partial
  // sums are stored by every block before they are summed, and the start
  // kernel resets the scalars: no clearing is needed
  const JacobiBufs B{v, {v + n, v + 2 * n}, {v + 3 * n, v + 4 * n}, {v + 5 * n, v + 6 * n},
                     base + kScrPart, reinterpret_cast<Scal*>(base + kScrScal), false};
  if (c->h.n_nat_c) cgp::launch_zero_masked(phi, c->nat_c, c->nc, s);
  int rc = jacobi_pcg64(c, b, phi, st, s, B);
  if (rc == CGP_ERR_HIP) return rc;
  if (c->h.n_nat_c == 0) {
    cgp::launch_weighted_sums(c->nc, phi, c->lumped_c, B.part, c->nb_c, s);
    cgp::launch_remove_mean(c->nc, phi, B.part, c->nb_c, c->lumped_c, s);
  }
  HIPCHK(hipGetLastError());
  return rc;
}

int cgp_prolong(cgp_ctx* c, const double* phic, double* phif, void* stream) {
  if (int rc = check_ready(c)) return rc;
  if (!phic || !phif) return fail(CGP_ERR_INVALID, "null device pointer");
  cgp::launch_prolong(c->nf, c->pcode, c->tri_c, c->prob.levels, phic, phif, as_stream(stream));
  HIPCHK(hipGetLastError());
  return CGP_OK;
}

int cgp_correct(cgp_ctx* c, const double* ut, const double* phi_f, const double* p_in,
                double* u_out, double* p_out, cgp_solve_stats st[3], void* stream) {
  if (int rc = check_ready(c)) return rc;
  const bool noninc = c->prob.scheme == CGP_SCHEME_NONINCREMENTAL;
  if (!ut || !phi_f || (!p_in && !noninc) || !u_out || !p_out)
    return fail(CGP_ERR_INVALID, "null device pointer");
  if (u_out == ut) return fail(CGP_ERR_INVALID, "u_out aliases u_tilde");
  int rc = run_correct(c, ut, phi_f, noninc ? nullptr : p_in, u_out, p_out, st, as_stream(stream));
  HIPCHK(hipGetLastError());
  return rc;
}

}  // extern "C"

namespace {

// The values of the lattice's coarse-vertex rows from a host CSR matrix in
// mesh numbering (rows 0 .. nV-1): every entry of those rows must be one of
// the table's columns and every table column an entry.
bool host_vertex_rows(const cgp::Lattice& L, int32_t n, const int32_t* rowptr, const int32_t* col,
                      const double* mval, std::vector<double>& vval) {
  vval.assign(L.vcol.size(), 0.0);
  std::vector<uint8_t> hit(L.vcol.size(), 0);
  for (int32_t v = 0; v < L.nV; ++v)
    for (int32_t s = rowptr[v]; s < rowptr[v + 1]; ++s) {
      if (col[s] < 0 || col[s] >= n) return false;
      const int32_t lc = L.lat_of[col[s]];
      int32_t k = 0;
      while (k < L.vw && !(L.vcol[(size_t)k * L.nV + v] == lc && L.vpos[(size_t)k * L.nV + v] >= 0 &&
                           !hit[(size_t)k * L.nV + v]))
        ++k;
      if (k == L.vw) return false;
      hit[(size_t)k * L.nV + v] = 1;
      vval[(size_t)k * L.nV + v] = mval[s];
    }
  for (size_t k = 0; k < hit.size(); ++k)
    if (L.vpos[k] >= 0 && !hit[k]) return false;
  return true;
}

// One Chebyshev step over the lattice nodes [l0, l1) as the single-step
// kernel computes it: out = x + ca (x - xm) + cb D^-1 (b - M x), values
// stored as T and combined in FP64.
template <typename T, int NR>
bool cheb_single_host(const cgp::LatDev& v, int32_t n, int32_t l0, int32_t l1, const T* b,
                      const T* xm, const T* x, double ca, double cb, T* out) {
  bool ok = true;
  for (int32_t l = l0; l < l1; ++l) {
    double y[NR], dg;
    cgp::lat_apply<NR, cgp::kCh2M>(v, l,
                                   [&](int32_t k, int d) {
                                     if (k < 0 || k >= n) {
                                       ok = false;
                                       return 0.0;
                                     }
                                     return (double)x[(int64_t)k * NR + d];
                                   },
                                   y, dg);
    const bool masked = v.ldir[l] != 0;
    const double di = 1.0 / dg;
    for (int d = 0; d < NR; ++d) {
      const double xl = x[(int64_t)l * NR + d];
      out[(int64_t)l * NR + d] =
          (T)((d < 2 && masked) ? 0.0
                                : xl + ca * (xl - (double)xm[(int64_t)l * NR + d]) +
                                      cb * di * ((double)b[(int64_t)l * NR + d] - y[d]));
    }
  }
  return ok;
}

// A whole mass solve of `iters` Chebyshev steps on the host, launch by
// launch as the device solve runs it: a first step on every node (x_0 = 0),
// then with pairs (lattice size 8) the step pairs -- a single step over
// [EB & ~3, n), the interior kernel block by block (each phase for every
// thread before the next), a single step again -- and single steps on every
// node for the rest; without pairs single steps throughout.  Lattice-ordered
// vectors stored as T; the three iterate buffers start as NaN, so a value
// read before any launch wrote it shows up in the result.
template <typename T, int NR>
bool cheb_solve_host(const cgp::LatDev& v, int32_t n, const T* b, int iters, bool pairs,
                     T* out) {
  using namespace cgp;
  constexpr int kPer = 16 / (int)sizeof(T);
  const size_t len = (size_t)n * NR;
  std::vector<T> xs[3];
  for (auto& x : xs) x.assign(len, (T)std::nan(""));
  T* x[3] = {xs[0].data(), xs[1].data(), xs[2].data()};
  // (ca_k, cb_k) of the three-term recurrence on [1/2, 2]
  std::vector<double> ca(iters), cb(iters);
  {
    const double theta = 1.25, delta = 0.75, sigma = theta / delta;
    double rho = 1.0 / sigma;
    for (int k = 0; k < iters; ++k) {
      ca[k] = 0.0;
      cb[k] = 1.0 / theta;
      if (k > 0) {
        const double rn = 1.0 / (2.0 * sigma - rho);
        ca[k] = rn * rho;
        cb[k] = 2.0 * rn / delta;
        rho = rn;
      }
    }
  }
  for (int32_t l = 0; l < n; ++l) {
    const double di = 1.0 / lat_diag(v, l);
    const bool masked = v.ldir[l] != 0;
    for (int d = 0; d < NR; ++d) {
      x[1][(int64_t)l * NR + d] = (T)((d < 2 && masked) ? 0.0 : cb[0] * di * (double)b[(int64_t)l * NR + d]);
      x[0][(int64_t)l * NR + d] = (T)0;
    }
  }
  bool ok = true;
  ch2_fault = false;
  auto cp16 = [](const T* src, T* dst) {
    for (int j = 0; j < kPer; ++j) dst[j] = src[j];
  };
  static constexpr Ch2NbTable nbt = ch2_make_nb_table();
  auto S = std::make_unique<Cheb2Shared<T, NR>>();
  const int32_t lb = v.EB & ~3;
  const int nblk = (v.nT + kCh2Tris - 1) / kCh2Tris;
  for (int k = 1; k < iters;) {
    if (!pairs || k + 1 >= iters) {
      ok = ok && cheb_single_host<T, NR>(v, n, 0, n, b, x[(k + 2) % 3], x[k % 3], ca[k], cb[k],
                                         x[(k + 1) % 3]);
      k += 1;
      continue;
    }
    ok = ok && cheb_single_host<T, NR>(v, n, lb, n, b, x[(k + 2) % 3], x[k % 3], ca[k], cb[k],
                                       x[(k + 1) % 3]);
    const Cheb2Args<T> A{n, b, x[(k + 2) % 3], x[k % 3], x[(k + 1) % 3], x[(k + 2) % 3],
                         ca[k], cb[k], ca[k + 1], cb[k + 1]};
    for (int blk = 0; blk < nblk; ++blk) {
      std::fill_n(reinterpret_cast<T*>(S.get()), sizeof(Cheb2Shared<T, NR>) / sizeof(T),
                  (T)std::nan(""));
      for (int t = 0; t < kCh2Threads; ++t) ch2_stage<T, NR>(v, A, blk, t, *S, cp16, cp16);
      for (int t = 0; t < kCh2Threads; ++t) ch2_step1<T, NR>(v, A, blk, t, nbt.w, *S);
      for (int t = 0; t < kCh2Threads; ++t) ch2_step2<T, NR>(v, A, blk, t, nbt.w, *S);
      for (int t = 0; t < kCh2Threads; ++t) ch2_write<T, NR>(v, A, blk, t, *S, cp16);
    }
    ok = ok && cheb_single_host<T, NR>(v, n, lb, n, b, x[k % 3], x[(k + 1) % 3], ca[k + 1],
                                       cb[k + 1], x[(k + 2) % 3]);
    k += 2;
  }
  ok = ok && !ch2_fault;
  std::copy(x[iters % 3], x[iters % 3] + len, out);
  return ok;
}

// The mixed-precision solve as the device runs it: float solve of b's float
// copy (d1), FP64 residual r = b - M d1 stored as float, float solve of r
// (d2); x = d1 + d2 in FP64.
template <int NR>
bool cheb_mixed_host(const cgp::LatDev& v, int32_t n, const double* b, int iters, bool pairs,
                     double* out) {
  const size_t len = (size_t)n * NR;
  std::vector<float> b32(len), d1(len), r32(len), d2(len);
  for (size_t i = 0; i < len; ++i) b32[i] = (float)b[i];
  bool ok = cheb_solve_host<float, NR>(v, n, b32.data(), iters, pairs, d1.data());
  for (int32_t l = 0; l < n; ++l) {
    double y[NR], dg;
    cgp::lat_apply<NR, cgp::kCh2M>(v, l,
                                   [&](int32_t k, int d) {
                                     if (k < 0 || k >= n) {
                                       ok = false;
                                       return 0.0;
                                     }
                                     return (double)d1[(size_t)k * NR + d];
                                   },
                                   y, dg);
    const bool masked = v.ldir[l] != 0;
    for (int d = 0; d < NR; ++d)
      r32[(size_t)l * NR + d] = (d < 2 && masked) ? 0.0f : (float)(b[(size_t)l * NR + d] - y[d]);
  }
  ok = ok && cheb_solve_host<float, NR>(v, n, r32.data(), iters, pairs, d2.data());
  for (size_t i = 0; i < len; ++i) out[i] = (double)d1[i] + (double)d2[i];
  return ok;
}

}  // namespace

extern "C" {

int cgp_lattice_mass_apply_host(const cgp_ctx* c, const int32_t* rowptr, const int32_t* col,
                                const double* mval, const double* x, double* y, double* diag) {
  if (!c || !rowptr || !col || !mval || !x || !y || !diag) return fail(CGP_ERR_INVALID, "null argument");
  const cgp::Lattice& L = c->lat;
  cgp::LatDev v = L.host_view();
  const int32_t n = c->nf;
  std::vector<double> vval;
  if (!host_vertex_rows(L, n, rowptr, col, mval, vval))
    return fail(CGP_ERR_INVALID, "vertex rows: column out of range or entries differ");
  v.vval = vval.data();
  std::vector<double> xl(n);
  std::vector<int32_t> node(n);
  for (int32_t i = 0; i < n; ++i) {
    xl[L.lat_of[i]] = x[i];
    node[L.lat_of[i]] = i;
  }
  bool in_range = true, diag_ok = true;
  const bool known = cgp::lat_dispatch(v.m, [&](auto lat) {
    constexpr int M = decltype(lat)::kM;
    for (int32_t l = 0; l < n; ++l) {
      double yy[1], dg;
      cgp::lat_apply<1, M>(v, l,
                           [&](int32_t k, int) {
                             if (k < 0 || k >= n) {
                               in_range = false;
                               return 0.0;
                             }
                             return xl[k];
                           },
                           yy, dg);
      y[node[l]] = yy[0];
      diag[node[l]] = dg;
      if (cgp::lat_diag(v, l) != dg) diag_ok = false;
    }
  });
  if (!known) return fail(CGP_ERR_INVALID, "unsupported lattice size");
  if (!in_range) return fail(CGP_ERR_INVALID, "lattice stencil index out of range");
  if (!diag_ok) return fail(CGP_ERR_INVALID, "lattice diagonals disagree");
  return CGP_OK;
}

int cgp_lattice_cheb_solve_host(const cgp_ctx* c, const int32_t* rowptr, const int32_t* col,
                                const double* mval, int32_t nr, const double* b, int32_t iters,
                                int32_t pairs, int32_t mixed, double* x) {
  if (!c || !rowptr || !col || !mval || !b || !x) return fail(CGP_ERR_INVALID, "null argument");
  if (nr != 2 && nr != 3) return fail(CGP_ERR_INVALID, "nr must be 2 or 3");
  if (iters < 1 || iters > 1000) return fail(CGP_ERR_INVALID, "iters must be 1..1000");
  const cgp::Lattice& L = c->lat;
  if (pairs && L.m != cgp::kCh2M) return fail(CGP_ERR_INVALID, "step pairs need lattice size 8");
  if (!pairs && L.m != cgp::kCh2M) return fail(CGP_ERR_INVALID, "the host solve needs lattice size 8");
  cgp::LatDev v = L.host_view();
  const int32_t n = c->nf;
  std::vector<double> vval;
  if (!host_vertex_rows(L, n, rowptr, col, mval, vval))
    return fail(CGP_ERR_INVALID, "vertex rows: column out of range or entries differ");
  v.vval = vval.data();
  const size_t len = (size_t)n * nr;
  std::vector<double> bl(len), xl(len);
  for (int32_t i = 0; i < n; ++i)
    for (int d = 0; d < nr; ++d) bl[(size_t)L.lat_of[i] * nr + d] = b[(size_t)i * nr + d];
  bool ok;
  if (mixed)
    ok = nr == 3 ? cheb_mixed_host<3>(v, n, bl.data(), iters, pairs != 0, xl.data())
                 : cheb_mixed_host<2>(v, n, bl.data(), iters, pairs != 0, xl.data());
  else
    ok = nr == 3 ? cheb_solve_host<double, 3>(v, n, bl.data(), iters, pairs != 0, xl.data())
                 : cheb_solve_host<double, 2>(v, n, bl.data(), iters, pairs != 0, xl.data());
  if (!ok) return fail(CGP_ERR_INVALID, "mass solve: index out of range");
  for (int32_t i = 0; i < n; ++i)
    for (int d = 0; d < nr; ++d) x[(size_t)i * nr + d] = xl[(size_t)L.lat_of[i] * nr + d];
  return CGP_OK;
}

int cgp_lattice_correct_rhs_host(const cgp_ctx* c, const double* phi_f, const double* phi_c,
                                 const double* u_tilde, double* rhs) {
  if (!c || (!phi_f && !phi_c) || !u_tilde || !rhs) return fail(CGP_ERR_INVALID, "null argument");
  const cgp::Lattice& L = c->lat;
  const cgp::LatDev v = L.host_view();
  const int32_t n = c->nf;
  std::vector<double> v4(4 * (size_t)n);
  cgp::corr_fault = false;
  for (int32_t l = 0; l < n; ++l)
    cgp::corr_gather(n, L.node_of.data(), phi_c ? nullptr : phi_f, u_tilde, l, v4.data());
  const cgp::CorrLatArgs A{n,         c->h.coarse.xy.data(), c->h.cn_ptr.data(), c->h.cn_tri.data(),
                           v4.data(), phi_c, c->prob.dt, c->prob.nu, c->prob.chi};
  const bool known = cgp::lat_dispatch(v.m, [&](auto lat) {
    constexpr int M = decltype(lat)::kM;
    for (int32_t l = 0; l < n; ++l) {
      double out[3];
      if (phi_c)
        cgp::corr_node<M, true>(v, A, l, out);
      else
        cgp::corr_node<M, false>(v, A, l, out);
      const int32_t i = L.node_of[l];
      for (int d = 0; d < 3; ++d) rhs[3 * (int64_t)i + d] = out[d];
    }
  });
  if (!known) return fail(CGP_ERR_INVALID, "unsupported lattice size");
  if (cgp::corr_fault) return fail(CGP_ERR_INVALID, "correction stencil index out of range");
  return CGP_OK;
}

int cgp_lattice_momentum_host(const cgp_ctx* c, const double* u_prev, const double* u,
                              const double* p, const double* u_dir, const double* f,
                              const double* t_nat, int32_t* rowptr, int32_t* col, double* aval,
                              double* rhs, double* x0, double* r0) {
  if (!c || !u_prev || !u || !u_dir || !rowptr || !col || !aval || !rhs || !x0 || !r0)
    return fail(CGP_ERR_INVALID, "null argument");
  const cgp::Lattice& L = c->lat;
  if (!L.mom_ok) return fail(CGP_ERR_INVALID, "no lattice form of the momentum rows on this context");
  const cgp::Graph& g = c->h.gf;
  const int32_t n = c->nf;
  const size_t nnz = g.col.size();
  std::copy(g.rowptr.begin(), g.rowptr.end(), rowptr);
  std::copy(g.col.begin(), g.col.end(), col);
  const double nan = std::nan("");
  std::fill_n(aval, nnz, nan);
  std::fill_n(rhs, 2 * (size_t)n, nan);
  std::fill_n(x0, 2 * (size_t)n, nan);
  std::fill_n(r0, 2 * (size_t)n, nan);
  std::vector<double> invd(n, nan);
  // the fields of the assembly pre-pass
  const double dt = c->prob.dt;
  std::vector<double2> W(n), R(n);
  for (int32_t i = 0; i < n; ++i) {
    const double ux = u[i], uy = u[n + i], px = u_prev[i], py = u_prev[n + i];
    double rx = 2.0 * ux - 0.5 * px, ry = 2.0 * uy - 0.5 * py;
    if (f) {
      rx += dt * f[i];
      ry += dt * f[n + i];
    }
    W[i] = make_double2(2.0 * ux - px, 2.0 * uy - py);
    R[i] = make_double2(rx, ry);
  }
  const cgp::MomLatArgs A{n, L.nV, g.rowptr.data(), L.mslot.data(), c->mrow_h.data(),
                          c->mtri_h.data(), c->h.dir_index.data(), W.data(), R.data(), p, u_dir,
                          c->ndir, t_nat, dt, dt * c->prob.nu, aval, invd.data(), rhs, x0, r0};
  auto put = [&](int32_t s, double val) { aval[s] = val; };
  for (int32_t i = L.nV; i < n; ++i) {
    if (t_nat)
      cgp::mom_row<true>(A, i, put);
    else
      cgp::mom_row<false>(A, i, put);
  }
  return CGP_OK;
}

int cgp_query_ndchol(const cgp_ctx* c, cgp_ndchol_info* out) {
  if (!c || !out) return fail(CGP_ERR_INVALID, "null argument");
  const cgp::NdFactor& f = c->nd;
  out->n_factored = f.nfac;
  out->n_supernodes = (int32_t)f.sn.size();
  out->height = f.height;
  out->max_front = f.max_front;
  out->g_entries = f.g_entries;
  return CGP_OK;
}

int cgp_ca_plan_host(int32_t n, const int32_t* rowptr, const int32_t* col, const double* xy,
                     int32_t* perm, int32_t* own_off, int32_t* info) {
  if (n < 1 || !rowptr || !col || !xy || !perm || !own_off || !info)
    return fail(CGP_ERR_INVALID, "null or empty argument");
  if (rowptr[0] != 0) return fail(CGP_ERR_INVALID, "rowptr[0] must be 0");
  for (int32_t i = 0; i < n; ++i)
    if (rowptr[i + 1] <= rowptr[i]) return fail(CGP_ERR_INVALID, "every row needs its diagonal");
  std::vector<int32_t> rp(rowptr, rowptr + n + 1), cl(col, col + rowptr[n]);
  for (int32_t j : cl)
    if (j < 0 || j >= n) return fail(CGP_ERR_INVALID, "column out of range");
  for (int64_t i = 0; i < 2 * (int64_t)n; ++i)
    if (!std::isfinite(xy[i])) return fail(CGP_ERR_INVALID, "node coordinates must be finite");
  cgp::CaPlan pl;
  std::string err;
  try {
    err = cgp::ca_plan(n, rp, cl, xy, cgp::kCaS, cgp::kCaThreads, cgp::kCaExtMax, cgp::kCaEllMax, pl);
  } catch (const std::exception& e) {
    err = e.what();
  }
  if (!err.empty()) return fail(CGP_ERR_INVALID, err);
  std::memcpy(perm, pl.perm.data(), sizeof(int32_t) * n);
  std::memcpy(own_off, pl.own_off.data(), sizeof(int32_t) * pl.own_off.size());
  info[0] = pl.ntiles;
  info[1] = pl.max_own;
  info[2] = pl.max_ext;
  info[3] = pl.width;
  return CGP_OK;
}

int cgp_ndchol_solve_host(int32_t n, const int32_t* rowptr, const int32_t* col,
                          const double* val, const double* xy, const uint8_t* skip,
                          const double* r, double* z, cgp_ndchol_info* info) {
  if (n < 1 || !rowptr || !col || !val || !xy || !skip || !r || !z)
    return fail(CGP_ERR_INVALID, "null argument or n < 1");
  if (rowptr[0] != 0) return fail(CGP_ERR_INVALID, "rowptr[0] must be 0");
  for (int32_t i = 0; i < n; ++i)
    if (rowptr[i + 1] < rowptr[i]) return fail(CGP_ERR_INVALID, "rowptr not monotone");
  for (int32_t e = 0; e < rowptr[n]; ++e)
    if (col[e] < 0 || col[e] >= n) return fail(CGP_ERR_INVALID, "column index out of range");
  std::vector<int32_t> rp(rowptr, rowptr + n + 1), cl(col, col + rowptr[n]);
  std::vector<uint8_t> sk(skip, skip + n);
  cgp::NdFactor f;
  std::string err;
  try {
    err = cgp::nd_symbolic(n, rp, cl, xy, sk, f);
    if (err.empty()) err = cgp::nd_numeric(rp, cl, val, f);
  } catch (const std::exception& e) {
    err = std::string("factorisation failed: ") + e.what();
  }
  if (!err.empty()) return fail(CGP_ERR_INVALID, err);
  cgp::nd_solve_host(f, r, z);
  if (info) {
    info->n_factored = f.nfac;
    info->n_supernodes = (int32_t)f.sn.size();
    info->height = f.height;
    info->max_front = f.max_front;
    info->g_entries = f.g_entries;
  }
  return CGP_OK;
}

}  // extern "C"

namespace {

// One step (Eqs. 21-26); `theta` (learned guess) or `guess` may be given.
int project_step(cgp_ctx* c, cgp_state* S, const double* u_dir, const double* f,
                 const double* t_nat, const double* guess, const float* theta,
                 cgp_step_stats* st, void* stream) {
  if (int rc = check_ready(c)) return rc;
  if (!S || !S->u_prev || !S->u || !S->p || (c->ndir && !u_dir))
    return fail(CGP_ERR_INVALID, "null state or boundary pointer");
  if (t_nat && c->h.n_nat_c == 0) return fail(CGP_ERR_INVALID, "traction given but no boundary is natural");
  for (int k = 0; k < 4; ++k)
    if (!S->phi_hist[k]) return fail(CGP_ERR_INVALID, "null phi_hist pointer");
  hipStream_t s = as_stream(stream);
  cgp_step_stats local{};
  cgp_step_stats* T = st ? st : &local;
  const bool noninc = c->prob.scheme == CGP_SCHEME_NONINCREMENTAL;
  int rc = run_momentum(c, S->u_prev, S->u, noninc ? nullptr : S->p, u_dir, f, t_nat, c->ut,
                        T->momentum, s);
  if (rc < 0) return rc;
  run_restrict(c, c->ut, c->bc, s);
  double* phi_new = S->phi_hist[3];
  if (theta) {
    // learned candidate, kept only if its FP64 initial residual is not worse
    // than that of the previous increment
    const double* hist[4] = {S->phi_hist[0], S->phi_hist[1], S->phi_hist[2], S->phi_hist[3]};
    cgp::net::launch_pack(theta, c->net_wb, s);
    cgp::net::launch_forward(c->C, c->Kc, theta, c->net_wb, c->net, c->bc, hist, c->hbar,
                             c->net_dpart, c->net_scal, s);
    cgp::net::launch_decode(c->C, theta, c->net, c->net_scal, nullptr, c->guess_tmp, c->nat_c,
                            c->net_lpart, s);
    cgp::launch_guard(c->C, c->Kc, c->bc, c->guess_tmp, S->phi_hist[0], phi_new, c->chose,
                      c->part, c->nb_c, s);
  } else {
    cgp::launch_copy(guess ? guess : S->phi_hist[0], phi_new, c->nc, s);
  }
  rc = worst(rc, run_pcg(c, c->bc, phi_new, &T->poisson, s));
  if (rc < 0) return rc;
  cgp::launch_prolong(c->nf, c->pcode, c->tri_c, c->prob.levels, phi_new, c->phi_f, s);
  cgp_solve_stats cs[3];
  rc = worst(rc, run_correct(c, c->ut, c->phi_f, noninc ? nullptr : S->p, S->u_prev, S->p, cs, s,
                             phi_new));
  if (rc < 0) return rc;
  T->mass[0] = cs[0];
  T->mass[1] = cs[1];
  T->prot = cs[2];
  double* np1 = S->u_prev;
  S->u_prev = S->u;
  S->u = np1;
  double* h3 = S->phi_hist[3];
  S->phi_hist[3] = S->phi_hist[2];
  S->phi_hist[2] = S->phi_hist[1];
  S->phi_hist[1] = S->phi_hist[0];
  S->phi_hist[0] = h3;
  S->step += 1;
  HIPCHK(hipGetLastError());
  T->guess_net = 0;
  if (st) {
    if (theta) {
      HIPCHK(hipMemcpyAsync(&c->pinned[15].iters, c->chose, sizeof(int32_t),
                            hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      T->guess_net = c->pinned[15].iters == 0 ? 1 : 0;
    } else {
      HIPCHK(hipStreamSynchronize(s));
    }
  }
  return rc;
}

// host-side seeded uniform generator (xorshift64*)
struct Rng {
  uint64_t x;
  explicit Rng(uint64_t seed) : x(seed * 0x9E3779B97F4A7C15ull + 0x2545F4914F6CDD1Dull) {
    if (!x) x = 1;
  }
  double uniform() {
    x ^= x >> 12;
    x ^= x << 25;
    x ^= x >> 27;
    return (double)((x * 0x2545F4914F6CDD1Dull) >> 11) * (1.0 / 9007199254740992.0);
  }
};

int net_check(cgp_ctx* c, const float* theta, const double* b, const double* const* hist) {
  if (int rc = check_ready(c)) return rc;
  if (!theta || !b || !hist) return fail(CGP_ERR_INVALID, "null argument");
  for (int k = 0; k < 4; ++k)
    if (!hist[k]) return fail(CGP_ERR_INVALID, "null history pointer");
  return CGP_OK;
}

}  // namespace

extern "C" {

int cgp_project_step(cgp_ctx* c, cgp_state* S, const double* u_dir, const double* f,
                     const double* t_nat, const double* guess, cgp_step_stats* st,
                     void* stream) {
  return project_step(c, S, u_dir, f, t_nat, guess, nullptr, st, stream);
}

int cgp_project_step_net(cgp_ctx* c, cgp_state* S, const double* u_dir, const double* f,
                         const double* t_nat, const float* theta, cgp_step_stats* st,
                         void* stream) {
  if (!theta) return fail(CGP_ERR_INVALID, "null network parameters");
  return project_step(c, S, u_dir, f, t_nat, nullptr, theta, st, stream);
}

int cgp_net_init(float* theta, uint64_t seed) {
  if (!theta) return fail(CGP_ERR_INVALID, "null argument");
  namespace N = cgp::net;
  Rng rng(seed);
  std::memset(theta, 0, sizeof(float) * N::kParams);
  auto fill = [&](int ofs, int rows, int cols, double scale) {
    const double lim = scale * std::sqrt(6.0 / cols);
    for (int k = 0; k < rows * cols; ++k) theta[ofs + k] = (float)((2.0 * rng.uniform() - 1.0) * lim);
  };
  fill(N::kWe, 32, 5, 1.0);
  for (int r = 0; r < N::kRounds; ++r) {
    const int o = N::round_ofs(r);
    fill(o + N::kA, 32, 32, 1.0);
    fill(o + N::kBm, 32, 32, 1.0);
    fill(o + N::kC, 32, 3, 1.0);
    fill(o + N::kU, 32, 64, 0.1);
  }
  for (int k = 0; k < 32; ++k) theta[N::kW + k] = (float)((2.0 * rng.uniform() - 1.0) * 0.01);
  return CGP_OK;
}

int cgp_net_guess(cgp_ctx* c, const float* theta, const double* b, const double* const* hist,
                  double* guess, void* stream) {
  if (int rc = net_check(c, theta, b, hist)) return rc;
  if (!guess) return fail(CGP_ERR_INVALID, "null guess pointer");
  hipStream_t s = as_stream(stream);
  cgp::net::launch_pack(theta, c->net_wb, s);
  cgp::net::launch_forward(c->C, c->Kc, theta, c->net_wb, c->net, b, hist, c->hbar,
                           c->net_dpart, c->net_scal, s);
  cgp::net::launch_decode(c->C, theta, c->net, c->net_scal, nullptr, guess, c->nat_c,
                          c->net_lpart, s);
  HIPCHK(hipGetLastError());
  return CGP_OK;
}

int cgp_net_grad(cgp_ctx* c, const float* theta, const double* b, const double* const* hist,
                 const double* target, float* grad, float* loss, void* stream) {
  if (int rc = net_check(c, theta, b, hist)) return rc;
  if (!target) return fail(CGP_ERR_INVALID, "null target");
  hipStream_t s = as_stream(stream);
  cgp::net::launch_pack(theta, c->net_wb, s);
  cgp::net::launch_forward(c->C, c->Kc, theta, c->net_wb, c->net, b, hist, c->hbar,
                           c->net_dpart, c->net_scal, s);
  cgp::net::launch_decode(c->C, theta, c->net, c->net_scal, target, nullptr, nullptr,
                          c->net_lpart, s);
  cgp::net::launch_backward(c->C, theta, c->net_wb, c->net, c->net_lpart,
                            loss ? loss : c->net_loss, s);
  if (grad)
    HIPCHK(hipMemcpyAsync(grad, c->net.grad, sizeof(float) * cgp::net::kParams,
                          hipMemcpyDeviceToDevice, s));
  HIPCHK(hipGetLastError());
  return CGP_OK;
}

int cgp_net_train_step(cgp_ctx* c, float* theta, float* m, float* v, int32_t step, float lr,
                       const double* b, const double* const* hist, const double* target,
                       float* loss, void* stream) {
  if (!m || !v || step < 1 || !(lr > 0.0f)) return fail(CGP_ERR_INVALID, "bad Adam arguments");
  if (int rc = cgp_net_grad(c, theta, b, hist, target, nullptr, loss, stream)) return rc;
  cgp::net::launch_adam(theta, c->net.grad, m, v, step, lr, as_stream(stream));
  HIPCHK(hipGetLastError());
  return CGP_OK;
}

int cgp_extrapolate(cgp_ctx* c, const double* const* hist, double* q, void* stream) {
  if (int rc = check_ready(c)) return rc;
  if (!hist || !hist[0] || !hist[1] || !hist[2] || !q) return fail(CGP_ERR_INVALID, "null argument");
  cgp::net::launch_extrapolate(c->nc, hist[0], hist[1], hist[2], c->nat_c, q, as_stream(stream));
  HIPCHK(hipGetLastError());
  return CGP_OK;
}

int cgp_guess_guard(cgp_ctx* c, const double* b, const double* cand, const double* prev,
                    double* out, int32_t* chose, void* stream) {
  if (int rc = check_ready(c)) return rc;
  if (!b || !cand || !prev || !out) return fail(CGP_ERR_INVALID, "null argument");
  cgp::launch_guard(c->C, c->Kc, b, cand, prev, out, chose ? chose : c->chose, c->part, c->nb_c,
                    as_stream(stream));
  HIPCHK(hipGetLastError());
  return CGP_OK;
}

int cgp_intermediates(cgp_ctx* c, const double** ut, const double** bc, const double** phif) {
  if (int rc = check_ready(c)) return rc;
  if (ut) *ut = c->ut;
  if (bc) *bc = c->bc;
  if (phif) *phif = c->phi_f;
  return CGP_OK;
}

int cgp_timing_enable(cgp_ctx* c, int kernel_id) {
  if (!c) return fail(CGP_ERR_INVALID, "null context");
  if (kernel_id < 0 || kernel_id > CGP_K_MASS_PAIR) return fail(CGP_ERR_INVALID, "unknown kernel id");
  c->timed_id = kernel_id;
  c->tev_used = 0;
  return CGP_OK;
}

int cgp_timing_read(cgp_ctx* c, double* total_ms, int64_t* launches) {
  if (!c || !total_ms || !launches) return fail(CGP_ERR_INVALID, "null argument");
  double sum = 0.0;
  for (size_t k = 0; k + 1 < c->tev_used; k += 2) {
    HIPCHK(hipEventSynchronize(c->tev[k + 1]));
    float ms = 0.0f;
    HIPCHK(hipEventElapsedTime(&ms, c->tev[k], c->tev[k + 1]));
    sum += ms;
  }
  *total_ms = sum;
  *launches = (int64_t)(c->tev_used / 2);
  return CGP_OK;
}

void cgp_destroy(cgp_ctx* c) {
  if (!c) return;
  for (hipEvent_t e : c->tev) (void)hipEventDestroy(e);
  for (int k = 0; k < 2; ++k)
    if (c->ev[k]) (void)hipEventDestroy(c->ev[k]);
  delete c;
}

}  // extern "C"
