// Internal declarations shared by the kernels (kernels.hip) and the C-ABI
// orchestration (api.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "lattice.hpp"

namespace cgp {

constexpr int kBlock = 256;    // threads per block (4 wave64)
constexpr int kNbMax = 1280;   // blocks per solver launch (partial-sum slots)
// the fine BiCGSTAB launches up to kNbMax blocks: five per CU, as many as the
// products' 30 KB LDS tiles allow; the coarse solvers up to kNbCoarse
constexpr int kNbCoarse = 1024;
constexpr int kEllPad = 8;     // ELL widths are multiples of this
constexpr int kSlots = 8;      // reduction slots per right-hand side

// CSR node graph with edge sides (see mesh.hpp), on the device.
struct DLevel {
  int32_t n;
  int32_t nnz;
  const int32_t* rowptr;
  const int32_t* col;
  const int32_t* side;
  const double2* xy;
  const int32_t* tile;   // row tiles of the LDS-staged products
  int32_t ntiles;
};

// Per right-hand-side solver scalars.  done_stamp is the (iteration, phase)
// stamp of the kernel that finished the solve, 0 while running; a kernel
// skips a right-hand side whose stamp is smaller than its own, so the kernel
// that takes the decision (every block of it computes the same value) never
// races with its own write.
struct Scal {
  double rho[2];    // PCG: gamma of even / odd iterations; BiCGSTAB: rho[0] current
  double rho_old;
  double alpha;
  double omega;
  double bb;        // ||b||^2
  double rel;       // last relative residual seen by the stopping test
  double pcg_alpha[2];  // PCG: alpha of even / odd iterations
  int32_t done_stamp;
  int32_t iters;
  int32_t status;   // 0 converged, 2 NaN
  int32_t pad_;
};

inline int stamp(int it, int phase) { return it * 8 + phase; }

// ---------------------------------------------------------------- assembly
void launch_mass_assemble(const DLevel& L, double* Mval, hipStream_t s);
// vval[k] = Mval[vpos[k]], 0 where vpos[k] < 0 (k < n)
void launch_vertex_rows(int64_t n, const int32_t* vpos, const double* Mval, double* vval,
                        hipStream_t s);
void launch_coarse_assemble(const DLevel& L, const uint8_t* nat, double* Kval, float* Kval32,
                            double* Dxval, double* Dyval, double* invd, float* invd32,
                            double* lumped, hipStream_t s);
// Lattice form of the momentum rows (momlat.hpp): rows from row0 on (the
// rows of the coarse vertices come first in mesh numbering).
struct MomRow;
struct MomTri;
struct MomLattice {
  const uint8_t* slot;      // [N][8]
  const MomRow* rows;       // [N]
  const MomTri* tris;       // [nT]
  int32_t row0;
};
// ml == nullptr: every row side-based
void launch_momentum_assemble(const DLevel& L, const int32_t* dir_index, double dt, double nu,
                              const double* u_prev, const double* u, const double* p,
                              const double* u_dir, int32_t n_dir, const double* f,
                              const double* t_nat, double* Aval, double* invdA, double* rhs,
                              double* x0, double* r0, double* scratch_w, double* scratch_r,
                              hipStream_t s, hipEvent_t* ev = nullptr,
                              const MomLattice* ml = nullptr);

// ---------------------------------------------------------------- BiCGSTAB (2 rhs)
// x, r, rhat, p, v, t, b: [2][n] (one right-hand side after the other);
// phat = D^-1 p and shat = D^-1 s: [n][2] (the two right-hand sides
// interleaved), so that the products gather both with one 16-byte load
struct BicgVecs {
  double *x, *r, *rhat, *p, *v, *phat, *shat, *t;
  const double* b;
  const double* invd;
};
// the start of the momentum BiCGSTAB: the assembly wrote r = b - A x0
// (launch_momentum_assemble's r0); r^ = r and the partial sums of (r, r),
// (b, b)
void launch_bicg_start(int32_t n, const BicgVecs& V, Scal* sc, double* part, int nb,
                       hipStream_t s);
// `ev`, when not null, is a pair of events recorded around the SpMV kernel
// v = A p^ (measurement hook).
void launch_bicg_iter(const DLevel& L, const double* Aval, const BicgVecs& V, Scal* sc,
                      double* part, int nb, int it, double tol, bool check_only,
                      hipStream_t s, hipEvent_t* ev = nullptr);

// ---------------------------------------------------------------- PCG (one rhs)
template <typename T>
struct PcgVecs {
  T* x;             // solution (in: initial guess)
  T* p;             // direction
  T* r[2];          // residual, alternating between iterations
  T* w[2];          // A D^-1 r, alternating
  T* s[2];          // A p, alternating
  const T* b;
  const T* invd;
  const T* val;       // CSR values (set-up kernels)
  // fixed-width (ELL) copy of the matrix for the iteration kernel, column
  // major: entry k of row i at [k * n + i]; width a multiple of kEllPad,
  // short rows padded with (i, 0); values scaled by column, K_ij / K_jj
  const int32_t* ell_col;
  const T* ell_val;
  int32_t ell_w;
};
template <typename T>
void launch_pcg_init(const DLevel& L, const PcgVecs<T>& V, bool zero_x0, Scal* sc, double* part,
                     int nb, hipStream_t s);
// ELL copies (see PcgVecs) of a CSR matrix: its FP64 values, and its values
// scaled by column (K D^-1, with invd = 1 / diag) in FP64 and FP32
void launch_make_ell(const DLevel& L, const double* val, const double* invd, int w,
                     int32_t* ell_col, double* ell_val, double* ell_sval, float* ell_sval32,
                     hipStream_t s);
// `ev`, when not null, is a pair of events recorded around the iteration kernel.
template <typename T>
void launch_pcg_iter(const DLevel& L, const PcgVecs<T>& V, Scal* sc, double* part, int nb, int it,
                     double tol, bool check_only, hipStream_t s, hipEvent_t* ev = nullptr);

// ---------------------------------------------------------------- Chebyshev mass solves
int cheb_iterations(double tol);
// Solves M x = b for nr (2 or 3) right-hand sides interleaved [n][nr] in the
// lattice layout (velocity components 0 at Dirichlet nodes); returns the
// buffer (one of x[0..2]) holding the result, or nullptr (nothing launched)
// when b or an iterate is not 16-byte aligned or the lattice size is not one
// of 1, 2, 4, 8.  `timer(tctx, which)`, when given, supplies an event pair per
// launch of a single step after the first (which = kChebTimedSingle) and per
// launch of the interior two-step kernel (kChebTimedPair), or nullptr.
constexpr int kChebTimedSingle = 0;
constexpr int kChebTimedPair = 1;
double* launch_cheb(const LatDev& L, int32_t n, const double* b, int nr,
                    double* const x[3], int iters, hipStream_t s,
                    hipEvent_t* (*timer)(void*, int), void* tctx);
// Mixed precision: FP64 iterative refinement around two float Chebyshev solves
// of `iters` steps each (iterates stored as float, combined in FP64): d1 from
// M d1 = b (b's float copy in y[3]), then the residual r = b - M d1 (FP64,
// over y[3]), then d2 from M d2 = r; the solution is d1 + d2.  y: five float
// buffers [n][nr], 16-byte aligned.  Returns false (nothing launched) for an
// unsupported lattice size or misaligned buffers.
bool launch_cheb_mixed(const LatDev& L, int32_t n, const double* b, int nr, float* const y[5],
                       int iters, hipStream_t s, hipEvent_t* (*timer)(void*, int), void* tctx,
                       const float** d1, const float** d2);

// ---------------------------------------------------------------- restriction / prolongation
void launch_restrict_galerkin(const int32_t* tri_f, int32_t n_fine_tris, const double2* xy_f,
                              int levels, const double* ut, int64_t stride, double* tripart,
                              hipStream_t s);
void launch_restrict_nodes(int32_t n_c, const int32_t* cn_ptr, const int32_t* cn_tri,
                           const double* tripart, const uint8_t* nat, double scale, double* b,
                           double* part, int nb, hipStream_t s);
void launch_restrict_inject(const DLevel& C, const uint8_t* nat, const double* ut,
                            int64_t stride, double scale, double* b, double* part, int nb,
                            hipStream_t s);
void launch_remove_mean(int32_t n, double* v, const double* part, int nb, const double* weights,
                        hipStream_t s);
void launch_weighted_sums(int32_t n, const double* v, const double* w, double* part, int nb,
                          hipStream_t s);
void launch_prolong(int32_t n_f, const int32_t* pcode, const int32_t* tri_c, int levels,
                    const double* phic, double* phif, hipStream_t s);

// ---------------------------------------------------------------- correction
// rhs [n][2 + chi]: velocity right-hand sides, then (chi = 1) the rotational one
// right-hand sides of the mass solves (interleaved [n][nr]) or, for the
// lumped modes, the lumped updates written to u_out / p_out directly
void launch_correct_rhs(const DLevel& L, const int32_t* dir_index, const double* Mval,
                        double dt, double nu, int chi, int mass_mode, const double* phi_f,
                        const double* ut, const double* p_in, double* rhs, double* u_out,
                        double* p_out, const int32_t* lat_of, hipStream_t s);
// the same right-hand sides for mass mode CGP_MASS_CONSISTENT on the lattice
// layout (corrlat.hpp): first A.v4 ([n][4] from phi_f and U~, or [n][2] from
// U~ when A.phi_c is given, phi_f then being its prolongation) through
// node_of, then rhs [n][2 + chi]; rhs and A.v4 16-byte aligned; false
// (nothing launched) for a misaligned buffer or an unsupported lattice size
bool launch_correct_rhs_lattice(const LatDev& L, const int32_t* node_of, const double* phi,
                                const double* ut, const struct CorrLatArgs& A, double* rhs,
                                float* rhs32, hipStream_t s);
// U = U~ + dU from the solved increments du [n][nr]; P = P + phi (+ du[2]
// when nr = 3) unless write_p is false
void launch_final_update(int32_t n, const double* ut, const double* du, const double* p_in,
                         const double* phi_f, int nr, bool write_p, double* u_out,
                         double* p_out, const int32_t* lat_of, hipStream_t s);
// the same with dU (and dp) = d1 + d2 from the two float solves of
// launch_cheb_mixed, added in FP64
void launch_final_update2(int32_t n, const double* ut, const float* d1, const float* d2,
                          const double* p_in, const double* phi_f, int nr, bool write_p,
                          double* u_out, double* p_out, const int32_t* lat_of, hipStream_t s);

// ---------------------------------------------------------------- small vector ops
void launch_copy(const double* src, double* dst, int64_t n, hipStream_t s);
void launch_zero_masked(double* x, const uint8_t* nat, int32_t n, hipStream_t s);
// x += d; with `skip`, nothing once that record's solve is done
void launch_axpy_f32(const float* d, double* x, int64_t n, hipStream_t s,
                     const Scal* skip = nullptr);
void launch_fill32(float* x, float v, int64_t n, hipStream_t s);
// n <= 5 scalar records into host-mapped pinned memory
void launch_mirror(const Scal* src, Scal* host_dst, int n, hipStream_t s);
void launch_residual64(const DLevel& C, const double* Kval, const double* b, const double* x,
                       double* r, float* r32, double* part, int nb, hipStream_t s);
void launch_reduce_check(const double* part, int nb, double tol, Scal* sc, int outer,
                         hipStream_t s);

// one iteration of PCG with the factor preconditioner, after z = M^-1 r:
// p_it = z + beta p_{it-1} (p alternates between p[0] and p[1]), q = K p_it,
// x += alpha p_it, r -= alpha q; leaves the partials of (r, r) in the RR slot.
// With skip != nullptr the kernels return at once when skip->done_stamp is set.
void launch_fpcg_iter(int32_t n, const int32_t* ell_col, const double* ell_val, int ell_w,
                      const double* z, double* const p[2], double* q, double* x, double* r,
                      Scal* sc, double* part, int nb, int it, hipStream_t s,
                      const Scal* skip = nullptr);
void launch_fill(double* x, double v, int64_t n, hipStream_t s);

}  // namespace cgp
