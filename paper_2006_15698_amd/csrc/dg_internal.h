// Internal declarations shared by the host library and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dg.h"

#define DG_MAXN 8
#define DG_NF 5

// Per-context constant tables, passed by value as a kernel argument.
// Section II-B: collocated Gauss-Legendre nodal basis (Eqs. (6)-(7)).
struct DGTables {
  double Dh[DG_MAXN * DG_MAXN];  // Dh[i*N+a] = w_a l_i'(xi_a) / w_i: the
                                 // volume term of Eq. (5) on one 1-D line,
                                 // mass matrix already divided out
  double lm[DG_MAXN];            // l_i(-1): face interpolation weights
  double lp[DG_MAXN];            // l_i(+1)
  double liftm[DG_MAXN];         // l_i(-1) / w_i: surface term of Eq. (5)
  double liftp[DG_MAXN];         // l_i(+1) / w_i   lifted by M^{-1}
  double w[DG_MAXN];             // Gauss-Legendre weights
  double rs[DG_MAXN];            // rs[i] = sum_a Dh[i*N+a] (free-stream identity:
                                 // (l_i(1) - l_i(-1)) / w_i up to rounding)
  float Dh32[DG_MAXN * DG_MAXN]; // Dh rounded to FP32 (matrix-core variant)
  float lm32[DG_MAXN];           // l_i(-1), l_i(+1) rounded to FP32
  float lp32[DG_MAXN];
  double sc[3];                  // 2 / h_d (reference-to-physical metric)
  double hinv[3];                // 1 / h_d
  double J;                      // h_x h_y h_z / 8 (volume Jacobian)
  double gamma;                  // ratio of specific heats, Eq. (3)
  double gm1;                    // gamma - 1
  int nx, ny, nz;
  int E;                         // nx*ny*nz
};

struct dg_ctx {
  int nx, ny, nz, p, N;
  int64_t E;
  double gamma;
  double L[3];
  double xi[DG_MAXN], w[DG_MAXN];
  hipStream_t stream;
  int precision;
  char* ws;
  size_t ws_bytes;
  DGTables tab;
  int timing_on;
  void* timing;   // DGTiming*, owned, created by dg_set_timing
  int exchange;   // DG_EXCHANGE_TRACES or DG_EXCHANGE_NEIGHBOUR (FP64 path)
  int xcd_remap;  // XCD-aware workgroup -> block mapping (neighbour path)
  int order;      // DG_ORDER_LINEAR or DG_ORDER_PENCIL
  int pencil_x;   // pencil extent along x in elements (0: whole row)
  int pencil_z;   // pencil extent along z in element planes
  int visc_fused; // viscous FP64 standard form: inviscid rate inside the viscous-flux launch
  // viscous terms (dg_set_viscosity): dynamic viscosity, Prandtl number and
  // conductivity mu gamma / ((gamma - 1) Pr); mu = 0 is the Euler equations
  double mu, prandtl, kappa;
  int volume_form;  // DG_VOLUME_STANDARD or DG_VOLUME_KEP (dg_set_volume_form)
  // graph replay of whole steps (dg_rk_graph_steps): one executable graph
  // per ping-pong parity, valid while the arrays, dt and `epoch` (bumped by
  // every setter that changes what a launch does) are unchanged
  unsigned epoch;
  hipStream_t gstream;
  hipEvent_t ev_in, ev_out;
  hipGraphExec_t gexec[2];
  const double* gQ;
  const double* gR;
  double gdt;
  unsigned gepoch;
};

// Order in which a neighbour-read stage launch visits its element blocks
// (kernel argument).  A block is EPB consecutive elements of one x-row (the
// last block of a row may be short).  Blocks are visited z-slab by z-slab
// (tz planes), inside a slab pencil by pencil along x (tx blocks), inside a
// pencil y-row by y-row, and inside that z-plane by z-plane, x fastest.
// Index order is the special case of whole-row pencils one plane deep.
struct DGOrder {
  int xcd;      // chunk the visiting order per XCD
  int nxb;      // blocks per x-row
  int tx;       // blocks of a pencil along x
  int tz;       // element planes of a pencil along z
};

// Visiting order and grid size of a neighbour-read stage launch with EPB
// elements per block.
inline DGOrder dg_order(const dg_ctx* c, int epb, unsigned* grid) {
  DGOrder o;
  const bool pencil = c->order == DG_ORDER_PENCIL;
  o.xcd = c->xcd_remap;
  o.nxb = (c->nx + epb - 1) / epb;
  const int px = pencil && c->pencil_x > 0 && c->pencil_x < c->nx ? c->pencil_x : c->nx;
  o.tx = (px + epb - 1) / epb;
  o.tz = !pencil || c->pencil_z < 1 ? 1 : (c->pencil_z > c->nz ? c->nz : c->pencil_z);
  *grid = (unsigned)((int64_t)o.nxb * c->ny * c->nz);
  return o;
}

// Workspace carve-up (byte offsets, each 256-aligned).
struct DGWorkspace {
  size_t trace_bytes;   // one face-trace buffer: 30 * N^2 * E doubles
  size_t off_trace0, off_trace1;
  size_t off_red;       // reduction partials
  size_t off_vjp;       // adjoint scratch: two state-sized buffers
  size_t off_q2;        // second state buffer of the neighbour-read path
  size_t off_visc_r;    // viscous terms only (mu > 0): the inviscid rate of a stage (5 N^3 E doubles)
  size_t off_visc_fv;   //   and the nodal viscous flux (12 N^3 E doubles)
  size_t total;
};
DGWorkspace dg_workspace_layout(const dg_ctx* c);

// Number of blocks used by the reduction kernels (fixed: the summation
// order, and hence the result, does not depend on the device).
#define DG_RED_BLOCKS 1024
#define DG_RED_VALS 8

// ---- launchers (return hipError_t as int) -------------------------------
// Face traces of Q on all six faces of every element.
int dg_launch_trace(const dg_ctx* c, const double* Q, double* T);
// RHS: R = dQ/dt using traces Tin of Q.
int dg_launch_rhs(const dg_ctx* c, const double* Q, const double* Tin, double* R);
// One RK stage in place; writes the traces of the updated Q to Tout when
// Tout != nullptr.
int dg_launch_stage(const dg_ctx* c, double* Q, double* res, const double* Tin,
                    double* Tout, double a, double b, double dt, int first);
// Neighbour-read stage: Qin -> Qout; mode 0 writes RR = dQ/dt, mode 1 the
// RK update (res = RR in place).
int dg_launch_stage_nb(const dg_ctx* c, const double* Qin, double* Qout, double* RR, int mode, double a, double b,
                       double dt, int first);
// Reductions: per-block partials then a fixed-order final pass into
// red[DG_RED_BLOCKS*DG_RED_VALS .. +DG_RED_VALS).
int dg_launch_reduce(const dg_ctx* c, const double* Q, double* red);
// Adjoint RHS.
int dg_launch_vjp(const dg_ctx* c, const double* Q, const double* gR, double* gQ, char* scratch);

// Viscous terms (kern_visc.hip): the nodal viscous flux of Q into Fv (with
// `rate` also the inviscid rate of the standard form into R), then mode 0:
// R += the viscous rate; mode 1: the LSERK45 stage in place on Qu and res
// with R the inviscid rate of the stage.
int dg_launch_visc(const dg_ctx* c, const double* Q, double* Fv, double* R, double* Qu, double* res, int mode,
                   double a, double b, double dt, int first, bool rate);

// Kinetic-energy-preserving split form (kern_split.hip): mode 0 RR = dQ/dt;
// mode 1 the LSERK45 stage Qin -> Qout with res = RR in place; mode 2 the
// first stage.
int dg_launch_split(const dg_ctx* c, const double* Qin, double* Qout, double* RR, int mode, double a, double b,
                    double dt);

// Gradient of the kinetic-energy integral with respect to Q.
int dg_launch_ke_grad(const dg_ctx* c, const double* Q, double* G);

int dg_launch_axpy(const dg_ctx* c, int64_t n, const double* x, double b, const double* y, double* out);
int dg_launch_rk_reverse(const dg_ctx* c, int64_t n, const double* v, double dt, double a, const double* gtot,
                         double* gQ, double* gres);

// FP32 matrix-core variants.  Their trace buffers hold FP32 deviations
// [face][field][E][N^2] followed (256-aligned) by FP64 anchors [field][E];
// they fit in the same workspace regions as the FP64 traces.
int dg_launch_trace_f32(const dg_ctx* c, const double* Q, char* buf);
int dg_launch_rhs_f32(const dg_ctx* c, const double* Q, const char* tin, double* R);
int dg_launch_stage_f32(const dg_ctx* c, double* Q, double* res, const char* tin, char* tout, double a,
                        double b, double dt, int first);
bool dg_f32_supported(int N);
int dg_launch_stage_nb_f32(const dg_ctx* c, const double* Qin, double* Qout, double* RR, int mode, double a,
                           double b, double dt, int first);
