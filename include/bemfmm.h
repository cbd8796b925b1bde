/*
 * bemfmm -- fast-multipole boundary-element electrostatics on one MI355X.
 *
 * The method is that of Yokota, Bardhan, Knepley, Barba and Hamada,
 * "Biomolecular electrostatics using a fast multipole BEM on up to 512 GPUs
 * and a billion unknowns" (arXiv:1007.4591):
 *
 *   Section 2.1 (continuum model, eq. ASC, eq. reac, matrix statement):
 *     flat triangular panels, one piecewise-constant unknown per panel,
 *     one quadrature point at the centroid;  A x = f E,  E = B q,
 *     A = (1 - f/2) I - f K',  f = 1 - eps_in/eps_out,
 *     K'_ij = a_j n_i . grad G(c_i, c_j), K'_ii = 0,  G = 1/(4 pi |r - r'|),
 *     phi = C x,  (C x)_q = sum_j a_j x_j G(r_q, c_j),
 *     dG = (2 pi K / eps_in) q^T C x,  K = 332.06 kcal A / (mol e^2).
 *   Section 2.2 (BIBEE, eq. CFA and the scale factors 0 and +1/2 named
 *     after it): the principal-value operator K' is replaced by -1/2, 0 or
 *     +1/2 times the identity, which gives x = f E (CFA), f E / (1 - f/2)
 *     (P) or f E / (1 - f); the energy is then computed as above.
 *   Section 4.4 (eq. binding-free-energy-estimate): the binding energy is
 *     the solvation energy of the complex minus those of its two parts.
 *   Section 2.3 (FMM): every product with K', B, C and their transposes is
 *     a fast-multipole sum over an octree (P2M, M2M, M2L, L2L, L2P, P2P).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Arrays are DEVICE pointers (memory of the current HIP device), FP64, in
 *   the caller's original order, row-major (x,y,z) for 3-vectors, unless the
 *   argument name ends in _host.  A tree lives on the device that was
 *   current when it was built; calls on it run there (the library makes
 *   that device current for the call and restores the caller's), so their
 *   arrays and stream must belong to that device.  The caller owns every argument buffer;
 *   the library copies what it keeps, so inputs may be freed after a call.
 * - All device work is enqueued on `stream` (a hipStream_t; NULL is the
 *   null stream).  Entry points that return host scalars or solve iteratively
 *   synchronise that stream.  A tree may be used by one stream at a time.
 * - Every function returns a bemfmm_status.  On failure, outputs are
 *   unspecified and bemfmm_last_error() returns a message (thread-local).
 *   The tree stays valid except after BEMFMM_EDEVICE.
 * - Expansion order p means degrees 0..p-1 (p^2 real coefficients per
 *   expansion; p = 10 gives the 55 complex coefficients of Section 3.2).
 * - Each tree also owns one non-blocking stream (default priority) on which
 *   the near field of a product runs beside the multipole passes.  Events
 *   order it after the caller's earlier work on `stream` and before the
 *   product's last kernel on `stream`, so the caller sees plain stream order.
 * - Every product is deterministic: the same tree, inputs and precision
 *   give bitwise the same result (no floating-point atomics).
 * - Environment switches, read when a tree runs its first product (or, for
 *   the cache, on first use): BEMFMM_CONCURRENT_P2P=0 runs the near field
 *   on `stream` after the multipole passes; BEMFMM_M2L_PERSISTENT=0 uses one
 *   workgroup per M2L tile instead of persistent workgroups (which the FP32
 *   M2L uses, and the FP64 M2L when it is large: at least 32 tiles of 256
 *   pairs per compute unit); BEMFMM_M2L_SPLIT=0 runs the persistent FP32 M2L
 *   of order 10 of the panel-to-panel products (A, A^T) on FP32 matrix-core
 *   products instead of bf16 ones on operands split into three bf16 parts
 *   (products from or to charges always use the FP32 ones);
 *   BEMFMM_FORK_AT=0, 1, 2 or 3 starts the near field at the start of the
 *   product, after P2M, after M2M or after M2L (default: after M2M when the
 *   M2L has at least 32 tiles of 256 pairs per compute unit, or 8 for the
 *   split-bf16 FP32 M2L, else after P2M);
 *   BEMFMM_CACHE_LIMIT_MB caps the device memory kept for reuse per device
 *   (default: half of the device's memory, see bemfmm_release_cache).
 *   Results do not depend on BEMFMM_CONCURRENT_P2P or BEMFMM_FORK_AT.  The
 *   split-bf16 M2L (the default for FP32 A and A^T at order 10) and the FP32
 *   ones selected by the two M2L switches agree to FP32 rounding; the FP32
 *   ones agree with each other bitwise.
 */
#ifndef BEMFMM_H
#define BEMFMM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct bemfmm_tree bemfmm_tree; /* opaque; owns its device memory */

typedef enum {
  BEMFMM_OK = 0,
  BEMFMM_EINVAL = 1,  /* bad argument, mesh or parameter */
  BEMFMM_ENOMEM = 2,  /* device allocation failed */
  BEMFMM_EDEVICE = 3, /* HIP runtime error */
  BEMFMM_ENOCONV = 4, /* iterative solve reached maxit; outputs hold the last iterate */
  BEMFMM_ESTATE = 5   /* NULL or destroyed tree */
} bemfmm_status;

typedef enum {
  BEMFMM_FP64 = 0,        /* every FMM stage in FP64 */
  BEMFMM_FP32 = 1,        /* P2P and expansions in FP32 (M2L on FP32 MFMA) */
  BEMFMM_FP32_REFINED = 2 /* solves: FP32 inner GMRES inside an FP64-residual
                             iterative refinement; single products: as FP32 */
} bemfmm_precision;

typedef enum {
  BEMFMM_OP_A = 0,  /* y[N] = (1 - f/2) x - f K' x,            x[N]   */
  BEMFMM_OP_AT = 1, /* y[N] = (1 - f/2) x - f K'^T x,          x[N]   */
  BEMFMM_OP_B = 2,  /* y[N] = E = B x (normal field),          x[Q]   */
  BEMFMM_OP_BT = 3, /* y[Q] = B^T x = DL(x)(r_q),              x[N]   */
  BEMFMM_OP_C = 4,  /* y[Q] = C x,                             x[N]   */
  BEMFMM_OP_CT = 5  /* y[N] = C^T x,                           x[Q]   */
} bemfmm_op;

/* BIBEE surface charge x = s f E: the principal-value operator K' replaced
 * by -1/2 (CFA, s = 1), 0 (P, s = 1/(1 - f/2)) or +1/2 (s = 1/(1 - f)). */
typedef enum { BEMFMM_BIBEE_CFA = 0, BEMFMM_BIBEE_P = 1, BEMFMM_BIBEE_PLUS_HALF = 2 } bemfmm_bibee;

/* How bemfmm_binding_energy computes each solvation energy: the full BEM
 * solve (bemfmm_solve_bem + bemfmm_solvation_energy) or one BIBEE variant. */
typedef enum {
  BEMFMM_ENERGY_BEM = 0,
  BEMFMM_ENERGY_BIBEE_CFA = 1,
  BEMFMM_ENERGY_BIBEE_P = 2,
  BEMFMM_ENERGY_BIBEE_PLUS_HALF = 3
} bemfmm_energy_method;

/* Multipole acceptance between two same-level cells whose integer offset
 * (in cell widths) is o:
 *   THETA:    far iff 3 < theta^2 |o|^2, i.e. (R_a + R_b) < theta |d| with
 *             R the box half-diagonal (strict; ties are near);
 *   ADJACENT: far iff max|o_i| > 1 (the interaction list of Section 2.3:
 *             children of the parent's neighbours that are not adjacent). */
typedef enum { BEMFMM_MAC_THETA = 0, BEMFMM_MAC_ADJACENT = 1 } bemfmm_mac;

typedef struct {
  int p;          /* expansion order, 1..11 (degrees 0..p-1) */
  int ncrit;      /* target leaf occupancy >= 1: the leaf level is the one whose
                     mean panels per non-empty cell is closest to ncrit on a
                     log scale, among the first level with mean <= ncrit and
                     the level above it (uniform-depth sparse octree) */
  double theta;   /* MAC parameter for BEMFMM_MAC_THETA, 0.3..1 */
  int mac;        /* bemfmm_mac */
  double eps_in;  /* solute permittivity > 0 */
  double eps_out; /* solvent permittivity > 0 */
  double near_quad; /* 0: one centroid point for every panel pair (Section 2.1).
                       nu in (0, 16]: near quadrature -- the K' entry of a panel
                       pair with |c_i - c_j| < nu rho_j (rho_j: the largest
                       distance from c_j to a vertex of panel j) takes the exact
                       integral over flat panel j (Section 2.1, discretisation
                       paragraph: analytic integrals for planar elements); used
                       by A and A^T and everything built on them.  EINVAL if such
                       a pair could fall outside the near field (then lower nu
                       or raise ncrit). */
} bemfmm_params;

typedef struct {
  int iters;           /* total inner (matvec) iterations */
  int outer_iters;     /* refinement steps (1 for plain solves) */
  int converged;       /* 1 if rel_residual <= tol */
  double rel_residual; /* explicit |b - A x| / |b| with the FP64 FMM operator */
  double seconds;      /* wall time of the call */
} bemfmm_solve_info;

typedef struct {
  int64_t n_panels, n_charges;
  int leaf_level;           /* L */
  int64_t n_cells;          /* all levels 0..L */
  int64_t n_leaves;
  int64_t n_near_pairs;     /* leaf-level near (P2P) cell pairs */
  int64_t n_far_pairs;      /* M2L cell pairs, all levels */
  int64_t n_m2l_panel_pairs;/* M2L pairs whose cells both hold panels (the A, A^T work) */
  int64_t n_offsets;        /* distinct M2L translation offsets */
  int64_t p2p_pairs_panels; /* sum over near cell pairs of n_t * n_s (panels -> panels) */
  double lo[3];             /* root cube corner */
  double side;              /* root cube side */
  int64_t n_nearquad_pairs; /* close panel pairs with exact integrals (0 unless near_quad > 0) */
} bemfmm_tree_info;

/* Build the octree and interaction lists for a mesh and a set of charges
 * (Section 2.3 hierarchy; Section 3.1 Morton ordering), entirely on the GPU:
 * panel geometry, bounding cube, 30-bit Morton keys, stable radix sort,
 * cells of every level, near (P2P) and far (M2L) lists grouped by
 * translation offset.  verts: [nv*3]; tris: [nt*3] int32 vertex indices,
 * counter-clockwise seen from outside (the normal points into the solvent);
 * charge_pos: [nq*3] (nq may be 0).  The mesh is fixed for the tree's
 * lifetime.  EINVAL: nt == 0, an index out of range, a zero-area or
 * non-finite triangle, a non-finite charge, or parameters out of range --
 * among them p outside 1..11: the matrix-core translation kernels hold an
 * expansion of p^2 coefficients padded to at most eight column tiles of 16
 * (p^2 <= 128), so p = 12 and above are refused.
 * *out receives a new tree, to be released with bemfmm_tree_destroy. */
int bemfmm_build_tree(const double *verts, int64_t nv, const int32_t *tris, int64_t nt,
                      const double *charge_pos, int64_t nq, const bemfmm_params *params,
                      void *stream, bemfmm_tree **out);

/* Move the charges (charge_pos [nq*3], same count and order) without
 * rebuilding: every charge keeps its leaf cell, so the FMM operator changes
 * continuously (finite differences on a frozen tree).  EINVAL if a charge
 * leaves its leaf box by more than 1/1000 of the leaf side (beyond that the
 * near/far lists, built for charges inside their leaves, would no longer
 * guarantee the MAC's separation); the charges are then left unchanged. */
int bemfmm_set_charges(bemfmm_tree *tree, const double *charge_pos, void *stream);

/* Bytes of the fixed per-device scratch array of bemfmm_set_charges_noalloc
 * (a 256-byte error word, then 16 + 32 bytes of staged positions per
 * charge): it holds up to 699,040 charges. */
#define BEMFMM_NOALLOC_SCRATCH_BYTES (32u << 20)

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving or optimisation loops, harnesses that forbid
 * hipMalloc): bemfmm_set_charges with the same arguments, checks and
 * results, bitwise, that allocates nothing.  Its error word and staged
 * positions live in a fixed library array of BEMFMM_NOALLOC_SCRATCH_BYTES
 * that every device the library runs on holds until the process ends, and
 * it reads charge_pos in place (the caller keeps it valid until the call
 * returns; the call synchronises `stream`).  EINVAL, with the tree
 * unchanged, if the tree holds more than 699,040 charges (use
 * bemfmm_set_charges), or in bemfmm_set_charges' cases.  Every call on one
 * GPU shares that GPU's array, which keeps the last call's contents: calls
 * that overlap on one GPU (two host threads, or two streams) race, so
 * serialise them. */
int bemfmm_set_charges_noalloc(bemfmm_tree *tree, const double *charge_pos, void *stream);

int bemfmm_tree_destroy(bemfmm_tree *tree);

/* Sizes of the built tree (host struct). */
int bemfmm_tree_get_info(const bemfmm_tree *tree, bemfmm_tree_info *info_host);

/* One fast-multipole product with the operator `op` (see bemfmm_op):
 * x and y are device FP64 arrays of the sizes listed there.  The result is
 * the FMM approximation of the dense discrete operator of Section 2.1. */
int bemfmm_fmm_matvec(bemfmm_tree *tree, int op, int precision, const double *x, double *y,
                      void *stream);

/* Solve A x = f B q (Section 2.1) by GMRES(restart) from x = 0 until the
 * explicit relative residual |f B q - A x| / |f B q| (FP64 FMM operator)
 * is <= tol or maxit inner iterations were spent.  q: [Q]; x: [N] output.
 * precision FP32_REFINED runs FP32-FMM GMRES inside an FP64 refinement
 * loop.  info_host may be NULL.  ENOCONV if not converged. */
int bemfmm_solve_bem(bemfmm_tree *tree, const double *q, double *x, double tol, int maxit,
                     int restart, int precision, bemfmm_solve_info *info_host, void *stream);

/* BIBEE energy (Section 2.2, eq. CFA and its scale-factor 0 and +1/2
 * variants): x = f E (CFA), f E / (1 - f/2) (P) or f E / (1 - f)
 * (PLUS_HALF), then dG = (2 pi K/eps_in) q^T C x, written to *dG_host in
 * kcal/mol.  q: [Q].  EINVAL for another kind. */
int bemfmm_bibee_energy(bemfmm_tree *tree, const double *q, int kind, int precision,
                        double *dG_host, void *stream);

/* Solvation energy dG = (2 pi K/eps_in) q^T C x for a given surface charge
 * x [N] (Section 2.1 energy; C by FMM), in kcal/mol, to *dG_host. */
int bemfmm_solvation_energy(bemfmm_tree *tree, const double *q, const double *x, int precision,
                            double *dG_host, void *stream);

/* Gradient of dG(q, r) = kappa q^T C A^-1 f B q (kappa = 2 pi K/eps_in),
 * given the forward solution x [N] of A x = f B q: solves A^T y = C^T q
 * (the transposed operator is a dipole-source FMM) and returns
 *   dG_dq   [Q]   = kappa (C x + f B^T y),
 *   dG_dpos [Q*3] = kappa q_q [grad SL(a x) + f grad DL(y)](r_q)
 * (the force on charge q is -dG_dpos; the mesh is held fixed).
 * Either output may be NULL.  info_host (may be NULL) describes the
 * adjoint solve. */
int bemfmm_adjoint_grad(bemfmm_tree *tree, const double *q, const double *x, double tol, int maxit,
                        int restart, int precision, double *dG_dq, double *dG_dpos,
                        bemfmm_solve_info *info_host, void *stream);

/* Electrostatic binding energy (Section 4.4, eq.
 * binding-free-energy-estimate): dG_bind = dG_complex - dG_protein -
 * dG_inhibitor, each the solvation energy of its own tree (surface and
 * charges) and charge values q_* [Q of that tree].  method is a
 * bemfmm_energy_method: BEM solves each system to `tol` (maxit, restart
 * and precision as for bemfmm_solve_bem; the energies' C products then run
 * in FP64 unless precision is FP32); a BIBEE method takes that variant's
 * surface charge at `precision` (tol, maxit and restart unused).
 * dG_host[4] receives (bind, complex, protein, inhibitor) in kcal/mol.  The
 * three trees must live on one device; they may be the same tree.  ENOCONV
 * if a BEM solve did not converge (dG_host then unspecified). */
int bemfmm_binding_energy(bemfmm_tree *complex_tree, const double *q_complex, bemfmm_tree *protein_tree,
                          const double *q_protein, bemfmm_tree *inhibitor_tree, const double *q_inhibitor,
                          int method, int precision, double tol, int maxit, int restart, double *dG_host,
                          void *stream);

/* Thread-local message for the last failure on this thread ("" if none). */
/* ------------------------------------------------------------------------
 * Linearised Poisson-Boltzmann solvent (Section 2.1: the screened equation
 * lap phi = kappa^2 phi outside the molecule, named there and in Section 5
 * as the method's next extension).  The paper gives no integral equation;
 * the one solved here is the second-kind pair for the surface potential
 * u = phi and its interior normal derivative v = d phi/dn (n outward), with
 * eps = eps_out/eps_in, G0 = 1/(4 pi r), Gk = exp(-kappa r)/(4 pi r):
 *   (1+eps)/2 u + (K0 - eps Kk) u - (V0 - Vk) v = S
 *   (1+1/eps)/2 v - (K0' - Kk'/eps) v + (D0 - Dk) u = dS/dn
 * (V single layer, K double layer, K' its adjoint, D the normal derivative of
 * the double layer; S = sum_k q_k G0(., r_k)/eps_in), collocated at the
 * centroids with one point per panel; the self terms of V0 - Vk and D0 - Dk
 * are exact integrals over the flat panel, the others vanish.  The far field
 * of Gk is a screened-kernel FMM on the same tree (per-level operators built
 * on the GPU at the first call with a new kappa); everything runs in FP64.
 * uv and y are [2N] = (u, v) in caller panel order; kappa > 0 in 1/A with
 * kappa * (root cube side) <= 400 (EINVAL otherwise).
 *
 * y = M uv (the operator above). */
int bemfmm_lpb_matvec(bemfmm_tree *tree, double kappa, const double *uv, double *y, void *stream);

/* Solve M uv = [S; dS/dn] by GMRES(restart) from 0 to the relative residual
 * tol (explicit, in info); ENOCONV at maxit with uv the last iterate. */
int bemfmm_lpb_solve(bemfmm_tree *tree, const double *q, double kappa, double *uv, double tol, int maxit,
                     int restart, bemfmm_solve_info *info, void *stream);

/* Solvation energy of a solution uv: dG = 2 pi K sum_k q_k phi_reac(r_k),
 * phi_reac = SL0(a v) - DL0(a u) the reaction potential (kcal/mol). */
int bemfmm_lpb_energy(bemfmm_tree *tree, const double *q, const double *uv, double *dG_host, void *stream);

const char *bemfmm_last_error(void);

/* Device memory of destroyed trees and of grown workspaces is kept by the
 * library, per device, and reused by later builds of a similar size (up to
 * BEMFMM_CACHE_LIMIT_MB per device, default half of the device's memory; a
 * failed allocation of the library empties the cache and retries).  Other
 * allocators in the process (PyTorch's) do not see this memory as free:
 * this call returns every cached block of every device to the driver after
 * synchronising each device; memory of live trees is untouched. */
int bemfmm_release_cache(void);

/* ----------------------------------------------------------------------
 * Inspection (used by parity tests; not needed to solve).
 * ---------------------------------------------------------------------- */

/* Copy tree arrays to host buffers the caller allocated with the sizes from
 * bemfmm_tree_info.  Any pointer may be NULL.
 *   panel_perm [N], charge_perm [Q]: sorted position -> caller index.
 *   panel_key [N], charge_key [Q]: 30-bit Morton keys in sorted order.
 *   cell_key [n_cells] (level prefix), cell_level [n_cells],
 *   cell_range [n_cells*4] = panel begin, end, charge begin, end,
 *   cell_parent [n_cells] (global cell index, -1 for the root);
 *   cells are stored level by level (0..L), each level in increasing key.
 *   near_ptr [n_leaves+1], near_idx [n_near_pairs]: leaf-level CSR, leaf
 *   indices local to level L, sources in increasing order;
 *   far_pairs [n_far_pairs*3] = (level, target, source) with level-local
 *   indices, ordered by level, then target, then source. */
int bemfmm_tree_export(const bemfmm_tree *tree, int32_t *panel_perm_host, int32_t *charge_perm_host,
                       uint32_t *panel_key_host, uint32_t *charge_key_host,
                       uint32_t *cell_key_host, int32_t *cell_level_host, int32_t *cell_range_host,
                       int32_t *cell_parent_host, int32_t *near_ptr_host, int32_t *near_idx_host,
                       int32_t *far_pairs_host);

/* Expansions left by the last bemfmm_fmm_matvec at `precision` on this
 * tree: which = 0 for multipole, 1 for local; out_host [n_cells * p*p]
 * FP64, cell-major in the cell order of bemfmm_tree_export, scaled and
 * packed as: a cell of side s stores M_n^m / s^n and s^(n+1) L_n^m of the
 * 1/|x-y| kernel, with R_n^m = r^n P_n^m(cos t) e^{i m phi}/(n+m)! and
 * I_n^m = (n-m)! P_n^m(cos t) e^{i m phi}/r^(n+1) (Condon-Shortley phase),
 * M_n^m = sum w conj(R_n^m(y - X)), L_n^m = sum w conj(I_n^m(y - X));
 * per degree n: Re m=0, then Re, Im of m = 1..n. */
int bemfmm_debug_expansions(bemfmm_tree *tree, int precision, int which, double *out_host);

/* enable = 1: the products that follow also record their near (P2P) and
 * far (L2P) parts for bemfmm_debug_fields (two extra FP64 writes per
 * target); 0 (the default) stops recording. */
int bemfmm_debug_record(bemfmm_tree *tree, int enable);

/* Near (P2P) and far (L2P) parts of the raw field of the last
 * bemfmm_fmm_matvec at `precision` made while recording was on
 * (bemfmm_debug_record; ESTATE otherwise), per target in the caller's order,
 * before the operator's combination (kernel 1/(4 pi |x - y|)): for panel
 * targets the normal derivative (A, B) or potential (A^T, C^T); for charge
 * targets the potential.  near_host, far_host: [n_targets]. */
int bemfmm_debug_fields(bemfmm_tree *tree, int precision, double *near_host, double *far_host);

/* Per-stage device time of FMM products since the last reset, from HIP
 * events recorded on the stream that runs each stage (enable = 1 starts
 * recording, 0 stops; reset clears).  Stage names: "p2m", "m2m", "m2l",
 * "l2l" (downward pass incl. the batched L2L), "p2p" (near field, on the
 * second stream), "l2p" (far-field evaluation and final combination),
 * "other" (packing of the inputs).  A name alone sums every product; "name/op/
 * precision" (e.g. "p2p/0/1") restricts it to one operator (BEMFMM_OP_*) at
 * one precision (BEMFMM_FP64 = 0, BEMFMM_FP32 = 1).  ms_host and
 * count_host receive the total time and the number of stage instances. */
int bemfmm_profile(bemfmm_tree *tree, int enable, int reset);
/* Restrict recording to products of one operator (BEMFMM_OP_*, or -1 for
 * any) at one precision (BEMFMM_FP64, BEMFMM_FP32, or -1 for any; a refined
 * solve runs FP32 and FP64 products).  Other products then record no events
 * and wait for nothing. */
int bemfmm_profile_select(bemfmm_tree *tree, int op, int precision);
int bemfmm_profile_get(bemfmm_tree *tree, const char *stage, double *ms_host, int64_t *count_host);

#ifdef __cplusplus
}
#endif

#endif /* BEMFMM_H */
