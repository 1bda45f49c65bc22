/*
 * nsasm -- element-by-element assembly of the incompressible Navier-Stokes
 * momentum right-hand side over linear tetrahedra, on one AMD MI355X (gfx950).
 *
 * The operation is the RHS assembly of an explicit-momentum fractional-step LES
 * (Owen, Ernst et al., "Alya towards Exascale", Sec. II), specialised as in
 * Sec. V-B: linear tetrahedra (4 nodes, constant shape-function gradients),
 * constant density and viscosity, an eddy viscosity evaluated once per element
 * on the fly, and the elemental RHS computed directly without elemental
 * matrices (Sec. V-A).  For element e with vertices a = 0..3 and nodal
 * velocity u_a, pressure p_a:
 *
 *   J = [x1-x0 | x2-x0 | x3-x0],  V = |det J| / 6,
 *   grad N_a = row a of J^-1 (a = 1..3),  grad N_0 = -(grad N_1 + grad N_2 + grad N_3),
 *   G = grad u = sum_a u_a (x) grad N_a,  q = grad p = sum_a p_a grad N_a,
 *   mu_e = mu + mu_t(G, V)  (eddy viscosity, see nsasm_params.eddy_model),
 *   R^e_a = int_e N_a (-rho G u_h - q + rho f) dx - mu_e V G grad N_a,
 *   rhs_n = sum over (e, a) with node(e, a) = n of R^e_a,
 *
 * where u_h is the P1 interpolant and the integral is the 4-point Gauss rule
 * (exact here, since the integrand has degree 2).  The paper prints no
 * discrete equations; the forms above (advective convection, gradient-form
 * pressure, Laplacian viscous term, Smagorinsky eddy viscosity, constant body
 * acceleration) are this library's reading of it.
 *
 * Conventions for every entry point:
 *  - Array arguments are DEVICE pointers (hipMalloc / torch CUDA tensors) on
 *    the current device; host pointers are rejected with
 *    NSASM_ERR_INVALID_ARGUMENT.  Arrays are dense, row-major, 64-bit indexed.
 *  - Field element type: double for NSASM_FP64, float for NSASM_MIXED.
 *    Coordinates are always double.
 *  - `stream` is a hipStream_t (NULL = the null stream).  Assembly calls are
 *    asynchronous on it and report launch errors only.  nsasm_mesh_create is
 *    synchronous.
 *  - The caller owns every argument buffer; the library keeps no caller
 *    pointer.  A mesh owns its internal device buffers until destroyed.
 *  - No call throws or aborts; each returns an nsasm_status and, when it is
 *    not NSASM_OK, sets a thread-local message read by nsasm_last_error().
 *  - A mesh's description is immutable after creation.  With the atomic and
 *    patch scatters, concurrent assembly calls on one mesh are safe when their
 *    output buffers differ; with the gather scatter they share the mesh's
 *    partial-sum buffer and must not overlap in time.
 */
#ifndef NSASM_H
#define NSASM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct nsasm_mesh nsasm_mesh; /* opaque, immutable after create */

typedef enum {
    NSASM_OK = 0,
    NSASM_ERR_INVALID_ARGUMENT = 1,   /* null/host pointer, bad size, bad enum */
    NSASM_ERR_BAD_CONNECTIVITY = 2,   /* node id out of range or repeated in a tet */
    NSASM_ERR_DEGENERATE_ELEMENT = 3, /* det J within rounding of zero, subnormal, or not finite */
    NSASM_ERR_OUT_OF_MEMORY = 4,
    NSASM_ERR_DEVICE = 5,             /* HIP runtime / launch failure */
    NSASM_ERR_UNSUPPORTED = 6         /* valid request the mesh cannot serve */
} nsasm_status;

typedef enum {
    NSASM_FP64 = 0,  /* all arithmetic and fields in double */
    NSASM_MIXED = 1  /* geometry (det J, J^-1, V) in double; fields, element
                        arithmetic and scatter-add in float */
} nsasm_precision;

typedef enum {
    NSASM_SCATTER_AUTO = 0,   /* PATCH_GATHER when the mesh allows it, else ATOMIC;
                                 with PATCH_GATHER, assembly calls on one mesh
                                 must not overlap in time (see below) */
    NSASM_SCATTER_ATOMIC = 1, /* one thread per element, 12 global atomic adds */
    NSASM_SCATTER_PATCH = 2,  /* element patches staged through LDS: nodes gathered
                                 once per patch, element contributions summed per
                                 node in LDS, one global atomic add per patch node
                                 and component */
    NSASM_SCATTER_PATCH_GATHER = 3 /* as PATCH, but each patch writes its per-node sums
                                 to a partial-sum buffer owned by the mesh and a
                                 second kernel sums them per node in a fixed order:
                                 no atomics, bitwise reproducible; assembly calls
                                 on one mesh must not overlap in time */
} nsasm_scatter;

/* Set in nsasm_params.flags: add into the output instead of overwriting it. */
#define NSASM_ACCUMULATE 1u

/* Eddy-viscosity models (nsasm_params.eddy_model), both evaluated once per
 * element from its constant velocity gradient G = grad u, with filter width
 * Delta = V^(1/3) and C_s = smagorinsky_cs (Sec. V-B computes the model on the
 * fly, once per element):
 *   SMAGORINSKY: mu_t = rho (C_s Delta)^2 |S|, S = (G + G^T)/2, |S| = sqrt(2 S:S).
 *   VREMAN (the paper's model; Vreman, Phys. Fluids 16, 2004): with
 *     alpha_ij = du_j/dx_i, beta_ij = Delta^2 sum_m alpha_mi alpha_mj,
 *     B = b11 b22 - b12^2 + b11 b33 - b13^2 + b22 b33 - b23^2,
 *     mu_t = rho c sqrt(B / alpha:alpha), c = 2.5 C_s^2, and mu_t = 0 where
 *     alpha:alpha = 0 or B <= 0.
 * The VJP differentiates mu_t, taking d mu_t / d G = 0 where the model is not
 * differentiable (|S| = 0; B = 0). */
#define NSASM_EDDY_SMAGORINSKY 0u
#define NSASM_EDDY_VREMAN 1u

/* Convective forms (nsasm_params.convective_form).  The paper calls Alya's
 * convection scheme energy preserving (Sec. II) without printing its discrete
 * form; these are the standard Galerkin forms of the same continuous term
 * rho (u . grad) u, replacing rho G u_h in the integrand of R^e_a:
 *   ADVECTIVE   (u . grad) u                          = G u
 *   DIVERGENCE  div(u (x) u)                          = G u + tr(G) u
 *   SKEW        the mean of the two above             = G u + tr(G) u / 2
 *   ROTATIONAL  (curl u) x u                          = G u - G^T u
 *   EMAC        2 D(u) u + (div u) u, D = (G + G^T)/2 = G u + G^T u + tr(G) u
 * (EMAC: Charnyi, Heister, Olshanskii, Rebholz, J. Comput. Phys. 2017).  With
 * the 4-point rule these integrate exactly, so summed over the mesh the
 * skew-symmetric, rotational and EMAC forms exchange no kinetic energy
 * (sum_n u_n . R^conv_n) except through the boundary flux of u |u|^2 (zero
 * for ROTATIONAL, and for the others when u = 0 on the boundary). */
#define NSASM_CONVECTIVE_ADVECTIVE 0u
#define NSASM_CONVECTIVE_DIVERGENCE 1u
#define NSASM_CONVECTIVE_SKEW 2u
#define NSASM_CONVECTIVE_ROTATIONAL 3u
#define NSASM_CONVECTIVE_EMAC 4u

typedef struct {
    double rho;            /* density, constant (> 0) */
    double mu;             /* molecular dynamic viscosity, constant (>= 0) */
    double smagorinsky_cs; /* model constant C_s; 0 disables the eddy viscosity */
    double body_force[3];  /* constant body-force acceleration f; term is +rho f */
    uint32_t flags;        /* bitwise OR of NSASM_ACCUMULATE, or 0 */
    uint32_t eddy_model;   /* NSASM_EDDY_SMAGORINSKY (0) or NSASM_EDDY_VREMAN */
    uint32_t convective_form; /* NSASM_CONVECTIVE_* (0 = advective) */
    uint32_t reserved;     /* must be 0 */
} nsasm_params;

typedef struct {
    int32_t renumber;    /* 1 (default): sort elements along a Hilbert curve and
                            renumber nodes by first touch; 0: keep user order */
    int32_t scatter;     /* nsasm_scatter */
    int32_t patch_elems; /* elements per patch, 32..256 in steps of 32; 0 = 256,
                            or 128 when a 256-element patch would touch more
                            than 256 distinct nodes */
    int32_t reserved;    /* must be 0 */
} nsasm_mesh_options;

typedef struct {
    int64_t n_nodes;
    int64_t n_elems;
    int32_t scatter;         /* resolved nsasm_scatter: ATOMIC, PATCH or PATCH_GATHER */
    int32_t renumbered;      /* 1 if mesh order differs from user order */
    int32_t n_patches;       /* 0 when scatter == ATOMIC */
    int32_t patch_elems;
    int32_t max_patch_nodes; /* largest number of distinct nodes in one patch */
    int32_t reserved;
    int64_t patch_node_refs; /* sum over patches of their distinct nodes */
} nsasm_mesh_info_t;

/*
 * Build a mesh: validate the connectivity, then (renumber = 1) order elements
 * along a Hilbert curve of their centroids, renumber nodes in order of first
 * use by that element order, and cut the element sequence into patches.
 * Locality of nodal gathers and scatters is what this buys (Sec. V-C:
 * indirect nodal accesses dominate once intermediates live in registers, and
 * nodal reuse happens in the cache shared by the threads).
 *
 * coords  : device, n_nodes x 3 doubles, user node order.
 * conn    : device, n_elems x 4 int32 node ids in [0, n_nodes), 4 distinct per
 *           element; local vertex order and orientation are free.
 * opts    : may be NULL (defaults above).
 * out     : receives the handle; set to NULL on failure (nothing is leaked).
 * Errors  : INVALID_ARGUMENT (null/host pointers, n <= 0, n_nodes >= 2^31,
 *           n_elems >= 2^29, bad options), BAD_CONNECTIVITY, DEGENERATE_ELEMENT
 *           (|det J| <= 64 eps |d1||d2||d3| with d_k = x_k - x_0, a subnormal
 *           det J or a non-finite vertex: within rounding of a flat element,
 *           where 1/det J would be noise), OUT_OF_MEMORY, DEVICE; UNSUPPORTED
 *           when scatter = PATCH is asked for and some patch has more than 256
 *           distinct nodes.
 */
nsasm_status nsasm_mesh_create(const double *coords, int64_t n_nodes, const int32_t *conn,
                               int64_t n_elems, const nsasm_mesh_options *opts, void *stream,
                               nsasm_mesh **out);

/* Library helper, no passage of the paper.  Free a mesh and its device
 * buffers (synchronises the device).  NULL is OK. */
nsasm_status nsasm_mesh_destroy(nsasm_mesh *mesh);

/* Library helper, no passage of the paper.  Sizes and layout decisions of a
 * mesh, written to the caller's host struct `info`.  Errors: INVALID_ARGUMENT
 * for a NULL mesh or info. */
nsasm_status nsasm_mesh_info(const nsasm_mesh *mesh, nsasm_mesh_info_t *info);

/* Library helper, no passage of the paper (the renumbering of
 * nsasm_mesh_create).  mesh_id_of_user: device, n_nodes int32 (caller-owned);
 * entry k is the mesh-order index of user node k (identity when not
 * renumbered).  Asynchronous on stream.  Errors: INVALID_ARGUMENT (NULL mesh,
 * non-device pointer), DEVICE. */
nsasm_status nsasm_mesh_permutation(const nsasm_mesh *mesh, int32_t *mesh_id_of_user, void *stream);

/* Library helper, no passage of the paper.  Internal connectivity: conn_mesh
 * (device, n_elems x 4 int32, mesh node ids, mesh element order) and
 * user_elem (device, n_elems int32, user index of each mesh-order element),
 * both caller-owned.  Either may be NULL.  Asynchronous on stream.  Errors:
 * INVALID_ARGUMENT (NULL mesh, non-device pointer), DEVICE. */
nsasm_status nsasm_mesh_connectivity(const nsasm_mesh *mesh, int32_t *conn_mesh, int32_t *user_elem,
                                     void *stream);

/* Library helper, no passage of the paper.  Reorder a per-node field with
 * ncomp (1..16) components between user order and mesh order:
 * mesh_ordered[perm[k]] = user[k] and back.  Both arrays are device,
 * n_nodes x ncomp, caller-owned, element type per precision (double / float),
 * and must not overlap.  Asynchronous on stream.  Errors: INVALID_ARGUMENT
 * (NULL mesh, bad ncomp or precision, non-device or identical pointers),
 * DEVICE. */
nsasm_status nsasm_to_mesh_order(const nsasm_mesh *mesh, int32_t ncomp, nsasm_precision precision,
                                 const void *user, void *mesh_ordered, void *stream);
nsasm_status nsasm_from_mesh_order(const nsasm_mesh *mesh, int32_t ncomp, nsasm_precision precision,
                                   const void *mesh_ordered, void *user, void *stream);

/*
 * Assemble the momentum RHS (definition at the top of this file; Sec. II for
 * the operation, Sec. V-A and V-B for its per-element form).
 * u   : device, n_nodes x 3, mesh order.    p : device, n_nodes, mesh order.
 * rhs : device, n_nodes x 3, mesh order; overwritten (or added to with
 *       NSASM_ACCUMULATE).  Must not overlap u or p.
 * With NSASM_SCATTER_PATCH_GATHER (the default where the mesh allows it) the
 * summation order is fixed and results are bitwise reproducible; with the
 * atomic scatters it is unspecified and results may differ between calls by
 * rounding.  Calls on one gather-scatter mesh share its partial-sum buffer:
 * they must not overlap in time (one stream, or ordered by events).  No
 * allocation, memset or host synchronisation happens inside, so the call may
 * be captured in a HIP graph.  Asynchronous on stream.
 * Errors: INVALID_ARGUMENT (null/host pointers, rho <= 0, mu < 0, cs < 0,
 * non-finite parameters, unknown precision, flags, eddy model or convective
 * form, non-zero reserved field), DEVICE.
 */
nsasm_status nsasm_assemble_rhs(const nsasm_mesh *mesh, const nsasm_params *params,
                                nsasm_precision precision, const void *u, const void *p, void *rhs,
                                void *stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * operation, arguments, ordering and results as nsasm_assemble_rhs, bit for
 * bit, but with the gather scatter the per-patch partial sums go to a fixed
 * 64 MiB region that the library holds on each GPU from its load until the
 * process ends, not to the mesh's buffer.  No hipMalloc, hipFree, memset or
 * allocating library routine is called.  (The other scatters use no scratch
 * memory; for them this is nsasm_assemble_rhs.)
 * Limit: 3 x (patch node references, nsasm_mesh_info_t.patch_node_refs) x
 * (8 bytes FP64, 4 bytes MIXED) must not exceed 64 MiB, i.e. about 6 M
 * tetrahedra in FP64 and 12 M in MIXED on cube-like meshes; larger meshes
 * are refused with UNSUPPORTED.
 * Every such call on one GPU uses the same region, whatever the mesh: calls
 * that overlap in time on one GPU (several streams, several threads) race
 * and give wrong results.  The region keeps the last call's contents; every
 * partial sum a call reads was written by that call, so nothing needs
 * clearing.
 * Errors: as nsasm_assemble_rhs, plus INVALID_ARGUMENT when the current
 * device is not the mesh's device and UNSUPPORTED beyond the limit.
 */
nsasm_status nsasm_assemble_rhs_noalloc(const nsasm_mesh *mesh, const nsasm_params *params,
                                        nsasm_precision precision, const void *u, const void *p,
                                        void *rhs, void *stream);

/*
 * Velocity vector-Jacobian product of the assembled RHS:
 *   grad_u = (d rhs / d u)^T adjoint,
 * the transpose of the linearisation of the Sec. II / V-B operation (the
 * paper states no adjoint; this is its exact derivative),
 * recomputing the element quantities (nothing is stored by the forward call).
 * The pressure and body-force terms do not depend on u.  The eddy viscosity
 * is differentiated as stated at nsasm_params.
 * u, adjoint : device, n_nodes x 3, mesh order.
 * grad_u     : device, n_nodes x 3, mesh order; overwritten (or added to with
 *              NSASM_ACCUMULATE).  Must not overlap the inputs.
 * Errors and ordering as nsasm_assemble_rhs.
 */
nsasm_status nsasm_assemble_rhs_vjp(const nsasm_mesh *mesh, const nsasm_params *params,
                                    nsasm_precision precision, const void *u, const void *adjoint,
                                    void *grad_u, void *stream);

/*
 * Pressure vector-Jacobian product of the assembled RHS:
 *   grad_p = (d rhs / d p)^T adjoint
 * (exact derivative of the Sec. II / V-B operation; the paper states none).
 * The RHS depends on p only through the pressure-gradient term, which is
 * linear in p (per element -(V/4) grad p at every vertex), so grad_p does not
 * depend on u and the eddy viscosity plays no part.
 * adjoint : device, n_nodes x 3, mesh order.
 * grad_p  : device, n_nodes, mesh order; overwritten (or added to with
 *           NSASM_ACCUMULATE).  Must not overlap adjoint.
 * Errors and ordering as nsasm_assemble_rhs.
 */
nsasm_status nsasm_assemble_rhs_vjp_p(const nsasm_mesh *mesh, const nsasm_params *params,
                                      nsasm_precision precision, const void *adjoint, void *grad_p,
                                      void *stream);

/*
 * Jacobian-vector product (directional derivative) of the assembled RHS
 * (exact derivative of the Sec. II / V-B operation; the paper states none):
 *   drhs = (d rhs / d u) du + (d rhs / d p) dp,
 * recomputing the element quantities; the eddy viscosity is differentiated as
 * stated at nsasm_params.  This is the product a Jacobian-free Newton-Krylov
 * solver of an implicit momentum step needs.
 * u, du : device, n_nodes x 3, mesh order.   dp : device, n_nodes, or NULL (0).
 * drhs  : device, n_nodes x 3, mesh order; overwritten (or added to with
 *         NSASM_ACCUMULATE).  Must not overlap the inputs.
 * Errors and ordering as nsasm_assemble_rhs.
 */
nsasm_status nsasm_assemble_rhs_jvp(const nsasm_mesh *mesh, const nsasm_params *params,
                                    nsasm_precision precision, const void *u, const void *du,
                                    const void *dp, void *drhs, void *stream);

/*
 * Lumped volume of every node, V^L_n = sum over the elements e containing n
 * of V_e / 4: the row sums of the P1 mass matrix divided by the density,
 * computed once at mesh creation (the mass of the explicit momentum stage of
 * Sec. II).  lumped: device, n_nodes doubles, mesh order, caller-owned; 0 at
 * nodes no element references.  Asynchronous on stream.  Errors:
 * INVALID_ARGUMENT (NULL mesh, non-device pointer), DEVICE.
 */
nsasm_status nsasm_mesh_lumped_volume(const nsasm_mesh *mesh, double *lumped, void *stream);

/*
 * One explicit momentum stage of the fractional-step scheme (Sec. II: the
 * momentum equation is integrated explicitly; the RHS assembled here is what
 * the stage advances).  With the lumped mass M_L,n = rho V^L_n:
 *   rhs   = the assembled RHS of (u, p)       (as nsasm_assemble_rhs)
 *   u_new[n][i] = u[n][i] + dt rhs[n][i] / (rho V^L_n)   if bit i of mask[n] is 0,
 *   u_new[n][i] = u[n][i]                               if it is 1
 * (Dirichlet components keep the value the caller stored in u).  A node that
 * no element references has V^L_n = 0 and rhs 0 and keeps u_new = u.
 * u              : device, n_nodes x 3, mesh order.   p : device, n_nodes.
 * dirichlet_mask : device, n_nodes bytes (bits 0..2 = x, y, z), or NULL (none).
 * rhs            : device, n_nodes x 3, receives the assembled RHS; may be NULL
 *                  when the mesh uses NSASM_SCATTER_PATCH_GATHER (the update is
 *                  then fused into the gather kernel and the RHS never reaches
 *                  memory), required otherwise.
 * u_new          : device, n_nodes x 3; may be u itself (in-place update) but
 *                  must not otherwise overlap an input.
 * dt: finite.  params->flags must be 0.  Asynchronous on stream.
 * Errors: as nsasm_assemble_rhs, plus INVALID_ARGUMENT for a non-finite dt,
 * non-zero flags, a missing rhs or overlapping buffers.
 */
nsasm_status nsasm_explicit_update(const nsasm_mesh *mesh, const nsasm_params *params,
                                   nsasm_precision precision, double dt, const void *u, const void *p,
                                   const uint8_t *dirichlet_mask, void *rhs, void *u_new, void *stream);

/*
 * Attainable memory bandwidth: b[k] = s * a[k] for k < n, the Scale kernel
 * whose measured rate, against the FP64 peak, gives the machine balance that
 * the paper's roofline analysis uses (Sec. III-C).  One read and one write
 * stream, 16 bytes moved per element; with arrays well beyond the last-level
 * cache the rate is what a streaming kernel can draw from HBM.
 * a, b : device, n doubles each; must not overlap (the caller owns both).
 *        Both 16-byte aligned -> 16-byte accesses; otherwise 8-byte ones.
 * n    : >= 0; 0 does nothing and checks no pointer.
 * Asynchronous on stream.
 * Errors: INVALID_ARGUMENT for n < 0, a NULL or non-device pointer, or
 * overlapping arrays; DEVICE if the launch fails.
 */
nsasm_status nsasm_stream_scale(const double *a, double *b, int64_t n, double s, void *stream);

/*
 * Atomic scatter rate: out[index[k] * ncomp + c] += value for k < n and
 * c < ncomp, each a device-scope atomic add, one thread per index entry in
 * index order.  This is the immediate scatter of the paper's final GPU kernel
 * (Sec. V-D: each element adds its local RHS straight into the global
 * vector), without the element arithmetic, so a caller can price an atomic:
 * with index = the mesh-order connectivity (4 entries per element) and
 * ncomp = 3 it issues exactly the atomics of an atomic-scatter assembly.
 * index : device, n int32 row numbers; entries outside [0, n_out_rows) are
 *         skipped.
 * out   : device, n_out_rows x ncomp, double (NSASM_FP64) or float
 *         (NSASM_MIXED); accumulated into, not cleared.
 * ncomp : 1..16.  n, n_out_rows : >= 0; n = 0 does nothing.
 * Asynchronous on stream.  The order of the additions is unspecified.
 * Errors: INVALID_ARGUMENT (NULL or non-device pointer, bad sizes, unknown
 * precision), DEVICE.
 */
nsasm_status nsasm_scatter_add(const int32_t *index, int64_t n, int32_t ncomp, nsasm_precision precision,
                               double value, void *out, int64_t n_out_rows, void *stream);

/*
 * Library helper for measurement, no passage of the paper (the paper times
 * its kernels one by one, Sec. III-A; this lets a caller do the same with HIP
 * events, live).  The next assembly call made on this thread
 * (nsasm_assemble_rhs, _noalloc, _vjp, _vjp_p, _jvp, nsasm_explicit_update)
 * launches its element kernel (patch kernel or per-element atomic kernel)
 * with element_start / element_stop and its node kernel (the gather of the
 * gather scatter, or the update kernel) with gather_start / gather_stop
 * through hipExtLaunchKernelGGL, which records each event at its kernel's
 * own start or end: hipEventElapsedTime(start, stop) is that kernel's
 * duration.  Each argument is a hipEvent_t created by the caller (who keeps
 * owning it) or NULL (not recorded); four NULLs cancel a pending request.
 * The call consumes the events whether it succeeds or not; no other function
 * records them.  Always returns NSASM_OK.
 */
nsasm_status nsasm_set_kernel_events(void *element_start, void *element_stop, void *gather_start,
                                     void *gather_stop);

/* Library helper, no passage of the paper.  Message for the last non-OK
 * status on this thread ("" if none); the string is owned by the library and
 * valid until the next call on this thread. */
const char *nsasm_last_error(void);

/* Library helper, no passage of the paper.  Library version string, e.g.
 * "0.2.0" (static storage). */
const char *nsasm_version(void);

#ifdef __cplusplus
}
#endif

#endif /* NSASM_H */
