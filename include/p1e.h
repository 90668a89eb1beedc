/*
 * p1e.h -- C ABI of libp1e: P1 finite-element energies and their gradients on one AMD
 * Instinct MI355X (gfx950).
 *
 * Method: Moskovka & Valdman, "Fast MATLAB evaluation of nonlinear energies using FEM in 2D
 * and 3D: Nodal elements" (arXiv 2109.01158). For a P1 (linear nodal) field v on a triangle
 * or tetrahedron mesh the library evaluates, for every element at once,
 *
 *     J(v) = J_grad(v) - b . v,   J_grad(v) = sum_T |T| W(F_T(v))      (Sections 1, 3.1, 3.2)
 *
 * with b = M f (consistent P1 mass matrix times the nodal load), and the gradient of J over
 * every free degree of freedom at once, either exactly (Section 6.2) or by patch central
 * differences (Section 6.1). Densities: compressible Neo-Hookean (eq. neoHook, 2D and 3D)
 * and the scalar p-Laplacian (eq. pLaplacian).
 *
 * Conventions shared by every entry point
 *   - DOF numbering: DOF n = d*i + j for node i and component j (Section 5, eq. bvvectors).
 *     A DOF is free unless the mesh description prescribes it (Dirichlet). The vector
 *     "vhat" holds the free DOFs of v in ascending n; gradients come back in the same order.
 *   - Sign of the linear part: J = J_grad - b.v, so dJ/dv = dJ_grad/dv - b.
 *   - Neo-Hookean v is the deformation (v = x is the undeformed state); the Dirichlet
 *     values of v are taken from the mesh description.
 *   - An element with det F <= 0 or a non-finite density is "bad": the energy becomes +Inf
 *     and the number of bad elements is written to *flag. Gradients are then undefined.
 *   - Device pointers: every pointer named *_dev, vhat, g, out3, flag is device memory on the
 *     current HIP device; "stream" is a hipStream_t (NULL = default stream). Compute entry
 *     points only enqueue work on that stream and return without synchronising.
 *   - Memory: the library never allocates device memory. p1e_mesh_bind places the mesh and
 *     all scratch arrays in one caller-owned device buffer that the caller keeps alive until
 *     p1e_mesh_destroy (or a re-bind). Host arrays passed to p1e_mesh_create are copied. The
 *     one device array of its own is the fixed static scratch of p1e_grad_exact_static.
 *   - Threads: a mesh handle is not thread-safe, and two calls on the same mesh must not
 *     overlap on the device (they share its scratch arrays); distinct handles are independent.
 *   - Errors: entry points return P1E_OK (0) or a negative status; p1e_last_error() gives a
 *     thread-local message for the last failure on the calling thread. No C++ exception
 *     crosses this interface.
 */
#ifndef P1E_H
#define P1E_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------------ status codes */
#define P1E_OK 0
#define P1E_EINVAL (-1)  /* bad argument (null pointer, dimension, index out of range, ...) */
#define P1E_EDEGEN (-2)  /* a degenerate element (zero size) in the mesh */
#define P1E_ENOMEM (-3)  /* device buffer too small for what was asked */
#define P1E_EHIP (-4)    /* a HIP runtime call or kernel launch failed */
#define P1E_EDOMAIN (-5) /* no admissible point (bad elements) where one was required */
#define P1E_EBUSY (-6)   /* queue full */
#define P1E_ESTATE (-7)  /* call made in the wrong state (e.g. mesh not bound for a mode) */

/* ------------------------------------------------------------------ energy kinds */
#define P1E_PLAPLACE 1 /* W(g) = |g|^p / p, scalar field (d = 1), p > 1 (eq. pLaplacian) */
#define P1E_NEOHOOKE 2 /* W(F) = C1 (|F|^2 - dim - 2 log det F) + D1 (det F - 1)^2,
                          vector field (d = dim) (eq. neoHook) */
#define P1E_SVK 3      /* St. Venant-Kirchhoff, the extension Section 2 names after eq. neoHook:
                          W(F) = C1 |E|^2 + D1 (tr E)^2 with E = (F^T F - I) / 2, i.e.
                          C1 = mu and D1 = lambda / 2 (Lame constants); vector field (d = dim),
                          finite for every F (no bad elements but non-finite values). Energy,
                          exact gradient and patch differences; not served by p1e_server. */
#define P1E_PLAPLACE_ORTHO 5 /* the p-Laplacian with the component-wise norm of the gradient,
                          W(g) = sum_m |g_m|^p / p, scalar field (d = 1), p > 1: the density whose
                          minima Benchmark 6 prints (Table 6; eq. pLaplacian writes |g|^p / p,
                          P1E_PLAPLACE). Everything P1E_PLAPLACE has, minimizer and server
                          included. */
#define P1E_GINZBURG_LANDAU 4 /* Ginzburg-Landau, the scalar first-gradient problem Section 7
                          names: W = C1 |grad u|^2 + D1 (u^2 - 1)^2 (C1 = eps/2, D1 = 1/4 for the
                          textbook energy eps/2 |grad u|^2 + (u^2 - 1)^2 / 4), scalar field
                          (d = 1); the potential is integrated exactly over each element
                          (a quartic of the P1 field). Energy, exact gradient and patch
                          differences; not served by p1e_server or p1e_minimize. */

/* ------------------------------------------------------------------ precision modes */
/* Each compute call names one mode; p1e_mesh_bind takes a bit mask of the modes to prepare. */
#define P1E_FP64 1  /* all element arithmetic, sums and gradients in FP64 */
#define P1E_MIXED 2 /* element arithmetic in FP32 on the displacement gradient; log det F,
                       the energy sum (compensated) and gradient accumulation in FP64 */
#define P1E_FD 4    /* bind-only bit: arrays for the patch central-difference gradient (FP64) */

/* ------------------------------------------------------------------ mesh flags */
/* Internal numbering (never visible in vhat or gradients): the elements are grouped into
 * tiles of consecutive elements, each evaluated by one workgroup with its nodal values and
 * element results in on-chip memory, and the nodes are numbered in order of first use. By
 * default the elements are first sorted along a Morton curve of their centroids, which makes
 * tiles compact. P1E_INPUT_ORDER keeps the caller's element order instead (for callers that
 * already number elements in compact clusters). Either choice changes only the order of
 * floating-point sums. */
#define P1E_INPUT_ORDER 1
/* Element geometry (B^-1 and |T|, Section 4.1). By default, element records that agree to
 * 2^-40 of each component's largest magnitude share one class, and a mesh with at most 64
 * classes (uniformly refined structured meshes have a few) whose every record lies within
 * 2^-42 of its class's first record (relative to each component's largest magnitude; the
 * deviation is reported in p1e_mesh_info) stores one record per class and a one-byte class
 * per element; the elements of a class then use its first record, which differs from their
 * own only by the rounding of node coordinates. Any other mesh stores no per-element
 * geometry: its tiles (then of at most 512 nodes) keep each node's coordinates as an offset
 * from the tile's centroid (FP32 in mixed mode, FP64 otherwise) and the element pass forms
 * B^-1 and |T| from its vertices' offsets. P1E_FULL_GEOMETRY: always store B^-1 and |T| per
 * element instead. */
#define P1E_FULL_GEOMETRY 4

typedef struct p1e_mesh p1e_mesh;

/* Material constants of a deformation density from Young's modulus E > 0 and Poisson's ratio
 * -1 < nu < 1/2 (host only). kind = P1E_NEOHOOKE: the constants of Benchmark 2 (Section 7),
 * C1 = mu / 2 and D1 = K / 2 with mu = E / (2 (1 + nu)) and the bulk modulus
 * K = E / (3 (1 - 2 nu)), used unchanged in 2D; kind = P1E_SVK: C1 = mu and D1 = lambda / 2
 * with lambda = E nu / ((1 + nu)(1 - 2 nu)). Writes *C1, *D1; P1E_EINVAL for another kind,
 * null outputs or E, nu out of range. */
int p1e_material_constants(int kind, double E, double nu, double *C1, double *D1);

/* Mesh and problem description (all arrays are host memory, row-major, 0-based). */
typedef struct p1e_mesh_desc {
  int32_t dim;   /* 2 (triangles) or 3 (tetrahedra) */
  int32_t ncomp; /* d: 1 for P1E_PLAPLACE(_ORTHO) and P1E_GINZBURG_LANDAU, dim for
                    P1E_NEOHOOKE and P1E_SVK */
  int32_t kind;  /* P1E_PLAPLACE, P1E_PLAPLACE_ORTHO, P1E_NEOHOOKE, P1E_SVK or
                    P1E_GINZBURG_LANDAU */
  int32_t flags; /* 0 or P1E_INPUT_ORDER | P1E_FULL_GEOMETRY */
  int64_t nn; /* number of nodes, 1 <= nn < 2^28 */
  int64_t ne; /* number of elements, 0 <= ne < 2^29 */
  const int32_t *conn;       /* [ne][dim+1] vertex indices, distinct, in [0, nn) */
  const double *coords;      /* [nn][dim] node coordinates */
  const uint8_t *dirichlet;  /* [nn][ncomp], nonzero = prescribed DOF; NULL = none */
  const double *dirichlet_values; /* [nn][ncomp] values of prescribed DOFs; NULL = 0 */
  const double *load;        /* [nn][ncomp] nodal values of the P1 load f; NULL = 0 */
  double p;                  /* p-Laplacian exponent, p > 1 */
  double C1, D1;             /* Neo-Hookean constants (C1 = mu/2, D1 = K/2 in Benchmark 2);
                                St. Venant-Kirchhoff: C1 = mu, D1 = lambda/2; Ginzburg-Landau:
                                the coefficients of |grad u|^2 and (u^2 - 1)^2 */
} p1e_mesh_desc;

typedef struct p1e_mesh_info {
  int64_t nn, ne;
  int64_t n_free_nodes; /* nodes with at least one free DOF (Remark 1) */
  int64_t n_free_dofs;  /* length of vhat and of gradients */
  int64_t nnz;          /* patch incidences of free nodes: sum over free nodes of |T^i| */
  int32_t dim, ncomp, kind, max_valence; /* max_valence = largest |T^i| */
  double total_volume, min_volume, max_volume;
  double dirichlet_bv; /* sum over prescribed DOFs of b_n v_n (constant part of b.v) */
  uint64_t alignment;  /* required alignment of the bound device buffer (bytes) */
  int32_t geometry_classes; /* distinct element records kept as a table (0: none) */
  int32_t geometry_mode;    /* 0: B^-1 and |T| stored per element; 1: geometry classes; 2: formed
                               in the element pass from the vertex coordinates */
  int64_t n_tiles;      /* element tiles */
  int64_t n_tile_nodes; /* sum over tiles of the distinct nodes of the tile */
  int64_t n_halo_rows;  /* free nodes whose patch spans several tiles (or no element) */
  int64_t n_halo_slots; /* partial patch sums of halo rows (one per tile and halo row) */
  double geometry_class_deviation; /* largest |record - class record| of an element, relative
                                      to the component's largest magnitude (0: no classes) */
} p1e_mesh_info;

/* Build a mesh handle: validates the description, computes element geometry (|T| and basis
 * gradients, Section 4.1), the free-node patch lists (Section 4.2, split by element tiles
 * into rows of (element, local vertex) pairs), the DOF maps and b = M f (Section 3.2).
 * Host-only; needs no GPU. Returns P1E_EINVAL or P1E_EDEGEN on bad input, and P1E_EINVAL for
 * a mesh beyond the library's limits: fewer than 2^28 free DOFs, and every per-node, per-DOF
 * and per-halo-slot array of the bound buffer below 4 GiB. */
int p1e_mesh_create(const p1e_mesh_desc *desc, p1e_mesh **out);

/* Release the handle (host memory only; the bound device buffer belongs to the caller). */
void p1e_mesh_destroy(p1e_mesh *mesh);

int p1e_mesh_get_info(const p1e_mesh *mesh, p1e_mesh_info *out);

/* Device bytes p1e_mesh_bind needs for the modes in mask (P1E_FP64 | P1E_MIXED | P1E_FD).
 * Returns 0 for an invalid mask or handle. */
uint64_t p1e_workspace_bytes(const p1e_mesh *mesh, int mode_mask);

/* Lay the mesh arrays and scratch out in the caller-owned device buffer dev_buf (aligned to
 * info.alignment, at least p1e_workspace_bytes(mesh, mode_mask) bytes) and upload them on
 * stream. Synchronises stream before returning. P1E_ENOMEM if bytes is too small. The
 * first bind whose mask holds P1E_MIXED also reorders, on the host and once per handle, where
 * each tile keeps its nodal values in LDS (fewer LDS bank conflicts for 16-byte float reads);
 * results do not depend on it. Not thread-safe against other calls on the same handle. */
int p1e_mesh_bind(p1e_mesh *mesh, void *dev_buf, uint64_t bytes, int mode_mask, void *stream);

/* Energy (Section 5). vhat: [n_free_dofs] FP64. out3: 3 doubles {J, J_grad, b.v}.
 * flag: 1 int32 = number of bad elements. prec: P1E_FP64 or P1E_MIXED (must be bound). */
int p1e_energy(p1e_mesh *mesh, const double *vhat, int prec, double *out3, int32_t *flag,
               void *stream);

/* Exact gradient (Section 6.2): g[n] = dJ/dv_n for the free DOFs, FP64, in vhat order.
 * Element forces |T| dW/dF grad phi are formed per element and summed per free node over
 * its patch in a fixed order (no atomics): within an element tile from on-chip memory, then
 * over the tiles the patch spans. out3 (nullable) receives the energy of the same call, as
 * in p1e_energy; flag receives the bad-element count. */
int p1e_grad_exact(p1e_mesh *mesh, const double *vhat, int prec, double *g, double *out3,
                   int32_t *flag, void *stream);

/* p1e_grad_exact with its scratch in a fixed array inside the library, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid allocation). Same arguments, results and stream semantics as p1e_grad_exact (bitwise
 * the same values); the call allocates nothing. Its scratch (tile partials [2][n_tiles] of
 * 16 bytes, bad counts [n_tiles] of 4 bytes, halo partials [n_halo_slots][ncomp] of 8 bytes,
 * each region rounded up to 256 bytes) lives in one static device array of
 * P1E_STATIC_SCRATCH_BYTES per GPU, held from the library's first use of a device until the
 * process ends; a mesh that needs more returns P1E_ENOMEM. Every call on one GPU shares that
 * array: calls that overlap on the device (other streams, other threads) race and must be
 * ordered by the caller. The mesh's own scratch region is not touched. */
#define P1E_STATIC_SCRATCH_BYTES (64ull << 20)
int p1e_grad_exact_static(p1e_mesh *mesh, const double *vhat, int prec, double *g, double *out3,
                          int32_t *flag, void *stream);

/* The exact gradient in two calls, for a differentiation hook whose backward pass runs later
 * than its forward pass:
 *   p1e_energy_forces  energy as p1e_energy, and the exact gradient (as p1e_grad_exact)
 *                      kept in the mesh's scratch arrays;
 *   p1e_grad_gather    g[n] = s * (kept gradient)[n] with s = *scale (a device double; NULL
 *                      means 1), which is s * (patch sum of the element forces - b_n).
 * p1e_grad_gather returns P1E_ESTATE unless a p1e_energy_forces call with the same prec came
 * before it (p1e_minimize clears the kept gradient). Calls must be enqueued in that order on
 * one stream, or ordered by the caller. */
int p1e_energy_forces(p1e_mesh *mesh, const double *vhat, int prec, double *out3,
                      int32_t *flag, void *stream);
int p1e_grad_gather(p1e_mesh *mesh, int prec, const double *scale, double *g, void *stream);

/* The backward pass of a differentiation hook whose forward pass wrote the exact gradient
 * (p1e_grad_exact, Section 6.2) into a buffer of its own: g[n] *= s in place for the
 * mesh's n_free_dofs entries, s = *scale (a device double, not NULL). When s == 1 the kernel
 * writes nothing (every product would return g[n] bitwise). g: device, caller-owned. Stream
 * ordered. P1E_ESTATE if the mesh is not bound. */
int p1e_grad_scale(p1e_mesh *mesh, const double *scale, double *g, void *stream);

/* Patch central differences (Section 6.1, eqs. CD, CDS, sumpatch), FP64 throughout:
 * g[n] = [sum_{T in T^(n)} |T| W(F_T(v + eps e_n)) - sum |T| W(F_T(v - eps e_n))]/(2 eps) - b_n
 * with an absolute step eps > 0 for every DOF. Only the perturbed row of F_T changes
 * (F_T +- eps e_j (x) grad phi_l). Needs the P1E_FD bind bit. flag as above. */
int p1e_grad_patch_fd(p1e_mesh *mesh, const double *vhat, double eps, double *g,
                      int32_t *flag, void *stream);

/* The fourth-order central-difference scheme, the higher-accuracy generalisation Section 6.1
 * mentions after eq. CD, on the same patches and under the same contract as
 * p1e_grad_patch_fd:
 * g[n] = [8 (S_n(eps) - S_n(-eps)) - (S_n(2 eps) - S_n(-2 eps))] / (12 eps) - b_n with
 * S_n(h) = sum_{T in T^(n)} |T| W(F_T(v + h e_n)); truncation error O(eps^4). */
int p1e_grad_patch_fd4(p1e_mesh *mesh, const double *vhat, double eps, double *g,
                       int32_t *flag, void *stream);

/* ------------------------------------------------------------------ minimization
 * A first-order minimization of J over vhat with the exact gradient, as the paper feeds J and
 * grad J to an optimizer (Section 7; the paper uses a trust-region method, this library
 * L-BFGS): memory m, initial inverse Hessian (s.y / y.y) I, a new pair kept only if
 * s.y > 1e-12 |s||y|, Armijo backtracking (c1 = 1e-4, halving, at most 40 trials), the first
 * step (and any step after a restart) scaled so that the largest nodal update is 0.1 h with h
 * the edge of the smallest element's reference cell, and a restart from steepest descent when
 * the L-BFGS direction is not a descent direction. Exactly max_iters accepted iterations
 * unless the gradient vanishes or the line search stalls. */
typedef struct p1e_lbfgs_opts {
  int32_t history;   /* m, 1..8 */
  int32_t max_iters; /* accepted iterations */
  int32_t prec;      /* P1E_FP64 or P1E_MIXED (the mesh must be bound for it) */
  int32_t reserved;
} p1e_lbfgs_opts;

/* status values of a finished minimization */
#define P1E_MIN_OK 0         /* max_iters iterations done */
#define P1E_MIN_STALLED 1    /* 40 halvings without sufficient decrease */
#define P1E_MIN_CONVERGED 2  /* zero gradient */
#define P1E_MIN_BAD_START (-5) /* the start point has bad elements */

typedef struct p1e_min_report {
  int32_t status, iterations, evaluations, reserved;
  double J;      /* final energy */
  double J_grad; /* J_grad of the last evaluated point */
} p1e_min_report;

/* Device workspace bytes of p1e_minimize for this mesh and options. */
uint64_t p1e_minimize_workspace_bytes(const p1e_mesh *mesh, const p1e_lbfgs_opts *opts);

/* Minimize from vhat (device, in/out) on a mesh bound for opts->prec. ws: caller-owned device
 * buffer (256-byte aligned, p1e_minimize_workspace_bytes). Synchronous on stream. Overwrites
 * the mesh's scratch arrays (a following p1e_grad_gather returns P1E_ESTATE). P1E_EDOMAIN if
 * the start point has bad elements; P1E_EINVAL for a P1E_SVK mesh (the minimizer and the
 * server cover the paper's two densities). */
int p1e_minimize(p1e_mesh *mesh, double *vhat, const p1e_lbfgs_opts *opts, void *ws,
                 uint64_t ws_bytes, p1e_min_report *report, void *stream);

/* ------------------------------------------------------------------ serving
 * Continuous batching of many minimizations (as p1e_minimize) of different meshes on one GPU.
 * Requests are submitted with their mesh description; worker threads build the meshes; a
 * request is admitted into a slot, in arrival order, once a slot and enough bytes of the
 * caller's device pool are free; every p1e_server_step advances all admitted requests by one
 * line-search trial with one fixed sequence of batched launches (replayed from a hipGraph when
 * use_graph is set), and retires finished ones, freeing their slot and pool bytes. Each
 * request's result is bitwise the same as when it runs alone. The server is driven by one
 * thread (submit/step/poll); submission may come from any thread. */
typedef struct p1e_server p1e_server;

typedef struct p1e_server_opts {
  int32_t max_slots;     /* requests on the device at once, 1..4096 */
  int32_t history;       /* L-BFGS memory, 1..8 */
  int32_t max_iters;     /* accepted iterations per request */
  int32_t prec;          /* P1E_FP64 or P1E_MIXED */
  int32_t use_graph;     /* replay the step from a captured hipGraph (needs a non-NULL stream) */
  int32_t setup_threads; /* host threads building meshes */
  uint64_t pool_bytes;   /* size of pool */
  void *pool;            /* caller-owned device buffer, 256-byte aligned, kept alive until destroy */
  void *stream;          /* hipStream_t for all device work */
} p1e_server_opts;

typedef struct p1e_request_info {
  int64_t id;
  int32_t status;      /* P1E_MIN_* or a negative P1E_E* setup/admission error */
  int32_t iterations, evaluations, n_free_dofs;
  double J, J_grad;
  double t_submit, t_admit, t_done; /* seconds on the server clock (p1e_server_clock) */
  uint64_t device_bytes;            /* pool bytes the request held */
} p1e_request_info;

/* Bytes at the head of the pool used for the engine tables. */
uint64_t p1e_server_table_bytes(int32_t max_slots, uint64_t pool_bytes);
int p1e_server_create(const p1e_server_opts *opts, p1e_server **out);
void p1e_server_destroy(p1e_server *server);
double p1e_server_clock(const p1e_server *server);
/* Copies the description (and the optional start point vhat0[n0] on the host; NULL: the
 * prescribed values, v = x for Neo-Hookean and 0 for the p-Laplacian); returns its id. */
int p1e_server_submit(p1e_server *server, const p1e_mesh_desc *desc, const double *vhat0,
                      int64_t n0, int64_t *id);
/* As p1e_server_submit for a request that arrives at t_arrival on the server clock (in the
 * future or now): it is neither built nor admitted before then. For replaying arrival traces. */
int p1e_server_submit_at(p1e_server *server, const p1e_mesh_desc *desc, const double *vhat0,
                         int64_t n0, double t_arrival, int64_t *id);
/* Retire finished requests, admit waiting ones, enqueue one step; reports the numbers of
 * admitted and of submitted-but-not-admitted requests. */
int p1e_server_step(p1e_server *server, int32_t *n_active, int32_t *n_waiting);
/* p1e_server_step in a loop until nothing is active or waiting, or max_steps (<= 0: no limit)
 * steps or max_seconds (<= 0: no limit) have passed. */
int p1e_server_run(p1e_server *server, int64_t max_steps, double max_seconds, int32_t *n_active,
                   int32_t *n_waiting);
/* Finished requests not reported before (up to cap). */
int p1e_server_poll(p1e_server *server, p1e_request_info *out, int32_t cap, int32_t *n);
/* Final vhat of a finished request (host copy of n doubles), until p1e_server_release. */
int p1e_server_result_vhat(p1e_server *server, int64_t id, double *dst, int64_t n);
int p1e_server_release(p1e_server *server, int64_t id);

/* Thread-local message of the last failure ("" if none). */
const char *p1e_last_error(void);

/* ------------------------------------------------------------------ kernel timing
 * For measurement harnesses: while enabled, every kernel the library launches is bracketed
 * by HIP events on its launch stream. p1e_prof_collect synchronises the recorded events and
 * returns, per kernel name, the launch count and the summed duration in milliseconds
 * (names are written as one '\n'-separated string into names[names_cap]). */
int p1e_prof_enable(int on);
int p1e_prof_reset(void);
int p1e_prof_collect(char *names, int64_t names_cap, int64_t *counts, double *total_ms,
                     int32_t cap, int32_t *n_out);

#ifdef __cplusplus
}
#endif

#endif /* P1E_H */
