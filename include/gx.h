/*
 * gx.h -- C ABI of libgx, the MI355X (gfx950) interaction engine for the
 * N-body/SPH galaxy integrator of Hirashima et al. (SC '25, arXiv 2510.23330).
 *
 * Scope: the per-step particle-interaction hot path -- Morton-ordered octree,
 * group interaction lists, softened monopole+quadrupole tree gravity, SPH
 * density/pressure and hydro force, FP64 kick/drift and energy audit.
 *
 * Conventions shared by every call
 * --------------------------------
 * Memory      Every array argument named "device" is a pointer into device
 *             memory owned by the caller (contiguous, one element per particle,
 *             structure of arrays, original particle order).  The library never
 *             frees or reallocates caller memory.  It owns only its internal
 *             scratch (sorted copies, tree, lists, sort buffers), kept inside the
 *             context, grow-only, released by gx_destroy.  Arguments named "host"
 *             are host pointers.
 * Streams     Work is enqueued on the context's stream (gx_create / gx_set_stream)
 *             and is asynchronous unless stated otherwise.  Calls that fill a
 *             host gx_stats* or a host output synchronise that stream.
 * Errors      Every int-returning call returns GX_OK (0) or a negative gx_status.
 *             gx_last_error() gives a message for the last failure on a context.
 *             No C++ exception crosses this interface.  A context serves one host
 *             thread at a time.
 * Precision   Positions, velocities, masses, accelerations, potentials, u and
 *             du/dt are FP64.  Pairwise arithmetic is FP32 on coordinates made
 *             relative to each receiving group's centre (Sec. 4.3), with FP32
 *             per-tile partial sums combined in FP64.  GX_PREC_FP64 runs the same
 *             kernels with FP64 pair arithmetic (error audits).
 * Units       Any consistent system; G is an argument.
 */
#ifndef GX_H
#define GX_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gx_ctx gx_ctx;

typedef enum {
    GX_OK = 0,
    GX_EINVAL = -1,     /* null/misaligned pointer, n < 0, bad enum or parameter */
    GX_ENOMEM = -2,     /* device scratch allocation failed */
    GX_EHIP = -3,       /* a HIP runtime call failed (text in gx_last_error) */
    GX_ENOTBUILT = -4,  /* forces requested before gx_tree_build on that slot */
    GX_ESTALE = -5,     /* particle count or pointers differ from the built tree */
    GX_ENOCONV = -6     /* kernel-size iteration hit max_iter somewhere; outputs written */
} gx_status;

/* Tree slots: one tree over all particles (gravity) and one over gas (SPH). */
enum { GX_TREE_ALL = 0, GX_TREE_GAS = 1 };

/* Gravity flags. */
enum {
    GX_QUAD = 1,      /* add the quadrupole term of accepted cells */
    GX_DIRECT = 2,    /* direct sum over all particles (no cells), same kernel */
    GX_PREC_FP64 = 4  /* FP64 pair arithmetic instead of FP32 */
};

/* Counters returned by calls that take a gx_stats* (zeroed by each such call). */
typedef struct {
    int64_t n_pp;        /* particle-particle interactions (self pairs included) */
    int64_t n_pc;        /* particle-cell interactions */
    int64_t n_sph_list;  /* SPH candidate pairs evaluated (list length x receivers) */
    int64_t n_sph_ngb;   /* SPH pairs inside the kernel support */
    int64_t n_groups;    /* receiving groups */
    int64_t n_nodes;     /* tree nodes */
    int64_t n_iter_max;  /* largest kernel-size iteration count */
    int64_t n_noconv;    /* receivers whose kernel size did not converge */
    int64_t n_rewalk;    /* groups whose SPH list had to be rebuilt */
    double ms;           /* wall time of the call on the stream, milliseconds */
    double ms_kernel;    /* time of the call's pairwise kernel alone (HIP events), ms */
} gx_stats;

/* Particle view: device pointers, original order, n elements each.
 * eps2 is the squared softening of each particle and must be > 0 for gravity
 * (the self pair then contributes a finite potential term that is removed).
 * vx/vy/vz are the velocities the SPH force uses (time-centred predictions). */
typedef struct {
    const double *x, *y, *z;
    const double *vx, *vy, *vz;
    const double *m;
    const float *eps2;
    const int64_t *id;
    const uint8_t *type;
    int64_t n;
} gx_particles;

/* Gas state: device pointers, same order and length as the gas gx_particles.
 * u      specific internal energy (the force reads the predicted value)
 * dudt   output of gx_sph_forces
 * H64    kernel size; input guess (<= 0 or NaN means none) and output, FP64
 * H, rho, P, cs, vsig   FP32 outputs (vsig from gx_sph_forces) */
typedef struct {
    double *u, *dudt, *H64;
    float *H, *rho, *P, *cs, *vsig;
    int64_t n;
} gx_gas;

/* Create a context on HIP device `device`, enqueueing on `hip_stream`
 * (a hipStream_t, or NULL for the default stream).  *out receives the handle. */
int gx_create(gx_ctx** out, int device, void* hip_stream);
int gx_destroy(gx_ctx* ctx);
int gx_set_stream(gx_ctx* ctx, void* hip_stream);
const char* gx_last_error(const gx_ctx* ctx);
/* Library build string (architecture and compile options); static storage. */
const char* gx_version(void);

/*
 * gx_tree_build -- Barnes-Hut octree over Morton-sorted particles (Sec. 3.4)
 * with receiving groups that share one interaction list (Sec. 5.2.2, 5.2.4).
 *
 *  1. Root cube: corner x0 = componentwise minimum, side
 *     L = (largest extent) * (1 + 2^-40) (1 if all points coincide).
 *  2. Keys: per axis c = min(2^21 - 1, floor((x - x0) * (2^21 / L))), 63-bit key
 *     interleaving the three 21-bit coordinates, x the most significant bit of
 *     each triple.  FP contraction is off for this arithmetic.
 *  3. Stable sort by key (ties keep input order).
 *  4. Nodes: a node at level l is a run of keys sharing their top 3l bits; it is
 *     split while it holds more than n_leaf particles and l < 21.  Nodes are
 *     numbered in depth-first pre-order with children in key order.
 *  5. Moments (FP64): mass, centre of mass, traceless quadrupole
 *     Q_ab = sum m (3 d_a d_b - |d|^2 delta_ab) about the centre of mass, mass-
 *     weighted mean eps^2, tight bounding box.
 *  6. Groups: maximal nodes holding at most n_group particles (or leaves).
 *
 * p         device particle view (x, y, z, m, eps2 read; eps2 may be NULL for
 *           GX_TREE_GAS, which then uses zero softening moments)
 * which     GX_TREE_ALL or GX_TREE_GAS (independent slots)
 * n_leaf    1..64; n_group n_leaf..4096
 * perm_out  optional device int32[n]: perm_out[s] = original index of sorted slot s
 * stats     optional host; n_nodes and n_groups filled.  This call always
 *           synchronises once (node and group counts size the next kernels).
 */
int gx_tree_build(gx_ctx* ctx, const gx_particles* p, int which, int n_leaf, int n_group,
                  int32_t* perm_out, gx_stats* stats);

/*
 * gx_gravity_forces -- tree gravity from the GX_TREE_ALL slot.
 *
 * Pair law, Eq. 1 (Sec. 3.5): a_i = -G sum_j m_j r_ij / (r_ij^2 + eps_i^2 + eps_j^2)^{3/2},
 * potential phi_i = -G sum_j m_j / (r_ij^2 + eps_i^2 + eps_j^2)^{1/2}, self pair excluded.
 * Walk: for each group G with tight box B_G, a node c with geometric side
 * l_c = L 2^-level and tight box B_c is accepted when l_c^2 < theta^2 d^2,
 * d = minimum distance between B_G and B_c; accepted nodes act through their
 * monopole (+ quadrupole with GX_QUAD):
 *   phi += -G [M/R + r.Q.r/(2 R^5)],  a += -G [M r/R^3 - Q r/R^5 + (5/2)(r.Q.r) r/R^7],
 *   r = r_i - s, R^2 = |r|^2 + eps_i^2 + <eps^2>_c.
 * Rejected leaves contribute their particles pairwise.  Coordinates are made
 * relative to the group's box centre in FP64 and rounded to FP32 (Sec. 4.3).
 *
 * p          the same particle view the tree was built from (GX_ESTALE otherwise)
 * G, theta   gravitational constant, opening angle (theta > 0; ignored with GX_DIRECT)
 * flags      GX_QUAD | GX_DIRECT | GX_PREC_FP64
 * ax..pot    device FP64 outputs [n], overwritten, original order
 * stats      optional host: n_pp, n_pc, n_groups, ms (synchronises)
 */
int gx_gravity_forces(gx_ctx* ctx, const gx_particles* p, double G, double theta, int flags,
                      double* ax, double* ay, double* az, double* pot, gx_stats* stats);

/*
 * gx_sph_density -- kernel size, density and pressure (the kernel-size and
 * density/pressure items of Table 3; Sec. 5.2.5).
 *
 * Kernel: Wendland C4 with compact support H,
 *   W(r, H) = 495 / (32 pi H^3) (1 - q)^6 (1 + 6 q + 35 q^2 / 3),  q = r / H < 1.
 * Each receiver solves (4 pi / 3) H_i^3 rho_i / m_i = n_ngb with
 * rho_i = sum_j m_j W(r_ij, H_i) (self included) by Newton's method kept inside
 * a bracket, until |N_eff - n_ngb| <= tol or max_iter.  Then
 * P = (gamma - 1) rho u, c = sqrt(gamma (gamma - 1) u).
 * Uses the GX_TREE_GAS slot built from `gas`.  g->H64 seeds the iteration when
 * positive; otherwise a seed comes from the group's mean density.
 * Returns GX_ENOCONV (outputs still written) if any receiver hit max_iter.
 */
int gx_sph_density(gx_ctx* ctx, const gx_particles* gas, gx_gas* g, double n_ngb, double gamma,
                   double tol, int max_iter, gx_stats* stats);

/*
 * gx_sph_forces -- hydro force (Table 3/4 "hydro force"), symmetric form
 *   dv_i/dt = -sum_j m_j [A_i gW_i + A_j gW_j + Pi_ij (gW_i + gW_j) / 2] r_ij
 *   du_i/dt =  sum_j m_j [A_i gW_i + Pi_ij (gW_i + gW_j) / 4] (v_ij . r_ij)
 * A = P / rho^2, gW_k r_ij = grad_i W(r_ij, H_k) = -1155/(4 pi H_k^5)(1 + 5q)(1 - q)^5 r_ij,
 * w = v_ij . r_ij / r_ij, v_sig = c_i + c_j - 3 min(w, 0),
 * Pi_ij = -alpha v_sig w / (rho_i + rho_j) when w < 0 else 0, over j != i with
 * r_ij < max(H_i, H_j).  vsig_i = max(c_i, max_j v_sig).  P, rho, H, cs come
 * from gx_sph_density; velocities from gas->vx/vy/vz and u from g->u.
 * ax, ay, az   device FP64 [n]: the hydro acceleration is ADDED to them
 * g->dudt, g->vsig  overwritten
 */
int gx_sph_forces(gx_ctx* ctx, const gx_particles* gas, gx_gas* g, double gamma, double alpha,
                  double* ax, double* ay, double* az, gx_stats* stats);

/*
 * gx_kick_drift -- one half of the second-order leapfrog (Sec. 3.2), FP64
 * (Sec. 4.3 keeps positions and velocities in double precision):
 *   v += a dt_kick;  u += dudt dt_kick;  x += v dt_drift;
 *   vpred = v + a dt_kick;  upred = u + dudt dt_kick   (predictions for the
 *   hydro force at the drifted positions).
 * Call (dt/2, dt) then, after the force, (dt/2, 0).
 * u/dudt/upred may be NULL (then n_u is ignored); they cover the first n_u
 * entries of u (the gas).  vpred_xyz, when non-NULL, is device FP64 [3 n]
 * laid out as vx[n], vy[n], vz[n].  u is floored at u_floor when u_floor > 0.
 */
int gx_kick_drift(gx_ctx* ctx, int64_t n, double dt_kick, double dt_drift, double* x, double* y,
                  double* z, double* vx, double* vy, double* vz, const double* ax,
                  const double* ay, const double* az, int64_t n_u, double* u, const double* dudt,
                  double u_floor, double* vpred_xyz, double* upred);

/*
 * gx_energy -- FP64 energy audit, deterministic two-level reduction:
 *   out[0] = sum m |v|^2 / 2, out[1] = sum m phi / 2, out[2] = sum_gas m u.
 * p: all particles (m, vx, vy, vz), pot: device [n]; m_gas/u: device [n_gas]
 * (may be NULL with n_gas = 0).  out: host double[3].  Synchronises.
 */
int gx_energy(gx_ctx* ctx, const gx_particles* p, const double* pot, int64_t n_gas,
              const double* m_gas, const double* u, double* out);

/*
 * gx_sph_timestep -- Courant step dt = c_cfl min_i H_i / vsig_i (Sec. 1: the
 * fluid-element size over the signal speed), per system or per cube.
 * cube_id: device int32 [n] in [0, n_cubes) or NULL (one system, n_cubes = 1).
 * dt_out: device double [n_cubes].
 */
int gx_sph_timestep(gx_ctx* ctx, const gx_gas* g, double c_cfl, const int32_t* cube_id,
                    int n_cubes, double* dt_out);

/* ---- inspection (tests, tooling); host outputs, synchronous -------------- */

/* Node and group counts of a built slot. */
int gx_tree_counts(gx_ctx* ctx, int which, int64_t* n_nodes, int64_t* n_groups);

/* Copy a built tree to host arrays (any pointer may be NULL):
 * keys[n] sorted keys, perm[n] sorted slot -> original index, box4 = x0,y0,z0,L;
 * per node (pre-order): begin, end, next (pre-order id after the subtree),
 * level, leaf, mass, com[3], quad[6] (xx,yy,zz,xy,xz,yz), eps2bar, lo[3], hi[3];
 * groups[n_groups] node id of each group. */
int gx_tree_export(gx_ctx* ctx, int which, uint64_t* keys, int32_t* perm, double* box4,
                   int32_t* begin, int32_t* end, int32_t* next, int32_t* level, int8_t* leaf,
                   double* mass, double* com, float* quad, float* eps2bar, double* lo,
                   double* hi, int32_t* groups);

/* Sizes of the interaction lists of the last gx_gravity_forces call. */
int gx_gravity_list_sizes(gx_ctx* ctx, int64_t* n_groups, int64_t* n_pc, int64_t* n_pp_ranges);

/* Copy them: pc_off[n_groups+1], pc_node[n_pc]; pp_off[n_groups+1] and
 * pp_begin/pp_end[n_pp_ranges] (sorted-slot ranges of opened leaves, merged
 * where contiguous). */
int gx_gravity_list_export(gx_ctx* ctx, int64_t* pc_off, int32_t* pc_node, int64_t* pp_off,
                           int32_t* pp_begin, int32_t* pp_end);

#ifdef __cplusplus
}
#endif
#endif /* GX_H */
