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
 *             host gx_stats* or a host output synchronise that stream, and so
 *             do the calls whose next launches depend on device-computed sizes
 *             or convergence: gx_tree_build (twice), gx_gravity_forces in tree
 *             mode (once: the list totals), gx_sph_density (once per Newton
 *             pass and list round), gx_sph_forces (list totals, long-list
 *             chunk count); each says so below.
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
    int64_t n_sph_list;  /* SPH candidate pairs evaluated: list length x receivers, and
                            for the density summed over all kernel-size passes */
    int64_t n_sph_ngb;   /* SPH pairs inside the kernel support: force, pairs with
                            r < max(H_i, H_j); density, evaluations with r < H_i
                            summed over all kernel-size passes */
    int64_t n_groups;    /* receiving groups */
    int64_t n_nodes;     /* tree nodes */
    int64_t n_iter_max;  /* largest kernel-size iteration count (SPH density);
                            deepest stack of the one-pass list walk (gravity) */
    int64_t n_noconv;    /* receivers whose kernel size did not converge */
    int64_t n_rewalk;    /* re-walk rounds of the SPH density list (SPH density);
                            1 when the gravity lists took the two-pass path */
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
/* Test hook of the gravity list walk: entries > 0 limits its small LDS stack
 * to min(entries, 2048) and has the one-pass list construction try it first,
 * so that a stack overflow and the retry with the large stack happen on small
 * workloads (lists and forces do not change, only the work done); 0 restores
 * the normal choice.  Kept by the context until changed. */
int gx_set_walk_stack_limit(gx_ctx* ctx, int entries);

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
 *           synchronises twice: the node count and level histogram size the
 *           node arrays and the per-level moment launches, the group count
 *           sizes the group list.
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
 * In tree mode the call synchronises once before the pairwise kernel: the
 * list totals tell whether every group's list fit its slot (else the exact
 * two-pass construction runs, with a second synchronisation).  GX_DIRECT
 * without stats does not synchronise.
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
 * Synchronises after the candidate walk (list totals), after each pass over
 * long lists and after each round (whether any group must be walked again
 * with a larger radius).
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
 * Synchronises after the candidate walk (list totals) and after counting the
 * long lists' chunks (their number sizes the chunked pass).
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
 * gx_add_accel -- a += b, then b = 0, per component, for n particles (all
 * six arrays device FP64 [n], a and b not overlapping).  The acceleration of a
 * particle is the sum of its gravity and hydro terms (Sec. 3.2); this folds a
 * set evaluated separately (e.g. gx_sph_forces, which adds into its outputs,
 * run into a zeroed set on another context's stream beside the gravity
 * kernel) into the total and leaves the set zeroed for the next evaluation.
 * Each element is added once, so the total equals adding into a directly.
 * Enqueued on the context's stream; errors: GX_EINVAL for a null pointer or
 * n < 0.
 */
int gx_add_accel(gx_ctx* ctx, int64_t n, double* ax, double* ay, double* az, double* bx,
                 double* by, double* bz);

/*
 * gx_kick_drift_cubes -- gx_kick_drift for independent systems (SN cubes)
 * that each take their own Courant step: particle i of cube c = cube_id[i]
 * uses dt_kick = f_kick dt_cube[c] and dt_drift = f_drift dt_cube[c]
 * (dt_cube device double [n_cubes], e.g. from gx_sph_timestep with cube_id;
 * a cube with dt 0 stays put).  All n particles are gas: u, dudt, upred and
 * vpred_xyz (layout of gx_kick_drift) cover all of them, or are NULL.
 */
int gx_kick_drift_cubes(gx_ctx* ctx, int64_t n, const int32_t* cube_id, const double* dt_cube,
                        double f_kick, double f_drift, double* x, double* y, double* z, double* vx,
                        double* vy, double* vz, const double* ax, const double* ay,
                        const double* az, double* u, const double* dudt, double u_floor,
                        double* vpred_xyz, double* upred);

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

/* ======================================================================== */
/* Supernova surrogate (Sec. 3.2 steps 1-4, Sec. 3.3)                       */
/* ======================================================================== */

/*
 * gx_sn_extract -- pick up the gas in the box of side 2 half_side around each
 * of k SN sites (Sec. 3.2 step 2: the (60 pc)^3 box around the exploding
 * star).  Membership: c - h <= x < c + h on every axis.
 * gas      device particle view (x, y, z read), original order
 * centers  device double [k][3]
 * offsets  device int32 [k+1] (output CSR offsets); idx device int32 [cap]
 *          (output: original indices, ascending within each cube)
 * total    host: number of memberships.  Synchronises; GX_EINVAL if > cap.
 */
int gx_sn_extract(gx_ctx* ctx, const gx_particles* gas, const double* centers, int k,
                  double half_side, int32_t* offsets, int32_t* idx, int64_t cap, int64_t* total);

/*
 * gx_sn_inject -- thermal energy injection of one SN (1e51 erg in the paper,
 * Sec. 1): the k_inj members of each cube nearest its centre (ties broken by
 * index) receive energy / (their total mass) of specific internal energy.
 * gas: x, y, z, m read; offsets/idx from gx_sn_extract (device); u device,
 * indexed like the gas arrays, updated in place.
 */
int gx_sn_inject(gx_ctx* ctx, const gx_particles* gas, const int32_t* offsets, const int32_t* idx,
                 const double* centers, int k, int k_inj, double energy, double* u);

/*
 * gx_sn_ambient -- ambient state of each extracted box, the value of voxels
 * that no particle kernel reaches (Sec. 3.3 mapping): amb[c] = (log10 of the
 * members' total mass over side^3, log10 of their mass-weighted temperature
 * u * u_to_T floored at 10 K, mass-weighted vx, vy, vz).  Boxes with no
 * member get (-30, 1, 0, 0, 0).
 * offsets/idx from gx_sn_extract (device); u device FP64 per gas particle;
 * amb device float [k][5] (output).
 */
int gx_sn_ambient(gx_ctx* ctx, const gx_particles* gas, const double* u, const int32_t* offsets,
                  const int32_t* idx, int k, double side, double u_to_T, float* amb);

/*
 * gx_sn_gather -- hand a region to the surrogate (Sec. 3.2 step 2): pack the
 * members of each box (CSR offsets/idx from gx_sn_extract) into compact
 * device arrays in the box's own frame: position (x - centers[c]) * scale +
 * dst[c], velocity, mass and u unchanged, kernel size H * scale (Ho may be
 * NULL; H NULL writes -1, i.e. unknown).  n_max bounds the members of one
 * box.  Outputs are indexed like idx (length offsets[k]).
 */
int gx_sn_gather(gx_ctx* ctx, const gx_particles* gas, const double* u, const float* H,
                 const int32_t* offsets, const int32_t* idx, int k, int64_t n_max,
                 const double* centers, const double* dst, double scale, double* x, double* y,
                 double* z, double* vx, double* vy, double* vz, double* m, double* uo, float* Ho);

/*
 * gx_sn_unframe -- back to the simulation frame, in place, for replacement
 * particles in CSR order: x = (x - src[c]) / scale + centers[c] + v_c dt, with
 * v_c the box's bulk velocity (amb columns 2..4 of gx_sn_ambient; amb NULL:
 * no drift) and dt the hand-over delay in simulation time units.
 */
int gx_sn_unframe(gx_ctx* ctx, const int32_t* offsets, int k, int64_t n_max, const double* src,
                  const double* centers, const float* amb, double dt, double scale, double* x,
                  double* y, double* z);

/*
 * gx_sn_voxelize -- particle-to-grid mapping by SPH kernel convolution with
 * Shepard normalisation (Sec. 3.3) on grid^3 voxels covering a cube of the
 * given side centred on each site:
 *   rho_v = sum_j m_j W(|x_v - x_j|, H_j),
 *   T_v = sum_j T_j W_j / sum_j W_j,  v_v = sum_j v_j W_j / sum_j W_j,
 * W the Wendland C4 kernel of gx_sph_density, T = u * u_to_T.  Channels:
 * log10 rho (floored at 1e-6 of the ambient density), log10 T (floored at
 * 10 K), vx, vy, vz; voxels no kernel reaches take the ambient values.
 * Uses the GX_TREE_GAS slot built from `gas` (every particle whose kernel
 * reaches a voxel contributes, not only extracted members).
 * u, H      device gas arrays (FP64 u, FP32 kernel size), original order
 * amb       device float [k][5]: ambient (log10 rho, log10 T, vx, vy, vz)
 * out_bf16  optional device bf16 [k][grid^3][cpad]: (channel - mean) / std,
 *           channels 5..cpad-1 zero (chan_mean/chan_std device float [5])
 * out_f32   optional device float [k][grid^3][5]: the physical channels
 * Voxel order is z-major, x fastest; grid must be a multiple of 4.
 */
int gx_sn_voxelize(gx_ctx* ctx, const gx_particles* gas, const double* u, const float* H,
                   const double* centers, int k, double side, int grid, double u_to_T,
                   const float* amb, const float* chan_mean, const float* chan_std,
                   uint16_t* out_bf16, int cpad, float* out_f32);

/*
 * gx_sn_resample -- grid-to-particle mapping (Sec. 3.3; the paper samples by
 * Gibbs sampling, here by exact inverse-CDF draws from the same piecewise-
 * constant density).  For cube c, out_off[c+1] - out_off[c] particles (as many
 * as entered, so mass is conserved): voxel chosen with probability
 * proportional to 10^(log10 rho_v) using uniforms[4j], position uniform in the
 * voxel from uniforms[4j+1..3]; T and velocity of the voxel; u = T * T_to_u.
 * pred      device float [k][grid^3][5] physical channels
 * uniforms  device float [4 * total] in [0, 1)
 * outputs   device double [total]; n_out_max = largest per-cube count
 */
int gx_sn_resample(gx_ctx* ctx, const float* pred, int k, int grid, double side,
                   const double* centers, const int32_t* out_off, int64_t n_out_max,
                   const float* uniforms, double T_to_u, double* x, double* y, double* z,
                   double* vx, double* vy, double* vz, double* u);

/*
 * gx_sn_resample_gibbs -- grid-to-particle mapping by Gibbs sampling, the
 * Markov-chain method Sec. 3.3 names.  Particle j of cube c (CSR out_off,
 * as in gx_sn_resample) runs a chain over voxel indices (X, Y, Z) that starts
 * at the voxel holding (x0, y0, z0)[j] (floor((p - (centre - side/2)) /
 * (side/grid)) per axis, clamped to the grid); each of `sweeps` sweeps draws
 * X from the weights 10^(log10 rho) along the line through the current
 * (Y, Z), then Y given (X, Z), then Z given (X, Y): the first index whose
 * inclusive prefix sum (FP64, in index order) exceeds u * (the line total),
 * the last index if none does.  The position is then uniform in the final
 * voxel; T and velocity are that voxel's; u = T * T_to_u.  sweeps = 0 keeps
 * the start voxel.
 * pred        device float [k][grid^3][5] physical channels
 * x0, y0, z0  device double [total] start positions, frame of `centers`
 * uniforms    device float [total][3 * sweeps + 3] in [0, 1): entries 3s,
 *             3s+1, 3s+2 drive the x, y, z draws of sweep s, the last three
 *             the position inside the voxel
 * outputs     device double [total]; n_out_max = largest per-cube count.
 * Scratch: 3 k grid^3 doubles (the line sums) in the context.
 */
int gx_sn_resample_gibbs(gx_ctx* ctx, const float* pred, int k, int grid, double side,
                         const double* centers, const int32_t* out_off, int64_t n_out_max,
                         const double* x0, const double* y0, const double* z0, int sweeps,
                         const float* uniforms, double T_to_u, double* x, double* y, double* z,
                         double* vx, double* vy, double* vz, double* u);

/*
 * gx_sn_encode8 -- the eight input cubes of Sec. 3.3: from physical rows
 * (log10 rho, log10 T, vx, vy, vz) of in_stride floats, out8 [V][8] =
 * (log10 rho, log10 T, log10(v0 + max(vx, 0)), log10(v0 + max(-vx, 0)), the
 * same for vy and vz).  The paper takes the logarithm of each sign's
 * magnitude; the offset v0 > 0 (same unit as v) keeps it finite where a
 * cube is empty.  FP64 arithmetic, FP32 storage.  Device pointers.
 * gx_sn_decode8 -- the inverse on rows of in_stride >= 8 floats: out5 [V][5]
 * with v = 10^(c+) - 10^(c-) per component (v0 cancels).
 */
int gx_sn_encode8(gx_ctx* ctx, int64_t V, const float* in5, int in_stride, double v0,
                  float* out8);
int gx_sn_decode8(gx_ctx* ctx, int64_t V, const float* in8, int in_stride, float* out5);

/*
 * gx_sn_check -- trust check of a prediction before replacement (an addition
 * to Sec. 3.2 step 4: a region whose prediction leaves the training targets'
 * range keeps the plain integrator).  ok[c] = 1 when every value of cube c is
 * finite and lo[ch] <= value <= hi[ch] for its channel ch (compared in FP32).
 * pred   device float [k][grid^3][5] physical channels
 * lo, hi host double [5]
 * ok     host uint8 [k] (output).  Synchronises.  k = 0 is a no-op.
 */
int gx_sn_check(gx_ctx* ctx, const float* pred, int k, int grid, const double* lo,
                const double* hi, uint8_t* ok);

/*
 * gx_sn_check_noalloc -- gx_sn_check for callers that cannot allocate device
 * memory: code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc.  It allocates nothing, does not synchronise, and writes
 * the flags to device memory; the outcome per region is that of gx_sn_check.
 * pred    device float [k][grid^3][5] physical channels
 * lo, hi  host double [5] (read during the call)
 * ok_dev  device uint8 [k] (output: 1 = trusted)
 * Its scratch (one 32-bit flag per region) is a static device array of
 * GX_NOALLOC_MAX_REGIONS entries that each device keeps for the life of the
 * process; gx_create takes its address.  k > GX_NOALLOC_MAX_REGIONS returns
 * GX_EINVAL with a message.  Every call on one device shares that array, so
 * calls that overlap on one device (two streams, two host threads) race;
 * calls in stream order do not.  k = 0 is a no-op.
 */
#define GX_NOALLOC_MAX_REGIONS 16384
int gx_sn_check_noalloc(gx_ctx* ctx, const float* pred, int k, int grid, const double* lo,
                        const double* hi, uint8_t* ok_dev);

/*
 * gx_sn_replace -- replace particles by ID (Sec. 3.2 step 4).  id: device
 * int64 [n] ids of the main arrays (each in [0, id_cap)); new particles with
 * ids new_id[m] overwrite position and velocity; u (device, index i - u_offset
 * for main index i >= u_offset) and H64 (same indexing; set to -1 so the next
 * kernel-size solve reseeds) may be NULL.  n_missing (host, may be NULL)
 * counts new ids absent from the main set.  Synchronises when n_missing.
 * An ID listed more than once among the new particles takes the values of
 * its last entry (deterministic).
 */
int gx_sn_replace(gx_ctx* ctx, int64_t n, const int64_t* id, int64_t id_cap, double* x, double* y,
                  double* z, double* vx, double* vy, double* vz, double* u, int64_t u_offset,
                  double* H64, int64_t m, const int64_t* new_id, const double* nx, const double* ny,
                  const double* nz, const double* nvx, const double* nvy, const double* nvz,
                  const double* nu, int64_t* n_missing);

/* ---- 3-D convolutional network blocks (BF16 operands, FP32 accumulate) ---
 * Activations are NDHWC bf16 [B][S][S][S][C] (x fastest, channels innermost);
 * weights bf16 [Cout][kvol][Cin] with kvol = 27 (3^3 kernel, zero padding 1,
 * tap = (dz*3 + dy)*3 + dx) or 1; biases and master weights FP32.  Cin must
 * be a multiple of 8 and Cout of 16 (pad with zero channels).
 */

/* out = act(conv(in, w) + bias); act 1 = LeakyReLU(0.1), 0 = identity.  Writes
 * out_bf16 and/or out_f32 ([B][S^3][Cout]); bias may be NULL. */
int gx_conv3d_fwd(gx_ctx* ctx, const uint16_t* in, int B, int S, int Cin, const uint16_t* w,
                  const float* bias, int ksize, int Cout, int act, uint16_t* out_bf16,
                  float* out_f32);
/* 3^3 convolution (as gx_conv3d_fwd) of an input assembled on the fly:
 * channels [0, c1) from `in` ([B][..][c1]) and [c1, Cin) from `in2`
 * ([B][..][Cin - c1]; NULL: all Cin channels from `in`, c1 = Cin); with
 * upsample = 1 both sources hold (S/2)^3 voxels and are read with nearest x2
 * upsampling.  Equals gx_upsample2 / gx_concat followed by gx_conv3d_fwd
 * without materialising their outputs (the U-Net's up-path convolutions at
 * inference).  c1 a multiple of 8; S even when upsampling. */
int gx_conv3d_fwd_fused(gx_ctx* ctx, const uint16_t* in, int c1, const uint16_t* in2, int upsample,
                        int B, int S, int Cin, const uint16_t* w, const float* bias, int Cout,
                        int act, uint16_t* out_bf16, float* out_f32);
/* 1^3 convolution (the network head) whose first nc of its Cout outputs are
 * written as out[v * out_stride + c] = fmaf(value, scale[c], shift[c]) (scale,
 * shift device float [nc]); the other outputs are not stored.  Equals
 * gx_conv3d_fwd (ksize 1, FP32 output) followed by gx_chan_affine with
 * in_stride Cout, bit for bit. */
int gx_conv_head(gx_ctx* ctx, const uint16_t* in, int B, int S, int Cin, const uint16_t* w,
                 const float* bias, int Cout, int nc, const float* scale, const float* shift,
                 float* out, int out_stride);
/* 3^3 convolution (as gx_conv3d_fwd, bf16 output) that also writes the 2^3
 * average pooling of that output, pool_bf16 [B][(S/2)^3][Cout]: equals
 * gx_conv3d_fwd followed by gx_avgpool2, bit for bit (the U-Net's encoder
 * convolutions before each pooling).  S even. */
int gx_conv3d_fwd_pool(gx_ctx* ctx, const uint16_t* in, int B, int S, int Cin, const uint16_t* w,
                       const float* bias, int Cout, int act, uint16_t* out_bf16,
                       uint16_t* pool_bf16);
/* din = dL/din from dout = dL/dout ([B][S^3][Cout]) for the layer of weights w
 * ([Cout][kvol][Cin]); when y_in (the layer input, itself the LeakyReLU output
 * of the previous layer) is given, din is multiplied by that activation's
 * derivative.  Cin must be a multiple of 16. */
int gx_conv3d_bwd_data(gx_ctx* ctx, const uint16_t* dout, int B, int S, int Cin, const uint16_t* w,
                       int ksize, int Cout, const uint16_t* y_in, uint16_t* din);
/* dw [Cout][kvol][Cin] += sum over voxels of dout x im2col(in); dbias [Cout] +=
 * sum of dout (may be NULL).  Accumulates: zero them first. */
int gx_conv3d_bwd_weight(gx_ctx* ctx, const uint16_t* in, const uint16_t* dout, int B, int S,
                         int Cin, int ksize, int Cout, float* dw, float* dbias);
/* gx_conv3d_bwd_weight with the layer input described as gx_conv3d_fwd_fused
 * takes it: channels 0 .. c1 - 1 from in ([B][V][c1]) and c1 .. Cin - 1 from
 * in2 ([B][V][Cin - c1]; NULL: c1 = Cin), and with upsample = 1 both read at
 * the nearest voxel of the (S/2)^3 grid, so that training needs no
 * concatenated or upsampled copy of the U-Net's up-path inputs.  Equals
 * gx_conv3d_bwd_weight on the materialised input, bit for bit.  Needs S a
 * power of two >= 8, Cin and Cout <= 256, c1 a multiple of 8 (GX_EINVAL
 * otherwise). */
int gx_conv3d_bwd_weight_fused(gx_ctx* ctx, const uint16_t* in, int c1, const uint16_t* in2,
                               int upsample, const uint16_t* dout, int B, int S, int Cin,
                               int ksize, int Cout, float* dw, float* dbias);
/* 2^3 average pooling of in [B][S^3][C] -> out [B][(S/2)^3][C]; backward = 1:
 * in is dL/dout at S/2 and out is dL/din at S. */
int gx_avgpool2(gx_ctx* ctx, const uint16_t* in, int B, int S, int C, uint16_t* out, int backward);
/* nearest x2 upsampling in [B][S^3][C] -> out [B][(2S)^3][C]; backward = 1:
 * in is dL/dout at 2S, out is dL/din at S (sum of the 8 fine cells). */
int gx_upsample2(gx_ctx* ctx, const uint16_t* in, int B, int S, int C, uint16_t* out, int backward);
/* out[v] = (a[v], b[v]) along channels for V voxels; split = 1 reverses it. */
int gx_concat(gx_ctx* ctx, uint16_t* a, int Ca, uint16_t* b, int Cb, int64_t V, uint16_t* out,
              int split);
/* loss = mean over V voxels and nc channels of (pred - target)^2 (pred fp32
 * [V][Cp], target fp32 [V][nc]); dpred (bf16 [V][Cp], may be NULL) = dloss/dpred.
 * loss: host.  Synchronises. */
int gx_mse(gx_ctx* ctx, const float* pred, int Cp, const float* target, int nc, int64_t V,
           uint16_t* dpred, double* loss);
/* Adam (Kingma & Ba 2015) at step t >= 1 on n FP32 parameters with moments m,
 * v; refreshes the bf16 copy when w_bf16 is non-NULL. */
int gx_adam_step(gx_ctx* ctx, int64_t n, float* w, const float* grad, float* m, float* v,
                 double lr, double b1, double b2, double eps, int64_t t, uint16_t* w_bf16);
/* Per-channel sums over V rows of in (fp32, row stride `stride`, channels
 * [0, nc), nc <= 16): sums[c] += sum_v x, sums[nc + c] += sum_v x^2 (device
 * double [2 nc]); FP64, fixed summation order.  Gives the training-set mean
 * and standard deviation used to standardise the network's channels. */
int gx_chan_stats(gx_ctx* ctx, int64_t V, const float* in, int stride, int nc, double* sums);
/* y[v][c] = in[v][c] * scale[c] + shift[c], c < nc (scale/shift device float
 * [nc]): standardisation ((x - mean) / std) or its inverse on predictions.
 * out: fp32 rows of out_stride (NULL: skipped); out_bf16: bf16 rows of
 * bf_stride with channels nc.. zero (NULL: skipped); in place is allowed for
 * out when out_stride == in_stride. */
int gx_chan_affine(gx_ctx* ctx, int64_t V, const float* in, int in_stride, int nc,
                   const float* scale, const float* shift, float* out, int out_stride,
                   uint16_t* out_bf16, int bf_stride);
/* One of the 48 symmetries of the cube per sample (training augmentation):
 * out[b] = in[b] mapped by sym[b] = perm * 8 + flips (device int32 [B]; perm
 * in [0, 6) selects the axis permutation (x,y,z), (x,z,y), (y,x,z), (y,z,x),
 * (z,x,y), (z,y,x) taken by output axes x, y, z; flip bit a reverses output
 * axis a).  in/out fp32 [B][S^3][C], voxel order z-major, x fastest; the
 * vector channels vc..vc+2 (vc < 0: none) are permuted and negated with the
 * axes.  in and out must not overlap. */
int gx_cube_sym(gx_ctx* ctx, const float* in, int B, int S, int C, int vc, const int32_t* sym,
                float* out);
/* y = bf16(x), round to nearest even. */
int gx_f32_to_bf16(gx_ctx* ctx, const float* x, int64_t n, uint16_t* y);
/* out = (a + b) * LeakyReLU'(y) elementwise over n bf16 values (b, y may be
 * NULL: no addition / no derivative); gradient routing at skip connections. */
int gx_grad_combine(gx_ctx* ctx, int64_t n, const uint16_t* a, const uint16_t* b, const uint16_t* y,
                    uint16_t* out);

/* ---- the whole network (Sec. 3.3) ----------------------------------------
 * The U-Net as one call per pass, the layer sequence run inside the library
 * over the blocks above.  Per level l < levels (channels base * 2^l): two 3^3
 * convolutions (zero padding 1, bias, LeakyReLU 0.1); 2^3 average pooling
 * down; nearest x2 upsampling followed by a 3^3 convolution up; the skip
 * joined by channel concatenation (upsampled path first); a linear 1^3 head
 * with cout outputs.  Layer order e0a e0b ... e{L-1}a e{L-1}b, then for
 * l = L-2 .. 0: u{l}c d{l}a d{l}b, then head; the flat parameter array holds
 * every layer's weights [Cout][kvol][Cin] in that order, then every bias.
 */
typedef struct {
    int levels;              /* 2..6 */
    int base;                /* channels of level 0, a multiple of 16 */
    int cin;                 /* input channels (physical ones zero padded), multiple of 8 */
    int cout;                /* head outputs, multiple of 16 */
    const uint16_t* w_bf16;  /* device bf16 [n_params]: the weights are read from here */
    const float* w_f32;      /* device fp32 [n_params]: the biases are read from here */
} gx_unet;

/* Parameter and layer counts of a network description (no device work). */
int gx_unet_sizes(int levels, int base, int cin, int cout, int64_t* n_params, int64_t* n_layers);
/* Layer `index` of that description: name (e.g. "d0a"), channels, kernel size
 * and offsets of its weights and bias in the flat parameter array. */
int gx_unet_layer(int levels, int base, int cin, int cout, int index, char* name, int name_cap,
                  int* cin_out, int* cout_out, int* ksize, int64_t* w_off, int64_t* b_off);
/*
 * gx_unet_forward -- one forward pass of B samples of S^3 voxels.
 * in        device bf16 [B][S^3][cin] (standardised channels)
 * save      1: keep every activation in the context for gx_unet_backward (the
 *           upsampled and concatenated inputs are materialised); 0: inference,
 *           the up-path convolutions read them on the fly (same results)
 * out_f32   device fp32 [B][S^3][cout] head output, or NULL
 * out_phys  device fp32 [B][S^3][nc]: the first nc head outputs mapped by
 *           out = y * scale[c] + shift[c] (scale, shift device fp32 [nc]),
 *           or NULL.  At least one output.
 * S must be divisible by 2^(levels - 1).  Activations are library scratch.
 */
int gx_unet_forward(gx_ctx* ctx, const gx_unet* net, const uint16_t* in, int B, int S, int save,
                    float* out_f32, int nc, const float* scale, const float* shift,
                    float* out_phys);
/*
 * gx_unet_backward -- parameter gradients of the last saving forward pass
 * (same network, B and S; GX_ESTALE otherwise).
 * in    the forward input; dout device bf16 [B][S^3][cout] = dL/d(head output)
 * grad  device fp32 [n_params], ACCUMULATED (zero it first)
 */
int gx_unet_backward(gx_ctx* ctx, const gx_unet* net, const uint16_t* in, int B, int S,
                     const uint16_t* dout, float* grad);
/* Copy a tensor written by the last forward pass (gradient = 0: the
 * activation `name`, e.g. "e1b", "p0", "u0c", "d0a", and with save = 1 also
 * the up path's upsampled and concatenated inputs "up0", "c0", formed again
 * from the kept activations where the pass did not keep them) or by the
 * backward pass after it (gradient = 1: the gradient of that activation's
 * pre-activation, or "skip{l}") to device bf16 dst (cap elements), stream
 * ordered; *count gets its element count (dst may be NULL to ask only for
 * it).  Inspection for tests. */
int gx_unet_saved(gx_ctx* ctx, const char* name, int gradient, uint16_t* dst, int64_t cap,
                  int64_t* count);
/* Standardisation of the network's channels from FP64 sums (gx_chan_stats
 * over count rows): mean = s / count, std = max(sqrt(max(s2 / count -
 * mean^2, 0)), min_std), scale = 1 / std, shift = -mean / std (device fp32
 * [nc] each, any may be NULL). */
int gx_chan_moments(gx_ctx* ctx, const double* sums, int nc, double count, double min_std,
                    float* mean, float* std_out, float* scale, float* shift);

#ifdef __cplusplus
}
#endif
#endif /* GX_H */
