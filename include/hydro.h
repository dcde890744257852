/*
 * hydro.h -- C ABI of the MI355X (gfx950) patch-group hydrodynamic solver.
 *
 * The library advances batches of patch groups -- 2x2x2 patches of 8^3
 * cells, i.e. 16^3 interior cells plus a ghost layer -- of the 3D Euler
 * equations by one step with the directionally unsplit schemes of
 * Schive, Zhang & Chiueh, arXiv:1103.3373:
 *   Sec. 2      : MUSCL-Hancock (MHM), the VL variant and the six-solve CTU
 *                 scheme; PLM / PPM reconstruction with the generalized
 *                 minmod, van Leer, van Albada or hybrid limiter, applied to
 *                 primitive or characteristic variables; Roe (with detection
 *                 of linearization failure and HLLE/HLLC fallback), HLLC and
 *                 HLLE Riemann solvers; steps (1)-(5): reconstruction (plus
 *                 characteristic tracing for CTU), Riemann solves, transverse
 *                 correction (CTU), conservative update, patch-boundary
 *                 fluxes.
 *   Sec. 3.1    : one patch group per work unit, data array[z][y][x] with x
 *                 fastest, fluxes across patch boundaries stored as soon as
 *                 they are computed.
 *   Sec. 4.1-4.2: inputs are the interior plus ghost cells of each group
 *                 (the "preparation step"), outputs the updated interiors.
 *   Sec. 4.3    : the evolution time step (CFL condition).
 *
 * Conventions for every entry point
 *  - Pointers are DEVICE pointers unless marked (host).  The caller allocates
 *    and owns every buffer; the library never frees caller memory.
 *  - Buffers hold float, or double when flags contain HYDRO_F64.
 *  - Conserved variables (rho, rho*u, rho*v, rho*w, E), ideal gas.
 *  - Calls are asynchronous on `stream` (a hipStream_t; NULL = null stream).
 *    Kernel faults surface at the caller's next synchronization.
 *  - Return 0 on success or a negative HYDRO_E* code; hydro_last_error()
 *    gives the message of the last failure on the calling thread.
 *  - Numerical trouble is never an error: Roe fallbacks and floor
 *    activations are counted on the device (hydro_get_diag).
 *  - Library-owned device memory: the diagnostics counters and a pool of
 *    reduction partials are allocated at the first call on a device; the
 *    plain path's temporaries, the VL half-step scratch and the per-group
 *    partials of hydro_cfl_dt_batch are allocated per (device, stream) the
 *    first time a call needs them at a given size (growing synchronizes the
 *    device).  A call that would allocate must not be the first of its kind
 *    inside a graph capture; hydro_cfl_dt and hydro_conserved_sums never
 *    allocate after the first call on the device (up to 64 streams).
 *    hydro_shutdown frees all of it.
 */
#ifndef HYDRO_H
#define HYDRO_H

#ifdef __cplusplus
extern "C" {
#endif

/* Schemes (Sec. 2). */
enum hydro_scheme { HYDRO_MHM = 0, HYDRO_VL = 1, HYDRO_CTU = 2 };
/* Reconstruction (Sec. 2). */
enum hydro_recon { HYDRO_PLM = 0, HYDRO_PPM = 1 };
/* Riemann solvers (Sec. 2).  The exact solver (Newton iteration on the
 * star pressure, then sampling on the face) runs on the plain path only:
 * hydro_solve_groups takes that path for it, and the fused-only calls
 * (hydro_solve_batch, hydro_step_box, hydro_autotune) return
 * HYDRO_EUNSUPPORTED.  With HYDRO_EXACT the first diagnostic counter counts
 * faces that generate vacuum or do not converge. */
enum hydro_riemann { HYDRO_ROE = 0, HYDRO_HLLC = 1, HYDRO_HLLE = 2, HYDRO_EXACT = 3 };
/* Slope limiters (Sec. 2).  The hybrid limiter is the van Leer slope bounded
 * by the generalized minmod slope; theta = 1.5 for both. */
enum hydro_limiter { HYDRO_LIM_GMINMOD = 0, HYDRO_LIM_VANLEER = 1, HYDRO_LIM_VANALBADA = 2, HYDRO_LIM_HYBRID = 3 };

/* flags */
#define HYDRO_F64 0x01          /* buffers hold double (default float) */
#define HYDRO_CHAR 0x02         /* limit characteristic variables (Sec. 2) */
#define HYDRO_FLUX_MID 0x04     /* flux_out also holds the internal patch mid planes */
#define HYDRO_PLAIN 0x08        /* plain per-group path (Sec. 3.1 design); default: fused path */
#define HYDRO_ROE_FB_HLLC 0x10  /* Roe fallback flux = HLLC (default HLLE) */
#define HYDRO_BOX_GROUPED 0x20  /* hydro_fill_ghosts_periodic: box is [G][5][16][16][16] */
#define HYDRO_BOX_SEGS 0x40     /* hydro_solve_batch: every segment is a periodic box (box == 1) */
#define HYDRO_ROE_FB_EXACT 0x80 /* Roe fallback flux = exact solver (plain path; Sec. 2) */

/* error codes */
#define HYDRO_OK 0
#define HYDRO_EINVAL (-1)       /* bad argument */
#define HYDRO_EUNSUPPORTED (-2) /* combination not built */
#define HYDRO_EHIP (-3)         /* HIP runtime error (message in hydro_last_error) */
#define HYDRO_EALIAS (-4)       /* input and output buffers overlap */

/*
 * Ghost width g needed by a scheme's stencil: MHM and CTU: PLM 2, PPM 3;
 * VL: PLM 3, PPM 4 (the first-order predictor adds one layer).  Group input
 * arrays are (16 + 2g)^3 per variable.  Returns -1 for a bad enum.
 */
int hydro_ghost_width(int scheme, int reconstruction);

/*
 * Advance n_groups patch groups by one step of size dt (Sec. 2, steps 1-5).
 *   in        [n_groups][5][N][N][N], N = 16 + 2*hydro_ghost_width(...): the
 *             interior and ghost cells of each group (Sec. 4.2), x fastest.
 *   out       [n_groups][5][16][16][16]: the updated interiors.  Must not
 *             overlap `in` or `flux_out` (HYDRO_EALIAS).
 *   flux_out  NULL, or [n_groups][3][nf][5][16][16]: the final physical flux
 *             F (not F*dt) on the group's faces (Sec. 2 step 5), dir x,y,z;
 *             face index 0 = lower face (interior offset 0), 1 = upper face
 *             (offset 16), and with HYDRO_FLUX_MID nf = 3 and index 2 = the
 *             internal patch boundary (offset 8); otherwise nf = 2.  The two
 *             transverse indices are (slow, fast) = (z,y) for x faces, (z,x)
 *             for y faces, (y,x) for z faces.
 *   dt, dh    time step and cell size (host doubles, > 0, finite); dt/dh is
 *             formed in double and rounded once for the float path.
 *   gamma     ratio of specific heats, > 1.
 * n_groups == 0 is a successful no-op.  Errors: HYDRO_EINVAL, HYDRO_EALIAS,
 * HYDRO_EUNSUPPORTED, HYDRO_EHIP.
 */
int hydro_solve_groups(const void* in, void* out, void* flux_out, int n_groups, double dt, double dh, double gamma,
                       int scheme, int reconstruction, int riemann, int limiter, int flags, void* stream);

/*
 * CFL time step (Sec. 4.3) in FP64 from interior cells U[n_groups][5][4096]:
 *   dt = cfl * dh / max over cells of max_d(|v_d| + c).
 * Written to dt_out (device, 1 double).  The maximum is order-free, so the
 * result equals a serial FP64 evaluation on the same (upcast) data.
 */
int hydro_cfl_dt(const void* U, int n_groups, double dh, double gamma, double cfl, int flags, double* dt_out,
                 void* stream);

/*
 * FP64 conserved sums over interior cells U[n_groups][5][4096]:
 *   sums_out[v] = dh^3 * sum U_v  (device, 5 doubles), fixed reduction order.
 */
int hydro_conserved_sums(const void* U, int n_groups, double dh, int flags, double* sums_out, void* stream);

/*
 * Both of the above (Sec. 4.3 time step and the FP64 conserved sums) in one
 * pass over U[n_groups][5][4096]: dt_out (device, 1 double) and sums_out
 * (device, 5 doubles) are bit-identical to hydro_cfl_dt and
 * hydro_conserved_sums on the same data, and the state is read once.
 * dt_out and sums_out must not overlap (HYDRO_EALIAS).
 */
int hydro_cfl_dt_sums(const void* U, int n_groups, double dh, double gamma, double cfl, int flags, double* dt_out,
                      double* sums_out, void* stream);

/*
 * Preparation step (Sec. 4.2), periodic box: build the ghosted groups
 * [G][5][N][N][N] (N = 16 + 2g, G = (gz*ngy + gy)*ngx + gx) from a box
 * [5][nz][ny][nx] (or [G][5][16][16][16] with HYDRO_BOX_GROUPED).  nx, ny,
 * nz must be positive multiples of 16 with fewer than 2^31 groups;
 * 0 <= g <= 16 (else HYDRO_EINVAL).
 */
int hydro_fill_ghosts_periodic(const void* box, int nx, int ny, int nz, int g, int flags, void* groups_out,
                               void* stream);

/*
 * Preparation step (Sec. 4.2) for AMR-shaped groups: every cell of each
 * padded group is the trilinear interpolation, at the cell centre, of a
 * periodic coarse field coarse[5][cn][cn][cn] on the unit box (spatial
 * interpolation at coarse-fine boundaries).  layout (device int32
 * [n_groups][4]) = (level, ox, oy, oz): the group's first interior cell on
 * the level grid of spacing base_dh / 2^level.
 */
int hydro_fill_groups_interp(const void* coarse, int cn, const int* layout, int n_groups, int g, double base_dh,
                             int flags, void* groups_out, void* stream);

/*
 * AMR levels for the preparation step of groups next to coarse-fine
 * boundaries (Sec. 4.2).  Level l (0 <= l < n_levels <= HYDRO_MAX_LEVELS)
 * spans the periodic unit box with ng_l = ng0 << l groups, i.e. 16 ng_l
 * cells, per side.  A group's layout entry (level, ox, oy, oz) gives its
 * first interior cell on its level grid; the origins are multiples of 16
 * in [0, 16 ng_l).
 *
 * The group map (device int32, hydro_group_map_len(ng0, n_levels) entries)
 * holds, level after level, the index of the group at each group position
 * or -1: map[off_l + (gz ng_l + gy) ng_l + gx] with off_l = sum over m < l of
 * ng_m^3.  hydro_group_map_len returns that length, or -1 for ng0 <= 0, a
 * level count outside [1, HYDRO_MAX_LEVELS] or 2^31 entries or more.
 */
#define HYDRO_MAX_LEVELS 8
long long hydro_group_map_len(int ng0, int n_levels);

/*
 * Builds the group map from layout (device int32 [n_groups][4]) into map_out
 * (device, caller-owned, hydro_group_map_len entries).  Entries whose level is
 * out of range or whose origin is off the level's 16-cell grid are left out;
 * where two groups share a position the higher index is kept.
 * Errors: HYDRO_EINVAL (bad ng0 / n_levels / n_groups, null pointer).
 */
int hydro_build_group_map(const int* layout, int n_groups, int ng0, int n_levels, int* map_out, void* stream);

/*
 * Preparation step (Sec. 4.2) with spatial and temporal interpolation:
 * builds each group's padded input [n_groups][5][N][N][N] (N = 16 + 2g,
 * 0 <= g <= 4) from
 *  - its own interior, fine[group][5][16][16][16] (the level's state at the
 *    fine time);
 *  - for a ghost cell that a group of the same level covers (by the map,
 *    periodic on the level grid): that group's value;
 *  - for every other ghost cell: the coarse state at the fine time,
 *    (1 - alpha[l]) coarse0 + alpha[l] coarse1 (both [5][cn][cn][cn],
 *    periodic on the unit box, at the start and the end of the coarse
 *    step), interpolated trilinearly to the cell centre.
 * alpha is a HOST array of n_levels weights in [0, 1].  Copies are exact;
 * interpolated values are formed in FP64 and rounded to the buffer type.
 * The map must be the one built for this layout (hydro_build_group_map);
 * entries naming no group of the call count as empty.  flags: HYDRO_F64 or 0.
 * Errors: HYDRO_EINVAL (sizes, g, alpha, flags, null pointers),
 * HYDRO_EALIAS (groups_out overlaps fine or a coarse state), HYDRO_EHIP.
 */
int hydro_fill_groups_amr(const void* fine, const int* layout, int n_groups, const int* map, int ng0, int n_levels,
                          const void* coarse0, const void* coarse1, int cn, const double* alpha, int g, int flags,
                          void* groups_out, void* stream);

/*
 * Coarse-grid correction after one coarse step (Sec. 2 step 5: the fluxes
 * stored on patch boundaries; Sec. 4.3: correcting the coarse-grid data),
 * in place on coarse (the state after the coarse step, a periodic n^3 box
 * in patch-group order [G][5][16][16][16], n a multiple of 16):
 *  - refluxing: a coarse cell that no fine group covers, next across a face
 *    to one that a fine group covers, had its update formed with the coarse
 *    flux Fc of that face; it is corrected to the mean Ff of the four fine
 *    fluxes on that face: U -= dt/dh (Ff - Fc) when the fine side is its +
 *    side, U += dt/dh (Ff - Fc) when it is its - side;
 *  - restriction: each covered coarse cell becomes the mean of its 8
 *    children.
 * The fine level has ratio 2; fine group f (fine_layout[f] = (unused, ox,
 * oy, oz), origins on the fine grid's 16-cell grid, so each fine group
 * covers one 8^3 coarse patch) has interiors fine[f][5][16][16][16] and face
 * fluxes fine_flux[f][3][2][5][16][16] averaged over its sub-steps (weights
 * dt_sub / dt, see hydro_accumulate).  fine_map is the fine level's group
 * map from hydro_build_group_map(fine_layout, n_fine, n / 8, 1, ...), which
 * takes only entries whose level field is 0 (fine groups with another level
 * entry are left out of the map and so neither reflux nor restrict).
 * coarse_flux [G][3][3][5][16][16] holds the coarse step's fluxes on every
 * patch face (faces -, + and the mid plane, i.e. a solve with
 * HYDRO_FLUX_MID).  dt, dh: the coarse step and cell size.  The correction
 * conserves the domain totals of a coarse step and its fine sub-steps.
 * flags: HYDRO_F64 or 0.  Errors: HYDRO_EINVAL, HYDRO_EALIAS (coarse
 * overlaps an input), HYDRO_EHIP.
 */
int hydro_amr_correct(void* coarse, int n, const void* coarse_flux, const void* fine, const int* fine_layout,
                      int n_fine, const int* fine_map, const void* fine_flux, double dt, double dh, int flags,
                      void* stream);

/*
 * acc[i] += w * x[i] for n elements (float, or double with HYDRO_F64),
 * evaluated in FP64: the sub-step average of fine face fluxes for
 * hydro_amr_correct.  acc == x is allowed; a partial overlap is
 * HYDRO_EALIAS.
 */
int hydro_accumulate(void* acc, const void* x, double w, long long n, int flags, void* stream);

/* One segment of a batched launch: `count` groups advanced by
 * dt = (*dt) * dt_scale with cell size dh.  `dt` points to a device double,
 * so the time step can be produced on the device (e.g. by hydro_cfl_dt) and
 * the launch captured in a graph.
 *   box == 0: in is [count][5][N][N][N] (ghosted groups, N = 16 + 2g).
 *   box == 1: in is a periodic box stored as groups [count][5][16][16][16],
 *             count = ngx*ngy*ngz, group index (gz*ngy + gy)*ngx + gx; the
 *             ghost cells are read from the neighbouring groups (the
 *             preparation step fused into the solver).  Fused path only.
 *             A z-slab of groups (ngx*ngy groups) must hold less than 4 GiB
 *             (FP32: at most 52,428 groups, FP64: 26,214); a segment beyond
 *             that gets NaN outputs.
 * out is [count][5][16][16][16], flux as for hydro_solve_groups or NULL. */
struct hydro_seg {
  const void* in;
  void* out;
  void* flux;          /* may be NULL */
  const double* dt;    /* device */
  double dt_scale;
  double dh;
  long long first;     /* global index of the segment's first group */
  long long count;     /* groups in the segment */
  int ngx, ngy, ngz;   /* box == 1: groups per dimension */
  int box;
};

/*
 * One step of a periodic box held in patch-group order (HYDRO_BOX_GROUPED
 * layout): box_in, box_out [G][5][16][16][16], G = (nx/16)(ny/16)(nz/16),
 * with dt read from the device double *dt_dev (times dt_scale).  The ghost
 * cells are read from the neighbouring groups of box_in, so no ghosted copy
 * is made (the preparation step of Sec. 4.2 fused into the solver).  nx,
 * ny, nz positive multiples of 16 with a z-slab of (nx/16)(ny/16) groups
 * below 4 GiB (else HYDRO_EINVAL); box_out must not overlap box_in.
 * flux_out as for hydro_solve_groups, or NULL.  Fused path only
 * (HYDRO_EUNSUPPORTED otherwise).
 */
int hydro_step_box(const void* box_in, void* box_out, void* flux_out, int nx, int ny, int nz, const double* dt_dev,
                   double dt_scale, double dh, double gamma, int scheme, int reconstruction, int riemann, int limiter,
                   int flags, void* stream);

/*
 * Batched CFL time step (Sec. 4.3): for every segment of the table, the FP64
 * dt of its `out` state ([count][5][4096] interiors) is written to the
 * segment's `dt` pointer: dt = cfl * dh / max over the segment's cells of
 * max_d(|v_d| + c) (dt_scale is not applied).  Bit-identical to
 * hydro_cfl_dt on each segment alone.  Segments sorted by `first`, covering
 * [0, n_groups_total).  Two launches for the whole table.
 */
int hydro_cfl_dt_batch(const struct hydro_seg* segs, int n_segs, long long n_groups_total, double gamma, double cfl,
                       int flags, void* stream);

/*
 * hydro_cfl_dt_batch for callers that cannot allocate device memory: code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  Same arguments, layouts, results (bit for bit) and errors as
 * hydro_cfl_dt_batch, but it calls no hipMalloc / hipFree: the per-group
 * maxima go to a library-owned static device array of
 * HYDRO_NOALLOC_MAX_GROUPS doubles (8 MiB, one copy on every device the
 * library runs on, held until the process ends).  Every slot a call reads
 * is written by the same call first, so nothing needs clearing.
 * n_groups_total > HYDRO_NOALLOC_MAX_GROUPS -> HYDRO_EINVAL (checked before
 * any device call).  All calls on one device share that array: calls
 * ordered on one stream are safe, calls that overlap in time on one device
 * (unordered streams) race and give wrong time steps.
 */
#define HYDRO_NOALLOC_MAX_GROUPS (1 << 20)
int hydro_cfl_dt_batch_noalloc(const struct hydro_seg* segs, int n_segs, long long n_groups_total, double gamma,
                               double cfl, int flags, void* stream);

/* Specialization of a batched launch (all segments share it). */
struct hydro_spec {
  int scheme, reconstruction, riemann, limiter, flags;
  double gamma;
};

/*
 * Batched solve (uneven levels / simulations in one launch): one persistent
 * launch of the fused kernel over segs[0..n_segs) (device table, segments in
 * increasing `first`, covering [0, n_groups_total)).  The launch shape comes
 * from the autotune cache (hydro_autotune) or a default.  Same layouts and
 * errors as hydro_solve_groups; HYDRO_PLAIN is not accepted here.
 */
int hydro_solve_batch(const struct hydro_seg* segs, int n_segs, long long n_groups_total,
                      const struct hydro_spec* spec, void* stream);
/* With HYDRO_BOX_SEGS in spec->flags the caller asserts that every segment
 * is a periodic box; VL then computes its half step once per cell instead of
 * once per ghosted group.  A launch whose table contradicts the flag writes
 * NaN to the outputs of the offending segments. */

/*
 * Autotuner: times the fused kernel's launch shapes for `spec` on a
 * synthetic batch of n_groups_hint groups (allocates and frees its own
 * buffers; synchronizes `stream`) and records the fastest in the in-process
 * cache used by hydro_solve_groups / hydro_solve_batch.  If the environment
 * variable HYDRO_TUNE_CACHE names a file, the cache is appended there and
 * read back at the first call.  Returns the chosen workgroup count (> 0).
 */
int hydro_autotune(const struct hydro_spec* spec, int n_groups_hint, void* stream);

/*
 * Pins the launch shape of the fused kernel for `spec`'s specialization in
 * the in-process cache (as if the autotuner had chosen it), for callers that
 * tune offline or need a fixed shape.  grid = persistent workgroup count (0
 * = default: one or twelve workgroups per compute unit, by variant; a grid
 * larger than a launch's work-item count is clamped to it).  variant =
 * register budget variant: 2 (one workgroup per CU, no register spills) or 4
 * (two workgroups per CU; FP32 only).  zrun = tile depth of a box step
 * without flux output (hydro_step_box; for VL, of its second stage): each
 * workgroup marches through zrun z-consecutive patch groups of one column in
 * one pass (a 16 x 16 x 16*zrun tile), so the work items are the box's
 * groups / zrun; 0 = default (the largest of 4, 2 that divides the box's
 * group count in z and leaves two items per resident workgroup slot).
 * Depths 2 and 4 are built for the FP32 van Leer / characteristic
 * specialization with variant 4 only (CTU with PLM or PPM, MHM and VL with
 * PPM); the depth used is the largest built one, not above the request, that
 * divides the box's group count in z.  At one tile depth, results do not
 * depend on the grid or variant (bit for bit).  Tile depths differ in the
 * last bits on the first planes of a group that continues a run, whose z
 * slopes and edges come from the kernel's loop body rather than its z
 * prologue (two copies of the same arithmetic the compiler may contract
 * differently). HYDRO_EINVAL for other values (zrun outside 0..64).
 */
int hydro_set_launch_shape(const struct hydro_spec* spec, int grid, int variant, int zrun);

/*
 * The launch shape hydro_step_box would use for `spec` on an nx x ny x nz
 * box without flux output (host outputs: workgroups, register variant, and
 * groups per z-run).  No device work.
 * HYDRO_EINVAL for bad sizes or options.
 */
int hydro_get_launch_shape(const struct hydro_spec* spec, int nx, int ny, int nz, int* grid, int* variant,
                           int* zrun);

/* Device diagnostics accumulated since the last reset. */
struct hydro_diag {
  unsigned long long roe_fallbacks; /* interfaces where Roe's linearization failed */
  unsigned long long floor_hits;    /* density/pressure floor activations */
};
/* Synchronizes `stream`, copies the counters to *out (host); reset != 0
 * clears them afterwards. */
int hydro_get_diag(struct hydro_diag* out, int reset, void* stream);

/* Message of the last error on the calling thread ("" if none). */
const char* hydro_last_error(void);

/* Frees the library's internal workspaces (plain-path temporaries,
 * reduction partials, tuning state).  Synchronizes the device. */
void hydro_shutdown(void);

#ifdef __cplusplus
}
#endif

#endif /* HYDRO_H */
