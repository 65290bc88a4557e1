/*
 * mcheis.h -- C ABI of the MI355X Metropolis library for the classical
 * anisotropic Heisenberg model.
 *
 * Model (Charilaou, arXiv:2106.11286, Eq. (1)):
 *     H = -J sum_<ij> S_i . S_j  -  K sum_i (S_i . e)^2
 * with unit three-component spins, nearest-neighbour bonds counted once, and a
 * uniaxial easy axis e.  Dynamics: single-spin Metropolis (the paper's Monte
 * Carlo paragraph): propose a new orientation uniformly on the sphere, accept
 * if dH <= 0 or if P <= exp(-dH/T) for a uniform P in (0,1).  Magnetisation:
 * Eq. (2), M = sum_i S_i / (N |S|), here with |S| = 1.
 *
 * Sites are updated by sublattice colour: every site of one colour in one
 * parallel pass (no bond joins two sites of one colour), colours 0..C-1 in
 * order; one sweep = C passes = one attempted move per occupied site.
 * C = 2 for simple cubic (sc) and body-centred cubic (bcc), 4 for
 * face-centred cubic (fcc).
 *
 * Random numbers: Philox4x32-10 with key (seed lo32, seed hi32) and counter
 * (s, replica_id, t, tag), where s is the canonical site index
 * s = ((z*Ly + y)*Lx + x)*n_basis + b, t the replica's sweep counter, tag 0 for
 * moves and 1 for the random initial state.  Word 0 gives z = 2u-1, word 1 the
 * azimuth 2 pi u, word 2 the acceptance number P, with u = (k + 1/2) 2^-23 from
 * the top 23 bits.  Results therefore depend only on (seed, replica_id, t, s),
 * never on tiling, batching or thread order.
 *
 * Conventions for every function:
 *  - the return value is an mc_status; nothing throws, aborts or exits;
 *  - on error a thread-local message is available from mc_last_error();
 *  - device pointers are HIP device memory on the current device, owned by
 *    the caller, and must outlive the handle; the library never frees them;
 *  - a handle is not thread-safe; calls on one handle must not overlap.
 */
#ifndef MCHEIS_H
#define MCHEIS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MC_OK = 0,
    MC_E_ARG = -1,         /* invalid argument value or NULL out-pointer          */
    MC_E_UNSUPPORTED = -2, /* valid model the library cannot colour / lay out     */
    MC_E_BUFFER = -3,      /* NULL, too small, misaligned or host buffer           */
    MC_E_DEVICE = -4,      /* no device, or a HIP error (message has the reason)   */
    MC_E_STATE = -5        /* call not valid in the handle's current state         */
} mc_status;

typedef enum { MC_SC = 0, MC_BCC = 1, MC_FCC = 2 } mc_lattice_kind;
typedef enum { MC_F32 = 0, MC_F64 = 1 } mc_precision;
typedef enum { MC_INIT_RANDOM = 0, MC_INIT_ALIGNED = 1, MC_INIT_USER = 2 } mc_init_mode;

/* mc_sweep / mc_schedule flags */
#define MC_MEASURE 1u    /* reduce observables on every sweep of this call            */
#define MC_TUNED_LAUNCH 4u /* launch as mc_autotune with this flag chose: per-pass   */
                           /* launches replayed as HIP graphs, or one persistent     */
                           /* launch (per-pass before any such tuning and after a    */
                           /* later mc_set_tile); not with MC_PERSISTENT.  Results   */
                           /* are bitwise the same in either mode.                   */
#define MC_PERSISTENT 2u /* run the sweeps as one persistent launch: work units       */
                         /* (sweep, colour, tile) are claimed in order by the resident */
                         /* workgroups, each replica advancing as soon as its previous */
                         /* pass is complete (no grid-wide barrier).  Results are      */
                         /* bitwise identical to the default launches.  Tiles without */
                         /* a persistent kernel (strips of 1 or 8 rows, pairs and     */
                         /* bands of pairs of 4 rows) give MC_E_UNSUPPORTED.  Queues: */
                         /* see mc_set_persistent_mode.                               */

/* One replica: lattice geometry and model parameters (Eq. (1)).
 *  kind          sc / bcc / fcc conventional cubic cells.
 *  Lx, Ly, Lz    cells per axis (>= 1).  sc needs Lx even (colour packing) and
 *                an even length on every periodic axis (2-colouring).
 *  periodic_mask bit0 x, bit1 y, bit2 z: periodic axes; open faces drop bonds.
 *  sphere_radius <= 0: every site of the box is occupied.  > 0: a site at
 *                position r (cells) is occupied iff |r - (Lx,Ly,Lz)/2| <= R.
 *                Unoccupied sites hold S = 0, are never updated and have no
 *                bonds.  A simple-cubic replica cut to a sphere runs on the
 *                tile (0) and LDS (3) kernels only (mc_set_tile gives
 *                MC_E_UNSUPPORTED for the others); bcc and fcc on every kernel.
 *  J, K          exchange and anisotropy (units of energy, k_B = 1).
 *  e             easy axis, normalised by the library (must be nonzero).
 *  T             temperature: 0 = greedy (accept iff dH <= 0), +inf = every
 *                move accepted; must not be negative or NaN.
 *  replica_id    counter word 1 of the random stream. */
typedef struct {
    int32_t kind;
    int32_t Lx, Ly, Lz;
    uint32_t periodic_mask;
    uint32_t replica_id;
    double sphere_radius;
    double J, K, e[3];
    double T;
} mc_replica_desc;

/* Spin storage of one replica: three device planes (x, y, z components), each
 * of capacity_sites elements of the precision's type (float or double).
 * Layout (colour-major, unoccupied sites hold 0):
 *  sc:      colour c = (x+y+z) & 1,
 *           idx = c*(N/2) + ((z*Ly + y)*Lx + x) / 2,  N = Lx*Ly*Lz;
 *  bcc/fcc: colour = basis site b,
 *           idx = b*(Lx*Ly*Lz) + (z*Ly + y)*Lx + x.
 * Alignment: each plane 16-byte aligned. */
typedef struct {
    void *sx, *sy, *sz;
    uint64_t capacity_sites;
} mc_spin_buffers;

/* Observables of one replica after one sweep (FP64 accumulation).
 *  sweep       sweeps completed by the replica when measured;
 *  n_sites     occupied sites N;  n_accepted  accepted moves in that sweep;
 *  M           magnetisation per spin, Eq. (2);  absM = |M|;
 *  E_exch      -J sum_bonds S_i.S_j;  E_anis  -K sum_i (S_i.e)^2;
 *  E           E_exch + E_anis (extensive, units of J). */
typedef struct {
    uint64_t sweep, n_sites, n_accepted;
    double M[3];
    double absM;
    double E, E_exch, E_anis;
} mc_obs;

/* Temperature schedule for mc_run_schedule.  For each of n_T steps: set the
 * temperatures T[step*n_reps + r], run n_equil unmeasured sweeps, then n_meas
 * sweeps, recording every measure_every-th of them (measure_every >= 1).  The
 * state is carried from one step to the next. */
typedef struct {
    int32_t n_T;
    const double *T; /* host array [n_T][n_reps] */
    uint32_t n_equil, n_meas, measure_every;
    uint32_t flags;  /* 0, MC_PERSISTENT or MC_TUNED_LAUNCH */
} mc_schedule;

/* Summary statistics of one replica's series (equilibrium averages over the
 * measured sweeps, per spin; errors by Flyvbjerg-Petersen blocking). */
typedef struct {
    uint64_t n;
    double abs_m, abs_m_err, m2, m2_err, m4, m4_err, e, e_err;
    double U4;  /* Binder cumulant 1 - <m^4>/(3 <m^2>^2) */
    double C;   /* specific heat per spin, (<E^2> - <E>^2)/(N T^2) */
    double chi; /* susceptibility per spin, N (<m^2> - <|m|>^2)/T */
    double acceptance;
    double U4_err; /* jackknife over 32 contiguous blocks (record i in block
                    * floor(32 i / n); n blocks of one record when n < 32) */
} mc_stats;

typedef struct mc_sim mc_sim; /* opaque handle */

/* Elements per spin plane that a replica needs (the box, all colours). */
mc_status mc_required_sites(const mc_replica_desc *d, uint64_t *sites_per_component);

/* Occupied sites N of a replica (sphere mask applied). */
mc_status mc_occupied_sites(const mc_replica_desc *d, uint64_t *n_sites);

/* Bytes of device scratch the handle needs for n_reps replicas (descriptors,
 * work list, per-workgroup FP64 partial sums, observable records, counters). */
mc_status mc_required_scratch(const mc_replica_desc *reps, int32_t n_reps, uint64_t *bytes);

/* Create a handle over n_reps replicas of one lattice kind and precision, and
 * write the initial state into the caller's buffers (unless MC_INIT_USER:
 * then the buffers already hold the state in the layout above).  The lattice
 * and its parameters are those of Eq. (1) and of the paper's simulation-setup
 * paragraph (cubic lattices, J, K, easy axis, T); the random start draws
 * each spin uniformly on the sphere, the aligned start sets S = e.
 *  bufs[n_reps]  spin planes per replica (device memory);
 *  scratch       device memory of at least mc_required_scratch bytes, 256-byte
 *                aligned, owned by the caller, used only by this handle;
 *  hip_stream    hipStream_t every call enqueues on (NULL = default stream).
 * Random start: spin s = sphere(Philox(seed, (s, replica_id, 0, 1))).
 * Errors: MC_E_ARG (n_reps < 1, lengths < 1, T < 0 or NaN, |e| = 0, mixed
 * lattice kinds, NULL out), MC_E_UNSUPPORTED (sc with odd Lx or with an odd
 * periodic length; box over 2^31 sites), MC_E_BUFFER (NULL / short /
 * misaligned / host memory), MC_E_DEVICE. */
mc_status mc_init_lattice(const mc_replica_desc *reps, int32_t n_reps, mc_precision prec,
                          uint64_t seed, mc_init_mode init, const mc_spin_buffers *bufs,
                          void *scratch, uint64_t scratch_bytes, void *hip_stream, mc_sim **out);

/* Enqueue n_sweeps sweeps of every replica (colour passes 0..C-1 each, sweep
 * counters t, t+1, ...).  Each site of a pass takes the Metropolis step of
 * the paper's Monte Carlo paragraph: field h = J sum of its neighbours' spins,
 * a proposal S' uniform on the sphere, dH = -h.(S'-S) - K[(S'.e)^2 - (S.e)^2]
 * from Eq. (1), acceptance if dH <= 0 or P <= exp(-dH/T), S <- S'/|S'|.  With MC_MEASURE every sweep also reduces the FP64
 * observables (fused into the passes; no extra spin traffic).  Asynchronous:
 * returns once the work is enqueued; device faults surface at the next
 * synchronising call. */
mc_status mc_sweep(mc_sim *h, uint32_t n_sweeps, uint32_t flags);

/* mc_sweep with HIP events recorded on the handle's stream around every
 * colour-pass launch; synchronises and returns the mean duration of one pass
 * launch (with the fused sweep kernel 9: of its one launch per sweep) and the
 * total time of the call (milliseconds).  For measuring the kernels in place;
 * results are identical to mc_sweep. */
mc_status mc_sweep_timed(mc_sim *h, uint32_t n_sweeps, uint32_t flags, double *pass_ms_avg,
                         double *total_ms);

/* Synchronise the stream and return the observables of the most recent
 * measured sweep of each replica (out[n_reps]): the magnetisation of Eq. (2)
 * and the two energy terms of Eq. (1).  MC_E_STATE if no sweep has
 * been measured since the handle was created. */
mc_status mc_observables(mc_sim *h, mc_obs *out, int32_t n_reps);

/* Observables of the current state recomputed from scratch: Eq. (2)'s
 * magnetisation sum and both terms of Eq. (1), every nearest-neighbour bond
 * counted once from a table of bond vectors, every product and sum in FP64.
 * A separate kernel that shares no code with the pass kernels, so it checks
 * their fused reduction independently.  n_accepted is 0; MC_E_DEVICE if the
 * kernel visits a number of occupied sites other than the lattice's.  Uses
 * the handle's scratch; synchronises. */
mc_status mc_measure_state(mc_sim *h, mc_obs *out, int32_t n_reps);

/* Bytes of device workspace a from-scratch measurement of caller buffers
 * needs (mc_measure_buffers): FP64 partial sums of up to 1024 workgroups. */
#define MC_MEASURE_WORKSPACE_BYTES 65536u

/* Observables of one replica's spins, held in caller buffers in the library
 * layout, computed from scratch as by mc_measure_state (Eq. (2)'s
 * magnetisation sum and both terms of Eq. (1); every bond once; FP64
 * products and sums) without a handle.  Enqueued on hip_stream (0: the null
 * stream) and asynchronous: record_dev (device memory, 8 doubles) receives
 * {M_x, M_y, M_z (sums), E_exch, E_anis, occupied sites, 0, 0} when the
 * stream reaches it.  workspace: caller-owned device memory of at least
 * MC_MEASURE_WORKSPACE_BYTES bytes, 256-byte aligned; it must not be used by
 * another call until this one has run.  Nothing is allocated; no argument is
 * kept after the call.  Errors: MC_E_ARG (descriptor, precision, NULL),
 * MC_E_UNSUPPORTED (descriptor), MC_E_BUFFER (too small, misaligned or not
 * device memory), MC_E_DEVICE (launch). */
mc_status mc_measure_buffers(const mc_replica_desc *d, mc_precision prec,
                             const mc_spin_buffers *bufs, void *workspace,
                             uint64_t workspace_bytes, double *record_dev, void *hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): mc_measure_buffers
 * with its workspace replaced by a static device array of the library
 * (64 KiB per GPU, held until the process ends); same arguments otherwise,
 * same results bit for bit.  Calls no allocating routine.  Every call on one
 * GPU shares that GPU's array: calls that overlap on one GPU (other streams,
 * other host threads) race and must be ordered by the caller.  No state
 * carries over between calls (each call writes every partial it reads).
 * MC_E_DEVICE if the array's device address cannot be found. */
mc_status mc_measure_buffers_static(const mc_replica_desc *d, mc_precision prec,
                                    const mc_spin_buffers *bufs, double *record_dev,
                                    void *hip_stream);

/* Run a temperature schedule: at each temperature thermalise, then average
 * (the paper's Monte Carlo and simulation-setup paragraphs: equilibration
 * sweeps followed by measurement sweeps per temperature).  Sweeps are replayed
 * as captured HIP graphs.
 * series receives the records in order [step][record][replica]; capacity is
 * its length in mc_obs elements and must be at least
 * n_T * (n_meas / measure_every) * n_reps.  n_written (may be NULL) receives
 * the count.  Synchronises. */
mc_status mc_run_schedule(mc_sim *h, const mc_schedule *s, mc_obs *series, uint64_t capacity,
                          uint64_t *n_written);

/* Change the temperatures (T[n_reps], same rules as the descriptor).  Ends a
 * replica exchange started with mc_exchange_init.  Synchronises. */
mc_status mc_set_temperatures(mc_sim *h, const double *T, int32_t n_reps);

/* One colour pass of every replica at the current sweep counter, without
 * advancing it, writing per-site diagnostics in the spin layout of the pass
 * colour: dH (working precision, element type of the spins) and the decision
 * (uint8 0/1).  Sites of other colours and unoccupied sites are not written.
 * Buffers are device memory of capacity_sites elements per replica, indexed
 * as the spin planes (pointer arrays of n_reps entries).  For checking
 * single-pass accuracy against a reference; not part of a sweep. */
mc_status mc_debug_pass(mc_sim *h, int32_t colour, void *const *dh, void *const *accepted);

/* Copy a replica's spins between the library layout and natural order
 * (canonical index s, see above) on the device.  to_natural != 0: packed ->
 * natural; 0: natural -> packed.  nx, ny, nz are device arrays of
 * mc_required_sites elements of the precision's type. */
mc_status mc_layout_copy(mc_sim *h, int32_t replica, int32_t to_natural, void *nx, void *ny,
                         void *nz);

/* Checkpoint / resume: the state is the spin buffers plus the sweep counter
 * (the counter-based stream makes a resumed run bitwise identical). */
mc_status mc_get_sweep(const mc_sim *h, uint64_t *t);
mc_status mc_set_sweep(mc_sim *h, uint64_t t);

/* Kernel and tile shape of the colour passes.  A tile is tx row columns x ty
 * rows x zc planes (a row column is a packed pair of sites for sc, a cell for
 * bcc/fcc).
 *  kernel 0 (any lattice): tx*ty <= 256 threads, one column and row each;
 *  kernel 1 (sc only): tx threads along the row (64, 128, 192 or 256), each
 *    holding ty consecutive rows (1, 2, 4 or 8), with the other colour kept in
 *    registers across planes;
 *  kernel 2 (sc only; the default for short or odd rows): as kernel 1, but
 *    rows grouped in bands of ty rows (2 or 4) and the (band, column)
 *    positions dealt to the tx threads contiguously, so no lane idles
 *    whatever the row length; a tile is tx positions x zc planes;
 *  kernel 3 (any lattice whose three component planes fit one workgroup's
 *    LDS; the default then): whole sweeps in LDS, one workgroup of tx threads
 *    (64 .. 1024, multiple of 64) per replica, colour passes separated by
 *    workgroup barriers; ty and zc are ignored.  Single passes (mc_debug_pass,
 *    mc_measure_state) keep using the previous pass kernel.  A replica too
 *    large gives MC_E_UNSUPPORTED;
 *  kernel 4 (sc only, every row of an even number of packed columns; the
 *    default when every row also has at least 96 packed columns): as
 *    kernel 1 with two adjacent columns per thread, read and written as one
 *    8-byte (FP32) or 16-byte (FP64) access; tx threads (64 .. 256) cover 2 tx
 *    columns, ty rows per thread (1, 2 or 4; persistent sweeps: 1 or 2);
 *  kernel 5 (sc only, even packed rows): as kernel 2 with two adjacent
 *    columns per thread: tx (64 .. 256) (band, pair) positions per workgroup,
 *    bands of ty rows (2 or 4; FP64 and persistent sweeps: 2);
 *  kernel 6 (bcc and fcc): tx lanes along x (64, 128, 192 or 256) times ty
 *    rows (tx*ty <= 256), zc planes walked in z with the other basis sites'
 *    planes kept in registers and the x neighbour taken from the adjacent
 *    lane (persistent sweeps run the kernel-0 body on the same tile);
 *  kernel 7 (bcc and fcc, every replica with Lx even; the default then, up
 *    to 4 GiB per spin component array): two adjacent cells of one basis per
 *    thread (one 8-byte FP32 / 16-byte FP64 access per component), bands of
 *    ty rows (1 or 2), tx (64 .. 256) (band, pair) positions per workgroup,
 *    zc planes walked in z with the other bases' rows kept in registers.  A
 *    larger array or an odd Lx gives MC_E_UNSUPPORTED;
 *  kernel 8 (sc only, rows a multiple of 16 bytes: Lx/2 a multiple of 4 in
 *    FP32, of 2 in FP64): tiles of ty whole rows (at most two (row, pair)
 *    positions per thread) walked over zc planes by tx = 256 threads; each
 *    plane's rows (other colour y0-1 .. y0+ty, own colour y0 .. y0+ty-1) are
 *    copied into LDS by asynchronous global-to-LDS loads one plane ahead of
 *    the arithmetic (double buffered, at most 60 KiB per workgroup), and the
 *    neighbour field is read from LDS.  No persistent sweeps;
 *  kernel 9 (sc only, even packed rows, every replica given a second buffer
 *    set by mc_set_second_buffers, component arrays below 4 GiB): the fused
 *    sweep -- both colours in one launch per sweep, reading the current
 *    state once and writing the next one into the other buffer set (24 bytes
 *    per update in FP32).  Tiles of ty whole rows (1 .. 64) walked over zc
 *    planes by tx = 256, 512 or 1024 threads, each lane holding up to three
 *    (row, pair) positions of rows y0-1 .. y0+ty (1024 threads: one; FP64:
 *    one, and tx <= 512); the new colour-0 spins of those rows are computed by
 *    the tile itself (also those outside it) and exchanged through
 *    6 (ty+2) Lx/2 spin values of LDS.  Shapes beyond these limits or the
 *    device's LDS give MC_E_UNSUPPORTED.  After each sweep the two buffer sets trade places
 *    (mc_get_state_buffers names the current one).  No persistent sweeps and
 *    no mc_debug_pass (MC_E_UNSUPPORTED).
 * The spins do not depend on the choice (only the FP64 summation order of the
 * observables does).  A shape whose work list does not fit the handle's
 * scratch gives MC_E_BUFFER.  Choosing any kernel but 3 discards the record of the
 * last measured sweep.  Synchronises; a deferred error of an earlier
 * persistent launch (watchdog, undrained queue) is returned first. */
mc_status mc_set_tile(mc_sim *h, int32_t kernel, int32_t tx, int32_t ty, int32_t zc);

/* Second buffer set of every replica (bufs[n_reps], same layout and
 * capacity as the state's, device memory, 16-byte aligned, not overlapping
 * the current state), used by the fused sweep kernel (9): a fused sweep reads
 * the current set and writes the other, after which the two trade places.
 * The caller owns the buffers and keeps them alive while the handle may run
 * kernel 9.  Sets the buffer set that does not hold the current state; the
 * state stays where it is.  MC_E_BUFFER for missing, small, misaligned or
 * overlapping buffers.  Synchronises. */
mc_status mc_set_second_buffers(mc_sim *h, const mc_spin_buffers *bufs);

/* The buffer set that holds a replica's current state: the one given to
 * mc_init_lattice, or (after an odd number of fused sweeps) the second set.
 * Host only; reflects every sweep enqueued so far. */
mc_status mc_get_state_buffers(const mc_sim *h, int32_t replica, mc_spin_buffers *out);
mc_status mc_get_tile(const mc_sim *h, int32_t *kernel, int32_t *tx, int32_t *ty, int32_t *zc,
                      uint64_t *n_items);

/* Autotuner (a property of this implementation, not of the method): time
 * candidate kernels and tile shapes on the handle's own lattices
 * (trial_sweeps sweeps each, with `flags` as for mc_sweep) and keep the
 * fastest (the fused sweep kernel 9 is a candidate once every replica has a
 * second buffer set).  The trial sweeps are ordinary sweeps of the chain: they advance
 * the state and the sweep counter (results stay bitwise independent of the
 * shape).  cache_path (may be NULL) names a text file of earlier choices
 * keyed by device (mc_tune_device_key of the handle's device), lattices,
 * precision and flags; a matching entry skips the trials, a new choice is
 * appended.  The chosen shape is returned through the out pointers (each may
 * be NULL).  Synchronises. */
mc_status mc_autotune(mc_sim *h, uint32_t trial_sweeps, uint32_t flags, const char *cache_path,
                      int32_t *kernel, int32_t *tx, int32_t *ty, int32_t *zc);

/* The launch mode the autotuner chose with MC_TUNED_LAUNCH (there it times
 * every candidate tile both as graph-replayed per-pass launches and, where the
 * tile has a persistent kernel, as one persistent launch, and keeps the
 * fastest pair): *persistent = 1 for the persistent launch, 0 otherwise
 * (also before any such tuning). */
mc_status mc_get_tuned_launch(const mc_sim *h, int32_t *persistent);

/* The device part of the autotuner's cache key: architecture name (the
 * device's gcnArchName), compute units and XCDs (both change with the
 * partition mode), as "<arch>-cu<n_cu>-xcd<n_xcd>" with separators of the
 * cache's text format replaced.  Writes a NUL-terminated string of at most
 * `capacity` bytes to out; MC_E_ARG for NULL pointers, negative counts or a
 * too small buffer.  Host only (no device access). */
mc_status mc_tune_device_key(const char *arch, int32_t n_cu, int32_t n_xcd, char *out,
                             uint64_t capacity);

/* Number of colours (passes per sweep) of the handle's lattice kind. */
mc_status mc_num_colours(const mc_sim *h, int32_t *n_colours);

/* Equilibrium statistics of one replica's records (stride: elements between
 * consecutive records of that replica, e.g. n_reps for mc_run_schedule
 * output), at temperature T (used by C and chi): thermal averages of the
 * Eq. (2) magnetisation and of the Eq. (1) energy per spin, with blocked
 * errors; the Binder cumulant locates T_C as in the accuracy paragraph.
 * MC_E_ARG for NULL pointers, n < 2 or stride < 1. */
mc_status mc_series_stats(const mc_obs *series, uint64_t n, uint64_t stride, double T,
                          mc_stats *out);

/* Bounded wait of persistent launches: a work unit waiting for its replica's
 * previous pass gives up after `spins` polls (about 0.1 us each; default
 * 2^24).  A launch that gave up sets the handle's watchdog flag, which later
 * launches keep: the next synchronising call returns MC_E_DEVICE (and clears
 * the flag) and the spins of that call are incomplete.  Every workgroup still
 * exits normally.  Waits for the handle's enqueued work first. */
mc_status mc_set_watchdog(mc_sim *h, uint32_t spins);

/* Replica exchange (parallel tempering) between the handle's replicas, an
 * extension of the paper's one-temperature runs for batches of identical
 * lattices (standard replica exchange: Swendsen and Wang; Hukushima and
 * Nemoto).  mc_exchange_init takes the replicas' current temperatures as the
 * ladder T_0 <= ... <= T_{n-1} (slot k; ties in replica order), each replica
 * at the slot of its own T; all replicas must differ only in T (0 < T < inf)
 * and replica_id (else MC_E_ARG); at least 2 replicas.
 * mc_exchange_sweep runs n_rounds rounds: sweeps_per_round sweeps (the last
 * one measured; with MC_PERSISTENT all of them, in one launch per round),
 * then one exchange step on the
 * device: round r attempts the slot pairs (k, k+1), k = r mod 2, r mod 2 + 2,
 * ..., with Delta = (1/T_k - 1/T_{k+1}) (E_i - E_j) for the replicas i at k and
 * j at k+1 and E the total Eq. (1) energy of the measured sweep; accepted iff
 * Delta >= 0 or u < exp(Delta), u the uniform of Philox counter
 * (k, 0, t, 2) under the handle's seed, t the sweeps done.  An accepted pair
 * swaps temperatures (the spins stay).  Asynchronous.
 * mc_exchange_state synchronises and returns replica_at_slot[n], T_slot[n],
 * attempted[n-1] and accepted[n-1] per pair (k, k+1) and the rounds done
 * (any pointer may be NULL); afterwards each replica's T in the handle is its
 * current slot's.  mc_set_temperatures (and mc_run_schedule) end the
 * exchange; mc_exchange_sweep then gives MC_E_STATE until the next init. */
mc_status mc_exchange_init(mc_sim *h);
mc_status mc_exchange_sweep(mc_sim *h, uint32_t n_rounds, uint32_t sweeps_per_round,
                            uint32_t flags);
mc_status mc_exchange_state(mc_sim *h, int32_t *replica_at_slot, double *T_slot,
                            uint64_t *attempted, uint64_t *accepted, uint64_t *rounds);

/* The paper's block scheme (implementation paragraph), for comparison with
 * the colour sweep; simple cubic lattices only (else MC_E_UNSUPPORTED).  The
 * canonical sites s = (z Ly + y) Lx + x are cut into blocks of n consecutive
 * sites (the last one shorter); in step j block k makes one Metropolis attempt
 * at site k n + floor(w3 m_k / 2^32), m_k its size, with w the Philox block of
 * counter (k, replica_id, j, 3) under the handle's seed (proposal from w0, w1,
 * acceptance uniform from w2, as in a colour pass).  Concurrent blocks read
 * each other's neighbours; this form makes that definite: every attempt of a
 * step sees the state before the step and the accepted moves are written
 * together (two launches per step and replica).  n steps are one sweep's
 * worth of attempts; the sweep counter does not move.  Every replica of the
 * handle takes the steps step0 .. step0 + n_steps - 1.
 * The caller supplies a device workspace of mc_block_workspace bytes
 * (256-byte aligned; else MC_E_BUFFER) whose first three 64-bit words count
 * attempts (occupied chosen sites), accepted moves and conflicts (attempts
 * with an attempted nearest neighbour in the same step, counted with
 * MC_BLOCK_CONFLICTS only); MC_BLOCK_RESET zeroes them first.
 * mc_block_counts synchronises, returns the three counts and zeroes them. */
#define MC_BLOCK_CONFLICTS 4u
#define MC_BLOCK_RESET 8u
mc_status mc_block_workspace(const mc_sim *h, uint32_t n, uint64_t *bytes);
mc_status mc_block_steps(mc_sim *h, uint32_t n, uint32_t step0, uint32_t n_steps, uint32_t flags,
                         void *work, uint64_t work_bytes);
mc_status mc_block_counts(mc_sim *h, void *work, uint64_t counts[3]);

/* Work queues of persistent launches (MC_PERSISTENT).  The replicas of a
 * handle are independent Markov chains, so a launch may serve each replica
 * from one XCD:
 *  MC_PERSIST_GLOBAL  one queue of all work units; a unit's spin stores are
 *                     written back from its XCD's L2 before the replica's
 *                     next pass may read them.
 *  MC_PERSIST_XCD     eight queues: the replicas are dealt to the eight XCDs
 *                     (largest first, each to the least loaded XCD, load =
 *                     work units of a sweep) and only workgroups running on
 *                     XCD g take units of queue g, so a replica's spins stay
 *                     in one L2 for the whole launch and no write-back is
 *                     needed.  Needs a device that deals workgroups to eight
 *                     XCDs in turn (checked once per device when a handle is
 *                     created); otherwise MC_E_UNSUPPORTED.
 *  MC_PERSIST_AUTO    (default) XCD queues when the device allows them, the
 *                     batch has at least 8 replicas and the most loaded queue
 *                     holds at most 1.25 times the mean load; else one queue.
 * Both give spins, records and observables bitwise identical to the default
 * launches.  The choice applies to later persistent calls, also after
 * mc_set_tile and mc_autotune (which re-deal the replicas); it drops captured
 * graphs.  mc_get_persistent_queues returns the queues in effect (1 or 8). */
typedef enum { MC_PERSIST_AUTO = 0, MC_PERSIST_GLOBAL = 1, MC_PERSIST_XCD = 2 } mc_persist_mode;
mc_status mc_set_persistent_mode(mc_sim *h, mc_persist_mode mode);
mc_status mc_get_persistent_queues(const mc_sim *h, int32_t *n_queues);

/* Wait for all enqueued work of the handle and report deferred errors
 * (device faults, a tripped persistent-launch watchdog). */
mc_status mc_synchronize(mc_sim *h);

/* Release the handle (never the caller's buffers, scratch or stream). */
void mc_destroy(mc_sim *h);

/* Measurement aid (no handle): the HBM access pattern of one simple-cubic
 * colour pass without its arithmetic, as a ceiling for the pass kernels.
 * x, y, z: caller-owned device arrays of 2*half_elems elements of `prec`
 * each (one component plane per colour, like the spin planes); their
 * contents are overwritten.  Each launch reads both halves and writes the
 * first in place (24 B read, 12 B written per FP32 element of the first
 * half), two elements per lane per access, on `grid` workgroups of 256
 * threads.  One untimed launch, then `reps` timed launches on hip_stream
 * (NULL: the default stream); *ms = mean time per launch.  half_elems must
 * be even and >= 2, grid in [1, 2^20], reps >= 1; MC_E_BUFFER for a NULL or
 * too small array.  Synchronises. */
mc_status mc_stream_probe(mc_precision prec, void *x, void *y, void *z, uint64_t half_elems,
                          uint32_t grid, uint32_t reps, void *hip_stream, double *ms);

/* Message of the last error on this thread ("" if none). */
const char *mc_last_error(void);

/* Library version string. */
const char *mc_version(void);

#ifdef __cplusplus
}
#endif

#endif /* MCHEIS_H */
