/*
 * pch.h - exact geodesic distance on triangle meshes with the Parallel
 * Chen-Han (PCH) method on AMD Instinct MI355X (gfx950).
 *
 * Problem (Algorithm 1, "Require"/"Ensure"): given a triangle mesh
 * M = (V, E, F) and source vertices S, compute for every vertex the length of
 * the shortest path to S on the polyhedral surface. Only edge lengths are
 * needed (Section 4.1), so a mesh can be given by coordinates or by
 * per-half-edge lengths.
 *
 * Each round of the method (Section 4.2) runs as device kernels: window
 * selection, window propagation (Algorithm 2), data organization
 * (Algorithm 3) and event processing (Algorithm 4). All state stays in device
 * memory; the host only enqueues rounds.
 *
 * Conventions
 *  - Every call returns pch_status: PCH_OK (0) or a negative error code. The
 *    message of the last error on the calling thread is pch_last_error().
 *  - Faces are int32 [nf][3], counter-clockwise; half-edge j = 3 f + i runs
 *    from faces[f][i] to faces[f][(i + 1) % 3] (Section 4.1).
 *  - Host arrays passed in are read during the call and not kept (the
 *    library copies what it needs). Output arrays marked "device" must be
 *    device memory (e.g. a torch tensor's data_ptr()) of at least the stated
 *    size; the caller owns them.
 *  - hip_stream is a hipStream_t (NULL = the default stream). Work is
 *    ordered on that stream; calls return after the result is complete.
 *  - Unreachable vertices get +infinity; sources get 0.
 *  - The library keeps no global mutable state apart from the thread-local
 *    error text; a mesh handle must not be used by two threads at once.
 */
#ifndef PCH_H
#define PCH_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  PCH_OK = 0,
  PCH_EINVAL = -1,    /* bad argument: null pointer, size, source index, option */
  PCH_EMESH = -2,     /* non-manifold edge or vertex, inconsistent orientation,
                         zero-area face */
  PCH_ENOMEM = -3,    /* device or host allocation failed */
  PCH_EDEVICE = -4,   /* a HIP call failed (message has the HIP error) */
  PCH_EOVERFLOW = -5, /* window pool would exceed options.pool_limit */
  PCH_ENUMERIC = -6   /* non-finite value in window geometry */
} pch_status;

typedef struct pch_mesh_s* pch_mesh;

/* Mesh from vertex coordinates.
 *  xyz    host double [nv][3]
 *  faces  host int32  [nf][3], CCW, indices in [0, nv)
 * Edge lengths are sqrt((dx*dx + dy*dy) + dz*dz). The handle owns device
 * copies of the half-edge geometry (Section 4.1 and Table 1) until
 * pch_mesh_destroy. Errors: PCH_EINVAL (sizes, indices), PCH_EMESH. */
pch_status pch_mesh_create(const double* xyz, int64_t nv, const int32_t* faces, int64_t nf,
                           void* hip_stream, pch_mesh* out);

/* Mesh from the metric only (Section 4.1: "it needs only the metric").
 *  he_len host double [3 nf]: length of half-edge j; the two half-edges of
 *         an interior edge must agree to 1e-9 relative. */
pch_status pch_mesh_create_from_lengths(const int32_t* faces, int64_t nf, int64_t nv,
                                        const double* he_len, void* hip_stream, pch_mesh* out);

void pch_mesh_destroy(pch_mesh mesh);

/* Sizes and classification: counts of vertices, faces, boundary half-edges
 * and pseudo-source vertices (boundary or saddle, Section 3). Any output
 * pointer may be NULL. */
pch_status pch_mesh_info(pch_mesh mesh, int64_t* nv, int64_t* nf, int64_t* n_boundary_he,
                         int64_t* n_pseudo);

/* Host copies of the per-vertex tables: total angle (double [nv]) and flags
 * (uint8 [nv]: bit 0 boundary, bit 1 pseudo-source). Either may be NULL. */
pch_status pch_mesh_vertex_tables(pch_mesh mesh, double* theta, uint8_t* flags);

/* Selection rules (Section 4.2 step 1 and Section 5.1). */
enum {
  PCH_SELECT_KTH = 0,   /* the k smallest keys, to 36 bits below the top
                           differing bit of the pool's key range; ties kept */
  PCH_SELECT_DELTA = 1, /* keys up to the pool's smallest key plus a step that
                           starts at delta0 and is scaled after each round by
                           k / selected (clamped to [1/2, 2]); no histogram */
  PCH_SELECT_TABLE = 2,  /* per-round cutoff values from options.cutoff_table
                           (select key <= cutoff); after the table, KTH */
  PCH_SELECT_LEARNED = 3, /* cutoff from predicted vertex distances
                           (options.predicted): with C(r) the number of
                           vertices predicted within r, m the pool's smallest
                           key and w the windows processed per vertex within m
                           so far (w0 before any), select keys up to
                           C^-1(C(m) + f k / w), where the factor f starts at
                           1 and is scaled after each such round by
                           k / selected (clamped to [1/2, 2]); predictions
                           only steer the rounds, the distances stay exact */
  PCH_SELECT_STRIDED = 4 /* the paper's approximate selection (Section 6):
                           the pool scan runs on T = k threads (rounded up to
                           whole workgroups) and thread i selects the nearest
                           non-stale window among pool positions i, i + T,
                           i + 2T, ...; one launch, no histogram; children
                           of its rounds take no further hop. The result
                           depends on the pool's layout (the distances do
                           not) */
};

typedef struct {
  int32_t select_mode;        /* PCH_SELECT_* (default PCH_SELECT_KTH) */
  int32_t filters;            /* bit 0 CH one-angle-one-split, bit 1 ICH window
                                 filter, bit 2 full fans, bit 3 stronger
                                 filtering: a window takes the two endpoint
                                 tests of the ICH filter again with the
                                 round-start distances when it propagates
                                 (its drops count as ICH drops) (default 3) */
  int64_t k;                  /* windows per round for PCH_SELECT_KTH (default 16384) */
  double eps_tiny;            /* drop children narrower than eps_tiny * edge
                                 length (Section 5.3 uses 1e-6; default 0) */
  int64_t pool_capacity;      /* initial window capacity; 0 = from mesh size */
  int64_t pool_limit;         /* growth cap in windows; 0 = no cap */
  int32_t collect_stats;      /* 1 = per-round counts (see pch_round_log) */
  int32_t rounds_per_sync;    /* rounds enqueued between host polls (default 16) */
  const double* cutoff_table; /* host, n_cutoff values, PCH_SELECT_TABLE */
  int64_t n_cutoff;
  int32_t collect_timing;     /* n > 0: time the phases of every n-th round
                                 with HIP events on hip_stream
                                 (pch_stats.ms_phase, ms_propagate) */
  int32_t hops;               /* propagation hops per round, 1..16 (default 1:
                                 every selected window crosses one face, as in
                                 Algorithm 1). With h > 1, children that pass
                                 the round's own selection test propagate
                                 again in the same round, up to h times,
                                 against the round-start geod_dist and
                                 angle_split; distances are unchanged (the
                                 order of propagation does not matter and
                                 stale values only prune less), rounds drop */
  double delta0;              /* first step of PCH_SELECT_DELTA; 0 = twice the
                                 mean edge length */
  const float* predicted;     /* device, nv predicted distances (LEARNED) */
  double w0;                  /* windows per vertex before the first round of
                                 LEARNED (default 4) */
  int32_t organize;           /* 1 = before they propagate, group each round's
                                 selected windows by edge (a one-pass bucket
                                 sort on the half-edge index, 4096 buckets;
                                 data organization, Algorithm 3); the order
                                 changes no result (default 0) */
  int32_t counts;             /* 1 = count windows created, events, fans and
                                 dropped windows for pch_stats (default); 0 =
                                 skip these statistics counters (fewer
                                 same-address atomics per launch); rounds,
                                 processed windows and timing are still
                                 filled. collect_stats implies 1. */
  int32_t fuse_hops;          /* 1 = with hops <= 6, one launch propagates all
                                 hops of a round: each workgroup takes the
                                 hopping children of its own windows from
                                 lists in LDS, depth first (default); 0 = one
                                 launch per hop. Same windows, events and
                                 results either way */
  int32_t fuse_scan;          /* with fused hops, the pool scan of the
                                 selection runs in the same launch: each
                                 workgroup propagates the windows it selects
                                 at once, with no selection buffer (not with
                                 PCH_SELECT_STRIDED or organize). 2 = a
                                 thread's first hopping child stays in its
                                 registers, later ones go to the LDS lists
                                 (default); 1 = every hopping child goes to
                                 the LDS lists; 0 = a partition launch first.
                                 Same windows, events and results either
                                 way */
  int32_t round_graph;        /* 1 = enqueue each rounds_per_sync rounds as one
                                 captured HIP graph (kept in the mesh handle
                                 and replayed while the launch arguments stay
                                 the same; not with collect_timing or an odd
                                 rounds_per_sync); 0 = launch by launch
                                 (default) */
} pch_options;

/* Fill opts with the defaults above. */
void pch_options_default(pch_options* opts);

typedef struct {
  int64_t rounds, created, processed, stale, tiny, ich_dropped, dist_events, angle_events,
      fans, fan_windows, deferred, peak_pool, restarts;
  double ms_total;           /* host wall time of the call */
  double ms_propagate;       /* summed time of the timed propagation launches */
  int64_t propagate_launches; /* launches timed in ms_propagate (rounds with work) */
  double delta0;             /* first step used by PCH_SELECT_DELTA */
  int64_t hop_launches;      /* propagation launches per round: 1 when the
                                hops are fused, else hops */
  double ms_phase[4];        /* with collect_timing: GPU time of the timed
                                rounds' phases, from HIP events between them
                                on hip_stream: [0] selection (histogram passes
                                and partition), [1] propagation (=
                                ms_propagate), [2] organization by edge,
                                [3] events (Algorithm 4 and the next round's
                                set-up) */
  int64_t timed_rounds;      /* rounds timed in ms_phase */
  int64_t pool_windows;      /* sum over rounds of the live windows in the
                                pool at round start (what the selection
                                scans) */
  int64_t selected;          /* windows the selection took from the pool,
                                summed over rounds (processed minus those that
                                hopped on); with counts only */
  int32_t scan_fused;        /* the round's launch plan (fuse_scan): 0 = a
                                partition launch, then propagation; 1 = the
                                pool scan inside the propagation launch;
                                2 = the same with each thread's first
                                hopping child held in registers */
  int32_t fused_workgroups;  /* workgroups of the fused plans' propagation
                                launch: as many as the device holds at once
                                (the occupancy of that launch times the
                                compute units); 0 for the partition plan */
} pch_stats;

/* Exact geodesic distance from the sources (Algorithm 1).
 *  sources  host int32 [m]; m > 1 gives the min field over all sources
 *           (Section 4.2); duplicates are allowed
 *  dist     device double [nv], written in full
 *  opts     NULL = defaults; stats may be NULL
 * If the window pool outgrows its capacity the run restarts with twice the
 * capacity (stats->restarts counts them); PCH_EOVERFLOW if that would pass
 * opts->pool_limit. Errors: PCH_EINVAL (source out of range, m < 1, bad
 * option), PCH_ENOMEM, PCH_EDEVICE (a HIP error, or a window or event whose
 * half-edge or vertex index lies outside the mesh: every such index is
 * range-checked before it is gathered and none is dereferenced),
 * PCH_ENUMERIC (a window's apex crossing was not finite). */
pch_status pch_geodesic(pch_mesh mesh, const int32_t* sources, int32_t m, double* dist,
                        void* hip_stream, const pch_options* opts, pch_stats* stats);

/* pch_geodesic for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same fields, bit for bit, and the same arguments, but no hipMalloc,
 * hipFree or other allocation. The work buffers of the field (window pools,
 * selection, event buffers, and the device copies of the sources, cutoff
 * table and predicted-distance table) come from one static device array of
 * 256 MiB per GPU, which the library holds until the process ends; the mesh
 * handle's own state (created by pch_mesh_create) is used as by
 * pch_geodesic. Limits: at most 1024 sources; the work buffers of a pool of
 * capacity c take about 572 c bytes (c = opts->pool_capacity, else
 * max(2^18, 2 * 3 nf)), so the default capacity fits meshes up to about
 * 78,000 faces, and larger ones with a smaller pool_capacity (an overflowing
 * pool doubles within the 256 MiB). A field that would need more returns
 * PCH_EOVERFLOW before any device work. opts may not set collect_timing,
 * collect_stats, organize, or hops > 1 with fuse_hops = 0 (PCH_EINVAL);
 * round_graph is ignored (instantiating a graph allocates).
 * Every call on one GPU shares that GPU's array: calls that overlap on one
 * GPU (two host threads, or two streams) race and must not be made. */
pch_status pch_geodesic_noalloc(pch_mesh mesh, const int32_t* sources, int32_t m, double* dist,
                                void* hip_stream, const pch_options* opts, pch_stats* stats);

/* Per-round integer log of the last pch_geodesic call on this mesh that had
 * opts->collect_stats set, one int64 [14] record per round:
 *   pool size at round start, cutoff (bit pattern >> shift, -1 = all or
 *   strided), shift (-2 table, -3 adaptive step, -4 learned, -5 strided
 *   selection), selected, stale dropped, children kept, tiny dropped, ICH
 *   dropped, distance events from propagation, angle events, fans,
 *   fan windows kept, deferred fan events, pool size at round end.
 * Writes min(max_rounds, rounds) records to out (host); *n_rounds = rounds. */
pch_status pch_round_log(pch_mesh mesh, int64_t* out, int64_t max_rounds, int64_t* n_rounds);

/* ------------------------------------------------------------------------
 * Batched fields: many independent single-source fields on meshes of uneven
 * size in one persistent launch. Each workgroup takes the next field from a
 * device queue (most expected time first: 24 windows per half-edge before
 * the first run, then the workgroup time each field took in the previous
 * run) and runs
 * its rounds with the adaptive-step selection (PCH_SELECT_DELTA) or the
 * learned cutoff (PCH_SELECT_LEARNED, each field with its own predictions);
 * results equal pch_geodesic with the same rule, k, hops and (for LEARNED)
 * predictions bit for bit. With gang > 1 a
 * workgroup may instead join a running field of its own XCD when that field's
 * expected time left per workgroup exceeds the next queued field's; the field's
 * rounds are then split over its workgroups from the next round on. Fields
 * whose windows outgrow a workgroup's pool are rerun with pch_geodesic.
 * ---------------------------------------------------------------------- */
typedef struct pch_batch_s* pch_batch;

typedef struct {
  int64_t k;             /* windows per round and field (default 1024) */
  int32_t teams_per_cu;  /* resident workgroups per compute unit (default 2) */
  int32_t filters;       /* as pch_options.filters (default 3) */
  double eps_tiny;       /* as pch_options.eps_tiny (default 0) */
  int64_t pool_capacity; /* windows per workgroup; 0 = from the largest mesh
                            and k (at least 3 k, at most 2^21) */
  int32_t use_graph;     /* 1 = replay a captured HIP graph of the launch (default) */
  int32_t team_threads;  /* threads of the workgroup that runs one field: 256
                            (default), 512 or 1024 */
  int32_t hops;          /* as pch_options.hops (default 1) */
  int32_t gang;          /* most workgroups on one field, 1..32 (default 1):
                            with more than 1, a workgroup that finds no field
                            left joins a running field of its own XCD, whose
                            rounds are then split over its workgroups */
  int64_t wait_ticks;    /* longest wait of a shared field's workgroups for each
                            other, in ticks of the device's 100 MHz wall clock
                            (0 = 2 s); when a wait runs out the field is rerun
                            with pch_geodesic */
  int32_t select_mode;   /* PCH_SELECT_DELTA (default) or PCH_SELECT_LEARNED */
  const float* predicted; /* PCH_SELECT_LEARNED: device float [offsets[n_fields]],
                            the predicted distances of field f at
                            predicted[offsets[f] .. offsets[f + 1]) (the layout
                            of the output, see pch_batch_offsets); read at
                            every pch_batch_run, so the caller keeps it alive
                            and may change its values between runs */
  double w0;             /* as pch_options.w0 (default 4) */
} pch_batch_options;

typedef struct {
  int64_t fields, reruns, max_rounds, processed, created, teams, k;
  double ms_total; /* host wall time of the call */
} pch_batch_stats;

void pch_batch_options_default(pch_batch_options* opts);

/* meshes: n_meshes handles created on the current device (kept by reference:
 * they must outlive the batch). Field f is the distance field from vertex
 * field_source[f] of mesh field_mesh[f]. Errors: PCH_EINVAL (index out of
 * range, n_fields < 1), PCH_ENOMEM, PCH_EDEVICE. */
pch_status pch_batch_create(const pch_mesh* meshes, int32_t n_meshes, const int32_t* field_mesh,
                            const int32_t* field_source, int32_t n_fields, const pch_batch_options* opts,
                            pch_batch* out);
void pch_batch_destroy(pch_batch batch);

/* offsets: host int64 [n_fields + 1]; field f occupies dist[offsets[f] ..
 * offsets[f + 1]) in the output of pch_batch_run. */
pch_status pch_batch_offsets(pch_batch batch, int64_t* offsets);

/* dist: device double [offsets[n_fields]] (caller-owned). */
pch_status pch_batch_run(pch_batch batch, double* dist, void* hip_stream, pch_batch_stats* stats);

/* Status of a batched field (first column of pch_batch_field_stats). Every
 * field whose status is not PCH_FIELD_OK is rerun with pch_geodesic and the
 * same rule: a pool overflow, the round limit, an abandoned gang or a field
 * no workgroup finished then complete normally, while non-finite window
 * geometry makes pch_batch_run return PCH_ENUMERIC and an index outside the
 * mesh PCH_EDEVICE (the single-field checks). */
enum {
  PCH_FIELD_OK = 0,
  PCH_FIELD_OVERFLOW = 1,   /* the workgroup's window pool overflowed */
  PCH_FIELD_MAX_ROUNDS = 2, /* no termination within the round limit */
  PCH_FIELD_ABANDONED = 3,  /* a shared field whose workgroups stopped waiting */
  PCH_FIELD_NOT_RUN = 4,    /* no workgroup finished the field */
  PCH_FIELD_NONFINITE = 5,  /* a window's apex crossing was not finite */
  PCH_FIELD_BAD_INDEX = 6   /* a window or event named a half-edge or vertex
                               outside the mesh (an internal error: such an
                               index is never dereferenced) */
};
const char* pch_field_status_string(int64_t status);

/* Per-field record of the last run, host int64 [n_fields][10]: status
 * (PCH_FIELD_*, after any rerun the status of the batched attempt), rounds,
 * windows processed, windows created, fans,
 * peak pool, stale windows, the time from the start of the field to its end
 * in ticks of the device's constant-rate wall clock (100 MHz on MI355X; 0
 * after a rerun), the helper workgroups that joined it, and the ticks they
 * spent in it. The time of leader and helpers and the windows processed set
 * the next run's order (most time first) and how helpers choose among
 * running fields. */
pch_status pch_batch_field_stats(pch_batch batch, int64_t* out);

/* Autotuner: times k in {8192, 16384, 32768, 65536} with workgroup shapes
 * (256 threads, 1 per CU), (512, 1) and (1024, 1) and 1 or 4 hops per round,
 * with up to 8 workgroups per field, then gang sizes 1, 2, 4 and 16 at the
 * best of those, each on the whole batch (into dist); keeps the fastest in
 * the batch and returns it in chosen (may be NULL). */
pch_status pch_batch_tune(pch_batch batch, double* dist, void* hip_stream, pch_batch_options* chosen);

/* Tuner cache. pch_batch_tune records its choice for the batch's size
 * bucket: the GPU architecture, and floor(log2) of the largest mesh's
 * half-edges, of the half-edges summed over the fields, and of the field
 * count. pch_batch_tune_cached applies the recorded choice for the batch's
 * bucket (*hit = 1, no trial runs), or runs pch_batch_tune when there is none
 * (*hit = 0). The cache lives in the process. pch_tune_cache_save and
 * pch_tune_cache_load write and read it as text, one bucket per line (load
 * adds to it; PCH_EINVAL on an unreadable file or a malformed line). */
pch_status pch_batch_tune_cached(pch_batch batch, double* dist, void* hip_stream, pch_batch_options* chosen,
                                 int32_t* hit);
pch_status pch_tune_cache_save(const char* path);
pch_status pch_tune_cache_load(const char* path);

/* Geodesic Voronoi labels (the multi-source setting of Section 4 and the
 * paper's outlook on Voronoi diagrams): for every vertex the index in
 * sources[0..m) of its nearest source (ties to the lowest index; -1 when no
 * source reaches it) and the distance to it. Computed as the m single-source
 * fields in one batched launch (opts as for pch_batch_create; NULL =
 * defaults) and a per-vertex minimum, so every distance is exact. dist
 * (double) and label (int32) are caller-owned device arrays of nv entries;
 * the call allocates m * nv doubles of device memory for the fields and
 * returns after the work on hip_stream is done. Errors: as pch_batch_create,
 * PCH_ENOMEM, PCH_EDEVICE. */
pch_status pch_voronoi(pch_mesh mesh, const int32_t* sources, int32_t m, double* dist, int32_t* label,
                       void* hip_stream, const pch_batch_options* opts);

/* Iso-contours of a distance field (an application of the exact per-vertex
 * distances, like the geodesic Voronoi diagram the paper's future work names).
 * The contour of level c is that of the linear interpolant of the vertex
 * distances over each face (marching triangles): a face whose three values
 * are not all on the same side of c (side: d >= c) holds one segment between
 * the two crossing points of its edges; a face with a non-finite vertex
 * value holds none.
 *  faces      device int32 [nf][3] (the mesh's faces; half-edge j of face f
 *             is j = 3 f + k, from vertex faces[f][k] to faces[f][(k+1) % 3])
 *  dist       device double [nv], e.g. the output of pch_geodesic
 *  levels     host double [n_levels], finite, 1 <= n_levels <= PCH_ISO_MAX_LEVELS
 *  seg_he     device int32 [cap][2]: the half-edges of the two endpoints
 *  seg_t      device double [cap][2]: each endpoint's fraction along its
 *             half-edge from the start vertex, (c - d_a) / (d_b - d_a)
 *  seg_level  device int32 [cap]: the level index of the segment
 *  cap        segments the outputs hold (0: count only; outputs may be NULL)
 *  n_segments host: the number of segments (also when they exceed cap)
 * Segments come in no particular order; each (face, level) pair gives at most
 * one, so cap = nf * n_levels always suffices. Returns after the work on
 * hip_stream is done; allocates 16 bytes of device memory per call.
 * Errors: PCH_EINVAL (bad sizes or levels, a face index outside [0, nv)),
 * PCH_EOVERFLOW (more than cap segments: the first cap found are written and
 * n_segments holds the count), PCH_ENOMEM, PCH_EDEVICE. */
#define PCH_ISO_MAX_LEVELS 64
pch_status pch_isolines(const int32_t* faces, int64_t nf, int64_t nv, const double* dist, const double* levels,
                        int32_t n_levels, int32_t* seg_he, double* seg_t, int32_t* seg_level, int64_t cap,
                        int64_t* n_segments, void* hip_stream);

/* ------------------------------------------------------------------------
 * Learned distance predictor for PCH_SELECT_LEARNED: an MLP 7 -> 64 -> 64 -> 1
 * (ReLU) on features [(v - c) / R, (s - c) / R, |v - s| / R] of vertex v,
 * source s, mesh centre c and radius R. Output |v - s| (1 + softplus(y)).
 * FP32 master weights; weights and activations rounded to BF16 before each
 * product, FP32 accumulation. Parameters (PCH_MLP_NPARAM floats, host
 * copies): W1[7][64], b1[64], W2[64][64], b2[64], W3[64], b3.
 * ---------------------------------------------------------------------- */
#define PCH_MLP_NPARAM 4737
typedef struct pch_mlp_s* pch_mlp;

pch_status pch_mlp_create(uint64_t seed, pch_mlp* out);
void pch_mlp_destroy(pch_mlp mlp);
pch_status pch_mlp_get_params(pch_mlp mlp, float* host_params);
pch_status pch_mlp_set_params(pch_mlp mlp, const float* host_params); /* resets AdamW state */

/* xyz device double [nv][3]; center host double [3]; feats device float
 * [nv][7]; base device float [nv] (the chord |v - s|). */
pch_status pch_mlp_features(const double* xyz, int64_t nv, int32_t source, const double* center, double radius,
                            float* feats, float* base, void* hip_stream);
/* pred device float [n]. */
pch_status pch_mlp_forward(pch_mlp mlp, const float* feats, const float* base, int64_t n, float* pred,
                           void* hip_stream);
/* Loss mean(((pred - target) / scale)^2) over n samples and its gradient
 * (host float [PCH_MLP_NPARAM], may be NULL) without updating. */
pch_status pch_mlp_gradients(pch_mlp mlp, const float* feats, const float* base, const float* target,
                             const float* scale, int64_t n, float* grads_host, float* loss_host, void* hip_stream);
/* One AdamW step (beta 0.9 / 0.999, eps 1e-8, decoupled weight decay on the
 * weights) on that loss; loss_host (may be NULL) receives the loss before it. */
pch_status pch_mlp_train_step(pch_mlp mlp, const float* feats, const float* base, const float* target,
                              const float* scale, int64_t n, float lr, float weight_decay, float* loss_host,
                              void* hip_stream);

const char* pch_status_string(pch_status s);
const char* pch_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* PCH_H */
