// Kernel parameter block shared by the host runtime (runtime.cpp) and the
// device engine (engine_lane.h, compiled per model at run time).  Passed by
// value as the single kernel argument; plain fields only, fixed layout.
#ifndef CWC_KPARAMS_H
#define CWC_KPARAMS_H

struct cwc_kparams {
    unsigned long long seed;
    long long G;              // trajectories in this launch
    long long R;              // replicas per instance
    long long g_base;         // global id of this launch's first trajectory
    long long max_events;     // 0 = unlimited
    double dt;
    int K1;                   // sample points
    unsigned int cap;         // count cap (<= INT32_MAX)
    int rate_stride;          // 0: one shared rate row; else n_rules
    int init_stride;          // 0: one shared init row; else n_cells
    int KR;                   // accumulator (and trajectory) rows per instance
    int k_base;               // sample index of row 0
    int k_stop;               // suspend before recording this sample (streamed
                              // runs, time-sliced kernels only); >= K1: never
    int k_slice;              // time-sliced kernels: a slice also ends before a
                              // trajectory records its k_slice-th sample point
                              // of the slice (constant simulation time); 0: no
    int want_traj;
    int want_digest;
    const double *rates;      // [I or 1][n_rules]
    const int *init;          // [I or 1][n_cells]
    // per-trajectory outputs, indexed by local id g - g_base
    int *final_counts;        // [G][C]
    long long *events;        // [G]
    double *t_final;          // [G]
    unsigned long long *digest;  // [G]
    unsigned char *status;    // [G]
    int *n_recorded;          // [G]
    int *traj;                // [KR][C][G] (trajectory fastest) or null
    int *final_term;          // general models: [G][max_comp][3 + 2 NS] or null
    // on-line moments, indexed by instance ((g - g_base) / R) and sample
    unsigned long long *s1;       // [I][KR][C]
    unsigned long long *s2_hi32;  // [I][KR][C]
    unsigned long long *s2_lo32;  // [I][KR][C]
    unsigned long long *rec_hist; // [I][K1+1] trajectories by recorded count, or null
    unsigned long long *n_rows;   // [I][KR] trajectories that recorded each row, or
                                  // null (streamed runs count here instead)
    unsigned long long *cursor;   // persistent form: next unclaimed item
    const int *order;             // persistent form (also when its grid holds
                                  // every item and runs without the queue):
                                  // instance of the i-th group of R items in
                                  // claim order (null = identity)
    int nslot;                    // lane layout: accumulator rows per wavefront
                                  // (power of two, 1..64)
    long long chunk;              // persistent lane form: 1 = lanes claim single
                                  // items; >= 64 = a wavefront claims `chunk`
                                  // consecutive items into its own window
    // time-sliced (serving) form: per-trajectory checkpoint and progress
    int *ck_counts;               // [G][C] counts of a suspended trajectory
    double *ck_t;                 // [G]
    unsigned long long *ck_e;     // [G] applied events
    unsigned long long *ck_dig;   // [G]
    int *ck_kn;                   // [G] next sample index
    unsigned char *ck_state;      // [G] 0 not started, 1 suspended, 2 finished
    unsigned long long *done_count;  // trajectories finished so far
};

// Resident serving kernels: the queue of (job, trajectory) items that the
// host publishes while the kernel runs, passed by value beside the job
// table.  Items are CWC_RQ_ITEM words: job slot, first trajectory, job id,
// unused.
#define CWC_RQ_ITEM 4
struct cwc_rq {
    unsigned long long *head;   // device memory: items claimed so far
    const long long *tail;      // coherent host memory: items published
    const long long *items;     // coherent host memory: ring [mask + 1][CWC_RQ_ITEM]
    const int *stop;            // coherent host memory: nonzero = claim nothing more
    long long *done;            // coherent host memory [slots]: id of the job whose
                                // last item has finished, by job slot
    long long mask;             // ring entries - 1 (a power of two minus one)
    long long idle_ticks;       // wall-clock ticks a wavefront waits for an item
    int nslot;                  // lane layout: accumulator rows per wavefront
};

#endif
