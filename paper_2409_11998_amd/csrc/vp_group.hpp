// Group execution structures shared by the batched API (vp_batch.hip, which
// also holds the kernels and the host code) and the serving loop
// (vp_server.hip).  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>

#include <vector>

#include "vp_device.hpp"

namespace vp {

// Device descriptors of one instance (plan + workspace) and its two levels.
struct LevelDesc {
    LevelGeom g;
    const int* vol_start; const int* vol_ij; const void* vol_dx; const void* vol_dy; const int* vol_idx;
    const int* bnd_start; const int* bnd_ij; const void* bnd_dx; const void* bnd_dy; const int* bnd_idx;
    const int* tgt_start; const int* tgt_ij; const void* tgt_dx; const void* tgt_dy; const int* tgt_idx;
    void* grid;
    void* spec;
    void* dgrid[2];  // double-layer channel grids and spectra of a level with dip (else NULL)
    void* dspec[2];
    const void* mult;
    const void* tw;
    void* hist;
    const double* horner;
    const double* horner_i;
    const float* horner_if;  // float32 plans: the interpolation table as float32
    const WorkUnit* sp_units;
    const WorkUnit* in_units;
    int n_sp_units;
};

struct InstDesc {
    int64_t n_src, n_bnd, n_tgt;
    const double* w;
    const double* nx;
    const double* ny;
    double* dc;
    unsigned long long* smax;
    void* str;
    dev::LocalArgs loc;  // geometry pointers and constants; per-call fields come from CallDesc
    int has_vol, has_bnd;
};

// Densities and output of one call (NULL density = kind not evaluated).
struct CallDesc {
    const double* f;
    const double* jet6;
    const double* sigma;
    const double* sj;
    const double* mu;
    const double* mj;
    double* out;
};

// A stage's work: segments of `count` units of (instance, level), items
// [begin, begin + count rounded up to 8).  In the spread, row-pass and
// forward-column stages level = l + 2 c addresses channel c of level l
// (c = 1, 2: the double-layer channels of a level with dip).
struct Seg {
    int inst;
    int level;
    int count;
    int begin;
};

struct StageTab {
    int nseg;
    int nitems;
    const Seg* seg;
};

struct HostStage {
    std::vector<Seg> seg;
    int nitems = 0;
    int w = 0;       // spreading width (spread / interpolation stages)
    int mma = 0;     // spread stage on matrix cores (float32 levels on kMmaTile tiles)
    size_t lds = 0;  // dynamic LDS bytes of the launch
    void add(int inst, int level, int count);
};

// Host image of everything one launch sequence reads: descriptors, call
// table and segment tables, laid out as in the device buffer.
struct GroupPlan {
    int precision = VP_FP64;
    std::vector<InstDesc> inst;
    std::vector<LevelDesc> lv;
    std::vector<CallDesc> call;
    HostStage zero, str, row, colf, col, c2r, local;
    std::vector<HostStage> spread, interp;  // one per distinct spreading width
    size_t off_inst = 0, off_lv = 0, off_call = 0, off_seg = 0, bytes = 0;
    std::vector<unsigned char> blob;
};

// Device-side views of a group placed at some device address.
struct GroupTabs {
    const InstDesc* inst = nullptr;
    const LevelDesc* lv = nullptr;
    CallDesc* call = nullptr;
    StageTab zero{}, str{}, row{}, colf{}, col{}, c2r{}, local{};
    std::vector<StageTab> spread, interp;
};

// Build the host image of a group (all plans of one precision).  args[i]:
// densities of instance i (NULL = kind not evaluated); kinds: VP_KIND_* the
// calls will pass whatever args holds now (a batch fixes its kinds when it is
// built and its densities per call).
vp_status group_build(const std::vector<const Plan*>& plans, const std::vector<Workspace>& ws,
                      const std::vector<vp_eval_args>& args, GroupPlan& G, int kinds = 0);
// Place the segment tables into G's image for a device buffer at dev_base.
GroupTabs group_tabs(GroupPlan& G, unsigned char* dev_base);
// Stage kinds a group launch times (vp_batch_get_timing).
constexpr int kBatchStages = VP_BATCH_STAGES;
// Enqueue every stage of a group whose image has been copied to the device;
// ev: NULL, or kBatchStages + 1 events recorded around the stage kinds.
hipError_t group_launch(const GroupPlan& G, const GroupTabs& T, hipStream_t st, hipEvent_t* ev = nullptr);
// Upper bound of the device image of a group of n instances.
size_t group_bytes_bound(size_t n);
// Build a group, stage its image in host_buf (pinned), copy it to dev_buf
// (stream-ordered) and launch it.  Both buffers (buf_bytes each) must stay
// untouched until the group has completed.  *enqueued tells whether the copy
// was issued (then, on a later failure, the stream must drain before host_buf
// is reused).
vp_status group_enqueue(const std::vector<const Plan*>& plans, const std::vector<Workspace>& ws,
                        const std::vector<vp_eval_args>& args, void* dev_buf, unsigned char* host_buf,
                        size_t buf_bytes, hipStream_t st, bool* enqueued);

}  // namespace vp
