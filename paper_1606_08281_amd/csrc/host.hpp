// host.hpp -- host-side objects of liblik: network handles and the
// network-specialised propagation kernels compiled at run time.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <map>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "../../include/lik.h"
#include "lik_internal.hpp"

namespace lik {
// Work partitioning used unless a caller sets another (lik_network_set_tuning).
constexpr lik_tuning kDefaultTuning = {1, 6, 1536, 1, 1, 0, 160, 0, 1, 16000, 60};
}  // namespace lik

struct lik_network {
    int32_t U, R;
    int32_t umax, rmax;  // size bucket of the generic kernels
    std::vector<int32_t> orders, stoich;
    int32_t kind[LIK_MAX_REACTIONS];
    int32_t s1[LIK_MAX_REACTIONS], s2[LIK_MAX_REACTIONS];
    uint32_t nu[LIK_MAX_REACTIONS][4];
    lik::Net4x8 n4;
    lik::Net8x16 n8;
    lik::Net32x64 n32;
    lik_tuning tuning = lik::kDefaultTuning;
    // (device, precision) -> loaded specialised kernel
    std::mutex spec_lock;
    struct SpecKernels {
        hipModule_t mod = nullptr;
        hipFunction_t item = nullptr;        // lik_propagate_spec
        hipFunction_t persistent = nullptr;  // lik_propagate_spec_p (R <= 16), or null
        hipFunction_t flow = nullptr;        // lik_flow_spec
    };
    std::map<std::pair<int, int>, SpecKernels> spec;
    // captured launch sequences of lik_eval_batch_device (LIK_FLAG_GRAPH)
    struct Graph {
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
        hipGraphNode_t admit = nullptr;  // the node whose seed changes per call
        lik::FilterDesc *desc = nullptr;
        lik::EngineArgs e;
        lik::RequestArgs r;
        unsigned admit_blocks = 0;
    };
    std::mutex graph_lock;
    std::map<std::string, Graph> graphs;
};

namespace lik {

// Source of the propagation kernel with this network's reaction tables as
// compile-time constants (same body as the generic kernels).
std::string specialized_source(const lik_network &net, int precision);

// The specialised kernel for the current device, compiled with hipRTC on
// first use (or read from the on-disk cache).  Returns nullptr and sets *err
// on failure.
enum SpecKind { kSpecItem = 0, kSpecPersistent = 1, kSpecFlow = 2 };
hipFunction_t specialized_kernel(lik_network &net, int precision, std::string *err,
                                 int kind = kSpecItem);

// The specialised kernel if an earlier call has already loaded it on the
// current device, else nullptr; never compiles or loads (no allocation).
hipFunction_t loaded_specialized_kernel(lik_network &net, int precision, int kind = kSpecItem);

// The flow kernel for filters of several networks (group g = nets[g]), each
// item running its network's specialised body; compiled with hipRTC (cached on
// disk) and loaded once per device for the life of the process.
std::string specialized_multi_source(const std::vector<lik_network *> &nets, int precision);
hipFunction_t specialized_multi_kernel(const std::vector<lik_network *> &nets, int precision,
                                       std::string *err);
bool precompile_multi(const std::vector<lik_network *> &nets, int precision, std::string *err);

// Code object of a generated kernel source (compiled with hipRTC, or read
// from the on-disk kernel cache keyed by the source, headers and compiler).
bool rtc_code(const std::string &src, std::vector<char> *code, std::string *err);

// Compile (or find in the disk cache) without loading: needs no device.
bool precompile_specialized(const lik_network &net, int precision, std::string *err);

// Release every captured graph of this network.
void release_graphs(lik_network &net);

// Release every module loaded for this network.
void release_specialized(lik_network &net);

// Kernel timing (lik_timing_enable): an event opening a propagation launch
// (null while timing is off), and the one closing it.
hipEvent_t timing_begin(hipStream_t s);
void timing_end_propagate(hipEvent_t begin, hipStream_t s);

// The fixed candidate tunings the autotuners time.
const lik_tuning *autotune_candidates(int *n);

// Error reporting (thread-local message for lik_last_error).
int fail(int code, const std::string &msg);
int hip_fail(hipError_t e, const char *where);
uint32_t compute_units();  // of the current device
unsigned persistent_waves();  // grid of the persistent propagation kernels
bool tuning_valid(const lik_tuning &t);
const char *tuning_rule();
inline size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// Argument checks shared by the entry points.
int check_common(lik_network_t net, const lik_obs_model *obs, const lik_eval_opts *opts,
                 int32_t n_theta, int32_t n_traj, int32_t n_particles);
int check_offsets(const int32_t *offs, int32_t M, int *t_max, int64_t *total);
int check_host_data(const lik_network *net, const lik_obs_model *obs, const lik_data *data,
                    int32_t n_theta, const uint32_t *theta_ids);

// One (network, precision) group of an engine iteration.
struct GroupLaunch {
    hipFunction_t spec = nullptr;    // network-specialised kernel, or null for generic
    hipFunction_t spec_p = nullptr;  // its persistent variant, or null
    bool persistent = false;         // take items from the group's counter (R <= 16)
    unsigned persistent_waves = 0;   // grid of the persistent variant
    const void *netargs = nullptr;   // generic kernel's network tables
    int umax = 0, rmax = 0, precision = 0;
    unsigned max_items = 0;          // upper bound on the group's work items
};

// One iteration: order the work, propagate every group, weigh/resample.
// `timed`: bracket the launches with timing events while timing is enabled.
hipError_t engine_iteration(const EngineArgs &e, const GroupLaunch *groups, int n_groups,
                            hipStream_t s, bool timed = true);

// The specialised kernel if the variant and the amount of work call for it.
// Returns false only when LIK_KERNEL_SPECIALIZED was asked for and failed.
bool choose_specialized(lik_network &net, int precision, int variant, double work,
                        hipFunction_t *fn, std::string *err);

const void *generic_netargs(const lik_network &net);

// Embedded kernel headers for run-time compilation (generated at build time).
int rtc_headers(const char *const **sources, const char *const **names);

}  // namespace lik
