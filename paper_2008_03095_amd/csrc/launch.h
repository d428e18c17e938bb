// Host-side launchers of the gfx950 kernels (one definition per .hip file).
#pragma once

#include "common.h"
#include "direct.h"

namespace infuse {

// sampler.hip
void launch_edge_hash(const GraphView& g, uint32_t seed, uint2* edges, hipStream_t st);
uint32_t x_sort_scratch_elems(uint32_t R);
void launch_x_sort(uint32_t seed, uint32_t R, uint32_t Rs, uint64_t* scratch, uint32_t* xs,
                   uint32_t* inv, uint32_t* pos, hipStream_t st);
uint32_t x_sort_single_max();  // largest R the batched set-up sorts itself
// batched set-up (kBpPrep) over the jobs of b; `blocks` = the phase's total
void launch_prep_batch(const BuildBatch& b, uint32_t blocks, hipStream_t st);

// cc.hip
void launch_fill_u32(uint32_t* p, uint64_t count, uint32_t value, hipStream_t st);
void launch_hook_rows(const GraphView& g, const MemoView& m, hipStream_t st);
void launch_hook_hubs(const GraphView& g, const MemoView& m, uint32_t chunk_tiles, hipStream_t st);
void launch_lists(const MemoView& m, hipStream_t st);
void launch_link(const GraphView& g, const MemoView& m, uint32_t blocks, hipStream_t st);
void launch_link_hubs(const GraphView& g, const MemoView& m, hipStream_t st);
void launch_flatten(const MemoView& m, uint32_t blocks, hipStream_t st);
void launch_count(const MemoView& m, hipStream_t st);
void launch_gain0(const MemoView& m, uint32_t blocks, hipStream_t st);

// batched labelling: the shape of one graph's job (hook_hubs and count
// parameters; workgroups per phase into blocks[kBatchPhases], prep excluded)
// and one phase's launch over all jobs of b (`blocks` = the phase's total)
void build_job_shape(const GraphView& g, const MemoView& m, uint32_t chunk_tiles, uint32_t list_blocks, BuildJob* job,
                     uint32_t* blocks);
void launch_build_batch(const BuildBatch& b, uint32_t phase, uint32_t blocks, hipStream_t st);

// celf.hip
uint32_t celf_topw_blocks(uint32_t n);
// A persistent job description as kernel-argument words (at most 512 bytes).
constexpr uint32_t kJobWords = 128;
struct JobWords {
  uint32_t w[kJobWords];
};
// Set-up of one selection in one launch: coverage words of the listed tiles
// cleared, keys from the initial gains, the persistent kernel's state
// cleared and, with `job` (host memory of kJobWords words), its description
// written to `pjob`.
void launch_celf_setup(const CelfView& c, uint32_t* pscratch, uint32_t scratch_words, const void* job,
                       void* pjob, hipStream_t st);
void launch_celf_step(const CelfView& c, uint32_t bulk_blocks, hipStream_t st);
void launch_celf_topw(const CelfView& c, hipStream_t st);
void launch_celf_eval(const CelfView& c, hipStream_t st);
// many selections (im_batch_select): their set-up in one launch (`blocks`
// = first[njobs]) and the packing of their results into the records at out
void launch_celf_prepare_batch(const CelfBatchJob* jobs, const uint32_t* first, uint32_t njobs, uint32_t blocks,
                               hipStream_t st);
void launch_celf_collect_batch(const CelfBatchJob* jobs, uint32_t njobs, unsigned char* out, hipStream_t st);
void launch_celf_bulk(const CelfView& c, uint32_t bulk_blocks, hipStream_t st);

// celf_persistent.hip
uint64_t pcelf_scratch_bytes();
uint64_t pcelf_err_offset();   // u32 error flag of the persistent kernel
uint64_t pcelf_prof_offset();  // 16 x u64: phase ticks (100 MHz) x10, -, -, barriers, rounds, rebuilds/bulks, look-ahead commits
uint64_t pcelf_work_offset();  // 2 x u64 (profiling): listed tiles evaluated, their non-singleton columns
uint32_t pcelf_grid(int device);
uint64_t pcelf_job_bytes();
// Writes the description of one selection (for a group of group_blocks
// workgroups) into host memory of pcelf_job_bytes() bytes.
// prof: bit 0 phase clock, bit 1 work counts (listed tiles and gathers)
void pcelf_fill_job(void* host_job, const CelfView& c, void* scratch, uint32_t* blist, uint32_t group_blocks,
                    uint32_t round0, uint32_t prof);
// jobs: device array of njobs descriptions.  first: device prefix sums of
// workgroups per description (njobs + 1 entries, each at least one), or
// nullptr for grid / group_blocks equal groups taking descriptions in turn.
hipError_t launch_celf_persistent(const void* jobs, uint32_t njobs, uint32_t grid, uint32_t group_blocks,
                                  const uint32_t* first, hipStream_t st);

// query.hip
uint32_t sigma_pair_max();
void launch_sigma_pair(const MemoView& m, const uint32_t* S, uint32_t len, unsigned long long* out,
                       hipStream_t st);
void launch_sigma_bitmap(const MemoView& m, const uint32_t* S, uint32_t len, uint32_t* bm,
                         uint32_t cwords, unsigned long long* out, hipStream_t st);
void launch_export(const MemoView& m, const uint32_t* pos, uint32_t r0, uint32_t cnt, uint32_t v0,
                   uint32_t nv, int mode, int32_t* out, hipStream_t st);

}  // namespace infuse
