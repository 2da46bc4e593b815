// Host-callable launchers of the shsph kernels (internal to the library).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include "common.hpp"

namespace shsph {

// Caller-order particle fields (structure of arrays, storage type T).
template <class T> struct FieldPtrs {
    const T *x, *y, *z, *vx, *vy, *vz, *u, *h, *ax, *ay, *az, *du;
    const u32* pid;
};

// Key-order working arrays owned by the context.
template <class T> struct SortedPtrs {
    vec4<T>* posh;     // x, y, z, h (h = current smoothing length)
    vec4<T>* velu;     // v*, u* (velocity and energy the derivatives use)
    vec4<T>* vhalf;    // v^{n+1/2}, u^{n+1/2} (stepping only)
    T* hn;             // h at the start of the step (normalises the h iteration)
    T* hcache;         // h the neighbour cache was built with (chi check)
    u32* pid;          // particle ids carried through the reordering
};

// Karras tables (App. B.7) plus node-indexed links for the traversals.
struct TreePtrs {
    u32 *lchild, *rchild, *endrange;   // local leaf/internal ids per instance
    u8 *lflag, *rflag;
    u32* child;                        // 2 per internal node: global node ids
    u32* parent;                       // per node (internal, then leaves)
};

// Caller-order outputs of a step (written at the particle's key-order slot).
template <class T> struct OutPtrs {
    T *x, *y, *z, *vx, *vy, *vz, *u, *h, *ax, *ay, *az, *du, *rho, *omega;
    u32* pid;
};

// The group neighbour cache: per group, its union of neighbour leaves
// (uleaf, with the union slot where each leaf starts, uslot; ucnt leaves,
// ustot slots; capacity cap per group), and per particle its neighbours as
// 16-bit union slots, four per word, ELL layout with a capacity per group:
// nlist[(gbase[g] + j / 4) * GROUP + lane]; ncnt[a] of them (32-bit slots,
// two per word, for a union of more than 65535 particles: see slot32_of).
struct CacheView {
    const u32 *uleaf, *uslot, *ucnt, *ustot;
    i64 cap;
    const u64* nlist;
    const u32* ncnt;
    const u64* gbase;         // first word of each group (words of GROUP lanes)
    const void *glo, *ghi;    // group boxes (vec4<T>) for the interior test
    const void* blo;          // node boxes: h_max of each instance's root
    const u32* root;
    double rk;                // R chi
    u64* work;                // work counters, 64 slots x 2 (profiling), or null
    const u32* skip;          // force: a device word that switches the launch off, or null
};

// Per-block partial sums of the corrector (instance id, or -1 if the block
// spans two instances and added its lanes directly).
struct BlockPart {
    int inst;
    int pad;
    double dv2, v2;
};

struct SphParams {
    double hfact, gamma, alpha, beta, beta_u, chi, lambda, eps_h, c_cour, c_force, r_kern;
    int max_iter;
    int kernel;             // KernelId (Sect. 2.1.1)
    double alpha_min, alpha_max, sigma_decay;   // shock-detection switch (App. G)
    int force_split;        // threads per particle in the force kernel (1 or 2)
};

// scan.hip
size_t scan_tmp_bytes(i64 n);
void scan_u8_u32(const u8* in, u32* out, i64 n, void* tmp, hipStream_t st);
void scan_u32_u32(const u32* in, u32* out, i64 n, void* tmp, hipStream_t st);
void scan_u32_u64(const u32* in, u64* out, i64 n, void* tmp, hipStream_t st);

// sort.hip
size_t radix_state_words(i64 n, int nseg);
int radix_sort_pairs(u64* k0, u32* v0, u64* k1, u32* v1, i64 n, int key_bits, const i64* seg_off,
                     int nseg, u32* state, u32* err, u32* host_word, hipStream_t st);

// tree.hip
template <class T>
void launch_predict_morton(const FieldPtrs<T>& f, i64 n, const InstDev* inst, const i64* p_off,
                           int ninst, const double* dt_inst, u64* keys, u32* vals, int bits,
                           hipStream_t st);
template <class T>
void launch_gather(const FieldPtrs<T>& f, i64 n, const InstDev* inst, const i64* p_off, int ninst,
                   const double* dt_inst, const u32* eps, const SortedPtrs<T>& s, hipStream_t st);
template <class T>
void launch_bbox(const FieldPtrs<T>& f, i64 n, InstDev* inst, const i64* p_off, int ninst,
                 const double* dt_inst, u64* bb, hipStream_t st);
void launch_mask_init(const u64* mu, i64 n, const i64* p_off, int ninst, u8* xi, hipStream_t st);
void launch_reduce_pass(const u64* mu, i64 n, const i64* p_off, int ninst, const u8* xold, u8* xnew,
                        hipStream_t st);
// Keep mask + nred reduction passes + scan + compaction in one kernel; `state`
// holds leaves_fused_state_words(n) words (cleared here); flag[0] is set if
// some tile could not be resolved in its window (then nothing it wrote is
// valid: run the separate passes), flag[1] on a look-back overrun.
size_t leaves_fused_state_words(i64 n);
void launch_leaves_fused(const u64* mu, i64 n, const i64* p_off, int ninst, int nred, u32* state,
                         u8* xi, u32* xscan, u32* id, u64* mu_leaf, u32* flag, hipStream_t st);
void launch_compact(const u64* mu, const u8* xi, const u32* xscan, i64 n, u32* id, u64* mu_leaf,
                    hipStream_t st);
// Tree node numbering: internal nodes 0 .. ni-1, leaf j at node lbase + j
// with lbase = n - ninst (the most internal nodes n particles can give), so
// the layout does not depend on the leaf count.  The Karras and box kernels
// read the leaf count from leaf_off[ninst] (device); their grids are sized
// from the caller's bound (the leaf count when known, else n).
void launch_inst_leaves(const i64* p_off, int ninst, const u32* xscan, i64 n, i64* leaf_off,
                        i64* ioff, u32* root, u32* parent, i64 lbase, hipStream_t st);
void launch_karras(const u64* mu_leaf, const i64* leaf_off, const i64* ioff, int ninst,
                   i64 lbase, i64 grid_internal, const TreePtrs& t, hipStream_t st);
template <class T>
void launch_boxes_up(const vec4<T>* posh, const u32* id, i64 grid_leaves, i64 lbase,
                     const u32* child, const u32* parent, const u32* endrange, const i64* ioff,
                     const i64* leaf_off, int ninst, u32* arrive, u32* rec, u32* nrec,
                     u32* rscan, void* scan_tmp, vec4<T>* blo, vec4<T>* bhi, u32* flags,
                     hipStream_t st, const u32* skip = nullptr);
size_t boxes_rec_count(i64 n_leaf);
// Export in compact numbering (leaf j at row n_internal + j).
void launch_prefix_boxes(const u64* mu_leaf, const i64* leaf_off, const i64* ioff, int ninst,
                         i64 n_internal, i64 n_leaf, i64 lbase, const u32* endrange,
                         const u32* parent, u32* pbox, i32* plen, int shift, hipStream_t st);

// neigh.hip
template <class T>
void launch_group_boxes(const vec4<T>* posh, const GroupMap& gm, i64 ngroups, vec4<T>* glo,
                        vec4<T>* ghi, hipStream_t st, const u32* skip = nullptr);
template <class T>
void launch_group_leaves(const vec4<T>* blo, const vec4<T>* bhi, const u32* child, const u32* id,
                         const u32* xscan, i64 n_internal, const vec4<T>* glo, const vec4<T>* ghi,
                         i64 ngroups,
                         const GroupMap& gm, const u32* root, const InstDev* inst, double rk,
                         i64 cap, u32 spread, bool serial, u32* uleaf, u32* uslot, u32* ucnt,
                         u32* ustot, u32* flags, const u8* redo, hipStream_t st);
template <class T>
void launch_group_cache(const vec4<T>* posh, const vec4<T>* blo, const vec4<T>* bhi, const u32* id,
                        const u32* xscan, i64 n_internal, const GroupMap& gm, i64 ngroups, const InstDev* inst,
                        double rk, double rkc, i64 cap, const u32* uleaf, const u32* uslot,
                        const u32* ucnt, const u32* ustot, const u64* gbase, const u32* gcap,
                        u64 words_alloc, u32* gneed, const u8* gredo, u64* nlist, u32* ncnt,
                        u32* flags, const vec4<T>* glo, const vec4<T>* ghi, const u32* root,
                        u64* work, int mode, const u8* redo, hipStream_t st);
// Per-group cache capacities (words per lane) for a build: from the need the
// group showed in the previous build (gneed, words; 0 = none yet: `dflt`),
// with a quarter's headroom, never above what the group's union could fill;
// gbase = exclusive scan of the capacities (gbase[ngroups] = total words).
void launch_cache_plan(const u32* ustot, const u32* gneed, i64 ngroups, u32 dflt, u32* gcap,
                       u64* gbase, void* scan_tmp, hipStream_t st, const u32* skip = nullptr);
// After an overflow: groups whose need exceeds their capacity get a larger
// range appended at the end (gbase[ngroups] grows) and gredo = 1; the others
// keep theirs (gredo = 0).
void launch_cache_regrow(const u32* gneed, i64 ngroups, u32* gcap, u64* gbase, u8* gredo,
                         hipStream_t st);
void launch_cache_to_global(const u32* id, const GroupMap& gm, i64 ngroups, i64 cap,
                            const u32* uleaf, const u32* uslot, const u32* ucnt, const u32* ustot,
                            const u64* gbase, const u64* nlist, const u32* ncnt, const u64* off,
                            u32* list, hipStream_t st);

// sph.hip
void launch_fill_u32(u32* p, i64 n, u32 v, hipStream_t st);
void launch_iota_u32(u32* p, i64 n, hipStream_t st);
// skip (device word, optional) on these launches: when nonzero the launch
// does nothing (a captured pass switches later stages off on the device).
void launch_stat_reset(InstStat* s, int ninst, int what, const u8* redo, hipStream_t st,
                       const u32* skip = nullptr);
template <class T>
void launch_root_hmax(const vec4<T>* blo, const u32* root, int ninst, double* out, hipStream_t st);
void launch_dt_select(double* dt_inst, const InstStat* s, const double* dt_host, int ninst,
                      hipStream_t st);
// Captured passes (see sph.hip): gs[0] abort word, gs[1 + r] re-run round r
// switched off; gate[k] the density's per-instance switch; redo[k] and
// reruns[k] the corrector re-runs.
void launch_gate_build(const u32* flags, u32 mask0, int w_sort, int w_leaves, const double* rhmax,
                       const InstDev* inst, int ninst, double rk, u32* gs, u8* gate, u32* reruns,
                       hipStream_t st);
void launch_gate_density(const InstStat* stat, int ninst, u32* gs, u8* gate, hipStream_t st);
void launch_gate_exceed(const InstStat* stat, int ninst, const u32* gs, u32* skw, u8* rx,
                        hipStream_t st);
void launch_flag_and(u32* f, u32 mask, hipStream_t st);     // f[0] &= mask
void launch_gate_round(const u32* flags, u32 mask0, const double* rhmax, const InstDev* inst,
                       int ninst, double rk, const u32* skw, u32* gs, u8* rx, hipStream_t st);
void launch_rerun_decide(const InstStat* stat, const i64* p_off, int ninst, double eps_v,
                         int max_reruns, int r, u32* gs, u8* redo, u32* reruns, hipStream_t st);
template <class T>
void launch_copy_h(const vec4<T>* posh, T* hc, i64 n, hipStream_t st, const u32* skip = nullptr);
template <class T>
void launch_density(const SortedPtrs<T>& s, const u32* id, const GroupMap& gm, i64 ngroups,
                    const InstDev* inst, const SphParams& P, const CacheView& cv, T* omega,
                    vec4<T>* thermo, u8* status, InstStat* stat, const u8* redo, hipStream_t st);
// Density then force in one persistent cooperative launch (see sph.hip);
// the force runs only if no particle left chi h_cache.  Returns 0, or -1 if
// the launch was not possible (the caller then runs the separate kernels).
template <class T>
int launch_density_force(const SortedPtrs<T>& s, const vec4<T>* thermo, const u32* id,
                         const GroupMap& gm, i64 ngroups, int ninst, const InstDev* inst,
                         const SphParams& P, const CacheView& cvd, const CacheView& cvf, T* omega,
                         u8* status, InstStat* stat, vec4<T>* acc, T* vsig, hipStream_t st);
template <class T>
void launch_force(const SortedPtrs<T>& s, const vec4<T>* thermo, const u32* id, const GroupMap& gm,
                  i64 ngroups, const InstDev* inst, const SphParams& P, const CacheView& cv,
                  vec4<T>* acc, T* vsig, InstStat* stat, hipStream_t st);
template <class T>
void launch_correct(const SortedPtrs<T>& s, const vec4<T>* acc, const T* omega, i64 n,
                    const i64* p_off, int ninst, const InstDev* inst, const double* dt_inst,
                    double hfact, const OutPtrs<T>& o, InstStat* stat, BlockPart* part,
                    hipStream_t st, const u32* skip = nullptr);
void launch_fold_parts(const BlockPart* part, i64 nblocks, int ninst, InstStat* stat, hipStream_t st,
                       const u32* skip = nullptr);
template <class T>
void launch_gather_velu(const u32* eps, i64 n, const T* vx, const T* vy, const T* vz, const T* u,
                        vec4<T>* velu, hipStream_t st);
template <class T>
void launch_alpha(const SortedPtrs<T>& s, const vec4<T>* acc_n, const T* omega, const u32* id,
                  const GroupMap& gm, i64 ngroups, const InstDev* inst, const SphParams& P,
                  const CacheView& cv, const double* dt_inst, T* alpha, vec4<T>* thermo,
                  hipStream_t st);
template <class T> void launch_gather1(const u32* eps, i64 n, const T* src, T* dst, hipStream_t st);
template <class T>
void launch_velu_from_out(const OutPtrs<T>& o, i64 n, const i64* p_off, int ninst,
                          const InstDev* inst, const u8* redo, vec4<T>* velu, hipStream_t st);
template <class T>
void launch_thermo(const vec4<T>* posh, const vec4<T>* velu, const T* omega, i64 n,
                   const i64* p_off, int ninst, const InstDev* inst, double hfact, double gamma,
                   double alpha, const T* alpha_s, vec4<T>* thermo, hipStream_t st,
                   const u32* skip = nullptr);
template <class T>
void launch_scatter(const u32* eps, i64 n, const vec4<T>* src4, int comp, const T* src1,
                    T* dst, hipStream_t st);
template <class T>
void launch_scatter_rho(const u32* eps, i64 n, const vec4<T>* posh, const i64* p_off, int ninst,
                        const InstDev* inst, double hfact, T* dst, hipStream_t st);

}  // namespace shsph
