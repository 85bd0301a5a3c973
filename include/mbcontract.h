/*
 * mbcontract.h -- C ABI of the MI355X (gfx950) implementation of the
 * recursive multibaryon contraction method of Guenther, Toth and Varnhorst,
 * "A recursive approach to determine correlation functions in multibaryon
 * systems" (arXiv:1301.4895).
 *
 * Three calls carry the method:
 *   mb_build_term_list      the per-nucleus, configuration-independent part
 *                           (Sec. 3-5, 7): L by the recursion of eq. recr_L,
 *                           the required components of every stage and the
 *                           operation lists Lambda, built once on the host.
 *   mb_make_blocks          the baryon blocks f_P, f_N of Sec. 2 (with the
 *                           several-source form of Sec. 6) from quark
 *                           propagators in device memory, antisymmetrised in
 *                           their same-flavour quark indices (Sec. 4), and
 *                           for a system with a Lambda its block f_L.
 *   mb_contract_correlator  the recursion F_-^(n+1) = F_-^(n) . f (eq. recr_F)
 *                           over the operation lists and the final contraction
 *                           with L (eq. C_final, eq. C_final_moresource).
 *
 * Conventions (0-based).  Quark index xi = N_s*(3*spin + colour) + source;
 * with nonrelativistic operators only spins 0, 1 enter (Sec. 7), so xi runs
 * over 3*D*N_s values with D = 4 (relativistic) or 2.  Baryon index
 * psi (sink) or chi (source) = N_s*alpha + s, D*N_s values; at the sink s
 * selects the sink function.  Within a correlator the baryons are ordered
 * protons first, then neutrons, then the Lambda, each species in ascending
 * index, identically at sink and source; the result is C(delta set; alpha
 * set) of eq. C_final with the
 * normalisation that makes it equal the Wick contraction of Sec. 2 (no
 * overall Grassmann sign).
 *
 * Ownership.  A term list is an opaque host object owned by the caller
 * (free it with mb_term_list_free).  Every device buffer -- propagators, sink
 * weights, exponents, blocks, correlators, workspaces and the device image of
 * the term list -- is allocated and owned by the caller; the library never
 * allocates device memory.  Device calls are asynchronous on the given HIP
 * stream (NULL = default stream); device faults surface at the caller's next
 * synchronisation.
 *
 * Errors.  Every call returns MB_OK (0) or a negative MB_E* code; arguments,
 * and the existence of a kernel for every launch of the call, are validated
 * on the host before anything is launched, and nothing is launched when a
 * call fails validation (MB_EHIP from the runtime during the launches can
 * leave earlier launches of the call queued).  mb_last_error() gives a
 * message for the last failure of the calling thread.
 */
#ifndef MBCONTRACT_H
#define MBCONTRACT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MB_OK 0
#define MB_EINVAL (-1)        /* malformed argument                          */
#define MB_EPAULI (-2)        /* more baryons/quarks than indices (Sec. 6)    */
#define MB_EUNSUPPORTED (-3)  /* outside what this build supports             */
#define MB_ENOWORKSPACE (-4)  /* buffer smaller than the queried size         */
#define MB_EHIP (-5)          /* a HIP runtime call failed                    */
#define MB_ENOMEM (-6)        /* host allocation failed                       */

#define MB_PATH_AUTO 0         /* more numerous species first, neutrons on a tie (Sec. 7) */
#define MB_PATH_PROTONS_FIRST 1
#define MB_PATH_NEUTRONS_FIRST 2
#define MB_PATH_EXPLICIT 3     /* the order given in mb_nucleus.order */
#define MB_PATH_BEST 4         /* the order with the fewest operations (below) */

#define MB_C64 0               /* complex float (re, im)   */
#define MB_C128 1              /* complex double (re, im)  */

#define MB_FP64 0              /* recursion stages stored in double              */
#define MB_MIXED 1             /* recursion stages stored in float (half the
                                  memory traffic of the bandwidth-bound gathers);
                                  blocks stored in double, every product and sum
                                  formed in double                                */
#define MB_MIXED_F32B 2        /* as MB_MIXED, and the recursion steps read float
                                  copies of the block entries (rounded once from
                                  the scaled double blocks); the first stage and
                                  every product and sum as in MB_MIXED.  The
                                  LDS-staged step kernel (MB_TUNE_KERNEL = 1) is
                                  refused with it (MB_EUNSUPPORTED)               */

/* A nucleus of n_P protons and n_N neutrons (Sec. 7), and optionally one
 * Lambda hyperon.
 *   rel    1: Gamma_1 = 1, Gamma_2 = C gamma_5; 0: the nonrelativistic
 *          Gamma_1 = P_nr, Gamma_2 = C gamma_5 P_nr (Dirac representation).
 *   n_src  number of orthogonal quark sources N_s (Sec. 6): 1 or 2, and 3
 *          with nonrelativistic operators (18 quark indices per flavour);
 *          MB_EUNSUPPORTED otherwise.
 *   path   order of the recursion (MB_PATH_*).  AUTO, PROTONS_FIRST and
 *          NEUTRONS_FIRST add all baryons of one species before the other.
 *          EXPLICIT: bit i of `order` set means that the (i+1)-th baryon added
 *          is a proton (n_P bits among the low n_P + n_N).  BEST: of every
 *          order (C(A, n_P) of them) the one with the fewest operations
 *          n_lambda for this request (Sec. 7: the best path is decided case by
 *          case); ties go to the AUTO order, then to the smaller mask.  The
 *          search counts the required sets of every order backwards from the
 *          final ones, without operation tables; MB_EUNSUPPORTED with side
 *          requests.  The correlators do not depend on the order.
 *   order  see EXPLICIT (ignored otherwise)
 *   n_Lambda  0, or 1 for a system with one Lambda: the baryon form of Sec. 1
 *          (eq. C_baryons) with (q1, q2, q3) = (s, u, d) and the nucleons'
 *          Gamma_1, Gamma_2, a third quark flavour s whose propagator is
 *          mb_problem.prop_s.  The Lambda is added after the nucleons (the
 *          last step of the path; its operations split one u, one d and the
 *          s index off every final component).  Supported with up to 12
 *          quark indices per flavour (relativistic with one source,
 *          nonrelativistic with one or two) and without side requests,
 *          projection or MB_PATH_BEST; n_P + n_N may be 0 (a single Lambda).
 *          MB_EUNSUPPORTED otherwise.                                        */
typedef struct {
    int n_P, n_N;
    int rel;
    int n_src;
    int path;
    uint32_t order;
    int n_Lambda;
} mb_nucleus;

/* Which components of C(delta set; alpha set) are wanted (Sec. 5, Sec. 8).
 *   all_components != 0: every sink set over the D*N_s baryon indices and,
 *          with one source, every source set; with several sources the
 *          source sets that put min(n, D) baryons of a species on source 0,
 *          min(rest, D) on source 1 and the rest on source 2 (the
 *          convention of Tables 1-3).  The other fields are ignored.
 *   otherwise: sink_P, sink_N are bit masks of the sink baryon indices; the
 *          output rows are every n_P-subset of sink_P times every
 *          n_N-subset of sink_N.  alpha[2*i], alpha[2*i+1] are the proton
 *          and neutron source index sets (bit masks, popcounts n_P and n_N)
 *          of output column i, 0 <= i < n_alpha.  A single spin component
 *          (Sec. 8) has sink_P = alpha[0], sink_N = alpha[1], n_alpha = 1.
 *   sink_L, alpha_L  with a Lambda: the Lambda's sink base set (rows: every
 *          proton set, then neutron set, then Lambda index of it, Lambda
 *          fastest) and alpha_L[i] its one-bit source set of column i; with
 *          all_components every index at the sink and, at the source, each
 *          of source 0's.  Ignored without a Lambda.
 *   proj   NULL: every (sink set, source set) component is an output.
 *          Otherwise the projection of Sec. 5: real weights
 *          proj[delta * n_alpha + alpha] over the sink sets (in the order
 *          of MB_EXPORT_DELTA) and source sets (MB_EXPORT_ALPHA) that the
 *          same request without proj gives; the output is the single value
 *          C_M = sum_{delta, alpha} proj[delta][alpha] C(delta set; alpha set)
 *          per lane.  The final sum uses the projected list
 *          L_M(delta; z) = sum_alpha proj[delta][alpha] c_alpha(z), and only
 *          the quark parts z with a nonzero L_M for some delta are kept,
 *          together with the components of earlier stages they need.  Every
 *          sink set of the masks stays a spin part (the stage layout is
 *          spin parts x quark parts), so restrict sink_P / sink_N to prune
 *          spin parts.  The weights are read during the build only.         */
typedef struct {
    int all_components;
    uint32_t sink_P, sink_N;
    int n_alpha;
    const uint32_t *alpha;
    const double *proj;
    uint32_t sink_L;
    const uint32_t *alpha_L;
} mb_spin_request;

/* A smaller nucleus on the recursion path (Sec. 7): the nucleus of the
 * first stage+1 baryons of the path, whose correlators are read from stage
 * `stage` of the same recursion with their own list L, so that the stages
 * are shared.  Its sink sets are the spin parts of that stage (every subset
 * of the main request's sink base sets with the nucleus' baryon counts, in
 * the order of MB_EXPORT_SPIN for that stage).
 *   stage           0 <= stage < A - 1
 *   all_components  every source set (as in mb_spin_request), else
 *   alpha           [n_alpha][2] proton and neutron source sets             */
typedef struct {
    int stage;
    int all_components;
    int n_alpha;
    const uint32_t *alpha;
} mb_side_request;

typedef struct mb_term_list mb_term_list;

/* Builds the term list of a nucleus and spin request (Sec. 3-5, 7): the
 * antisymmetrised G of each baryon type, L on sorted index sets by
 * L^(n+1) = L^(n) . G (eq. recr_L) restricted to the requested source sets,
 * the final required components (requested sink sets times every index set
 * with a nonzero L), the required components of every earlier stage and the
 * operation list of every step, in the factorised form
 *     (quark split of the output) x (baryon-index split of the output),
 * which is the split of eq. antis_product_2 with its sign.  Host only,
 * deterministic, independent of any gauge configuration.
 * Returns MB_EPAULI when a species has more baryons than baryon indices or a
 * flavour more quarks than quark indices, MB_EUNSUPPORTED beyond 16 baryons
 * or 24 quark indices, MB_EINVAL for malformed requests.  On success *out
 * owns the list.                                                           */
int mb_build_term_list(const mb_nucleus *nuc, const mb_spin_request *req,
                       mb_term_list **out);

/* Same as mb_build_term_list but builds only the required-component sets
 * and counts (the memory-saving mode of Sec. 3): no operation tables, no
 * device image.  mb_term_list_counts works on the result.                  */
int mb_build_term_list_counts_only(const mb_nucleus *nuc, const mb_spin_request *req,
                                   mb_term_list **out);

/* mb_build_term_list with n_side smaller nuclei on the path (Sec. 7): every
 * stage a side request reads also keeps the quark parts its list L needs,
 * and the operations of the earlier steps grow accordingly (n_lambda counts
 * them once).  The contraction writes the side correlators after the main
 * output (see mb_contract_correlator).  MB_EUNSUPPORTED with a projection. */
int mb_build_term_list_path(const mb_nucleus *nuc, const mb_spin_request *req, int n_side,
                            const mb_side_request *side, mb_term_list **out);

void mb_term_list_free(mb_term_list *tl);

/* Term lists are built once per nucleus and request, independently of any
 * gauge configuration (Sec. 3, 7).  mb_term_list_save writes a host term
 * list (not its device image or launch tuning) to the file `path` in a
 * versioned binary format of this library, native byte order; MB_EINVAL if
 * the file cannot be written.  mb_term_list_load reads it back into a new
 * list, owned by the caller (upload it before contracting); MB_EINVAL for a
 * missing, truncated or foreign file, MB_EUNSUPPORTED for another format
 * version.  A loaded list exports and contracts exactly as the saved one.   */
int mb_term_list_save(const mb_term_list *tl, const char *path);
int mb_term_list_load(const char *path, mb_term_list **out);

#define MB_MAX_STAGES 16
#define MB_MAX_BATCH 65535     /* lanes per call */

/* Sizes of a term list.  Stage s (0-based) holds the components with the
 * first s+1 baryons of the path; step s (s >= 1) forms stage s from stage
 * s-1 and the block of baryon path[s].
 *   n_lambda        total operations (one complex multiply-add each; the
 *                   count the paper's tables report)
 *   n_lambda_step   operations of step s (entry 0 is 0)
 *   n_req           |required components| of stage s
 *   n_quark         distinct (u set, d set[, s set]) parts of stage s
 *   n_spin          distinct (proton set, neutron set[, Lambda set]) parts
 *                   of stage s
 *   n_L             nonzero entries of L over all requested source sets
 *   n_U             distinct quark parts with a nonzero L (final stage)
 *   n_delta, n_alpha  sink sets / source sets of the request (the output
 *                   rows / columns unless projected)
 *   n_psi, n_xi     D*N_s and 3*D*N_s
 *   device_bytes    size of the device image (0 in counts-only mode)
 *   projected       1 for a projected request (one output per lane), else 0
 *   n_LM            nonzero entries of the projected list L_M (0 if not
 *                   projected); n_L then counts the entries of c on the
 *                   kept quark parts
 *   n_side          side requests (smaller nuclei on the path)
 *   n_out           complex outputs per lane: main output and side outputs
 *   rel, n_src      the operators and sources of the nucleus
 *   n_Lambda        0 or 1 (the last stage then adds the Lambda: path entry
 *                   MB_LAMBDA)                                             */
typedef struct {
    int n_stages;
    int path[MB_MAX_STAGES];
    int64_t n_lambda;
    int64_t n_lambda_step[MB_MAX_STAGES];
    int64_t n_req[MB_MAX_STAGES];
    int64_t n_quark[MB_MAX_STAGES];
    int32_t n_spin[MB_MAX_STAGES];
    int64_t n_L;
    int64_t n_U;
    int32_t n_delta, n_alpha;
    int32_t n_psi, n_xi;
    int64_t device_bytes;
    int32_t projected;
    int64_t n_LM;
    int32_t n_side;
    int64_t n_out;
    int32_t rel, n_src;
    int32_t n_Lambda;
} mb_counts;

#define MB_PROTON 0    /* species numbers of mb_counts.path */
#define MB_NEUTRON 1
#define MB_LAMBDA 2

int mb_term_list_counts(const mb_term_list *tl, mb_counts *out);

/* Export of the term list for inspection and tests (host memory).  If buf is
 * NULL, *bytes receives the size; otherwise *bytes must be at least that
 * size.  `stage` selects the stage where relevant.
 *   MB_EXPORT_QUARK  uint32 [n_quark][2]: (u mask, d mask) in the stage's
 *                    order: ascending in (d, u) for a stage reached by adding
 *                    a proton (after the first), else ascending in (u, d)
 *   MB_EXPORT_SPIN   uint32 [n_spin][2]: (proton mask, neutron mask) in the
 *                    stage's order (proton rank major)
 *   MB_EXPORT_QSPLIT uint32 [n_quark][S][2] for stage >= 1: per output quark
 *                    part, per split: (quark part index in stage-1,
 *                    block quark index | sign bit 31 set for -1); the splits
 *                    of an output are ordered by the added baryon's single
 *                    quark index (d of a proton, u of a neutron), then by
 *                    the rank of its same-flavour pair
 *   MB_EXPORT_SSPLIT int32 [n_spin][k][3] for stage >= 1: per output spin
 *                    part, per split: (spin part index in stage-1, baryon
 *                    index psi of the added baryon, sign +1/-1)
 *   MB_EXPORT_COEF   int64 [n_alpha+1] row starts, then int64 [n_L] final
 *                    quark part indices, then int64 [n_L] values of L on
 *                    sorted sets (the coefficient c of the final sum)
 *   MB_EXPORT_DELTA  uint32 [n_delta][2] sink sets, MB_EXPORT_ALPHA uint32
 *                    [n_alpha][2] source sets (proton mask, neutron mask)
 *   MB_EXPORT_PROJ   projected lists only: int64 [n_delta+1] row starts,
 *                    int64 [n_LM] final quark part indices, double [n_LM]
 *                    values of L_M(delta; z)
 *   MB_EXPORT_SIDE   side request `stage` (its index, not a stage): int64
 *                    stage, int64 n_alpha, then uint32 [n_alpha][2] source
 *                    sets, then the coefficients as for MB_EXPORT_COEF with
 *                    quark part indices of that stage
 *   MB_EXPORT_QUARK_S  uint32 [n_quark]: the s mask of each quark part (0
 *                    before the Lambda's stage)
 *   MB_EXPORT_SPIN_L uint32 [n_spin]: the Lambda mask of each spin part (0
 *                    before the Lambda's stage)
 *   MB_EXPORT_DELTA_L, MB_EXPORT_ALPHA_L  uint32 [n_delta] / [n_alpha]: the
 *                    Lambda's sink / source set of each row / column
 * The block quark index of a proton split with u pair (a<b) and d index c is
 * (b*(b-1)/2 + a)*n_xi + c; of a neutron split with u index c and d pair
 * (a<b) it is c*(n_xi*(n_xi-1)/2) + b*(b-1)/2 + a; of the Lambda with s
 * index e, u index c and d index f it is (e*n_xi + c)*n_xi + f.  A Lambda
 * step's splits are ordered by the u index, then the d index.              */
#define MB_EXPORT_QUARK 1
#define MB_EXPORT_SPIN 2
#define MB_EXPORT_QSPLIT 3
#define MB_EXPORT_SSPLIT 4
#define MB_EXPORT_COEF 5
#define MB_EXPORT_DELTA 6
#define MB_EXPORT_ALPHA 7
#define MB_EXPORT_PROJ 8
#define MB_EXPORT_SIDE 9
#define MB_EXPORT_QUARK_S 10
#define MB_EXPORT_SPIN_L 11
#define MB_EXPORT_DELTA_L 12
#define MB_EXPORT_ALPHA_L 13
int mb_term_list_export(const mb_term_list *tl, int what, int stage, void *buf,
                        size_t *bytes);

/* Launch tuning of recursion step `step` (1..A-1; -1 = every step), chosen by
 * an autotuner; results do not depend on it (up to the order of sums).
 *   MB_TUNE_PASS_GROUP  passthrough spin parts per thread: 0 = automatic
 *                       (3, 2 or 1, the largest that divides their count),
 *                       or 1, 2, 3, 6 (must divide the count; the LDS kernel
 *                       takes 6 as automatic)
 *   MB_TUNE_LDS_BYTES   LDS reserved per workgroup (0..65536), which caps the
 *                       number of resident workgroups per CU (fewer operands
 *                       in flight per L2)
 *   MB_TUNE_LANE_TILE   lanes per wavefront, 64 (default) or 16 (four
 *                       sub-waves share the quark splits of an output)
 *   MB_TUNE_UNROLL      splits whose loads a wavefront of the direct kernel
 *                       issues together: 1 or 2 (0 = automatic)
 *   MB_TUNE_GROUP       outputs per wavefront: 1 (default), or 2 or 4 with
 *                       64 lanes, where neighbouring outputs share the block
 *                       rows they read at the same split position (applies
 *                       with passthrough groups up to 3)
 *   MB_TUNE_PAIRED      1 (default): the float stage this step reads is stored
 *                       with neighbouring spin parts of a lane together
 *                       when every thread of the step takes both (one
 *                       16-byte load instead of two); 0: plain layout
 *   MB_TUNE_TWO_PHASE   0 (default) or 1 (direct kernel only): the step runs
 *                       in two parts.  Part A computes, for every output and
 *                       every single-flavour index c of it (d of a proton,
 *                       u of a neutron), the sum over the splits whose added
 *                       baryon takes c -- all of them read previous-stage
 *                       parts with the same single-flavour set, and part A
 *                       runs those work items together, so that the parts
 *                       they read stay in L2 -- and writes it as a partial;
 *                       part B adds the partials of every output.  The
 *                       contraction workspace then holds the partials of
 *                       the largest such step (query it after tuning).
 *   MB_TUNE_KERNEL      0 (default): every thread gathers its block entries
 *                       from global memory; 1: the block rows of one single
 *                       quark index at a time are staged in LDS per
 *                       workgroup of 16 lanes x 16 outputs (lane tile and
 *                       LDS bytes are then fixed; up to 12 quark indices)
 * Steps whose species has more than four sink indices (three sources) run
 * the direct kernel with one passthrough part per thread and no output
 * grouping: other kernel, passthrough-group or grouping settings there make
 * the contraction return MB_EUNSUPPORTED before any launch.
 * With step 0 (or -1):
 *   MB_TUNE_BLOCKS      the site sums of mb_make_blocks: 0 (default) on the
 *                       matrix cores where the shape has that kernel (every
 *                       shape up to 12 quark indices), else on the vector
 *                       units; 1 matrix cores (MB_EUNSUPPORTED beyond 12
 *                       quark indices); 2 vector units, register-tiled
 * Returns MB_EINVAL for an unknown item, step or value.                      */
#define MB_TUNE_PASS_GROUP 1
#define MB_TUNE_LDS_BYTES 2
#define MB_TUNE_LANE_TILE 3
#define MB_TUNE_KERNEL 4
#define MB_TUNE_UNROLL 5
#define MB_TUNE_GROUP 6
#define MB_TUNE_PAIRED 7
#define MB_TUNE_TWO_PHASE 8
#define MB_TUNE_BLOCKS 9
int mb_term_list_tune(mb_term_list *tl, int step, int what, int value);

/* Copies the operation tables to device memory `dev` (caller-owned, at least
 * counts.device_bytes, 256-byte aligned) and binds the term list to it; the
 * buffer must stay alive while the term list is used on the device.  A term
 * list may be bound to one buffer at a time (a later call rebinds it).
 * Synchronous with respect to the host copy (the host tables may be freed
 * with the term list afterwards).                                          */
int mb_term_list_upload(mb_term_list *tl, void *dev, size_t bytes, void *stream);

/* One batch of independent (problem, timeslice) units ("lanes").
 *   batch      B, number of lanes, 1..MB_MAX_BATCH (MB_EUNSUPPORTED above;
 *              larger sets of lanes are cut into several calls)
 *   V          sink sites per timeslice
 *   in_dtype   MB_C64 or MB_C128, element type of the propagators
 *   precision  MB_FP64, MB_MIXED or MB_MIXED_F32B
 *   prop_u, prop_d  device, [B][V][n_src][12][12] complex of in_dtype:
 *              element [b][x][s][row][col] = S(x)[(spin,colour) row at the
 *              sink; source spin-colour col of source s]; prop_d may equal
 *              prop_u (isospin limit: one diquark, one block serves both
 *              species).
 *   sink_w     device, complex double [n_src][V]: sink function s' at site
 *              x (Sec. 2, 6); NULL means s(x) = 1 for every sink function.
 *   scale_exp  device, int32 [B]: the propagators of lane b are read
 *              multiplied by 2^scale_exp[b] (exact); NULL means 0.
 *   prop_s     device, the strange propagator in the layout of prop_u, for
 *              a term list with a Lambda (MB_EINVAL if NULL there); ignored
 *              otherwise.  It may equal prop_u or prop_d.                   */
typedef struct {
    int64_t batch;
    int64_t V;
    int in_dtype;
    int precision;
    const void *prop_u;
    const void *prop_d;
    const double *sink_w;
    const int32_t *scale_exp;
    const void *prop_s;
} mb_problem;

/* Device buffer sizes for one batch:
 *   blocks_bytes     output of mb_make_blocks / input of the contraction
 *   blocks_ws_bytes  workspace of mb_make_blocks (site-chunk partial sums)
 *   contract_ws_bytes workspace of mb_contract_correlator (two stages of F;
 *                    for a projected term list also the per-sink-set sums;
 *                    with MB_TUNE_TWO_PHASE the partials of the largest
 *                    two-phase step, so the size depends on the tuning)   */
int mb_workspace_query(const mb_term_list *tl, const mb_problem *p,
                       size_t *blocks_bytes, size_t *blocks_ws_bytes,
                       size_t *contract_ws_bytes);

/* Baryon blocks (Sec. 2; Sec. 6 with one sink function per source index)
 *   f_B(psi; xi1, xi2, xi3) = sum_x s_{s'(psi)}(x) eps_abc
 *        (Gamma_1)_{alpha(psi) beta} (Gamma_2)_{gamma delta}
 *        S_q1[(beta,a), xi1] S_q2[(gamma,b), xi2] S_q3[(delta,c), xi3]
 * for the proton (u,u,d) and neutron (d,u,d), antisymmetrised without
 * normalisation in the two same-flavour slots (Sec. 4), for every lane.
 * The sum over sites runs in double precision and the blocks are stored in
 * double in every precision mode (MB_MIXED_F32B adds float copies).
 * With a Lambda also f_L of (q1, q2, q3) = (s, u, d), which has no two
 * slots of one flavour and is stored as it is.
 * Output layout (complex double in every precision mode): proton block
 * [block quark index][lane / 16][psi][lane % 16] followed by the neutron
 * block (and the Lambda block, n_xi^3 block quark indices), lanes padded to
 * a multiple of 64, then int32 e[lane] (padded lanes included): the blocks
 * of a lane are stored multiplied by 2^-e[lane] (exact), e chosen so that
 * their largest real or imaginary part lies in [1/2, 1) (e = 0 for an
 * all-zero lane).  Products of many blocks then stay near 1 in float stage
 * storage whatever the size of the propagators; the final sum multiplies by
 * 2^(A e).  With MB_MIXED_F32B the exponents are padded to a multiple of 256
 * bytes and followed by the scaled block entries again as complex float,
 * same layout and order, each rounded to nearest.                          */
int mb_make_blocks(const mb_term_list *tl, const mb_problem *p, void *blocks,
                   size_t blocks_bytes, void *ws, size_t ws_bytes, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): exactly
 * mb_make_blocks -- same kernels, same chunking, bit-identical blocks --
 * with the site-chunk partial sums in a fixed device array of
 * MB_NOALLOC_SCRATCH_BYTES that the library holds on every GPU it runs on
 * until the process ends, instead of a workspace argument.  The caller
 * still passes the propagators and the blocks buffer.  Sizes beyond the
 * array (mb_workspace_query's blocks_ws_bytes above
 * MB_NOALLOC_SCRATCH_BYTES) fail with MB_ENOWORKSPACE before anything is
 * launched.  No allocating call is made.  Every call on one GPU shares that
 * GPU's array: calls that overlap on one GPU (different streams without
 * ordering, other host threads) race and must be serialised by the caller.
 * Nothing in the array needs to start at zero.                             */
#define MB_NOALLOC_SCRATCH_BYTES (64u << 20)
int mb_make_blocks_noalloc(const mb_term_list *tl, const mb_problem *p, void *blocks,
                           size_t blocks_bytes, void *stream);

/* Correlators from blocks: the recursion of eq. recr_F over the operation
 * lists, then C(delta; alpha) = sum_z F_-(delta; z) L(alpha; z) / (n_P! n_N!)
 * (eq. C_final with the sum over sorted index sets), the final sum in double.
 *   corr_out  device, complex double [B][n_delta][n_alpha]; for a projected
 *             term list [B]: C_M = sum_z F_-(delta; z) L_M(delta; z) /
 *             (n_P! n_N!) summed over delta (eq. CM_final), the sum over
 *             delta in a fixed order.  Side requests follow in order, each
 *             [B][n_spin of its stage][its n_alpha]; a side nucleus of A_i
 *             baryons carries the exponent 3*A_i*scale_exp[b] (exp_out holds
 *             the main nucleus' 3*A*scale_exp[b])
 *   exp_out   device, int32 [B] or NULL: 3*A*scale_exp[b], so that the
 *             correlator of the unscaled propagators is corr_out * 2^-exp_out
 *   err_out   device, double [B][n_out][2] or NULL: for every output of
 *             corr_out (same order, main then side outputs), an a-posteriori
 *             estimate of how far the MB_MIXED (or MB_MIXED_F32B) result
 *             lies from the MB_FP64 result for the same blocks, in the units
 *             of corr_out:
 *               [0]  sigma: standard deviation of that difference when the
 *                    rounding errors of the float stage storage (and of the
 *                    float block copies with MB_MIXED_F32B) are taken as
 *                    independent (each stored real rounded to nearest, error
 *                    uniform on half an ulp each side), propagated through
 *                    every step of eq. recr_F and the sum of eq. C_final.
 *                    One rounded block copy enters many splits, whose
 *                    errors then add coherently: with MB_MIXED_F32B sigma
 *                    can fall well short of the deviation (by up to 7x
 *                    measured on one-component 8Be outputs);
 *               [1]  bound: the same propagation with absolute values, a
 *                    bound to first order in u = 2^-24 (it ignores u^2 terms
 *                    and the double-precision rounding common to both paths).
 *             The propagation runs extra kernels over two error stages (one
 *             float pair per component) and needs mb_workspace_query_err
 *             more workspace bytes after contract_ws_bytes.  MB_FP64 writes
 *             zeros (no extra workspace).  The correlators themselves do not
 *             change.
 * The term list must be uploaded.                                           */
int mb_contract_correlator(const mb_term_list *tl, const mb_problem *p,
                           const void *blocks, size_t blocks_bytes, double *corr_out,
                           int32_t *exp_out, double *err_out, void *ws, size_t ws_bytes,
                           void *stream);

/* Additional contraction workspace (bytes, after contract_ws_bytes) that
 * mb_contract_correlator needs with err_out != NULL: two error stages of
 * 8 bytes per component and lane, plus per-sink-set estimates of a projected
 * list; 0 for MB_FP64.                                                     */
int mb_workspace_query_err(const mb_term_list *tl, const mb_problem *p, size_t *err_ws_bytes);

/* One part of mb_contract_correlator, for timing the parts separately:
 * step 0 copies the first baryon's block into stage 0, step s in 1..A-1 is
 * recursion step s (eq. recr_F), step A is the final sum (corr_out, exp_out
 * as above; ignored for the other steps).  Running steps 0..A in order on
 * one stream is exactly mb_contract_correlator with err_out = NULL; the
 * workspace carries the stages between the calls.                           */
int mb_contract_step(const mb_term_list *tl, const mb_problem *p, const void *blocks,
                     size_t blocks_bytes, int step, double *corr_out, int32_t *exp_out, void *ws,
                     size_t ws_bytes, void *stream);

/* ---- Batched runs of uneven work (many nuclei, volumes, lanes) ----------
 * Lanes of different nuclei or volumes cannot share a launch, so a batch is
 * a list of items, each one (term list, problem) with its own buffers, run
 * as one captured HIP graph: the items are spread over n_branches
 * concurrent branches (forked from and joined back into the launch stream),
 * every branch running its items one after the other (blocks, then every
 * contraction step).  Small items then overlap with large ones.  Every
 * computation is that of mb_make_blocks + mb_contract_correlator (Sec. 2,
 * eq. recr_F, eq. C_final); only the order of independent launches differs. */
typedef struct {
    const mb_term_list *tl;   /* uploaded; its launch tuning is read at capture */
    mb_problem prob;
    void *blocks;             /* device buffers sized by mb_workspace_query  */
    size_t blocks_bytes;
    void *blocks_ws;
    size_t blocks_ws_bytes;
    void *contract_ws;
    size_t contract_ws_bytes;
    double *corr_out;         /* as for mb_contract_correlator               */
    int32_t *exp_out;         /* may be NULL                                 */
    int branch;               /* 0..n_branches-1                             */
} mb_batch_item;

/* Host-side scheduler: estimates the cost of every item (algorithmic flops
 * of its blocks and of its recursion, over its lanes; written to cost_out
 * if not NULL) and assigns the items to branches longest first, each to the
 * branch with the least work so far (branch_out[n_items]).  Items on one
 * branch run one after the other, so they may share their blocks and
 * workspace buffers; items on different branches may not.                 */
int mb_batch_plan(const mb_term_list *const *tls, const mb_problem *probs, int n_items,
                  int n_branches, int *branch_out, double *cost_out);

typedef struct mb_batch mb_batch;

/* Validates every item (as the single calls would), checks that no two
 * items on different branches share a blocks or workspace buffer, and
 * records the launches of all items into a HIP graph (on streams of its own,
 * default priority) which it instantiates.  Items on one branch run in the
 * order given.  Nothing runs until mb_batch_launch.  The buffers and term
 * lists must stay alive and keep their addresses while the batch exists;
 * their contents are read at launch time.  MB_EHIP if capture fails;
 * MB_EUNSUPPORTED for a projected term list.                                */
int mb_batch_create(const mb_batch_item *items, int n_items, int n_branches, mb_batch **out);

/* Launches the whole batch on `stream` (one graph launch).  Launches of one
 * batch on streams that are not ordered with each other race.              */
int mb_batch_launch(mb_batch *b, void *stream);

/* Number of kernel nodes of the recorded graph. */
int mb_batch_kernel_count(const mb_batch *b, int64_t *out);

void mb_batch_free(mb_batch *b);

/* Message of the last failed call on this thread ("" if none). */
const char *mb_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* MBCONTRACT_H */
