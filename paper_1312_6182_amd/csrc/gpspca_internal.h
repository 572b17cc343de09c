// Internal declarations of the gfx950 GP-SPCA library: device control block,
// kernel parameter blocks and the host-side launchers of every kernel.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <string>

#include "../../include/gpspca.h"

namespace gpspca {

constexpr int kMaxM = GPSPCA_MAX_M;
// rows per workgroup of the single-unit partial reduction (one Gram partial each)
constexpr int kRm1Rows = 32;

// Device-resident state of one solve.  Written only by single-workgroup
// kernels (stop test / projection) and by the control reset kernel.
struct Ctrl {
    int k;                 // index of the next pass
    int done;              // 1 once the stopping rule fired (or an error)
    int status;            // GPSPCA_* status of the solve
    int n_iter;            // passes made
    int ndead;             // dead components at the last retraction
    int degenerate_seen;   // some retraction completed dead components / F = 0
    int max_iter;
    int warm;              // the previous retraction's eigenvectors may seed the next
    int nact;              // columns with any active component in the current pass (the
                           // correlation kernels add to it; the stop kernel clears it)
    double tol;
    double last_F;
};

// Problem constants passed by value to every pass kernel.
struct PassParams {
    const float* A;        // column-major p x n FP32 (dtype F32)
    const uint16_t* Abf;   // bf16 storage (dtype BF16)
    const uint8_t* Af8;    // e4m3 storage (dtype F8E4M3)
    const float* scale;    // per-column scales or nullptr
    int64_t lda;
    int64_t n;
    int p;
    int ldx;               // leading dimension of the internal X buffers (multiple of 4)
    int m;
    int l0;                // 1 for the l0 (hard threshold) forms
    double gamma;
    float muf[kMaxM];      // mu_j in FP32 (for the back-projection weights)
    double mu[kMaxM];      // mu_j in FP64 (for the threshold)
    double gam[kMaxM];     // gamma of component j (all equal, except on a gamma path)
    // frozen-support passes (refinement): only the columns list[0 .. *nlist-1]
    // are visited, and s_ij = 0 wherever bit (i, j) of mask is clear
    const int* list;       // ascending column indices, or nullptr (all columns)
    const int* nlist;      // device count of list entries
    const uint32_t* mask;  // mask[j * mask_words + i / 32] bit i % 32, or nullptr
    int64_t mask_words;
    int* nact;             // &Ctrl::nact: active-column count of the pass
};

// Balanced partition of the FP32 matrix-core correlation: every wave owns q
// whole tiles of 16 columns, and the rem leftover tiles are split by rows over
// all waves; xpart holds the partial sums of those splits (2 x 256 floats per
// wave and component group), and the objective partials have nwp = waves + rem
// slots per component.
struct BalArgs {
    float* xpart;
    int q, rem, nwp;
};

// A configuration of the correlation kernel: the autotuner's unit of choice.
enum TuneKernel { kTuneDefault = 0, kTuneMfma = 1, kTuneVx = 2, kTuneValu = 3, kTuneRd = 4,
                  kTuneWg = 5, kTuneRd128 = 6, kTuneX3 = 7, kTuneQw = 8 };
struct Tune {
    int kernel;            // TuneKernel
    int stages;            // LDS stages (matrix-core kernels), 0 = default
    int waves;             // workgroups per CU (matrix-core kernels), 0 = default
};

// Layout of the caller's workspace for one solve (byte offsets).
struct Plan {
    // problem
    int64_t p, n, lda;
    int m, form, l0, max_iter;
    int ldx;
    int mpad;              // columns of the internal X buffers (zero padded to the group size)
    // kernel choice
    int fused_m1;          // 1: single fused pass kernel (m == 1), else corr + back-projection
    int m1_threads, m1_kq, m1_grid;
    int corr_M, corr_grid; // corr kernel: padded component count and grid
    int bp_kq, bp_rb, bp_cr; // back-projection: quads per thread, row blocks, column ranges
    int bp_thr;            // column ranges with >= bp_thr/1024 active columns are back-projected
                           // densely on the matrix cores (> 1024: never)
    int npart;             // number of G partials
    int nwave_part;        // objective partial slots per component (fpart[j * nwave_part + w])
    int red_split;         // split of the partial reduction
    int gram_rows, gram_grid;
    int fused_gram;        // m <= 16: partial reduction and Gram in one kernel (64-row blocks)
    int gram_blocks;       // number of Gram partials of a pass
    size_t xil_bytes;      // bytes of each interleaved copy of X (0: none)
    int fin_grid;
    int topm_grid;
    int vec4;              // float4 loads of A are legal
    int dtype;             // storage of A (GPSPCA_F32 | BF16 | F8E4M3)
    int use_q;             // 16/8-bit storage: bfloat16 matrix-core correlation
    int use_qw;            // ... by four-wave workgroups that share each X stage
    int restricted;        // frozen-support passes over a column list (VALU correlation)
    int use_mfma;          // block correlation on the matrix cores (LDS DMA staging)
    int bal, bal_q, bal_rem; // ... balanced partition: q whole tiles per wave, rem leftover
                           // tiles split by rows (k_corr_bal_fix finishes them)
    int mfma_stages;       // stages in flight of the matrix-core kernels (FP32 and 16/8-bit)
    int waves_per_cu;      // resident matrix-core workgroups per CU
    int use_rd;            // matrix-core correlation with register-direct operand loads
    int use_x3;            // FP32 correlation on the bfloat16 matrix cores (three-part split)
    int use_wg;            // matrix-core correlation, four waves sharing X per workgroup
    int rd_depth;          // its software-pipeline depth (stages of 32 rows)
    int rd128;             // register-direct loads of whole 128-byte lines (8 columns each)
    int use_vx;            // block correlation with X held in registers (m <= 8, p <= 10240)
    int vx_threads, vx_kq;
    int use_mv;            // block correlation on the matrix cores, A staged through registers
    int path;              // gamma path: independent single-unit columns (normalize, per-column stop)
    const double* defl_q;  // deflated component: basis of the earlier components (p x defl_k, FP64)
    int exact;             // block L1 from its original form: F = sum_j ||s_j||, G column j / ||s_j||
    int defl_k;            // ... and their count (0: no deflation)
    // workspace offsets (bytes)
    size_t o_ctrl, o_trace, o_x0, o_x1, o_s, o_act, o_gpart, o_touched, o_fpart, o_nnzpart,
        o_l1, o_g64, o_gram, o_coef, o_norms, o_cand_v, o_cand_i, o_idx, o_fin, o_invn, o_fcomp,
        o_pstate, o_list, o_xil0, o_xil1, o_fsum, o_xpart;
    size_t total;
};

// ---- launchers (defined in the .hip files) --------------------------------
// pass kernels (k_pass.hip)
hipError_t launch_pass_m1(const Plan& pl, const PassParams& pp, const float* x, float* S,
                          float* gpart, double* fpart, int* nnzpart, const Ctrl* ctrl,
                          hipStream_t st);
hipError_t launch_corr(const Plan& pl, const PassParams& pp, const float* X, float* S,
                       uint8_t* act, double* fpart, int* nnzpart, const Ctrl* ctrl,
                       hipStream_t st);
hipError_t launch_corr_vx(const Plan& pl, const PassParams& pp, const float* X, float* S,
                          uint8_t* act, double* fpart, int* nnzpart, const Ctrl* ctrl,
                          hipStream_t st);
hipError_t launch_corr_wg(const Plan& pl, const PassParams& pp, const float* X, const float* Xil,
                          float* S, uint8_t* act, double* fpart, int* nnzpart, const Ctrl* ctrl,
                          hipStream_t st);
hipError_t launch_corr_rd(const Plan& pl, const PassParams& pp, const float* X, const float* Xil,
                          float* S, uint8_t* act, double* fpart, int* nnzpart, const Ctrl* ctrl,
                          hipStream_t st);
hipError_t launch_corr_x3(const Plan& pl, const PassParams& pp, const float* X, const float* Xil,
                          float* S, uint8_t* act, double* fpart, int* nnzpart, const Ctrl* ctrl,
                          hipStream_t st);
int corr_mfma_blocks_per_cu(int m, int stages);
hipError_t launch_corr_mv(const Plan& pl, const PassParams& pp, const float* X, float* S,
                          uint8_t* act, double* fpart, int* nnzpart, const Ctrl* ctrl,
                          hipStream_t st);
// Xil: X in the row-quad-interleaved layout of launch_x_interleave.
// Kernel timing: while the solve driver times a launch of the pass's
// correlation kernel, these events are set and that launch records them at its
// own start and end (hipExtLaunchKernelGGL puts them on the dispatch itself,
// so no separate event packets sit around the kernel).  Null otherwise.
struct KernelEvents {
    hipEvent_t start = nullptr, stop = nullptr;
};
extern thread_local KernelEvents g_kev;

// Launch of a correlation kernel that records g_kev when it is set.
#define GPSPCA_LAUNCH_TIMED(KERNEL, GRID, BLOCK, SHM, STREAM, ...)                               \
    do {                                                                                         \
        if (::gpspca::g_kev.start)                                                               \
            hipExtLaunchKernelGGL(KERNEL, GRID, BLOCK, SHM, STREAM, ::gpspca::g_kev.start,       \
                                  ::gpspca::g_kev.stop, 0, __VA_ARGS__);                        \
        else                                                                                     \
            hipLaunchKernelGGL(KERNEL, GRID, BLOCK, SHM, STREAM, __VA_ARGS__);                   \
    } while (0)

hipError_t launch_corr_mfma(const Plan& pl, const PassParams& pp, const float* X, const float* Xil,
                            float* S, uint8_t* act, double* fpart, int* nnzpart, float* xpart,
                            const Ctrl* ctrl, hipStream_t st);
hipError_t launch_backproj(const Plan& pl, const PassParams& pp, const float* S,
                           const uint8_t* act, float* gpart, int* touched, const Ctrl* ctrl,
                           hipStream_t st);
hipError_t launch_colnorm(const PassParams& pp, int dtype, double* norms, int grid,
                          hipStream_t st);
hipError_t launch_mask_list(const uint32_t* mask, int64_t words, int m, int64_t n, int* list,
                            int* nlist, hipStream_t st);
// reduced-precision storage (k_quant.hip)
hipError_t launch_quantize(const float* A, int64_t lda, int p, int64_t n, int to, void* out,
                           int64_t ldq, float* scale, hipStream_t st);
int corr_q_stages(int dtype, int m, int want);
int corr_q_blocks_per_cu(int dtype, int m, int stages);
hipError_t launch_corr_q(const Plan& pl, const PassParams& pp, const float* X, const float* Xil,
                         float* S,
                         uint8_t* act, double* fpart, int* nnzpart, const Ctrl* ctrl,
                         hipStream_t st);
hipError_t launch_corr_qw(const Plan& pl, const PassParams& pp, const float* X, const float* Xil,
                         float* S,
                         uint8_t* act, double* fpart, int* nnzpart, const Ctrl* ctrl,
                         hipStream_t st);

// reductions, retraction, stop test (k_reduce.hip)
hipError_t launch_fill_zero(void* ptr, size_t bytes, hipStream_t st);
hipError_t launch_ctrl_reset(Ctrl* ctrl, int max_iter, double tol, hipStream_t st);
// Buffers that the start of a solve clears (whole 4-byte words).
struct StartZero {
    uint32_t* ptr[8];
    size_t words[8];
    int n;
};
// One launch: control block reset, the StartZero buffers cleared, and, with X0
// given (device p x m, leading dim ldx0), g64 = X0 in FP64.
hipError_t launch_start(Ctrl* ctrl, int max_iter, double tol, const StartZero& z, int m, int p,
                        const float* X0, int ldx0, double* g64, hipStream_t st);
hipError_t launch_reduce_partials(const Plan& pl, const float* gpart, const int* touched,
                                  double* l1, const Ctrl* ctrl, hipStream_t st);
hipError_t launch_gram(const Plan& pl, const double* l1, int nsplit, const float* X,
                       int with_x, double* g64, double* gram, const Ctrl* ctrl,
                       hipStream_t st);
// m = 1 after the fused pass: g64 = the sum of the npart partials, and the
// cdiv(p, kRm1Rows) Gram partials of ||g||^2 (entry 0 of each 3-entry block).
hipError_t launch_reduce_m1(const Plan& pl, const float* gpart, double* g64, double* gram,
                            const Ctrl* ctrl, hipStream_t st);
// Xn (m = 1 only, may be NULL): write x_{k+1} = g / ||g|| from g64 as well.
hipError_t launch_stop(const Plan& pl, const double* fpart, const int* nnzpart,
                       const double* gram, double* trace, double* coef, double* fcomp,
                       double* vprev, const double* g64, float* Xn, double* fsum, Ctrl* ctrl,
                       hipStream_t st);
hipError_t launch_reduce_gram(const Plan& pl, const float* gpart, const int* touched,
                              const float* X, int with_x, double* g64, double* gram,
                              const Ctrl* ctrl, hipStream_t st);
// fsum (may be NULL): also sum the objective and support-size partials per
// component into fsum[0..m) and fsum[m..2m).
hipError_t launch_gram_sum(const Plan& pl, int nent, int ngram, const double* gram, double* coef,
                           const Ctrl* ctrl, hipStream_t st, const double* fpart = nullptr,
                           const int* nnzpart = nullptr, double* fsum = nullptr);
// gamma path: per-column objective, trace, stopping and normalization
struct PathState {
    int frozen;            // 1 once this column's stopping rule fired
    int n_iter;            // passes of this column
    int status;            // GPSPCA_* status of this column
    int degenerate;        // F = 0 was reached
    double last_F;
};
hipError_t launch_stop_path(const Plan& pl, const double* fpart, const int* nnzpart,
                            const double* gram, double* trace, double* coef, double* fcomp,
                            PathState* ps, Ctrl* ctrl, hipStream_t st);
hipError_t launch_bcast_col0(const Plan& pl, float* X, hipStream_t st);
hipError_t launch_project_diag(const Plan& pl, const double* gram, double* coef, Ctrl* ctrl,
                               hipStream_t st);
hipError_t launch_project(const Plan& pl, const double* gram, double* coef, Ctrl* ctrl,
                          hipStream_t st);
// X (component-major, leading dim ldx) -> Xil: blocks of 16 components, each
// block row-quad-major, Xil[((b * ldx/4 + q) * 16 + c) * 4 + e] = X[16b + c][4q + e],
// so that the matrix-core kernels stage 4 row quads x 16 components of X with
// one contiguous 1 KB read.
hipError_t launch_x_interleave(const Plan& pl, const float* X, float* Xil, hipStream_t st);
// Xil_n (may be NULL): also write X_{k+1} in the interleaved layout.
hipError_t launch_apply(const Plan& pl, const double* g64, const float* Xk, const double* coef,
                        float* Xn, float* Xil_n, const Ctrl* ctrl, hipStream_t st);
hipError_t launch_load_g64(const Plan& pl, const float* X0, int ldx0, double* g64,
                           hipStream_t st);

// init and finalize (k_init_fin.hip)
hipError_t launch_topm(const Plan& pl, const double* norms, double* cand_v, int64_t* cand_i,
                       int64_t* idx, hipStream_t st);
hipError_t launch_gather(const Plan& pl, const PassParams& pp, const int64_t* idx, double* g64,
                         hipStream_t st);
hipError_t launch_finalize(const Plan& pl, const float* S, double* fin, double* invn, float* Z,
                           uint32_t* support, hipStream_t st);
hipError_t launch_copy_x(const Plan& pl, const float* Xint, float* Xout, hipStream_t st);
// X_{n_iter - 1} (Xa when n_iter is odd, Xb when even, read from ctrl on the
// device) -> Xout (leading dim p)
hipError_t launch_copy_x_last(const Plan& pl, const float* Xa, const float* Xb, const Ctrl* ctrl,
                              float* Xout, hipStream_t st);

// Offsets of the coefficient block (doubles) written by the stop / projection kernels.
inline size_t coef_omega(int m) { return 0; }
inline size_t coef_psi(int m) { return (size_t)m * m; }

// Deflated single-unit components: x <- P x / ||P x|| with P = I - Q Q^T,
// the column norms of P A, and Q[:, k] <- x.
hipError_t launch_deflate(int p, int k, const double* Q, const double* x, float* out,
                          double* scratch, const Ctrl* ctrl, hipStream_t st);
hipError_t launch_defl_norms(const float* A, int64_t lda, int p, int64_t n, int k,
                             const double* Q, double* norms, int grid, hipStream_t st);
hipError_t launch_append_basis(int p, const float* x, double* q, hipStream_t st);

// ---- host driver (gpspca_abi.cpp), shared with the server (serve.cpp) ----

int fail(int code, const std::string& msg);
int check_problem(const gpspca_matrix* A, int form, int m, double gamma, const double* mu);
int solve_core(const gpspca_matrix* A, int form, int m, double gamma, const double* mu,
               const double* gammas, int path, const uint32_t* mask, const float* X0,
               double tol, int max_iter, void* workspace, size_t ws_bytes, hipStream_t st,
               float* X, float* Z, uint32_t* support, double* obj_trace, int* n_iter,
               int* status_out, const double* norms_in, int multistart = 0,
               const double* defl_q = nullptr, int defl_k = 0, int exact = 0,
               int noalloc = 0);

}  // namespace gpspca
