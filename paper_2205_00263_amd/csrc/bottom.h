// Fused bottom-of-pass kernel (first convolution + ReLU layer 0): arguments and launcher.
#pragma once

#include "kernels.h"

namespace mnb {

struct BottomArgs {
    int mode;        // 0: intermediate rows (update l/u), 1: spec rows (lb + best), 2: lb only
    float margin;    // rounding margin factor: 2^-20 for spec rows, 0 for intermediate rows
    int src_mode;    // 0: rows read from A; 1: rows built from the objective convolution's filter
    const float* A;  // [M, d1] coefficients on the output of ReLU layer 0 (src_mode 0)
    const float* c;  // [M] (src_mode 0)
    const float* cpart; int ldcp, ncp;
    // objective convolution (src_mode 1): its input is the output of ReLU layer 0
    const float* Wobj; const float* bias_obj;
    int oCi, oHi, oWi, oCo, oHo, oWo, ok, os, op;
    const RowDesc* rows; const InstDesc* inst; const int32_t* slots; const int32_t* qid;
    int M, d1, d0;
    // first convolution: input (Ci,Hi,Wi) -> ReLU layer 0 input (Co,Ho,Wo)
    int Ci, Hi, Wi, Co, Ho, Wo, k, s, p;
    const float* W1; const float* b1; const float* bias1;
    const float* l; const float* u; const int8_t* S; long ld_state;
    const float* alpha; const float* beta; long ld_param; int n_sets;
    const float* v; const float* vhat; const float* gp;
    const float* lo; const float* hi;
    // outputs
    float* lw; float* uw; int state_off_obj;
    float* lb_out; float* best; uint8_t* improved; uint8_t* xbits;
    int adjoint;
    float* Gout; float* Ap_out;
    float* d_alpha; float* d_beta; long ldg;
    float* gsum_hat; float* gsum_out;
    // row chunks: block b handles rows [cr0[b], cr1[b]) of instance cinst[b]; gradient
    // partials [n_chunk][3][d1] are summed per instance in chunk order
    const int* cinst; const int* cr0; const int* cr1; int n_chunk;
    const int* ichunk0; const int* ichunk1;   // [n_inst] chunk range of each instance
    float* part;
    int box_lds;     // set by launch_bottom: the query's box is staged in LDS
};

bool bottom_supported(int d1, int d0, int n_weights);
void launch_bottom(const BottomArgs& a, int n_inst, hipStream_t st);
// MFMA variant for first-layer convolutions into 16 channels with at most 32 taps per channel
// (launch_bottom dispatches to it)
bool bottom_mf_supported(int Co, int Ci, int k, int s, int Ho, int Wo, int d0, int d1, bool mnc);
void launch_bottom_mf(const BottomArgs& a, hipStream_t st);
// instance gradients from the chunk partials (after launch_bottom with adjoint)
void launch_bottom_reduce(const BottomArgs& a, int n_inst, hipStream_t st);
constexpr int BOTTOM_CHUNK_ROWS = 32;

// Window-sparse variant for intermediate rows whose objective is ReLU layer 1 fed by a
// convolution of ReLU layer 0 (no MNC): one workgroup per (instance, window position).
// A row of a window: pass row index r (~r for an upper-bound row), objective neuron,
// signed objective bias and the objective neuron's bound before the pass (mode 0).
struct WinEnt {
    int32_t r, j;
    float cb, old;
};
struct WinArgs {
    int mode;        // 0: update l/u of the objective layer, 2: lb only
    const RowDesc* rows; const InstDesc* inst; const int32_t* qid;
    int d1, d0;
    // first convolution: input (Ci,Hi,Wi) -> ReLU layer 0 input (C1,Ho,Wo)
    int Ci, Hi, Wi, C1, Ho, Wo, k, s, p;
    const float* W1; const float* b1;
    // objective convolution on the output of ReLU layer 0
    int oCi, oHi, oWi, oCo, oHo, oWo, ok, os, op;
    const float* Wobj; const float* bobj;   // bobj: bias per objective neuron
    const float* l; const float* u; const int8_t* S; long ld_state;
    const float* alpha; const float* beta; long ld_param; int n_sets;
    const float* lo; const float* hi;
    float* lw; float* uw; int state_off_obj;
    float* lb_out;
    int adjoint;
    // per instance: A_s [n_inst][d0] and {sum min(A_s lo, A_s hi), sum |A_s| max(|lo|,|hi|), S beta . b, 0}
    float* asplit; float* scal;
    // per (instance, window): alpha partials [E], x* sums minus n x*_s [Ci IH IH], row counts
    float* part_a; float* part_x; int* part_n;
    float* d_alpha; float* d_beta; long ldg;
    // per instance and window position: first entry in win_ent ([n_inst][nwin + 1]); the
    // entries of a window are its rows in pass order (built by launch_bottom_win)
    int* win_ptr; WinEnt* win_ent;
};

bool win_supported(int C1, int Ci, int k, int s, int ok, int oCo, int d1, int d0);
// per-window row lists of a pass (win_ptr, win_ent); needed once per pass before launch_bottom_win
void launch_win_rows(const WinArgs& a, int n_inst, hipStream_t st);
void launch_bottom_win(const WinArgs& a, int n_inst, hipStream_t st);
void launch_bottom_win_reduce(const WinArgs& a, int n_inst, hipStream_t st);

}  // namespace mnb
