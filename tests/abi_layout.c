/* Prints the size and field offsets of the C ABI's structs, so the Python
 * ctypes mirrors can be checked against the compiler's layout. */
#include <stddef.h>
#include <stdio.h>
#include "mt.h"

#define F(T, f) printf(#T " " #f " %zu\n", offsetof(T, f))

int main(void) {
    printf("mt_params sizeof %zu\n", sizeof(mt_params));
    F(mt_params, step_m); F(mt_params, max_steps); F(mt_params, p_min); F(mt_params, seed);
    F(mt_params, n_variants); F(mt_params, scales); F(mt_params, mode); F(mt_params, block);
    F(mt_params, compact_every); F(mt_params, use_graph); F(mt_params, ckpt_every);
    F(mt_params, ckpt); F(mt_params, tape); F(mt_params, trace); F(mt_params, n_trace);
    F(mt_params, trace_steps); F(mt_params, tally); F(mt_params, z_det); F(mt_params, r_ap);
    F(mt_params, r_scale); F(mt_params, sampler); F(mt_params, interp);
    F(mt_params, stage_field);
    printf("mt_muons sizeof %zu\n", sizeof(mt_muons));
    F(mt_muons, x); F(mt_muons, y); F(mt_muons, z); F(mt_muons, px); F(mt_muons, py);
    F(mt_muons, pz); F(mt_muons, q);
    printf("mt_result sizeof %zu\n", sizeof(mt_result));
    F(mt_result, status); F(mt_result, n_steps); F(mt_result, volume);
    return 0;
}
