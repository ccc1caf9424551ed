// Prints the field offsets and sizes of the C-ABI structs (include/cggm.h)
// for comparison with the ctypes mirrors of the Python binding.
#include <stdio.h>
#include <stddef.h>
#include "cggm.h"
int main(){
#define R(f) printf("req %s %zu\n", #f, offsetof(cggm_request, f));
R(X)R(Y)R(n)R(p)R(q)R(npath)R(lamL)R(lamT)R(tol)R(precision)R(max_iter)R(lambda_passes)R(mixed_min_q)R(Lambda_out)R(Theta_out)R(dtype)R(tile)
printf("req size %zu\n", sizeof(cggm_request));
#define O(f) printf("opt %s %zu\n", #f, offsetof(cggm_options, f));
O(max_iter)O(max_ls)O(ls_beta)O(ls_sigma)O(stall_iters)O(sweep)O(tile)O(lambda_passes)O(precision)O(mixed_min_q)O(workspace_budget)O(warm_Lambda)O(warm_Theta)O(trace)O(trace_cap)O(trace_len)O(kstats)O(theta_passes)O(split_level)O(split_adapt)O(blockwise)O(sxx_cache_bytes)O(graphs)
printf("opt size %zu\n", sizeof(cggm_options));
#define I(f) printf("info %s %zu\n", #f, offsetof(cggm_request_info, f));
I(status)I(slot)I(iters_total)I(t_submit_ms)I(t_admit_ms)I(t_done_ms)I(footprint)
printf("info size %zu\n", sizeof(cggm_request_info));
#define S(f) printf("stats %s %zu\n", #f, offsetof(cggm_server_stats, f));
S(submitted)S(completed)S(rejected)S(max_running)S(pool_bytes)S(peak_bytes_in_use)
printf("stats size %zu\n", sizeof(cggm_server_stats));
#define T(f) printf("trace %s %zu\n", #f, offsetof(cggm_trace_entry, f));
T(iter)T(ls_trials)T(sweep_fallbacks)T(sweep_split)T(f)T(subgrad_l1)T(l1)T(alpha)T(m_Lambda)T(m_Theta)
T(nnz_Lambda)T(nnz_Theta)T(t_end_ms)T(ms_gradient)T(ms_lambda_cd)T(ms_line_search)T(ms_theta_cd)T(delta)
printf("trace size %zu\n", sizeof(cggm_trace_entry));
#define K(f) printf("kstats %s %zu\n", #f, offsetof(cggm_kernel_stats, f));
K(waves)K(tiles)K(ms)K(bytes)K(flops)
printf("kstats size %zu\n", sizeof(cggm_kernel_stats));
return 0;}
