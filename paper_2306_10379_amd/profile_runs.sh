#!/bin/bash
# Regenerates the rocprofv3 summaries under profiles/. Run from the repository root on a
# machine with the GPU (the library built): bash paper_2306_10379_amd/profile_runs.sh
# Raw databases go to /tmp/gsi_prof (they are too large to keep with the results); the
# rocprofv3 logs go to $GSI_PROF_LOGS (default: prof_logs/ at the repository root). Each
# summary records the command that produced it.
# rocprofv3 may exit with a segmentation fault after the profiled program has finished and
# its database is complete; a step counts as done when its database exists.
R=$(pwd)
O=/tmp/gsi_prof
K=${GSI_PROF_LOGS:-prof_logs}
case "$K" in /*) ;; *) K=$R/$K ;; esac  # the steps run from /tmp
mkdir -p "$O" "$K"
export TMPDIR=/tmp
db() { find "$1" -name '*.db' | head -1; }
step() {  # step <dir> <timeout> <rocprofv3 arguments...>; counter runs are killed outright at the limit
  local d=$1 t=$2
  shift 2
  echo "== rocprofv3 $* (${d})"
  if [ "$1" = "--pmc" ]; then
    (cd /tmp && timeout -s KILL "$t" rocprofv3 "$@" > "$K/$(basename "$d").log" 2>&1)
  else
    (cd /tmp && timeout -k 10 "$t" rocprofv3 "$@" > "$K/$(basename "$d").log" 2>&1)
  fi
  local rc=$?
  if [ -z "$(db "$d")" ]; then echo "no database from ${d} (status $rc)"; return 1; fi
  echo "   done (status $rc)"
}
B="python3 $R/bench.py"
step "$O/c2_trace" 600 --kernel-trace --stats -d "$O/c2_trace" -o c2 -- $B --no-cpu --legs none --steps 1 --warmup 0 || exit 1
step "$O/c2_fetch" 120 --pmc FETCH_SIZE -d "$O/c2_fetch" -o f -- $B --profile-steps 3 || exit 1
step "$O/c2_write" 120 --pmc WRITE_SIZE -d "$O/c2_write" -o w -- $B --profile-steps 3 || exit 1
step "$O/c3_trace" 300 --kernel-trace --stats -d "$O/c3_trace" -o c3 -- $B --profile-steps 20 --profile-matrix spiked --profile-precision bf16 || exit 1
step "$O/c3_fetch" 180 --pmc FETCH_SIZE -d "$O/c3_fetch" -o f -- $B --profile-steps 3 --profile-matrix spiked --profile-precision bf16 || exit 1
step "$O/c3_write" 180 --pmc WRITE_SIZE -d "$O/c3_write" -o w -- $B --profile-steps 3 --profile-matrix spiked --profile-precision bf16 || exit 1
step "$O/w128_trace" 300 --kernel-trace --stats -d "$O/w128_trace" -o w128 -- $B --profile-steps 20 --profile-matrix spiked --profile-precision fp64 --p 128 || exit 1
step "$O/w128_fetch" 180 --pmc FETCH_SIZE -d "$O/w128_fetch" -o f -- $B --profile-steps 3 --profile-matrix spiked --profile-precision fp64 --p 128 || exit 1
step "$O/w128_write" 180 --pmc WRITE_SIZE -d "$O/w128_write" -o w -- $B --profile-steps 3 --profile-matrix spiked --profile-precision fp64 --p 128 || exit 1
step "$O/st_fetch" 120 --pmc FETCH_SIZE -d "$O/st_fetch" -o f -- $B --profile-steps 3 --profile-matrix stencil || exit 1
step "$O/st_write" 120 --pmc WRITE_SIZE -d "$O/st_write" -o w -- $B --profile-steps 3 --profile-matrix stencil || exit 1
step "$O/c4_trace" 400 --kernel-trace --stats -d "$O/c4_trace" -o c4 -- $B --legs-only --legs batched --steps 1 --warmup 0 || exit 1
step "$O/fno_trace" 300 --kernel-trace --stats -d "$O/fno_trace" -o fno -- python3 -m pytest $R/tests/test_gpu_fno.py -q -m gpu -p no:cacheprovider || exit 1
step "$O/warm_trace" 400 --kernel-trace --stats -d "$O/warm_trace" -o warm -- $B --legs-only --legs none --warm --no-cpu --warm-train 128 --warm-test 32 --warm-chunk 128 --warm-chunk-test 32 || exit 1
cd "$R"
S="python3 -m paper_2306_10379_amd.profsum"
C="bash paper_2306_10379_amd/profile_runs.sh (rocprofv3"
$S trace "$(db "$O/c2_trace")" "$C --kernel-trace --stats -- $B --no-cpu --legs none --steps 1 --warmup 0)" > profiles/kernels_laplace3d_128_p64_fp64.md
$S traffic "$(db "$O/c2_fetch")" "$(db "$O/c2_write")" "$C --pmc FETCH_SIZE / WRITE_SIZE -- $B --profile-steps 3)" profiles/traffic_laplace3d_128_p64_fp64.json > /dev/null
$S trace "$(db "$O/c3_trace")" "$C --kernel-trace --stats -- $B --profile-steps 20 --profile-matrix spiked --profile-precision bf16)" > profiles/kernels_spiked4M_p64_bf16.md
$S traffic "$(db "$O/c3_fetch")" "$(db "$O/c3_write")" "$C --pmc FETCH_SIZE / WRITE_SIZE -- $B --profile-steps 3 --profile-matrix spiked --profile-precision bf16)" profiles/traffic_spiked4M_p64_bf16.json > /dev/null
$S trace "$(db "$O/w128_trace")" "$C --kernel-trace --stats -- $B --profile-steps 20 --profile-matrix spiked --profile-precision fp64 --p 128)" > profiles/kernels_spiked4M_p128_fp64.md
$S traffic "$(db "$O/w128_fetch")" "$(db "$O/w128_write")" "$C --pmc FETCH_SIZE / WRITE_SIZE -- $B --profile-steps 3 --profile-matrix spiked --profile-precision fp64 --p 128)" profiles/traffic_spiked4M_p128_fp64.json > /dev/null
$S traffic "$(db "$O/st_fetch")" "$(db "$O/st_write")" "$C --pmc FETCH_SIZE / WRITE_SIZE -- $B --profile-steps 3 --profile-matrix stencil)" profiles/traffic_laplace3d_128_p64_fp64_stencil.json > /dev/null
$S trace "$(db "$O/c4_trace")" "$C --kernel-trace --stats -- $B --legs-only --legs batched --steps 1 --warmup 0)" > profiles/kernels_schrodinger_batch512.md
$S trace "$(db "$O/fno_trace")" "$C --kernel-trace --stats -- python3 -m pytest tests/test_gpu_fno.py)" > profiles/kernels_warmstart_network.md
$S trace "$(db "$O/warm_trace")" "$C --kernel-trace --stats -- $B --legs-only --legs none --warm --no-cpu --warm-train 128 --warm-test 32 --warm-chunk 128 --warm-chunk-test 32)" > profiles/kernels_warmstart_c5_bf16_small.md
cp profiles/*.md profiles/*.json "$K/" 2>/dev/null
echo "summaries written"
