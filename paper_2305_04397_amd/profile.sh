#!/bin/bash
# rocprofv3 summaries of bench.py on the 50x100 workload (one warm-up step and
# one timed step): a kernel trace with per-kernel statistics, then one counter
# pass each for FETCH_SIZE and WRITE_SIZE, then the HBM bytes per sweep launch
# (traffic.txt).  The model upload's FP64->FP32 conversion kernels (a plain
# stream of known size: 8 bytes read, 4 written per element) calibrate the
# byte counters.  Two SQ counter passes follow (instruction mix, wave
# occupancy and waits of every kernel).  Output under $1 (default
# ./profile_out); $2 (optional) adds bench.py arguments, e.g. "--schedule 39"
# for the LDS-staged sweep.
set -o pipefail
OUT=${1:-profile_out}
EXTRA=${2:-}
REPO=$(cd "$(dirname "$0")/.." && pwd)
mkdir -p "$OUT"
OUT=$(cd "$OUT" && pwd)
cd /tmp && export TMPDIR=/tmp
# --no-graph: launches are enqueued one by one (rocprofv3's kernel tracing
# crashed the process replaying captured graphs); kernel durations do not
# depend on how the launches are submitted
ARGS="$REPO/bench.py --steps 1 --warmup 1 --queries 0 --proposer-queries 0 --no-cpu-baseline --no-graph $EXTRA"
SUM="python3 -m paper_2305_04397_amd.profile_summary"
echo "profile: kernel trace" && \
timeout -k 10 600 rocprofv3 --kernel-trace --stats -d "$OUT/trace" -o run --output-format csv -- python3 $ARGS \
    > "$OUT/trace.json" 2> "$OUT/trace.log" && (cd "$REPO" && $SUM "$OUT/trace" --delete-raw > /dev/null) && \
echo "profile: FETCH_SIZE" && \
timeout -s KILL 600 rocprofv3 --pmc FETCH_SIZE -d "$OUT/fetch" -o run --output-format csv -- python3 $ARGS \
    > "$OUT/fetch.log" 2>&1 && (cd "$REPO" && $SUM "$OUT/fetch" --delete-raw > /dev/null) && \
echo "profile: WRITE_SIZE" && \
timeout -s KILL 600 rocprofv3 --pmc WRITE_SIZE -d "$OUT/write" -o run --output-format csv -- python3 $ARGS \
    > "$OUT/write.log" 2>&1 && (cd "$REPO" && $SUM "$OUT/write" --delete-raw > /dev/null) && \
echo "profile: traffic" && \
(cd "$REPO" && $SUM traffic "$OUT/fetch" "$OUT/write" "$OUT/trace.json" "$OUT/traffic.txt" > /dev/null) && \
echo "profile: SQ counters (1)" && \
timeout -s KILL 600 rocprofv3 --pmc SQ_WAVES SQ_BUSY_CYCLES SQ_WAVE_CYCLES SQ_WAIT_ANY SQ_WAIT_INST_ANY SQ_ACTIVE_INST_ANY \
    SQ_ACTIVE_INST_VALU SQ_ACTIVE_INST_LDS -d "$OUT/sq1" -o run --output-format csv -- python3 $ARGS \
    > "$OUT/sq1.log" 2>&1 && (cd "$REPO" && $SUM "$OUT/sq1" --delete-raw > /dev/null) && \
echo "profile: SQ counters (2)" && \
timeout -s KILL 600 rocprofv3 --pmc SQ_INSTS_VALU SQ_INSTS_SALU SQ_INSTS_SMEM SQ_INSTS_LDS SQ_INSTS_VMEM_RD SQ_INSTS_VMEM_WR \
    SQ_LDS_BANK_CONFLICT TCC_HIT_sum -d "$OUT/sq2" -o run --output-format csv -- python3 $ARGS \
    > "$OUT/sq2.log" 2>&1 && (cd "$REPO" && $SUM "$OUT/sq2" --delete-raw > /dev/null)
