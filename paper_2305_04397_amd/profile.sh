#!/bin/bash
# rocprofv3 summaries of bench.py on the 50x100 workload (one warm-up step and
# one timed step): a kernel trace with per-kernel statistics, then one counter
# pass each for FETCH_SIZE and WRITE_SIZE, then the HBM bytes per sweep launch
# (traffic.txt).  The model upload's FP64->FP32 conversion kernels (a plain
# stream of known size: 8 bytes read, 4 written per element) calibrate the
# byte counters.  Output under $1 (default ./profile_out).
set -o pipefail
OUT=${1:-profile_out}
REPO=$(cd "$(dirname "$0")/.." && pwd)
mkdir -p "$OUT"
OUT=$(cd "$OUT" && pwd)
cd /tmp && export TMPDIR=/tmp
ARGS="$REPO/bench.py --steps 1 --warmup 1 --queries 0 --proposer-queries 0 --no-cpu-baseline"
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
(cd "$REPO" && $SUM traffic "$OUT/fetch" "$OUT/write" "$OUT/trace.json" "$OUT/traffic.txt" > /dev/null)
