#!/bin/bash
# Host-only AddressSanitizer + UndefinedBehaviorSanitizer run of the oracle:
# builds oracle/liboracle_san.so and runs the CPU tests that call it (pins,
# lottery-loop traces, workload checks) with libasan preloaded into python.
# Any invalid access, leak-free heap misuse or undefined behaviour aborts the run.
set -euo pipefail
cd "$(dirname "$0")/.."
export ORACLE_SANITIZE=1
export ASAN_OPTIONS=detect_leaks=0:abort_on_error=1
export UBSAN_OPTIONS=print_stacktrace=1:halt_on_error=1
LD_PRELOAD="$(gcc -print-file-name=libasan.so):$(gcc -print-file-name=libubsan.so)" \
    python -m pytest tests -x -q -m "not gpu" -p no:cacheprovider "$@"
