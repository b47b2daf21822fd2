"""Where the report-writing GPU tests put their JSON: the directory named by
DHT_REPORT_DIR when it is set and exists, else nowhere."""
import json
import os


def write_report(name: str, data) -> None:
    d = os.environ.get("DHT_REPORT_DIR")
    if d and os.path.isdir(d):
        with open(os.path.join(d, name), "w") as f:
            json.dump(data, f, indent=1)
